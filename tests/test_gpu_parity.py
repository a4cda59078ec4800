"""GPU parity: the HIP path through the C ABI against the FP64 oracle on identical seeded inputs.

Gate (FP32 path): ||s_gpu - s_oracle||_2 / ||s_oracle||_2 <= 1e-5 and, per element,
max_m |s_gpu - s_oracle| / max_m |s_oracle| <= 1e-5.  The oracle draws its directions
with its own generator (oracle.directions) and the test asserts that the library's
plan holds the same ones; the sort permutation is bit-exact against the stable
argsort of the GPU's own FP32 projections (the sort's input).

The FP32 tolerance: the projection of a point has a rounding error of about
d 2^-24 sum_i |u_i xi_i| (a few 1e-7 relative), everything after it is FP32 with FP64
prefix sums and coefficient tables, and the measured errors are 1e-8 .. 2e-6.
"""
import math
import sys

import numpy as np
import pytest

import workloads as wlm

try:
    import torch  # noqa: F401  (import cost outside the per-test time limit)
except ImportError:  # pragma: no cover
    torch = None
from oracle import directions as odirs
from oracle import sliced

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def oracle_directions(d, P, seed, plan=None):
    """The oracle's own directions; asserts that a plan holds the same ones."""
    xi = odirs.directions(d, P, seed)
    if plan is not None:
        assert np.array_equal(plan.directions(), xi), "plan directions differ from the oracle's"
    return xi


def run_gpu(kernel, x, y, w, P, seed=0, probe=False, directions=None, **params):
    torch = _torch()
    import paper_2401_08260_amd as ks
    d = x.shape[1]
    plan = ks.Plan(d, P, kernel, seed=seed, directions=directions, **params)
    if directions is None:
        xi = oracle_directions(d, P, seed, plan)
    else:
        xi = np.asarray(directions, dtype=np.float64)
        assert np.array_equal(plan.directions(), xi)
    dev = torch.device("cuda:0")
    xt, yt, wt = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (x, y, w))
    N, M = x.shape[0], y.shape[0]
    pr = None
    if probe:
        pr = dict(z=torch.empty((P, M + N), dtype=torch.float32, device=dev),
                  bounds=torch.empty((P, 2), dtype=torch.float64, device=dev),
                  t=torch.empty((P, M), dtype=torch.float32, device=dev),
                  perm=torch.empty((P, M + N), dtype=torch.int32, device=dev) if kernel != "gaussian" else None)
    s = plan(xt, yt, wt, probe=pr)
    torch.cuda.synchronize()
    out = {"s": s.cpu().numpy().astype(np.float64), "xi": xi}
    if pr:
        for k, v in pr.items():
            if v is not None:
                out[k] = v.cpu().numpy()
    return out


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_s(kernel, x, y, w, xi, sigma=1.0, method="sort", n_coeff=0, T=0.0, slices=False, coeff_eps=0.0):
    return sliced.sliced_sum(kernel, x, y, w, xi, sigma, method, n_coeff, T, return_slices=slices,
                             coeff_eps=coeff_eps)


def max_rel(a, ref):
    """max_m |a_m - ref_m| / max_m |ref_m| (per-element error on the scale of the result)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))


def assert_parity(a, ref, tol=TOL, what="s"):
    """Normwise and per-element gate against the oracle."""
    e2, em = sliced.rel_l2(a, ref), max_rel(a, ref)
    note(f"  {what}: rel l2 {e2:.3e}, max elementwise {em:.3e}")
    assert e2 <= tol, (what, e2)
    assert em <= tol, (what, em)
    return e2


# ---------------------------------------------------------------------------
def test_projection_and_bounds():
    rng = np.random.default_rng(21)
    for (N, M, d, P) in [(300, 200, 784, 16), (1000, 77, 50, 130), (5, 3, 10, 1), (129, 1, 3, 2)]:
        note(f"projection N={N} M={M} d={d} P={P}")
        x = rng.random((N, d), dtype=np.float32)
        y = rng.standard_normal((M, d)).astype(np.float32)
        w = np.full(N, 1.0 / N, dtype=np.float32)
        r = run_gpu("negdist", x, y, w, P, seed=5, probe=True)
        xi = r["xi"]
        u = np.concatenate([y, x]).astype(np.float64)
        zref = (u @ xi.T).T                       # (P, M+N)
        bound = 4 * d * 2.0 ** -24 * (np.abs(u) @ np.abs(xi).T).T + 1e-30
        assert np.all(np.abs(r["z"] - zref) <= bound)
        z = r["z"].astype(np.float64)
        assert np.array_equal(r["bounds"][:, 0], z.min(axis=1))
        assert np.array_equal(r["bounds"][:, 1], z.max(axis=1))


def _check_perm(z, perm):
    for p in range(z.shape[0]):
        ref = np.argsort(z[p], kind="stable")
        assert np.array_equal(perm[p], ref), f"slice {p}"


@pytest.mark.parametrize("N,M,d,P", [(3000, 2000, 784, 16), (1, 1, 3, 2), (1, 5, 1, 1), (7, 1, 17, 3),
                                     (129, 130, 64, 5), (5000, 1, 8, 2), (20000, 30000, 32, 4)])
def test_negdist_parity_and_permutation(N, M, d, P):
    note(f"negdist N={N} M={M} d={d} P={P}")
    rng = np.random.default_rng(N + 7 * M + d)
    x = rng.random((N, d), dtype=np.float32)
    y = rng.random((M, d), dtype=np.float32)
    w = rng.random(N).astype(np.float32)
    r = run_gpu("negdist", x, y, w, P, seed=1, probe=True)
    _check_perm(r["z"], r["perm"])
    ref, ts = oracle_s("negdist", x, y, w, r["xi"], slices=True)
    assert_parity(r["s"], ref)
    assert_parity(r["t"], ts, what="t")


def test_negdist_max_buckets_large_union():
    """A union of 1.2 million points takes the largest bucket count of the sort path (2048):
    two buckets per thread in the scatter's tile scan, many groups per slice.  Permutations
    bit-exact, per-slice sums and the average against the oracle."""
    rng = np.random.default_rng(2048)
    N, M, d, P = 600000, 600000, 8, 4
    x = rng.standard_normal((N, d)).astype(np.float32)
    y = rng.standard_normal((M, d)).astype(np.float32)
    w = rng.random(N).astype(np.float32)
    note(f"negdist max buckets N={N} M={M} d={d} P={P}")
    r = run_gpu("negdist", x, y, w, P, seed=3, probe=True)
    _check_perm(r["z"], r["perm"])
    ref, ts = oracle_s("negdist", x, y, w, r["xi"], slices=True)
    assert_parity(r["s"], ref)
    assert_parity(r["t"], ts, what="t")


def test_negdist_more_slices_than_a_batch():
    """P = 2100 slices with the default slice batch, which the library caps at 1024: three
    batches (1024, 1024, 52) and the running average across them; ragged N, M."""
    rng = np.random.default_rng(2100)
    N, M, d, P = 700, 450, 12, 2100
    x = rng.random((N, d), dtype=np.float32)
    y = rng.random((M, d), dtype=np.float32)
    w = rng.random(N).astype(np.float32)
    note(f"negdist P={P} N={N} M={M} d={d}")
    r = run_gpu("negdist", x, y, w, P, seed=21, probe=True)
    _check_perm(r["z"][::97], r["perm"][::97])
    ref, ts = oracle_s("negdist", x, y, w, r["xi"], slices=True)
    assert_parity(r["s"], ref)
    assert_parity(r["t"], ts, what="t")


def test_negdist_signed_weights_and_ties():
    """Integer-valued coordinates give many equal projections (ties inside and across x, y)."""
    rng = np.random.default_rng(3)
    N, M, d, P = 6000, 4000, 4, 6
    x = rng.integers(0, 3, (N, d)).astype(np.float32)
    y = rng.integers(0, 3, (M, d)).astype(np.float32)
    w = rng.standard_normal(N).astype(np.float32)
    note("negdist ties")
    r = run_gpu("negdist", x, y, w, P, seed=2, probe=True)
    _check_perm(r["z"], r["perm"])
    ref = oracle_s("negdist", x, y, w, r["xi"])
    assert_parity(r["s"], ref)


def test_negdist_identical_points_large_group():
    """All sources at one point: one bucket far larger than LDS (streaming sort path)."""
    rng = np.random.default_rng(4)
    N, M, d, P = 20000, 3000, 16, 3
    x = np.tile(rng.random((1, d), dtype=np.float32), (N, 1))
    y = rng.random((M, d), dtype=np.float32)
    w = rng.random(N).astype(np.float32)
    note("negdist identical sources")
    r = run_gpu("negdist", x, y, w, P, seed=3, probe=True)
    _check_perm(r["z"], r["perm"])
    ref = oracle_s("negdist", x, y, w, r["xi"])
    assert_parity(r["s"], ref)
    # everything at one point: all projections equal, s = 0
    x2 = np.zeros((50, d), dtype=np.float32)
    r2 = run_gpu("negdist", x2, x2[:7].copy(), np.ones(50, np.float32), 2, probe=True)
    assert np.all(r2["s"] == 0.0)


def test_negdist_determinism_and_batching():
    rng = np.random.default_rng(5)
    N, M, d, P = 5000, 4000, 100, 12
    x = rng.random((N, d), dtype=np.float32)
    y = rng.random((M, d), dtype=np.float32)
    w = rng.random(N).astype(np.float32)
    note("negdist determinism")
    a = run_gpu("negdist", x, y, w, P, seed=9)["s"]
    b = run_gpu("negdist", x, y, w, P, seed=9)["s"]
    assert np.array_equal(a, b)
    c = run_gpu("negdist", x, y, w, P, seed=9, slice_batch=5)["s"]
    assert sliced.rel_l2(c, a) <= 1e-6


def test_gauss_ndft_workload_full_size_f64_input():
    wl = wlm.WORKLOADS["gauss_ndft"]
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    note("gauss_ndft full size")
    r = run_gpu("gaussian", x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=wl.n_coeff, T=wl.T,
                method="ndft")
    ref = oracle_s("gaussian", x, y, w, r["xi"], sigma, "ndft", wl.n_coeff, wl.T)
    assert_parity(r["s"], ref)


def test_gauss_ndft_ragged_fp32():
    rng = np.random.default_rng(6)
    for (N, M, d, P) in [(4097, 300, 10, 3), (1, 2, 5, 1), (9000, 5000, 30, 4)]:
        x = rng.standard_normal((N, d)).astype(np.float32)
        y = rng.standard_normal((M, d)).astype(np.float32)
        w = rng.random(N).astype(np.float32)
        sigma = float(np.sqrt(2 * d))
        note(f"gauss ndft N={N} M={M} d={d} P={P}")
        r = run_gpu("gaussian", x, y, w, P, seed=4, sigma=sigma, n_coeff=64, T=0.045, method="ndft", probe=True)
        ref = oracle_s("gaussian", x, y, w, r["xi"], sigma, "ndft", 64, 0.045)
        assert_parity(r["s"], ref)


@pytest.mark.parametrize("n_coeff", [2, 16, 30])
def test_gauss_ndft_coefficient_counts(n_coeff):
    """The NDFT adjoint takes its coefficients in groups of 8, one block per group: K + 1 = 2
    (one partial group), 9 (a full group and one) and 16 (two full groups), with two chunks of
    sources and a partial target chunk."""
    rng = np.random.default_rng(n_coeff)
    N, M, d, P = 5000, 700, 10, 5
    x = rng.standard_normal((N, d)).astype(np.float32)
    y = rng.standard_normal((M, d)).astype(np.float32)
    w = rng.random(N).astype(np.float32)
    sigma = float(np.sqrt(2 * d))
    note(f"gauss ndft n_coeff={n_coeff}")
    r = run_gpu("gaussian", x, y, w, P, seed=8, sigma=sigma, n_coeff=n_coeff, T=0.045, method="ndft")
    ref = oracle_s("gaussian", x, y, w, r["xi"], sigma, "ndft", n_coeff, 0.045)
    assert_parity(r["s"], ref)


def test_gauss_nfft_workload_reduced():
    wl = wlm.scaled(wlm.WORKLOADS["gauss_nfft"], N=20000, M=15000, P=6)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    note("gauss_nfft reduced")
    r = run_gpu("gaussian", x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=wl.n_coeff, T=wl.T,
                method="nfft", oversample=2, window_m=6)
    ref = oracle_s("gaussian", x, y, w, r["xi"], sigma, "nfft", wl.n_coeff, wl.T)
    assert_parity(r["s"], ref)


@pytest.mark.parametrize("m,tol", [(2, 1e-3), (3, 1e-4), (4, TOL), (5, TOL), (7, TOL), (8, TOL)])
def test_gauss_nfft_window_widths(m, tol):
    """The NFFT with other Kaiser-Bessel half-widths m than the workloads' 6 (each m is its own
    kernel instance).  The oracle sums the truncated Fourier series exactly, so the difference
    is the window's aliasing error, which falls roughly like exp(-2 pi m sqrt(1 - 1/sigma)) for
    oversampling sigma = 2 (about 1e-4 at m = 2, 1e-6 at m = 3), above the FP32 floor only for
    m <= 3: the tolerance is 1e-5 from m = 4 on."""
    wl = wlm.scaled(wlm.WORKLOADS["gauss_nfft"], N=6000, M=4000, P=4)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    note(f"gauss_nfft window m={m}")
    r = run_gpu("gaussian", x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=wl.n_coeff, T=wl.T,
                method="nfft", oversample=2, window_m=m)
    ref = oracle_s("gaussian", x, y, w, r["xi"], sigma, "nfft", wl.n_coeff, wl.T)
    assert_parity(r["s"], ref, tol)


@pytest.mark.parametrize("kernel,n_coeff,oversample", [("gaussian", 64, 2), ("gaussian", 256, 2),
                                                      ("gaussian", 128, 4), ("laplacian", 512, 2)])
def test_nfft_grid_sizes(kernel, n_coeff, oversample):
    """Other coefficient counts and oversampling factors than the workloads': FFT lengths 128
    to 1024 in LDS, and with them other window widths and lane sharing in the spread."""
    base = "gauss_nfft" if kernel == "gaussian" else "laplace"
    wl = wlm.scaled(wlm.WORKLOADS[base], N=5000, M=3500, P=4)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    note(f"{kernel} nfft n_coeff={n_coeff} oversample={oversample}")
    r = run_gpu(kernel, x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=n_coeff, T=wl.T,
                method="nfft", oversample=oversample, window_m=6)
    ref = oracle_s(kernel, x, y, w, r["xi"], sigma, "nfft", n_coeff, wl.T)
    assert_parity(r["s"], ref)


def test_laplace_workload_reduced():
    wl = wlm.scaled(wlm.WORKLOADS["laplace"], N=4000, M=3000, P=6)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    note("laplace reduced")
    r = run_gpu("laplacian", x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=wl.n_coeff, T=wl.T,
                probe=True)
    _check_perm(r["z"], r["perm"])
    ref = oracle_s("laplacian", x, y, w, r["xi"], sigma, "nfft", wl.n_coeff, wl.T)
    assert_parity(r["s"], ref)


@pytest.mark.parametrize("n_coeff", [128, 512])
def test_laplace_coefficient_transforms(n_coeff):
    """The Laplacian's smooth-part coefficients come from 16 n_coeff samples: up to 4096 of
    them (128 coefficients: 2048 samples) the set-up takes an FFT, beyond that (512: 8192)
    its direct transform.  Both against the oracle's own quadrature."""
    rng = np.random.default_rng(96 + n_coeff)
    N, M, d, P = 2500, 1800, 24, 5
    x = rng.random((N, d), dtype=np.float32)
    y = rng.random((M, d), dtype=np.float32)
    w = rng.random(N).astype(np.float32)
    sigma = float(np.sqrt(d / 6.0))
    note(f"laplace coefficients n_coeff={n_coeff}")
    r = run_gpu("laplacian", x, y, w, P, seed=9, sigma=sigma, n_coeff=n_coeff, T=0.125, probe=True)
    ref, ts = oracle_s("laplacian", x, y, w, r["xi"], sigma, "nfft", n_coeff, 0.125, slices=True)
    assert_parity(r["s"], ref)
    assert_parity(r["t"], ts, what="t")


def test_negdist_workload_full_size():
    """The negative-distance workload at its full size (N=M=1e5, d=784, P=256)."""
    wl = wlm.WORKLOADS["negdist"]
    x, y, w = wlm.generate(wl)
    note("negdist full size")
    r = run_gpu("negdist", x, y, w, wl.P, seed=wl.dir_seed)
    ref = oracle_s("negdist", x, y, w, r["xi"])
    assert_parity(r["s"], ref)


def test_matern_reduced():
    """Matern nu = 3/2 with the paper's NFFT setting (1024 coefficients), mixture data."""
    wl = wlm.scaled(wlm.WORKLOADS["gauss_nfft"], N=20000, M=15000, P=4)
    x, y, w = wlm.generate(wl)
    beta = wlm.median_heuristic(x, y)
    note("matern reduced")
    r = run_gpu("matern", x, y, w, wl.P, seed=6, sigma=beta, n_coeff=1024, T=0.125, probe=True)
    ref, ts = oracle_s("matern", x, y, w, r["xi"], beta, "nfft", 1024, 0.125, slices=True)
    assert_parity(r["s"], ref)
    assert_parity(r["t"], ts, what="t")


def test_laplace_many_slices_batched_ragged():
    """Laplacian (NFFT + sort) with P = 70 in slice batches of 32 (so 32, 32, 6), ragged
    N and M: more slices than one LDS sub-batch of the interpolation holds for this
    window (57), batches of 8 slices with a partial last one, and the running sum
    across slice batches.  Per-slice sums and the average against the oracle."""
    rng = np.random.default_rng(70)
    N, M, d, P = 1500, 700, 48, 70
    x = rng.random((N, d), dtype=np.float32)
    y = rng.random((M, d), dtype=np.float32)
    w = rng.random(N).astype(np.float32)
    sigma = float(np.sqrt(d / 6.0))
    note(f"laplace batched N={N} M={M} d={d} P={P}")
    r = run_gpu("laplacian", x, y, w, P, seed=11, sigma=sigma, n_coeff=256, T=0.125, slice_batch=32, probe=True)
    ref, ts = oracle_s("laplacian", x, y, w, r["xi"], sigma, "nfft", 256, 0.125, slices=True)
    assert_parity(r["s"], ref)
    assert_parity(r["t"], ts, what="t")


# ---------------------------------------------------------------------------
# NFFT spread in several source chunks (Remark "Non-equispaced FFT", Sec. 3.1): a spread
# block takes 32 768 sources of a slice, so N = 3 * 32768 + 1001 gives three full chunks
# and a ragged fourth, and the grid kernel reduces four chunk partials per slice.
NFFT_CHUNK = 32768


@pytest.mark.parametrize("kernel", ["gaussian", "laplacian", "matern"])
def test_nfft_several_spread_chunks(kernel):
    base = "laplace" if kernel == "laplacian" else "gauss_nfft"
    wl = wlm.scaled(wlm.WORKLOADS[base], N=3 * NFFT_CHUNK + 1001, M=7000, d=12, P=3)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    n_coeff = 1024 if kernel == "matern" else wl.n_coeff
    T = 0.125 if kernel == "matern" else wl.T
    note(f"{kernel} nfft N={wl.N} (4 spread chunks) M={wl.M} d={wl.d} P={wl.P}")
    r = run_gpu(kernel, x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=n_coeff, T=T,
                method="nfft", probe=True)
    if kernel == "laplacian":
        _check_perm(r["z"], r["perm"])
    ref, ts = oracle_s(kernel, x, y, w, r["xi"], sigma, "nfft", n_coeff, T, slices=True)
    assert_parity(r["s"], ref)
    assert_parity(r["t"], ts, what="t")


@pytest.mark.timeout(900)
def test_gauss_nfft_workload_full_points():
    """The Gaussian NFFT workload at its full N = M = 1e6 and d = 50 (31 spread chunks per
    slice), with 4 of its 256 directions; every target against the oracle."""
    wl = wlm.scaled(wlm.WORKLOADS["gauss_nfft"], P=4)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    note(f"gauss_nfft full N={wl.N} M={wl.M} d={wl.d}, P={wl.P}")
    r = run_gpu("gaussian", x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=wl.n_coeff, T=wl.T,
                method="nfft", oversample=wl.oversample, window_m=wl.window_m)
    ref = oracle_s("gaussian", x, y, w, r["xi"], sigma, "nfft", wl.n_coeff, wl.T)
    assert_parity(r["s"], ref)


@pytest.mark.timeout(900)
def test_laplace_workload_full_points():
    """The Laplacian workload at its full N = M = 2e5 and d = 3072 (7 spread chunks, sort
    groups over 4e5 keys per slice), with 4 of its 512 directions; every target and every
    permutation against the oracle."""
    wl = wlm.scaled(wlm.WORKLOADS["laplace"], P=4)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    note(f"laplace full N={wl.N} M={wl.M} d={wl.d}, P={wl.P}")
    r = run_gpu("laplacian", x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=wl.n_coeff, T=wl.T,
                probe=True)
    _check_perm(r["z"], r["perm"])
    ref, ts = oracle_s("laplacian", x, y, w, r["xi"], sigma, "nfft", wl.n_coeff, wl.T, slices=True)
    assert_parity(r["s"], ref)
    assert_parity(r["t"], ts, what="t")


# ---------------------------------------------------------------------------
# The cutoff set of eq. "Fourier_cutoff" (Sec. 2.2): coefficients with |c_k| <= eps leave
# the sum.  eps is chosen so that the result moves well beyond the tolerance against
# eps = 0, and (checked on the oracle's coefficients) so that no coefficient lies within
# 1e-4 relative of eps, where an FP32 rescaling could take the other decision.
def _eps_margin(kernel, d, x, y, xi, sigma, method, n_coeff, T, eps):
    from oracle import kernels as kn
    zx, zy = sliced.project(x, xi), sliced.project(y, xi)
    K = sliced.cutoff_K(method, n_coeff)
    ks = np.arange(-K, K + 1)
    worst = np.inf
    for p in range(xi.shape[0]):
        _, _, tau = sliced.rescale(zx[:, p], zy[:, p], T, sigma)
        if kernel == "gaussian":
            c = kn.gauss_fourier_coeff(d, tau * sigma, ks)
        else:
            c = kn.laplace_smooth_coeffs(d, 1.0 / (sigma * tau), K, 16 * n_coeff)[1]
        c = np.abs(c[c != 0.0])
        worst = min(worst, float(np.min(np.abs(c / eps - 1.0))))
    return worst


@pytest.mark.parametrize("kernel,method,base", [("gaussian", "ndft", "gauss_ndft"), ("gaussian", "nfft", "gauss_nfft"),
                                                ("laplacian", "nfft", "laplace")])
def test_coeff_eps_cutoff(kernel, method, base):
    wl = wlm.scaled(wlm.WORKLOADS[base], N=6000, M=4000, d=20, P=5)
    x, y, w = wlm.generate(wl)
    if wl.dtype == "f64":
        x, y, w = (a.astype(np.float32) for a in (x, y, w))
    sigma = wlm.median_heuristic(x, y)
    xi = oracle_directions(wl.d, wl.P, wl.dir_seed)
    eps = {"gauss_ndft": 2e-3, "gauss_nfft": 3e-4, "laplace": 2e-2}[base]
    margin = _eps_margin(kernel, wl.d, x, y, xi, sigma, method, wl.n_coeff, wl.T, eps)
    assert margin > 1e-4, margin
    note(f"{kernel} {method} coeff_eps={eps} (closest coefficient {margin:.2e} relative from eps)")
    r = run_gpu(kernel, x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=wl.n_coeff, T=wl.T,
                method=method, coeff_eps=eps)
    ref = oracle_s(kernel, x, y, w, xi, sigma, method, wl.n_coeff, wl.T, coeff_eps=eps)
    ref0 = oracle_s(kernel, x, y, w, xi, sigma, method, wl.n_coeff, wl.T)
    moved = sliced.rel_l2(ref, ref0)
    note(f"  eps moves the oracle result by {moved:.3e}")
    assert moved > 10 * TOL
    assert_parity(r["s"], ref)
