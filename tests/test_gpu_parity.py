"""GPU parity: the HIP path through the C ABI against the FP64 oracle on identical seeded inputs.

Gate (FP32 path): ||s_gpu - s_oracle||_2 / ||s_oracle||_2 <= 1e-5, with the same
directions on both sides; the sort permutation is bit-exact against the stable
argsort of the GPU's own FP32 projections.
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
from oracle import sliced

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_gpu(kernel, x, y, w, P, seed=0, probe=False, **params):
    torch = _torch()
    import paper_2401_08260_amd as ks
    d = x.shape[1]
    plan = ks.Plan(d, P, kernel, seed=seed, **params)
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
    out = {"s": s.cpu().numpy().astype(np.float64), "xi": plan.directions()}
    if pr:
        for k, v in pr.items():
            if v is not None:
                out[k] = v.cpu().numpy()
    return out


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_s(kernel, x, y, w, xi, sigma=1.0, method="sort", n_coeff=0, T=0.0, slices=False):
    return sliced.sliced_sum(kernel, x, y, w, xi, sigma, method, n_coeff, T, return_slices=slices)


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
    assert sliced.rel_l2(r["s"], ref) <= TOL
    assert sliced.rel_l2(r["t"].astype(np.float64), ts) <= TOL


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
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= TOL
    assert sliced.rel_l2(r["t"].astype(np.float64), ts) <= TOL


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
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= TOL
    assert sliced.rel_l2(r["t"].astype(np.float64), ts) <= TOL


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
    assert sliced.rel_l2(r["s"], ref) <= TOL


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
    assert sliced.rel_l2(r["s"], ref) <= TOL
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
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= TOL


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
        assert sliced.rel_l2(r["s"], ref) <= TOL


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
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= TOL


def test_gauss_nfft_workload_reduced():
    wl = wlm.scaled(wlm.WORKLOADS["gauss_nfft"], N=20000, M=15000, P=6)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    note("gauss_nfft reduced")
    r = run_gpu("gaussian", x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=wl.n_coeff, T=wl.T,
                method="nfft", oversample=2, window_m=6)
    ref = oracle_s("gaussian", x, y, w, r["xi"], sigma, "nfft", wl.n_coeff, wl.T)
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= TOL


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
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= tol


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
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= TOL


def test_laplace_workload_reduced():
    wl = wlm.scaled(wlm.WORKLOADS["laplace"], N=4000, M=3000, P=6)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    note("laplace reduced")
    r = run_gpu("laplacian", x, y, w, wl.P, seed=wl.dir_seed, sigma=sigma, n_coeff=wl.n_coeff, T=wl.T,
                probe=True)
    _check_perm(r["z"], r["perm"])
    ref = oracle_s("laplacian", x, y, w, r["xi"], sigma, "nfft", wl.n_coeff, wl.T)
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= TOL


def test_negdist_workload_full_size():
    """The negative-distance workload at its full size (N=M=1e5, d=784, P=256)."""
    wl = wlm.WORKLOADS["negdist"]
    x, y, w = wlm.generate(wl)
    note("negdist full size")
    r = run_gpu("negdist", x, y, w, wl.P, seed=wl.dir_seed)
    ref = oracle_s("negdist", x, y, w, r["xi"])
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= TOL


def test_matern_reduced():
    """Matern nu = 3/2 with the paper's NFFT setting (1024 coefficients), mixture data."""
    wl = wlm.scaled(wlm.WORKLOADS["gauss_nfft"], N=20000, M=15000, P=4)
    x, y, w = wlm.generate(wl)
    beta = wlm.median_heuristic(x, y)
    note("matern reduced")
    r = run_gpu("matern", x, y, w, wl.P, seed=6, sigma=beta, n_coeff=1024, T=0.125, probe=True)
    ref, ts = oracle_s("matern", x, y, w, r["xi"], beta, "nfft", 1024, 0.125, slices=True)
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= TOL
    assert sliced.rel_l2(r["t"].astype(np.float64), ts) <= TOL


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
    err = sliced.rel_l2(r["s"], ref)
    note(f"  rel err {err:.3e}")
    assert err <= TOL
    assert sliced.rel_l2(r["t"].astype(np.float64), ts) <= TOL
