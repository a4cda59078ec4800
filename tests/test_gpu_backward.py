"""GPU parity of the backward pass (ksum_backward) against the FP64 oracle gradient, and a
finite-difference check of the GPU gradient on the Laplacian workload's shape.

The oracle computes everything itself: its own directions (oracle.directions) or the
explicit ones the test passes to both sides, its own FP64 projections, its own derivative
sums (oracle.gradient.sliced_grad).  Nothing it sees comes from the HIP path.

The derivative sums of the sort path (negative distance, the Laplacian's |.| part) jump
where two projections cross (sign(0) = 0, reading of the gradient), so FP32 and FP64
projections of random data could take different sign decisions.  Those tests use inputs
whose FP32 projections are exact: directions with 4^j nonzero entries +-2^-j (unit norm
exactly) and coordinates k 2^-b, so every product and partial sum of the projection is a
dyadic number within FP32's 24 bits, and the GPU's FP32 (or split-BF16) GEMM gives the FP64
projection bit for bit.  The smooth Fourier paths (Gaussian, Matern) use the workloads'
random directions and data.

Gate: relative l2 error and max elementwise error / max |ref| <= 1e-5 per gradient (FP32).
"""
import numpy as np
import pytest

import workloads as wlm
from oracle import gradient, sliced
from test_gpu_parity import assert_parity, note, oracle_directions

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dyadic_directions(d, P, rng):
    """P unit vectors with 4^j nonzeros +-2^-j on a random support (4^j <= min(d, 64))."""
    j = 0
    while 4 ** (j + 1) <= min(d, 64):
        j += 1
    s = 4 ** j
    xi = np.zeros((P, d))
    for p in range(P):
        idx = rng.choice(d, size=s, replace=False)
        xi[p, idx] = rng.choice([-1.0, 1.0], size=s) * 2.0 ** -j
    return xi, j


def dyadic_points(n, d, bits, rng):
    """n x d coordinates k 2^-bits, k uniform in [0, 2^bits): exact in FP32."""
    return (rng.integers(0, 2 ** bits, size=(n, d)) * 2.0 ** -bits).astype(np.float32)


def dyadic_case(N, M, d, P, seed, bits=None):
    rng = np.random.default_rng(seed)
    xi, j = dyadic_directions(d, P, rng)
    # |projection| < 2^j with resolution 2^-(bits+j): within 24 bits for bits <= 23 - 2j
    b = 23 - 2 * j if bits is None else bits
    x = dyadic_points(N, d, b, rng)
    y = dyadic_points(M, d, b, rng)
    w = rng.random(N).astype(np.float32)
    g = rng.standard_normal(M).astype(np.float32)
    return x, y, w, g, xi


def run_backward(kernel, x, y, w, g, P, seed=0, directions=None, **params):
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
    xt, yt, wt, gt = (torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev) for a in (x, y, w, g))
    gx, gy, gw = plan.backward(xt, yt, wt, gt)
    torch.cuda.synchronize()
    return dict(gx=gx.cpu().numpy().astype(np.float64), gy=gy.cpu().numpy().astype(np.float64),
                gw=gw.cpu().numpy().astype(np.float64), xi=xi)


def check(kernel, x, y, w, g, P, seed=0, directions=None, ref_kw=None, tol=TOL, **params):
    ref_kw = ref_kw or {}
    r = run_backward(kernel, x, y, w, g, P, seed=seed, directions=directions, **params)
    xd, yd, wd, gd = (np.asarray(a, dtype=np.float32).astype(np.float64) for a in (x, y, w, g))
    gx_ref, gy_ref, gw_ref = gradient.sliced_grad(kernel, xd, yd, wd, gd, r["xi"], **ref_kw)
    assert_parity(r["gx"], gx_ref, tol, "grad_x")
    assert_parity(r["gy"], gy_ref, tol, "grad_y")
    assert_parity(r["gw"], gw_ref, tol, "grad_w")
    return r


@pytest.mark.parametrize("N,M,d,P", [(3000, 2000, 64, 8), (1, 1, 3, 2), (700, 5, 17, 3), (5000, 4000, 784, 4)])
def test_backward_negdist(N, M, d, P):
    note(f"backward negdist N={N} M={M} d={d} P={P} (exact dyadic projections)")
    x, y, w, g, xi = dyadic_case(N, M, d, P, N + M + d)
    y[: min(M, N) // 2] = x[: min(M, N) // 2]          # targets on top of sources: ties
    check("negdist", x, y, w, g, P, directions=xi)


def test_backward_negdist_identical_points():
    # every projection of a slice equal: all groups go to the fallback kernel
    note("backward negdist identical points")
    N, M, d, P = 6000, 3000, 8, 3
    x = np.full((N, d), 0.25, dtype=np.float32)
    y = np.full((M, d), 0.25, dtype=np.float32)
    rng = np.random.default_rng(1)
    w = rng.random(N).astype(np.float32)
    g = rng.standard_normal(M).astype(np.float32)
    r = run_backward("negdist", x, y, w, g, P, seed=2)
    # sign(0) = 0 everywhere: no gradient with respect to the points
    assert np.all(r["gx"] == 0.0) and np.all(r["gy"] == 0.0)


def test_backward_negdist_large_ties_fallback():
    # a large group of equal keys with sources and targets mixed: the streaming fallback
    note("backward negdist large tie group")
    N, M, d, P = 12000, 9000, 4, 2
    x, y, w, g, xi = dyadic_case(N, M, d, P, 5)
    x[:7000] = 0.5
    y[:5000] = 0.5
    check("negdist", x, y, w, g, P, directions=xi)


@pytest.mark.parametrize("N,M,d,P", [(2000, 1500, 16, 6), (4097, 300, 10, 3)])
def test_backward_gauss_ndft(N, M, d, P):
    note(f"backward gauss ndft N={N} M={M} d={d} P={P}")
    rng = np.random.default_rng(N + d)
    x = rng.standard_normal((N, d)).astype(np.float32)
    y = rng.standard_normal((M, d)).astype(np.float32)
    w = rng.random(N).astype(np.float32)
    g = rng.standard_normal(M).astype(np.float32)
    sigma = float(np.sqrt(2 * d))
    kw = dict(sigma=sigma, method="ndft", n_coeff=64, T=0.045)
    check("gaussian", x, y, w, g, P, seed=1, ref_kw=kw, **kw)


def test_backward_gauss_nfft_reduced():
    wl = wlm.scaled(wlm.WORKLOADS["gauss_nfft"], N=20000, M=15000, P=4)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    g = np.random.default_rng(8).standard_normal(wl.M).astype(np.float32)
    note("backward gauss nfft reduced")
    kw = dict(sigma=sigma, method="nfft", n_coeff=wl.n_coeff, T=wl.T)
    check("gaussian", x, y, w, g, wl.P, seed=wl.dir_seed, ref_kw=kw, oversample=2, window_m=6, **kw)


def test_backward_laplace_reduced():
    """The Laplacian workload's d = 3072 with exact dyadic projections (N = 4000, M = 3000, P = 6)."""
    x, y, w, g, xi = dyadic_case(4000, 3000, 3072, 6, 9)
    w[:] = np.float32(1.0 / 4000)
    sigma = wlm.median_heuristic(x, y)
    note("backward laplace reduced (exact dyadic projections)")
    kw = dict(sigma=sigma, method="nfft", n_coeff=256, T=0.125)
    check("laplacian", x, y, w, g, 6, directions=xi, ref_kw=kw, **kw)


def test_backward_laplace_workload_shape_vs_oracle():
    """The Laplacian workload's d = 3072 with 64 directions and N = M = 1000 (exact dyadic
    projections): every gradient entry against the oracle gradient."""
    x, y, w, g, xi = dyadic_case(1000, 1000, 3072, 64, 10)
    w[:] = np.float32(1.0 / 1000)
    sigma = wlm.median_heuristic(x, y)
    note("backward laplace d=3072 P=64 vs oracle (exact dyadic projections)")
    kw = dict(sigma=sigma, method="nfft", n_coeff=256, T=0.125)
    check("laplacian", x, y, w, g, 64, directions=xi, ref_kw=kw, **kw)


def test_backward_laplace_workload_shape_finite_differences():
    """Central differences (h = 1e-3) of L = sum_m g_m s_m on 32 coordinates against the GPU
    gradient, on the Laplacian workload's shape (d = 3072, P = 512, its directions, sigma by
    the median heuristic, U[0,1] points, w = 1/N) with N = M = 48 points.

    The forward is linear in the sources and weights for fixed directions, and the sliced
    kernel is symmetric in its two arguments, so the central difference of L in x_{n,i} is
    sum_m g_m s'_m / (2h) for the forward s' with the two sources x_n +- h e_i and weights
    +-w_n (every other source cancels exactly), and in y_{m,i} it is g_m sum_n w_n s''_n / (2h)
    for the forward s'' with the two sources y_m +- h e_i, weights +-1 and targets x.  Computing
    the differences this way keeps the FP32 rounding of s (about 6e-8 |s|, larger than the
    change 2h |dL/dx| itself) out of them.  The rescaling bounds of these small forwards
    differ from the full one's, which changes the sums only by the truncation error.  For w
    the plain central difference of two full forwards is used (L is linear in w).

    Tolerance: the FD quotient differs from the derivative where a projection pair crosses
    within h (the |.| kink of the Laplacian's sorted part); with the oracle in FP64 on this
    case that is 5.5e-4 of max |grad|.  Gate: 1e-2 of max |grad| for x and y, 1e-3 relative
    for w."""
    torch = _torch()
    import paper_2401_08260_amd as ks
    wl = wlm.scaled(wlm.WORKLOADS["laplace"], N=48, M=48)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    g = np.random.default_rng(5).standard_normal(wl.M).astype(np.float32)
    kw = dict(sigma=sigma, method="nfft", n_coeff=wl.n_coeff, T=wl.T)
    plan = ks.Plan(wl.d, wl.P, "laplacian", seed=wl.dir_seed, **kw)
    dev = torch.device("cuda:0")

    def dev_(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

    xt, yt, wt, gt = dev_(x), dev_(y), dev_(w), dev_(g)
    gx, gy, gw = (t.cpu().numpy().astype(np.float64) for t in plan.backward(xt, yt, wt, gt))
    g64 = g.astype(np.float64)
    h = 1e-3
    rng = np.random.default_rng(1)
    note("backward laplace d=3072 P=512 N=M=48: finite differences on 32 coordinates")
    fd_xy, an_xy = [], []
    for _ in range(12):
        n, i = int(rng.integers(wl.N)), int(rng.integers(wl.d))
        src = np.stack([x[n], x[n]]).astype(np.float64)
        src[0, i] += h
        src[1, i] -= h
        src = src.astype(np.float32)                   # the step as the GPU sees it
        step = float(src[0, i]) - float(src[1, i])
        s = plan(dev_(src), yt, dev_([w[n], -w[n]])).cpu().numpy().astype(np.float64)
        fd_xy.append(g64 @ s / step)
        an_xy.append(gx[n, i])
    for _ in range(12):
        m, i = int(rng.integers(wl.M)), int(rng.integers(wl.d))
        src = np.stack([y[m], y[m]]).astype(np.float64)
        src[0, i] += h
        src[1, i] -= h
        src = src.astype(np.float32)
        step = float(src[0, i]) - float(src[1, i])
        s = plan(dev_(src), xt, dev_([1.0, -1.0])).cpu().numpy().astype(np.float64)
        fd_xy.append(g64[m] * (w.astype(np.float64) @ s) / step)
        an_xy.append(gy[m, i])
    fd_w, an_w = [], []
    for _ in range(8):
        n = int(rng.integers(wl.N))
        vals, wn = [], []
        for sg in (1.0, -1.0):
            ww = w.astype(np.float64).copy()
            ww[n] += sg * h
            ww = ww.astype(np.float32)
            wn.append(float(ww[n]))
            vals.append(g64 @ plan(xt, yt, dev_(ww)).cpu().numpy().astype(np.float64))
        fd_w.append((vals[0] - vals[1]) / (wn[0] - wn[1]))
        an_w.append(gw[n])
    fd_xy, an_xy, fd_w, an_w = map(np.asarray, (fd_xy, an_xy, fd_w, an_w))
    scale = max(np.abs(gx).max(), np.abs(gy).max())
    e_xy = float(np.max(np.abs(fd_xy - an_xy)) / scale)
    e_w = float(np.max(np.abs(fd_w - an_w) / np.abs(an_w)))
    note(f"  x, y: max |fd - grad| / max |grad| = {e_xy:.3e};  w: max relative {e_w:.3e}")
    assert e_xy <= 1e-2
    assert e_w <= 1e-3


def test_autograd_function_and_translation_invariance():
    torch = _torch()
    import paper_2401_08260_amd as ks
    note("autograd KernelSum")
    rng = np.random.default_rng(12)
    N, M, d, P = 3000, 2500, 32, 8
    dev = torch.device("cuda:0")
    x = torch.from_numpy(rng.random((N, d), dtype=np.float32)).to(dev).requires_grad_(True)
    y = torch.from_numpy(rng.random((M, d), dtype=np.float32)).to(dev).requires_grad_(True)
    w = torch.from_numpy(rng.random(N).astype(np.float32)).to(dev).requires_grad_(True)
    plan = ks.Plan(d, P, "negdist", seed=7)
    s = ks.KernelSum.apply(plan, x, y, w)
    loss = (s * s).sum()
    loss.backward()
    gx, gy, gw = plan.backward(x.detach(), y.detach(), w.detach(), (2 * s).detach())
    torch.cuda.synchronize()
    assert torch.equal(x.grad, gx) and torch.equal(y.grad, gy) and torch.equal(w.grad, gw)
    tot = (x.grad.double().sum(0) + y.grad.double().sum(0)).norm().item()
    scale = x.grad.double().abs().sum().item() + y.grad.double().abs().sum().item()
    note(f"  translation residual {tot / scale:.3e}")
    assert tot <= 1e-5 * scale


@pytest.mark.parametrize("kernel", ["negdist", "laplacian"])
def test_backward_subsets_and_batches(kernel):
    """Every subset of the gradients equals the full backward bitwise (the projections are
    shared between the sums of the gradient, or computed directly when only grad_x and grad_w
    are asked for), over three slice batches (32, 32, 6) with ragged N != M; the full set
    also against the oracle gradient (exact dyadic projections)."""
    torch = _torch()
    import paper_2401_08260_amd as ks
    N, M, d, P = 2100, 1300, 24, 70
    x, y, w, g, xi = dyadic_case(N, M, d, P, 33)
    kw = {}
    if kernel == "laplacian":
        kw = dict(sigma=float(np.sqrt(d / 6.0)), method="nfft", n_coeff=256, T=0.125)
    note(f"backward subsets {kernel} N={N} M={M} d={d} P={P}")
    r = check(kernel, x, y, w, g, P, directions=xi, ref_kw=kw, slice_batch=32, **kw)
    plan = ks.Plan(d, P, kernel, directions=xi, slice_batch=32, **kw)
    dev = torch.device("cuda:0")
    xt, yt, wt, gt = (torch.from_numpy(a).to(dev) for a in (x, y, w, g))
    full = [t.cpu().numpy() for t in plan.backward(xt, yt, wt, gt)]
    for need in [(True, False, False), (False, True, False), (False, False, True), (True, False, True),
                 (False, True, True), (True, True, False)]:
        part = plan.backward(xt, yt, wt, gt, need_x=need[0], need_y=need[1], need_w=need[2])
        torch.cuda.synchronize()
        for k in range(3):
            assert (part[k] is None) == (not need[k])
            if part[k] is not None:
                assert np.array_equal(part[k].cpu().numpy(), full[k]), (need, k)
    assert np.array_equal(full[0].astype(np.float64), r["gx"])


def test_backward_split_bf16():
    """Split-BF16 projection: coordinates with 16 significant bits split exactly into two
    bf16 halves and the directions +-2^-j are bf16 numbers, so the three products are exact
    and the gradients meet the FP32 gate."""
    note("backward split-bf16 negdist (exact dyadic projections)")
    N, M, d, P = 3000, 2000, 128, 6
    x, y, w, g, xi = dyadic_case(N, M, d, P, 21, bits=16)
    check("negdist", x, y, w, g, P, directions=xi, precision="split_bf16")


def test_backward_split_bf16_presplit():
    """The same with more than 8 tiles of 256 slices: the points are split once per call
    (for the union of the gradient's first layout) and the GEMM is fed by direct LDS
    copies; exact dyadic projections again meet the FP32 gate."""
    note("backward split-bf16 negdist, P = 2100 (points split once per call)")
    N, M, d, P = 1500, 1000, 64, 2100
    x, y, w, g, xi = dyadic_case(N, M, d, P, 23, bits=16)
    check("negdist", x, y, w, g, P, directions=xi, precision="split_bf16")


def test_backward_matern_reduced():
    rng = np.random.default_rng(31)
    N, M, d, P = 6000, 5000, 20, 3
    x = rng.standard_normal((N, d)).astype(np.float32)
    y = rng.standard_normal((M, d)).astype(np.float32)
    w = rng.random(N).astype(np.float32)
    g = rng.standard_normal(M).astype(np.float32)
    beta = wlm.median_heuristic(x, y)
    note("backward matern")
    kw = dict(sigma=beta, method="nfft", n_coeff=1024, T=0.125)
    check("matern", x, y, w, g, P, seed=2, ref_kw=kw, **kw)
