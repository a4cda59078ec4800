"""GPU parity of the backward pass (ksum_backward) against the FP64 oracle gradient.

The derivative sums of the sort path jump where two projections cross, so the
oracle's derivative sums are evaluated on the GPU's own FP32 projections (the
probe z of a forward call, bitwise the projections the backward computes): both
sides then take every sign decision on the same values.  grad_w is a forward sum
with the roles swapped and is compared with the oracle's sliced sum directly.
Gate: relative l2 error <= 1e-5 per gradient (FP32 path).
"""
import numpy as np
import pytest

import workloads as wlm
from oracle import gradient, sliced
from test_gpu_parity import note

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_backward(kernel, x, y, w, g, P, seed=0, **params):
    torch = _torch()
    import paper_2401_08260_amd as ks
    d = x.shape[1]
    N, M = x.shape[0], y.shape[0]
    plan = ks.Plan(d, P, kernel, seed=seed, **params)
    dev = torch.device("cuda:0")
    xt, yt, wt, gt = (torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev) for a in (x, y, w, g))
    z = torch.empty((P, M + N), dtype=torch.float32, device=dev)
    plan(xt, yt, wt, probe={"z": z})
    gx, gy, gw = plan.backward(xt, yt, wt, gt)
    torch.cuda.synchronize()
    zz = z.cpu().numpy().astype(np.float64)
    return dict(gx=gx.cpu().numpy().astype(np.float64), gy=gy.cpu().numpy().astype(np.float64),
                gw=gw.cpu().numpy().astype(np.float64), zy=zz[:, :M].T, zx=zz[:, M:].T, xi=plan.directions())


def check(kernel, x, y, w, g, P, seed=0, ref_kw=None, tol=TOL, **params):
    ref_kw = ref_kw or {}
    r = run_backward(kernel, x, y, w, g, P, seed=seed, **params)
    xd, yd, wd, gd = (np.asarray(a, dtype=np.float32).astype(np.float64) for a in (x, y, w, g))
    gx_ref, gy_ref = gradient.grad_from_projections(kernel, x.shape[1], r["zx"], r["zy"], wd, gd, r["xi"],
                                                    **ref_kw)
    gw_ref = sliced.sliced_sum(kernel, yd, xd, gd, r["xi"], **ref_kw)
    errs = {"x": sliced.rel_l2(r["gx"], gx_ref), "y": sliced.rel_l2(r["gy"], gy_ref),
            "w": sliced.rel_l2(r["gw"], gw_ref)}
    note(f"  rel err grad_x {errs['x']:.3e} grad_y {errs['y']:.3e} grad_w {errs['w']:.3e}")
    for k, v in errs.items():
        assert v <= tol, k
    return r


@pytest.mark.parametrize("N,M,d,P", [(3000, 2000, 64, 8), (1, 1, 3, 2), (700, 5, 17, 3), (5000, 4000, 784, 4)])
def test_backward_negdist(N, M, d, P):
    note(f"backward negdist N={N} M={M} d={d} P={P}")
    rng = np.random.default_rng(N + M + d)
    x = rng.random((N, d), dtype=np.float32)
    y = rng.random((M, d), dtype=np.float32)
    y[: min(M, N) // 2] = x[: min(M, N) // 2]          # targets on top of sources: ties
    w = rng.random(N).astype(np.float32)
    g = rng.standard_normal(M).astype(np.float32)
    check("negdist", x, y, w, g, P, seed=3)


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
    rng = np.random.default_rng(5)
    N, M, d, P = 12000, 9000, 4, 2
    x = rng.random((N, d), dtype=np.float32)
    y = rng.random((M, d), dtype=np.float32)
    x[:7000] = 0.5
    y[:5000] = 0.5
    w = rng.random(N).astype(np.float32)
    g = rng.standard_normal(M).astype(np.float32)
    check("negdist", x, y, w, g, P, seed=4)


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
    wl = wlm.scaled(wlm.WORKLOADS["laplace"], N=4000, M=3000, P=4)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    g = np.random.default_rng(9).standard_normal(wl.M).astype(np.float32)
    note("backward laplace reduced")
    kw = dict(sigma=sigma, method="nfft", n_coeff=wl.n_coeff, T=wl.T)
    check("laplacian", x, y, w, g, wl.P, seed=wl.dir_seed, ref_kw=kw, **kw)


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
    also against the oracle gradient."""
    torch = _torch()
    import paper_2401_08260_amd as ks
    rng = np.random.default_rng(33)
    N, M, d, P = 2100, 1300, 24, 70
    x = rng.random((N, d), dtype=np.float32)
    y = rng.random((M, d), dtype=np.float32)
    w = rng.random(N).astype(np.float32)
    g = rng.standard_normal(M).astype(np.float32)
    kw = {}
    if kernel == "laplacian":
        kw = dict(sigma=float(np.sqrt(d / 6.0)), method="nfft", n_coeff=256, T=0.125)
    note(f"backward subsets {kernel} N={N} M={M} d={d} P={P}")
    r = check(kernel, x, y, w, g, P, seed=4, ref_kw=kw, slice_batch=32, **kw)
    plan = ks.Plan(d, P, kernel, seed=4, slice_batch=32, **kw)
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
    note("backward split-bf16 negdist")
    rng = np.random.default_rng(21)
    N, M, d, P = 3000, 2000, 128, 6
    x = rng.random((N, d), dtype=np.float32)
    y = rng.random((M, d), dtype=np.float32)
    w = rng.random(N).astype(np.float32)
    g = rng.standard_normal(M).astype(np.float32)
    # grad_w is compared with the FP64-projection oracle: the split-BF16 projection's
    # error enters it as in the forward (the mixed-precision gate of the forward tests)
    check("negdist", x, y, w, g, P, seed=3, tol=1e-4, precision="split_bf16")


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
