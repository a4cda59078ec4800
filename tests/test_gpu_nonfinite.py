"""The opt-in input check (params.check_finite): a NaN or an infinity in x, y, w (or in
grad_s for the backward) makes the call return KSUM_ENONFINITE before any other work, so
no output is written; with finite inputs the checked call gives the unchecked result
bitwise."""
import numpy as np
import pytest

from test_gpu_parity import note

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _data(torch, N, M, d, dtype=np.float32, seed=0):
    rng = np.random.default_rng(seed)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(rng.random((N, d)).astype(dtype)).to(dev)
    y = torch.from_numpy(rng.random((M, d)).astype(dtype)).to(dev)
    w = torch.from_numpy(rng.random(N).astype(dtype)).to(dev)
    return x, y, w


KERNELS = [("negdist", {}), ("laplacian", dict(sigma=2.0)), ("gaussian", dict(sigma=2.0, n_coeff=128, T=0.02))]


@pytest.mark.parametrize("kernel,params", KERNELS, ids=[k for k, _ in KERNELS])
def test_checked_finite_inputs_give_the_unchecked_result(kernel, params):
    torch = _torch()
    import paper_2401_08260_amd as ks
    x, y, w = _data(torch, 5000, 4000, 24)
    a = ks.Plan(24, 16, kernel, seed=2, **params)(x, y, w)
    b = ks.Plan(24, 16, kernel, seed=2, check_finite=1, **params)(x, y, w)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("where", ["x", "y", "w"])
@pytest.mark.parametrize("value", [float("nan"), float("inf"), -float("inf")])
def test_nonfinite_input_is_refused_and_nothing_written(where, value):
    torch = _torch()
    import paper_2401_08260_amd as ks
    N, M, d = 3000, 2000, 16
    x, y, w = _data(torch, N, M, d, seed=1)
    t = {"x": x, "y": y, "w": w}[where]
    t.view(-1)[t.numel() // 2 + 7] = value
    plan = ks.Plan(d, 8, "laplacian", sigma=2.0, seed=3, check_finite=1)
    s = torch.full((M,), 7.0, dtype=torch.float32, device=x.device)
    with pytest.raises(ks.KsumError) as e:
        plan(x, y, w, out=s)
    assert e.value.status == ks.KSUM_ENONFINITE
    torch.cuda.synchronize()
    assert bool(torch.all(s == 7.0)), "a refused call must not write s"


def test_nonfinite_fp64_input_noalloc_and_backward():
    torch = _torch()
    import paper_2401_08260_amd as ks
    N, M, d = 2000, 1500, 10
    # FP64 inputs are checked before they are converted
    x, y, w = _data(torch, N, M, d, dtype=np.float64, seed=4)
    x[5, 3] = float("nan")
    plan = ks.Plan(d, 8, "gaussian", sigma=2.0, n_coeff=64, T=0.045, method="ndft", seed=1, check_finite=1)
    with pytest.raises(ks.KsumError) as e:
        plan(x, y, w)
    assert e.value.status == ks.KSUM_ENONFINITE
    # the no-allocation entry point checks too
    x, y, w = _data(torch, N, M, d, seed=5)
    w[N - 1] = float("inf")
    plan = ks.Plan(d, 8, "negdist", seed=1, check_finite=1)
    s = torch.full((M,), 3.0, dtype=torch.float32, device=x.device)
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(ks.KsumError) as e:
        ks.ksum_execute_noalloc(plan.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), s.data_ptr(), stream)
    assert e.value.status == ks.KSUM_ENONFINITE
    torch.cuda.synchronize()
    assert bool(torch.all(s == 3.0))
    # the backward checks grad_s as well; its outputs stay untouched
    w[N - 1] = 0.5
    gs = torch.ones(M, dtype=torch.float32, device=x.device)
    gs[17] = float("nan")
    with pytest.raises(ks.KsumError) as e:
        plan.backward(x, y, w, gs)
    assert e.value.status == ks.KSUM_ENONFINITE
    gs[17] = 1.0
    gx, gy, gw = plan.backward(x, y, w, gs)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(gx).all() and torch.isfinite(gy).all() and torch.isfinite(gw).all())
    note("  refusals: FP64 NaN in x, Inf weight through ksum_execute_noalloc, NaN grad_s in the backward")
