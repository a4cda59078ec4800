"""ksum_execute_noalloc, the forward sum that allocates nothing (its workspace is the
library's static per-GPU scratch), against ksum_execute with a caller workspace on the
same plan and inputs: two calls in a row, the second on a smaller input, so that the
second call runs on a scratch that still holds the first call's data.  The first call is
large enough that the scratch takes fewer slices per batch than the plan's own batch."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = 1e-5


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _inputs(torch, rng, N, M, d):
    dev = torch.device("cuda:0")
    x = torch.from_numpy(rng.random((N, d), dtype=np.float32)).to(dev)
    y = torch.from_numpy(rng.random((M, d), dtype=np.float32)).to(dev)
    w = torch.from_numpy(rng.random(N, dtype=np.float32)).to(dev)
    return x, y, w


def _rel(a, ref):
    a, ref = a.astype(np.float64), ref.astype(np.float64)
    return (float(np.linalg.norm(a - ref) / np.linalg.norm(ref)),
            float(np.max(np.abs(a - ref)) / np.max(np.abs(ref))))


CASES = [
    # kernel, plan parameters, d, P, (N, M) of the first and of the second call
    ("laplacian", dict(sigma=2.0, n_coeff=256, T=0.125), 32, 24, (600_000, 500_000), (3000, 2000)),
    ("gaussian", dict(sigma=1.5, n_coeff=128, T=0.02, method="nfft"), 16, 40, (1_000_000, 900_000), (7000, 5000)),
    ("negdist", dict(), 64, 30, (700_000, 600_000), (2500, 4100)),
]


@pytest.mark.parametrize("kernel,params,d,P,big,small", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_execute(kernel, params, d, P, big, small):
    torch = _torch()
    import paper_2401_08260_amd as ks
    kid = ks.KERNELS[kernel]
    plan = ks.Plan(d, P, kernel, seed=11, **params)
    ws_big = ks.ksum_workspace_size(plan.handle, *big)
    batch_fit = max(b for b in range(1, P + 1)
                    if ks.ksum_workspace_bytes(d, P, kid, ks.make_params(kid, seed=11, slice_batch=b, **params),
                                               *big) <= ks.KSUM_NOALLOC_SCRATCH_BYTES)
    note(f"{kernel} d={d} P={P}: first call N, M = {big} (workspace {ws_big / 2**20:.0f} MiB, "
         f"{batch_fit} slices per batch in the scratch), second call N, M = {small}")
    assert batch_fit < P, "the first call should need more than one batch in the scratch"
    rng = np.random.default_rng(5)
    calls = [_inputs(torch, rng, *big, d), _inputs(torch, rng, *small, d)]
    stream = torch.cuda.current_stream().cuda_stream
    # the two no-allocation calls back to back on one stream
    outs = []
    for (x, y, w) in calls:
        s = torch.full((y.shape[0],), float("nan"), dtype=torch.float32, device=x.device)
        ks.ksum_execute_noalloc(plan.handle, x.data_ptr(), x.shape[0], y.data_ptr(), y.shape[0], w.data_ptr(),
                                s.data_ptr(), stream)
        outs.append(s)
    torch.cuda.synchronize()
    for (x, y, w), s in zip(calls, outs):
        N, M = x.shape[0], y.shape[0]
        need = ks.ksum_workspace_size(plan.handle, N, M)
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
        ref = torch.empty(M, dtype=torch.float32, device=x.device)
        ks.ksum_execute(plan.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), ref.data_ptr(),
                        ws.data_ptr(), need, stream)
        torch.cuda.synchronize()
        a, r = s.cpu().numpy(), ref.cpu().numpy()
        e2, em = _rel(a, r)
        note(f"  N={N} M={M}: rel l2 {e2:.3e}, max elementwise {em:.3e}, bitwise equal {np.array_equal(a, r)}")
        assert np.all(np.isfinite(a))
        assert e2 <= TOL and em <= TOL, (e2, em)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    torch = _torch()
    import paper_2401_08260_amd as ks
    d, P = 2, 4
    plan = ks.Plan(d, P, "laplacian", sigma=2.0, seed=3)
    rng = np.random.default_rng(9)
    # one slice of 6e6 sources and 6e6 targets needs more than the scratch holds; the
    # buffers are real, so nothing would be read out of bounds even if a launch happened
    N = M = 6_000_000
    x, y, w = _inputs(torch, rng, N, M, d)
    s = torch.zeros(M, dtype=torch.float32, device=x.device)
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(ks.KsumError) as err:
        ks.ksum_execute_noalloc(plan.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), s.data_ptr(), stream)
    assert err.value.status == ks.KSUM_EWORKSPACE
    note(f"  refused: {err.value}")
    with pytest.raises(ks.KsumError) as err:
        ks.ksum_execute_noalloc(plan.handle, x.data_ptr(), N, None, M, w.data_ptr(), s.data_ptr(), stream)
    assert err.value.status == ks.KSUM_EINVAL
    torch.cuda.synchronize()
    assert float(s.abs().max()) == 0.0, "a refused call must not write its output"
    # the library still works after the refusals: a call that fits, against ksum_execute
    n, m = 4000, 3000
    s2 = torch.empty(m, dtype=torch.float32, device=x.device)
    ks.ksum_execute_noalloc(plan.handle, x.data_ptr(), n, y.data_ptr(), m, w.data_ptr(), s2.data_ptr(), stream)
    need = ks.ksum_workspace_size(plan.handle, n, m)
    ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    ref = torch.empty(m, dtype=torch.float32, device=x.device)
    ks.ksum_execute(plan.handle, x.data_ptr(), n, y.data_ptr(), m, w.data_ptr(), ref.data_ptr(), ws.data_ptr(),
                    need, stream)
    torch.cuda.synchronize()
    e2, em = _rel(s2.cpu().numpy(), ref.cpu().numpy())
    note(f"  after the refusals N={n} M={m}: rel l2 {e2:.3e}, max elementwise {em:.3e}")
    assert e2 <= TOL and em <= TOL, (e2, em)
