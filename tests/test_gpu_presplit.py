"""Split-BF16 plans with more than 8 tiles of 256 slices split the points to bf16 hi / lo
once per call into a step-tiled layout and feed the projection GEMM from it by direct
copies into LDS; the no-allocation entry point keeps the split inside the GEMM.  Both
take the same products in the same order, so the sums must agree bit for bit (the sort
and Fourier stages do not depend on the batch size)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


CASES = [
    # kernel, plan parameters, d (4-, 2- and 1-wide point loads of the in-GEMM split), P, N, M
    ("negdist", dict(), 64, 2100, 3001, 2003),
    ("laplacian", dict(sigma=2.0, n_coeff=128, T=0.125), 50, 2311, 2500, 1700),
    ("gaussian", dict(sigma=1.5, n_coeff=128, T=0.02, method="nfft"), 17, 2053, 4099, 777),
    # batches of 1000 slices: slice tiles start at rows that are not multiples of 32
    ("negdist", dict(slice_batch=1000), 96, 2600, 1800, 1300),
]


@pytest.mark.parametrize("kernel,params,d,P,N,M", CASES, ids=[f"{c[0]}-P{c[3]}" for c in CASES])
def test_presplit_matches_split_in_gemm(kernel, params, d, P, N, M):
    import torch
    import paper_2401_08260_amd as ks
    note(f"presplit {kernel} d={d} P={P} N={N} M={M}")
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(17)
    x = torch.from_numpy(rng.random((N, d), dtype=np.float32)).to(dev)
    y = torch.from_numpy(rng.random((M, d), dtype=np.float32)).to(dev)
    w = torch.from_numpy(rng.random(N, dtype=np.float32)).to(dev)
    plan = ks.Plan(d, P, kernel, seed=5, precision="split_bf16", **params)
    stream = torch.cuda.current_stream().cuda_stream
    need = ks.ksum_workspace_size(plan.handle, N, M)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    a = torch.full((M,), float("nan"), device=dev)
    b = torch.full((M,), float("nan"), device=dev)
    ks.ksum_execute(plan.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), a.data_ptr(), ws.data_ptr(), need,
                    stream)
    ks.ksum_execute_noalloc(plan.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), b.data_ptr(), stream)
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.all(np.isfinite(a))
    diff = int(np.count_nonzero(a != b))
    note(f"  {diff} of {M} sums differ")
    assert diff == 0
