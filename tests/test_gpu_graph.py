"""ksum_execute captured into a HIP graph (through torch's graph capture) and launched
again with new inputs in the same buffers: every launch must give the eager result
bit for bit.  The call enqueues kernels only (its clears are kernels of its own), so
a caller that cannot afford the launches one by one can capture it.  Between the
launches the test runs the eager call and synchronises, and checks every launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)


CASES = [
    # kernel, plan parameters, d, P, N, M
    ("laplacian", dict(sigma=2.0, n_coeff=128, T=0.125, precision="split_bf16"), 40, 2100, 2600, 1900),
    ("negdist", dict(precision="fp32"), 24, 96, 3001, 1777),
    ("gaussian", dict(sigma=1.5, n_coeff=128, T=0.02, method="nfft"), 17, 40, 4099, 2222),
]


@pytest.mark.parametrize("kernel,params,d,P,N,M", CASES, ids=[c[0] for c in CASES])
def test_execute_in_graph(kernel, params, d, P, N, M):
    import torch
    import paper_2401_08260_amd as ks
    note(f"graph {kernel} d={d} P={P} N={N} M={M}")
    dev = torch.device("cuda:0")
    plan = ks.Plan(d, P, kernel, seed=3, **params)
    need = ks.ksum_workspace_size(plan.handle, N, M)
    x = torch.empty((N, d), device=dev)
    y = torch.empty((M, d), device=dev)
    w = torch.empty(N, device=dev)
    s_graph = torch.full((M,), float("nan"), device=dev)
    ws_graph = torch.empty(need, dtype=torch.uint8, device=dev)
    ws_eager = torch.empty(need, dtype=torch.uint8, device=dev)
    rng = np.random.default_rng(41)

    def fill():
        x.copy_(torch.from_numpy(rng.random((N, d), dtype=np.float32)))
        y.copy_(torch.from_numpy(rng.random((M, d), dtype=np.float32)))
        w.copy_(torch.from_numpy(rng.random(N, dtype=np.float32)))

    def eager():
        s = torch.full((M,), float("nan"), device=dev)
        st = torch.cuda.current_stream().cuda_stream
        ks.ksum_execute(plan.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), s.data_ptr(), ws_eager.data_ptr(),
                        need, st)
        torch.cuda.synchronize()
        return s.cpu().numpy()

    fill()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        st = torch.cuda.current_stream().cuda_stream
        ks.ksum_execute(plan.handle, x.data_ptr(), N, y.data_ptr(), M, w.data_ptr(), s_graph.data_ptr(),
                        ws_graph.data_ptr(), need, st)
    torch.cuda.synchronize()
    for rep in range(3):
        if rep:
            fill()
            torch.cuda.synchronize()
        ref = eager()
        s_graph.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        got = s_graph.cpu().numpy()
        diff = int(np.count_nonzero(got != ref))
        note(f"  launch {rep}: {diff} of {M} sums differ from the eager call")
        assert np.all(np.isfinite(ref))
        assert diff == 0
    del graph
    torch.cuda.synchronize()
