"""The request server (continuous batching): every result is bitwise the same alone and in the
mix, admission respects the HBM arena, and a request that can never fit is refused."""
import numpy as np
import pytest

from test_gpu_parity import note

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _params(kernel, d):
    if kernel == "gaussian":
        return dict(sigma=float(np.sqrt(2 * d)), n_coeff=128, T=0.02, method="nfft")
    if kernel == "laplacian":
        return dict(sigma=float(np.sqrt(2 * d)), n_coeff=256, T=0.125)
    return {}


def test_server_results_match_alone_and_respect_arena():
    torch = _torch()
    import paper_2401_08260_amd as ks
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(24):
        kernel = ["gaussian", "laplacian", "negdist"][i % 3]
        d = [16, 128][(i // 3) % 2]
        N, M = int(rng.integers(1000, 20000)), int(rng.integers(1000, 20000))
        prec = "split_bf16" if i % 4 == 3 else "fp32"
        x = torch.from_numpy(rng.standard_normal((N, d)).astype(np.float32)).to(dev)
        y = torch.from_numpy(rng.standard_normal((M, d)).astype(np.float32)).to(dev)
        w = torch.from_numpy(rng.random(N).astype(np.float32)).to(dev)
        g = torch.from_numpy(rng.standard_normal(M).astype(np.float32)).to(dev) if i % 3 == 1 else None
        reqs.append(dict(kernel=kernel, d=d, P=64, x=x, y=y, w=w, g=g,
                         params=dict(_params(kernel, d), precision=prec, seed=i % 5)))
    arena = 256 << 20
    srv = ks.Server(slots=4, hbm_bytes=arena)
    outs = {}
    for i, r in enumerate(reqs):
        N, M = r["x"].shape[0], r["y"].shape[0]
        s = torch.empty(M, dtype=torch.float32, device=dev)
        grads = (None, None, None)
        if r["g"] is not None:
            grads = (torch.empty((N, r["d"]), dtype=torch.float32, device=dev),
                     torch.empty((M, r["d"]), dtype=torch.float32, device=dev),
                     torch.empty(N, dtype=torch.float32, device=dev))
        outs[i] = (s, grads)
        srv.submit(i, r["kernel"], r["d"], r["P"], r["x"], r["y"], r["w"], s, params=r["params"],
                   grad_s=r["g"], grads=grads)
    srv.drain()
    done = srv.poll(1000)
    st = srv.stats()
    note(f"  server stats {st}")
    assert len(done) == len(reqs) and all(c["status"] == 0 for c in done)
    assert st["arena_peak"] <= arena and st["finished"] == len(reqs)
    assert all(c["t_submit"] <= c["t_start"] <= c["t_end"] for c in done)
    srv.close()
    torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        plan = ks.Plan(r["d"], r["P"], r["kernel"], **r["params"])
        s_alone = plan(r["x"], r["y"], r["w"])
        s_mix, grads = outs[i]
        assert torch.equal(s_alone, s_mix), f"request {i} forward"
        if r["g"] is not None:
            gx, gy, gw = plan.backward(r["x"], r["y"], r["w"], r["g"])
            assert torch.equal(gx, grads[0]) and torch.equal(gy, grads[1]) and torch.equal(gw, grads[2]), \
                f"request {i} backward"
    torch.cuda.synchronize()


def test_server_refuses_request_larger_than_arena():
    torch = _torch()
    import paper_2401_08260_amd as ks
    dev = torch.device("cuda:0")
    srv = ks.Server(slots=2, hbm_bytes=1 << 20)
    N = M = 20000
    x = torch.rand((N, 64), device=dev)
    y = torch.rand((M, 64), device=dev)
    w = torch.rand(N, device=dev)
    s = torch.empty(M, device=dev)
    srv.submit(7, "negdist", 64, 64, x, y, w, s)
    srv.drain()
    done = srv.poll()
    assert len(done) == 1 and done[0]["tag"] == 7 and done[0]["status"] == ks.KSUM_ENOMEM
    srv.close()
