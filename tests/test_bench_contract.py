"""Host-side checks of bench.py: the single-GPU refusal and the algorithmic work it
prices each kernel launch with (no GPU needed)."""
import importlib.util
import os
import subprocess
import sys

import pytest

import workloads as wlm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr + r.stdout
    assert r.stdout.strip() == ""          # no JSON line for a refused run


@pytest.mark.parametrize("name", ["negdist", "laplace", "gauss_nfft", "gauss_ndft"])
def test_projection_flops_per_launch(name):
    b = _bench()
    wl = wlm.WORKLOADS[name]
    bound, amount, unit, peak = b.kernel_work("project", wl, wl.P)
    assert (bound, unit) == ("mfma", "TFLOP/s")
    # one multiply and one add per coordinate, point and slice
    assert amount * 1e12 == pytest.approx(2.0 * (wl.N + wl.M) * wl.d * wl.P, rel=1e-12)
    assert peak == pytest.approx(157.3)


def test_negdist_sort_bytes_per_launch():
    b = _bench()
    wl = wlm.WORKLOADS["negdist"]
    N, M, P = wl.N, wl.M, wl.P
    L = N + M
    # keys and indices read once, a weight per source, a t value per target
    assert b.kernel_work("sort_group", wl, P)[1] * 1e9 == pytest.approx((8 * L + 4 * N + 4 * M) * P)
    # projection read and (key, index) written once per entry
    assert b.kernel_work("sort_scatter", wl, P)[1] * 1e9 == pytest.approx(12 * L * P)
    assert b.kernel_work("sort_hist", wl, P)[0] == "hbm"
    assert b.kernel_work("no_such_stage", wl, P) is None
