"""Host checks of the seeded input generators (shapes, ranges and the serving stream's statistics)."""
import math

import numpy as np

import workloads as wlm


def test_serving_stream_statistics():
    reqs = wlm.serving_stream(20000, 200.0, seed=4)
    t = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 1 / 200.0) < 0.05 / 200.0
    for key in ("N", "M"):
        v = np.array([r[key] for r in reqs])
        assert v.min() >= 1000 and v.max() <= 500000
        # log-uniform: the mean of the log is the midpoint of [log 1e3, log 5e5]
        assert abs(np.mean(np.log(v)) - 0.5 * (math.log(1e3) + math.log(5e5))) < 0.05
    assert {r["d"] for r in reqs} == {16, 128, 784, 3072}
    assert {r["kernel"] for r in reqs} == {"gaussian", "laplacian", "negdist"}
    assert {r["P"] for r in reqs} == {64, 256}
    assert abs(np.mean([r["grad"] for r in reqs]) - 0.3) < 0.02
    # the stream is reproducible
    assert wlm.serving_stream(20000, 200.0, seed=4) == reqs


def test_workload_inputs_shapes_and_dtypes():
    for name, wl in wlm.WORKLOADS.items():
        small = wlm.scaled(wl, N=300, M=200, P=4)
        x, y, w = wlm.generate(small)
        dt = np.float64 if wl.dtype == "f64" else np.float32
        assert x.shape == (300, wl.d) and y.shape == (200, wl.d) and w.shape == (300,)
        assert x.dtype == dt and y.dtype == dt and w.dtype == dt
        if wl.weights == "inv_n":
            assert np.allclose(w, 1.0 / 300)
