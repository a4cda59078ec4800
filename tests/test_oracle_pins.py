"""Pins for two oracle parts that no closed form of the paper covers.

* The direction generator's SplitMix64 stream (the paper only says "draw P random
  directions", Sec. 2.3) against the published outputs of the reference generator
  (tests/golden/splitmix64.json).
* The cutoff set of eq. "Fourier_cutoff" (Sec. 2.2), C = {k : |k| <= K_max, |c_k| > eps}:
  - for the Gaussian on d = 1 the coefficients fall monotonically in |k|, so the eps cutoff
    is the same sum as a smaller K_max with eps = 0 (a reduction to the K_max-only path);
  - for d > 1 and the tapered Laplacian coefficients, the difference to eps = 0 is bounded
    by sum over the dropped k of |c_k| * sum_n |w_n| (triangle inequality on the dropped
    terms of the Fourier sum) and is not zero;
  - an eps above every |c_k| empties C, so the Fourier sum is 0.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import directions, kernels as kn, sliced

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.json")) as f:
        gold = json.load(f)
    for st in gold["streams"]:
        got = [directions.splitmix64(st["seed"], c) for c in range(len(st["outputs"]))]
        assert got == [int(v) for v in st["outputs"]], st["seed"]


def _slice_inputs(seed, n=300, m=200):
    rng = np.random.default_rng(seed)
    zx = rng.standard_normal(n)
    zy = rng.standard_normal(m)
    w = rng.uniform(0, 1, n)
    return zx, zy, w


def test_eps_cutoff_d1_gaussian_equals_smaller_kmax():
    zx, zy, w = _slice_inputs(1)
    sigma, T, n_coeff = 0.4, 0.1, 64
    xt, yt, tau = sliced.rescale(zx, zy, T, sigma)
    ks = np.arange(-32, 33)
    c = kn.gauss_fourier_coeff(1, tau * sigma, ks)
    # eps between |c_K'| and |c_K'+1| for the k > 0 tail
    Kp = 9
    eps = math.sqrt(c[32 + Kp] * c[32 + Kp + 1])
    assert c[32 + Kp] > eps > c[32 + Kp + 1]
    t_eps = sliced.slice_sum("gaussian", 1, zx, zy, w, sigma, "ndft", n_coeff, T, coeff_eps=eps)
    t_k = sliced.slice_sum("gaussian", 1, zx, zy, w, sigma, "ndft", 2 * Kp, T)
    assert np.allclose(t_eps, t_k, rtol=1e-13, atol=1e-13 * np.max(np.abs(t_k)))
    t_full = sliced.slice_sum("gaussian", 1, zx, zy, w, sigma, "ndft", n_coeff, T)
    assert np.max(np.abs(t_full - t_eps)) > 1e-6 * np.max(np.abs(t_full))


@pytest.mark.parametrize("kernel,d,method,n_coeff,T", [("gaussian", 10, "ndft", 64, 0.045),
                                                      ("laplacian", 50, "nfft", 256, 0.125),
                                                      ("matern", 20, "nfft", 1024, 0.125)])
def test_eps_cutoff_bound_on_dropped_terms(kernel, d, method, n_coeff, T):
    zx, zy, w = _slice_inputs(d)
    sigma = 1.5 if kernel == "gaussian" else 3.0
    xt, yt, tau = sliced.rescale(zx, zy, T, sigma)
    K = sliced.cutoff_K(method, n_coeff)
    ks = np.arange(-K, K + 1)
    if kernel == "gaussian":
        c = kn.gauss_fourier_coeff(d, tau * sigma, ks)
    elif kernel == "laplacian":
        c = kn.laplace_smooth_coeffs(d, 1.0 / (sigma * tau), K, 16 * n_coeff)[1]
    else:
        c = kn.matern_coeffs(d, sigma * tau, K, 16 * n_coeff)[1]
    eps = 1e-3 * np.max(np.abs(c))
    dropped = (np.abs(c) <= eps) & (c != 0.0)
    assert dropped.any() and (~dropped).any()
    t0 = sliced.slice_sum(kernel, d, zx, zy, w, sigma, method, n_coeff, T)
    te = sliced.slice_sum(kernel, d, zx, zy, w, sigma, method, n_coeff, T, coeff_eps=eps)
    # the Laplacian's sorted part does not depend on eps, so the same bound holds
    bound = np.sum(np.abs(c[dropped])) * np.sum(np.abs(w))
    diff = np.abs(te - t0)
    assert np.max(diff) <= bound * (1 + 1e-9) + 1e-12
    assert np.max(diff) > 0.0
    # eps above every coefficient: C is empty and the Fourier sum vanishes
    t_none = sliced.slice_sum(kernel, d, zx, zy, w, sigma, method, n_coeff, T,
                              coeff_eps=2.0 * np.max(np.abs(c)))
    if kernel == "laplacian":
        from oracle import onedim
        assert np.allclose(t_none, onedim.negdist_sum(zx, zy, w, kn.c_d(d) / sigma), rtol=0, atol=1e-12)
    else:
        assert np.all(t_none == 0.0)
