"""Pins for oracle.onedim: Algorithm "alg:fastsum_energy" and the NDFT Fourier summation (Sec. 3)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import kernels as kn
from oracle import onedim

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "alg2_hand.json")


def brute_negdist(z, v, cd):
    return np.array([-cd * sum(v[n] * abs(z[n] - z[m]) for n in range(len(z))) for m in range(len(z))])


def test_alg2_hand_cases():
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        z = np.array(c["z"], dtype=np.float64)
        order = np.argsort(z, kind="stable")
        assert np.array_equal(order, np.arange(len(z)))      # fixtures are already ascending
        t = onedim.negdist_sorted(z, np.array(c["v"], dtype=np.float64), float(c["cd"]))
        assert np.array_equal(t, np.array(c["t"], dtype=np.float64))


def test_alg2_bit_exact_on_small_integers():
    rng = np.random.default_rng(7)
    for L in (1, 2, 3, 17, 200):
        z = np.sort(rng.integers(-50, 50, size=L)).astype(np.float64)
        v = rng.integers(-9, 10, size=L).astype(np.float64)
        t = onedim.negdist_sorted(z, v, 3.0)
        zi = z.astype(np.int64)
        vi = v.astype(np.int64)
        ref = np.array([-3 * int(np.sum(vi * np.abs(zi - zi[m]))) for m in range(L)], dtype=np.float64)
        assert np.array_equal(t, ref)


def test_alg2_random_vs_brute_force():
    rng = np.random.default_rng(8)
    for L in (5, 64, 300):
        z = np.sort(rng.standard_normal(L))
        v = rng.standard_normal(L)
        t = onedim.negdist_sorted(z, v, 1.7)
        ref = brute_negdist(z, v, 1.7)
        assert np.max(np.abs(t - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_negdist_general_case_and_ties():
    rng = np.random.default_rng(9)
    N, M = 40, 30
    zx = rng.integers(-6, 6, size=N).astype(np.float64)     # many ties, also between x and y
    zy = rng.integers(-6, 6, size=M).astype(np.float64)
    w = rng.integers(-4, 5, size=N).astype(np.float64)
    t, perm = onedim.negdist_sum(zx, zy, w, 2.0, return_perm=True)
    ref = np.array([-2.0 * np.sum(w * np.abs(zx - zy[m])) for m in range(M)])
    assert np.array_equal(t, ref)
    z = np.concatenate([zy, zx])
    assert np.all(np.diff(z[perm]) >= 0)
    # stable: equal keys keep union-index order
    same = np.diff(z[perm]) == 0
    assert np.all(np.diff(perm)[same] > 0)


def test_negdist_tie_order_invariance():
    z = np.array([0.0, 1.0, 1.0, 1.0, 2.5])
    v = np.array([0.3, -1.25, 2.0, 0.5, 1.0])
    t1 = onedim.negdist_sorted(z, v, 1.0)
    t2 = onedim.negdist_sorted(z, v[[0, 3, 1, 2, 4]], 1.0)
    assert np.allclose(t1[[0, 4]], t2[[0, 4]], rtol=0, atol=1e-15)


def test_ndft_exact_for_trigonometric_polynomial():
    """If phi is a trigonometric polynomial with coefficients c_k on C, the NDFT summation is exact."""
    rng = np.random.default_rng(10)
    ks = np.arange(-5, 6)
    cs = rng.standard_normal(11)
    cs = 0.5 * (cs + cs[::-1])                        # real, even coefficients (C symmetric)
    xt = rng.uniform(-0.25, 0.25, 37)
    yt = rng.uniform(-0.25, 0.25, 23)
    w = rng.standard_normal(37)

    def phi(u):
        return np.real(np.sum(cs[:, None] * np.exp(-2j * math.pi * ks[:, None] * u[None, :]), axis=0))

    t = onedim.ndft_sum(xt, yt, w, ks, cs)
    ref = np.array([np.sum(w * phi(xt - y)) for y in yt])
    assert np.max(np.abs(t - ref)) < 1e-12


def test_ndft_asymmetric_phase_convention():
    """A non-even phi pins the exponent signs: t_m = sum_n w_n phi(x_n - y_m)."""
    ks = np.array([-1, 1])
    cs = np.array([0.0, 1.0])                          # phi(u) = exp(-2 pi i u), real part cos(2 pi u)
    xt = np.array([0.1])
    yt = np.array([0.0, 0.2])
    t = onedim.ndft_sum(xt, yt, np.array([1.0]), ks, cs)
    assert np.allclose(t, np.cos(2 * math.pi * (xt[0] - yt)), atol=1e-15)


@pytest.mark.parametrize("d", [1, 3, 10])
def test_gaussian_fourier_summation_vs_direct(d):
    """Sec. 2.2 + Sec. 3.1: with rescaling and the Lemma's coefficients, the NDFT sum matches f pointwise."""
    rng = np.random.default_rng(11 + d)
    sigma = 1.0
    zx = rng.uniform(-1.5, 1.5, 120)
    zy = rng.uniform(-1.5, 1.5, 90)
    w = rng.uniform(0, 1, 120)
    T = 0.06          # data range 3 sigma: truncation and periodization errors both below 1e-9 here
    cmin, cmax = min(zx.min(), zy.min()), max(zx.max(), zy.max())
    tau = 2 * T / (cmax - cmin)
    xt, yt = tau * (zx - cmin) - T, tau * (zy - cmin) - T
    ks = np.arange(-32, 33)
    cs = kn.gauss_fourier_coeff(d, tau * sigma, ks)
    t = onedim.ndft_sum(xt, yt, w, ks, cs)
    ref = onedim.direct_1d(zx, zy, w, lambda u: kn.counterpart_f("gaussian", d, u, sigma))
    assert np.max(np.abs(t - ref)) < 1e-9 * np.max(np.abs(ref))
