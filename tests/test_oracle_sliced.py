"""Pins for the sliced pipeline (Algorithm "alg:fast_Fourier_sliced") and the direction generator."""
import math

import mpmath
import numpy as np
import pytest

import workloads as wlm
from oracle import direct, directions, kernels as kn, sliced


def test_directions_unit_and_prefix():
    xi = directions.directions(7, 12, 5)
    assert np.allclose(np.linalg.norm(xi, axis=1), 1.0, atol=1e-15)
    xi4 = directions.directions(7, 4, 5)
    assert np.array_equal(xi[:4], xi4)
    assert not np.array_equal(directions.directions(7, 4, 6), xi4)


def test_directions_uniform_on_sphere():
    d, P = 5, 4000
    xi = directions.directions(d, P, 123)
    assert np.max(np.abs(xi.mean(axis=0))) < 4.0 / math.sqrt(P * d)
    cov = xi.T @ xi / P
    assert np.max(np.abs(cov - np.eye(d) / d)) < 0.02
    # the uniforms behind them are uniform: chi-square over 16 bins
    u = np.array([(directions.splitmix64(9, c) >> 11) * 2.0 ** -53 for c in range(16000)])
    counts = np.bincount((u * 16).astype(int), minlength=16)
    chi2 = np.sum((counts - 1000.0) ** 2 / 1000.0)
    assert chi2 < 40.0       # 15 dof, p ~ 5e-4


def test_median_heuristic_hand_case():
    x = np.array([[0.0, 0.0], [3.0, 0.0]])
    y = np.array([[0.0, 4.0], [6.0, 8.0]])
    # distances: |x0x1| 3, |x0y0| 4, |x0y1| 10, |x1y0| 5, |x1y1| sqrt(9+64), |y0y1| sqrt(36+16)
    d = sorted([3, 4, 10, 5, math.sqrt(73), math.sqrt(52)])
    assert wlm.median_heuristic(x, y) == pytest.approx(0.5 * (d[2] + d[3]))


# T = 0.1 for the Gaussian: data range ~4.5 sigma, so tau*sigma ~ 0.045 keeps |k| <= 32 enough
@pytest.mark.parametrize("kernel,method,nc,T", [("gaussian", "ndft", 64, 0.1), ("negdist", "sort", 0, 0.0),
                                                ("laplacian", "nfft", 256, 0.125), ("matern", "nfft", 1024, 0.125)])
def test_d1_slicing_is_exact(kernel, method, nc, T):
    """d = 1: every direction is +-1 and f = F, so the sliced sum equals the exact sum for any P."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((80, 1))
    y = rng.standard_normal((60, 1))
    w = rng.uniform(0, 1, 80)
    sigma = 1.2
    xi = directions.directions(1, 3, 0)
    s = sliced.sliced_sum(kernel, x, y, w, xi, sigma, method, nc, T)
    ref = direct.direct_sum(kernel, x, y, w, sigma)
    # Laplacian: the smooth part k1 has a |u|^3 kink, so 256 coefficients leave ~1e-7
    # Matern: f keeps a |u|^3 term too, 1024 coefficients leave ~1e-8
    tol = {"negdist": 1e-12, "gaussian": 1e-9, "laplacian": 3e-7, "matern": 3e-8}[kernel]
    assert sliced.rel_l2(s, ref) < tol


def _equispaced_2d(P):
    a = math.pi * np.arange(P) / P
    return np.stack([np.cos(a), np.sin(a)], axis=1)


def test_d2_equispaced_directions_converge():
    """d = 2, xi_p = (cos(pi p/P), sin(pi p/P)): the slice average is a quadrature of the
    expectation over S^1 and converges to the exact sum (spectrally for the Gaussian)."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((50, 2))
    y = rng.standard_normal((40, 2))
    w = rng.uniform(0, 1, 50)
    # (exact 1-D sums here: for d = 2 the counterpart decays only like 1/x^2, so the Fourier
    # path's periodisation error is ~1e-2 at this data range -- a property of the method at d = 2)
    ref_g = direct.direct_sum("gaussian", x, y, w, 1.5)
    errs = [sliced.rel_l2(sliced.sliced_direct("gaussian", x, y, w, _equispaced_2d(P), 1.5), ref_g)
            for P in (8, 16, 32)]
    assert errs[2] < 1e-12 and errs[1] < errs[0] * 1e-4
    ref_n = direct.direct_sum("negdist", x, y, w)
    errs_n = [sliced.rel_l2(sliced.sliced_sum("negdist", x, y, w, _equispaced_2d(P)), ref_n) for P in (16, 64)]
    assert errs_n[1] < errs_n[0] / 8          # at least second order in 1/P


def test_random_slicing_rate():
    """Prop. thm:accuracy_P / Thm. cor:error_bound: the slicing error decays like P^-1/2."""
    rng = np.random.default_rng(5)
    d = 6
    x = rng.standard_normal((60, d))
    y = rng.standard_normal((50, d))
    w = rng.uniform(0, 1, 60)
    ref = direct.direct_sum("negdist", x, y, w)
    Ps = np.array([8, 32, 128, 512])
    errs = []
    for P in Ps:
        e = [sliced.rel_l2(sliced.sliced_sum("negdist", x, y, w, directions.directions(d, P, seed)), ref)
             for seed in range(12)]
        errs.append(np.mean(e))
    slope = np.polyfit(np.log(Ps), np.log(errs), 1)[0]
    assert -0.65 < slope < -0.35


def _brute_sliced(kernel, x, y, w, xi, sigma):
    """Triple loop with mpmath counterparts (independent of the oracle's series)."""
    d = x.shape[1]
    P = xi.shape[0]
    out = np.zeros(y.shape[0])
    for m in range(y.shape[0]):
        acc = mpmath.mpf(0)
        for p in range(P):
            for n in range(x.shape[0]):
                t = abs(float(np.dot(xi[p], x[n] - y[m])))
                if kernel == "gaussian":
                    f = mpmath.hyp1f1(mpmath.mpf(d) / 2, 0.5, -t * t / (2 * sigma * sigma))
                elif kernel == "negdist":
                    f = -kn.c_d(d) * t
                elif kernel == "matern":
                    z = 0.75 * (t / sigma) ** 2
                    f = (mpmath.hyp1f2(mpmath.mpf(d) / 2, 0.5, -0.5, z)
                         + mpmath.sqrt(3 * mpmath.pi) * mpmath.gamma(mpmath.mpf(d) / 2 + 1.5)
                         / mpmath.gamma(mpmath.mpf(d) / 2) * (t / sigma) ** 3
                         * mpmath.hyp1f2(mpmath.mpf(d) / 2 + 1.5, 2, 2.5, z))
                else:
                    a = 1.0 / sigma
                    q = (a * t) ** 2 / 4
                    f = (mpmath.hyp1f2(mpmath.mpf(d) / 2, 0.5, 0.5, q)
                         - mpmath.sqrt(mpmath.pi) * a * t * mpmath.gamma((d + 1) / 2) / mpmath.gamma(d / 2)
                         * mpmath.hyp1f2((d + 1) / 2, 1, 1.5, q))
                acc += w[n] * f
        out[m] = float(acc / P)
    return out


@pytest.mark.parametrize("kernel,method,nc,T", [("gaussian", "ndft", 64, 0.045), ("negdist", "sort", 0, 0.0),
                                                ("laplacian", "nfft", 256, 0.125), ("matern", "nfft", 1024, 0.125)])
def test_pipeline_vs_brute_force_tiny(kernel, method, nc, T):
    rng = np.random.default_rng(6)
    d = 5
    x = rng.uniform(0, 1, (24, d))
    y = rng.uniform(0, 1, (16, d))
    w = rng.uniform(0, 1, 24)
    xi = directions.directions(d, 3, 11)
    sigma = 0.9
    s = sliced.sliced_sum(kernel, x, y, w, xi, sigma, method, nc, T)
    ref = _brute_sliced(kernel, x, y, w, xi, sigma)
    tol = {"negdist": 1e-13, "gaussian": 1e-8, "laplacian": 1e-7, "matern": 1e-8}[kernel]
    assert sliced.rel_l2(s, ref) < tol


def test_workload_small_case_matches_sliced_direct():
    """The gauss_ndft workload family: NDFT path vs exact 1-D sums, same directions."""
    wl = wlm.scaled(wlm.WORKLOADS["gauss_ndft"], N=300, M=200, P=8)
    x, y, w = wlm.generate(wl)
    sigma = wlm.median_heuristic(x, y)
    xi = directions.directions(wl.d, wl.P, wl.dir_seed)
    s = sliced.sliced_sum("gaussian", x, y, w, xi, sigma, "ndft", wl.n_coeff, wl.T)
    ref = sliced.sliced_direct("gaussian", x, y, w, xi, sigma)
    assert sliced.rel_l2(s, ref) < 1e-8
