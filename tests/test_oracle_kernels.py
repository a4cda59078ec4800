"""Pins for oracle.kernels: constants, 1-D counterparts and Fourier coefficients.

Each check compares the oracle with something independent of its own formula:
Gamma-function special values, closed forms for d = 1 and d = 3 (Cor.
"cor:existence_d3"), mpmath's hypergeometric functions, the Riemann-Liouville
transform of Prop. "prop:sliced_kernels" by quadrature, and quadrature of the
Fourier integral of Lemma "lem:Fourier_Gauss".
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate

from oracle import kernels as kn


def test_cd_special_values():
    # c_1 = 1, c_2 = pi/2, c_3 = 2 from Gamma(1/2) = sqrt(pi), Gamma(1) = 1, Gamma(3/2) = sqrt(pi)/2
    assert kn.c_d(1) == pytest.approx(1.0, rel=1e-15)
    assert kn.c_d(2) == pytest.approx(math.pi / 2, rel=1e-15)
    assert kn.c_d(3) == pytest.approx(2.0, rel=1e-15)
    # d = 3 via Cor. cor:existence_d3: F(t) = -t gives f = F + t F' = -2t
    # large d: Gamma((d+1)/2)/Gamma(d/2) ~ sqrt(d/2) (1 - 1/(4d))
    for d in (1000, 10000):
        assert kn.c_d(d) / (math.sqrt(math.pi * d / 2) * (1 - 1 / (4 * d))) == pytest.approx(1.0, abs=1e-6)


@pytest.mark.parametrize("d", [1, 3, 10, 50])
def test_gauss_counterpart_vs_mpmath(d):
    sigma = 1.3
    t = np.linspace(0.0, 2.5, 11)
    ours = kn.counterpart_f("gaussian", d, t, sigma)
    ref = np.array([float(mpmath.hyp1f1(d / 2, 0.5, -(tt ** 2) / (2 * sigma ** 2))) for tt in t])
    # FP64 series error bound: ~1e-16 * (number of terms) * sum_n |T_n|, and sum |T_n| = 1F1(d/2; 1/2; +z)
    absum = np.array([float(mpmath.hyp1f1(d / 2, 0.5, (tt ** 2) / (2 * sigma ** 2))) for tt in t])
    assert np.all(np.abs(ours - ref) <= 1e-14 * absum + 1e-15)


def test_gauss_counterpart_closed_forms():
    sigma = 0.8
    t = np.linspace(0, 3, 17)
    z = t ** 2 / (2 * sigma ** 2)
    # d = 1: the counterpart is the kernel itself
    assert np.allclose(kn.counterpart_f("gaussian", 1, t, sigma), np.exp(-z), atol=1e-14)
    # d = 3: f = F + t F' = exp(-z) (1 - 2 z)
    assert np.allclose(kn.counterpart_f("gaussian", 3, t, sigma), np.exp(-z) * (1 - 2 * z), atol=1e-13)


def _laplace_1f2(d, alpha, x):
    """App. C closed form: 1F2(d/2; 1/2, 1/2; a^2x^2/4) - sqrt(pi) a x Gamma((d+1)/2)/Gamma(d/2) 1F2((d+1)/2; 1, 3/2; a^2x^2/4)."""
    q = (alpha * x) ** 2 / 4
    pref = mpmath.sqrt(mpmath.pi) * alpha * x * mpmath.gamma((d + 1) / 2) / mpmath.gamma(d / 2)
    return mpmath.hyp1f2(d / 2, 0.5, 0.5, q) - pref * mpmath.hyp1f2((d + 1) / 2, 1, 1.5, q)


@pytest.mark.parametrize("d", [2, 5, 50, 3072])
def test_laplace_counterpart_vs_appendix_1f2(d):
    mpmath.mp.dps = 40
    alpha = 0.3 if d < 100 else 0.044
    t = np.linspace(0.0, 4.0, 9)
    ours = kn.counterpart_f("laplacian", d, t, 1.0 / alpha)
    ref = np.array([float(_laplace_1f2(d, alpha, tt)) for tt in t])
    scale = max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(ours - ref)) / scale < 1e-9
    mpmath.mp.dps = 15


def test_laplace_counterpart_closed_forms():
    alpha = 0.7
    t = np.linspace(0, 5, 21)
    assert np.allclose(kn.counterpart_f("laplacian", 1, t, 1 / alpha), np.exp(-alpha * t), atol=1e-14)
    # d = 3, Cor. cor:existence_d3: f = F + t F' = exp(-a t)(1 - a t)
    assert np.allclose(kn.counterpart_f("laplacian", 3, t, 1 / alpha),
                       np.exp(-alpha * t) * (1 - alpha * t), atol=1e-13)


def test_laplace_k1_removes_linear_term():
    d, alpha = 20, 0.4
    u = np.array([0.0, 1e-4, 0.5, 2.0])
    f = kn.counterpart_f("laplacian", d, u, 1 / alpha)
    k1 = kn.laplace_k1(d, alpha, u)
    assert np.allclose(k1 - f, alpha * kn.c_d(d) * np.abs(u), atol=1e-12)
    # k1 is flat at 0 to second order: (k1(h) - k1(0))/h -> 0
    h = 1e-5
    assert abs((kn.laplace_k1(d, alpha, h) - kn.laplace_k1(d, alpha, 0.0)) / h) < 1e-3


@pytest.mark.parametrize("kernel,d", [("gaussian", 3), ("gaussian", 10), ("laplacian", 4),
                                      ("laplacian", 10), ("negdist", 7), ("matern", 4), ("matern", 12)])
def test_riemann_liouville_transform(kernel, d):
    """Prop. prop:sliced_kernels: F(s) = 2Gamma(d/2)/(sqrt(pi)Gamma((d-1)/2)) int_0^1 f(ts)(1-t^2)^((d-3)/2) dt."""
    sigma = 1.1
    pref = 2 * math.gamma(d / 2) / (math.sqrt(math.pi) * math.gamma((d - 1) / 2))
    for s in (0.3, 1.0, 2.2):
        integrand = lambda t: float(kn.counterpart_f(kernel, d, t * s, sigma)) * (1 - t * t) ** ((d - 3) / 2)
        val, _ = integrate.quad(integrand, 0, 1, epsabs=1e-13, epsrel=1e-12, limit=200)
        assert pref * val == pytest.approx(float(kn.basis_F(kernel, s, sigma)), rel=1e-9, abs=1e-11)


def test_gauss_fourier_d1_textbook():
    # d = 1: f = exp(-x^2/(2 s^2)) has Fourier transform s sqrt(2 pi) exp(-2 pi^2 s^2 w^2)
    s = 0.37
    w = np.linspace(-3, 3, 13)
    ref = s * math.sqrt(2 * math.pi) * np.exp(-2 * math.pi ** 2 * s ** 2 * w ** 2)
    assert np.allclose(kn.gauss_fourier_coeff(1, s, w), ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("d", [3, 10])
def test_gauss_fourier_vs_quadrature(d):
    """Lemma lem:Fourier_Gauss against int f_sigma(x) cos(2 pi w x) dx with mpmath's 1F1."""
    mpmath.mp.dps = 30
    sigma = 0.9
    for w in (0.3, 0.7, 1.2):
        f = lambda x: mpmath.hyp1f1(mpmath.mpf(d) / 2, 0.5, -x * x / (2 * sigma ** 2)) * mpmath.cos(2 * mpmath.pi * w * x)
        val = 2 * mpmath.quadosc(f, [0, mpmath.inf], omega=2 * mpmath.pi * w)
        ours = float(kn.gauss_fourier_coeff(d, sigma, w))
        assert abs(ours - float(val)) < 1e-10 * max(1.0, abs(float(val)))
    mpmath.mp.dps = 15


@pytest.mark.parametrize("d", [1, 2, 10, 200])
def test_gauss_fourier_integrates_to_one(d):
    # Fourier inversion at x = 0: int f^_sigma(w) dw = f_sigma(0) = 1
    sigma = 0.6
    val, _ = integrate.quad(lambda w: float(kn.gauss_fourier_coeff(d, sigma, w)), -np.inf, np.inf,
                            epsabs=1e-13, limit=400)
    assert val == pytest.approx(1.0, abs=1e-10)


def test_laplace_smooth_coeffs_synthesis():
    """The taper-recipe coefficients resynthesise k1*W on the region the data can occupy.

    k1 has a |u|^3 kink at 0 (its series has odd powers from 3 on), so the truncated
    Fourier series converges like K^-3: loose at the default 256 coefficients, tight at 1024.
    """
    d, alpha_t = 3072, 0.5
    u = np.linspace(-0.25, 0.25, 41)
    ref = kn.laplace_k1(d, alpha_t, u) * kn.taper(u)
    assert np.all(np.abs(kn.taper(u) - 1) < 1e-9)
    for nf, tol in ((256, 2e-6), (1024, 5e-8)):
        K = nf // 2 - 1
        ks, cs = kn.laplace_smooth_coeffs(d, alpha_t, K, 16 * nf)
        assert np.array_equal(cs, cs[::-1])            # even in k
        synth = np.array([np.sum(cs * np.cos(2 * math.pi * ks * uu)) for uu in u])
        assert np.max(np.abs(synth - ref)) < tol * np.max(np.abs(ref))


@pytest.mark.parametrize("d", [1, 3])
def test_matern_counterpart_closed_forms(d):
    # d = 1: f = F; d = 3: f = F + t F' = (1 + a - a^2) exp(-a), a = sqrt(3) t / beta
    t = np.linspace(0.0, 4.0, 41)
    beta = 1.3
    a = math.sqrt(3.0) * t / beta
    ref = (1 + a) * np.exp(-a) if d == 1 else (1 + a - a * a) * np.exp(-a)
    assert np.allclose(kn.counterpart_f("matern", d, t, beta), ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("d", [2, 7, 50, 3072])
def test_matern_counterpart_vs_mpmath(d):
    # the FP64 series cancel: for (t / beta)^2 d <= 64 the error stays below 2e-8 f(0)
    beta = 0.8
    tmax = 8.0 * beta / math.sqrt(d)
    for t in (0.01 * tmax, 0.3 * tmax, tmax):
        z = 0.75 * (t / beta) ** 2
        ref = (mpmath.hyp1f2(mpmath.mpf(d) / 2, 0.5, -0.5, z)
               + mpmath.sqrt(3 * mpmath.pi) * mpmath.gamma(mpmath.mpf(d) / 2 + 1.5) / mpmath.gamma(mpmath.mpf(d) / 2)
               * (t / beta) ** 3 * mpmath.hyp1f2(mpmath.mpf(d) / 2 + 1.5, 2, 2.5, z))
        assert abs(float(kn.counterpart_f("matern", d, t, beta)) - float(ref)) <= 2e-8


def test_matern_coeffs_synthesis():
    d, beta_t, K = 10, 0.3, 511
    ks, c = kn.matern_coeffs(d, beta_t, K, 16 * 1024)
    u = np.linspace(-0.25, 0.25, 101)
    synth = (np.exp(2j * math.pi * np.outer(u, ks)) @ c).real
    ref = kn.matern32_f(d, u, beta_t)
    assert np.max(np.abs(synth - ref)) <= 1e-7 * np.max(np.abs(ref))
