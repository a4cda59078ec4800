"""Kernels, their one-dimensional counterparts and Fourier coefficients (FP64).

K(x,y) = F(||x-y||) on R^d and k(x,y) = f(|x-y|) on R are related by the slicing
identity K(x,y) = E_xi[k(<xi,x>, <xi,y>)] (eq. "sliced_kernel", Sec. 2).  The
pairs used here are the rows of Table "tab:kernels":

  Gaussian   F(r) = exp(-r^2/(2 sigma^2)),   f = 1F1(d/2; 1/2; -t^2/(2 sigma^2))
  Laplacian  F(r) = exp(-alpha r),            f = sum_n b_n t^n with
             b_n = (-alpha)^n sqrt(pi) Gamma((n+d)/2) / (n! Gamma(d/2) Gamma((n+1)/2))
  neg. dist. F(r) = -r,                       f = -c_d t,
             c_d = sqrt(pi) Gamma((d+1)/2) / Gamma(d/2)   (Sec. 3.2)
  Matern     nu = 3/2: F(r) = (1 + sqrt(3) r/beta) exp(-sqrt(3) r/beta), f from the
             1F2 form of the appendix on the Matern and Laplacian kernels

Parameters: `sigma` is the Gaussian bandwidth; the Laplacian uses alpha = 1/sigma;
the Matern kernel uses beta = sigma.
"""
from __future__ import annotations

import functools
import math

import numpy as np
from scipy.special import erfc

KERNELS = ("gaussian", "laplacian", "negdist", "matern")


def c_d(d: int) -> float:
    """c_d = sqrt(pi) Gamma((d+1)/2) / Gamma(d/2) (Sec. 3.2; Table "tab:kernels", negative distance)."""
    return math.sqrt(math.pi) * math.exp(math.lgamma((d + 1) / 2.0) - math.lgamma(d / 2.0))


def basis_F(kernel: str, r, sigma: float):
    """The d-dimensional basis function F(r) (first column of Table "tab:kernels")."""
    r = np.asarray(r, dtype=np.float64)
    if kernel == "gaussian":
        return np.exp(-r * r / (2.0 * sigma * sigma))
    if kernel == "laplacian":
        return np.exp(-r / sigma)
    if kernel == "negdist":
        return -r
    if kernel == "matern":
        a = math.sqrt(3.0) * r / sigma
        return (1.0 + a) * np.exp(-a)
    raise ValueError(kernel)


def _gauss_f_series(d: int, t, sigma: float):
    """1F1(d/2; 1/2; -z), z = t^2/(2 sigma^2), by its power series (Table "tab:kernels", Gaussian row).

    Term ratio T_{n+1}/T_n = (-z)(d/2+n) / ((1/2+n)(n+1)).  Plain FP64 summation:
    the absolute error is about 1e-16 times the largest term (<= e^z (1+z)^(d/2)).
    """
    z = np.asarray(t, dtype=np.float64) ** 2 / (2.0 * sigma * sigma)
    term = np.ones_like(z)
    total = np.ones_like(z)
    biggest = np.ones_like(z)
    n = 0
    while True:
        term = term * (-z) * (d / 2.0 + n) / ((0.5 + n) * (n + 1.0))
        n += 1
        total = total + term
        biggest = np.maximum(biggest, np.abs(term))
        if n > 8 and np.all(np.abs(term) <= 1e-18 * biggest):
            break
        if n > 20000:
            raise RuntimeError("1F1 series did not converge")
    return total


def _laplace_chains(d: int, t, alpha: float):
    """Even and odd partial sums of the Laplacian counterpart series (Table "tab:kernels").

    b_n t^n obeys T_{n+2} = T_n (alpha t)^2 (n+d) / ((n+1)^2 (n+2)) with
    T_0 = 1 and T_1 = -alpha t c_d; the even chain is positive, the odd chain negative.
    Returns (even_sum, odd_sum_from_n3, T_1).
    """
    at = alpha * np.asarray(t, dtype=np.float64)
    a2 = at * at
    even = np.ones_like(at)
    te = np.ones_like(at)
    t1 = -at * c_d(d)
    to = t1.copy()
    odd3 = np.zeros_like(at)
    biggest = np.ones_like(at)
    n = 0
    while True:
        te = te * a2 * (n + d) / ((n + 1.0) ** 2 * (n + 2.0))
        to = to * a2 * (n + 1 + d) / ((n + 2.0) ** 2 * (n + 3.0))
        even = even + te
        odd3 = odd3 + to
        biggest = np.maximum(biggest, np.maximum(np.abs(te), np.abs(to)))
        n += 2
        if n > 8 and np.all(np.abs(te) + np.abs(to) <= 1e-18 * biggest):
            break
        if n > 40000:
            raise RuntimeError("Laplacian series did not converge")
    return even, odd3, t1


def _hyp1f2(a: float, b1: float, b2: float, z):
    """1F2(a; b1, b2; z) by its power series, term ratio (a+n) z / ((b1+n) (b2+n) (n+1))."""
    z = np.asarray(z, dtype=np.float64)
    term = np.ones_like(z)
    total = np.ones_like(z)
    biggest = np.ones_like(z)
    n = 0
    while True:
        term = term * (a + n) * z / ((b1 + n) * (b2 + n) * (n + 1.0))
        n += 1
        total = total + term
        biggest = np.maximum(biggest, np.abs(term))
        if n > 8 and np.all(np.abs(term) <= 1e-18 * biggest):
            break
        if n > 20000:
            raise RuntimeError("1F2 series did not converge")
    return total


def matern32_f(d: int, t, beta: float):
    """1-D counterpart of the Matern kernel with nu = 3/2 (appendix, 1F2 form):
    f(t) = 1F2(d/2; 1/2, -1/2; z) + sqrt(3 pi) Gamma(d/2 + 3/2) / Gamma(d/2) (t/beta)^3
           1F2(d/2 + 3/2; 2, 5/2; z),   z = 3 t^2 / (4 beta^2)
    (the appendix's second term has the factor -Gamma(1 - nu) = 2 sqrt(pi) at nu = 3/2).
    The two FP64 series cancel: the error grows with (t/beta)^2 d; it stays below 2e-8 f(0)
    for (t/beta)^2 d <= 64 and reaches ~2e-7 f(0) at (t/beta)^2 d ~ 150, the edge of the
    range that rescaled data with beta of the size of the median distance reach."""
    x = np.abs(np.asarray(t, dtype=np.float64)) / beta
    z = 0.75 * x * x
    c3 = math.sqrt(3.0 * math.pi) * math.exp(math.lgamma(d / 2.0 + 1.5) - math.lgamma(d / 2.0))
    return _hyp1f2(d / 2.0, 0.5, -0.5, z) + c3 * x ** 3 * _hyp1f2(d / 2.0 + 1.5, 2.0, 2.5, z)


def counterpart_f(kernel: str, d: int, t, sigma: float):
    """The 1-D counterpart f(t), t >= 0 (fourth column of Table "tab:kernels")."""
    t = np.abs(np.asarray(t, dtype=np.float64))
    if kernel == "gaussian":
        return _gauss_f_series(d, t, sigma)
    if kernel == "laplacian":
        even, odd3, t1 = _laplace_chains(d, t, 1.0 / sigma)
        return even + t1 + odd3
    if kernel == "negdist":
        return -c_d(d) * t
    if kernel == "matern":
        return matern32_f(d, t, sigma)
    raise ValueError(kernel)


def laplace_k1(d: int, alpha: float, u):
    """Smooth part of the Laplacian counterpart (Sec. 3.3): k1(u) = f(|u|) + alpha c_d |u|.

    K1 = exp(-alpha r) + alpha r has counterpart f + alpha c_d |.|, i.e. the series
    of f with its linear term removed.
    """
    even, odd3, _ = _laplace_chains(d, np.abs(np.asarray(u, dtype=np.float64)), alpha)
    return even + odd3


def gauss_fourier_coeff(d: int, sigma: float, k):
    """Fourier transform of f_sigma = 1F1(d/2;1/2;-x^2/(2 sigma^2)) at omega = k (Lemma "lem:Fourier_Gauss").

    f^_sigma(w) = d pi sigma exp(-2 pi^2 sigma^2 w^2) (2 pi^2 sigma^2 w^2)^((d-1)/2) / (sqrt(2) Gamma((d+2)/2)),
    evaluated in log space (Sec. 2.2).  At w = 0 the value is sqrt(2 pi) sigma for d = 1 and 0 otherwise.
    """
    k = np.asarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    nz = k != 0
    z = 2.0 * math.pi ** 2 * sigma ** 2 * k[nz] ** 2
    logc = (math.log(d * math.pi * sigma / math.sqrt(2.0)) - math.lgamma((d + 2) / 2.0)
            - z + 0.5 * (d - 1) * np.log(z))
    out[nz] = np.exp(logc)
    if d == 1:
        out[~nz] = math.sqrt(2.0 * math.pi) * sigma
    return out


def taper(u, center: float = 0.375, width: float = 1.0 / 37.0):
    """W(u) = erfc((|u| - center)/width) / 2: ~1 for |u| <= 1/4, ~0 near |u| = 1/2."""
    return 0.5 * erfc((np.abs(np.asarray(u, dtype=np.float64)) - center) / width)


@functools.lru_cache(maxsize=8)
def _cos_matrix(K: int, L: int):
    """cos(2 pi k u_j) for k = 0..K and u_j = -1/2 + j/L, j = 0..L-1 (read-only)."""
    u = -0.5 + np.arange(L, dtype=np.float64) / L
    m = np.cos(2.0 * math.pi * np.outer(np.arange(K + 1, dtype=np.float64), u))
    m.setflags(write=False)
    return m


def tapered_coeffs(phi, K: int, L: int):
    """c_k = integral phi(u) W(u) exp(2 pi i k u) du, k = -K..K, on the torus [-1/2, 1/2) by the
    trapezoidal rule on u_j = -1/2 + j/L (phi even, so c_k is real and even in k):

        c_k = (1/L) sum_j phi(u_j) W(u_j) cos(2 pi k u_j)

    written out as the plain sum, as a product of the cosine matrix and the samples."""
    u = -0.5 + np.arange(L, dtype=np.float64) / L
    vals = phi(u) * taper(u)
    ks = np.arange(-K, K + 1)
    c_pos = _cos_matrix(K, L) @ vals / L          # k = 0..K
    return ks, c_pos[np.abs(ks)]


def laplace_smooth_coeffs(d: int, alpha_t: float, K: int, L: int):
    """Fourier coefficients c_k, k = -K..K, of the tapered smooth part on the torus [-1/2, 1/2).

    The paper computes the smooth part K1 of the Laplacian (Sec. 3.3) by fast
    Fourier summation without giving its coefficients.  Reading used here:
    phi(u) = k1(u) W(u) with k1 in rescaled units (alpha_t = alpha / tau) and the
    taper W above, and c_k = integral phi(u) exp(2 pi i k u) du by the trapezoidal
    rule on u_j = -1/2 + j/L, j = 0..L-1 (exact up to aliasing for periodic phi).
    phi is even, so c_k is real and even in k.
    """
    return tapered_coeffs(lambda u: laplace_k1(d, alpha_t, u), K, L)


def matern_coeffs(d: int, beta_t: float, K: int, L: int):
    """Fourier coefficients of the tapered Matern counterpart f(|u|) in rescaled units
    (beta_t = beta tau); f is continuously differentiable, so no part is split off (the
    paper's Matern runs use the NFFT on f directly)."""
    return tapered_coeffs(lambda u: matern32_f(d, u, beta_t), K, L)
