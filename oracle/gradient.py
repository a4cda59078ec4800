"""Gradients of the sliced kernel sum, FP64 -- TEST INFRASTRUCTURE ONLY.

For a loss with upstream gradient g_m = dL/ds_m of the sliced sum

  s_m = (1/P) sum_p t_{m,p},   t_{m,p} = sum_n w_n f(|<xi_p, x_n> - <xi_p, y_m>|)

(Algorithm "alg:fast_Fourier_sliced", Sec. 3) the chain rule through the
projections gives, with the directions held fixed,

  dL/dw_n = (1/P) sum_p sum_m g_m f(|z^x_{n,p} - z^y_{m,p}|)   (the sum with the roles of
                                                               sources and targets swapped)
  dL/dy_m = (g_m / P) sum_p D^y_{m,p} xi_p,   D^y_{m,p} = d/dz sum_n w_n f(|z^x_{n,p} - z|) at z = z^y_{m,p}
  dL/dx_n = (w_n / P) sum_p D^x_{n,p} xi_p,   D^x_{n,p} = d/dz sum_m g_m f(|z^y_{m,p} - z|) at z = z^x_{n,p}

The one-dimensional derivative sums D are computed the way the forward sums
are (Sec. 3.1 and 3.2):
  * Fourier summation: the derivative of sum_k c_k w^_k exp(2 pi i k y~) is the same
    sum with the coefficients 2 pi i k c_k, times tau (y~ = tau (y - c_min) - T);
  * sorting: d/dz of -c sum_n v_n |z_n - z| is -c (A_< - A_>), with A_< and A_> the sums
    of v over the points strictly below and strictly above z (sign(0) = 0, so a
    point coinciding with the target contributes nothing);
  * the Laplacian adds both parts (Sec. 3.3).
Readings: sign(0) = 0; c_min, c_max and tau of the rescaling are held constant
(the sums do not depend on them beyond the truncation error of Sec. 3.1).
"""
from __future__ import annotations

import math

import numpy as np

from . import kernels as kn
from . import onedim
from . import sliced


def ndft_deriv(xt, yt, w, ks, cs, tau: float, chunk: int = 4096):
    """tau * d/dy~ of the Fourier sum of onedim.ndft_sum at the targets yt."""
    xt = np.asarray(xt, dtype=np.float64)
    yt = np.asarray(yt, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    ks = np.asarray(ks, dtype=np.float64)
    cs = np.asarray(cs, dtype=np.float64)
    what = np.zeros(ks.shape[0], dtype=np.complex128)
    for s in range(0, xt.shape[0], chunk):
        what += np.exp(-2j * math.pi * np.outer(ks, xt[s:s + chunk])) @ w[s:s + chunk]
    h = (2j * math.pi * ks) * cs * what
    out = np.empty(yt.shape[0], dtype=np.float64)
    for s in range(0, yt.shape[0], chunk):
        out[s:s + chunk] = (np.exp(2j * math.pi * np.outer(yt[s:s + chunk], ks)) @ h).real
    return tau * out


def absdist_deriv_sum(zx, zy, w, c: float):
    """D_m = d/dz of -c sum_n w_n |zx_n - z| at z = zy_m, through the sorted sources:
    -c (A_<(m) - A_>(m)) with strict inequalities."""
    zx = np.asarray(zx, dtype=np.float64)
    zy = np.asarray(zy, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    order = np.argsort(zx, kind="stable")
    zs = zx[order]
    cum = np.concatenate([[0.0], np.cumsum(w[order])])
    lo = np.searchsorted(zs, zy, side="left")     # sources strictly below
    hi = np.searchsorted(zs, zy, side="right")    # sources below or equal
    a_lt = cum[lo]
    a_gt = cum[-1] - cum[hi]
    return -c * (a_lt - a_gt)


def slice_deriv(kernel: str, d: int, zx, zy, w, sigma: float, method: str, n_coeff: int, T: float,
                laplace_L_factor: int = 16, coeff_eps: float = 0.0):
    """Derivative sums D_m = d/dz sum_n w_n f(|zx_n - z|) at z = zy_m for one slice."""
    if kernel == "negdist":
        return absdist_deriv_sum(zx, zy, w, kn.c_d(d))
    K = sliced.cutoff_K(method, n_coeff)
    ks = np.arange(-K, K + 1)
    xt, yt, tau = sliced.rescale(zx, zy, T, sigma)
    if kernel == "gaussian":
        cs = sliced.cutoff(kn.gauss_fourier_coeff(d, tau * sigma, ks), coeff_eps)
        return ndft_deriv(xt, yt, w, ks, cs, tau)
    if kernel == "laplacian":
        alpha = 1.0 / sigma
        ks2, cs = kn.laplace_smooth_coeffs(d, alpha / tau, K, laplace_L_factor * n_coeff)
        return (ndft_deriv(xt, yt, w, ks2, sliced.cutoff(cs, coeff_eps), tau)
                + absdist_deriv_sum(zx, zy, w, alpha * kn.c_d(d)))
    if kernel == "matern":
        ks2, cs = kn.matern_coeffs(d, sigma * tau, K, laplace_L_factor * n_coeff)
        return ndft_deriv(xt, yt, w, ks2, sliced.cutoff(cs, coeff_eps), tau)
    raise ValueError(kernel)


def sliced_grad(kernel: str, x, y, w, g, xi, sigma: float = 1.0, method: str = "sort",
                n_coeff: int = 0, T: float = 0.0, coeff_eps: float = 0.0):
    """(dL/dx, dL/dy, dL/dw) of L with dL/ds = g for the sliced fast sum with directions xi."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    zx = sliced.project(x, xi)
    zy = sliced.project(y, xi)
    gx, gy = grad_from_projections(kernel, x.shape[1], zx, zy, w, g, xi, sigma, method, n_coeff, T, coeff_eps)
    grad_w = sliced.sliced_sum(kernel, y, x, g, xi, sigma, method, n_coeff, T, coeff_eps=coeff_eps)
    return gx, gy, grad_w


def grad_from_projections(kernel: str, d: int, zx, zy, w, g, xi, sigma: float = 1.0, method: str = "sort",
                          n_coeff: int = 0, T: float = 0.0, coeff_eps: float = 0.0):
    """(dL/dx, dL/dy) from given projections zx (N, P) and zy (M, P): the derivative sums of
    every slice and the back-projection onto the directions xi (P, d)."""
    zx = np.asarray(zx, dtype=np.float64)
    zy = np.asarray(zy, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    xi = np.asarray(xi, dtype=np.float64)
    P = xi.shape[0]
    Dy = np.empty((zy.shape[0], P))
    Dx = np.empty((zx.shape[0], P))
    for p in range(P):
        Dy[:, p] = slice_deriv(kernel, d, zx[:, p], zy[:, p], w, sigma, method, n_coeff, T, coeff_eps=coeff_eps)
        Dx[:, p] = slice_deriv(kernel, d, zy[:, p], zx[:, p], g, sigma, method, n_coeff, T, coeff_eps=coeff_eps)
    grad_y = (g / P)[:, None] * (Dy @ xi)
    grad_x = (w / P)[:, None] * (Dx @ xi)
    return grad_x, grad_y


def direct_deriv_1d(zx, zy, w, f, h: float = 1e-5):
    """D_m = sum_n w_n f'(|zy_m - zx_n|) sign(zy_m - zx_n), f' by a central difference of f
    (a brute-force reference for slice_deriv; sign(0) = 0)."""
    zx = np.asarray(zx, dtype=np.float64)
    zy = np.asarray(zy, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    out = np.empty(zy.shape[0])
    for m in range(zy.shape[0]):
        r = zy[m] - zx
        a = np.abs(r)
        fp = (f(a + h) - f(np.maximum(a - h, 0.0))) / (a + h - np.maximum(a - h, 0.0))
        out[m] = np.sum(w * fp * np.sign(r))
    return out
