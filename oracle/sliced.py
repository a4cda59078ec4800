"""Sliced kernel summation, Algorithm "alg:fast_Fourier_sliced" (Sec. 3), FP64.

  s_m ~= (1/P) sum_p t_{m,p},   t_{m,p} = sum_n w_n k(<xi_p, x_n>, <xi_p, y_m>)

with the 1-D sums by
  * sorting (negative distance, Sec. 3.2),
  * fast Fourier summation with direct NDFTs (Gaussian, Sec. 3.1 + Sec. 2.2),
  * both (Laplacian, Sec. 3.3: k = k1 + k2, k1 smooth, k2 = -alpha c_d |.|).

Readings of passages that are garbled or silent (all listed in the design notes):
  * Rescaling (Sec. 3.1): per slice c_min, c_max over sources and targets,
    tau = 2T/(c_max - c_min), x~ = tau (x - c_min) - T in [-T, T], and the
    rescaled kernel phi~(u) = phi(u / tau).  For the Gaussian f_sigma(u/tau) =
    f_{tau sigma}(u), so c_k = f^_{tau sigma}(k).  A slice whose points all
    project to one value uses c_max - c_min := sigma.
  * Cutoff set: "ndft" with n_coeff coefficients uses k = -n_coeff/2..n_coeff/2;
    "nfft" with n_coeff coefficients uses the index set -n_coeff/2..n_coeff/2-1 with
    c_{-n_coeff/2} := 0, i.e. k = -(n_coeff/2-1)..n_coeff/2-1.  (The NFFT is a fast
    approximation of the same NDFT, so the oracle evaluates the NDFT.)
  * Laplacian smooth part: coefficients from oracle.kernels.laplace_smooth_coeffs
    with L = 16 n_coeff samples; the Matern kernel (nu = 3/2) the same recipe on its
    whole counterpart (oracle.kernels.matern_coeffs).
  * Cutoff threshold (eq. "Fourier_cutoff", Sec. 2.2): C keeps the k of the index
    set above with |c_k| > eps; the others are left out of the sum (their c_k is
    taken as 0).  eps = 0 keeps every nonzero coefficient.
"""
from __future__ import annotations

import numpy as np

from . import kernels as kn
from . import onedim


def project(points, xi):
    """P_xi(x) = <xi, x> for every point and direction: (n, P), FP64."""
    return np.asarray(points, dtype=np.float64) @ np.asarray(xi, dtype=np.float64).T


def cutoff_K(method: str, n_coeff: int) -> int:
    """Largest |k| of the symmetric cutoff set used for a method and coefficient count."""
    if method == "ndft":
        return n_coeff // 2
    if method == "nfft":
        return n_coeff // 2 - 1
    raise ValueError(method)


def cutoff(cs, eps: float):
    """The cutoff set of eq. "Fourier_cutoff" (Sec. 2.2): coefficients with |c_k| <= eps are
    dropped from C, i.e. contribute nothing to the Fourier sum."""
    cs = np.asarray(cs, dtype=np.float64)
    return np.where(np.abs(cs) > eps, cs, 0.0)


def rescale(zx, zy, T: float, sigma: float):
    """Map one slice onto [-T, T] (Sec. 3.1, "Rescaling"); returns (x~, y~, tau)."""
    cmin = min(np.min(zx), np.min(zy))
    cmax = max(np.max(zx), np.max(zy))
    rng = cmax - cmin
    if not rng > 0.0:
        rng = sigma
    tau = 2.0 * T / rng
    return tau * (zx - cmin) - T, tau * (zy - cmin) - T, tau


def slice_sum(kernel: str, d: int, zx, zy, w, sigma: float, method: str, n_coeff: int, T: float,
              laplace_L_factor: int = 16, coeff_eps: float = 0.0):
    """t_m for one slice by the fast 1-D summation the kernel uses."""
    if kernel == "negdist":
        return onedim.negdist_sum(zx, zy, w, kn.c_d(d))
    K = cutoff_K(method, n_coeff)
    ks = np.arange(-K, K + 1)
    xt, yt, tau = rescale(zx, zy, T, sigma)
    if kernel == "gaussian":
        cs = cutoff(kn.gauss_fourier_coeff(d, tau * sigma, ks), coeff_eps)
        return onedim.ndft_sum(xt, yt, w, ks, cs)
    if kernel == "laplacian":
        alpha = 1.0 / sigma
        ks2, cs = kn.laplace_smooth_coeffs(d, alpha / tau, K, laplace_L_factor * n_coeff)
        t1 = onedim.ndft_sum(xt, yt, w, ks2, cutoff(cs, coeff_eps))
        t2 = onedim.negdist_sum(zx, zy, w, alpha * kn.c_d(d))
        return t1 + t2
    if kernel == "matern":
        ks2, cs = kn.matern_coeffs(d, sigma * tau, K, laplace_L_factor * n_coeff)
        return onedim.ndft_sum(xt, yt, w, ks2, cutoff(cs, coeff_eps))
    raise ValueError(kernel)


def sliced_sum(kernel: str, x, y, w, xi, sigma: float = 1.0, method: str = "sort",
               n_coeff: int = 0, T: float = 0.0, return_slices: bool = False, coeff_eps: float = 0.0):
    """Algorithm "alg:fast_Fourier_sliced": average of the P one-dimensional fast sums."""
    d = np.asarray(x).shape[1]
    zx = project(x, xi)
    zy = project(y, xi)
    P = zx.shape[1]
    ts = np.empty((P, zy.shape[0]), dtype=np.float64)
    for p in range(P):
        ts[p] = slice_sum(kernel, d, zx[:, p], zy[:, p], w, sigma, method, n_coeff, T, coeff_eps=coeff_eps)
    s = ts.sum(axis=0) / P
    if return_slices:
        return s, ts
    return s


def sliced_direct(kernel: str, x, y, w, xi, sigma: float = 1.0, return_slices: bool = False):
    """The slicing approximation with exact 1-D sums: (1/P) sum_p sum_n w_n f(|<xi_p, x_n - y_m>|)."""
    d = np.asarray(x).shape[1]
    zx = project(x, xi)
    zy = project(y, xi)
    P = zx.shape[1]
    ts = np.empty((P, zy.shape[0]), dtype=np.float64)

    def f(t):
        return kn.counterpart_f(kernel, d, t, sigma)

    for p in range(P):
        ts[p] = onedim.direct_1d(zx[:, p], zy[:, p], w, f)
    s = ts.sum(axis=0) / P
    if return_slices:
        return s, ts
    return s


def rel_l2(a, ref) -> float:
    """||a - ref||_2 / ||ref||_2."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def per_summand_error(a, ref, w) -> float:
    """The paper's error measure ||s_true - s||_1 / (M sum_n |w_n|) (Sec. 4.1)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sum(np.abs(a - ref)) / (ref.shape[0] * np.sum(np.abs(np.asarray(w, np.float64)))))
