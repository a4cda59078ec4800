"""One-dimensional kernel sums t_m = sum_n w_n k(x_n, y_m) (Sec. 3), FP64.

  direct_1d       the definition, O(MN)
  ndft_sum        fast Fourier summation with direct non-equispaced transforms (Sec. 3.1)
  negdist_sorted  Algorithm "alg:fastsum_energy" on an ascending sequence (Sec. 3.2)
  negdist_sum     the general case of Sec. 3.2 through a stable sorting permutation
"""
from __future__ import annotations

import math

import numpy as np


def direct_1d(zx, zy, w, f):
    """t_m = sum_n w_n f(|zx_n - zy_m|) by its definition (eq. "large_sum")."""
    zx = np.asarray(zx, dtype=np.float64)
    zy = np.asarray(zy, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    t = np.empty(zy.shape[0], dtype=np.float64)
    for m in range(zy.shape[0]):
        t[m] = np.sum(w * f(np.abs(zx - zy[m])))
    return t


def ndft_sum(xt, yt, w, ks, cs, chunk: int = 4096):
    """Fast Fourier summation of Sec. 3.1 with direct transforms.

    xt, yt: rescaled points in [-1/2, 1/2); ks: the cutoff set C (symmetric);
    cs: the coefficients c_k of phi(x) = sum_k c_k exp(-2 pi i k x).
      w^_k = sum_n w_n exp(-2 pi i k x_n)             (adjoint NDFT)
      t_m  = Re sum_k c_k w^_k exp(+2 pi i k y_m)       (NDFT)
    (The sign of the forward exponent is the one that makes t_m = sum_n w_n phi(x_n - y_m).)
    """
    xt = np.asarray(xt, dtype=np.float64)
    yt = np.asarray(yt, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    ks = np.asarray(ks, dtype=np.float64)
    cs = np.asarray(cs, dtype=np.float64)
    what = np.zeros(ks.shape[0], dtype=np.complex128)
    for s in range(0, xt.shape[0], chunk):
        e = np.exp(-2j * math.pi * np.outer(ks, xt[s:s + chunk]))
        what += e @ w[s:s + chunk]
    h = cs * what
    t = np.empty(yt.shape[0], dtype=np.float64)
    for s in range(0, yt.shape[0], chunk):
        e = np.exp(2j * math.pi * np.outer(yt[s:s + chunk], ks))
        t[s:s + chunk] = (e @ h).real
    return t


def negdist_sorted(z, v, cd: float):
    """Algorithm "alg:fastsum_energy": t_m = -sum_n c_d v_n |z_n - z_m| for ascending z.

    a = cumsum(c_d v); a~_i = a_i (z_{i+1} - z_i); b = cumsum(a~);
    t_m = b_{L-1} - 2 b_{m-1} - a_L (z_L - z_m), with the readings a~_L := 0 (z_{L+1}
    does not exist and a~_L is never used) and b_0 := 0.  Indices below are 0-based.
    """
    z = np.asarray(z, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    L = z.shape[0]
    if L == 0:
        return np.zeros(0)
    a = np.cumsum(cd * v)
    at = np.zeros(L, dtype=np.float64)
    at[:L - 1] = a[:L - 1] * (z[1:] - z[:L - 1])
    b = np.cumsum(at)
    b_prev = np.zeros(L, dtype=np.float64)      # b_{m-1} for m = 1..L (1-based)
    b_prev[1:] = b[:L - 1]
    b_last = b[L - 2] if L >= 2 else 0.0        # b_{L-1} (1-based)
    return b_last - 2.0 * b_prev - a[L - 1] * (z[L - 1] - z)


def negdist_sum(zx, zy, w, cd: float, return_perm: bool = False):
    """Sec. 3.2, general case: t_m = -sum_n c_d w_n |x_n - y_m| via sorting.

    Union z = (y_1..y_M, x_1..x_N), v = (0..0, w_1..w_N); sigma is the stable
    ascending permutation (ties in union-index order); Algorithm
    "alg:fastsum_energy" runs on z_sigma and the inverse permutation brings the
    results back.  Returns the first M entries (the targets).
    """
    zx = np.asarray(zx, dtype=np.float64)
    zy = np.asarray(zy, dtype=np.float64)
    M = zy.shape[0]
    z = np.concatenate([zy, zx])
    v = np.concatenate([np.zeros(M), np.asarray(w, dtype=np.float64)])
    perm = np.argsort(z, kind="stable")
    t_sorted = negdist_sorted(z[perm], v[perm], cd)
    t = np.empty_like(t_sorted)
    t[perm] = t_sorted
    if return_perm:
        return t[:M], perm
    return t[:M]
