"""Seeded synthetic workloads for the sliced kernel summation.

This module only draws inputs (points, weights) and states the workload
parameters.  It holds none of the summation method's arithmetic and is shared
by the FP64 oracle, the tests and the benchmark, so that both sides of a
parity check see identical inputs.

The shapes and distributions follow the paper's experimental setup (Sec. 4.1:
Gaussian points, uniform weights, M = N) and the four workload families the
implementation is measured on:

  gauss_ndft  Gaussian kernel, N=M=1000, d=10, x,y ~ N(0,I) (FP64), w ~ U[0,1],
              P=64 directions (seed 0), 64 Fourier coefficients, direct NDFT.
  negdist     negative distance kernel, N=M=1e5, d=784, x,y ~ U[0,1]^d (FP32),
              w = 1/N, P=256 directions (seed 1), sort + FP64 prefix sums.
  gauss_nfft  Gaussian kernel, N=M=1e6, d=50, x,y from a mixture of 10 isotropic
              Gaussians (means ~ N(0,4I), component std 1) (FP32), w ~ N(0,1),
              P=256 (seed 2), 128 coefficients, oversampling 2, KB half-width 6.
  laplace     Laplacian kernel exp(-||x-y||/sigma), N=M=2e5, d=3072,
              x,y ~ U[0,1]^d (FP32), w = 1/N, P=512 (seed 3), NFFT + sort.

sigma is the median pairwise distance of a 500-point subsample (the first 250
sources and the first 250 targets).  Data seeds are 1000 + workload number;
numpy's PCG64 generator draws everything.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    number: int          # 1..4, used for the data seed
    kernel: str          # "gaussian" | "negdist" | "laplacian"
    method: str          # "ndft" | "sort" | "nfft"
    N: int
    M: int
    d: int
    P: int
    dir_seed: int
    data: str            # "normal" | "uniform" | "mixture"
    weights: str         # "uniform01" | "inv_n" | "normal"
    dtype: str           # input dtype: "f64" or "f32"
    n_coeff: int = 0     # Fourier coefficients (0 = not used)
    T: float = 0.0       # rescaling threshold (0 = not used)
    oversample: int = 2
    window_m: int = 6


WORKLOADS = {
    "gauss_ndft": Workload("gauss_ndft", 1, "gaussian", "ndft", 1000, 1000, 10, 64, 0,
                           "normal", "uniform01", "f64", n_coeff=64, T=0.045),
    "negdist": Workload("negdist", 2, "negdist", "sort", 100_000, 100_000, 784, 256, 1,
                        "uniform", "inv_n", "f32"),
    "gauss_nfft": Workload("gauss_nfft", 3, "gaussian", "nfft", 1_000_000, 1_000_000, 50, 256, 2,
                           "mixture", "normal", "f32", n_coeff=128, T=0.02),
    "laplace": Workload("laplace", 4, "laplacian", "nfft", 200_000, 200_000, 3072, 512, 3,
                        "uniform", "inv_n", "f32", n_coeff=256, T=0.125),
}


def scaled(wl: Workload, N: Optional[int] = None, M: Optional[int] = None,
           d: Optional[int] = None, P: Optional[int] = None) -> Workload:
    """The same workload family at other sizes (used for small parity cases)."""
    return dataclasses.replace(wl, N=N if N is not None else wl.N, M=M if M is not None else wl.M,
                               d=d if d is not None else wl.d, P=P if P is not None else wl.P)


def _points(rng: np.random.Generator, kind: str, n: int, d: int, dtype, mix_means=None):
    if kind == "normal":
        return rng.standard_normal((n, d)).astype(dtype, copy=False)
    if kind == "uniform":
        if dtype == np.float32:
            return rng.random((n, d), dtype=np.float32)
        return rng.random((n, d))
    if kind == "mixture":
        comp = rng.integers(0, mix_means.shape[0], size=n)
        out = rng.standard_normal((n, d), dtype=np.float32) if dtype == np.float32 \
            else rng.standard_normal((n, d))
        out += mix_means[comp].astype(dtype)
        return out
    raise ValueError(kind)


def generate(wl: Workload, seed: Optional[int] = None):
    """Draw (x, y, w) for a workload.  x: (N,d), y: (M,d), w: (N,).

    Everything is drawn from one PCG64 stream in the order: mixture means (if
    any), x, y, w.  The dtype is FP64 for "f64" workloads and FP32 otherwise.
    """
    rng = np.random.default_rng(1000 + wl.number if seed is None else seed)
    dtype = np.float64 if wl.dtype == "f64" else np.float32
    means = None
    if wl.data == "mixture":
        means = 2.0 * rng.standard_normal((10, wl.d))      # means ~ N(0, 4I)
    x = _points(rng, wl.data, wl.N, wl.d, dtype, means)
    y = _points(rng, wl.data, wl.M, wl.d, dtype, means)
    if wl.weights == "uniform01":
        w = rng.random(wl.N).astype(dtype)
    elif wl.weights == "inv_n":
        w = np.full(wl.N, 1.0 / wl.N, dtype=dtype)
    elif wl.weights == "normal":
        w = rng.standard_normal(wl.N).astype(dtype)
    else:
        raise ValueError(wl.weights)
    return x, y, w


def median_heuristic(x: np.ndarray, y: np.ndarray, n_sub: int = 250) -> float:
    """Median pairwise distance of the first n_sub sources and first n_sub targets.

    All distances i < j among the 2*n_sub points, in FP64; for an even count the
    median is the mean of the two middle values.  Pure workload parameter
    selection (how the kernel bandwidth of a workload is chosen).
    """
    pts = np.concatenate([np.asarray(x[:n_sub], dtype=np.float64),
                          np.asarray(y[:n_sub], dtype=np.float64)], axis=0)
    n = pts.shape[0]
    dists = []
    for i in range(n - 1):
        diff = pts[i + 1:] - pts[i]
        dists.append(np.sqrt(np.einsum("ij,ij->i", diff, diff)))
    allv = np.sort(np.concatenate(dists))
    k = allv.shape[0]
    if k == 0:
        return 1.0
    if k % 2 == 1:
        return float(allv[k // 2])
    return float(0.5 * (allv[k // 2 - 1] + allv[k // 2]))


def kernel_scale(wl: Workload, x, y) -> float:
    """sigma for Gaussian/Laplacian workloads (Laplacian alpha = 1/sigma); 0 otherwise."""
    if wl.kernel in ("gaussian", "laplacian"):
        return median_heuristic(x, y)
    return 0.0


def subsample_targets(M: int, count: int = 2000) -> np.ndarray:
    """Indices of the targets on which the exact direct sum is evaluated (the first `count`)."""
    return np.arange(min(M, count))


def serving_stream(n_requests: int = 20000, rate: float = 200.0, seed: int = 4):
    """Request descriptors for the serving mix: Poisson arrivals, log-uniform N and M.

    Returns a list of dicts with arrival time (s), N, M, d, kernel, P, data kind and
    whether gradients are requested.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    lo, hi = math.log(1e3), math.log(5e5)
    out = []
    for i in range(n_requests):
        out.append(dict(
            arrival=float(t[i]),
            N=int(round(math.exp(rng.uniform(lo, hi)))),
            M=int(round(math.exp(rng.uniform(lo, hi)))),
            d=int(rng.choice([16, 128, 784, 3072])),
            kernel=str(rng.choice(["gaussian", "laplacian", "negdist"])),
            P=int(rng.choice([64, 256])),
            data=str(rng.choice(["normal", "uniform"])),
            grad=bool(rng.random() < 0.3),
        ))
    return out
