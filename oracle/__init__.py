"""FP64 CPU oracle for the sliced fast kernel summation -- TEST INFRASTRUCTURE ONLY.

Plain, slow, deliberately unoptimised reference code written from the paper
(J. Hertrich, "Fast Kernel Summation in High Dimensions via Slicing and Fourier
Transforms").  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import it; the GPU library never calls it and shares no code with it
(the two only share the seeded input generators in ``workloads``).

Modules
  directions  counter-based SplitMix64 + Box-Muller directions on S^{d-1}
  kernels     basis functions F, 1-D counterparts f (Table "tab:kernels"),
              c_d (Sec. 3.2), Gaussian Fourier coefficients (Lemma
              "lem:Fourier_Gauss"), Laplacian smooth-part coefficients
  onedim      1-D summations: direct, Fourier summation by NDFT (Sec. 3.1),
              sort + cumsum (Algorithm "alg:fastsum_energy", Sec. 3.2)
  sliced      Algorithm "alg:fast_Fourier_sliced" with the rescaling of Sec. 3.1
              and the Laplacian decomposition of Sec. 3.3
  direct      the exact O(MN) kernel sum (problem statement, Sec. 1 / Sec. 3)
  gradient    gradients of the sliced fast sum: derivative sums by Fourier
              summation with 2 pi i k c_k and by sorting (sign(0) = 0), and the
              back-projection onto the directions

Every floating-point computation is FP64.  Pinned by tests/test_oracle_*.py
against closed forms, independent library evaluations (mpmath), brute force on
tiny inputs, exactness on small integers and the O(P^-1/2) slicing rate.
"""
from . import directions, kernels, onedim, sliced, direct, gradient  # noqa: F401
