// Host-side tables of a plan: random directions and the Kaiser-Bessel window.
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "internal.h"

namespace ksum {

// ---------------------------------------------------------------------------
// Directions uniform on S^{d-1}: normalised standard Gaussian vectors.  The
// Gaussians come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", 2014) used as a counter-based generator and
// the Box-Muller transform (cosine branch).
// ---------------------------------------------------------------------------
static inline uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

void generate_directions(int32_t d, int32_t P, uint64_t seed, double *out) {
  std::vector<double> g(d);
  for (int32_t p = 0; p < P; ++p) {
    for (int32_t i = 0; i < d; ++i) {
      const uint64_t c = 2ull * ((uint64_t)p * (uint64_t)d + (uint64_t)i);
      const uint64_t o1 = splitmix64_at(seed, c);
      const uint64_t o2 = splitmix64_at(seed, c + 1);
      const double u1 = (double)((o1 >> 11) + 1) * 0x1.0p-53;
      const double u2 = (double)(o2 >> 11) * 0x1.0p-53;
      g[i] = std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
    double nrm2 = 0.0;
    for (int32_t i = 0; i < d; ++i) nrm2 += g[i] * g[i];
    const double nrm = std::sqrt(nrm2);
    for (int32_t i = 0; i < d; ++i) out[(int64_t)p * d + i] = g[i] / nrm;
  }
}

// ---------------------------------------------------------------------------
// Kaiser-Bessel window of the NFFT literature (the NFFT3 library the paper
// uses): grid size n, half-width m cells, shape b = pi (2 - 1/sigma_os).
//   phi(x)  = sinh(b sqrt(m^2 - (n x)^2)) / (pi sqrt(m^2 - (n x)^2)),  |n x| <= m
//   phi^(k) = I_0(m sqrt(b^2 - (2 pi k / n)^2)) / n
// (phi^ is the continuous Fourier transform of phi at integer frequency k).
// ---------------------------------------------------------------------------
static double bessel_i0(double x) {
  // power series sum_k (x^2/4)^k / (k!)^2; all terms positive
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 1000; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

static double kb_shape(int oversample) { return M_PI * (2.0 - 1.0 / (double)oversample); }

// phi at an offset of `cells` grid cells (cells = n x)
static double kb_phi_cells(int m, int oversample, double cells) {
  const double b = kb_shape(oversample);
  const double s2 = (double)m * m - cells * cells;
  if (s2 < 0.0) return 0.0;
  const double s = std::sqrt(s2);
  if (s < 1e-12) return b / M_PI;
  return std::sinh(b * s) / (M_PI * s);
}

double kb_phihat(int m, int n, int oversample, int k) {
  const double b = kb_shape(oversample);
  const double a = 2.0 * M_PI * (double)k / (double)n;
  const double arg = b * b - a * a;
  if (arg <= 0.0) return 0.0;
  return bessel_i0((double)m * std::sqrt(arg)) / (double)n;
}

int window_degree_for(int m);

// Fits phi((fr + m - 1 - j)/n) / phi(0), fr in [0,1), j = 0..m-1, by polynomials
// in x = fr - 1/2 of degree deg: Chebyshev interpolation at deg+1 Chebyshev
// nodes of [-1/2, 1/2] (near-minimax), converted to monomials.  The fit is
// checked on a fine grid; err receives a message if it is worse than 1e-6 (the
// degrees chosen reach 5e-8).
bool build_window_poly(int m, int n, int oversample, WindowPoly *out, std::string *err) {
  (void)n;
  const int deg = window_degree_for(m);
  if (2 * m > kMaxTaps || deg > kMaxPolyDeg) {
    *err = "window too wide";
    return false;
  }
  const double phi0 = kb_phi_cells(m, oversample, 0.0);
  out->taps = 2 * m;
  out->deg = deg;
  for (int j = 0; j < kMaxTaps; ++j)
    for (int q = 0; q <= kMaxPolyDeg; ++q) out->c[j][q] = 0.f;
  const int nn = deg + 1;
  double worst = 0.0;
  for (int j = 0; j < m; ++j) {
    // Chebyshev coefficients a_k of f(x), x = t/2, t in [-1,1]
    std::vector<double> fx(nn), a(nn, 0.0);
    for (int i = 0; i < nn; ++i) {
      const double t = std::cos(M_PI * (i + 0.5) / nn);
      const double fr = 0.5 * t + 0.5;
      fx[i] = kb_phi_cells(m, oversample, fr + m - 1 - j) / phi0;
    }
    for (int k = 0; k < nn; ++k) {
      double s = 0.0;
      for (int i = 0; i < nn; ++i) s += fx[i] * std::cos(M_PI * k * (i + 0.5) / nn);
      a[k] = (k == 0 ? 1.0 : 2.0) * s / nn;
    }
    // monomial coefficients in t: T_0 = 1, T_1 = t, T_{k+1} = 2t T_k - T_{k-1}
    std::vector<double> mono(nn, 0.0), tkm1(nn, 0.0), tk(nn, 0.0), tkp1(nn, 0.0);
    tkm1[0] = 1.0;
    if (nn > 1) tk[1] = 1.0;
    for (int q = 0; q < nn; ++q) mono[q] += a[0] * tkm1[q];
    if (nn > 1)
      for (int q = 0; q < nn; ++q) mono[q] += a[1] * tk[q];
    for (int k = 2; k < nn; ++k) {
      for (int q = 0; q < nn; ++q) tkp1[q] = -tkm1[q] + (q > 0 ? 2.0 * tk[q - 1] : 0.0);
      for (int q = 0; q < nn; ++q) mono[q] += a[k] * tkp1[q];
      tkm1 = tk;
      tk = tkp1;
    }
    // t = 2x: coefficient of x^q is mono[q] * 2^q
    for (int q = 0; q < nn; ++q) out->c[j][q] = (float)(mono[q] * std::ldexp(1.0, q));
    // check on a fine grid (double evaluation of the float coefficients)
    for (int i = 0; i <= 400; ++i) {
      const double x = -0.5 + i / 400.0;
      double v = 0.0;
      for (int q = nn - 1; q >= 0; --q) v = v * x + (double)out->c[j][q];
      const double ref = kb_phi_cells(m, oversample, x + 0.5 + m - 1 - j) / phi0;
      worst = std::fmax(worst, std::fabs(v - ref));
    }
  }
  if (worst > 1e-6) {
    *err = "window polynomial fit error " + std::to_string(worst);
    return false;
  }
  return true;
}

}  // namespace ksum
