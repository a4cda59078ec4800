/* Exact kernel sum s_m = sum_n w_n F(||x_n - y_m||) (problem statement, Sec. 1 and Sec. 3).
 *
 * Part of the FP64 CPU oracle (test infrastructure only).  Plain loops in the
 * order of the definition, FP64 arithmetic, one OpenMP thread per target block.
 * x: N*d, y: M*d, row-major; inputs may be FP32 or FP64 (converted exactly to FP64).
 * kernel: 1 Gaussian exp(-r^2/(2 sigma^2)), 2 Laplacian exp(-r/sigma), 3 negative distance -r,
 *         4 Matern nu = 3/2 (1 + sqrt(3) r/sigma) exp(-sqrt(3) r/sigma).
 */
#include <math.h>
#include <stdint.h>

static double basis(int kernel, double r2, double sigma) {
  if (kernel == 1) return exp(-r2 / (2.0 * sigma * sigma));
  if (kernel == 2) return exp(-sqrt(r2) / sigma);
  if (kernel == 4) {
    const double a = sqrt(3.0) * sqrt(r2) / sigma;
    return (1.0 + a) * exp(-a);
  }
  return -sqrt(r2);
}

#define DEFINE_DIRECT(NAME, T)                                                              \
  void NAME(const T *x, int64_t N, const T *y, int64_t M, int64_t d, const T *w,            \
            int kernel, double sigma, double *s) {                                          \
    _Pragma("omp parallel for schedule(dynamic, 1)")                                        \
    for (int64_t m = 0; m < M; ++m) {                                                       \
      const T *ym = y + m * d;                                                              \
      double acc = 0.0;                                                                     \
      for (int64_t n = 0; n < N; ++n) {                                                     \
        const T *xn = x + n * d;                                                            \
        double r2 = 0.0;                                                                    \
        for (int64_t i = 0; i < d; ++i) {                                                   \
          double diff = (double)xn[i] - (double)ym[i];                                      \
          r2 += diff * diff;                                                                \
        }                                                                                   \
        acc += (double)w[n] * basis(kernel, r2, sigma);                                     \
      }                                                                                     \
      s[m] = acc;                                                                           \
    }                                                                                       \
  }

DEFINE_DIRECT(oracle_direct_sum_f64, double)
DEFINE_DIRECT(oracle_direct_sum_f32, float)
