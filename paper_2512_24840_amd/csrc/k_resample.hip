// Flux-conserving resampling (Section 2.2, step 3; Eqs. 2-4) from a linear
// wavelength grid onto a grid uniform in log10.
//
// Eqs. 2-4 take the cumulative integral C of the piecewise-constant source
// at its bin edges, interpolate C linearly at the target edges and divide the
// differences by the target widths.  C is linear inside each source bin, so
// C(l_b) - C(l_a) is the integral of the source between l_a and l_b: the
// bins strictly inside plus the covered fractions of the two end bins.  Each
// thread forms that local sum for one target pixel directly, which needs no
// prefix scan across the row and carries no cancellation of two large
// cumulative values; it is the same quantity up to rounding.
#include "lasp_internal.h"

namespace lasp {
namespace {

// Position of wavelength l in source bins, l = e0 + (k + f) dlam, with
// 0 <= k < n_src and 0 <= f <= 1 (the range's end maps to k = n_src - 1,
// f = 1; edges a rounding step outside the range are clamped onto it).
__device__ inline void locate(double l, double e0, double dlam, int n_src, int &k, double &f) {
  const double x = (l - e0) / dlam;
  const double kf = fmin(fmax(floor(x), 0.0), (double)(n_src - 1));
  k = (int)kf;
  f = fmin(fmax(x - kf, 0.0), 1.0);
}

// Grid: (ceil(n_out / 256), up to 1024 row groups); threads own one target
// pixel and loop over rows.
__global__ __launch_bounds__(256) void k_resample(const float *src, int n_rows, int n_src,
                                                  int64_t ld_src, double e0, double dlam,
                                                  float *out, int n_out, int64_t ld_out,
                                                  double lg0, double dlog10) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n_out) return;
  const double la = pow(10.0, lg0 + ((double)j - 0.5) * dlog10);
  const double lb = pow(10.0, lg0 + ((double)j + 0.5) * dlog10);
  int ka, kb;
  double fa, fb;
  locate(la, e0, dlam, n_src, ka, fa);
  locate(lb, e0, dlam, n_src, kb, fb);
  const double scale = dlam / (lb - la);
  for (int r = blockIdx.y; r < n_rows; r += gridDim.y) {
    const float *x = src + (size_t)r * ld_src;
    // (C(l_b) - C(l_a)) / dlam = sum_{ka <= i < kb} x_i + fb x_kb - fa x_ka
    double acc = fb * (double)x[kb] - fa * (double)x[ka];
    for (int i = ka; i < kb; ++i) acc += (double)x[i];
    out[(size_t)r * ld_out + j] = (float)(acc * scale);
  }
}

}  // namespace

hipError_t launch_resample(const float *src, int n_rows, int n_src, int64_t ld_src, double lam0,
                           double dlam, float *out, int n_out, int64_t ld_out, double lg0,
                           double dlog10, hipStream_t st) {
  if (n_rows == 0 || n_out == 0) return hipSuccess;
  const dim3 grid((n_out + 255) / 256, n_rows < 1024 ? n_rows : 1024);
  hipLaunchKernelGGL(k_resample, grid, dim3(256), 0, st, src, n_rows, n_src, ld_src,
                     lam0 - 0.5 * dlam, dlam, out, n_out, ld_out, lg0, dlog10);
  return hipGetLastError();
}

}  // namespace lasp
