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

// Target pixel j spans the source positions ka + fa .. kb + fb; scale turns
// the sum over that span (in source pixels) into a mean over the target bin.
struct Span {
  int ka, kb;
  double fa, fb, scale;
};

__device__ inline Span span_of(int j, double e0, double dlam, int n_src, double lg0, double dlog10) {
  Span p;
  const double la = pow(10.0, lg0 + ((double)j - 0.5) * dlog10);
  const double lb = pow(10.0, lg0 + ((double)j + 0.5) * dlog10);
  locate(la, e0, dlam, n_src, p.ka, p.fa);
  locate(lb, e0, dlam, n_src, p.kb, p.fb);
  p.scale = dlam / (lb - la);
  return p;
}

// (C(l_b) - C(l_a)) / dlam = sum_{ka <= i < kb} x_i + fb x_kb - fa x_ka, as
// a mean over the bin; x is indexed from source pixel `base`.
__device__ inline float bin_mean(const Span &p, const float *x, int base) {
  double acc = p.fb * (double)x[p.kb - base] - p.fa * (double)x[p.ka - base];
  for (int i = p.ka; i < p.kb; ++i) acc += (double)x[i - base];
  return (float)(acc * p.scale);
}

// Tiled form: a block owns kRsThreads consecutive target pixels (one per
// thread) and loops over rows.  The pixel spans are computed once per block
// and kept in registers.  Per row, the source window of the block (at most
// KP * kRsThreads pixels) goes through registers into LDS with coalesced
// loads, and the bin sums are formed from LDS; the next row's window is
// loaded while this row's sums are formed.  A block whose window is wider
// than KP * kRsThreads (the host sizes KP from the widest block) reads the
// source from global memory instead.
// Grid: (ceil(n_out / kRsThreads), up to 1024 row groups).
constexpr int kRsThreads = 256;

template <int KP>
__global__ __launch_bounds__(kRsThreads) void k_resample_tiled(const float *src, int n_rows, int n_src,
                                                               int64_t ld_src, double e0, double dlam,
                                                               float *out, int n_out, int64_t ld_out,
                                                               double lg0, double dlog10) {
  __shared__ float win[KP * kRsThreads];
  __shared__ int w_lo, w_hi;
  const int t = threadIdx.x;
  const int j = blockIdx.x * kRsThreads + t;
  const bool has_j = j < n_out;
  const Span sp = span_of(has_j ? j : n_out - 1, e0, dlam, n_src, lg0, dlog10);
  // the block's window: the smallest ka to the largest kb of its pixels
  if (t == 0) {
    w_lo = n_src;
    w_hi = 0;
  }
  __syncthreads();
  atomicMin(&w_lo, sp.ka);
  atomicMax(&w_hi, sp.kb);
  __syncthreads();
  const int w0 = w_lo, nwin = w_hi - w_lo + 1;
  if (nwin > KP * kRsThreads) {  // block uniform
    for (int r = blockIdx.y; r < n_rows; r += gridDim.y)
      if (has_j) out[(size_t)r * ld_out + j] = bin_mean(sp, src + (size_t)r * ld_src, 0);
    return;
  }
  float pre[KP];
  auto fetch = [&](int r) {
    const float *x = src + (size_t)r * ld_src + w0;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int i = t + kRsThreads * k;
      pre[k] = i < nwin ? x[i] : 0.f;
    }
  };
  int r = blockIdx.y;
  if (r < n_rows) fetch(r);
  for (; r < n_rows; r += gridDim.y) {
#pragma unroll
    for (int k = 0; k < KP; ++k) win[t + kRsThreads * k] = pre[k];
    __syncthreads();
    if (r + (int)gridDim.y < n_rows) fetch(r + gridDim.y);  // in flight during the sums
    if (has_j) out[(size_t)r * ld_out + j] = bin_mean(sp, win, w0);
    __syncthreads();
  }
}

// Direct form, for spans too wide to stage: threads own one target pixel
// and loop over rows, reading the source from global memory.
// Grid: (ceil(n_out / 256), up to 1024 row groups).
__global__ __launch_bounds__(256) void k_resample(const float *src, int n_rows, int n_src,
                                                  int64_t ld_src, double e0, double dlam,
                                                  float *out, int n_out, int64_t ld_out,
                                                  double lg0, double dlog10) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n_out) return;
  const Span sp = span_of(j, e0, dlam, n_src, lg0, dlog10);
  for (int r = blockIdx.y; r < n_rows; r += gridDim.y)
    out[(size_t)r * ld_out + j] = bin_mean(sp, src + (size_t)r * ld_src, 0);
}

}  // namespace

// Source pixels of the widest block's window, from host arithmetic; two
// pixels of slack on each side cover a last-bit difference between the
// host's and the device's pow.
static int widest_window(int n_src, double e0, double dlam, int n_out, double lg0, double dlog10) {
  auto pos = [&](double edge) {
    const double l = pow(10.0, lg0 + edge * dlog10);
    const double x = floor((l - e0) / dlam);
    return (int)fmin(fmax(x, 0.0), (double)(n_src - 1));
  };
  int widest = 0;
  for (int j0 = 0; j0 < n_out; j0 += kRsThreads) {
    const int j1 = j0 + kRsThreads < n_out ? j0 + kRsThreads : n_out;
    const int w = pos((double)j1 - 0.5) - pos((double)j0 - 0.5) + 1;
    widest = w > widest ? w : widest;
  }
  return widest + 4;
}

hipError_t launch_resample(const float *src, int n_rows, int n_src, int64_t ld_src, double lam0,
                           double dlam, float *out, int n_out, int64_t ld_out, double lg0,
                           double dlog10, hipStream_t st) {
  if (n_rows == 0 || n_out == 0) return hipSuccess;
  const double e0 = lam0 - 0.5 * dlam;
  const int rows_y = n_rows < 1024 ? n_rows : 1024;
  const int nwin = widest_window(n_src, e0, dlam, n_out, lg0, dlog10);
  const dim3 tgrid((n_out + kRsThreads - 1) / kRsThreads, rows_y);
  if (nwin <= 8 * kRsThreads) {
    hipLaunchKernelGGL(k_resample_tiled<8>, tgrid, dim3(kRsThreads), 0, st, src, n_rows, n_src,
                       ld_src, e0, dlam, out, n_out, ld_out, lg0, dlog10);
  } else if (nwin <= 16 * kRsThreads) {
    hipLaunchKernelGGL(k_resample_tiled<16>, tgrid, dim3(kRsThreads), 0, st, src, n_rows, n_src,
                       ld_src, e0, dlam, out, n_out, ld_out, lg0, dlog10);
  } else if (nwin <= 32 * kRsThreads) {
    hipLaunchKernelGGL(k_resample_tiled<32>, tgrid, dim3(kRsThreads), 0, st, src, n_rows, n_src,
                       ld_src, e0, dlam, out, n_out, ld_out, lg0, dlog10);
  } else if (nwin <= 48 * kRsThreads) {
    hipLaunchKernelGGL(k_resample_tiled<48>, tgrid, dim3(kRsThreads), 0, st, src, n_rows, n_src,
                       ld_src, e0, dlam, out, n_out, ld_out, lg0, dlog10);
  } else {
    const dim3 grid((n_out + 255) / 256, rows_y);
    hipLaunchKernelGGL(k_resample, grid, dim3(256), 0, st, src, n_rows, n_src, ld_src, e0, dlam,
                       out, n_out, ld_out, lg0, dlog10);
  }
  return hipGetLastError();
}

}  // namespace lasp
