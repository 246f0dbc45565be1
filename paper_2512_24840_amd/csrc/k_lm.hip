// Levenberg-Marquardt polish of the grouped fit (the curvature step that the
// paper's Section 4.5, future improvements, proposes for the Adam stage): per
// spectrum, damped Gauss-Newton steps on the residual r = sqrt(W) (o - C F'') with the
// continuum profiled out.  The covariance kernel supplies the normal
// equations S du = q at the current u (S = Schur complement of the
// continuum block of J^T W J, q = Ju^T W e); a step solves
// (S + lambda diag(S)) du = q in FP64, the trial point is evaluated by the
// forward pass, and the step is kept when chi2 falls (lambda / 10) or
// dropped (lambda * 10), as in Marquardt's method.  Spectra run in lockstep
// but each has its own lambda, acceptance and stopping test.
#include "lasp_internal.h"

namespace lasp {
namespace {

constexpr int kLmBlock = 256;

// 5x5 symmetric positive definite solve (Cholesky, FP64); false if not SPD.
__device__ inline bool chol5(double (&a)[kNP][kNP], double (&x)[kNP]) {
#pragma unroll
  for (int j = 0; j < kNP; ++j) {
    double d = a[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= a[j][k] * a[j][k];
    if (!(d > 0.0) || !isfinite(d)) return false;
    const double l = sqrt(d);
    a[j][j] = l;
#pragma unroll
    for (int i = j + 1; i < kNP; ++i) {
      double v = a[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= a[i][k] * a[j][k];
      a[i][j] = v / l;
    }
  }
#pragma unroll
  for (int i = 0; i < kNP; ++i) {
    double v = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= a[i][k] * x[k];
    x[i] = v / a[i][i];
  }
#pragma unroll
  for (int i = kNP - 1; i >= 0; --i) {
    double v = x[i];
#pragma unroll
    for (int k = i + 1; k < kNP; ++k) v -= a[k][i] * x[k];
    x[i] = v / a[i][i];
  }
  return true;
}

__global__ void k_lm_init(Geometry g, LmState lm) {
  const int spec = blockIdx.x * blockDim.x + threadIdx.x;
  if (spec >= g.B) return;
  lm.lambda[spec] = 1e-3;
  lm.need_jac[spec] = 1;
  lm.flags[spec] = 0;
}

// Trial point u + du for every spectrum still iterating.
__global__ void k_lm_solve(Geometry g, State s, LmState lm) {
  const int spec = blockIdx.x * blockDim.x + threadIdx.x;
  if (spec >= g.B) return;
  float *ut = lm.u_trial + (size_t)spec * kNP;
  const float *u = s.u + (size_t)spec * kNP;
  if (lm.flags[spec] & kLmDone) {
#pragma unroll
    for (int t = 0; t < kNP; ++t) ut[t] = u[t];
    return;
  }
  const double *nrm = lm.normal + (size_t)spec * kNormalStride;
  const double lam = lm.lambda[spec];
  double a[kNP][kNP], x[kNP];
  double dmax = 0.0;
#pragma unroll
  for (int t = 0; t < kNP; ++t) dmax = fmax(dmax, nrm[t * kNP + t]);
#pragma unroll
  for (int i = 0; i < kNP; ++i) {
#pragma unroll
    for (int j = 0; j < kNP; ++j) a[i][j] = nrm[i * kNP + j];
    a[i][i] += lam * fmax(nrm[i * kNP + i], 1e-12 * dmax);
    x[i] = nrm[25 + i];
  }
  double dinf = 0.0;
  if (chol5(a, x)) {
    // predicted chi2 decrease of the Gauss-Newton model, du^T q: below the
    // tolerance there is nothing left to gain and the spectrum stops here
    double dec = 0.0;
#pragma unroll
    for (int t = 0; t < kNP; ++t) dec = fma(x[t], nrm[25 + t], dec);
    if (dec < kLmDecreaseTol) {
      lm.flags[spec] |= kLmDone;
#pragma unroll
      for (int t = 0; t < kNP; ++t) ut[t] = u[t];
      return;
    }
#pragma unroll
    for (int t = 0; t < kNP; ++t) {
      ut[t] = (float)((double)u[t] + x[t]);
      dinf = fmax(dinf, fabs(x[t]));
    }
  } else {
    dinf = NAN;  // no step: the accept kernel raises lambda
#pragma unroll
    for (int t = 0; t < kNP; ++t) ut[t] = u[t];
  }
  lm.step_inf[spec] = dinf;
}

// Keep or drop the trial step; stopping tests.
__global__ void k_lm_accept(Geometry g, State s, LmState lm, int last) {
  const int spec = blockIdx.x * blockDim.x + threadIdx.x;
  if (spec >= g.B) return;
  int fl = lm.flags[spec];
  if (fl & kLmDone) {
    lm.need_jac[spec] = 0;
    return;
  }
  const double c0 = lm.normal[(size_t)spec * kNormalStride + 30];
  const double c1 = lm.chi2_trial[spec];
  const double dinf = lm.step_inf[spec];
  double lam = lm.lambda[spec];
  bool done = false;
  if (isfinite(dinf) && isfinite(c1) && c1 < c0) {
#pragma unroll
    for (int t = 0; t < kNP; ++t) s.u[(size_t)spec * kNP + t] = lm.u_trial[(size_t)spec * kNP + t];
    lam = fmax(lam * 0.1, 1e-15);
    lm.need_jac[spec] = 1;
    done = (c0 - c1) <= kLmDropTol * c0 || dinf <= kLmStepTol;
  } else {
    lam *= 10.0;
    lm.need_jac[spec] = 0;
    done = lam > kLmLambdaMax || (isfinite(dinf) && dinf <= kLmStepTol) || !isfinite(c0);
  }
  lm.lambda[spec] = lam;
  if (done) {
    fl |= kLmDone;
    lm.need_jac[spec] = 0;
  } else if (last) {
    s.status[spec] |= kStPolishLimit;
  }
  lm.flags[spec] = fl;
}

// Number of spectra whose polish has not stopped, into *lm.active (one
// workgroup; the host reads it to stop enqueuing iterations).
__global__ __launch_bounds__(1024) void k_lm_active(Geometry g, LmState lm) {
  __shared__ int part[16];
  int n = 0;
  for (int i = threadIdx.x; i < g.B; i += 1024) n += (lm.flags[i] & kLmDone) ? 0 : 1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n += __shfl_down(n, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += part[w];
    *lm.active = t;
  }
}

}  // namespace

hipError_t launch_lm_active(const Geometry &g, const LmState &lm, hipStream_t st) {
  hipLaunchKernelGGL(k_lm_active, dim3(1), dim3(1024), 0, st, g, lm);
  return hipGetLastError();
}

hipError_t launch_lm_init(const Geometry &g, const LmState &lm, hipStream_t st) {
  hipLaunchKernelGGL(k_lm_init, dim3((g.B + kLmBlock - 1) / kLmBlock), dim3(kLmBlock), 0, st, g,
                     lm);
  return hipGetLastError();
}

hipError_t launch_lm_solve(const Geometry &g, const State &s, const LmState &lm, hipStream_t st) {
  hipLaunchKernelGGL(k_lm_solve, dim3((g.B + kLmBlock - 1) / kLmBlock), dim3(kLmBlock), 0, st, g,
                     s, lm);
  return hipGetLastError();
}

hipError_t launch_lm_accept(const Geometry &g, const State &s, const LmState &lm, int last,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_lm_accept, dim3((g.B + kLmBlock - 1) / kLmBlock), dim3(kLmBlock), 0, st, g,
                     s, lm, last);
  return hipGetLastError();
}

}  // namespace lasp
