// Interpolator contractions on the matrix cores (Eq. 1 read as a matrix
// product, F' = Phi(u) B, with B the [20 x (P+2M)] coefficient spectra) and
// the adjoint contraction Phi-bar = F-bar' B^T fused with the Adam update of
// Section 2.2 stage 8.
//
// v_mfma_f32_16x16x4f32 operand layout (wave64, one block):
//   A[i][k]: lane i + 16 k      B[k][j]: lane j + 16 k
//   D[i][j]: lane j + 16 (i / 4), register i % 4
#include "lasp_internal.h"

namespace lasp {
namespace {

constexpr int kFwdTiles = 8;  // 16-pixel tiles per wave in the forward GEMM

// Feature row t of spectrum s: t = 0 is phi(u), t = 1..3 is d phi / d u_t.
__device__ inline void feature_row(const float *u, int t, float *out) {
  const float x = u[0], y = u[1], z = u[2];
  if (t == 0) {
    features(x, y, z, out);
  } else {
    float d[3][kNB];
    feature_derivs(x, y, z, d);
#pragma unroll
    for (int k = 0; k < kNB; ++k) out[k] = d[t - 1][k];
  }
}

// F'[r][c] = sum_k Phi[r][k] basis[k][c] for r < rows (rows = B or 4B with
// derivative rows).  Grid: (ldF / (64 * kFwdTiles), ceil(rows / 16)).
__global__ __launch_bounds__(256) void k_interp_fwd(Geometry g, State s, int rows_per_spec) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rows = g.B * rows_per_spec;
  const int r0 = blockIdx.y * 16;
  const int my_row = r0 + (lane & 15);
  const int kq = lane >> 4;  // k offset inside a group of 4

  float bv[5];
  {
    float phi[kNB];
#pragma unroll
    for (int k = 0; k < kNB; ++k) phi[k] = 0.f;
    if (my_row < rows) {
      const int spec = my_row / rows_per_spec;
      const int t = my_row - spec * rows_per_spec;
      feature_row(s.u + (size_t)spec * kNP, t, phi);
    }
#pragma unroll
    for (int kk = 0; kk < 5; ++kk) bv[kk] = phi[4 * kk + kq];
  }

  const int cbase = (blockIdx.x * 4 + wave) * (16 * kFwdTiles);
  for (int n = 0; n < kFwdTiles; ++n) {
    const int c0 = cbase + 16 * n;
    if (c0 >= g.ldF) break;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 5; ++kk) {
      const float a = s.basis[(size_t)(4 * kk + kq) * g.ldF + c0 + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv[kk], acc, 0, 0, 0);
    }
    if (my_row < rows) {
      float4 *dst = reinterpret_cast<float4 *>(s.fp + (size_t)my_row * g.ldF + c0 + 4 * kq);
      *dst = make_float4(acc[0], acc[1], acc[2], acc[3]);
    }
  }
}

// Phi-bar[s][k] = sum_c F-bar'[s][c] basis[k][c], then the gradient of
// J = chi2/n_eff with respect to u and one Adam step (or, with grad_out,
// the gradient written out and no update).  One workgroup = 16 spectra; its
// four waves split the columns and combine through LDS.
__global__ __launch_bounds__(256) void k_interp_bwd(Geometry g, State s, AdamCfg adam,
                                                    int do_adam, float *grad_out) {
  __shared__ float red[4][16][32];
  __shared__ float pb[16][kNB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s0 = blockIdx.x * 16;
  const int i_row = lane & 15;   // spectrum within the tile (A rows) / basis row (B cols)
  const int kq = lane >> 4;
  const bool row_ok = s0 + i_row < g.B;
  const float *fb_row = s.fbar + (size_t)(s0 + i_row) * g.ldF;
  const float *b0_row = s.basis + (size_t)i_row * g.ldF;
  const bool b1_ok = i_row < kNB - 16;
  const float *b1_row = s.basis + (size_t)(16 + (b1_ok ? i_row : 0)) * g.ldF;

  floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  const int per_wave = ((g.ldF / 16 + 3) / 4) * 16;
  const int cb = wave * per_wave;
  const int ce = min(cb + per_wave, g.ldF);
  for (int c = cb; c < ce; c += 16) {
    const int cc = c + 4 * kq;
    float4 fa = make_float4(0.f, 0.f, 0.f, 0.f);
    if (row_ok) fa = *reinterpret_cast<const float4 *>(fb_row + cc);
    const float4 b0 = *reinterpret_cast<const float4 *>(b0_row + cc);
    float4 b1 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (b1_ok) b1 = *reinterpret_cast<const float4 *>(b1_row + cc);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.x, b0.x, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.x, b1.x, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.y, b0.y, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.y, b1.y, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.z, b0.z, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.z, b1.z, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.w, b0.w, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(fa.w, b1.w, acc1, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    red[wave][4 * kq + q][i_row] = acc0[q];
    red[wave][4 * kq + q][16 + i_row] = acc1[q];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * kNB; e += 256) {
    const int i = e / kNB, k = e - i * kNB;
    pb[i][k] = ((red[0][i][k] + red[1][i][k]) + red[2][i][k]) + red[3][i][k];
  }
  __syncthreads();

  const int t = threadIdx.x;
  if (t < 16 && s0 + t < g.B) {
    const int spec = s0 + t;
    float *u = s.u + (size_t)spec * kNP;
    float d[3][kNB];
    feature_derivs(u[0], u[1], u[2], d);
    float grad[kNP];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float acc = 0.f;
#pragma unroll
      for (int k = 1; k < kNB; ++k) acc = fmaf(pb[t][k], d[a][k], acc);
      grad[a] = acc;
    }
    grad[3] = s.g45[(size_t)spec * 2 + 0];
    grad[4] = s.g45[(size_t)spec * 2 + 1];
    if (grad_out) {
#pragma unroll
      for (int a = 0; a < kNP; ++a) grad_out[(size_t)spec * kNP + a] = grad[a];
    }
    if (do_adam) {
      const int step = s.t[spec] + 1;
      s.t[spec] = step;
      const float bc1 = 1.f - powf(adam.beta1, (float)step);
      const float bc2 = 1.f - powf(adam.beta2, (float)step);
      const float step_size = adam.lr / bc1;
      const float rbc2 = 1.f / sqrtf(bc2);
      float *m = s.m + (size_t)spec * kNP;
      float *v = s.v + (size_t)spec * kNP;
#pragma unroll
      for (int a = 0; a < kNP; ++a) {
        const float ga = grad[a];
        const float ma = adam.beta1 * m[a] + (1.f - adam.beta1) * ga;
        const float va = adam.beta2 * v[a] + (1.f - adam.beta2) * ga * ga;
        m[a] = ma;
        v[a] = va;
        const float denom = sqrtf(va) * rbc2 + adam.eps;
        u[a] = u[a] - step_size * (ma / denom);
      }
    }
  }
}

}  // namespace

hipError_t launch_interp_fwd(const Geometry &g, const State &s, int deriv_rows, int bf16x3,
                             hipStream_t st) {
  (void)bf16x3;
  const int rows_per_spec = deriv_rows ? 4 : 1;
  const int rows = g.B * rows_per_spec;
  const int cols_per_block = 4 * 16 * kFwdTiles;
  dim3 grid((g.ldF + cols_per_block - 1) / cols_per_block, (rows + 15) / 16);
  hipLaunchKernelGGL(k_interp_fwd, grid, dim3(256), 0, st, g, s, rows_per_spec);
  return hipGetLastError();
}

hipError_t launch_interp_bwd(const Geometry &g, const State &s, const AdamCfg *adam,
                             float *grad_out, hipStream_t st) {
  AdamCfg a = adam ? *adam : AdamCfg{0.f, 0.f, 0.f, 0.f};
  hipLaunchKernelGGL(k_interp_bwd, dim3((g.B + 15) / 16), dim3(256), 0, st, g, s, a,
                     adam ? 1 : 0, grad_out);
  return hipGetLastError();
}

}  // namespace lasp
