// Interpolator contractions on the matrix cores (Eq. 1 read as a matrix
// product, F' = Phi(u) B, with B the [20 x (P+2M)] coefficient spectra) and
// the adjoint contraction Phi-bar = F-bar' B^T fused with the Adam update of
// Section 2.2 stage 8.
//
// v_mfma_f32_16x16x4f32 operand layout (wave64, one block):
//   A[i][k]: lane i + 16 k      B[k][j]: lane j + 16 k
//   D[i][j]: lane j + 16 (i / 4), register i % 4
// v_mfma_f32_16x16x32_bf16: lane l supplies row i = l % 16 of A (column
// j = l % 16 of B) with eight k values; A and B use the same k assignment,
// so the sum over k does not depend on which eight each lane carries.
//
// BF16x3: x = x_hi + x_lo with x_hi = bf16(x), x_lo = bf16(x - x_hi); a
// product is a_hi b_hi + a_hi b_lo + a_lo b_hi (the dropped a_lo b_lo is
// 2^-16 relative), accumulated in FP32.  In the forward contraction the
// constant monomial's row (phi_0 = 1) is added in FP32 exactly and only
// rows 1..19 go through BF16x3.
#include "lasp_internal.h"

namespace lasp {
namespace {

constexpr int kFwdTiles = 8;  // 16-pixel tiles per wave in the forward GEMM

template <int V>
struct IntC {
  static constexpr int value = V;
};

// Feature row t of spectrum s: t = 0 is phi(u), t = 1..3 is d phi / d u_t.
__device__ inline void feature_row(const float *u, int t, float *out) {
  const float x = u[0], y = u[1], z = u[2];
  if (t == 0) {
    features(x, y, z, out);
  } else {
    float d[3][kNB];
    feature_derivs(x, y, z, d);
    // selects, not an indexed load: keeps d in registers
#pragma unroll
    for (int k = 0; k < kNB; ++k) out[k] = t == 1 ? d[0][k] : (t == 2 ? d[1][k] : d[2][k]);
  }
}

// The same row over the three emulator classes: entry 20 q + k is
// w_q phi_k, and its derivative rows carry d w_q / d u1 phi_k as well.
__device__ inline void feature_row_classes(const Geometry &g, const float *u, int t, float *out) {
  const float x = u[0], y = u[1], z = u[2];
  float phi[kNB], r[kNB], d[3][kNB];
  features(x, y, z, phi);
  feature_derivs(x, y, z, d);
#pragma unroll
  for (int k = 0; k < kNB; ++k)
    r[k] = t == 0 ? phi[k] : (t == 1 ? d[0][k] : (t == 2 ? d[1][k] : d[2][k]));
  float w[kMaxClasses], dw[kMaxClasses];
  class_weights(g, x, w, dw);
#pragma unroll
  for (int q = 0; q < kMaxClasses; ++q)
#pragma unroll
    for (int k = 0; k < kNB; ++k)
      out[kNB * q + k] = t == 1 ? fmaf(dw[q], phi[k], w[q] * r[k]) : w[q] * r[k];
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort8 __attribute__((ext_vector_type(8)));

// Round to nearest even (finite inputs).
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline void split8(const float *x, bf16x8 &hi, bf16x8 &lo) {
  ushort8 h, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint16_t a = f2bf(x[e]);
    h[e] = a;
    l[e] = f2bf(x[e] - bf2f(a));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  lo = __builtin_bit_cast(bf16x8, l);
}

// hi/lo copies of the padded basis: [20][ldF] for the adjoint contraction and
// [ldF][32] (k-major, rows 1..19, zeros elsewhere) for the forward one.
__global__ void k_split_basis(Geometry g, State s) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ldF) return;
#pragma unroll 1
  for (int k = 0; k < 32; ++k) {
    uint16_t hi = 0, lo = 0;
    if (k < kNB) {
      const float x = s.basis[(size_t)k * g.ldF + c];
      hi = f2bf(x);
      lo = f2bf(x - bf2f(hi));
      s.basis_hi[(size_t)k * g.ldF + c] = hi;
      s.basis_lo[(size_t)k * g.ldF + c] = lo;
    }
    const bool fwd = k >= 1 && k < kNB;
    s.basis_thi[(size_t)c * 32 + k] = fwd ? hi : 0;
    s.basis_tlo[(size_t)c * 32 + k] = fwd ? lo : 0;
  }
}

// Output staging of the forward contraction: a workgroup's 16 rows x 512
// columns pass through LDS so that each row leaves as contiguous 1 KB runs
// (the MFMA result layout alone gives 64-byte pieces of 16 rows).
constexpr int kFwdCols = 4 * 16 * kFwdTiles;  // columns per workgroup
constexpr int kFwdLd = kFwdCols + 4;           // LDS row stride (floats)

__device__ inline void fwd_stage(float *sT, int wave, int lane, int n, const floatx4 &v) {
  const int j = lane & 15, kq = lane >> 4;
  *reinterpret_cast<float4 *>(sT + j * kFwdLd + wave * 16 * kFwdTiles + 16 * n + 4 * kq) =
      make_float4(v[0], v[1], v[2], v[3]);
}

// F' rows of the block's 16 launch rows r0 + j: row r (entry r / rps of the
// work list, derivative row r % rps) lands in F' row spec * rps + r % rps.
// Threads 0..15 write dst; a barrier must follow before fwd_store.
__device__ inline void fwd_dst_rows(const State &s, int r0, int rows, int rps, int *dst) {
  const int j = threadIdx.x;
  if (j >= 16 || r0 + j >= rows) return;
  const int r = r0 + j;
  if (!s.order) {
    dst[j] = r;  // no work list: rows in place
  } else {
    const int e = r / rps;
    dst[j] = s.order[e] * rps + (r - e * rps);
  }
}

__device__ inline void fwd_store(const Geometry &g, const State &s, const float *sT,
                                 const int *dst, int r0, int rows) {
  const int c_base = blockIdx.x * kFwdCols;
#pragma unroll
  for (int q = 0; q < 16 * kFwdCols / 4 / 256; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int r = e / (kFwdCols / 4), c4 = e - r * (kFwdCols / 4);
    const int col = c_base + 4 * c4;
    if (r0 + r < rows && col < g.ldF)
      *reinterpret_cast<float4 *>(s.fp + (size_t)dst[r] * g.ldF + col) =
          *reinterpret_cast<const float4 *>(sT + r * kFwdLd + 4 * c4);
  }
}

// BF16x3 variant of k_interp_fwd (same grid and output layout).
__global__ __launch_bounds__(256) void k_interp_fwd_bf16(Geometry g, State s, int rows_per_spec, int skip_done) {
  __shared__ __align__(16) float sT[16 * kFwdLd];
  __shared__ int dst[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rows = work_count(g, s) * rows_per_spec;
  const int r0 = blockIdx.y * 16;
  if (r0 >= rows) return;  // past the work list (uniform over the block)
  const int my_row = r0 + (lane & 15);
  const int kq = lane >> 4;
  if (skip_done && s.target) {
    bool any = false;
    for (int r = 0; r < 16; ++r) {
      const int row = r0 + r;
      any = any || (row < rows && slot_active(s, work_spec(s, row / rows_per_spec)));
    }
    if (!any) return;
  }
  fwd_dst_rows(s, r0, rows, rows_per_spec, dst);
  bf16x8 b_hi, b_lo;
  float phi0 = 0.f;
  {
    float phi[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) phi[k] = 0.f;
    if (my_row < rows) {
      const int e = my_row / rows_per_spec;
      const int t = my_row - e * rows_per_spec;
      feature_row(s.u + (size_t)work_spec(s, e) * kNP, t, phi);
    }
    phi0 = phi[0];
    phi[0] = 0.f;  // constant row added in FP32 below
    float sel[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float v = phi[e];
#pragma unroll
      for (int q = 1; q < 4; ++q)
        if (kq == q) v = phi[8 * q + e];
      sel[e] = v;
    }
    split8(sel, b_hi, b_lo);
  }
  // phi_0 of the spectrum whose outputs this lane holds (column j = lane % 16)
  const int cbase = (blockIdx.x * 4 + wave) * (16 * kFwdTiles);
  for (int n = 0; n < kFwdTiles; ++n) {
    const int c0 = cbase + 16 * n;
    if (c0 >= g.ldF) break;
    const uint16_t *ah = s.basis_thi + (size_t)(c0 + (lane & 15)) * 32 + 8 * kq;
    const uint16_t *al = s.basis_tlo + (size_t)(c0 + (lane & 15)) * 32 + 8 * kq;
    const bf16x8 a_hi = __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushort8 *>(ah));
    const bf16x8 a_lo = __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushort8 *>(al));
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_lo, b_hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, b_lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, b_hi, acc, 0, 0, 0);
    const float4 b0 = *reinterpret_cast<const float4 *>(s.basis + c0 + 4 * kq);
    floatx4 out = {fmaf(phi0, b0.x, acc[0]), fmaf(phi0, b0.y, acc[1]), fmaf(phi0, b0.z, acc[2]),
                   fmaf(phi0, b0.w, acc[3])};
    fwd_stage(sT, wave, lane, n, out);
  }
  __syncthreads();
  fwd_store(g, s, sT, dst, r0, rows);
}

// F'[r][c] = sum_k Phi[r][k] basis[k][c] for r < rows (rows = B or 4B with
// derivative rows), k < NB (20, or 60 over three emulator classes).
// Grid: (ldF / (64 * kFwdTiles), ceil(rows / 16)).
template <int NB>
__global__ __launch_bounds__(256) void k_interp_fwd(Geometry g, State s, int rows_per_spec, int skip_done) {
  __shared__ __align__(16) float sT[16 * kFwdLd];
  __shared__ int dst[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rows = work_count(g, s) * rows_per_spec;
  const int r0 = blockIdx.y * 16;
  if (r0 >= rows) return;  // past the work list (uniform over the block)
  const int my_row = r0 + (lane & 15);
  const int kq = lane >> 4;  // k offset inside a group of 4
  if (skip_done && s.target) {
    bool any = false;
    for (int r = 0; r < 16; ++r) {
      const int row = r0 + r;
      any = any || (row < rows && slot_active(s, work_spec(s, row / rows_per_spec)));
    }
    if (!any) return;
  }
  fwd_dst_rows(s, r0, rows, rows_per_spec, dst);

  float bv[NB / 4];
  {
    float phi[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) phi[k] = 0.f;
    if (my_row < rows) {
      const int e = my_row / rows_per_spec;
      const int t = my_row - e * rows_per_spec;
      const float *ur = s.u + (size_t)work_spec(s, e) * kNP;
      if (NB == kNB)
        feature_row(ur, t, phi);
      else
        feature_row_classes(g, ur, t, phi);
    }
    // selects, not an indexed load: keeps phi in registers
#pragma unroll
    for (int kk = 0; kk < NB / 4; ++kk)
      bv[kk] = kq == 0 ? phi[4 * kk] : (kq == 1 ? phi[4 * kk + 1] : (kq == 2 ? phi[4 * kk + 2] : phi[4 * kk + 3]));
  }
  const int cbase = (blockIdx.x * 4 + wave) * (16 * kFwdTiles);
  // products over feature groups KK0 .. KK0 + NKK - 1 (4 features each)
  auto run = [&](auto kk0, auto nkk) {
    constexpr int KK0 = decltype(kk0)::value, NKK = decltype(nkk)::value;
    for (int n = 0; n < kFwdTiles; ++n) {
      const int c0 = cbase + 16 * n;
      if (c0 >= g.ldF) break;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = KK0; kk < KK0 + NKK; ++kk) {
        const float a = s.basis[(size_t)(4 * kk + kq) * g.ldF + c0 + (lane & 15)];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv[kk], acc, 0, 0, 0);
      }
      fwd_stage(sT, wave, lane, n, acc);
    }
  };
  if constexpr (NB == kNB) {
    run(IntC<0>{}, IntC<NB / 4>{});
  } else {
    // an emulator class whose weight and weight derivative are zero in all
    // 16 rows of the tile (spectra of other Teff regimes) has an all-zero
    // feature block; its products would add exact zeros and are left out
    int mask = 0;
#pragma unroll
    for (int q = 0; q < kMaxClasses; ++q) {
      bool nz = false;
#pragma unroll
      for (int kk = 5 * q; kk < 5 * q + 5; ++kk) nz = nz || bv[kk] != 0.f;
      mask |= (__ballot(nz) != 0) << q;
    }
    switch (mask) {  // wave uniform; every wave of the block sees the same rows
      case 1: run(IntC<0>{}, IntC<5>{}); break;
      case 2: run(IntC<5>{}, IntC<5>{}); break;
      case 4: run(IntC<10>{}, IntC<5>{}); break;
      case 3: run(IntC<0>{}, IntC<10>{}); break;
      case 6: run(IntC<5>{}, IntC<10>{}); break;
      default: run(IntC<0>{}, IntC<15>{}); break;
    }
  }
  __syncthreads();
  fwd_store(g, s, sT, dst, r0, rows);
}

// Gradient of J with respect to u from Phi-bar (pb, NB entries) and the
// fused pass's dJ/du4, dJ/du5, then the stopping rules and one Adam step of
// spectrum spec (or the gradient written out).
template <int NB>
__device__ inline void bwd_epilogue(const Geometry &g, const State &s, const AdamCfg &adam,
                                    int do_adam, float *grad_out, int spec, const float *pb) {
  float *u = s.u + (size_t)spec * kNP;
  float d[3][kNB];
  feature_derivs(u[0], u[1], u[2], d);
  float grad[kNP];
  if constexpr (NB == kNB) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float acc = 0.f;
#pragma unroll
      for (int k = 1; k < kNB; ++k) acc = fmaf(pb[k], d[a][k], acc);
      grad[a] = acc;
    }
  } else {
    // d (sum_q w_q phi . Phi-bar_q) / d u_a: the class weights depend on u1
    float phi[kNB], w[kMaxClasses], dw[kMaxClasses];
    features(u[0], u[1], u[2], phi);
    class_weights(g, u[0], w, dw);
#pragma unroll
    for (int a = 0; a < 3; ++a) grad[a] = 0.f;
#pragma unroll
    for (int q = 0; q < kMaxClasses; ++q) {
      const float *pq = &pb[kNB * q];
      float sp = 0.f, sd0 = 0.f, sd1 = 0.f, sd2 = 0.f;
#pragma unroll
      for (int k = 0; k < kNB; ++k) {
        sp = fmaf(pq[k], phi[k], sp);
        sd0 = fmaf(pq[k], d[0][k], sd0);
        sd1 = fmaf(pq[k], d[1][k], sd1);
        sd2 = fmaf(pq[k], d[2][k], sd2);
      }
      grad[0] = fmaf(dw[q], sp, fmaf(w[q], sd0, grad[0]));
      grad[1] = fmaf(w[q], sd1, grad[1]);
      grad[2] = fmaf(w[q], sd2, grad[2]);
    }
  }
  grad[3] = s.g45[(size_t)spec * 2 + 0];
  grad[4] = s.g45[(size_t)spec * 2 + 1];
  if (grad_out) {
#pragma unroll
    for (int a = 0; a < kNP; ++a) grad_out[(size_t)spec * kNP + a] = grad[a];
  }
  bool take = do_adam && slot_active(s, spec);
  if (take && adam.stop_window > 0) {
    // stopping rules of stage 8 on ell_t = sqrt(chi2 / n_eff) after t steps:
    // a change below stop_tol over the last W steps, or a rise at each of
    // them (the ring holds ell of the last W step counts)
    const int t0 = s.t[spec], W = adam.stop_window;
    const int n = s.neff[spec];
    const double ell = n > 0 ? sqrt(s.chi2[spec] / (double)n) : 0.0;
    double *h = s.lhist + (size_t)spec * W;
    int rise = s.nrise[spec];
    if (t0 >= 1) rise = ell > h[(t0 - 1) % W] ? rise + 1 : 0;
    uint32_t bit = 0;
    if (t0 >= W && fabs(h[t0 % W] - ell) < (double)adam.stop_tol)
      bit = kStStopFlat;
    else if (rise >= W)
      bit = kStStopRising;
    s.nrise[spec] = rise;
    h[t0 % W] = ell;
    if (bit) {
      s.target[spec] = t0;
      s.status[spec] |= bit;
      take = false;
    }
  }
  if (take) {
    const int step = s.t[spec] + 1;
    s.t[spec] = step;
    if (adam.stop_window > 0 && step >= s.target[spec]) s.status[spec] |= kStNotConverged;
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

// BF16x3 variant of the adjoint contraction (one emulator class): one
// workgroup = 16 spectra; its four waves split the columns and combine
// through LDS.
__global__ __launch_bounds__(256) void k_interp_bwd_bf16(Geometry g, State s, AdamCfg adam,
                                                         int do_adam, float *grad_out) {
  constexpr int NB = kNB;
  constexpr int NG = 2;
  __shared__ float red[4][16][16 * NG];
  __shared__ float pb[16][NB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s0 = blockIdx.x * 16;
  const int count = work_count(g, s);
  if (s0 >= count) return;  // past the work list (uniform over the block)
  const int i_row = lane & 15;   // spectrum within the tile (A rows) / basis row (B cols)
  const int kq = lane >> 4;
  const bool row_ok = s0 + i_row < count;
  const float *fb_row = s.fbar + (size_t)work_spec(s, row_ok ? s0 + i_row : s0) * g.ldF;
  bool b_ok[NG];
  int b_row[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    b_ok[q] = 16 * q + i_row < NB;
    b_row[q] = 16 * q + (b_ok[q] ? i_row : 0);
  }
  if (s.target) {  // the whole tile finished: nothing to do (uniform over the block)
    bool any = false;
    for (int r = 0; r < 16; ++r) any = any || (s0 + r < count && slot_active(s, work_spec(s, s0 + r)));
    if (!any) return;
  }

  floatx4 acc[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int per_wave = g.ldF / 4;  // ldF is a multiple of 128
  const int cb = wave * per_wave;
  const int ce = cb + per_wave;
  const uint16_t *h0 = s.basis_hi + (size_t)b_row[0] * g.ldF;
  const uint16_t *l0 = s.basis_lo + (size_t)b_row[0] * g.ldF;
  const uint16_t *h1 = s.basis_hi + (size_t)b_row[1] * g.ldF;
  const uint16_t *l1 = s.basis_lo + (size_t)b_row[1] * g.ldF;
  const bf16x8 zero = __builtin_bit_cast(bf16x8, ushort8{0, 0, 0, 0, 0, 0, 0, 0});
  for (int c = cb; c < ce; c += 32) {
    const int cc = c + 8 * kq;
    float fa[8];
    if (row_ok) {
      const float4 x0 = *reinterpret_cast<const float4 *>(fb_row + cc);
      const float4 x1 = *reinterpret_cast<const float4 *>(fb_row + cc + 4);
      fa[0] = x0.x; fa[1] = x0.y; fa[2] = x0.z; fa[3] = x0.w;
      fa[4] = x1.x; fa[5] = x1.y; fa[6] = x1.z; fa[7] = x1.w;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) fa[e] = 0.f;
    }
    bf16x8 a_hi, a_lo;
    split8(fa, a_hi, a_lo);
    const bf16x8 bh0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushort8 *>(h0 + cc));
    const bf16x8 bl0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushort8 *>(l0 + cc));
    bf16x8 bh1 = zero, bl1 = zero;
    if (b_ok[1]) {
      bh1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushort8 *>(h1 + cc));
      bl1 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushort8 *>(l1 + cc));
    }
    acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_lo, bh0, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_lo, bh1, acc[1], 0, 0, 0);
    acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, bl0, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, bl1, acc[1], 0, 0, 0);
    acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, bh0, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, bh1, acc[1], 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) red[wave][4 * kq + q][16 * gi + i_row] = acc[gi][q];
  __syncthreads();
  for (int e = threadIdx.x; e < 16 * NB; e += 256) {
    const int i = e / NB, k = e - i * NB;
    pb[i][k] = ((red[0][i][k] + red[1][i][k]) + red[2][i][k]) + red[3][i][k];
  }
  __syncthreads();

  const int t = threadIdx.x;
  if (t < 16 && s0 + t < count)
    bwd_epilogue<NB>(g, s, adam, do_adam, grad_out, work_spec(s, s0 + t), pb[t]);
}

// Phi-bar[s][k] = sum_c F-bar'[s][c] basis[k][c], then the gradient of
// J = chi2/n_eff with respect to u and one Adam step (or, with grad_out,
// the gradient written out and no update).  One workgroup = 32 spectra in
// two 16-row tiles; each of its eight waves covers ldF / 8 columns for both
// tiles, so one basis load feeds both, and the waves combine through LDS in
// a fixed order.  Basis rows go in groups of 16 (NG = 2 groups for 20 rows,
// 4 for 60); the loads of rows past NB are skipped and count as zero.
template <int NB>
__global__ __launch_bounds__(512) void k_interp_bwd(Geometry g, State s, AdamCfg adam,
                                                      int do_adam, float *grad_out) {
  constexpr int NG = (NB + 15) / 16;
  constexpr int NWV = 8;
  constexpr int kSLd = 36;                        // staging row stride (floats)
  constexpr int kStage = 36 * kSLd;               // one wave's [32 + 4 rows][32 columns]
  constexpr int kRed = 32 * 16 * NG;              // one wave's partial sums
  constexpr int kBuf = NWV * (kStage > kRed ? kStage : kRed);
  __shared__ __align__(16) float sbuf[kBuf];      // staging, then the partial sums
  __shared__ float pb[32][NB];
  auto red = reinterpret_cast<float (*)[32][16 * NG]>(sbuf);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s0 = blockIdx.x * 32;
  const int count = work_count(g, s);
  if (s0 >= count) return;  // past the work list (uniform over the block)
  const int i_row = lane & 15;
  const int kq = lane >> 4;
  bool row_ok[2];
  const float *fb_row[2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    row_ok[rt] = s0 + 16 * rt + i_row < count;
    fb_row[rt] = s.fbar + (size_t)work_spec(s, row_ok[rt] ? s0 + 16 * rt + i_row : s0) * g.ldF;
  }
  bool b_ok[NG];
  const float *b_ptr[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    b_ok[q] = 16 * q + i_row < NB;
    b_ptr[q] = s.basis + (size_t)(16 * q + (b_ok[q] ? i_row : 0)) * g.ldF;
  }
  if (s.target) {
    bool any = false;
    for (int r = 0; r < 32; ++r) any = any || (s0 + r < count && slot_active(s, work_spec(s, s0 + r)));
    if (!any) return;
  }
  floatx4 acc[2][NG];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int q = 0; q < NG; ++q) acc[rt][q] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int per_wave = g.ldF / NWV;  // ldF is a multiple of 128
  const int cb = wave * per_wave, ce = cb + per_wave;
  constexpr int kU = 2;  // 16-column MFMA blocks per stage
  // groups Q0 .. Q1 - 1 of 16 basis rows
  auto step = [&](auto q0, auto q1, const float4 (&fa)[2], const float4 (&bv)[NG]) {
    constexpr int Q0 = decltype(q0)::value, Q1 = decltype(q1)::value;
    float4 a[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) a[rt] = row_ok[rt] ? fa[rt] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int q = Q0; q < Q1; ++q) acc[rt][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt].x, bv[q].x, acc[rt][q], 0, 0, 0);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int q = Q0; q < Q1; ++q) acc[rt][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt].y, bv[q].y, acc[rt][q], 0, 0, 0);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int q = Q0; q < Q1; ++q) acc[rt][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt].z, bv[q].z, acc[rt][q], 0, 0, 0);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int q = Q0; q < Q1; ++q) acc[rt][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt].w, bv[q].w, acc[rt][q], 0, 0, 0);
  };
  auto load = [&](auto q0, auto q1, int cc, float4 (&fa)[2], float4 (&bv)[NG]) {
    constexpr int Q0 = decltype(q0)::value, Q1 = decltype(q1)::value;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) fa[rt] = *reinterpret_cast<const float4 *>(fb_row[rt] + cc);
#pragma unroll
    for (int q = Q0; q < Q1; ++q) {
      if (16 * q + 16 <= NB || b_ok[q])
        bv[q] = *reinterpret_cast<const float4 *>(b_ptr[q] + cc);
      else
        bv[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  // F-bar' goes through this wave's LDS stage, 32 rows x 32 columns at a
  // time, read with row-contiguous loads (128-byte runs per row); the MFMA
  // operands (16 rows x 4 columns per lane group) come from LDS.  The next
  // stage's F-bar' and basis loads are in flight during this stage's
  // products.
  float *stg = sbuf + wave * kStage;
  const float *rp[4];
  bool rv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int ri = 8 * j + (lane >> 3);
    rv[j] = s0 + ri < count;
    rp[j] = s.fbar + (size_t)work_spec(s, rv[j] ? s0 + ri : s0) * g.ldF + 4 * (lane & 7);
  }
  auto run = [&](auto q0, auto q1) {
    auto fetch = [&](int cc, float4 (&fv)[4], float4 (&bv)[kU][NG]) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        fv[j] = rv[j] ? *reinterpret_cast<const float4 *>(rp[j] + cc) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        float4 dummy[2];
        load(q0, q1, cc + 16 * u + 4 * kq, dummy, bv[u]);
      }
    };
    int c = cb;
    if (c + 16 * kU <= ce) {
      float4 fv[4], bv[kU][NG];
      fetch(c, fv, bv);
      for (; c + 16 * kU <= ce; c += 16 * kU) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          *reinterpret_cast<float4 *>(stg + (8 * j + (lane >> 3)) * kSLd + 4 * (lane & 7)) = fv[j];
        float4 bcur[kU][NG];
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
          for (int q = 0; q < NG; ++q) bcur[u][q] = bv[u][q];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (c + 32 * kU <= ce) fetch(c + 16 * kU, fv, bv);  // next stage
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          float4 fa[2];
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
            fa[rt] = *reinterpret_cast<const float4 *>(stg + (16 * rt + i_row) * kSLd + 16 * u + 4 * kq);
          step(q0, q1, fa, bcur[u]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    for (; c < ce; c += 16) {
      float4 fa[2], bv[NG];
      load(q0, q1, c + 4 * kq, fa, bv);
      step(q0, q1, fa, bv);
    }
  };
  floatx4 acc4 = {0.f, 0.f, 0.f, 0.f};
  if constexpr (NB == kNB) {
    // Basis rows 0-15 as one 16-row group of 16x16x4 products; rows 16-19
    // as sixteen 4x4x1 blocks, no zero rows: block b = g + 8 h (lanes 4b ..
    // 4b + 3) takes spectra 4g .. 4g + 3 and the h-th 16 columns of each
    // 32-column stage, so lane l supplies F-bar' of spectrum l & 31 and
    // basis row 16 + (l & 3), and accumulates spectra 4g + r x row 16 + (l & 3).
    const int hh = lane >> 5, r4 = lane & 31, j4 = lane & 3;
    const float *b4 = s.basis + (size_t)(16 + j4) * g.ldF;
    const float *fb4row = s.fbar + (size_t)work_spec(s, s0 + r4 < count ? s0 + r4 : s0) * g.ldF;
    float *stg = sbuf + wave * kStage;
    const float *rp[4];
    bool rv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int ri = 8 * j + (lane >> 3);
      rv[j] = s0 + ri < count;
      rp[j] = s.fbar + (size_t)work_spec(s, rv[j] ? s0 + ri : s0) * g.ldF + 4 * (lane & 7);
    }
    // lanes 0-31 stage basis rows 16-19 of the stage (row 32 + (lane >> 3))
    const float *bs = s.basis + (size_t)(16 + ((lane >> 3) & 3)) * g.ldF + 4 * (lane & 7);
    int c = cb;
    if (c + 32 <= ce) {
      float4 fv[4], fs, bv[kU];
      auto fetch = [&](int cc) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          fv[j] = rv[j] ? *reinterpret_cast<const float4 *>(rp[j] + cc) : make_float4(0.f, 0.f, 0.f, 0.f);
        fs = lane < 32 ? *reinterpret_cast<const float4 *>(bs + cc) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < kU; ++u) bv[u] = *reinterpret_cast<const float4 *>(b_ptr[0] + cc + 16 * u + 4 * kq);
      };
      fetch(c);
      for (; c + 32 <= ce; c += 32) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          *reinterpret_cast<float4 *>(stg + (8 * j + (lane >> 3)) * kSLd + 4 * (lane & 7)) = fv[j];
        if (lane < 32) *reinterpret_cast<float4 *>(stg + (32 + (lane >> 3)) * kSLd + 4 * (lane & 7)) = fs;
        float4 bcur[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) bcur[u] = bv[u];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (c + 64 <= ce) fetch(c + 32);  // next stage
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          float4 fa[2], b16[NG];
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
            fa[rt] = *reinterpret_cast<const float4 *>(stg + (16 * rt + i_row) * kSLd + 16 * u + 4 * kq);
          b16[0] = bcur[u];
          step(IntC<0>{}, IntC<1>{}, fa, b16);
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const float4 a4 = *reinterpret_cast<const float4 *>(stg + r4 * kSLd + 16 * hh + 4 * qq);
          const float4 w4 = *reinterpret_cast<const float4 *>(stg + (32 + j4) * kSLd + 16 * hh + 4 * qq);
          acc4 = __builtin_amdgcn_mfma_f32_4x4x1f32(a4.x, w4.x, acc4, 0, 0, 0);
          acc4 = __builtin_amdgcn_mfma_f32_4x4x1f32(a4.y, w4.y, acc4, 0, 0, 0);
          acc4 = __builtin_amdgcn_mfma_f32_4x4x1f32(a4.z, w4.z, acc4, 0, 0, 0);
          acc4 = __builtin_amdgcn_mfma_f32_4x4x1f32(a4.w, w4.w, acc4, 0, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    for (; c < ce; c += 16) {  // a 16-column tail: lanes of half 1 add zeros
      float4 fa[2], bv[NG];
      load(IntC<0>{}, IntC<1>{}, c + 4 * kq, fa, bv);
      step(IntC<0>{}, IntC<1>{}, fa, bv);
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        float4 a4 = *reinterpret_cast<const float4 *>(fb4row + c + 4 * qq);
        const float4 w4 = *reinterpret_cast<const float4 *>(b4 + c + 4 * qq);
        if (hh) a4 = make_float4(0.f, 0.f, 0.f, 0.f);
        acc4 = __builtin_amdgcn_mfma_f32_4x4x1f32(a4.x, w4.x, acc4, 0, 0, 0);
        acc4 = __builtin_amdgcn_mfma_f32_4x4x1f32(a4.y, w4.y, acc4, 0, 0, 0);
        acc4 = __builtin_amdgcn_mfma_f32_4x4x1f32(a4.z, w4.z, acc4, 0, 0, 0);
        acc4 = __builtin_amdgcn_mfma_f32_4x4x1f32(a4.w, w4.w, acc4, 0, 0, 0);
      }
    }
  } else {
    // an emulator class with zero weight and weight derivative for all 32
    // spectra (other Teff regimes) only ever multiplies its rows of
    // Phi-bar by zero: the 16-row groups that hold no other class's rows
    // are left out (classes are rows 0-19, 20-39, 40-59; groups 0-15,
    // 16-31, 32-47, 48-63)
    bool nz[kMaxClasses] = {false, false, false};
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      if (row_ok[rt]) {
        float w[kMaxClasses], dw[kMaxClasses];
        class_weights(g, s.u[(size_t)work_spec(s, s0 + 16 * rt + i_row) * kNP], w, dw);
#pragma unroll
        for (int q = 0; q < kMaxClasses; ++q) nz[q] = nz[q] || w[q] != 0.f || dw[q] != 0.f;
      }
    }
    int mask = 0;
#pragma unroll
    for (int q = 0; q < kMaxClasses; ++q) mask |= (__ballot(nz[q]) != 0) << q;
    switch (mask) {  // block uniform: all waves see the same 32 spectra
      case 1: run(IntC<0>{}, IntC<2>{}); break;
      case 2: run(IntC<1>{}, IntC<3>{}); break;
      case 4: run(IntC<2>{}, IntC<4>{}); break;
      case 3: run(IntC<0>{}, IntC<3>{}); break;
      case 6: run(IntC<1>{}, IntC<4>{}); break;
      default: run(IntC<0>{}, IntC<4>{}); break;
    }
  }
  __syncthreads();  // every wave is done with its stage: the buffer takes the partial sums
  if constexpr (NB == kNB) {
    // rows 0-15 from the 16-row group; rows 16-19 from the 4x4 blocks, the
    // two column halves in columns 16-19 and 20-23
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][16 * rt + 4 * kq + r][i_row] = acc[rt][0][r];
    const int g4 = (lane >> 2) & 7;
#pragma unroll
    for (int r = 0; r < 4; ++r) red[wave][4 * g4 + r][16 + (lane & 3) + 4 * (lane >> 5)] = acc4[r];
  } else {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < NG; ++q) red[wave][16 * rt + 4 * kq + r][16 * q + i_row] = acc[rt][q][r];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * NB; e += 512) {
    const int i = e / NB, k = e - i * NB;
    float v;
    if (NB == kNB && k >= 16) {
      v = red[0][i][k] + red[0][i][k + 4];
#pragma unroll
      for (int w = 1; w < NWV; ++w) v += red[w][i][k] + red[w][i][k + 4];
    } else {
      v = red[0][i][k];
#pragma unroll
      for (int w = 1; w < NWV; ++w) v += red[w][i][k];
    }
    pb[i][k] = v;
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 32 && s0 + t < count)
    bwd_epilogue<NB>(g, s, adam, do_adam, grad_out, work_spec(s, s0 + t), pb[t]);
}

}  // namespace

hipError_t launch_interp_fwd(const Geometry &g, const State &s, int deriv_rows, int bf16x3,
                             hipStream_t st) {
  const int rows_per_spec = deriv_rows ? 4 : 1;
  const int rows = g.B * rows_per_spec;
  const int cols_per_block = 4 * 16 * kFwdTiles;
  dim3 grid((g.ldF + cols_per_block - 1) / cols_per_block, (rows + 15) / 16);
  // derivative rows are only formed for final evaluations: never skip those
  const int skip_done = deriv_rows ? 0 : 1;
  if (bf16x3)
    hipLaunchKernelGGL(k_interp_fwd_bf16, grid, dim3(256), 0, st, g, s, rows_per_spec, skip_done);
  else if (g.nb == kNB)
    hipLaunchKernelGGL(k_interp_fwd<kNB>, grid, dim3(256), 0, st, g, s, rows_per_spec, skip_done);
  else
    hipLaunchKernelGGL(k_interp_fwd<kNB * kMaxClasses>, grid, dim3(256), 0, st, g, s,
                       rows_per_spec, skip_done);
  return hipGetLastError();
}

hipError_t launch_interp_bwd(const Geometry &g, const State &s, const AdamCfg *adam,
                             float *grad_out, int bf16x3, hipStream_t st) {
  AdamCfg a = adam ? *adam : AdamCfg{0.f, 0.f, 0.f, 0.f, 0, 0.f};
  const dim3 grid((g.B + 15) / 16);
  if (bf16x3)
    hipLaunchKernelGGL(k_interp_bwd_bf16, grid, dim3(256), 0, st, g, s, a, adam ? 1 : 0, grad_out);
  else if (g.nb == kNB)
    hipLaunchKernelGGL((k_interp_bwd<kNB>), dim3((g.B + 31) / 32), dim3(512), 0, st, g, s, a,
                       adam ? 1 : 0, grad_out);
  else
    hipLaunchKernelGGL((k_interp_bwd<kNB * kMaxClasses>), dim3((g.B + 31) / 32), dim3(512), 0,
                       st, g, s, a, adam ? 1 : 0, grad_out);
  return hipGetLastError();
}

hipError_t launch_split_basis(const Geometry &g, const State &s, hipStream_t st) {
  hipLaunchKernelGGL(k_split_basis, dim3((g.ldF + 255) / 256), dim3(256), 0, st, g, s);
  return hipGetLastError();
}

}  // namespace lasp
