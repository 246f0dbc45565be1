// Internal declarations of the HIP library: argument blocks, device helpers
// and kernel launchers.  Not part of the public ABI (include/lasp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lasp {

constexpr double kCkms = 299792.458;            // speed of light, km/s
constexpr double kLn10 = 2.302585092994045684;  // ln 10
constexpr float kSigmaFloorPx = 0.1f;           // lower bound of the kernel width, pixels
constexpr int kNB = 20;                         // interpolator terms (cubic in 3 coordinates)
constexpr int kMaxClasses = 3;                  // emulator temperature classes
constexpr int kNP = 5;                          // free parameters per spectrum
constexpr int kNPL = 17;                        // pixels owned by one lane in the fused pass
constexpr int kTB = 8;                          // taps per register block
constexpr int kMaxArms = 4;

// Status bits (same values as LASP_ST_* in lasp.h).
constexpr uint32_t kStNonfinite = 0x01u;
constexpr uint32_t kStNoData = 0x02u;
constexpr uint32_t kStSingular = 0x04u;
constexpr uint32_t kStContNonpos = 0x08u;
constexpr uint32_t kStOutOfBox = 0x10u;
constexpr uint32_t kStSigmaFloor = 0x20u;
constexpr uint32_t kStStopFlat = 0x40u;
constexpr uint32_t kStStopRising = 0x80u;
constexpr uint32_t kStNotConverged = 0x100u;
constexpr uint32_t kStPolishLimit = 0x200u;
constexpr int kMaxStopWindow = 4096;

// Levenberg-Marquardt polish: a spectrum stops when the predicted chi2
// decrease of its next step is below kLmDecreaseTol (chi2 units: the
// remaining improvement is 1e-3 standard deviations in any direction), when
// an accepted step lowers chi2 by less than kLmDropTol relative or moves u
// by less than kLmStepTol, or when the damping passes kLmLambdaMax.
constexpr double kLmDecreaseTol = 1e-6;
constexpr double kLmDropTol = 1e-10;
constexpr double kLmStepTol = 1e-7;
constexpr double kLmLambdaMax = 1e10;
constexpr int kLmDone = 1;
constexpr int kNormalStride = 32;

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Geometry shared by every per-step kernel.
struct Geometry {
  int B;        // spectra
  int P;        // pixels
  int M;        // margin
  int Pe;       // P + 2M basis columns
  int ldF;      // row stride of F' / F-bar' / padded basis (multiple of 64, >= Pe)
  int nd;       // continuum coefficients D + 1
  int block;    // threads of the fused pass
  int n_arms;   // >= 1
  int arm_start[kMaxArms + 1];  // arm a covers pixels [arm_start[a], arm_start[a+1])
  double arm_sig2[kMaxArms];    // instrumental sigma^2, (km/s)^2 (0 for a single bare arm)
  int bare;                     // 1: one arm without instrument term
  double inv_scale;             // pixels per km/s = 1 / (c ln10 dlog10)
  double rv_lo, rv_half;        // RV = rv_lo + (u4 + 1) rv_half
  double sg_lo, sg_half;        // sigma = sg_lo + (u5 + 1) sg_half
  int n_classes;                // 1, or 3 emulator temperature classes
  int nb;                       // basis rows: kNB * n_classes
  double lt_lo, lt_half;        // log10 Teff = lt_lo + (u1 + 1) lt_half
  double edges[4];              // Teff regime edges (K) of the class blend
  double hpow[11];              // h^n, h = 2 / P: pixel step of the continuum's x
};

// Per-spectrum state and scratch owned by the library.
struct State {
  float *u;         // [B][5] normalised parameters
  float *m;         // [B][5] Adam first moment
  float *v;         // [B][5] Adam second moment
  int *t;           // [B] Adam step count
  int *target;      // [B] step count at which a slot stops (NULL: every slot runs)
  float2 *ow;       // [B][kNPL][block] (o/w, W w^2) in lane-major order
  float *wscale;    // [B] flux weight w
  int *neff;        // [B]
  uint32_t *status; // [B]
  float *fp;        // [B][ldF] (or [B][4][ldF]) F'
  int fp_stride;    // floats between consecutive spectra in fp (ldF or 4 ldF)
  float *fbar;      // [B][ldF] F-bar'
  float *g45;       // [B][2] dJ/du4, dJ/du5
  double *chi2;     // [B]
  double *lhist;    // [B][stop window] loss history ring (stopping rules)
  int *nrise;       // [B] consecutive steps at which the loss rose
  // Optional list of the spectra still taking steps (stopping rules on):
  // the per-step kernels then work on order[0 .. *n_active) instead of
  // 0 .. B.  NULL: every spectrum, in index order.
  const int *order;     // [B] spectrum indices, active ones first
  const int *n_active;  // [1] length of the list
  float *basis;     // [nb][ldF] zero-padded copy of the basis
  uint16_t *basis_hi;  // [20][ldF] bf16 high part (BF16x3, adjoint contraction)
  uint16_t *basis_lo;  // [20][ldF] bf16 low part
  uint16_t *basis_thi; // [ldF][32] bf16 high part, k-major per column, rows 1..19 (forward)
  uint16_t *basis_tlo; // [ldF][32] bf16 low part
};

// Per-spectrum state of the Levenberg-Marquardt polish.
struct LmState {
  double *normal;      // [B][kNormalStride] S (25), q (5), chi2 at the current u
  double *lambda;      // [B] damping
  double *chi2_trial;  // [B] chi2 at the trial point
  double *step_inf;    // [B] max |du| of the trial step (NaN: no step)
  float *u_trial;      // [B][5]
  uint32_t *st_trial;  // [B] status of the trial evaluation (discarded)
  int *need_jac;       // [B] 1: normal equations needed at the current u
  int *flags;          // [B] kLmDone
  int *active;         // [1] spectra still iterating (k_lm_active)
};

// Inputs and outputs of the Clean mask kernel.  obs, ivar and model are
// [B][P] row-major in the units of obs.  With s.ow set, the kernel writes
// the new weights into the fused pass's (o/w, W w^2) array and n_eff; with
// s.target set, stopped spectra are skipped.
struct CleanArgs {
  const float *obs;
  const float *ivar;
  const float *model;
  float f_shift;
  uint8_t *keep_out;   // optional [B][P]: 1 kept, 0 clipped
  int32_t *masked_out; // optional [B]: clipped valid pixels
  State s;             // ow, wscale, neff, t, target (others unused)
};

struct AdamCfg {
  float lr, beta1, beta2, eps;
  int stop_window;  // 0: fixed step count
  float stop_tol;
};

// ---------------------------------------------------------------- host side
hipError_t launch_prepare(const Geometry &g, const State &s, const float *obs, const float *ivar,
                          const float *init_params, const double *box_lo, const double *box_hi,
                          float weight_quantile, int init_state, int target_steps, hipStream_t st);

// A spectrum takes Adam steps while t < target (always when target is NULL).
#ifdef __HIPCC__
__device__ inline bool slot_active(const State &s, int spec) {
  return s.target == nullptr || s.t[spec] < s.target[spec];
}
// Entries the per-step kernels cover, and the spectrum of entry i.
__device__ inline int work_count(const Geometry &g, const State &s) {
  return s.order ? *s.n_active : g.B;
}
__device__ inline int work_spec(const State &s, int i) { return s.order ? s.order[i] : i; }
#endif
// Writes the spectra with slot_active true to order -- in index order, or
// with several emulator classes in index order within each Teff regime,
// regimes by increasing Teff -- and their number to n_active (one
// workgroup).
hipError_t launch_compact(const Geometry &g, const State &s, int *order, int *n_active,
                          hipStream_t st);
hipError_t launch_interp_fwd(const Geometry &g, const State &s, int deriv_rows, int bf16x3,
                             hipStream_t st);
// set_status: 1 for a pass at the parameters a call returns (the
// evaluation bits of the status are replaced), 0 for the passes of the
// steps (status untouched).
hipError_t launch_fused(const Geometry &g, const State &s, int adjoint, float *model_out,
                        int set_status, hipStream_t st);
hipError_t launch_interp_bwd(const Geometry &g, const State &s, const AdamCfg *adam,
                             float *grad_out, int bf16x3, hipStream_t st);
hipError_t launch_split_basis(const Geometry &g, const State &s, hipStream_t st);
hipError_t launch_finalize(const Geometry &g, const State &s, const double *box_lo,
                           const double *box_hi, float *out_params, uint32_t *status_out,
                           double *chi2_out, int32_t *steps_out, hipStream_t st);
hipError_t launch_progress(const Geometry &g, const State &s, int32_t *steps, int32_t *done,
                           hipStream_t st);
// Covariance, model Jacobian and/or Gauss-Newton normal equations
// (out_normal [B][kNormalStride]: S row-major [25], q [5], chi2) for the
// spectra with active[spec] != 0 (every spectrum when active is NULL).
hipError_t launch_cov(const Geometry &g, const State &s, const double *box_lo, const double *box_hi,
                      double *out_cov, float *out_jac, double *out_normal, const int *active,
                      hipStream_t st);
hipError_t launch_outputs(const Geometry &g, const State &s, double *chi2_out, float *J_out,
                          int32_t *neff_out, uint32_t *status_out, hipStream_t st);
hipError_t launch_lm_init(const Geometry &g, const LmState &lm, hipStream_t st);
hipError_t launch_lm_solve(const Geometry &g, const State &s, const LmState &lm, hipStream_t st);
hipError_t launch_lm_active(const Geometry &g, const LmState &lm, hipStream_t st);
hipError_t launch_lm_accept(const Geometry &g, const State &s, const LmState &lm, int last,
                            hipStream_t st);
hipError_t launch_clean(const Geometry &g, const CleanArgs &a, hipStream_t st);
hipError_t launch_resample(const float *src, int n_rows, int n_src, int64_t ld_src, double lam0,
                           double dlam, float *out, int n_out, int64_t ld_out, double lg0,
                           double dlog10, hipStream_t st);
bool fused_supported(int block, int nd);
// Sets the calling thread's lasp_last_error() message; returns code.
int set_error(int code, const char *msg);
size_t fused_smem_bytes(const Geometry &g);

// -------------------------------------------------------------- device side
#ifdef __HIPCC__

// Eq. 1 features: monomials of total degree <= 3 in x = (u1, u2, u3),
// graded lexicographic order.
__device__ inline void features(float x, float y, float z, float *phi) {
  phi[0] = 1.f;
  phi[1] = x; phi[2] = y; phi[3] = z;
  phi[4] = x * x; phi[5] = x * y; phi[6] = x * z; phi[7] = y * y; phi[8] = y * z; phi[9] = z * z;
  phi[10] = x * x * x; phi[11] = x * x * y; phi[12] = x * x * z; phi[13] = x * y * y;
  phi[14] = x * y * z; phi[15] = x * z * z; phi[16] = y * y * y; phi[17] = y * y * z;
  phi[18] = y * z * z; phi[19] = z * z * z;
}

// Weights of the three emulator classes (cool, warm, hot) at u1 (Eq. 1 over
// the five Teff regimes): with a = clamp((T - e0) / (e1 - e0)) and
// b = clamp((T - e2) / (e3 - e2)) the weights are 1 - a, a (1 - b) and a b,
// so one class holds inside a regime and two blend linearly in Teff across a
// transition regime.  dw = d w / d u1 (zero where the blend is flat).  FP64
// inside, FP32 out.
__device__ inline void class_weights(const Geometry &g, float u1, float *w, float *dw) {
  const double lt = g.lt_lo + ((double)u1 + 1.0) * g.lt_half;
  const double T = exp(kLn10 * lt);
  const double dT = T * kLn10 * g.lt_half;
  const double w01 = g.edges[1] - g.edges[0], w23 = g.edges[3] - g.edges[2];
  double a = (T - g.edges[0]) / w01, da = dT / w01;
  if (!(T > g.edges[0] && T < g.edges[1])) da = 0.0;
  a = fmin(fmax(a, 0.0), 1.0);
  double b = (T - g.edges[2]) / w23, db = dT / w23;
  if (!(T > g.edges[2] && T < g.edges[3])) db = 0.0;
  b = fmin(fmax(b, 0.0), 1.0);
  w[0] = (float)(1.0 - a);
  w[1] = (float)(a * (1.0 - b));
  w[2] = (float)(a * b);
  dw[0] = (float)(-da);
  dw[1] = (float)(da * (1.0 - b) - a * db);
  dw[2] = (float)(da * b + a * db);
}

// d phi_k / d x_t for t = 0, 1, 2 (d[t][k]).
__device__ inline void feature_derivs(float x, float y, float z, float (*d)[kNB]) {
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int k = 0; k < kNB; ++k) d[t][k] = 0.f;
  d[0][1] = 1.f; d[1][2] = 1.f; d[2][3] = 1.f;
  d[0][4] = 2.f * x;
  d[0][5] = y; d[1][5] = x;
  d[0][6] = z; d[2][6] = x;
  d[1][7] = 2.f * y;
  d[1][8] = z; d[2][8] = y;
  d[2][9] = 2.f * z;
  d[0][10] = 3.f * x * x;
  d[0][11] = 2.f * x * y; d[1][11] = x * x;
  d[0][12] = 2.f * x * z; d[2][12] = x * x;
  d[0][13] = y * y; d[1][13] = 2.f * x * y;
  d[0][14] = y * z; d[1][14] = x * z; d[2][14] = x * y;
  d[0][15] = z * z; d[2][15] = 2.f * x * z;
  d[1][16] = 3.f * y * y;
  d[1][17] = 2.f * y * z; d[2][17] = y * y;
  d[1][18] = z * z; d[2][18] = 2.f * y * z;
  d[2][19] = 3.f * z * z;
}

// Butterfly reduce-scatter of N per-lane values over a 64-lane wave.
// On return every lane holds, in v[0], the wave-wide sum of value index
// lane / (64 / N); lanes with lane % (64 / N) == 0 are the writers.
template <int N, typename T>
__device__ inline T wave_reduce_scatter(T (&v)[N], int lane) {
  static_assert(N >= 1 && N <= 64 && (N & (N - 1)) == 0, "N must be a power of two <= 64");
  int off = 32;
#pragma unroll
  for (int cnt = N; cnt > 1; cnt >>= 1, off >>= 1) {
    const int half = cnt >> 1;
    const bool hi = (lane & off) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      T send = hi ? v[i] : v[half + i];
      T keep = hi ? v[half + i] : v[i];
      v[i] = keep + __shfl_xor(send, off, 64);
    }
  }
  T r = v[0];
  for (; off >= 1; off >>= 1) r += __shfl_xor(r, off, 64);
  return r;
}


// Makes the compiler treat x as a new value: computations from x after this
// point are not merged with the same computations before it (which would
// keep their results live across phases and raise register pressure).
template <typename T>
__device__ inline void opaque(T &x) {
  asm volatile("" : "+v"(x));
}

// Value of v in lane l (l wave uniform), through scalar registers.
__device__ inline double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}


template <int N>
struct Pow2 {
  static constexpr int v = N <= 1 ? 1 : 2 * Pow2<(N + 1) / 2>::v;
};
template <>
struct Pow2<1> {
  static constexpr int v = 1;
};

// Sum of NV per-lane doubles over the workgroup, result in out[0..NV).
// Chunks of 32 go through the wave butterfly, then across waves in a
// fixed order (deterministic).
template <int NW, int NV>
__device__ inline void block_sum_doubles(const double (&acc)[NV], double *red, double *out,
                                         int lane, int wave) {
  constexpr int kChunks = (NV + 31) / 32;
#pragma unroll
  for (int ch = 0; ch < kChunks; ++ch) {
    constexpr int kW = NV < 32 ? Pow2<NV>::v : 32;
    double tmp[kW];
#pragma unroll
    for (int i = 0; i < kW; ++i) tmp[i] = (ch * 32 + i < NV) ? acc[(ch * 32 + i) % NV] : 0.0;
    const double r = wave_reduce_scatter<kW, double>(tmp, lane);
    constexpr int kStride = 64 / kW;
    if ((lane % kStride) == 0) red[wave * 64 + lane / kStride] = r;
    __syncthreads();
    const int t = threadIdx.x;
    if (t < kW && ch * 32 + t < NV) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += red[w * 64 + t];
      out[ch * 32 + t] = s;
    }
    __syncthreads();
  }
}

// Orders a wave's LDS accesses so that lanes see each other's stores.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over each aligned group of eight lanes, returned in all eight, by DPP
// lane moves (no LDS round trip): swap neighbours, swap pairs within a
// quad, then mirror within the half row, which pairs the group's two quads.
// The additions form the same tree in every lane, so all eight agree.
template <int CTRL>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ inline int dpp_mov(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <typename T>
__device__ inline T group8_sum(T v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  return v;
}

__device__ inline int read_lane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Sum over the wave, the same value in every lane: eight-lane groups, then
// the row mirror pairs the two groups of each 16-lane row, then the four
// row sums are read through scalar registers and added in a fixed order.
template <typename T>
__device__ inline T wave_sum(T x) {
  x = group8_sum(x);
  x += dpp_mov<0x140>(x);  // row_mirror
  return (read_lane(x, 0) + read_lane(x, 16)) + (read_lane(x, 32) + read_lane(x, 48));
}

__device__ inline float wave_min(float x) {
  x = fminf(x, dpp_mov<0xB1>(x));
  x = fminf(x, dpp_mov<0x4E>(x));
  x = fminf(x, dpp_mov<0x141>(x));
  x = fminf(x, dpp_mov<0x140>(x));
  return fminf(fminf(read_lane(x, 0), read_lane(x, 16)), fminf(read_lane(x, 32), read_lane(x, 48)));
}

// Sum of NV per-lane doubles over one wave through LDS (no workgroup
// barrier: any single wave may call it).  scratch holds 8 x 64 doubles;
// out[0..NV) (LDS) is valid in every lane after the call.  Deterministic.
template <int NV>
__device__ inline void wave_sum_lds(const double (&acc)[NV], double *scratch, double *out,
                                    int lane) {
  const int tt = lane >> 3, part = lane & 7;
#pragma unroll
  for (int c = 0; c < (NV + 7) / 8; ++c) {
#pragma unroll
    for (int t = 0; t < 8; ++t) scratch[t * 64 + lane] = (8 * c + t < NV) ? acc[(8 * c + t) % NV] : 0.0;
    wave_lds_sync();
    const double *row = scratch + tt * 64 + 8 * part;
    double v = ((row[0] + row[1]) + (row[2] + row[3])) + ((row[4] + row[5]) + (row[6] + row[7]));
    v = group8_sum(v);
    if (part == 0 && 8 * c + tt < NV) out[8 * c + tt] = v;
    wave_lds_sync();
  }
}

// Sum of NV per-lane values over the workgroup through LDS: eight values at
// a time are widened to FP64 and transposed through scratch[wave][8][64]
// (one wave's region is 4 KB), each group of eight lanes adds one value's 64
// partials, then the waves' results are added in a fixed order.  out[0..NV)
// is valid for every thread after the call.  Deterministic.
template <int NW, int NV, typename T>
__device__ inline void block_sum_lds(const T (&acc)[NV], double *scratch, double *red,
                                     double *out, int lane, int wave) {
  double *sc = scratch + wave * 512;
  const int tt = lane >> 3, part = lane & 7;
#pragma unroll
  for (int c = 0; c < (NV + 7) / 8; ++c) {
    // FP32 partials are widened 8 at a time, so few doubles are live at once
#pragma unroll
    for (int t = 0; t < 8; ++t)
      sc[t * 64 + lane] = (8 * c + t < NV) ? (double)acc[(8 * c + t) % NV] : 0.0;
    wave_lds_sync();
    const double *row = sc + tt * 64 + 8 * part;
    double v = ((row[0] + row[1]) + (row[2] + row[3])) + ((row[4] + row[5]) + (row[6] + row[7]));
    v = group8_sum(v);
    if (part == 0) red[wave * 64 + 8 * c + tt] = v;
    wave_lds_sync();
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w * 64 + t];
    out[t] = s;
  }
  __syncthreads();
}

// block_sum_lds for FP32 partials: eight values at a time go through
// scratch[wave][8][64] as FP32 (2 KB per wave; half the registers and LDS of
// widening first); each group of eight lanes adds one value's eight-lane
// runs in FP32 and the rest -- across the groups, then the waves -- in FP64,
// in a fixed order.  out[0..NV) is
// valid for every thread after the call.  Deterministic.
template <int NW, int NV>
__device__ inline void block_sum_lds_f32(const float (&acc)[NV], float *scratch, double *red,
                                         double *out, int lane, int wave) {
  float *sc = scratch + wave * 8 * 64;
  const int tt = lane >> 3, part = lane & 7;
#pragma unroll
  for (int c = 0; c < (NV + 7) / 8; ++c) {
#pragma unroll
    for (int t = 0; t < 8; ++t) sc[t * 64 + lane] = (8 * c + t < NV) ? acc[(8 * c + t) % NV] : 0.f;
    wave_lds_sync();
    const float4 x0 = *reinterpret_cast<const float4 *>(sc + tt * 64 + 8 * part);
    const float4 x1 = *reinterpret_cast<const float4 *>(sc + tt * 64 + 8 * part + 4);
    double v = (double)(((x0.x + x0.y) + (x0.z + x0.w)) + ((x1.x + x1.y) + (x1.z + x1.w)));
    v = group8_sum(v);
    if (part == 0) red[wave * 64 + 8 * c + tt] = v;
    wave_lds_sync();
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w * 64 + t];
    out[t] = s;
  }
  __syncthreads();
}

#endif  // __HIPCC__

}  // namespace lasp
