// Once-per-fit preparation of each spectrum: pixel weights, the flux weight
// w of Eq. 6 (a flux quantile, Section 3.3 "Setting spectral weighting
// factors"), the lane-major (o/w, W w^2) layout read by the fused pass, and
// the initial Adam state.
#include "lasp_internal.h"

namespace lasp {
namespace {

constexpr int kPrepBlock = 256;

__device__ inline bool pixel_ok(float o, float iv) {
  return isfinite(o) && isfinite(iv) && iv > 0.f;
}

// Order-preserving map of a float to an unsigned key.
__device__ inline uint32_t fkey(float f) {
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float funkey(uint32_t k) {
  uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(b);
}

// Key of a pixel left out of the selection (no finite flux maps to it).
constexpr uint32_t kNoKey = 0xffffffffu;

// k-th smallest (0-based) flux among the valid pixels of one spectrum, by a
// four-pass 8-bit radix select over the order-preserving keys (staged in
// LDS, kNoKey for invalid pixels).  Each pass counts the candidates' digits
// into 256 bins (a wave whose candidates all share one digit adds them with
// one atomic: the first passes see nearly equal fluxes), then thread t
// takes bin t in a block-wide prefix sum and the one thread whose bin holds
// the k-th candidate records the digit and the rank within it.
__device__ float block_select(const uint32_t *keys, int P, uint32_t k, uint32_t *hist,
                              uint32_t *sh) {
  static_assert(kPrepBlock == 256, "one bin per thread");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t *wsum = sh + 2;  // [kPrepBlock / 64] bin totals of each wave's bins
  uint32_t prefix = 0, mask = 0;
  for (int shift = 24; shift >= 0; shift -= 8) {
    hist[tid] = 0;
    __syncthreads();
    for (int j = tid; j < P; j += kPrepBlock) {
      const uint32_t key = keys[j];
      const bool take = key != kNoKey && (key & mask) == prefix;
      const uint32_t bin = (key >> shift) & 255u;
      const uint64_t tk = __ballot(take);
      if (tk == 0) continue;
      const int first = __ffsll((unsigned long long)tk) - 1;
      const uint32_t b0 = __shfl(bin, first);
      if (__ballot(take && bin == b0) == tk) {
        if (lane == first) atomicAdd(&hist[b0], (uint32_t)__popcll(tk));
      } else if (take) {
        atomicAdd(&hist[bin], 1u);
      }
    }
    __syncthreads();
    const uint32_t h = hist[tid];
    uint32_t incl = h;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    for (int w = 0; w < wave; ++w) incl += wsum[w];
    const uint32_t excl = incl - h;
    // bins 0..254 hold the k-th candidate when excl <= k < incl; bin 255
    // takes whatever rank is past bin 254
    if (excl <= k && (tid == 255 || k < incl)) {
      sh[0] = (uint32_t)tid;
      sh[1] = k - excl;
    }
    __syncthreads();
    prefix |= sh[0] << shift;
    mask |= 255u << shift;
    k = sh[1];
    __syncthreads();
  }
  return funkey(prefix);
}

// The (k+1)-th smallest valid flux right after block_select(k) returned key0
// (its last pass left the digit and the rank in sh[0], sh[1] and the count of
// that exact key in hist): key0 again if another pixel holds it, else the
// smallest valid key above key0 -- the same value a second select would
// give, for one pass over the keys.
__device__ float block_select_next(const uint32_t *keys, int P, uint32_t key0,
                                   const uint32_t *hist, uint32_t *sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t *wmin = sh + 2;  // [kPrepBlock / 64]
  if (sh[1] + 1 < hist[sh[0]]) return funkey(key0);  // block uniform
  uint32_t m = kNoKey;  // above every valid key
  for (int j = tid; j < P; j += kPrepBlock) {
    const uint32_t key = keys[j];
    if (key > key0) m = min(m, key);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor(m, o));
  __syncthreads();  // every thread has read sh and hist
  if (lane == 0) wmin[wave] = m;
  __syncthreads();
  m = wmin[0];
#pragma unroll
  for (int w = 1; w < kPrepBlock / 64; ++w) m = min(m, wmin[w]);
  __syncthreads();
  return funkey(m);
}

__global__ __launch_bounds__(kPrepBlock) void k_prepare(Geometry g, State s, const float *obs,
                                                        const float *ivar, const float *init,
                                                        double blo0, double blo1, double blo2,
                                                        double blo3, double blo4, double bhi0,
                                                        double bhi1, double bhi2, double bhi3,
                                                        double bhi4, float quantile,
                                                        int init_state, int target_steps) {
  // [max(P, 2 * 64 * kNPL)]: the row's flux keys, then the layout staging
  extern __shared__ __align__(16) uint32_t keys[];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t sh[2 + kPrepBlock / 64];
  __shared__ int red_n[kPrepBlock / 64];
  __shared__ int red_bad[kPrepBlock / 64];
  const int spec = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const size_t row = (size_t)spec * g.P;
  const float *o_row = obs + row;
  const float *i_row = ivar + row;

  int n = 0, bad = 0;
  for (int j = tid; j < g.P; j += kPrepBlock) {
    const float o = o_row[j], iv = i_row[j];
    const bool ok = pixel_ok(o, iv);
    n += ok ? 1 : 0;
    bad |= (!isfinite(o) || !isfinite(iv)) ? 1 : 0;
    keys[j] = ok ? fkey(o) : kNoKey;
  }
  n = wave_sum(n);
  bad = wave_sum(bad);
  if (lane == 0) {
    red_n[wave] = n;
    red_bad[wave] = bad;
  }
  __syncthreads();
  int n_eff = 0, any_bad = 0;
  for (int w = 0; w < kPrepBlock / 64; ++w) {
    n_eff += red_n[w];
    any_bad |= red_bad[w];
  }

  // Flux weight: the requested quantile (linear interpolation between order
  // statistics), rounded to the nearest power of two so that o/w and W w^2
  // are exact in floating point.  The objective does not depend on w.
  float w = 1.f;
  if (quantile > 0.f && n_eff > 0) {
    const float pos = quantile * (float)(n_eff - 1);
    const uint32_t k0 = (uint32_t)floorf(pos);
    const float frac = pos - (float)k0;
    const float v0 = block_select(keys, g.P, k0, hist, sh);
    float q = v0;
    if (frac > 0.f && k0 + 1 < (uint32_t)n_eff) {
      const float v1 = block_select_next(keys, g.P, fkey(v0), hist, sh);
      q = v0 + frac * (v1 - v0);
    }
    if (q > 0.f && isfinite(q)) w = exp2f(rintf(log2f(q)));
    if (!(w > 0.f) || !isfinite(w) || !isfinite(1.f / (w * w))) w = 1.f;
  }
  const float inv_w = 1.f / w;
  const float w2 = w * w;

  // Lane-major layout for the fused pass: slot (i, lane) holds pixel
  // lane * kNPL + i, so a lane reads its pixels with coalesced loads.  The
  // pixels of 64 lanes at a time go through LDS (the keys' space, free
  // after the selects): read in pixel order, written in slot order, both
  // coalesced.
  float2 *dst = s.ow + (size_t)spec * kNPL * g.block;
  float2 *stage = reinterpret_cast<float2 *>(keys);  // [64 * kNPL]
  constexpr int kChunk = 64 * kNPL;
  for (int ln0 = 0; ln0 < g.block; ln0 += 64) {
    __syncthreads();  // the keys, or the previous chunk, are no longer read
    for (int q = tid; q < kChunk; q += kPrepBlock) {
      const int j = ln0 * kNPL + q;
      float2 val = make_float2(0.f, 0.f);
      if (j < g.P) {
        const float o = o_row[j], iv = i_row[j];
        if (pixel_ok(o, iv)) val = make_float2(o * inv_w, iv * w2);
      }
      stage[q] = val;
    }
    __syncthreads();
    for (int q = tid; q < kChunk; q += kPrepBlock) {
      const int i = q >> 6, l = q & 63;
      dst[(size_t)i * g.block + ln0 + l] = stage[l * kNPL + i];
    }
  }

  if (tid == 0) {
    uint32_t st = 0;
    if (any_bad) st |= kStNonfinite;
    if (n_eff <= kNP + g.nd) st |= kStNoData;
    s.status[spec] = st;
    s.neff[spec] = n_eff;
    s.wscale[spec] = w;
    if (init_state) {
      const double lo[5] = {blo0, blo1, blo2, blo3, blo4};
      const double hi[5] = {bhi0, bhi1, bhi2, bhi3, bhi4};
      for (int t = 0; t < kNP; ++t) {
        double th = (double)init[(size_t)spec * kNP + t];
        if (t == 0) th = log10(th);
        s.u[(size_t)spec * kNP + t] = (float)(2.0 * (th - lo[t]) / (hi[t] - lo[t]) - 1.0);
        s.m[(size_t)spec * kNP + t] = 0.f;
        s.v[(size_t)spec * kNP + t] = 0.f;
      }
      s.t[spec] = 0;
      if (s.target) s.target[spec] = target_steps;
      if (s.nrise) s.nrise[spec] = 0;
    }
  }
}

// OUT_OF_BOX of the parameters u (|u_t| > 1.5 for some t, or not finite).
__device__ inline uint32_t box_bit(const float *u) {
  uint32_t b = 0;
  for (int t = 0; t < kNP; ++t)
    if (!(fabsf(u[t]) <= 1.5f)) b = kStOutOfBox;
  return b;
}

// Physical parameters, status and chi2 at the end of a fit.  OUT_OF_BOX is
// replaced by that of the returned parameters.
__global__ void k_finalize(Geometry g, State s, double blo0, double blo1, double blo2, double blo3,
                           double blo4, double bhi0, double bhi1, double bhi2, double bhi3,
                           double bhi4, float *out_params, uint32_t *status_out,
                           double *chi2_out, int32_t *steps_out) {
  const int spec = blockIdx.x * blockDim.x + threadIdx.x;
  if (spec >= g.B) return;
  const double lo[5] = {blo0, blo1, blo2, blo3, blo4};
  const double hi[5] = {bhi0, bhi1, bhi2, bhi3, bhi4};
  uint32_t st = (s.status[spec] & ~kStOutOfBox) | box_bit(s.u + (size_t)spec * kNP);
  for (int t = 0; t < kNP; ++t) {
    const double u = (double)s.u[(size_t)spec * kNP + t];
    double th = lo[t] + 0.5 * (u + 1.0) * (hi[t] - lo[t]);
    if (t == 0) th = exp10(th);
    out_params[(size_t)spec * kNP + t] = (float)th;
  }
  s.status[spec] = st;
  if (status_out) status_out[spec] = st;
  if (chi2_out) chi2_out[spec] = s.chi2[spec];
  if (steps_out) steps_out[spec] = s.t[spec];
}

// Steps taken and stopped flag of each slot.
// The spectra still taking steps, in index order within each Teff regime
// (with several emulator classes: cool, cool/warm blend, warm, warm/hot
// blend, hot, from the current parameters), regimes in that order, so that
// the contraction tiles mostly hold one regime.  Each thread counts the
// active spectra of its contiguous chunk per regime, workgroup-wide scans of
// the counts give each chunk's first position in each regime, and each
// thread writes its chunk.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_compact(Geometry g, State s, int *order,
                                                  int *n_active) {
  constexpr int kKeys = 5;
  __shared__ int cnt[kKeys][1024];
  __shared__ int first[kKeys + 1];
  const int t = threadIdx.x;
  const int nk = g.n_classes > 1 ? kKeys : 1;
  // regime boundaries in the normalised log Teff coordinate
  double ue[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) ue[e] = (log10(g.edges[e]) - g.lt_lo) / g.lt_half - 1.0;
  auto key = [&](int i) {
    if (nk == 1) return 0;
    const double u1 = s.u[(size_t)i * kNP];
    int k = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) k += u1 > ue[e] ? 1 : 0;
    return k;
  };
  const int chunk = (g.B + 1023) / 1024;
  const int b0 = min(t * chunk, g.B), b1 = min(b0 + chunk, g.B);
  int c[kKeys] = {0, 0, 0, 0, 0};
  for (int i = b0; i < b1; ++i) {
    if (!slot_active(s, i)) continue;
    const int k = key(i);
#pragma unroll
    for (int q = 0; q < kKeys; ++q) c[q] += q == k ? 1 : 0;
  }
#pragma unroll
  for (int q = 0; q < kKeys; ++q) cnt[q][t] = c[q];
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive scans
    int v[kKeys];
#pragma unroll
    for (int q = 0; q < kKeys; ++q) v[q] = (t >= off && q < nk) ? cnt[q][t - off] : 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kKeys; ++q) cnt[q][t] += v[q];
    __syncthreads();
  }
  if (t == 0) {
    first[0] = 0;
    for (int q = 0; q < kKeys; ++q) first[q + 1] = first[q] + cnt[q][1023];
  }
  __syncthreads();
  int pos[kKeys];
#pragma unroll
  for (int q = 0; q < kKeys; ++q) pos[q] = first[q] + cnt[q][t] - c[q];
  for (int i = b0; i < b1; ++i) {
    if (!slot_active(s, i)) continue;
    const int k = key(i);
#pragma unroll
    for (int q = 0; q < kKeys; ++q)
      if (q == k) order[pos[q]++] = i;
  }
  if (t == 1023) *n_active = first[kKeys];
}

__global__ void k_progress(Geometry g, State s, int32_t *steps, int32_t *done) {
  const int spec = blockIdx.x * blockDim.x + threadIdx.x;
  if (spec >= g.B) return;
  const int t = s.t[spec];
  if (steps) steps[spec] = t;
  if (done) done[spec] = (s.target && t >= s.target[spec]) ? 1 : 0;
}

// Per-spectrum results of a forward evaluation: chi2, the objective
// J = chi2 / n_eff of Eq. 9 (read per spectrum), n_eff and status (with
// OUT_OF_BOX of the evaluated u).
__global__ void k_outputs(Geometry g, State s, double *chi2_out, float *J_out, int32_t *neff_out,
                          uint32_t *status_out) {
  const int spec = blockIdx.x * blockDim.x + threadIdx.x;
  if (spec >= g.B) return;
  const double c = s.chi2[spec];
  const int n = s.neff[spec];
  const uint32_t st = (s.status[spec] & ~kStOutOfBox) | box_bit(s.u + (size_t)spec * kNP);
  s.status[spec] = st;
  if (chi2_out) chi2_out[spec] = c;
  if (J_out) J_out[spec] = n > 0 ? (float)(c / (double)n) : 0.f;
  if (neff_out) neff_out[spec] = n;
  if (status_out) status_out[spec] = st;
}

}  // namespace

hipError_t launch_outputs(const Geometry &g, const State &s, double *chi2_out, float *J_out,
                          int32_t *neff_out, uint32_t *status_out, hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL(k_outputs, dim3((g.B + bs - 1) / bs), dim3(bs), 0, st, g, s, chi2_out, J_out,
                     neff_out, status_out);
  return hipGetLastError();
}

hipError_t launch_prepare(const Geometry &g, const State &s, const float *obs, const float *ivar,
                          const float *init_params, const double *lo, const double *hi,
                          float weight_quantile, int init_state, int target_steps,
                          hipStream_t st) {
  const size_t lds = sizeof(uint32_t) * (size_t)(g.P > 2 * 64 * kNPL ? g.P : 2 * 64 * kNPL);
  hipLaunchKernelGGL(k_prepare, dim3(g.B), dim3(kPrepBlock), lds, st,
                     g, s, obs, ivar, init_params,
                     lo[0], lo[1], lo[2], lo[3], lo[4], hi[0], hi[1], hi[2], hi[3], hi[4],
                     weight_quantile, init_state, target_steps);
  return hipGetLastError();
}

hipError_t launch_finalize(const Geometry &g, const State &s, const double *lo, const double *hi,
                           float *out_params, uint32_t *status_out, double *chi2_out,
                           int32_t *steps_out, hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL(k_finalize, dim3((g.B + bs - 1) / bs), dim3(bs), 0, st, g, s, lo[0], lo[1],
                     lo[2], lo[3], lo[4], hi[0], hi[1], hi[2], hi[3], hi[4], out_params,
                     status_out, chi2_out, steps_out);
  return hipGetLastError();
}

hipError_t launch_compact(const Geometry &g, const State &s, int *order, int *n_active,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, g, s, order, n_active);
  return hipGetLastError();
}

hipError_t launch_progress(const Geometry &g, const State &s, int32_t *steps, int32_t *done,
                           hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL(k_progress, dim3((g.B + bs - 1) / bs), dim3(bs), 0, st, g, s, steps, done);
  return hipGetLastError();
}

}  // namespace lasp
