// Clean outlier mask (Section 2.2, step 6: the three-step clipping of the
// Clean strategy), per spectrum, from the residual eps = o - m against the
// current model m:
//   B  |eps_j| - f G_j > k sigma, k = 3 relaxed to 4, 5, 7 while more than
//      3 % of the valid pixels would be clipped;
//   C  a neighbour of a B outlier with |eps| - f G > 2 sigma;
//   D  a neighbour j' of an outlier j with eps_j eps_j' > 0,
//      |eps_j'| <= |eps_j| and |eps_j'| - f G_j' > sigma', repeated until it
//      does not change (at most 20 passes);
// with G_j = max |m_j - m_{j+-1}| (the flux gradient), sigma the sample
// standard deviation of eps over the valid pixels and sigma' over those
// kept by B and C.  Decisions in FP64.  Only pixels with positive finite
// weight are tested or seed a neighbour test.
//
// One workgroup per spectrum; thread l owns pixels [17 l, 17 l + 17) (the
// layout of the fused pass), so a new mask can be written straight into its
// (o/w, W w^2) array.
#include "lasp_internal.h"

namespace lasp {
namespace {

constexpr int kMaxDPasses = 20;

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_clean(Geometry g, CleanArgs a) {
  constexpr int NW = BLOCK / 64;
  __shared__ double sRed[NW * 64];
  __shared__ double sOut[8];
  __shared__ double sScr[NW * 512];
  __shared__ double sEL[BLOCK], sER[BLOCK];  // eps of each thread's first and last pixel
  __shared__ double sML[BLOCK], sMR[BLOCK];  // model of the same pixels
  __shared__ uint32_t sOL[BLOCK], sOR[BLOCK];  // outlier flag of the same pixels
  const int spec = blockIdx.x;
  if (a.s.target && a.s.t[spec] >= a.s.target[spec]) return;  // a stopped fit keeps its mask
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int P = g.P;
  const int j0 = tid * kNPL;
  const size_t row = (size_t)spec * P;

  double eps[kNPL], m[kNPL];
  uint32_t valid = 0;
#pragma unroll
  for (int i = 0; i < kNPL; ++i) {
    const int j = j0 + i;
    double e = 0.0, mm = 0.0;
    if (j < P) {
      const float o = a.obs[row + j], iv = a.ivar[row + j];
      mm = (double)a.model[row + j];
      if (isfinite(o) && isfinite(iv) && iv > 0.f) {
        valid |= 1u << i;
        e = (double)o - mm;
      }
    }
    eps[i] = e;
    m[i] = mm;
  }
  sML[tid] = m[0];
  sMR[tid] = m[kNPL - 1];
  sEL[tid] = eps[0];
  sER[tid] = eps[kNPL - 1];
  __syncthreads();
  // flux gradient G_j = max(|m_j - m_{j-1}|, |m_j - m_{j+1}|), ends use one side
  double G[kNPL];
#pragma unroll
  for (int i = 0; i < kNPL; ++i) {
    const int j = j0 + i;
    const double ml = i > 0 ? m[i - 1] : (tid > 0 ? sMR[tid - 1] : 0.0);
    const double mr = i < kNPL - 1 ? m[i + 1] : (tid + 1 < BLOCK ? sML[tid + 1] : 0.0);
    const double gl = j > 0 ? fabs(m[i] - ml) : 0.0;
    const double gr = j + 1 < P ? fabs(m[i] - mr) : 0.0;
    G[i] = fmax(gl, gr);
  }
  const double f = (double)a.f_shift;

  // sample standard deviation of eps over the valid pixels
  auto stats = [&](uint32_t sel, double &sd, double &n_out) {
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int i = 0; i < kNPL; ++i)
      if (sel >> i & 1u) {
        acc[0] += 1.0;
        acc[1] += eps[i];
      }
    block_sum_lds<NW, 2>(acc, sScr, sRed, sOut, lane, wave);
    const double n = sOut[0], mean = n > 0.0 ? sOut[1] / n : 0.0;
    double v[1] = {0.0};
#pragma unroll
    for (int i = 0; i < kNPL; ++i)
      if (sel >> i & 1u) v[0] += (eps[i] - mean) * (eps[i] - mean);
    block_sum_lds<NW, 1>(v, sScr, sRed, sOut + 2, lane, wave);
    sd = n > 1.0 ? sqrt(sOut[2] / (n - 1.0)) : 0.0;
    n_out = n;
  };
  double sigma, nv;
  stats(valid, sigma, nv);

  // B with the relaxed thresholds k = 3, 4, 5, 7 (k is set before each count,
  // so the last one stands if every count is above 3 %)
  double k = 3.0;
  for (int q = 0; q < 4; ++q) {
    k = q == 0 ? 3.0 : (q == 1 ? 4.0 : (q == 2 ? 5.0 : 7.0));
    double c[1] = {0.0};
#pragma unroll
    for (int i = 0; i < kNPL; ++i)
      if ((valid >> i & 1u) && fabs(eps[i]) - f * G[i] > k * sigma) c[0] += 1.0;
    block_sum_lds<NW, 1>(c, sScr, sRed, sOut + 3, lane, wave);
    if (sOut[3] <= 0.03 * nv) break;
  }
  uint32_t bout = 0;
#pragma unroll
  for (int i = 0; i < kNPL; ++i)
    if ((valid >> i & 1u) && fabs(eps[i]) - f * G[i] > k * sigma) bout |= 1u << i;

  // neighbour flags across thread boundaries
  auto exchange = [&](uint32_t flags, uint32_t &left, uint32_t &right) {
    __syncthreads();
    sOL[tid] = flags & 1u;
    sOR[tid] = flags >> (kNPL - 1) & 1u;
    __syncthreads();
    left = tid > 0 ? sOR[tid - 1] : 0u;           // flag of pixel j0 - 1
    right = tid + 1 < BLOCK ? sOL[tid + 1] : 0u;  // flag of pixel j0 + 17
  };
  uint32_t bl, br;
  exchange(bout, bl, br);
  // C: neighbours of B outliers above 2 sigma
  uint32_t cout = 0;
#pragma unroll
  for (int i = 0; i < kNPL; ++i) {
    const bool nb = (i > 0 ? (bout >> (i - 1) & 1u) : bl) || (i < kNPL - 1 ? (bout >> (i + 1) & 1u) : br);
    if ((valid >> i & 1u) && nb && fabs(eps[i]) - f * G[i] > 2.0 * sigma) cout |= 1u << i;
  }
  double sigma2, n2;
  stats(valid & ~bout & ~cout, sigma2, n2);

  // D: grow from the outliers through same-sign, not larger neighbours
  const double el = tid > 0 ? sER[tid - 1] : 0.0;           // eps of pixel j0 - 1
  const double er = tid + 1 < BLOCK ? sEL[tid + 1] : 0.0;  // eps of pixel j0 + 17
  uint32_t dout = 0;
  for (int pass = 0; pass < kMaxDPasses; ++pass) {
    const uint32_t o = (bout | cout | dout) & valid;
    uint32_t ol, orr;
    exchange(o, ol, orr);
    uint32_t nd = dout;
#pragma unroll
    for (int i = 0; i < kNPL; ++i) {
      if (!(valid >> i & 1u)) continue;
      const double ae = fabs(eps[i]);
      if (!(ae - f * G[i] > sigma2)) continue;
      const bool sl = i > 0 ? (o >> (i - 1) & 1u) : ol;
      const double es = i > 0 ? eps[i - 1] : el;
      const bool sr = i < kNPL - 1 ? (o >> (i + 1) & 1u) : orr;
      const double et = i < kNPL - 1 ? eps[i + 1] : er;
      if ((sl && es * eps[i] > 0.0 && ae <= fabs(es)) || (sr && et * eps[i] > 0.0 && ae <= fabs(et)))
        nd |= 1u << i;
    }
    const int changed = __syncthreads_or(nd != dout);
    dout = nd;
    if (!changed) break;
  }

  // outputs: keep flags, the new weights of the fused pass, n_eff
  const uint32_t masked = (bout | cout | dout) & valid;
  if (a.keep_out) {
#pragma unroll
    for (int i = 0; i < kNPL; ++i)
      if (j0 + i < P) a.keep_out[row + j0 + i] = (masked >> i & 1u) ? 0 : 1;
  }
  double cnt[1] = {(double)__popc(valid & ~masked)};
  block_sum_lds<NW, 1>(cnt, sScr, sRed, sOut + 4, lane, wave);
  if (a.s.ow) {
    const float w = a.s.wscale[spec];
    const float w2 = w * w;
    float2 *dst = a.s.ow + (size_t)spec * kNPL * BLOCK + tid;
#pragma unroll
    for (int i = 0; i < kNPL; ++i) {
      const int j = j0 + i;
      if (j < P && (valid >> i & 1u)) dst[i * BLOCK].y = (masked >> i & 1u) ? 0.f : a.ivar[row + j] * w2;
    }
    if (tid == 0) a.s.neff[spec] = (int)sOut[4];
  }
  if (a.masked_out && tid == 0) a.masked_out[spec] = (int)(nv - sOut[4]);
}

}  // namespace

hipError_t launch_clean(const Geometry &g, const CleanArgs &a, hipStream_t st) {
  switch (g.block) {
    case 128: hipLaunchKernelGGL(k_clean<128>, dim3(g.B), dim3(128), 0, st, g, a); break;
    case 256: hipLaunchKernelGGL(k_clean<256>, dim3(g.B), dim3(256), 0, st, g, a); break;
    case 512: hipLaunchKernelGGL(k_clean<512>, dim3(g.B), dim3(512), 0, st, g, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lasp
