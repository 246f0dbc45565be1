// Fused per-spectrum pass of one Adam step (Section 2.2, stages 4-8):
//   Eq. 5  Gaussian kernel G(mu, sigma) and F'' = F' (x) G, F' staged in LDS
//   Eq. 6  continuum by weighted least squares: moments of W F''^2 and
//          W F'' o against Chebyshev polynomials (per-lane FP32 sums over 17
//          pixels, FP64 across lanes), normal equations solved in FP64
//          (Gauss-Jordan, one lane per row)
//   Eq. 7  residual e = o - C F'' (C by Horner in a power series of the
//          pixel offset, re-centred on each lane's pixels);  Eq. 9
//          chi2 = sum W e^2 (per spectrum)
//   adjoint of J = chi2 / n_eff with the continuum at its least-squares
//          value (envelope theorem): g_j = -2 W e C / n_eff, the lag
//          correlation R(m) = sum_j g_j F'_{j-m+M} giving dJ/dmu and
//          dJ/dsigma, and the transposed convolution F-bar' that the
//          backward contraction turns into dJ/du_{1..3}.
//
// The continuum space {polynomials of degree <= D} is spanned here by
// Chebyshev polynomials: the least-squares fit, its residual, chi2 and the
// gradient are the same as with the paper's Legendre basis (only the
// coefficient vector differs), and T_m T_n = (T_{m+n} + T_{|m-n|}) / 2
// turns the Gram matrix into 2D + 1 moments.
//
// One workgroup owns one spectrum; lane l owns pixels [17 l, 17 l + 17) (an
// odd stride, so lanes hit distinct LDS banks).  Taps run in register blocks
// of 8 against a 24-value window.  The lag correlation takes g from
// registers, so the g-bar row the transposed convolution reads replaces F'
// in LDS once F' has been read for the last time.
#include <type_traits>

#include "lasp_internal.h"

namespace lasp {
namespace {

constexpr int kOffF = 16;  // F' column c lives at sF[kOffF + c]
constexpr int kMid = kNPL / 2;  // each lane expands the continuum about its pixel j0 + kMid

// [x^n] T_k(x) for k, n <= 10, from T_k = 2x T_{k-1} - T_{k-2}.
struct ChebPow {
  int c[11][11];
};
constexpr ChebPow make_cheb_pow() {
  ChebPow t{};
  t.c[0][0] = 1;
  t.c[1][1] = 1;
  for (int k = 2; k < 11; ++k)
    for (int n = 0; n <= k; ++n) t.c[k][n] = (n > 0 ? 2 * t.c[k - 1][n - 1] : 0) - t.c[k - 2][n];
  return t;
}
constexpr ChebPow kChebPow = make_cheb_pow();

// LDS of one workgroup.  Row region A holds, in turn, F' (column c at
// kOffF + c) until the lag correlation has read it, then the g-bar row
// (pixel j at 2M + j, j in [-2M, P + 2M + 32), zero outside [0, P)) for the
// transposed convolution, then F-bar' on its way out.  Scratch region B
// holds, in turn, the moments' reduction transposes, the lag correlation's
// per-wave transposes [NW][kTB][64] and wave 0's mu / sigma sums.
struct FusedLayout {
  int a_len;      // floats of region A
  int gb_base;    // 2M: g-bar pixel j at sF[gb_base + j]
  int b_off;      // float offset of region B
  int b_len;      // floats of region B
  int ks;         // taps buffer stride per arm
  int k_off;      // float offset of the taps
  int r_off;      // float offset of per-wave R(m) partials [NW][n_arms][ks]
  int rs_off;     // float offset of R(m) sums [n_arms][ks]
  int d_off;      // byte offset of the double scratch
  int bytes;
};

__host__ __device__ inline FusedLayout fused_layout(const Geometry &g, int nwaves, int nmom_pad) {
  FusedLayout L;
  const int f_len = kOffF + g.ldF + 32;
  const int g_len = g.P + 4 * g.M + 32;
  L.a_len = ((f_len > g_len ? f_len : g_len) + 3) & ~3;
  L.gb_base = 2 * g.M;
  const int mom = nwaves * 8 * 64;                          // FP32 moment transposes
  const int lag = nwaves * kTB * 64;
  const int musig = 2 * (8 * 64 + 8);                     // wave_sum_lds scratch + sums
  L.b_len = mom > lag ? mom : lag;
  if (L.b_len < musig) L.b_len = musig;
  L.b_off = L.a_len;
  L.ks = ((2 * g.M + 1 + 7) & ~7) + 8;
  L.k_off = L.b_off + L.b_len;
  L.r_off = L.k_off + g.n_arms * L.ks;
  L.rs_off = L.r_off + nwaves * g.n_arms * L.ks;
  const int fl_end = L.rs_off + g.n_arms * L.ks;
  L.d_off = ((fl_end * 4) + 15) & ~15;
  // doubles: reduction scratch [nwaves][64], moments [nmom_pad], the
  // continuum's power series [32], scalars [32] (flag, per-arm H and sigma)
  L.bytes = L.d_off + 8 * (nwaves * 64 + nmom_pad + 32 + 32);
  return L;
}

// set_status != 0: this pass evaluates the returned parameters; it replaces
// the evaluation bits (SINGULAR, CONT_NONPOS, SIGMA_FLOOR) of the spectrum's
// status with those of this pass.  0 (the passes of the Adam steps): the
// status is left alone, so a condition seen only on the way does not reach
// the result.
//
// Four waves per SIMD: the register budget is held to 128 per lane, so with
// the LDS above four 256-thread or two 512-thread workgroups share a CU.  The
// price is a few spills: at 3,900 pixels 40 bytes per lane (some of the
// lane's (o/w, W w^2) pairs, parked in scratch between the moments and the
// residual: one store and one load each per pass); measured faster than
// three waves per SIMD without spills, for both pixel counts.
template <int BLOCK, int ND, bool ADJ, bool MULTI>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_fused(
    Geometry g, State s, float *model_out, int set_status) {
  constexpr int NW = BLOCK / 64;
  constexpr int NNU = 2 * ND - 1;  // nu_0 .. nu_{2D}
  constexpr int NMOM = NNU + ND;   // plus r_0 .. r_D
  constexpr int NWIN = kNPL + kTB - 1;
  extern __shared__ __align__(16) unsigned char smem[];
  const FusedLayout L = fused_layout(g, NW, NMOM);
  float *sF = reinterpret_cast<float *>(smem);  // region A
  float *sGb = sF + L.gb_base;  // sGb[j], j in [-2M, P + 2M + 32), once F' is read
  float *sB = sF + L.b_off;     // region B
  float *sK = sF + L.k_off;
  float *sRp = sF + L.r_off;
  float *sRs = sF + L.rs_off;
  float *sRt = sB + (threadIdx.x >> 6) * (kTB * 64);
  double *sRed = reinterpret_cast<double *>(smem + L.d_off);
  double *sMom = sRed + NW * 64;
  double *sBd = sMom + NMOM;  // continuum power series m_n h^n
  double *sScal = sBd + 32;
  int *sHa = reinterpret_cast<int *>(sScal + 16);      // [kMaxArms]
  double *sSp = sScal + 24;                            // [kMaxArms]

  if ((int)blockIdx.x >= work_count(g, s)) return;  // past the active list
  const int spec = work_spec(s, blockIdx.x);
  if (ADJ && !slot_active(s, spec)) return;  // finished slot: no step
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int P = g.P, M = g.M;
  const int j0 = tid * kNPL;           // first pixel (and basis column) of this lane
  // waves whose every lane has kNPL pixels in the row skip the per-pixel
  // range tests: wave-uniform branches
  const bool pix_inside = (__builtin_amdgcn_readfirstlane(wave) + 1) * 64 * kNPL <= g.P;
  auto branch = [](bool c, auto &&f) {
    if (c)
      f(std::true_type{});
    else
      f(std::false_type{});
  };
  const bool has_pix = j0 < P;
  const int jr = has_pix ? j0 : 0;     // window origin kept in range for idle lanes

  // ---- loads: the velocity and width first, then F' and the data, so that
  //      the F' stores below need not wait for the data ---------------------
  const double u4 = (double)s.u[(size_t)spec * kNP + 3];
  const double u5 = (double)s.u[(size_t)spec * kNP + 4];
  // 17 * BLOCK >= ldF, so every thread stages at most five float4 of F'.
  constexpr int kStage = (kNPL * BLOCK / 4 + BLOCK - 1) / BLOCK;
  const int n4 = g.ldF / 4;
  float4 fst[kStage];
  {
    const float4 *src = reinterpret_cast<const float4 *>(s.fp + (size_t)spec * s.fp_stride);
#pragma unroll
    for (int k = 0; k < kStage; ++k) fst[k] = src[min(tid + k * BLOCK, n4 - 1)];
  }
  float2 ow[kNPL];  // (o / w, W w^2), lane-major: coalesced
  {
    const float2 *src = s.ow + (size_t)spec * kNPL * BLOCK + tid;
#pragma unroll
    for (int i = 0; i < kNPL; ++i) ow[i] = src[i * BLOCK];
  }
  // threads past the row store the last float4 again (the same value)
#pragma unroll
  for (int k = 0; k < kStage; ++k)
    *reinterpret_cast<float4 *>(sF + kOffF + 4 * min(tid + k * BLOCK, n4 - 1)) = fst[k];
  for (int q = tid; q < kOffF; q += BLOCK) sF[q] = 0.f;
  for (int q = tid; q < 32; q += BLOCK) sF[kOffF + g.ldF + q] = 0.f;
  for (int q = tid; q < NW * g.n_arms * L.ks; q += BLOCK) sRp[q] = 0.f;

  // ---- Eq. 5 kernel parameters: mu, sigma in pixels, H per arm (FP64) ----
  // Wave 0's serial sections (these taps, the continuum solve, dJ/dmu and
  // dJ/dsigma) run at raised wave priority: the other waves of the
  // workgroup wait on them, the waves of other workgroups do not.
  const double rv = g.rv_lo + (u4 + 1.0) * g.rv_half;
  const double sg = g.sg_lo + (u5 + 1.0) * g.sg_half;
  const double mu = rv * g.inv_scale;
  if (wave == 0) {
    __builtin_amdgcn_s_setprio(3);
    for (int a = 0; a < g.n_arms; ++a) {
      const double seff = g.bare ? sg : sqrt(sg * sg + g.arm_sig2[a]);
      double spx = seff * g.inv_scale;
      if (!(spx >= (double)kSigmaFloorPx)) spx = (double)kSigmaFloorPx;
      double hf = ceil(fabs(mu) + 5.0 * spx);
      if (!(hf <= (double)M)) hf = (double)M;  // also catches NaN
      const int H = (int)hf, T = 2 * H + 1;
      const double inv2s2 = 0.5 / (spx * spx);
      double gv[3];
      double part = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int idx = lane + 64 * k;
        double v = 0.0;
        if (64 * k < T && idx < T) {  // first test is wave uniform
          const double d = (double)(idx - H) - mu;
          v = exp(-d * d * inv2s2);
        }
        gv[k] = v;
        part += v;
      }
      const double inv_sum = 1.0 / wave_sum(part);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int idx = lane + 64 * k;
        if (idx < L.ks) sK[a * L.ks + idx] = (float)(gv[k] * inv_sum);
      }
      if (lane == 0) {
        sHa[a] = H;
        sSp[a] = spx;
      }
    }
  }
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();

  // ---- arms touched by this wave's output pixels (wave uniform) ---------
  constexpr bool multi = MULTI;  // several spectrograph arms
  const int wp0 = wave * 64 * kNPL;
  const int wp1 = min(wp0 + 64 * kNPL, P) - 1;
  int wa_lo = 0, wa_hi = 0;
  for (int a = 1; a < g.n_arms; ++a) {
    if (g.arm_start[a] <= wp0) wa_lo = a;
    if (g.arm_start[a] <= wp1) wa_hi = a;
  }

  // ---- Eq. 5: F''_j = sum_m G(m) F'_{j-m+M} ------------------------------
  float fpp[kNPL];
#pragma unroll
  for (int i = 0; i < kNPL; ++i) fpp[i] = 0.f;
  if (has_pix) {
    for (int a = wa_lo; a <= wa_hi; ++a) {
      const int H = __builtin_amdgcn_readfirstlane(sHa[a]), T = 2 * H + 1;
      const float *K = sK + a * L.ks;
      float acc[kNPL];
#pragma unroll
      for (int i = 0; i < kNPL; ++i) acc[i] = 0.f;
      for (int mb = 0; mb < T; mb += kTB) {
        const float *wsrc = sF + kOffF + j0 + M + H - mb - (kTB - 1);
        float w[NWIN];
#pragma unroll
        for (int q = 0; q < NWIN; ++q) w[q] = wsrc[q];
#pragma unroll
        for (int t = 0; t < kTB; ++t) {
          if (mb + t >= T) break;  // wave uniform: no work on the block's padding
          const float gk = K[mb + t];
#pragma unroll
          for (int i = 0; i < kNPL; ++i) acc[i] = fmaf(gk, w[i - t + kTB - 1], acc[i]);
        }
      }
      if constexpr (!multi) {
#pragma unroll
        for (int i = 0; i < kNPL; ++i) fpp[i] = acc[i];
      } else {
        const int lo = g.arm_start[a], hi = g.arm_start[a + 1];
#pragma unroll
        for (int i = 0; i < kNPL; ++i)
          if (j0 + i >= lo && j0 + i < hi) fpp[i] = acc[i];
      }
    }
  }

  // ---- Eq. 6 moments: nu_l = sum W F''^2 T_l (l <= 2D), r_n = sum W F'' o T_n
  //      (n <= D), in one pass over the lane's pixels with T_0 .. T_D only:
  //      T_{D+k} = 2 T_D T_k - T_{D-k}, so nu_{D+k} = 2 q_k - nu_{D-k} with
  //      q_k = sum W F''^2 T_D T_k (k = 1..D).  Each lane sums its 17 pixels
  //      in FP32, eight lanes' sums are added in FP32 on their way through
  //      LDS; the sums over those groups and the waves, the combination and
  //      the solve are FP64.
  {
    const float two_over_p = 2.f / (float)P;
    const float x0 = fmaf((float)j0, two_over_p, -1.f);
#pragma unroll
    for (int i = 0; i < kNPL; ++i) {
      opaque(fpp[i]);
      opaque(ow[i]);
    }
    float nu[ND], q[ND], rr[ND];  // nu_0..nu_D, q_1..q_D (q[0] unused), r_0..r_D
#pragma unroll
    for (int k = 0; k < ND; ++k) nu[k] = q[k] = rr[k] = 0.f;
#pragma unroll
    for (int i = 0; i < kNPL; ++i) {
      const float x = fmaf((float)i, two_over_p, x0);
      const float wf = ow[i].y * fpp[i];
      const float y = wf * fpp[i];   // W F''^2
      const float z = wf * ow[i].x;  // W F'' o
      const float x2 = x + x;
      float t[ND];  // T_0(x) .. T_D(x)
      t[0] = 1.f;
      t[1] = x;
#pragma unroll
      for (int l = 2; l < ND; ++l) t[l] = fmaf(x2, t[l - 1], -t[l - 2]);
      const float yd = y * t[ND - 1];
      nu[0] += y;
      rr[0] += z;
#pragma unroll
      for (int l = 1; l < ND; ++l) {
        nu[l] = fmaf(y, t[l], nu[l]);
        q[l] = fmaf(yd, t[l], q[l]);
        rr[l] = fmaf(z, t[l], rr[l]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // lane partials in the order nu_0..nu_D, q_1..q_D, r_0..r_D
    float acc[NMOM];
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[k] = nu[k];
#pragma unroll
    for (int k = 1; k < ND; ++k) acc[ND - 1 + k] = q[k];
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[NNU + k] = rr[k];
    block_sum_lds_f32<NW, NMOM>(acc, sB, sRed, sMom, lane, wave);
  }

  // ---- normal equations A b = r (A_mn = (nu_{m+n} + nu_|m-n|)/2), solved
  //      in FP64 by Gauss-Jordan elimination, lane i holding row i.  sMom
  //      holds nu_0..nu_D, then q_1..q_D with nu_{D+k} = 2 q_k - nu_{D-k}.
  if (wave == 0) {
    __builtin_amdgcn_s_setprio(3);
    constexpr int D = ND - 1;
    // nu_0 .. nu_2D mirrored about index D (sNu[D + l] = sNu[D - l] = nu_l),
    // so row i reads nu_{i+n} and nu_{|i-n|} at fixed offsets from sNu + i
    double *sNu = sRed;  // [3 D + 1], free until the residual's chi2 sums
    {
      const int l = min(lane, NNU - 1);
      const double lo = sMom[l], hi = sMom[l <= D ? l : 2 * D - l];
      const double nu = l <= D ? lo : fma(2.0, lo, -hi);
      if (lane < NNU) sNu[D + lane] = nu;
      if (lane >= 1 && lane <= D) sNu[D - lane] = nu;
    }
    // lanes past row D repeat row D; only rows 0..D are read or stored
    const bool row = lane < ND;
    double a[ND + 1];
    a[ND] = sMom[NNU + min(lane, ND - 1)];
    wave_lds_sync();
    {
      const double *nr = sNu + min(lane, ND - 1);
#pragma unroll
      for (int n = 0; n < ND; ++n) a[n] = 0.5 * (nr[D + n] + nr[D - n]);
    }
    // Gauss-Jordan without scaling the pivot rows: row k stays as it is and
    // every other row loses its column-k entry; b_i = a_i[ND] / a_i[i] at
    // the end.  The pivots are those of the scaled form.
    bool ok = true;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      double piv[ND + 1];
#pragma unroll
      for (int n = k; n <= ND; ++n) piv[n] = read_lane(a[n], k);
      ok = ok && (piv[k] > 0.0) && isfinite(piv[k]);
      // 1 / pivot: the hardware estimate and two Newton steps
      double rp = __builtin_amdgcn_rcp(piv[k]);
      rp = fma(rp, fma(-piv[k], rp, 1.0), rp);
      rp = fma(rp, fma(-piv[k], rp, 1.0), rp);
      const double f = lane == k ? 0.0 : a[k] * rp;
#pragma unroll
      for (int n = k + 1; n <= ND; ++n) a[n] = fma(-f, piv[n], a[n]);
    }
    {
      double dg = a[0];
#pragma unroll
      for (int n = 1; n < ND; ++n) dg = lane == n ? a[n] : dg;
      a[ND] = a[ND] / dg;
    }
    // The continuum as a power series in the pixel offset v = j - P/2 from
    // the row's centre: x_j = h v with h = 2 / P, so C = sum_n m_n h^n v^n
    // with m_n = sum_k b_k [x^n] T_k.  b goes through LDS to every lane of
    // the wave, the coefficients m_n h^n back to LDS; each lane re-centres
    // the series on its own pixels below.
    if (row) sBd[16 + lane] = ok ? a[ND] : 0.0;
    wave_lds_sync();
    double bk[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) bk[k] = sBd[16 + k];
    double mm[ND];
#pragma unroll
    for (int n = 0; n < ND; ++n) {
      double m = 0.0;
#pragma unroll
      for (int k = n; k < ND; k += 2) m = fma(bk[k], (double)kChebPow.c[k][n], m);
      mm[n] = m * g.hpow[n];
    }
    if (lane == 0) {
#pragma unroll
      for (int n = 0; n < ND; ++n) sBd[n] = mm[n];
    }
    if (lane == 0) sScal[0] = ok ? 1.0 : 0.0;
    __builtin_amdgcn_s_setprio(0);
  }
  __syncthreads();

  // ---- Eq. 7 residual, Eq. 9 chi2, adjoint seed g = dJ/dF'' ---------------
  const bool ok = __builtin_amdgcn_readfirstlane((int)(sScal[0] != 0.0)) != 0;
  const int n_eff = s.neff[spec];
  const float gscale = n_eff > 0 ? -2.f / (float)n_eff : 0.f;
  const float wsc = s.wscale[spec];
  float gb[kNPL];
  float chi2_part = 0.f;  // this lane's 17 terms; lanes and waves add in FP64
  float cmin = INFINITY;
  {
    // Taylor coefficients of t -> C(x_{j0 + kMid} + h t): the series in v
    // shifted to v0 = j0 + kMid - P/2 by repeated synthetic division (FP64),
    // then evaluated by Horner in FP32 at t = i - kMid, |h t| <= 16 / P.
    float cf[ND];
    {
      double a[ND];
#pragma unroll
      for (int n = 0; n < ND; ++n) a[n] = sBd[n];
      const double v0 = (double)(j0 + kMid) - 0.5 * (double)P;
#pragma unroll
      for (int k = 0; k < ND - 1; ++k)
#pragma unroll
        for (int n = ND - 2; n >= k; --n) a[n] = fma(v0, a[n + 1], a[n]);
#pragma unroll
      for (int n = 0; n < ND; ++n) cf[n] = (float)a[n];
    }
    auto residual = [&](auto inside) {
#pragma unroll
      for (int i = 0; i < kNPL; ++i) {
        const int j = j0 + i;
        const float t = (float)(i - kMid);
        float C = cf[ND - 1];
#pragma unroll
        for (int k = ND - 2; k >= 0; --k) C = fmaf(C, t, cf[k]);
        const float mdl = C * fpp[i];
        const float e = ow[i].x - mdl;
        const float we = ow[i].y * e;
        chi2_part = fmaf(we, e, chi2_part);
        gb[i] = (we * C) * gscale;
        if constexpr (decltype(inside)::value)
          cmin = fminf(cmin, C);
        else
          cmin = fminf(cmin, j < P ? C : INFINITY);
        if (model_out != nullptr) {
          if (j < P) model_out[(size_t)spec * P + j] = mdl * wsc;
        }
      }
    };
    // (the three-arm kernel keeps one copy of the loop: two copies there
    // moved its spills and measured slower)
    if constexpr (MULTI)
      residual(std::false_type{});
    else
      branch(pix_inside, residual);
    if (!ok) {
#pragma unroll
      for (int i = 0; i < kNPL; ++i) gb[i] = 0.f;
    }
  }
  {
    const double cs = wave_sum((double)chi2_part);
    const float cm = wave_min(cmin);
    if (lane == 0) {
      sRed[wave * 64 + 0] = cs;
      sRed[wave * 64 + 1] = (double)cm;
    }
  }
  __syncthreads();
  if (tid == 0) {
    double cs = 0.0, cm = INFINITY;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      cs += sRed[w * 64 + 0];
      cm = fmin(cm, sRed[w * 64 + 1]);
    }
    s.chi2[spec] = cs;
    if (set_status) {
      uint32_t st = s.status[spec] & ~(kStSingular | kStContNonpos | kStSigmaFloor);
      if (!ok) st |= kStSingular;
      if (!(cm > 0.0)) st |= kStContNonpos;
      for (int a = 0; a < g.n_arms; ++a) {
        const double seff = g.bare ? sg : sqrt(sg * sg + g.arm_sig2[a]);
        if (!(seff * g.inv_scale >= (double)kSigmaFloorPx)) st |= kStSigmaFloor;
      }
      s.status[spec] = st;
    }
  }
  if (!ADJ) return;

  // ---- lag correlation R_a(m) = sum_{j in arm a} g_j F'_{j-m+M} ----------
  if (wp0 < P) {
    for (int a = wa_lo; a <= wa_hi; ++a) {
      const int H = __builtin_amdgcn_readfirstlane(sHa[a]), T = 2 * H + 1;
      float gm[kNPL];
      if constexpr (!multi) {
        branch(pix_inside, [&](auto inside) {
#pragma unroll
          for (int i = 0; i < kNPL; ++i)
            gm[i] = (decltype(inside)::value || has_pix) ? gb[i] : 0.f;
        });
      } else {
        const int lo = g.arm_start[a], hi = g.arm_start[a + 1];
#pragma unroll
        for (int i = 0; i < kNPL; ++i)
          gm[i] = (has_pix && j0 + i >= lo && j0 + i < hi) ? gb[i] : 0.f;
      }
      for (int mb = 0; mb < T; mb += kTB) {
        const float *wsrc = sF + kOffF + jr + M + H - mb - (kTB - 1);
        float w[NWIN];
#pragma unroll
        for (int q = 0; q < NWIN; ++q) w[q] = wsrc[q];
        float r[kTB];
#pragma unroll
        for (int t = 0; t < kTB; ++t) {
          float acc = 0.f;
          if (mb + t < T) {  // wave uniform
#pragma unroll
            for (int i = 0; i < kNPL; ++i) acc = fmaf(gm[i], w[i - t + kTB - 1], acc);
          }
          r[t] = acc;
        }
        // wave-wide sums of the kTB partials: transpose through LDS, each
        // group of 8 lanes adds one tap's 64 partials (fixed order)
#pragma unroll
        for (int t = 0; t < kTB; ++t) sRt[t * 64 + lane] = r[t];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        {
          const int tt = lane >> 3, part = lane & 7;
          const float4 x0 = *reinterpret_cast<const float4 *>(sRt + tt * 64 + 8 * part);
          const float4 x1 = *reinterpret_cast<const float4 *>(sRt + tt * 64 + 8 * part + 4);
          float v = ((x0.x + x0.y) + (x0.z + x0.w)) + ((x1.x + x1.y) + (x1.z + x1.w));
          v = group8_sum(v);
          if (part == 0) sRp[(wave * g.n_arms + a) * L.ks + mb + tt] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
  __syncthreads();  // every read of F' is done: region A takes the g-bar row
  branch(pix_inside, [&](auto inside) {
#pragma unroll
    for (int i = 0; i < kNPL; ++i)
      if (decltype(inside)::value || j0 + i < P) sGb[j0 + i] = gb[i];
  });
  for (int q = tid; q < 2 * M; q += BLOCK) sGb[q - 2 * M] = 0.f;
  for (int q = tid; q < 2 * M + 32; q += BLOCK) sGb[P + q] = 0.f;
  for (int q = tid; q < g.n_arms * L.ks; q += BLOCK) {
    float acc = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) acc += sRp[w * g.n_arms * L.ks + q];
    sRs[q] = acc;
  }
  __syncthreads();

  // ---- dJ/dmu, dJ/dsigma per arm and the chain to u4, u5 (wave 0) -------
  if (wave == 0) {
    __builtin_amdgcn_s_setprio(3);
    double g4 = 0.0, g5 = 0.0;
    for (int a = 0; a < g.n_arms; ++a) {
      const int H = __builtin_amdgcn_readfirstlane(sHa[a]), T = 2 * H + 1;
      double s1 = 0, s2 = 0, rg = 0, rgd = 0, rgd2 = 0;
      for (int idx = lane; idx < T; idx += 64) {
        const double d = (double)(idx - H) - mu;
        const double G = (double)sK[a * L.ks + idx];
        const double R = (double)sRs[a * L.ks + idx];
        s1 += G * d;
        s2 += G * d * d;
        rg += R * G;
        rgd += R * G * d;
        rgd2 += R * G * d * d;
      }
      {
        // region B is free once the lag correlation is done
        const double part[5] = {s1, s2, rg, rgd, rgd2};
        double *tot = reinterpret_cast<double *>(sB) + 512;
        wave_sum_lds<5>(part, reinterpret_cast<double *>(sB), tot, lane);
        s1 = tot[0];
        s2 = tot[1];
        rg = tot[2];
        rgd = tot[3];
        rgd2 = tot[4];
      }
      const double sp = sSp[a];
      const double dmu = (rgd - s1 * rg) / (sp * sp);
      const double dsig = (rgd2 - s2 * rg) / (sp * sp * sp);
      g4 += dmu * g.rv_half * g.inv_scale;
      const double seff = g.bare ? sg : sqrt(sg * sg + g.arm_sig2[a]);
      const bool fl = !(seff * g.inv_scale >= (double)kSigmaFloorPx);
      const double dsdu = fl ? 0.0 : g.sg_half * g.inv_scale * (g.bare ? 1.0 : sg / seff);
      g5 += dsig * dsdu;
    }
    if (lane == 0) {
      s.g45[(size_t)spec * 2 + 0] = ok ? (float)g4 : 0.f;
      s.g45[(size_t)spec * 2 + 1] = ok ? (float)g5 : 0.f;
    }
    __builtin_amdgcn_s_setprio(0);
  }

  // ---- transposed convolution F-bar'_c = sum_m G(m) g_{c+m-M} ------------
  const int c0 = j0;
  float fb[kNPL];
#pragma unroll
  for (int i = 0; i < kNPL; ++i) fb[i] = 0.f;
  if (c0 < g.Pe) {
    // arms whose pixels the columns of this wave can reach (wave uniform)
    int ta_lo = 0, ta_hi = 0;
    if constexpr (multi) {
      const int jlo = wave * 64 * kNPL - 2 * M;
      const int jhi = (wave + 1) * 64 * kNPL - 1;
      for (int a = 1; a < g.n_arms; ++a) {
        if (g.arm_start[a] <= jlo) ta_lo = a;
        if (g.arm_start[a] <= jhi) ta_hi = a;
      }
    }
    for (int a = ta_lo; a <= ta_hi; ++a) {
      const int H = __builtin_amdgcn_readfirstlane(sHa[a]), T = 2 * H + 1;
      const float *K = sK + a * L.ks;
      const int lo = multi ? g.arm_start[a] : 0;
      const int hi = multi ? g.arm_start[a + 1] : P;
      for (int mb = 0; mb < T; mb += kTB) {
        const int base = c0 - H + mb - M;
        float w[NWIN];
#pragma unroll
        for (int q = 0; q < NWIN; ++q) w[q] = sGb[base + q];
        if constexpr (multi) {
#pragma unroll
          for (int q = 0; q < NWIN; ++q) w[q] = (base + q >= lo && base + q < hi) ? w[q] : 0.f;
        }
#pragma unroll
        for (int t = 0; t < kTB; ++t) {
          if (mb + t >= T) break;  // wave uniform
          const float gk = K[mb + t];
#pragma unroll
          for (int i = 0; i < kNPL; ++i) fb[i] = fmaf(gk, w[i + t], fb[i]);
        }
      }
    }
  }
  __syncthreads();  // every read of the g-bar row is done: region A takes F-bar'
#pragma unroll
  for (int i = 0; i < kNPL; ++i)
    if (c0 + i < g.ldF) sF[kOffF + c0 + i] = (c0 + i < g.Pe) ? fb[i] : 0.f;
  __syncthreads();
  {
    float4 *dst = reinterpret_cast<float4 *>(s.fbar + (size_t)spec * g.ldF);
    for (int q = tid; q < g.ldF / 4; q += BLOCK)
      dst[q] = *reinterpret_cast<const float4 *>(sF + kOffF + 4 * q);
  }
}

template <int BLOCK, int ND, bool ADJ, bool MULTI>
hipError_t launch_fused_k(const Geometry &g, const State &s, float *model_out, int set_status,
                          hipStream_t st) {
  const FusedLayout L = fused_layout(g, BLOCK / 64, 3 * ND - 1);
  auto k = k_fused<BLOCK, ND, ADJ, MULTI>;
  hipError_t e =
      hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, L.bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(g.B), dim3(BLOCK), L.bytes, st, g, s, model_out, set_status);
  return hipGetLastError();
}

template <int BLOCK, int ND>
hipError_t launch_fused_t(const Geometry &g, const State &s, int adjoint, float *model_out,
                          int set_status, hipStream_t st) {
  const bool multi = g.n_arms > 1;
  if (adjoint)
    return multi ? launch_fused_k<BLOCK, ND, true, true>(g, s, model_out, set_status, st)
                 : launch_fused_k<BLOCK, ND, true, false>(g, s, model_out, set_status, st);
  return multi ? launch_fused_k<BLOCK, ND, false, true>(g, s, model_out, set_status, st)
               : launch_fused_k<BLOCK, ND, false, false>(g, s, model_out, set_status, st);
}

template <int BLOCK>
hipError_t launch_fused_b(const Geometry &g, const State &s, int adjoint, float *model_out,
                          int set_status, hipStream_t st) {
  switch (g.nd) {
    case 5: return launch_fused_t<BLOCK, 5>(g, s, adjoint, model_out, set_status, st);
    case 7: return launch_fused_t<BLOCK, 7>(g, s, adjoint, model_out, set_status, st);
    case 9: return launch_fused_t<BLOCK, 9>(g, s, adjoint, model_out, set_status, st);
    case 11: return launch_fused_t<BLOCK, 11>(g, s, adjoint, model_out, set_status, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool fused_supported(int block, int nd) {
  return (block == 128 || block == 256 || block == 512) &&
         (nd == 5 || nd == 7 || nd == 9 || nd == 11);
}

size_t fused_smem_bytes(const Geometry &g) {
  return (size_t)fused_layout(g, g.block / 64, 3 * g.nd - 1).bytes;
}

hipError_t launch_fused(const Geometry &g, const State &s, int adjoint, float *model_out,
                        int set_status, hipStream_t st) {
  switch (g.block) {
    case 128: return launch_fused_b<128>(g, s, adjoint, model_out, set_status, st);
    case 256: return launch_fused_b<256>(g, s, adjoint, model_out, set_status, st);
    case 512: return launch_fused_b<512>(g, s, adjoint, model_out, set_status, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lasp
