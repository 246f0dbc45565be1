// Parameter covariance at the final point (Section 2.2 stage 9: linear
// error propagation Sigma = s^2 (J^T J)^{-1} with s^2 = chi2 / (n_eff - 5)).
//
// The residual r_j = sqrt(W_j) (o_j - C_j F''_j) depends on the five
// parameters u and on the continuum coefficients b.  The u-block of the
// inverse normal matrix is the inverse of the Schur complement
//   S = Ju^T Ju - Ju^T Jb (Jb^T Jb)^{-1} Jb^T Ju,
// so with Jb^T Jb = A (the continuum Gram matrix) and X = Jb^T Ju only 5x5
// and (D+1)x5 sums are needed.  The five columns dF''/du are formed in
// forward mode: dF''/du_t = G (x) dF'/du_t for t = 1..3 (dF'/du_t from the
// derivative rows of the interpolator contraction) and
// dF''/du_{4,5} = (dG/dmu, dG/dsigma) (x) F' times the chain factors.
// Optionally the model Jacobian d(C F'')/du at fixed continuum is written,
// and the Gauss-Newton normal equations of the profiled residual, S du = q
// with q = Ju^T W e (no continuum term: Jb^T W e = 0 at the least-squares
// continuum), for the Levenberg-Marquardt polish.
#include "lasp_internal.h"

namespace lasp {
namespace {

constexpr int kOffF = 16;

template <int V>
struct IntC {
  static constexpr int value = V;
};

struct CovLayout {
  int ks;
  int k_off;   // floats: taps [n_arms][3][ks]
  int d_off;   // floats: columns dF''/du_{1..3} [3][kNPL * block], lane-major pixels
  int x_off;   // bytes: doubles
  int bytes;
};

// The staged F' row region (floats [0, k_off)) is reused as the reduction
// scratch of block_sum_lds once every convolution is done.
__host__ __device__ inline CovLayout cov_layout(const Geometry &g, int nwaves) {
  CovLayout L;
  int cols = kOffF + (g.ldF > kNPL * g.block ? g.ldF : kNPL * g.block) + 32;
  if (cols < nwaves * 1024) cols = nwaves * 1024;
  L.ks = ((2 * g.M + 1 + 7) & ~7) + 8;
  L.k_off = (cols + 3) & ~3;
  L.d_off = (L.k_off + g.n_arms * 3 * L.ks + 3) & ~3;
  const int fl_end = L.d_off + 3 * kNPL * g.block;
  L.x_off = ((fl_end * 4) + 15) & ~15;
  // doubles: reduction [nwaves][64], moments [64], JuJu + q + chi2 [32],
  // X [16][8], work [64], scalars [16]
  L.bytes = L.x_off + 8 * (nwaves * 64 + 64 + 32 + 128 + 64 + 16);
  return L;
}

// Two waves per SIMD (two workgroups per CU, as the LDS allows) although the
// registers then spill some values to scratch: the measured time per
// launch falls by about a fifth against one wave per SIMD without spills.
template <int BLOCK, int ND>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2))) void k_cov(Geometry g, State s, double blo0, double bhi0,
                                               double blo1, double bhi1, double blo2, double bhi2,
                                               double out_scale3, double out_scale4,
                                               double *out_cov, float *out_jac,
                                               double *out_normal, const int *active) {
  constexpr int NW = BLOCK / 64;
  constexpr int NNU = 2 * ND - 1;
  constexpr int NMOM = NNU + ND;
  constexpr int NWIN = kNPL + kTB - 1;
  constexpr int NCOL = kNPL * BLOCK;  // stride of one staged column
  extern __shared__ __align__(16) unsigned char smem[];
  const CovLayout L = cov_layout(g, NW);
  float *sF = reinterpret_cast<float *>(smem);
  float *sK = sF + L.k_off;
  float *sD = sF + L.d_off;
  double *sRed = reinterpret_cast<double *>(smem + L.x_off);
  double *sMom = sRed + NW * 64;
  double *sJJ = sMom + 64;    // JuJu packed [15], q [5], chi2
  double *sX = sJJ + 32;      // [ND][5]
  double *sW = sX + 128;      // work
  double *sScal = sW + 64;
  float *sBf = reinterpret_cast<float *>(sScal);       // [16] (b as float)
  int *sHa = reinterpret_cast<int *>(sScal + 8);        // [kMaxArms]
  float *sCs = reinterpret_cast<float *>(sScal + 12);   // [kMaxArms] chain factor for sigma

  const int spec = blockIdx.x;
  if (active && !active[spec]) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int P = g.P, M = g.M;
  const int j0 = tid * kNPL;
  const bool has_pix = j0 < P;
  const bool multi = g.n_arms > 1;

  for (int q = tid; q < 3 * NCOL; q += BLOCK) sD[q] = 0.f;

  // ---- taps G, dG/dmu, dG/dsigma per arm ---------------------------------
  const double u4 = (double)s.u[(size_t)spec * kNP + 3];
  const double u5 = (double)s.u[(size_t)spec * kNP + 4];
  const double rv = g.rv_lo + (u4 + 1.0) * g.rv_half;
  const double sg = g.sg_lo + (u5 + 1.0) * g.sg_half;
  const double mu = rv * g.inv_scale;
  const float cmu = (float)(g.rv_half * g.inv_scale);
  if (wave == 0) {
    for (int a = 0; a < g.n_arms; ++a) {
      const double seff = g.bare ? sg : sqrt(sg * sg + g.arm_sig2[a]);
      double spx = seff * g.inv_scale;
      const bool fl = !(spx >= (double)kSigmaFloorPx);
      if (fl) spx = (double)kSigmaFloorPx;
      double hf = ceil(fabs(mu) + 5.0 * spx);
      if (!(hf <= (double)M)) hf = (double)M;
      const int H = (int)hf, T = 2 * H + 1;
      double gv[3], dv[3];
      double part = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int idx = lane + 64 * k;
        double v = 0.0, d = 0.0;
        if (64 * k < T && idx < T) {
          d = (double)(idx - H) - mu;
          v = exp(-d * d / (2.0 * spx * spx));
        }
        gv[k] = v;
        dv[k] = d;
        part += v;
      }
      const double inv_sum = 1.0 / wave_sum(part);
      double s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        gv[k] *= inv_sum;
        s1 += gv[k] * dv[k];
        s2 += gv[k] * dv[k] * dv[k];
      }
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      const double sp = spx;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int idx = lane + 64 * k;
        if (idx < L.ks) {
          const bool in = idx < T;
          sK[(a * 3 + 0) * L.ks + idx] = in ? (float)gv[k] : 0.f;
          sK[(a * 3 + 1) * L.ks + idx] = in ? (float)(gv[k] * (dv[k] - s1) / (sp * sp)) : 0.f;
          sK[(a * 3 + 2) * L.ks + idx] =
              in ? (float)(gv[k] * (dv[k] * dv[k] - s2) / (sp * sp * sp)) : 0.f;
        }
      }
      if (lane == 0) {
        sHa[a] = H;
        sCs[a] = fl ? 0.f : (float)(g.sg_half * g.inv_scale * (g.bare ? 1.0 : sg / seff));
      }
    }
  }

  // ---- forward-mode columns: F'' and dF''/du_t, one staged row at a time.
  //      Row 0 gives F'' and the mu, sigma columns (kept in registers); rows
  //      1..3 give the u1..u3 columns (kept in LDS) -----------------------
  float f[kNPL], d3[kNPL], d4[kNPL];
#pragma unroll
  for (int i = 0; i < kNPL; ++i) f[i] = d3[i] = d4[i] = 0.f;
  const int wp0 = wave * 64 * kNPL;
  const int wp1 = min(wp0 + 64 * kNPL, P) - 1;
  int wa_lo = 0, wa_hi = 0;
  for (int a = 1; a < g.n_arms; ++a) {
    if (g.arm_start[a] <= wp0) wa_lo = a;
    if (g.arm_start[a] <= wp1) wa_hi = a;
  }
  constexpr int kStage = (kNPL * BLOCK / 4 + BLOCK - 1) / BLOCK;
  const int n4 = g.ldF / 4;
  for (int row = 0; row < 4; ++row) {
    __syncthreads();
    {
      const float4 *src = reinterpret_cast<const float4 *>(s.fp + (size_t)spec * s.fp_stride +
                                                           (size_t)row * g.ldF);
      float4 fst[kStage];
#pragma unroll
      for (int k = 0; k < kStage; ++k) fst[k] = src[min(tid + k * BLOCK, n4 - 1)];
#pragma unroll
      for (int k = 0; k < kStage; ++k)
        *reinterpret_cast<float4 *>(sF + kOffF + 4 * min(tid + k * BLOCK, n4 - 1)) = fst[k];
      for (int q = tid; q < kOffF; q += BLOCK) sF[q] = 0.f;
      for (int q = tid; q < 32; q += BLOCK) sF[kOffF + g.ldF + q] = 0.f;
    }
    __syncthreads();
    if (!has_pix) continue;
    for (int a = wa_lo; a <= wa_hi; ++a) {
      const int H = sHa[a], T = 2 * H + 1;
      const int nk = row == 0 ? 3 : 1;
      float acc[3][kNPL];
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int i = 0; i < kNPL; ++i) acc[q][i] = 0.f;
      for (int mb = 0; mb < T; mb += kTB) {
        const float *wsrc = sF + kOffF + j0 + M + H - mb - (kTB - 1);
        float w[NWIN];
#pragma unroll
        for (int q = 0; q < NWIN; ++q) w[q] = wsrc[q];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (q < nk) {
            const float *K = sK + (a * 3 + q) * L.ks;
#pragma unroll
            for (int t = 0; t < kTB; ++t) {
              const float gk = K[mb + t];
#pragma unroll
              for (int i = 0; i < kNPL; ++i) acc[q][i] = fmaf(gk, w[i - t + kTB - 1], acc[q][i]);
            }
          }
        }
      }
      const int lo = multi ? g.arm_start[a] : 0;
      const int hi = multi ? g.arm_start[a + 1] : 0x7fffffff;
      const float cs = sCs[a];
#pragma unroll
      for (int i = 0; i < kNPL; ++i) {
        if (j0 + i >= lo && j0 + i < hi) {
          if (row == 0) {
            f[i] = acc[0][i];
            d3[i] = cmu * acc[1][i];
            d4[i] = cs * acc[2][i];
          } else {
            sD[(row - 1) * NCOL + j0 + i] = acc[0][i];
          }
        }
      }
    }
  }
  // data (lane-major, coalesced)
  float2 ow[kNPL];
  {
    const float2 *src = s.ow + (size_t)spec * kNPL * BLOCK + tid;
#pragma unroll
    for (int i = 0; i < kNPL; ++i) ow[i] = src[i * BLOCK];
  }
  __syncthreads();  // every read of the staged row is done: sF becomes scratch
  double *scratch = reinterpret_cast<double *>(sF);

  // ---- continuum least squares (as in the fused pass): nu_l = sum W F''^2
  //      T_l (l <= 2D) and r_n = sum W F'' o T_n (n <= D) from T_0 .. T_D
  //      only (nu_{D+k} = 2 q_k - nu_{D-k}, q_k = sum W F''^2 T_D T_k); each
  //      lane sums its pixels in FP32, the sums across lanes and waves are
  //      FP64 ------------------------------------------------------------------
  {
    constexpr int D = ND - 1;
    const float two_over_p = 2.f / (float)P;
    float nu[ND], q[ND], rr[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) nu[k] = q[k] = rr[k] = 0.f;
#pragma unroll
    for (int i = 0; i < kNPL; ++i) {
      const float x = fmaf((float)(j0 + i), two_over_p, -1.f);
      const float wf = ow[i].y * f[i];
      const float y = wf * f[i];
      const float z = wf * ow[i].x;
      const float x2 = x + x;
      float t[ND];
      t[0] = 1.f;
      t[1] = x;
#pragma unroll
      for (int l = 2; l < ND; ++l) t[l] = fmaf(x2, t[l - 1], -t[l - 2]);
      const float yd = y * t[D];
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
    float acc[NMOM];  // nu_0..nu_D, q_1..q_D, r_0..r_D
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[k] = nu[k];
#pragma unroll
    for (int k = 1; k < ND; ++k) acc[D + k] = q[k];
#pragma unroll
    for (int k = 0; k < ND; ++k) acc[NNU + k] = rr[k];
    block_sum_lds_f32<NW, NMOM>(acc, reinterpret_cast<float *>(scratch), sRed, sW, lane, wave);
    if (tid < NMOM) sMom[tid] = (tid > D && tid < NNU) ? fma(2.0, sW[tid], -sW[2 * D - tid]) : sW[tid];
    __syncthreads();
  }
  if (wave == 0) {
    double a[ND + 1];
    const bool row = lane < ND;
#pragma unroll
    for (int n = 0; n < ND; ++n) {
      const int dd = lane > n ? lane - n : n - lane;
      a[n] = row ? 0.5 * (sMom[min(lane + n, NNU - 1)] + sMom[min(dd, NNU - 1)]) : 0.0;
    }
    a[ND] = row ? sMom[NNU + min(lane, ND - 1)] : 0.0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      double piv[ND + 1];
#pragma unroll
      for (int n = k; n <= ND; ++n) piv[n] = read_lane(a[n], k);
      ok = ok && (piv[k] > 0.0) && isfinite(piv[k]);
      const double rp = 1.0 / piv[k];
      if (lane == k) {
#pragma unroll
        for (int n = k; n <= ND; ++n) a[n] *= rp;
      } else {
        const double fct = a[k] * rp;
#pragma unroll
        for (int n = k + 1; n <= ND; ++n) a[n] = fma(-fct, piv[n], a[n]);
        a[k] = 0.0;
      }
    }
    if (row) sBf[lane] = ok ? (float)a[ND] : 0.f;
    if (lane == 0) sScal[15] = ok ? 1.0 : 0.0;
  }
  __syncthreads();

  // ---- one pass per pixel: continuum C, residual e, the residual Jacobian
  //      columns ju_t = C dF''/du_t (scaled in place: registers for mu and
  //      sigma, LDS for u1..u3), and Ju^T W Ju (15), q = Ju^T W e (5) and
  //      chi2 in FP64 ------------------------------------------------------
  {
    float c[ND];
#pragma unroll
    for (int k = 0; k < ND; ++k) c[k] = sBf[k];
#pragma unroll
    for (int i = 0; i < kNPL; ++i) {
      opaque(f[i]);
      opaque(ow[i]);
    }
    const float two_over_p = 2.f / (float)P;
    float acc[20];  // Ju^T W Ju packed (15), q = Ju^T W e (5): FP32 per lane
#pragma unroll
    for (int k = 0; k < 20; ++k) acc[k] = 0.f;
    double chi2 = 0.0;
#pragma unroll
    for (int i = 0; i < kNPL; ++i) {
      const float x = fmaf((float)(j0 + i), two_over_p, -1.f);
      float b1 = 0.f, b2 = 0.f;
#pragma unroll
      for (int k = ND - 1; k >= 1; --k) {
        const float bk = fmaf(x + x, b1, c[k] - b2);
        b2 = b1;
        b1 = bk;
      }
      const float C = fmaf(x, b1, c[0] - b2);
      const float e = ow[i].x - C * f[i];
      float dd[kNP];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        // j0 + i < kNPL * BLOCK for every thread; columns are zero where no
        // pixel is
        const float v = sD[t * NCOL + j0 + i] * C;
        sD[t * NCOL + j0 + i] = v;
        dd[t] = v;
      }
      d3[i] *= C;
      d4[i] *= C;
      dd[3] = d3[i];
      dd[4] = d4[i];
      const float w = ow[i].y;
      const float we = w * e;
      int k = 0;
#pragma unroll
      for (int p = 0; p < kNP; ++p) {
        const float wd = w * dd[p];
#pragma unroll
        for (int q = 0; q <= p; ++q) {
          acc[k] = fmaf(wd, dd[q], acc[k]);
          ++k;
        }
      }
#pragma unroll
      for (int p = 0; p < kNP; ++p) acc[15 + p] = fmaf(we, dd[p], acc[15 + p]);
      chi2 = fma((double)ow[i].y * (double)e, (double)e, chi2);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (out_jac && has_pix) {
      const float wsc = s.wscale[spec];
#pragma unroll
      for (int i = 0; i < kNPL; ++i)
        if (j0 + i < P) {
          float *o = out_jac + (size_t)spec * kNP * P + j0 + i;
#pragma unroll
          for (int t = 0; t < 3; ++t) o[(size_t)t * P] = sD[t * NCOL + j0 + i] * wsc;
          o[(size_t)3 * P] = d3[i] * wsc;
          o[(size_t)4 * P] = d4[i] * wsc;
        }
    }
    if (out_cov == nullptr && out_normal == nullptr) return;
    block_sum_lds_f32<NW, 20>(acc, reinterpret_cast<float *>(scratch), sRed, sJJ, lane, wave);
    double c2[1] = {chi2};
    block_sum_lds<NW, 1>(c2, scratch, sRed, sJJ + 20, lane, wave);
  }
  // X[n][t] = Jb^T W Ju = sum W F'' T_n ju_t (Chebyshev T_n), FP32 per lane
  // and FP64 across lanes: one pass for the LDS columns u1..u3 and one for
  // the register columns mu, sigma, T_0 .. T_D formed once per pixel and pass
  // (a pass that picked a register column by a run-time index would make
  // the compiler keep them in memory).
  auto xpass = [&](auto ncol, int t0, auto column) {
    constexpr int NCX = decltype(ncol)::value;
    int jb = j0;
    opaque(jb);
#pragma unroll
    for (int i = 0; i < kNPL; ++i) {
      opaque(f[i]);
      opaque(ow[i]);
    }
    float acc[NCX * ND];  // [column][n]
#pragma unroll
    for (int n = 0; n < NCX * ND; ++n) acc[n] = 0.f;
    const float two_over_p = 2.f / (float)P;
#pragma unroll
    for (int i = 0; i < kNPL; ++i) {
      const float x = fmaf((float)(jb + i), two_over_p, -1.f);
      const float x2 = x + x;
      const float wf = ow[i].y * f[i];
      float v[NCX];
#pragma unroll
      for (int c = 0; c < NCX; ++c) {
        v[c] = wf * column(c, i);
        acc[c * ND] += v[c];
        acc[c * ND + 1] = fmaf(v[c], x, acc[c * ND + 1]);
      }
      float tm = 1.f, tc = x;
#pragma unroll
      for (int n = 2; n < ND; ++n) {
        const float tn = fmaf(x2, tc, -tm);
#pragma unroll
        for (int c = 0; c < NCX; ++c) acc[c * ND + n] = fmaf(v[c], tn, acc[c * ND + n]);
        tm = tc;
        tc = tn;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    block_sum_lds_f32<NW, NCX * ND>(acc, reinterpret_cast<float *>(scratch), sRed, sW, lane, wave);
    if (tid < NCX * ND) sX[(tid % ND) * kNP + t0 + tid / ND] = sW[tid];
    __syncthreads();
  };
  xpass(IntC<3>{}, 0, [&](int c, int i) { return sD[c * NCOL + j0 + i]; });
  xpass(IntC<2>{}, 3, [&](int c, int i) { return c == 0 ? d3[i] : d4[i]; });

  // ---- wave 0: Y = A^{-1} X, S = JuJu - X^T Y, Sigma_u = s^2 S^{-1} --------
  if (wave == 0) {
    constexpr int NC = ND + kNP;
    double a[NC];
    const bool row = lane < ND;
#pragma unroll
    for (int n = 0; n < ND; ++n) {
      const int dd = lane > n ? lane - n : n - lane;
      a[n] = row ? 0.5 * (sMom[min(lane + n, NNU - 1)] + sMom[min(dd, NNU - 1)]) : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kNP; ++t) a[ND + t] = row ? sX[min(lane, ND - 1) * kNP + t] : 0.0;
    bool ok = sScal[15] != 0.0;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
      double piv[NC];
#pragma unroll
      for (int n = k; n < NC; ++n) piv[n] = read_lane(a[n], k);
      ok = ok && (piv[k] > 0.0) && isfinite(piv[k]);
      const double rp = 1.0 / piv[k];
      if (lane == k) {
#pragma unroll
        for (int n = k; n < NC; ++n) a[n] *= rp;
      } else {
        const double fct = a[k] * rp;
#pragma unroll
        for (int n = k + 1; n < NC; ++n) a[n] = fma(-fct, piv[n], a[n]);
        a[k] = 0.0;
      }
    }
    if (row) {
#pragma unroll
      for (int t = 0; t < kNP; ++t) sW[lane * kNP + t] = a[ND + t];  // Y[n][t]
    }
    if (lane == 0) sScal[14] = ok ? 1.0 : 0.0;
  }
  __syncthreads();
  if (wave == 0) {
    bool ok = sScal[14] != 0.0;
    // lanes 0..4 own rows of S, then invert S by Gauss-Jordan on [S | I]
    double sr[2 * kNP];
    const int r = lane < kNP ? lane : 0;
#pragma unroll
    for (int q = 0; q < kNP; ++q) {
      const int p = r > q ? r : q, qq = r > q ? q : r;
      double v = sJJ[p * (p + 1) / 2 + qq];
#pragma unroll
      for (int n = 0; n < ND; ++n) v -= sX[n * kNP + r] * sW[n * kNP + q];
      sr[q] = v;
      sr[kNP + q] = (r == q) ? 1.0 : 0.0;
    }
    if (out_normal && lane < kNP) {
      // Gauss-Newton normal equations of the residual with the continuum
      // profiled out: S du = q (rows of S, then q, then chi2)
      double *o = out_normal + (size_t)spec * kNormalStride;
#pragma unroll
      for (int q = 0; q < kNP; ++q) o[lane * kNP + q] = sr[q];
      o[25 + lane] = sJJ[15 + lane];
      if (lane == 0) o[30] = ok ? sJJ[20] : NAN;
    }
    if (out_cov) {
#pragma unroll
      for (int k = 0; k < kNP; ++k) {
        double piv[2 * kNP];
#pragma unroll
        for (int n = 0; n < 2 * kNP; ++n) piv[n] = read_lane(sr[n], k);
        ok = ok && (piv[k] > 0.0) && isfinite(piv[k]);
        const double rp = 1.0 / piv[k];
        if (lane == k) {
#pragma unroll
          for (int n = 0; n < 2 * kNP; ++n) sr[n] *= rp;
        } else {
          const double fct = sr[k] * rp;
#pragma unroll
          for (int n = 0; n < 2 * kNP; ++n) sr[n] = fma(-fct, piv[n], sr[n]);
        }
      }
      const int n_eff = s.neff[spec];
      const double chi2 = sJJ[20];
      const double s2 = n_eff > kNP ? chi2 / (double)(n_eff - kNP) : NAN;
      if (lane < kNP) {
        // physical units: Teff via dTeff = Teff ln10 dlog10Teff, the others by
        // the box half-widths
        const double lt = blo0 + 0.5 * ((double)s.u[(size_t)spec * kNP] + 1.0) * (bhi0 - blo0);
        double jd[kNP];
        jd[0] = 0.5 * (bhi0 - blo0) * exp10(lt) * kLn10;
        jd[1] = 0.5 * (bhi1 - blo1);
        jd[2] = 0.5 * (bhi2 - blo2);
        jd[3] = out_scale3;
        jd[4] = out_scale4;
        double jr = jd[0];
#pragma unroll
        for (int q = 1; q < kNP; ++q)
          if (q == lane) jr = jd[q];
#pragma unroll
        for (int q = 0; q < kNP; ++q) {
          const double v = ok ? s2 * sr[kNP + q] * jr * jd[q] : NAN;
          out_cov[((size_t)spec * kNP + lane) * kNP + q] = v;
        }
      }
      if (lane == 0 && !ok) s.status[spec] |= kStSingular;
    }
  }
}

template <int BLOCK, int ND>
hipError_t launch_cov_t(const Geometry &g, const State &s, const double *lo, const double *hi,
                        double *out_cov, float *out_jac, double *out_normal, const int *active,
                        hipStream_t st) {
  const CovLayout L = cov_layout(g, BLOCK / 64);
  auto k = k_cov<BLOCK, ND>;
  hipError_t e =
      hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, L.bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(g.B), dim3(BLOCK), L.bytes, st, g, s, lo[0], hi[0], lo[1], hi[1],
                     lo[2], hi[2], 0.5 * (hi[3] - lo[3]), 0.5 * (hi[4] - lo[4]), out_cov, out_jac,
                     out_normal, active);
  return hipGetLastError();
}

template <int BLOCK>
hipError_t launch_cov_b(const Geometry &g, const State &s, const double *lo, const double *hi,
                        double *out_cov, float *out_jac, double *out_normal, const int *active,
                        hipStream_t st) {
  switch (g.nd) {
    case 5: return launch_cov_t<BLOCK, 5>(g, s, lo, hi, out_cov, out_jac, out_normal, active, st);
    case 7: return launch_cov_t<BLOCK, 7>(g, s, lo, hi, out_cov, out_jac, out_normal, active, st);
    case 9: return launch_cov_t<BLOCK, 9>(g, s, lo, hi, out_cov, out_jac, out_normal, active, st);
    case 11:
      return launch_cov_t<BLOCK, 11>(g, s, lo, hi, out_cov, out_jac, out_normal, active, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_cov(const Geometry &g, const State &s, const double *lo, const double *hi,
                      double *out_cov, float *out_jac, double *out_normal, const int *active,
                      hipStream_t st) {
  switch (g.block) {
    case 128: return launch_cov_b<128>(g, s, lo, hi, out_cov, out_jac, out_normal, active, st);
    case 256: return launch_cov_b<256>(g, s, lo, hi, out_cov, out_jac, out_normal, active, st);
    case 512: return launch_cov_b<512>(g, s, lo, hi, out_cov, out_jac, out_normal, active, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lasp
