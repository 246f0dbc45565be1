// C ABI (include/lasp.h): argument validation, cached device scratch and the
// launch sequence of a grouped fit.  Every number is computed by the device
// kernels; this file only checks shapes and enqueues work.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <map>
#include <vector>
#include <mutex>
#include <string>
#include <utility>

#include "lasp.h"
#include "lasp_internal.h"

namespace {

using lasp::Geometry;
using lasp::State;

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int dev_fail(hipError_t e, const char *where) {
  return fail(LASP_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Device scratch of one (device, stream) pair, grown on demand.
struct Workspace {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t cap_B = 0, cap_ow = 0, cap_fp = 0, cap_fbar = 0, cap_basis = 0, cap_hist = 0, cap_lm = 0;
  size_t cap_tsplit = 0;  // entries of the transposed BF16 split basis
  size_t cap_order = 0;
  int *order = nullptr;     // [B] active list of the stopping rules, then its length
  int *h_active = nullptr;  // pinned [2]: lengths read back by the host
  hipEvent_t ev[2] = {nullptr, nullptr};
  size_t cap_model = 0;
  float *model = nullptr;  // [B][P] model for the Clean updates
  State s{};
  lasp::LmState lm{};
  // a chunk of plain Adam steps as one HIP graph (lasp_fit_group), with the
  // bytes of the arguments it was captured with
  hipStream_t cap_st = nullptr;  // capture only: nothing runs on it
  hipGraphExec_t steps_exec = nullptr;
  std::vector<unsigned char> steps_key;
};

std::mutex g_mu;
std::map<std::pair<int, void *>, Workspace *> g_ws;

template <typename T>
hipError_t grow(T *&p, size_t &cap, size_t need) {
  if (need <= cap && p != nullptr) return hipSuccess;
  if (p) {
    hipError_t e = hipFree(p);
    if (e != hipSuccess) return e;
    p = nullptr;
    cap = 0;
  }
  hipError_t e = hipMalloc((void **)&p, need * sizeof(T) + 256);
  if (e == hipSuccess) cap = need;
  return e;
}

void free_ws(Workspace *w) {
  State &s = w->s;
  void *ptrs[] = {s.u,        s.m,        s.v,        s.t,       s.target, s.nrise, s.lhist,
                  s.ow,       s.wscale,   s.neff,     s.status,  s.fp,     s.fbar,  s.g45,
                  s.chi2,     s.basis,    s.basis_hi, s.basis_lo, s.basis_thi, s.basis_tlo};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  lasp::LmState &l = w->lm;
  void *lptrs[] = {l.normal, l.lambda, l.chi2_trial, l.step_inf, l.u_trial, l.st_trial,
                   l.need_jac, l.flags};
  for (void *p : lptrs)
    if (p) (void)hipFree(p);
  if (w->model) (void)hipFree(w->model);
  w->model = nullptr;
  w->cap_model = 0;
  if (w->order) (void)hipFree(w->order);
  w->order = nullptr;
  w->cap_order = 0;
  if (w->h_active) (void)hipHostFree(w->h_active);
  w->h_active = nullptr;
  for (hipEvent_t &e : w->ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (w->steps_exec) (void)hipGraphExecDestroy(w->steps_exec);
  w->steps_exec = nullptr;
  w->steps_key.clear();
  if (w->cap_st) (void)hipStreamDestroy(w->cap_st);
  w->cap_st = nullptr;
  w->s = State{};
  w->lm = lasp::LmState{};
  w->cap_B = w->cap_ow = w->cap_fp = w->cap_fbar = w->cap_basis = w->cap_hist = w->cap_lm = 0;
  w->cap_tsplit = 0;
}

// Grows the buffers of w to hold g.B spectra of geometry g (fp_rows rows of F'
// per spectrum, a loss history of hist_w entries when the stopping rules are
// on).  Earlier work on the stream may still use old buffers, so the stream
// is synchronised before anything is freed.
int ensure_buffers(Workspace *w, const Geometry &g, int fp_rows, int hist_w, hipStream_t st,
                   bool lm = false, bool want_order = false) {
  const size_t B = (size_t)g.B;
  const size_t need_hist = B * (size_t)hist_w;
  const size_t need_lm = lm ? B : 0;
  const size_t need_ow = B * lasp::kNPL * g.block;
  const size_t need_fp = B * fp_rows * g.ldF;
  const size_t need_fbar = B * g.ldF;
  const size_t need_basis = (size_t)g.nb * g.ldF;
  const size_t need_tsplit = (size_t)32 * g.ldF;
  const size_t need_order = (hist_w > 0 || want_order) ? B + 1 : 0;
  const bool regrow = B > w->cap_B || need_ow > w->cap_ow || need_fp > w->cap_fp ||
                      need_fbar > w->cap_fbar || need_basis > w->cap_basis ||
                      need_tsplit > w->cap_tsplit || need_order > w->cap_order ||
                      need_hist > w->cap_hist || need_lm > w->cap_lm || !w->s.u;
  if (!regrow) return LASP_OK;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return dev_fail(e, "hipStreamSynchronize");
  State &s = w->s;
  const size_t cb = w->cap_B;
  size_t c1 = cb, c2 = cb, c3 = cb, c4 = cb, c5 = cb, c6 = cb, c7 = cb, c8 = cb, c9 = cb;
  size_t c10 = cb, c11 = cb;
  hipError_t r = hipSuccess;
  if (B > cb || !s.u) {
    r = grow(s.u, c1, B * lasp::kNP);
    if (r == hipSuccess) r = grow(s.m, c2, B * lasp::kNP);
    if (r == hipSuccess) r = grow(s.v, c3, B * lasp::kNP);
    if (r == hipSuccess) r = grow(s.t, c4, B);
    if (r == hipSuccess) r = grow(s.wscale, c5, B);
    if (r == hipSuccess) r = grow(s.neff, c6, B);
    if (r == hipSuccess) r = grow(s.status, c7, B);
    if (r == hipSuccess) r = grow(s.g45, c8, B * 2);
    if (r == hipSuccess) r = grow(s.chi2, c9, B);
    if (r == hipSuccess) r = grow(s.target, c10, B);
    if (r == hipSuccess) r = grow(s.nrise, c11, B);
    if (r == hipSuccess) w->cap_B = B;
  }
  if (r == hipSuccess && need_hist > 0) r = grow(s.lhist, w->cap_hist, need_hist);
  if (r == hipSuccess && need_order > 0) r = grow(w->order, w->cap_order, need_order);
  if (r == hipSuccess && need_lm > w->cap_lm) {
    lasp::LmState &l = w->lm;
    const size_t cl = w->cap_lm;
    size_t a1 = cl, a2 = cl, a3 = cl, a4 = cl, a5 = cl, a6 = cl, a7 = cl, a8 = cl;
    r = grow(l.normal, a1, need_lm * lasp::kNormalStride);
    if (r == hipSuccess) r = grow(l.lambda, a2, need_lm);
    if (r == hipSuccess) r = grow(l.chi2_trial, a3, need_lm);
    if (r == hipSuccess) r = grow(l.step_inf, a4, need_lm);
    if (r == hipSuccess) r = grow(l.u_trial, a5, need_lm * lasp::kNP);
    if (r == hipSuccess) r = grow(l.st_trial, a6, need_lm);
    if (r == hipSuccess) r = grow(l.need_jac, a7, need_lm);
    if (r == hipSuccess) r = grow(l.flags, a8, need_lm + 1);
    if (r == hipSuccess) {
      l.active = l.flags + need_lm;
      w->cap_lm = need_lm;
    }
  }
  if (r == hipSuccess) r = grow(s.ow, w->cap_ow, need_ow);
  if (r == hipSuccess) r = grow(s.fp, w->cap_fp, need_fp);
  if (r == hipSuccess) r = grow(s.fbar, w->cap_fbar, need_fbar);
  if (r == hipSuccess) {
    size_t cap = w->cap_basis, cap2 = w->cap_basis, cap3 = w->cap_basis;
    r = grow(s.basis, cap, need_basis);
    if (r == hipSuccess) r = grow(s.basis_hi, cap2, need_basis);
    if (r == hipSuccess) r = grow(s.basis_lo, cap3, need_basis);
    if (r == hipSuccess) w->cap_basis = cap;
  }
  if (r == hipSuccess) {
    size_t cap4 = w->cap_tsplit, cap5 = w->cap_tsplit;
    r = grow(s.basis_thi, cap4, need_tsplit);
    if (r == hipSuccess) r = grow(s.basis_tlo, cap5, need_tsplit);
    if (r == hipSuccess) w->cap_tsplit = cap4;
  }
  if (r != hipSuccess) {
    free_ws(w);
    (void)hipGetLastError();
    return fail(r == hipErrorOutOfMemory ? LASP_E_NOMEM : LASP_E_DEVICE,
                std::string("device allocation: ") + hipGetErrorString(r));
  }
  return LASP_OK;
}

int get_workspace(const Geometry &g, int fp_rows, int hist_w, hipStream_t st, Workspace **out,
                  bool lm = false, bool want_order = false) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, (void *)st);
  Workspace *w = g_ws[key];
  if (!w) {
    w = new Workspace();
    w->device = dev;
    w->stream = st;
    g_ws[key] = w;
  }
  int rc = ensure_buffers(w, g, fp_rows, hist_w, st, lm, want_order);
  if (rc) return rc;
  *out = w;
  return LASP_OK;
}

// Per-spectrum pointers shifted to start at slot0 (fp_rows rows of F' each).
State offset_state(const State &s, const Geometry &g, int slot0, int fp_rows, int hist_w) {
  State o = s;
  const size_t k = (size_t)slot0;
  o.u += k * lasp::kNP;
  o.m += k * lasp::kNP;
  o.v += k * lasp::kNP;
  o.t += k;
  if (o.target) o.target += k;
  if (o.nrise) o.nrise += k;
  if (o.lhist) o.lhist += k * (size_t)hist_w;
  o.ow += k * lasp::kNPL * g.block;
  o.wscale += k;
  o.neff += k;
  o.status += k;
  o.g45 += 2 * k;
  o.chi2 += k;
  o.fp += k * fp_rows * g.ldF;
  o.fbar += k * g.ldF;
  return o;
}

// Validates options and the wavelength grid and fills the geometry.
int make_geometry(const lasp_opts *o, const double *wave_grid, Geometry *g) {
  if (!o) return fail(LASP_E_ARG, "opts is NULL");
  if (o->n_spec < 0) return fail(LASP_E_ARG, "n_spec < 0");
  if (o->n_pix < 32) return fail(LASP_E_ARG, "n_pix must be >= 32");
  if (o->n_classes != 1 && o->n_classes != LASP_MAX_CLASSES)
    return fail(LASP_E_ARG, "n_classes must be 1 or 3");
  if (o->n_basis != LASP_N_BASIS * o->n_classes)
    return fail(LASP_E_ARG, "n_basis must be 20 * n_classes");
  if (o->n_classes > 1) {
    for (int i = 0; i < 4; ++i)
      if (!(o->class_edges[i] > 0.0) || !isfinite(o->class_edges[i]) ||
          (i > 0 && !(o->class_edges[i] > o->class_edges[i - 1])))
        return fail(LASP_E_ARG, "class_edges must be positive, finite and increasing");
    if (o->precision != LASP_PREC_FP32)
      return fail(LASP_E_UNSUPPORTED, "more than one emulator class needs LASP_PREC_FP32");
  }
  if (o->margin < 1 || o->margin > 80) return fail(LASP_E_ARG, "margin must be in [1, 80]");
  if (!(o->degree == 4 || o->degree == 6 || o->degree == 8 || o->degree == 10))
    return fail(LASP_E_UNSUPPORTED, "degree must be one of 4, 6, 8, 10");
  if (o->precision != LASP_PREC_FP32 && o->precision != LASP_PREC_BF16X3)
    return fail(LASP_E_UNSUPPORTED, "precision must be LASP_PREC_FP32 or LASP_PREC_BF16X3");
  for (int t = 0; t < LASP_N_PAR; ++t)
    if (!(o->box_hi[t] > o->box_lo[t]) || !isfinite(o->box_lo[t]) || !isfinite(o->box_hi[t]))
      return fail(LASP_E_ARG, "box_hi must exceed box_lo (finite)");
  if (!(o->lr > 0.f) || !(o->beta1 >= 0.f && o->beta1 < 1.f) || !(o->beta2 >= 0.f && o->beta2 < 1.f) ||
      !(o->eps > 0.f))
    return fail(LASP_E_ARG, "invalid Adam hyper-parameters");
  if (o->n_arms < 0 || o->n_arms > LASP_MAX_ARMS) return fail(LASP_E_ARG, "n_arms must be 0..4");
  if (o->stop_window < 0 || o->stop_window > lasp::kMaxStopWindow)
    return fail(LASP_E_ARG, "stop_window must be in [0, 4096]");
  if (!(o->stop_tol >= 0.f) || !std::isfinite(o->stop_tol))
    return fail(LASP_E_ARG, "stop_tol must be finite and >= 0");
  if (o->polish_iters < 0 || o->polish_iters > 1000)
    return fail(LASP_E_ARG, "polish_iters must be in [0, 1000]");
  if (o->clean_every < 0 || o->clean_max < 0)
    return fail(LASP_E_ARG, "clean_every and clean_max must be >= 0");
  if (!wave_grid) return fail(LASP_E_ARG, "wave_grid is NULL");

  const int P = o->n_pix;
  for (int j = 0; j < P; ++j)
    if (!(wave_grid[j] > 0.0) || !isfinite(wave_grid[j]))
      return fail(LASP_E_GRID, "wave_grid must be positive and finite");
  const double dl = log10(wave_grid[P - 1] / wave_grid[0]) / (double)(P - 1);
  if (!(dl > 0.0)) return fail(LASP_E_GRID, "wave_grid must increase");
  for (int j = 0; j + 1 < P; ++j) {
    const double st = log10(wave_grid[j + 1] / wave_grid[j]);
    if (fabs(st - dl) > 1e-6 * dl) {
      char buf[160];
      snprintf(buf, sizeof buf, "wave_grid not uniform in log10 at pixel %d (step %.9g vs %.9g)", j,
               st, dl);
      return fail(LASP_E_GRID, buf);
    }
  }

  memset(g, 0, sizeof(*g));
  g->B = o->n_spec;
  g->P = P;
  g->M = o->margin;
  g->Pe = P + 2 * o->margin;
  g->ldF = (g->Pe + 127) & ~127;
  g->nd = o->degree + 1;
  g->block = 0;
  for (int b : {128, 256, 512})
    if (lasp::kNPL * b >= g->ldF) {
      g->block = b;
      break;
    }
  if (!g->block) return fail(LASP_E_UNSUPPORTED, "n_pix + 2*margin exceeds 8704");
  if (o->n_arms == 0) {
    g->n_arms = 1;
    g->bare = 1;
    g->arm_start[0] = 0;
    g->arm_start[1] = P;
  } else {
    g->n_arms = o->n_arms;
    g->bare = 0;
    if (o->arm_start[0] != 0) return fail(LASP_E_ARG, "arm_start[0] must be 0");
    for (int a = 0; a < o->n_arms; ++a) {
      if (a > 0 && o->arm_start[a] <= o->arm_start[a - 1])
        return fail(LASP_E_ARG, "arm_start must increase");
      if (o->arm_start[a] >= P) return fail(LASP_E_ARG, "arm_start beyond n_pix");
      if (!(o->arm_sigma_kms[a] >= 0.f) || !isfinite(o->arm_sigma_kms[a]))
        return fail(LASP_E_ARG, "arm_sigma_kms must be finite and >= 0");
      g->arm_start[a] = o->arm_start[a];
      g->arm_sig2[a] = (double)o->arm_sigma_kms[a] * (double)o->arm_sigma_kms[a];
    }
    g->arm_start[o->n_arms] = P;
  }
  g->inv_scale = 1.0 / (lasp::kCkms * lasp::kLn10 * dl);
  g->hpow[0] = 1.0;
  for (int n = 1; n < 11; ++n) g->hpow[n] = g->hpow[n - 1] * (2.0 / (double)P);
  g->rv_lo = o->box_lo[3];
  g->rv_half = 0.5 * (o->box_hi[3] - o->box_lo[3]);
  g->sg_lo = o->box_lo[4];
  g->sg_half = 0.5 * (o->box_hi[4] - o->box_lo[4]);
  g->n_classes = o->n_classes;
  g->nb = lasp::kNB * o->n_classes;
  g->lt_lo = o->box_lo[0];
  g->lt_half = 0.5 * (o->box_hi[0] - o->box_lo[0]);
  for (int i = 0; i < 4; ++i) g->edges[i] = o->class_edges[i];
  if (lasp::fused_smem_bytes(*g) > 160 * 1024)
    return fail(LASP_E_UNSUPPORTED, "shape needs more LDS than a workgroup has");
  return LASP_OK;
}

// Copies the caller's basis into the zero-padded [nb][ldF] layout.
__global__ void k_copy_basis(const float *src, float *dst, int Pe, int ldF) {
  const int k = blockIdx.y;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ldF; c += gridDim.x * blockDim.x)
    dst[(size_t)k * ldF + c] = c < Pe ? src[(size_t)k * Pe + c] : 0.f;
}

int copy_basis(const Geometry &g, const State &s, const float *basis, int bf16x3,
               hipStream_t st) {
  hipLaunchKernelGGL(k_copy_basis, dim3((g.ldF + 255) / 256, g.nb), dim3(256), 0, st, basis,
                     s.basis, g.Pe, g.ldF);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && bf16x3) e = lasp::launch_split_basis(g, s, st);
  return e == hipSuccess ? LASP_OK : dev_fail(e, "copy basis");
}

// ---- optional kernel timing (lasp_profile_*) ------------------------------
struct ProfRecord {
  int cls;
  hipEvent_t beg, end;
};
// Launches may come from several host threads (the server's worker among
// them): the event lists are guarded by g_prof_mu.
std::atomic<uint32_t> g_prof_mask{0};
std::mutex g_prof_mu;
std::vector<ProfRecord> g_prof;       // recorded, not yet read
std::vector<hipEvent_t> g_event_pool;  // free events
double g_prof_ms[LASP_NK];
int64_t g_prof_n[LASP_NK];

hipEvent_t pool_event() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events when its class is being timed.
struct ProfScope {
  int cls;
  hipStream_t st;
  hipEvent_t beg = nullptr;
  ProfScope(int c, hipStream_t s) : cls(c), st(s) {
    if (g_prof_mask & (1u << c)) {
      beg = pool_event();
      if (beg) (void)hipEventRecord(beg, st);
    }
  }
  ~ProfScope() {
    if (!beg) return;
    hipEvent_t end = pool_event();
    if (!end) return;
    (void)hipEventRecord(end, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back(ProfRecord{cls, beg, end});
  }
};

void prof_drain() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto &r : g_prof) {
    float ms = 0.f;
    if (hipEventSynchronize(r.end) == hipSuccess && hipEventElapsedTime(&ms, r.beg, r.end) == hipSuccess) {
      g_prof_ms[r.cls] += ms;
      g_prof_n[r.cls] += 1;
    }
    g_event_pool.push_back(r.beg);
    g_event_pool.push_back(r.end);
  }
  g_prof.clear();
}

#define LASP_TIMED(cls, st) ProfScope prof_scope_##__LINE__((cls), (st))

// Steps between two compactions of the active list (stopping rules on).
constexpr int kCompactEvery = 16;
// Polish iterations between two counts of the spectra still iterating.
constexpr int kLmCheckEvery = 4;

#define LASP_CHECK(call, what)                 \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) return dev_fail(e_, what); \
  } while (0)

// Launch sequence of a forward evaluation at fixed u on the buffers of s
// (fp rows: 4 when the Jacobian or covariance is wanted, else 1).
int forward_enqueue(const Geometry &g, State s, const float *obs, const float *ivar,
                    const float *basis, const float *u, float *out_model, double *out_chi2,
                    float *out_J, int32_t *out_neff, float *out_grad, float *out_jac,
                    double *out_cov, const lasp_opts *opts) {
  hipStream_t st = (hipStream_t)opts->stream;
  const bool rows4 = out_jac || out_cov;
  s.target = nullptr;
  const int bf16 = opts->precision == LASP_PREC_BF16X3;
  int rc = copy_basis(g, s, basis, bf16, st);
  if (rc) return rc;
  {
    LASP_TIMED(LASP_K_PREPARE, st);
    LASP_CHECK(lasp::launch_prepare(g, s, obs, ivar, nullptr, opts->box_lo, opts->box_hi,
                                    opts->weight_quantile, 0, 0, st),
               "prepare");
  }
  LASP_CHECK(hipMemcpyAsync(s.u, u, sizeof(float) * lasp::kNP * g.B, hipMemcpyDeviceToDevice, st),
             "copy u");
  s.fp_stride = rows4 ? 4 * g.ldF : g.ldF;
  {
    LASP_TIMED(LASP_K_INTERP_FWD, st);
    LASP_CHECK(lasp::launch_interp_fwd(g, s, rows4 ? 1 : 0, bf16, st), "interpolator contraction");
  }
  {
    LASP_TIMED(LASP_K_FUSED, st);
    LASP_CHECK(lasp::launch_fused(g, s, out_grad ? 1 : 0, out_model, 1, st), "fused pass");
  }
  if (out_grad) {
    LASP_TIMED(LASP_K_INTERP_BWD, st);
    LASP_CHECK(lasp::launch_interp_bwd(g, s, nullptr, out_grad, bf16, st), "adjoint contraction");
  }
  if (rows4) {
    LASP_TIMED(LASP_K_COV, st);
    LASP_CHECK(lasp::launch_cov(g, s, opts->box_lo, opts->box_hi, out_cov, out_jac, nullptr, nullptr, st),
               "covariance / model Jacobian");
  }
  LASP_CHECK(lasp::launch_outputs(g, s, out_chi2, out_J, out_neff, opts->status, st), "outputs");
  return LASP_OK;
}

// ---- fixed scratch of the allocation-free forward evaluation ----------------
// One array per device, held from the library's first kernel launch on that
// device until the process ends.  Host code never passes the array's name to
// a kernel or a copy: it passes the device address that hipGetSymbolAddress
// returns for the current device.
constexpr size_t kScratchBytes = LASP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch array (looked up once per
// device, with that device current).
int scratch_address(unsigned char **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(LASP_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return dev_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
  }
  *out = g_scratch_ptr[dev];
  return LASP_OK;
}

// Lays the buffers of a forward evaluation (fp_rows rows of F' per spectrum)
// out back to back from base, each 256-byte aligned, and returns the bytes
// they take; base == nullptr only measures.
size_t carve_forward_state(const Geometry &g, int fp_rows, int bf16, unsigned char *base,
                           State *s) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void * {
    void *p = base ? (void *)(base + off) : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  const size_t B = (size_t)g.B, ld = (size_t)g.ldF;
  *s = State{};
  s->u = (float *)take(B * lasp::kNP * sizeof(float));
  s->m = (float *)take(B * lasp::kNP * sizeof(float));
  s->v = (float *)take(B * lasp::kNP * sizeof(float));
  s->t = (int *)take(B * sizeof(int));
  s->wscale = (float *)take(B * sizeof(float));
  s->neff = (int *)take(B * sizeof(int));
  s->status = (uint32_t *)take(B * sizeof(uint32_t));
  s->g45 = (float *)take(B * 2 * sizeof(float));
  s->chi2 = (double *)take(B * sizeof(double));
  s->ow = (float2 *)take(B * lasp::kNPL * g.block * sizeof(float2));
  s->fp = (float *)take(B * fp_rows * ld * sizeof(float));
  s->fbar = (float *)take(B * ld * sizeof(float));
  s->basis = (float *)take((size_t)g.nb * ld * sizeof(float));
  if (bf16) {
    s->basis_hi = (uint16_t *)take((size_t)g.nb * ld * sizeof(uint16_t));
    s->basis_lo = (uint16_t *)take((size_t)g.nb * ld * sizeof(uint16_t));
    s->basis_thi = (uint16_t *)take((size_t)32 * ld * sizeof(uint16_t));
    s->basis_tlo = (uint16_t *)take((size_t)32 * ld * sizeof(uint16_t));
  }
  return off;
}

// Adam steps per replay of the cached step graph, and the largest group that
// uses it: beyond that each step's kernels run long enough that launching
// them one by one costs nothing (the replay measured 0.4 % slower at 16,384
// spectra, 6 % faster for one spectrum).
constexpr int kGraphSteps = 25;
constexpr int kGraphMaxSpectra = 4096;

// Enqueues chunks x kGraphSteps plain Adam steps (interpolator contraction,
// fused pass, adjoint contraction + Adam; no stopping rules, one emulator
// class, no Clean) on st as replays of one HIP graph.  The graph is captured
// on the workspace's own stream (nothing runs there) and kept until the
// arguments change: the kernels take (g, s, adam, bf16) by value, so equal
// bytes of those mean an equal launch sequence.  The graph holds kernel
// nodes only.
int replay_steps(Workspace *w, const Geometry &g, const State &s, const lasp::AdamCfg &adam,
                 int bf16, int chunks, hipStream_t st) {
  std::vector<unsigned char> key(sizeof(Geometry) + sizeof(State) + sizeof(adam) + sizeof(int));
  unsigned char *k = key.data();
  memcpy(k, &g, sizeof(Geometry));
  memcpy(k + sizeof(Geometry), &s, sizeof(State));
  memcpy(k + sizeof(Geometry) + sizeof(State), &adam, sizeof(adam));
  memcpy(k + sizeof(Geometry) + sizeof(State) + sizeof(adam), &bf16, sizeof(int));
  if (!w->steps_exec || w->steps_key != key) {
    if (w->steps_exec) (void)hipGraphExecDestroy(w->steps_exec);
    w->steps_exec = nullptr;
    w->steps_key.clear();
    hipError_t e = hipSuccess;
    if (!w->cap_st) e = hipStreamCreateWithFlags(&w->cap_st, hipStreamNonBlocking);
    if (e != hipSuccess) return dev_fail(e, "step graph stream");
    e = hipStreamBeginCapture(w->cap_st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return dev_fail(e, "step graph capture");
    hipError_t le = hipSuccess;
    for (int it = 0; it < kGraphSteps && le == hipSuccess; ++it) {
      le = lasp::launch_interp_fwd(g, s, 0, bf16, w->cap_st);
      if (le == hipSuccess) le = lasp::launch_fused(g, s, 1, nullptr, 0, w->cap_st);
      if (le == hipSuccess) le = lasp::launch_interp_bwd(g, s, &adam, nullptr, bf16, w->cap_st);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(w->cap_st, &graph);
    if (le != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return dev_fail(le != hipSuccess ? le : e, "step graph capture");
    }
    e = hipGraphInstantiate(&w->steps_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      w->steps_exec = nullptr;
      (void)hipGetLastError();
      return dev_fail(e, "step graph instantiation");
    }
    w->steps_key = key;
  }
  for (int c = 0; c < chunks; ++c) {
    hipError_t e = hipGraphLaunch(w->steps_exec, st);
    if (e != hipSuccess) return dev_fail(e, "step graph launch");
  }
  return LASP_OK;
}

__global__ void k_zero16(uint4 *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

namespace lasp {
int set_error(int code, const char *msg) { return fail(code, msg ? msg : ""); }
}  // namespace lasp

extern "C" {

void lasp_default_opts(lasp_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->n_basis = LASP_N_BASIS;
  o->margin = 64;
  o->degree = 10;
  o->precision = LASP_PREC_FP32;
  const double lo[5] = {log10(4000.0), 1.0, -2.5, -300.0, 50.0};
  const double hi[5] = {log10(8000.0), 5.0, 0.5, 300.0, 150.0};
  for (int t = 0; t < 5; ++t) {
    o->box_lo[t] = lo[t];
    o->box_hi[t] = hi[t];
  }
  o->lr = 1e-2f;
  o->beta1 = 0.9f;
  o->beta2 = 0.999f;
  o->eps = 1e-8f;
  o->weight_quantile = 0.5f;
  o->stop_window = 0;
  o->stop_tol = 1e-5f;
  o->clean_max = 11;
  o->n_classes = 1;
  const double edges[4] = {4000.0, 4550.0, 7000.0, 9000.0};
  for (int i = 0; i < 4; ++i) o->class_edges[i] = edges[i];
  o->step_graph = 1;
}

const char *lasp_last_error(void) { return g_err.c_str(); }

int lasp_profile_enable(uint32_t mask) {
  prof_drain();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int k = 0; k < LASP_NK; ++k) {
    g_prof_ms[k] = 0.0;
    g_prof_n[k] = 0;
  }
  g_prof_mask = mask;
  return LASP_OK;
}

int lasp_profile_read(double *total_ms, int64_t *launches, int32_t n) {
  if (n < 0 || n > LASP_NK || (n > 0 && (!total_ms || !launches)))
    return fail(LASP_E_ARG, "lasp_profile_read: bad arguments");
  prof_drain();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int k = 0; k < n; ++k) {
    total_ms[k] = g_prof_ms[k];
    launches[k] = g_prof_n[k];
  }
  return LASP_OK;
}

void lasp_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto &kv : g_ws) {
    Workspace *w = kv.second;
    (void)hipSetDevice(w->device);
    (void)hipStreamSynchronize(w->stream);
    free_ws(w);
    delete w;
  }
  g_ws.clear();
  (void)hipSetDevice(cur);
}

int lasp_fit_group(const float *obs, const float *ivar, const double *wave_grid, const float *basis,
                   const float *init_params, float *out_params, double *out_cov, int32_t n_steps,
                   const lasp_opts *opts) {
  g_err.clear();
  Geometry g;
  int rc = make_geometry(opts, wave_grid, &g);
  if (rc) return rc;
  if (!obs || !ivar || !basis || !init_params || !out_params)
    return fail(LASP_E_ARG, "obs, ivar, basis, init_params and out_params are required");
  if (n_steps < 0) return fail(LASP_E_ARG, "n_steps < 0");
  if (g.B == 0) return LASP_OK;
  hipStream_t st = (hipStream_t)opts->stream;
  Workspace *w = nullptr;
  const int W = opts->stop_window;
  const int polish = opts->polish_iters;
  const int ce = opts->clean_every, cm = opts->clean_max;
  // several emulator classes: the work list also groups the spectra by Teff
  // regime (tiles of one regime skip the other classes' products)
  const bool regimes = g.n_classes > 1;
  rc = get_workspace(g, (out_cov || polish) ? 4 : 1, W, st, &w, polish > 0, regimes);
  if (rc) return rc;
  if (ce > 0) {
    const size_t need = (size_t)g.B * g.P;
    if (need > w->cap_model) {
      hipError_t e = hipStreamSynchronize(st);
      if (e == hipSuccess && w->model) e = hipFree(w->model);
      w->model = nullptr;
      w->cap_model = 0;
      if (e == hipSuccess) e = hipMalloc((void **)&w->model, need * sizeof(float));
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LASP_E_NOMEM, std::string("Clean model buffer: ") + hipGetErrorString(e));
      }
      w->cap_model = need;
    }
    if (opts->out_mask) {
      hipError_t e = hipMemsetAsync(opts->out_mask, 1, (size_t)g.B * g.P, st);
      if (e != hipSuccess) return dev_fail(e, "out_mask init");
    }
  }
  State s = w->s;
  if (W == 0) s.target = nullptr;  // every spectrum takes n_steps steps
  const int bf16 = opts->precision == LASP_PREC_BF16X3;
  rc = copy_basis(g, s, basis, bf16, st);
  if (rc) return rc;
  {
    LASP_TIMED(LASP_K_PREPARE, st);
    LASP_CHECK(lasp::launch_prepare(g, s, obs, ivar, init_params, opts->box_lo, opts->box_hi,
                                    opts->weight_quantile, 1, n_steps, st),
               "prepare");
  }
  const lasp::AdamCfg adam{opts->lr, opts->beta1, opts->beta2, opts->eps, W, opts->stop_tol};
  s.fp_stride = g.ldF;
  if ((W > 0 || polish > 0) && !w->h_active) {
    hipError_t e = hipHostMalloc((void **)&w->h_active, 2 * sizeof(int));
    for (int k = 0; e == hipSuccess && k < 2; ++k)
      e = hipEventCreateWithFlags(&w->ev[k], hipEventDisableTiming);
    if (e != hipSuccess) return dev_fail(e, "active-list events");
  }
  int it0 = 0;
  if (opts->step_graph && W == 0 && !regimes && ce == 0 && g_prof_mask.load() == 0 &&
      n_steps >= kGraphSteps && g.B <= kGraphMaxSpectra) {
    // the plain path launches the same three kernels with the same
    // arguments at every step: whole chunks replay one cached graph (not
    // while kernels are being timed, which brackets each launch)
    it0 = n_steps / kGraphSteps * kGraphSteps;
    rc = replay_steps(w, g, s, adam, bf16, n_steps / kGraphSteps, st);
    if (rc) return rc;
  }
  for (int it = it0; it < n_steps; ++it) {
    if ((W > 0 || regimes) && (it > 0 || regimes) && it % kCompactEvery == 0) {
      // the spectra still stepping, listed so that the per-step kernels cover
      // those only (a fit's arithmetic does not depend on its place)
      State all = s;
      all.order = nullptr;
      LASP_CHECK(lasp::launch_compact(g, all, w->order, w->order + g.B, st), "active list");
      s.order = w->order;
      s.n_active = w->order + g.B;
    }
    if (W > 0 && it > 0 && it % kCompactEvery == 0) {
      // once no fit is active, stop enqueuing steps: the host reads the list
      // length of the previous compaction, whose steps the device is still
      // working through, so the wait leaves no gap
      const int slot = (it / kCompactEvery) & 1;
      LASP_CHECK(hipMemcpyAsync(w->h_active + slot, w->order + g.B, sizeof(int),
                                hipMemcpyDeviceToHost, st),
                 "active count");
      LASP_CHECK(hipEventRecord(w->ev[slot], st), "active count event");
      if (it >= 2 * kCompactEvery) {
        LASP_CHECK(hipEventSynchronize(w->ev[slot ^ 1]), "active count wait");
        if (w->h_active[slot ^ 1] == 0) break;
      }
    }
    {
      LASP_TIMED(LASP_K_INTERP_FWD, st);
      LASP_CHECK(lasp::launch_interp_fwd(g, s, 0, bf16, st), "interpolator contraction");
    }
    if (ce > 0 && it > 0 && it % ce == 0 && it / ce <= cm) {
      // Clean update: residual of the current model, new mask and weights
      // (every spectrum, as without the active list)
      State sc = s;
      sc.order = nullptr;
      sc.n_active = nullptr;
      LASP_CHECK(lasp::launch_fused(g, sc, 0, w->model, 0, st), "fused pass (model)");
      lasp::CleanArgs ca{obs, ivar, w->model, it == ce ? 0.5f : 0.2f, opts->out_mask, nullptr, sc};
      LASP_CHECK(lasp::launch_clean(g, ca, st), "Clean mask");
    }
    {
      LASP_TIMED(LASP_K_FUSED, st);
      LASP_CHECK(lasp::launch_fused(g, s, 1, nullptr, 0, st), "fused pass");
    }
    {
      LASP_TIMED(LASP_K_INTERP_BWD, st);
      LASP_CHECK(lasp::launch_interp_bwd(g, s, &adam, nullptr, bf16, st), "adjoint contraction + Adam");
    }
  }
  // chi2 and status at the returned parameters (every spectrum, stopped or
  // not); derivative rows for the covariance
  s.target = nullptr;
  s.order = nullptr;
  s.n_active = nullptr;
  if (polish > 0) {
    // Levenberg-Marquardt polish from the Adam end point
    const lasp::LmState lm = w->lm;
    State trial = s;
    trial.u = lm.u_trial;
    trial.chi2 = lm.chi2_trial;
    trial.status = lm.st_trial;
    trial.fp_stride = g.ldF;
    LASP_CHECK(lasp::launch_lm_init(g, lm, st), "polish init");
    for (int it = 0; it < polish; ++it) {
      s.fp_stride = 4 * g.ldF;
      LASP_CHECK(lasp::launch_interp_fwd(g, s, 1, bf16, st), "interpolator contraction");
      {
        LASP_TIMED(LASP_K_COV, st);
        LASP_CHECK(lasp::launch_cov(g, s, opts->box_lo, opts->box_hi, nullptr, nullptr, lm.normal,
                                    lm.need_jac, st),
                   "normal equations");
      }
      LASP_CHECK(lasp::launch_lm_solve(g, s, lm, st), "polish step");
      LASP_CHECK(lasp::launch_interp_fwd(g, trial, 0, bf16, st), "interpolator contraction");
      LASP_CHECK(lasp::launch_fused(g, trial, 0, nullptr, 1, st), "fused pass");
      LASP_CHECK(lasp::launch_lm_accept(g, s, lm, it == polish - 1, st), "polish accept");
      if ((it + 1) % kLmCheckEvery == 0 && it + 1 < polish) {
        // once every spectrum has stopped the remaining iterations change
        // nothing: the host reads the count of kLmCheckEvery iterations
        // earlier (the device is still working through the ones since) and
        // stops enqueuing
        const int slot = ((it + 1) / kLmCheckEvery) & 1;
        LASP_CHECK(lasp::launch_lm_active(g, lm, st), "polish count");
        LASP_CHECK(hipMemcpyAsync(w->h_active + slot, lm.active, sizeof(int),
                                  hipMemcpyDeviceToHost, st),
                   "polish count");
        LASP_CHECK(hipEventRecord(w->ev[slot], st), "polish count event");
        if (it + 1 >= 2 * kLmCheckEvery) {
          LASP_CHECK(hipEventSynchronize(w->ev[slot ^ 1]), "polish count wait");
          if (w->h_active[slot ^ 1] == 0) break;
        }
      }
    }
  }
  s.fp_stride = out_cov ? 4 * g.ldF : g.ldF;
  LASP_CHECK(lasp::launch_interp_fwd(g, s, out_cov ? 1 : 0, bf16, st), "interpolator contraction");
  LASP_CHECK(lasp::launch_fused(g, s, 0, nullptr, 1, st), "fused pass");
  if (out_cov) {
    LASP_TIMED(LASP_K_COV, st);
    LASP_CHECK(lasp::launch_cov(g, s, opts->box_lo, opts->box_hi, out_cov, nullptr, nullptr, nullptr, st),
               "covariance");
  }
  {
    LASP_TIMED(LASP_K_FINALIZE, st);
    LASP_CHECK(lasp::launch_finalize(g, s, opts->box_lo, opts->box_hi, out_params, opts->status,
                                     opts->out_chi2, opts->out_steps, st),
               "finalize");
  }
  return LASP_OK;
}

int lasp_clean_mask(const float *obs, const float *ivar, const float *model, float f_shift,
                    uint8_t *keep, int32_t *n_masked, const double *wave_grid,
                    const lasp_opts *opts) {
  g_err.clear();
  Geometry g;
  int rc = make_geometry(opts, wave_grid, &g);
  if (rc) return rc;
  if (!obs || !ivar || !model || !keep)
    return fail(LASP_E_ARG, "obs, ivar, model and keep are required");
  if (!(f_shift >= 0.f) || !std::isfinite(f_shift)) return fail(LASP_E_ARG, "f_shift must be >= 0");
  if (g.B == 0) return LASP_OK;
  hipStream_t st = (hipStream_t)opts->stream;
  lasp::CleanArgs ca{obs, ivar, model, f_shift, keep, n_masked, State{}};
  LASP_CHECK(lasp::launch_clean(g, ca, st), "Clean mask");
  return LASP_OK;
}

int lasp_resample(const float *src, int32_t n_rows, int32_t n_src, int64_t ld_src, double lam0,
                  double dlam, float *out, int32_t n_out, int64_t ld_out, double lg0,
                  double dlog10, void *stream) {
  g_err.clear();
  if (n_rows < 0 || n_src < 1 || n_out < 0) return fail(LASP_E_ARG, "need n_rows >= 0, n_src >= 1, n_out >= 0");
  if (ld_src < n_src || ld_out < n_out) return fail(LASP_E_ARG, "ld_src >= n_src and ld_out >= n_out required");
  if (!isfinite(lam0) || !(dlam > 0.0) || !isfinite(dlam) || !isfinite(lg0) || !(dlog10 > 0.0) ||
      !isfinite(dlog10))
    return fail(LASP_E_ARG, "lam0, lg0 finite and dlam, dlog10 positive and finite required");
  if (n_rows == 0 || n_out == 0) return LASP_OK;
  if (!src || !out) return fail(LASP_E_ARG, "src and out are required");
  const char *s0 = (const char *)src, *s1 = (const char *)(src + (size_t)(n_rows - 1) * ld_src + n_src);
  const char *o0 = (const char *)out, *o1 = (const char *)(out + (size_t)(n_rows - 1) * ld_out + n_out);
  if (o0 < s1 && s0 < o1) return fail(LASP_E_ARG, "out must not overlap src");
  const double e0 = lam0 - 0.5 * dlam, e1 = e0 + (double)n_src * dlam;
  const double first = pow(10.0, lg0 - 0.5 * dlog10);
  const double last = pow(10.0, lg0 + ((double)n_out - 0.5) * dlog10);
  if (!(first >= e0) || !(last <= e1)) {
    char buf[200];
    snprintf(buf, sizeof buf, "target edges [%.6f, %.6f] leave the source range [%.6f, %.6f]",
             first, last, e0, e1);
    return fail(LASP_E_GRID, buf);
  }
  LASP_CHECK(lasp::launch_resample(src, n_rows, n_src, ld_src, lam0, dlam, out, n_out, ld_out,
                                   lg0, dlog10, (hipStream_t)stream),
             "resample");
  return LASP_OK;
}

int lasp_forward(const float *obs, const float *ivar, const double *wave_grid, const float *basis,
                 const float *u, float *out_model, double *out_chi2, float *out_J,
                 int32_t *out_neff, float *out_grad, float *out_jac, double *out_cov,
                 const lasp_opts *opts) {
  g_err.clear();
  Geometry g;
  int rc = make_geometry(opts, wave_grid, &g);
  if (rc) return rc;
  if (!obs || !ivar || !basis || !u || !out_chi2)
    return fail(LASP_E_ARG, "obs, ivar, basis, u and out_chi2 are required");
  if (g.B == 0) return LASP_OK;
  hipStream_t st = (hipStream_t)opts->stream;
  const bool rows4 = out_jac || out_cov;
  Workspace *w = nullptr;
  rc = get_workspace(g, rows4 ? 4 : 1, 0, st, &w);
  if (rc) return rc;
  return forward_enqueue(g, w->s, obs, ivar, basis, u, out_model, out_chi2, out_J, out_neff,
                         out_grad, out_jac, out_cov, opts);
}

int lasp_forward_noalloc(const float *obs, const float *ivar, const double *wave_grid,
                         const float *basis, const float *u, float *out_model, double *out_chi2,
                         float *out_J, int32_t *out_neff, float *out_grad, float *out_jac,
                         double *out_cov, const lasp_opts *opts) {
  g_err.clear();
  Geometry g;
  int rc = make_geometry(opts, wave_grid, &g);
  if (rc) return rc;
  if (!obs || !ivar || !basis || !u || !out_chi2)
    return fail(LASP_E_ARG, "obs, ivar, basis, u and out_chi2 are required");
  if (g.B == 0) return LASP_OK;
  hipStream_t st = (hipStream_t)opts->stream;
  const int rows = (out_jac || out_cov) ? 4 : 1;
  const int bf16 = opts->precision == LASP_PREC_BF16X3;
  State s;
  const size_t need = carve_forward_state(g, rows, bf16, nullptr, &s);
  if (need > kScratchBytes) {
    const size_t per = need / (size_t)g.B;
    char buf[240];
    snprintf(buf, sizeof buf,
             "lasp_forward_noalloc: %d spectra of this shape need %zu bytes of scratch; its "
             "fixed array holds %zu bytes (at most about %zu spectra of this shape)",
             g.B, need, kScratchBytes, per ? kScratchBytes / per : (size_t)0);
    return fail(LASP_E_NOMEM, buf);
  }
  unsigned char *base = nullptr;
  rc = scratch_address(&base);
  if (rc) return rc;
  carve_forward_state(g, rows, bf16, base, &s);
  // the previous call's contents stay in the array: clear the part this
  // call uses (a fill kernel, so that a captured call records no memset)
  hipLaunchKernelGGL(k_zero16, dim3(1024), dim3(256), 0, st, reinterpret_cast<uint4 *>(base),
                     need / 16);
  LASP_CHECK(hipGetLastError(), "scratch clear");
  return forward_enqueue(g, s, obs, ivar, basis, u, out_model, out_chi2, out_J, out_neff,
                         out_grad, out_jac, out_cov, opts);
}


// ---------------------------------------------------------------- pools --
}  // extern "C"

struct lasp_pool {
  Geometry g;          // g.B = capacity
  lasp_opts opts;
  hipStream_t st;
  int device;
  int bf16;
  Workspace w;
};

namespace {
// Device bytes of one pool slot: the per-spectrum buffers that
// ensure_buffers allocates for a pool (u, m, v, t, target, rise counter,
// weight, n_eff, status, d/du4,5, chi2, list entry, loss ring, the
// (o/w, W w^2) layout, four rows of F' and F-bar').
size_t slot_bytes_of(const Geometry &g, int stop_window) {
  return 3 * lasp::kNP * sizeof(float) + 7 * sizeof(int) + 2 * sizeof(float) +
         sizeof(double) + (size_t)stop_window * sizeof(double) +
         (size_t)lasp::kNPL * g.block * sizeof(float2) + (size_t)5 * g.ldF * sizeof(float);
}

// Device bytes of a pool independent of its capacity: the padded basis and
// its BF16 hi/lo splits (both layouts), and the list length.
size_t pool_fixed_bytes(const Geometry &g) {
  return (size_t)g.nb * g.ldF * (sizeof(float) + 2 * sizeof(uint16_t)) +
         (size_t)2 * 32 * g.ldF * sizeof(uint16_t) + sizeof(int);
}

int pool_geometry(const lasp_pool *p, int count, Geometry *g) {
  *g = p->g;
  g->B = count;
  return LASP_OK;
}
}  // namespace

extern "C" {

size_t lasp_pool_slot_bytes(const lasp_opts *opts, const double *wave_grid) {
  Geometry g;
  if (make_geometry(opts, wave_grid, &g)) return 0;
  return slot_bytes_of(g, opts->stop_window);
}

int lasp_pool_create(const double *wave_grid, const float *basis, const lasp_opts *opts,
                     lasp_pool **out) {
  g_err.clear();
  if (!out) return fail(LASP_E_ARG, "out is NULL");
  *out = nullptr;
  Geometry g;
  int rc = make_geometry(opts, wave_grid, &g);
  if (rc) return rc;
  if (!basis) return fail(LASP_E_ARG, "basis is NULL");
  if (g.B < 1) return fail(LASP_E_ARG, "pool capacity (n_spec) must be >= 1");
  lasp_pool *p = new lasp_pool();
  p->g = g;
  p->opts = *opts;
  p->st = (hipStream_t)opts->stream;
  p->bf16 = opts->precision == LASP_PREC_BF16X3;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return dev_fail(e, "hipGetDevice");
  }
  rc = ensure_buffers(&p->w, g, 4, opts->stop_window, p->st, false, true);
  if (!rc) {
    e = hipMemsetAsync(p->w.s.target, 0, sizeof(int) * g.B, p->st);
    if (e == hipSuccess) e = hipMemsetAsync(p->w.s.t, 0, sizeof(int) * g.B, p->st);
    if (e != hipSuccess) rc = dev_fail(e, "pool init");
  }
  if (!rc) rc = copy_basis(g, p->w.s, basis, p->bf16, p->st);
  if (rc) {
    lasp_pool_destroy(p);
    return rc;
  }
  *out = p;
  return LASP_OK;
}

int lasp_pool_load(lasp_pool *p, int32_t slot0, int32_t count, const float *obs,
                   const float *ivar, const float *init_params, int32_t n_steps) {
  g_err.clear();
  if (!p || !obs || !ivar || !init_params) return fail(LASP_E_ARG, "NULL argument");
  if (slot0 < 0 || count < 1 || slot0 + count > p->g.B || n_steps < 0)
    return fail(LASP_E_ARG, "slot range outside the pool or n_steps < 0");
  Geometry g;
  pool_geometry(p, count, &g);
  State s = offset_state(p->w.s, p->g, slot0, 4, p->opts.stop_window);
  LASP_TIMED(LASP_K_PREPARE, p->st);
  LASP_CHECK(lasp::launch_prepare(g, s, obs, ivar, init_params, p->opts.box_lo, p->opts.box_hi,
                                  p->opts.weight_quantile, 1, n_steps, p->st),
             "prepare");
  return LASP_OK;
}

int lasp_pool_step(lasp_pool *p, int32_t slot_end, int32_t k) {
  g_err.clear();
  if (!p) return fail(LASP_E_ARG, "pool is NULL");
  if (slot_end < 0 || slot_end > p->g.B || k < 0) return fail(LASP_E_ARG, "bad slot_end or k");
  if (slot_end == 0 || k == 0) return LASP_OK;
  Geometry g;
  pool_geometry(p, slot_end, &g);
  State s = p->w.s;
  s.fp_stride = g.ldF;
  const lasp::AdamCfg adam{p->opts.lr,  p->opts.beta1,       p->opts.beta2,
                           p->opts.eps, p->opts.stop_window, p->opts.stop_tol};
  // the slots below their step target, listed so that the step kernels skip
  // idle and finished slots (a fit's arithmetic does not depend on its place)
  LASP_CHECK(lasp::launch_compact(g, s, p->w.order, p->w.order + p->g.B, p->st), "active list");
  s.order = p->w.order;
  s.n_active = p->w.order + p->g.B;
  for (int it = 0; it < k; ++it) {
    {
      LASP_TIMED(LASP_K_INTERP_FWD, p->st);
      LASP_CHECK(lasp::launch_interp_fwd(g, s, 0, p->bf16, p->st), "interpolator contraction");
    }
    {
      LASP_TIMED(LASP_K_FUSED, p->st);
      LASP_CHECK(lasp::launch_fused(g, s, 1, nullptr, 0, p->st), "fused pass");
    }
    {
      LASP_TIMED(LASP_K_INTERP_BWD, p->st);
      LASP_CHECK(lasp::launch_interp_bwd(g, s, &adam, nullptr, p->bf16, p->st),
                 "adjoint contraction + Adam");
    }
  }
  return LASP_OK;
}

int lasp_pool_progress(lasp_pool *p, int32_t slot0, int32_t count, int32_t *steps,
                       int32_t *done) {
  g_err.clear();
  if (!p) return fail(LASP_E_ARG, "pool is NULL");
  if (slot0 < 0 || count < 1 || slot0 + count > p->g.B)
    return fail(LASP_E_ARG, "slot range outside the pool");
  if (!steps && !done) return LASP_OK;
  Geometry g;
  pool_geometry(p, count, &g);
  State s = offset_state(p->w.s, p->g, slot0, 4, p->opts.stop_window);
  LASP_CHECK(lasp::launch_progress(g, s, steps, done, p->st), "progress");
  return LASP_OK;
}

int lasp_pool_finish(lasp_pool *p, int32_t slot0, int32_t count, float *out_params,
                     double *out_cov, uint32_t *status, double *chi2) {
  g_err.clear();
  if (!p || !out_params) return fail(LASP_E_ARG, "NULL argument");
  if (slot0 < 0 || count < 1 || slot0 + count > p->g.B)
    return fail(LASP_E_ARG, "slot range outside the pool");
  Geometry g;
  pool_geometry(p, count, &g);
  const int rows = out_cov ? 4 : 1;
  State s = offset_state(p->w.s, p->g, slot0, rows, p->opts.stop_window);
  s.target = nullptr;  // the final evaluation covers every slot of the range
  s.fp_stride = rows * g.ldF;
  LASP_CHECK(lasp::launch_interp_fwd(g, s, out_cov ? 1 : 0, p->bf16, p->st),
             "interpolator contraction");
  LASP_CHECK(lasp::launch_fused(g, s, 0, nullptr, 1, p->st), "fused pass");
  if (out_cov) {
    LASP_TIMED(LASP_K_COV, p->st);
    LASP_CHECK(lasp::launch_cov(g, s, p->opts.box_lo, p->opts.box_hi, out_cov, nullptr, nullptr, nullptr,
                                p->st),
               "covariance");
  }
  LASP_TIMED(LASP_K_FINALIZE, p->st);
  LASP_CHECK(lasp::launch_finalize(g, s, p->opts.box_lo, p->opts.box_hi, out_params, status,
                                   chi2, nullptr, p->st),
             "finalize");
  return LASP_OK;
}

int lasp_pool_resize(lasp_pool *p, int32_t capacity, int32_t keep) {
  g_err.clear();
  if (!p) return fail(LASP_E_ARG, "pool is NULL");
  if (capacity < 1 || keep < 0 || keep > capacity || keep > p->g.B)
    return fail(LASP_E_ARG, "need capacity >= 1 and 0 <= keep <= min(capacity, current capacity)");
  if (capacity == p->g.B) return LASP_OK;
  Geometry g = p->g;
  g.B = capacity;
  const int W = p->opts.stop_window;
  Workspace nw;
  nw.device = p->device;
  nw.stream = p->st;
  int rc = ensure_buffers(&nw, g, 4, W, p->st, false, true);
  if (rc) return rc;
  const State &a = p->w.s;
  const State &b = nw.s;
  const size_t k = (size_t)keep, ld = (size_t)g.ldF;
  struct Piece {
    void *dst;
    const void *src;
    size_t bytes;
  };
  const Piece pieces[] = {
      {b.u, a.u, k * lasp::kNP * sizeof(float)},
      {b.m, a.m, k * lasp::kNP * sizeof(float)},
      {b.v, a.v, k * lasp::kNP * sizeof(float)},
      {b.t, a.t, k * sizeof(int)},
      {b.target, a.target, k * sizeof(int)},
      {b.nrise, a.nrise, k * sizeof(int)},
      {b.lhist, a.lhist, W > 0 ? k * W * sizeof(double) : 0},
      {b.ow, a.ow, k * lasp::kNPL * g.block * sizeof(float2)},
      {b.wscale, a.wscale, k * sizeof(float)},
      {b.neff, a.neff, k * sizeof(int)},
      {b.status, a.status, k * sizeof(uint32_t)},
      {b.g45, a.g45, k * 2 * sizeof(float)},
      {b.chi2, a.chi2, k * sizeof(double)},
      {b.fp, a.fp, k * 4 * ld * sizeof(float)},
      {b.fbar, a.fbar, k * ld * sizeof(float)},
      {b.basis, a.basis, (size_t)g.nb * ld * sizeof(float)},
      {b.basis_hi, a.basis_hi, p->bf16 ? (size_t)g.nb * ld * sizeof(uint16_t) : 0},
      {b.basis_lo, a.basis_lo, p->bf16 ? (size_t)g.nb * ld * sizeof(uint16_t) : 0},
      {b.basis_thi, a.basis_thi, p->bf16 ? (size_t)32 * ld * sizeof(uint16_t) : 0},
      {b.basis_tlo, a.basis_tlo, p->bf16 ? (size_t)32 * ld * sizeof(uint16_t) : 0},
  };
  hipError_t e = hipSuccess;
  for (const Piece &q : pieces)
    if (e == hipSuccess && q.bytes > 0)
      e = hipMemcpyAsync(q.dst, q.src, q.bytes, hipMemcpyDeviceToDevice, p->st);
  // slots past `keep` start idle (step count 0, target 0)
  if (e == hipSuccess && capacity > keep)
    e = hipMemsetAsync(b.target + keep, 0, sizeof(int) * (capacity - keep), p->st);
  if (e == hipSuccess && capacity > keep)
    e = hipMemsetAsync(b.t + keep, 0, sizeof(int) * (capacity - keep), p->st);
  // the old buffers are freed only once the copies (and every earlier step
  // on the pool's stream) have finished
  if (e == hipSuccess) e = hipStreamSynchronize(p->st);
  if (e != hipSuccess) {
    free_ws(&nw);
    return dev_fail(e, "pool resize");
  }
  free_ws(&p->w);
  p->w = nw;
  p->g.B = capacity;
  return LASP_OK;
}

size_t lasp_pool_bytes(const lasp_pool *p) {
  if (!p) return 0;
  return (size_t)p->g.B * slot_bytes_of(p->g, p->opts.stop_window) + pool_fixed_bytes(p->g);
}

int32_t lasp_pool_capacity(const lasp_pool *p) { return p ? p->g.B : 0; }

int lasp_pool_destroy(lasp_pool *p) {
  if (!p) return LASP_OK;
  (void)hipStreamSynchronize(p->st);
  free_ws(&p->w);
  delete p;
  return LASP_OK;
}

}  // extern "C"
