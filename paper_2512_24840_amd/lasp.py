"""ctypes binding of liblasp.so (include/lasp.h): argument marshalling only.

Every step of the fit runs in the HIP kernels behind the C ABI; this module
checks tensor shapes, dtypes and devices, fills ``lasp_opts`` and forwards
device pointers and the current HIP stream.  It raises if the library has
not been built -- there is no fallback path.
"""

from __future__ import annotations

import ctypes
import dataclasses
import math
import os

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "liblasp.so")

LASP_OK = 0
ERRORS = {-1: "LASP_E_ARG", -2: "LASP_E_GRID", -3: "LASP_E_DEVICE", -4: "LASP_E_NOMEM",
          -5: "LASP_E_UNSUPPORTED"}
ST_NONFINITE_INPUT = 0x01
ST_NO_DATA = 0x02
ST_SINGULAR = 0x04
ST_CONT_NONPOS = 0x08
ST_OUT_OF_BOX = 0x10
ST_SIGMA_FLOOR = 0x20
ST_STOP_FLAT = 0x40
ST_STOP_RISING = 0x80
ST_NOT_CONVERGED = 0x100
ST_POLISH_LIMIT = 0x200
PREC = {"fp32": 0, "bf16x3": 1}
N_BASIS = 20
N_PAR = 5
EXPORTED = ("lasp_default_opts", "lasp_fit_group", "lasp_forward", "lasp_last_error",
            "lasp_release", "lasp_profile_enable", "lasp_profile_read", "lasp_pool_slot_bytes",
            "lasp_pool_create", "lasp_pool_load", "lasp_pool_step", "lasp_pool_progress",
            "lasp_pool_finish", "lasp_pool_destroy", "lasp_clean_mask", "lasp_resample",
            "lasp_forward_noalloc", "lasp_pool_resize", "lasp_pool_bytes", "lasp_pool_capacity",
            "lasp_server_default_opts", "lasp_server_create", "lasp_server_add_shape",
            "lasp_server_submit", "lasp_server_poll", "lasp_server_stats", "lasp_server_destroy")
SERVER_MAX_SHAPES = 8
KERNELS = ("prepare", "interp_fwd", "fused", "interp_bwd", "cov", "finalize")


class LaspError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("n_steps", ctypes.c_int32),
                ("steps_per_tick", ctypes.c_int32), ("want_cov", ctypes.c_int32),
                ("capacity_quantum", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("shape", ctypes.c_int32), ("count", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("stopped", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("hbm_in_use", ctypes.c_size_t),
                ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("ticks", ctypes.c_int64), ("resizes", ctypes.c_int64),
                ("queued", ctypes.c_int32), ("active", ctypes.c_int32),
                ("finishing", ctypes.c_int32), ("n_shapes", ctypes.c_int32),
                ("capacity", ctypes.c_int32 * 8), ("used_slots", ctypes.c_int32 * 8)]


class LaspOpts(ctypes.Structure):
    _fields_ = [
        ("n_spec", ctypes.c_int32),
        ("n_pix", ctypes.c_int32),
        ("n_basis", ctypes.c_int32),
        ("margin", ctypes.c_int32),
        ("degree", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("box_lo", ctypes.c_double * 5),
        ("box_hi", ctypes.c_double * 5),
        ("lr", ctypes.c_float),
        ("beta1", ctypes.c_float),
        ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("weight_quantile", ctypes.c_float),
        ("n_arms", ctypes.c_int32),
        ("arm_start", ctypes.c_int32 * 4),
        ("arm_sigma_kms", ctypes.c_float * 4),
        ("stream", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("out_chi2", ctypes.c_void_p),
        ("stop_window", ctypes.c_int32),
        ("stop_tol", ctypes.c_float),
        ("out_steps", ctypes.c_void_p),
        ("polish_iters", ctypes.c_int32),
        ("clean_every", ctypes.c_int32),
        ("clean_max", ctypes.c_int32),
        ("out_mask", ctypes.c_void_p),
        ("n_classes", ctypes.c_int32),
        ("class_edges", ctypes.c_double * 4),
        ("step_graph", ctypes.c_int32),
    ]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load() -> ctypes.CDLL:
    """Load liblasp.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        lib.lasp_default_opts.argtypes = [ctypes.POINTER(LaspOpts)]
        lib.lasp_default_opts.restype = None
        lib.lasp_fit_group.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.c_int32,
                                       ctypes.POINTER(LaspOpts)]
        lib.lasp_fit_group.restype = ctypes.c_int
        lib.lasp_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                     ctypes.POINTER(LaspOpts)]
        lib.lasp_forward.restype = ctypes.c_int
        lib.lasp_forward_noalloc.argtypes = lib.lasp_forward.argtypes
        lib.lasp_forward_noalloc.restype = ctypes.c_int
        lib.lasp_last_error.argtypes = []
        lib.lasp_last_error.restype = ctypes.c_char_p
        lib.lasp_release.argtypes = []
        lib.lasp_release.restype = None
        lib.lasp_profile_enable.argtypes = [ctypes.c_uint32]
        lib.lasp_profile_enable.restype = ctypes.c_int
        lib.lasp_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
        lib.lasp_profile_read.restype = ctypes.c_int
        lib.lasp_pool_slot_bytes.argtypes = [ctypes.POINTER(LaspOpts), vp]
        lib.lasp_pool_slot_bytes.restype = ctypes.c_size_t
        lib.lasp_pool_create.argtypes = [vp, vp, ctypes.POINTER(LaspOpts),
                                         ctypes.POINTER(ctypes.c_void_p)]
        lib.lasp_pool_create.restype = ctypes.c_int
        lib.lasp_pool_load.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp,
                                       ctypes.c_int32]
        lib.lasp_pool_load.restype = ctypes.c_int
        lib.lasp_pool_step.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        lib.lasp_pool_step.restype = ctypes.c_int
        lib.lasp_pool_progress.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp]
        lib.lasp_pool_progress.restype = ctypes.c_int
        lib.lasp_pool_finish.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
        lib.lasp_pool_finish.restype = ctypes.c_int
        lib.lasp_clean_mask.argtypes = [vp, vp, vp, ctypes.c_float, vp, vp, vp,
                                        ctypes.POINTER(LaspOpts)]
        lib.lasp_clean_mask.restype = ctypes.c_int
        lib.lasp_resample.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_double, vp, ctypes.c_int32,
                                      ctypes.c_int64, ctypes.c_double, ctypes.c_double, vp]
        lib.lasp_resample.restype = ctypes.c_int
        lib.lasp_pool_destroy.argtypes = [vp]
        lib.lasp_pool_destroy.restype = ctypes.c_int
        lib.lasp_pool_resize.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        lib.lasp_pool_resize.restype = ctypes.c_int
        lib.lasp_pool_bytes.argtypes = [vp]
        lib.lasp_pool_bytes.restype = ctypes.c_size_t
        lib.lasp_pool_capacity.argtypes = [vp]
        lib.lasp_pool_capacity.restype = ctypes.c_int32
        lib.lasp_server_default_opts.argtypes = [ctypes.POINTER(ServerOpts)]
        lib.lasp_server_default_opts.restype = None
        lib.lasp_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
        lib.lasp_server_create.restype = ctypes.c_int
        lib.lasp_server_add_shape.argtypes = [vp, vp, vp, ctypes.POINTER(LaspOpts),
                                              ctypes.POINTER(ctypes.c_int32)]
        lib.lasp_server_add_shape.restype = ctypes.c_int
        lib.lasp_server_submit.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp,
                                           vp, vp, ctypes.POINTER(ctypes.c_int64)]
        lib.lasp_server_submit.restype = ctypes.c_int
        lib.lasp_server_poll.argtypes = [vp, ctypes.POINTER(RequestInfo), ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        lib.lasp_server_poll.restype = ctypes.c_int
        lib.lasp_server_stats.argtypes = [vp, ctypes.POINTER(ServerCounters)]
        lib.lasp_server_stats.restype = ctypes.c_int
        lib.lasp_server_destroy.argtypes = [vp]
        lib.lasp_server_destroy.restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != LASP_OK:
        raise LaspError(rc, load().lasp_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, name: str, dtype, shape):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


@dataclasses.dataclass
class Arms:
    start: tuple
    sigma_kms: tuple


def make_opts(n_spec, n_pix, *, margin=64, degree=10, precision="fp32", lr=1e-2,
              betas=(0.9, 0.999), eps=1e-8, weight_quantile=0.5, arms: Arms | None = None,
              box=None, stream=None, stop_window=0, stop_tol=1e-5, polish_iters=0,
              clean_every=0, clean_max=11, n_classes=1, class_edges=None,
              step_graph=True) -> LaspOpts:
    o = LaspOpts()
    load().lasp_default_opts(ctypes.byref(o))
    o.n_spec, o.n_pix, o.margin, o.degree = int(n_spec), int(n_pix), int(margin), int(degree)
    o.precision = PREC[precision]
    o.lr, o.beta1, o.beta2, o.eps = float(lr), float(betas[0]), float(betas[1]), float(eps)
    o.weight_quantile = float(weight_quantile)
    o.stop_window, o.stop_tol = int(stop_window), float(stop_tol)
    o.polish_iters = int(polish_iters)
    o.clean_every, o.clean_max = int(clean_every), int(clean_max)
    o.n_classes = int(n_classes)
    o.n_basis = N_BASIS * int(n_classes)
    o.step_graph = int(bool(step_graph))
    if class_edges is not None:
        for i in range(4):
            o.class_edges[i] = float(class_edges[i])
    if box is not None:
        lo, hi = box
        for t in range(5):
            o.box_lo[t], o.box_hi[t] = float(lo[t]), float(hi[t])
    if arms is not None and len(arms.start) > 0:
        o.n_arms = len(arms.start)
        for a, (s, g) in enumerate(zip(arms.start, arms.sigma_kms)):
            o.arm_start[a], o.arm_sigma_kms[a] = int(s), float(g)
    if stream is None:
        stream = torch.cuda.current_stream()
    o.stream = ctypes.c_void_p(stream.cuda_stream)
    return o


def _grid(wave_grid, n_pix):
    g = np.ascontiguousarray(np.asarray(wave_grid, dtype=np.float64))
    if g.shape != (n_pix,):
        raise ValueError(f"wave_grid must have shape ({n_pix},)")
    return g


@dataclasses.dataclass
class FitResult:
    params: torch.Tensor          # [B, 5] float32, physical units
    cov: torch.Tensor | None      # [B, 5, 5] float64, physical units
    status: torch.Tensor          # [B] int32 (LASP_ST_* bits)
    chi2: torch.Tensor            # [B] float64
    steps: torch.Tensor | None = None  # [B] int32 Adam steps taken
    mask: torch.Tensor | None = None   # [B, P] uint8 last Clean mask (1 kept)


def fit_group(obs, ivar, wave_grid, basis, init_params, n_steps, *, want_cov=False,
              margin=64, degree=10, precision="fp32", lr=1e-2, betas=(0.9, 0.999), eps=1e-8,
              weight_quantile=0.5, arms: Arms | None = None, box=None, stream=None,
              stop_window=0, stop_tol=1e-5, polish_iters=0, clean_every=0, clean_max=11,
              want_mask=False, n_classes=1, class_edges=None, step_graph=True,
              out: FitResult | None = None) -> FitResult:
    """lasp_fit_group on device tensors; returns after enqueueing (stream ordered).
    stop_window > 0 turns on the per-spectrum stopping rules (window, stop_tol);
    polish_iters > 0 adds that many Levenberg-Marquardt iterations at most;
    clean_every > 0 turns on the Clean mask updates (every clean_every steps,
    at most clean_max times); n_classes = 3 takes a [60, P + 2M] basis of
    three emulator temperature classes blended over the Teff regimes;
    step_graph=False launches every step's kernels instead of replaying the
    cached graph of 25 steps (same results)."""
    lib = load()
    B, P = obs.shape
    _dev(obs, "obs", torch.float32, (B, P))
    _dev(ivar, "ivar", torch.float32, (B, P))
    _dev(basis, "basis", torch.float32, (N_BASIS * n_classes, P + 2 * margin))
    _dev(init_params, "init_params", torch.float32, (B, N_PAR))
    grid = _grid(wave_grid, P)
    dev = obs.device
    if out is None:
        out = FitResult(torch.empty((B, N_PAR), dtype=torch.float32, device=dev),
                        torch.empty((B, N_PAR, N_PAR), dtype=torch.float64, device=dev)
                        if want_cov else None,
                        torch.empty(B, dtype=torch.int32, device=dev),
                        torch.empty(B, dtype=torch.float64, device=dev),
                        torch.empty(B, dtype=torch.int32, device=dev),
                        torch.empty((B, P), dtype=torch.uint8, device=dev) if want_mask else None)
    o = make_opts(B, P, margin=margin, degree=degree, precision=precision, lr=lr, betas=betas,
                  eps=eps, weight_quantile=weight_quantile, arms=arms, box=box, stream=stream,
                  stop_window=stop_window, stop_tol=stop_tol, polish_iters=polish_iters,
                  clean_every=clean_every, clean_max=clean_max, n_classes=n_classes,
                  class_edges=class_edges, step_graph=step_graph)
    o.status = ctypes.c_void_p(out.status.data_ptr())
    o.out_chi2 = ctypes.c_void_p(out.chi2.data_ptr())
    if out.steps is not None:
        o.out_steps = ctypes.c_void_p(out.steps.data_ptr())
    if out.mask is not None:
        o.out_mask = ctypes.c_void_p(out.mask.data_ptr())
    with torch.cuda.device(dev):
        rc = lib.lasp_fit_group(_ptr(obs), _ptr(ivar), grid.ctypes.data_as(ctypes.c_void_p),
                                _ptr(basis), _ptr(init_params), _ptr(out.params), _ptr(out.cov),
                                int(n_steps), ctypes.byref(o))
    _check(rc)
    return out


def forward(obs, ivar, wave_grid, basis, u, *, want_model=False, want_grad=False,
            want_jac=False, want_cov=False, margin=64, degree=10, precision="fp32",
            weight_quantile=0.5, arms: Arms | None = None, box=None, stream=None,
            n_classes=1, class_edges=None, noalloc=False) -> dict:
    """lasp_forward: model, chi2, J, n_eff, gradient, model Jacobian and
    covariance at fixed normalised u.  noalloc=True calls
    lasp_forward_noalloc (the library's fixed scratch array instead of its
    cached allocations; the result tensors are still allocated here)."""
    lib = load()
    B, P = obs.shape
    _dev(obs, "obs", torch.float32, (B, P))
    _dev(ivar, "ivar", torch.float32, (B, P))
    _dev(basis, "basis", torch.float32, (N_BASIS * n_classes, P + 2 * margin))
    _dev(u, "u", torch.float32, (B, N_PAR))
    grid = _grid(wave_grid, P)
    dev = obs.device
    res = dict(chi2=torch.empty(B, dtype=torch.float64, device=dev),
               J=torch.empty(B, dtype=torch.float32, device=dev),
               n_eff=torch.empty(B, dtype=torch.int32, device=dev),
               status=torch.empty(B, dtype=torch.int32, device=dev))
    res["model"] = torch.empty((B, P), dtype=torch.float32, device=dev) if want_model else None
    res["grad"] = torch.empty((B, N_PAR), dtype=torch.float32, device=dev) if want_grad else None
    res["jac"] = torch.empty((B, N_PAR, P), dtype=torch.float32, device=dev) if want_jac else None
    res["cov"] = (torch.empty((B, N_PAR, N_PAR), dtype=torch.float64, device=dev)
                  if want_cov else None)
    o = make_opts(B, P, margin=margin, degree=degree, precision=precision,
                  weight_quantile=weight_quantile, arms=arms, box=box, stream=stream,
                  n_classes=n_classes, class_edges=class_edges)
    o.status = ctypes.c_void_p(res["status"].data_ptr())
    with torch.cuda.device(dev):
        fn = lib.lasp_forward_noalloc if noalloc else lib.lasp_forward
        rc = fn(_ptr(obs), _ptr(ivar), grid.ctypes.data_as(ctypes.c_void_p),
                _ptr(basis), _ptr(u), _ptr(res["model"]), _ptr(res["chi2"]),
                _ptr(res["J"]), _ptr(res["n_eff"]), _ptr(res["grad"]),
                _ptr(res["jac"]), _ptr(res["cov"]), ctypes.byref(o))
    _check(rc)
    return res


def clean_mask(obs, ivar, model, wave_grid, f_shift, *, margin=64, stream=None):
    """lasp_clean_mask: (keep [B, P] uint8, n_masked [B] int32) device tensors."""
    lib = load()
    B, P = obs.shape
    for t, nm in ((obs, "obs"), (ivar, "ivar"), (model, "model")):
        _dev(t, nm, torch.float32, (B, P))
    grid = _grid(wave_grid, P)
    keep = torch.empty((B, P), dtype=torch.uint8, device=obs.device)
    nm_ = torch.empty(B, dtype=torch.int32, device=obs.device)
    o = make_opts(B, P, margin=margin, stream=stream)
    with torch.cuda.device(obs.device):
        _check(lib.lasp_clean_mask(_ptr(obs), _ptr(ivar), _ptr(model), float(f_shift), _ptr(keep),
                                   _ptr(nm_), grid.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o)))
    return keep, nm_


def resample(src, lam0, dlam, n_out, lg0, dlog10, *, out=None, stream=None):
    """lasp_resample: rows of src [R, n_src] (float32 device tensor, bin
    centres lam0 + i dlam) onto n_out log10-uniform pixels centred at
    10^(lg0 + j dlog10); returns out [R, n_out] float32 (stream ordered)."""
    lib = load()
    if src.dim() != 2:
        raise ValueError("src must be [rows, n_src]")
    R, n_src = src.shape
    _dev(src, "src", torch.float32, (R, n_src))
    if out is None:
        out = torch.empty((R, int(n_out)), dtype=torch.float32, device=src.device)
    _dev(out, "out", torch.float32, (R, int(n_out)))
    if stream is None:
        stream = torch.cuda.current_stream(src.device)
    with torch.cuda.device(src.device):
        _check(lib.lasp_resample(_ptr(src), int(R), int(n_src), int(n_src), float(lam0),
                                 float(dlam), _ptr(out), int(n_out), int(n_out), float(lg0),
                                 float(dlog10), ctypes.c_void_p(stream.cuda_stream)))
    return out


def release():
    load().lasp_release()


def profile_enable(kernels=()):
    """Time every later launch of the named kernel classes with HIP events."""
    mask = 0
    for k in kernels:
        mask |= 1 << KERNELS.index(k)
    _check(load().lasp_profile_enable(mask))


def profile_read() -> dict:
    """{kernel: (total_ms, launches)} since the last profile_enable()."""
    n = len(KERNELS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(load().lasp_profile_read(ms, cnt, n))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNELS)}


DEFAULT_BOX = (np.array([math.log10(4000.0), 1.0, -2.5, -300.0, 50.0]),
               np.array([math.log10(8000.0), 5.0, 0.5, 300.0, 150.0]))


class Pool:
    """Resident fit slots of one spectral shape (lasp_pool_*), on one stream."""

    def __init__(self, wave_grid, basis, capacity, *, margin=64, degree=10, precision="fp32",
                 lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_quantile=0.5,
                 arms: Arms | None = None, box=None, stream=None, stop_window=0, stop_tol=1e-5,
                 n_classes=1, class_edges=None):
        lib = load()
        P = int(np.asarray(wave_grid).shape[0])
        _dev(basis, "basis", torch.float32, (N_BASIS * n_classes, P + 2 * margin))
        self.n_pix, self.capacity = P, int(capacity)
        self.device = basis.device
        self.stream = stream or torch.cuda.Stream(device=self.device)
        self._grid = _grid(wave_grid, P)
        self._opts = make_opts(capacity, P, margin=margin, degree=degree, precision=precision,
                               lr=lr, betas=betas, eps=eps, weight_quantile=weight_quantile,
                               arms=arms, box=box, stream=self.stream, stop_window=stop_window,
                               stop_tol=stop_tol, n_classes=n_classes, class_edges=class_edges)
        self.stop_window = int(stop_window)
        self.slot_bytes = int(lib.lasp_pool_slot_bytes(ctypes.byref(self._opts),
                                                       self._grid.ctypes.data_as(ctypes.c_void_p)))
        self._p = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.lasp_pool_create(self._grid.ctypes.data_as(ctypes.c_void_p), _ptr(basis),
                                        ctypes.byref(self._opts), ctypes.byref(self._p)))

    def load(self, slot0, obs, ivar, init_params, n_steps):
        n = obs.shape[0]
        _dev(obs, "obs", torch.float32, (n, self.n_pix))
        _dev(ivar, "ivar", torch.float32, (n, self.n_pix))
        _dev(init_params, "init_params", torch.float32, (n, N_PAR))
        _check(load().lasp_pool_load(self._p, int(slot0), int(n), _ptr(obs), _ptr(ivar),
                                     _ptr(init_params), int(n_steps)))

    def step(self, slot_end, k):
        _check(load().lasp_pool_step(self._p, int(slot_end), int(k)))

    def progress(self, slot0, steps=None, done=None):
        """Steps taken and stopped flags of slots [slot0, slot0 + n) into
        int32 device tensors of length n (stream ordered)."""
        t = steps if steps is not None else done
        if t is None:
            return
        n = t.shape[0]
        for x, nm in ((steps, "steps"), (done, "done")):
            if x is not None:
                _dev(x, nm, torch.int32, (n,))
        _check(load().lasp_pool_progress(self._p, int(slot0), int(n), _ptr(steps), _ptr(done)))

    def finish(self, slot0, params, cov=None, status=None, chi2=None):
        n = params.shape[0]
        _dev(params, "params", torch.float32, (n, N_PAR))
        _check(load().lasp_pool_finish(self._p, int(slot0), int(n), _ptr(params), _ptr(cov),
                                       _ptr(status), _ptr(chi2)))

    def resize(self, capacity, keep):
        """lasp_pool_resize: hold `capacity` slots, keeping slots [0, keep)."""
        _check(load().lasp_pool_resize(self._p, int(capacity), int(keep)))
        self.capacity = int(load().lasp_pool_capacity(self._p))

    @property
    def bytes(self) -> int:
        return int(load().lasp_pool_bytes(self._p))

    def close(self):
        if self._p:
            load().lasp_pool_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
