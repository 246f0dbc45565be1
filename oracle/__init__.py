"""FP64 CPU oracle for grouped full-spectrum fitting -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never loads it.  The C source shares no code with the HIP
library.

Python side: ctypes marshalling only; every number comes from
``lasp_oracle.c``.  Calls release the GIL, so a thread pool fits spectra in
parallel.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lasp_oracle.c")
_LIB = os.path.join(_HERE, "liblasp_oracle.so")

NONFINITE, NO_DATA, SINGULAR, CONT_NONPOS, OUT_OF_BOX, NOT_CONVERGED, SIGMA_FLOOR = (
    1 << i for i in range(7))
N_PAR = 5
N_BASIS = 20


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fno-fast-math", "-std=c11", "-Wall", "-shared", "-fPIC",
                        _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("n_pix", ctypes.c_int),
        ("margin", ctypes.c_int),
        ("degree", ctypes.c_int),
        ("n_arms", ctypes.c_int),
        ("arm_start", ctypes.c_int * 4),
        ("arm_sigma", ctypes.c_double * 4),
        ("dlog10", ctypes.c_double),
        ("lo", ctypes.c_double * 5),
        ("hi", ctypes.c_double * 5),
        ("n_classes", ctypes.c_int),
        ("edges", ctypes.c_double * 4),
    ]

# Teff edges (K) of the emulator's five regimes: cool, cool->warm blend, warm,
# warm->hot blend, hot.
REGIME_EDGES = (4000.0, 4550.0, 7000.0, 9000.0)


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int)
        up = ctypes.POINTER(ctypes.c_uint)
        cp = ctypes.POINTER(_Cfg)
        lib.orc_features.argtypes = [dp, dp, dp]
        lib.orc_features.restype = None
        lib.orc_legendre.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.orc_legendre.restype = ctypes.c_double
        lib.orc_kernel.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp, dp]
        lib.orc_kernel.restype = ctypes.c_int
        lib.orc_convolve.argtypes = [dp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, dp]
        lib.orc_convolve.restype = None
        lib.orc_eval.argtypes = [cp, fp, fp, fp, dp, dp, dp, dp, dp, dp, ip, dp, dp, up]
        lib.orc_eval.restype = ctypes.c_int
        lib.orc_residual.argtypes = [cp, fp, fp, fp, dp, dp, dp, dp]
        lib.orc_residual.restype = ctypes.c_int
        lib.orc_fit.argtypes = [cp, fp, fp, fp, dp, ctypes.c_int, dp, dp, dp, ip, dp, dp, ip, up]
        lib.orc_fit.restype = ctypes.c_int
        lib.orc_covariance.argtypes = [cp, fp, fp, fp, dp, dp, dp]
        lib.orc_class_weights.argtypes = [cp, dp, dp, dp]
        lib.orc_class_weights.restype = None
        lib.orc_resample.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, fp,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_resample.restype = ctypes.c_int
        lib.orc_stop_rule.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        lib.orc_stop_rule.restype = ctypes.c_int
        lib.orc_stop_step.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ip]
        lib.orc_stop_step.restype = ctypes.c_int
        dd = ctypes.c_double
        lib.orc_adam_fit.argtypes = [cp, fp, fp, fp, dp, ctypes.c_int, dd, dd, dd, dd,
                                     ctypes.c_int, dd, ctypes.c_int, ctypes.c_int, dp, ip, ip, dp,
                                     ctypes.POINTER(ctypes.c_uint8)]
        lib.orc_adam_fit.restype = ctypes.c_int
        u8p = ctypes.POINTER(ctypes.c_uint8)
        lib.orc_clean.argtypes = [ctypes.c_int, fp, fp, dp, ctypes.c_double, u8p, dp, ip]
        lib.orc_clean.restype = ctypes.c_int
        lib.orc_covariance.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _d(a):
    return _p(a, ctypes.c_double)


def _f(a):
    return _p(a, ctypes.c_float)


class Config:
    """Grid/shape description for the oracle (plain values, no arithmetic)."""

    def __init__(self, n_pix, margin, degree, dlog10, box_lo, box_hi, arm_start=(), arm_sigma=(),
                 n_classes=1, edges=REGIME_EDGES):
        c = _Cfg()
        c.n_pix, c.margin, c.degree = int(n_pix), int(margin), int(degree)
        c.n_classes = int(n_classes)
        for i in range(4):
            c.edges[i] = float(edges[i])
        self.n_classes = c.n_classes
        c.n_arms = len(arm_start)
        for i, (s, g) in enumerate(zip(arm_start, arm_sigma)):
            c.arm_start[i] = int(s)
            c.arm_sigma[i] = float(g)
        c.dlog10 = float(dlog10)
        for i in range(5):
            c.lo[i] = float(box_lo[i])
            c.hi[i] = float(box_hi[i])
        self.c = c
        self.n_pix, self.margin, self.degree = c.n_pix, c.margin, c.degree
        self.n_ext = c.n_pix + 2 * c.margin
        self.box_lo = np.array(box_lo, dtype=np.float64)
        self.box_hi = np.array(box_hi, dtype=np.float64)

    @classmethod
    def from_shape(cls, shape, box_lo, box_hi, n_classes=1):
        return cls(shape.n_pix, shape.margin, shape.degree, shape.dlog10, box_lo, box_hi,
                   shape.arm_start, shape.arm_sigma_kms, n_classes=n_classes)

    def normalise(self, phys):
        """Physical (Teff K, logg, [Fe/H], RV, sigma) -> u in the box [-1, 1]."""
        phys = np.asarray(phys, dtype=np.float64)
        th = phys.copy()
        th[..., 0] = np.log10(phys[..., 0])
        return 2.0 * (th - self.box_lo) / (self.box_hi - self.box_lo) - 1.0

    def physical(self, u):
        u = np.asarray(u, dtype=np.float64)
        th = self.box_lo + 0.5 * (u + 1.0) * (self.box_hi - self.box_lo)
        th[..., 0] = 10.0 ** th[..., 0]
        return th


def features(x):
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    phi = np.empty(N_BASIS)
    dphi = np.empty((3, N_BASIS))
    lib.orc_features(_d(x), _d(phi), _d(dphi))
    return phi, dphi


def legendre(n, x):
    return _load().orc_legendre(int(n), float(x))


def kernel(mu, sig, margin):
    lib = _load()
    n = 2 * margin + 1
    G, Gm, Gs = np.zeros(n), np.zeros(n), np.zeros(n)
    H = lib.orc_kernel(float(mu), float(sig), int(margin), _d(G), _d(Gm), _d(Gs))
    T = 2 * H + 1
    return H, G[:T].copy(), Gm[:T].copy(), Gs[:T].copy()


def convolve(fp, G, margin, n_pix):
    lib = _load()
    fp = np.ascontiguousarray(fp, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    H = (G.size - 1) // 2
    out = np.zeros(n_pix)
    lib.orc_convolve(_d(fp), fp.size, _d(G), H, int(margin), 0, int(n_pix), _d(out))
    return out


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def evaluate(cfg: Config, obs, ivar, basis, u):
    """Model at fixed normalised u for one spectrum; dict of FP64 results."""
    lib = _load()
    obs, ivar, basis = _f32(obs), _f32(ivar), _f32(basis)
    u = np.ascontiguousarray(u, dtype=np.float64)
    P, nd = cfg.n_pix, cfg.degree + 1
    out = dict(fp=np.empty(cfg.n_ext), fpp=np.empty(P), b=np.empty(nd), model=np.empty(P),
               grad=np.empty(5), jac=np.empty((5, P)))
    chi2 = ctypes.c_double()
    neff = ctypes.c_int()
    flags = ctypes.c_uint()
    rc = lib.orc_eval(ctypes.byref(cfg.c), _f(obs), _f(ivar), _f(basis), _d(u), _d(out["fp"]),
                      _d(out["fpp"]), _d(out["b"]), _d(out["model"]), ctypes.byref(chi2),
                      ctypes.byref(neff), _d(out["grad"]), _d(out["jac"]), ctypes.byref(flags))
    out.update(rc=rc, chi2=chi2.value, n_eff=neff.value, flags=flags.value)
    out["J"] = chi2.value / neff.value if neff.value > 0 else float("nan")
    return out


def residual(cfg: Config, obs, ivar, basis, u, b, want_jac=True):
    lib = _load()
    obs, ivar, basis = _f32(obs), _f32(ivar), _f32(basis)
    u = np.ascontiguousarray(u, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    r = np.empty(cfg.n_pix)
    jac = np.empty((cfg.n_pix, 5 + cfg.degree + 1)) if want_jac else None
    lib.orc_residual(ctypes.byref(cfg.c), _f(obs), _f(ivar), _f(basis), _d(u), _d(b), _d(r), _d(jac))
    return (r, jac) if want_jac else r


def fit(cfg: Config, obs, ivar, basis, u0, max_iter=200):
    """Levenberg-Marquardt fit of one spectrum from normalised start u0."""
    lib = _load()
    obs, ivar, basis = _f32(obs), _f32(ivar), _f32(basis)
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    u = np.empty(5)
    b = np.empty(cfg.degree + 1)
    cov_u = np.empty((5, 5))
    cov_p = np.empty((5, 5))
    chi2 = ctypes.c_double()
    neff = ctypes.c_int()
    nit = ctypes.c_int()
    flags = ctypes.c_uint()
    rc = lib.orc_fit(ctypes.byref(cfg.c), _f(obs), _f(ivar), _f(basis), _d(u0), int(max_iter),
                     _d(u), _d(b), ctypes.byref(chi2), ctypes.byref(neff), _d(cov_u), _d(cov_p),
                     ctypes.byref(nit), ctypes.byref(flags))
    return dict(rc=rc, u=u, b=b, chi2=chi2.value, n_eff=neff.value, cov_u=cov_u, cov=cov_p,
                n_iter=nit.value, flags=flags.value, params=cfg.physical(u))


def covariance(cfg: Config, obs, ivar, basis, u):
    lib = _load()
    obs, ivar, basis = _f32(obs), _f32(ivar), _f32(basis)
    u = np.ascontiguousarray(u, dtype=np.float64)
    cov_u = np.empty((5, 5))
    cov_p = np.empty((5, 5))
    rc = lib.orc_covariance(ctypes.byref(cfg.c), _f(obs), _f(ivar), _f(basis), _d(u), _d(cov_u),
                            _d(cov_p))
    return dict(rc=rc, cov_u=cov_u, cov=cov_p)


def class_weights(cfg: Config, u):
    """Emulator class weights at normalised u and their derivatives in u_1."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64)
    w = np.zeros(3)
    dw = np.zeros(3)
    lib.orc_class_weights(ctypes.byref(cfg.c), _d(u), _d(w), _d(dw))
    return w[:max(cfg.n_classes, 1)], dw[:max(cfg.n_classes, 1)]


def resample(src, lam0, dlam, n_out, lg0, dlog10):
    """Flux-conserving resampling of rows of ``src`` (linear grid, bin
    centres lam0 + i dlam) onto the log grid 10^(lg0 + j dlog10), j < n_out.
    Returns (out [rows, n_out] float64, all targets inside the source)."""
    lib = _load()
    src = np.atleast_2d(_f32(src))
    out = np.empty((src.shape[0], n_out))
    ok = True
    for r in range(src.shape[0]):
        row = np.ascontiguousarray(src[r])
        o = np.empty(n_out)
        rc = lib.orc_resample(int(row.size), float(lam0), float(dlam), _f(row), int(n_out),
                              float(lg0), float(dlog10), _d(o))
        out[r] = o
        ok = ok and rc == 0
    return out, ok


def stop_step(ell, n_max, window, tol):
    """First step count at which stopping rule 2 or 3 holds on the loss
    history ell (ell[t] after t steps), else n_max; returns (t, rule)."""
    lib = _load()
    ell = np.ascontiguousarray(ell, dtype=np.float64)
    if ell.size < n_max:
        raise ValueError("ell needs at least n_max entries")
    rule = ctypes.c_int()
    t = lib.orc_stop_step(_d(ell), int(n_max), int(window), float(tol), ctypes.byref(rule))
    return t, rule.value


def adam_fit(cfg: Config, obs, ivar, basis, u0, n_max=500, lr=1e-2, betas=(0.9, 0.999),
             eps=1e-8, window=0, tol=1e-5, clean_every=0, clean_max=11):
    """FP64 Adam on chi2/n_eff from normalised start u0, with the stopping
    rules when window > 0 and the Clean mask updates when clean_every > 0.
    Returns u, steps, rule, loss history, final mask (keep) and params."""
    lib = _load()
    obs, ivar, basis = _f32(obs), _f32(ivar), _f32(basis)
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    u = np.empty(5)
    ell = np.empty(n_max + 1)
    steps = ctypes.c_int()
    rule = ctypes.c_int()
    keep = np.empty(cfg.n_pix, dtype=np.uint8)
    lib.orc_adam_fit(ctypes.byref(cfg.c), _f(obs), _f(ivar), _f(basis), _d(u0), int(n_max),
                     float(lr), float(betas[0]), float(betas[1]), float(eps), int(window),
                     float(tol), int(clean_every), int(clean_max), _d(u), ctypes.byref(steps),
                     ctypes.byref(rule), _d(ell), keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return dict(u=u, steps=steps.value, rule=rule.value, ell=ell[:steps.value + 1].copy(),
                keep=keep, params=cfg.physical(u))


def clean_mask(obs, ivar, model, f_shift):
    """Clean outlier mask of one spectrum: keep (1) / masked (0) per pixel,
    the number of masked valid pixels, the accepted k and the D passes."""
    lib = _load()
    obs, ivar = _f32(obs), _f32(ivar)
    model = np.ascontiguousarray(model, dtype=np.float64)
    n = obs.shape[0]
    keep = np.empty(n, dtype=np.uint8)
    k = ctypes.c_double()
    it = ctypes.c_int()
    masked = lib.orc_clean(int(n), _f(obs), _f(ivar), _d(model), float(f_shift),
                           keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(k),
                           ctypes.byref(it))
    return dict(keep=keep, masked=masked, k=k.value, d_iters=it.value)


def adam_fit_many(cfg: Config, obs, ivar, basis, init_phys, threads=None, **kw):
    """adam_fit of each row on a thread pool; returns a list of dicts."""
    n = obs.shape[0]
    u0 = cfg.normalise(init_phys)
    threads = threads or os.cpu_count() or 1
    basis = _f32(basis)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(adam_fit, cfg, obs[i], ivar[i], basis, u0[i], **kw) for i in range(n)]
        return [f.result() for f in futs]


def fit_many(cfg: Config, obs, ivar, basis, init_phys, max_iter=200, threads=None):
    """Fit each row independently on a thread pool; returns a list of dicts."""
    n = obs.shape[0]
    u0 = cfg.normalise(init_phys)
    threads = threads or os.cpu_count() or 1
    basis = _f32(basis)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        futs = [ex.submit(fit, cfg, obs[i], ivar[i], basis, u0[i], max_iter) for i in range(n)]
        return [f.result() for f in futs]
