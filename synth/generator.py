"""Seeded synthetic workloads with the shapes of the paper's surveys.

Stand-ins (the paper's LAMOST/DESI spectra and ELODIE emulator coefficients
are not available):

* LAMOST-like grids: logarithmic wavelength grid with a 1e-4 dex step
  (Section "Application to DESI" fixes that step; Section "Data
  Preprocessing" gives 1327 px over 4200-5700 A, which is that step).
* DESI-like grid: 3600-9800 A with resolving power rising from 2000 to 5000
  (Section "Application to DESI"), modelled as three equal-pixel arms with a
  fixed instrumental sigma each.
* Interpolator: K = 20 coefficient spectra, one per monomial of total degree
  <= 3 in the three normalised atmospheric coordinates, built from 300 seeded
  Gaussian absorption lines whose depths are polynomials in those coordinates
  (the role of the polynomial emulator of Eq. 1).

Every array is drawn from numpy ``Generator(PCG64)`` streams keyed by
``SeedSequence([id, index])`` so any single item regenerates on its own.

Observed spectra are simulated in closed form: each line, Doppler shifted by
exp(v/c) and convolved analytically with the Gaussian broadening profile, is
averaged over each pixel's wavelength bin, multiplied by a smooth continuum
written in the power basis, and given Gaussian noise.  None of this is the
discrete model that the fit evaluates.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import erf

C_KMS = 299792.458

# Normalisation box for (log10 Teff, log g, [Fe/H], RV km/s, sigma km/s): the
# prior ranges of the synthetic workloads.
BOX_LO = np.array([math.log10(4000.0), 1.0, -2.5, -300.0, 50.0])
BOX_HI = np.array([math.log10(8000.0), 5.0, 0.5, 300.0, 150.0])

# Exponents (a, b, c) of the 20 monomials x1^a x2^b x3^c, graded by total
# degree and lexicographic within a degree.  Row k of the basis multiplies
# monomial k.
EXPONENTS = (
    (0, 0, 0),
    (1, 0, 0), (0, 1, 0), (0, 0, 1),
    (2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2),
    (3, 0, 0), (2, 1, 0), (2, 0, 1), (1, 2, 0), (1, 1, 1), (1, 0, 2),
    (0, 3, 0), (0, 2, 1), (0, 1, 2), (0, 0, 3),
)
N_BASIS = len(EXPONENTS)
N_LINES = 300
_DEPTH_SCALE = {1: 0.25, 2: 0.08, 3: 0.03}
_WINDOW_SIGMAS = 7.0


@dataclasses.dataclass(frozen=True)
class Shape:
    name: str
    shape_id: int
    lam0: float          # centre of pixel 0, Angstrom
    dlog10: float        # grid step in log10(lambda)
    n_pix: int
    margin: int          # extra basis columns on each side of the pixel range
    degree: int          # continuum polynomial degree
    arm_start: tuple = ()       # first pixel of each arm (empty: one arm, no instrument term)
    arm_sigma_kms: tuple = ()   # instrumental Gaussian sigma of each arm, km/s

    @property
    def n_ext(self) -> int:
        return self.n_pix + 2 * self.margin


def _desi_shape() -> Shape:
    n = 7800
    step = math.log10(9800.0 / 3600.0) / (n - 1)
    res = (2000.0, 3500.0, 5000.0)
    sig = tuple(C_KMS / (2.0 * math.sqrt(2.0 * math.log(2.0)) * r) for r in res)
    return Shape("desi7800", 5, 3600.0, step, n, 64, 10, (0, 2600, 5200), sig)


_SHAPES = {
    "lamost1550": Shape("lamost1550", 1, 3850.0, 1e-4, 1550, 64, 8),
    "lamost3900": Shape("lamost3900", 2, 3700.0, 1e-4, 3900, 64, 10),
    "desi7800": _desi_shape(),
}


def shape_by_name(name: str, **overrides) -> Shape:
    """Named workload shape; keyword overrides build small test variants."""
    s = _SHAPES[name]
    return dataclasses.replace(s, **overrides) if overrides else s


def wave_grid(shape: Shape) -> np.ndarray:
    """Pixel-centre wavelengths (A), uniform in log10."""
    return shape.lam0 * 10.0 ** (shape.dlog10 * np.arange(shape.n_pix, dtype=np.float64))


def _ext_grid(shape: Shape) -> np.ndarray:
    j = np.arange(shape.n_ext, dtype=np.float64) - shape.margin
    return shape.lam0 * 10.0 ** (shape.dlog10 * j)


def _bin_edges(centres: np.ndarray, dlog10: float) -> np.ndarray:
    """Edges of log-uniform pixel bins around ``centres`` (len+1 values)."""
    lo = centres * 10.0 ** (-0.5 * dlog10)
    return np.concatenate([lo, centres[-1:] * 10.0 ** (0.5 * dlog10)])


def _binned_gaussians(edges: np.ndarray, centre: np.ndarray, sigma: np.ndarray,
                      amp: np.ndarray) -> np.ndarray:
    """Sum over lines of amp * (mean of exp(-(l-c)^2/2s^2) over each bin).

    ``centre``, ``sigma``, ``amp`` have shape [n, L] (n spectra, L lines);
    returns [n, len(edges)-1].  Each line is integrated only over the bins
    within 7 sigma of its centre; the truncated wings are below 1e-10.
    """
    n, n_lines = centre.shape
    n_bins = edges.size - 1
    width = np.diff(edges)
    log_e0 = math.log(edges[0])
    dln = math.log(edges[1] / edges[0])
    lo = np.floor((np.log(np.maximum(centre - _WINDOW_SIGMAS * sigma, 1e-3)) - log_e0) / dln)
    hi = np.ceil((np.log(centre + _WINDOW_SIGMAS * sigma) - log_e0) / dln)
    span = int(max(1, (hi - lo).max())) + 1
    first = np.clip(lo.astype(np.int64), 0, n_bins)
    k = first[..., None] + np.arange(span + 1)                       # edge indices
    valid_edge = k <= n_bins
    kk = np.minimum(k, n_bins)
    z = (edges[kk] - centre[..., None]) / (math.sqrt(2.0) * sigma[..., None])
    cdf = erf(z)
    seg = np.diff(cdf, axis=-1)                                       # [n, L, span]
    bins = kk[..., :-1]
    ok = valid_edge[..., 1:] & (bins < n_bins)
    contrib = (amp * sigma * math.sqrt(math.pi / 2.0))[..., None] * seg
    contrib = np.where(ok, contrib, 0.0)
    rows = np.broadcast_to(np.arange(n)[:, None, None], bins.shape)
    flat = (rows * n_bins + np.where(ok, bins, 0)).ravel()
    out = np.bincount(flat, weights=contrib.ravel(), minlength=n * n_bins)
    return out.reshape(n, n_bins) / width


@dataclasses.dataclass
class LineList:
    centre: np.ndarray    # [L] rest wavelength, A
    sigma: np.ndarray     # [L] intrinsic Gaussian sigma, A
    coef: np.ndarray      # [L, 20] depth polynomial coefficients


def _monomials(x: np.ndarray) -> np.ndarray:
    """x: [n, 3] -> [n, 20] values of the monomials listed in EXPONENTS."""
    e = np.asarray(EXPONENTS, dtype=np.float64)                       # [20, 3]
    return np.prod(x[:, None, :] ** e[None, :, :], axis=-1)


# Effective-temperature regimes of the multi-class emulator (K): the cool
# class alone below the first edge, cool -> warm blended linearly in Teff
# between the first two, warm alone, warm -> hot blended between the last
# two, hot alone above (the paper's five regimes of the ELODIE emulator).
REGIME_EDGES = (4000.0, 4550.0, 7000.0, 9000.0)


def class_weights(teff: np.ndarray, edges=REGIME_EDGES) -> np.ndarray:
    """[n] Teff (K) -> [n, 3] weights of the cool, warm and hot classes."""
    t = np.asarray(teff, dtype=np.float64)
    a = np.clip((t - edges[0]) / (edges[1] - edges[0]), 0.0, 1.0)   # cool -> warm
    b = np.clip((t - edges[2]) / (edges[3] - edges[2]), 0.0, 1.0)   # warm -> hot
    return np.stack([1.0 - a, a * (1.0 - b), a * b], axis=-1)


def _line_list(shape: Shape, cls: int = 0) -> LineList:
    key = [shape.shape_id, 0xBA515] if cls == 0 else [shape.shape_id, 0xBA515, cls]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(key)))
    ext = _ext_grid(shape)
    centre = rng.uniform(ext[0], ext[-1], N_LINES)
    sigma = rng.uniform(0.5, 3.0, N_LINES)
    a0 = rng.uniform(0.05, 0.6, N_LINES)
    coef = np.zeros((N_LINES, N_BASIS))
    coef[:, 0] = a0
    for k in range(1, N_BASIS):
        deg = sum(EXPONENTS[k])
        coef[:, k] = a0 * rng.normal(0.0, _DEPTH_SCALE[deg], N_LINES)
    return LineList(centre, sigma, coef)


def make_basis(shape: Shape, n_classes: int = 1):
    """Interpolator coefficient spectra [20 * n_classes, n_pix + 2*margin]
    (float32) and the line list (a list of n_classes lists when n_classes > 1).

    Row 0 of each class is the line-free unit level minus the constant part
    of every line's depth; row k > 0 carries monomial k's share of the
    depths.  Each line profile is averaged over the pixel's wavelength bin
    (flux conserving).  Class c (cool, warm, hot) has its own line depths.
    """
    edges = _bin_edges(_ext_grid(shape), shape.dlog10)
    all_lines = [_line_list(shape, c) for c in range(n_classes)]
    basis = np.zeros((N_BASIS * n_classes, shape.n_ext))
    for c, lines in enumerate(all_lines):
        for k in range(N_BASIS):
            prof = _binned_gaussians(edges, lines.centre[None, :], lines.sigma[None, :],
                                     lines.coef[None, :, k])[0]
            basis[c * N_BASIS + k] = (1.0 if k == 0 else 0.0) - prof
    return basis.astype(np.float32), (all_lines[0] if n_classes == 1 else all_lines)


def linear_grid_basis(shape: Shape, n_classes: int = 1, step: float = 0.2, pad: float = 20.0):
    """The same coefficient spectra sampled like an emulator's output: on a
    linear wavelength grid of ``step`` A covering the extended log grid with
    ``pad`` A to spare, each line averaged over the linear bins.  Returns
    (lambda0 [A, centre of the first bin], step, [rows, n] float32)."""
    ext = _ext_grid(shape)
    lo = ext[0] * 10.0 ** (-0.5 * shape.dlog10) - pad
    hi = ext[-1] * 10.0 ** (0.5 * shape.dlog10) + pad
    n = int(math.ceil((hi - lo) / step))
    centres = lo + step * (np.arange(n) + 0.5)
    edges = lo + step * np.arange(n + 1)
    all_lines = [_line_list(shape, c) for c in range(n_classes)]
    out = np.zeros((N_BASIS * n_classes, n))
    for c, lines in enumerate(all_lines):
        for k in range(N_BASIS):
            prof = _linear_binned_gaussians(edges, lines.centre, lines.sigma, lines.coef[:, k])
            out[c * N_BASIS + k] = (1.0 if k == 0 else 0.0) - prof
    return float(centres[0]), float(step), out.astype(np.float32)


def _linear_binned_gaussians(edges, centre, sigma, amp):
    """Sum of amp * (mean of each Gaussian over linear bins ``edges``)."""
    width = np.diff(edges)
    out = np.zeros(edges.size - 1)
    for c, s, a in zip(centre, sigma, amp):
        i0 = max(0, int(np.searchsorted(edges, c - _WINDOW_SIGMAS * s)) - 1)
        i1 = min(edges.size - 1, int(np.searchsorted(edges, c + _WINDOW_SIGMAS * s)) + 1)
        e = edges[i0:i1 + 1]
        cdf = erf((e - c) / (math.sqrt(2.0) * s))
        out[i0:i1] += a * s * math.sqrt(math.pi / 2.0) * np.diff(cdf)
    return out / width


def _normalise(theta: np.ndarray) -> np.ndarray:
    return 2.0 * (theta - BOX_LO) / (BOX_HI - BOX_LO) - 1.0


@dataclasses.dataclass
class SpectraBatch:
    obs: np.ndarray        # [n, P] float32
    ivar: np.ndarray       # [n, P] float32, 0 = masked
    init: np.ndarray       # [n, 5] float32 (Teff K, log g, [Fe/H], RV km/s, sigma km/s)
    truth: np.ndarray      # [n, 5] float64, same units
    snr: np.ndarray        # [n]
    scale: np.ndarray      # [n] continuum scale


def _item_rng(config_id: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([config_id, index])))


def make_spectra(shape: Shape, lines: LineList, config_id: int, start: int, count: int,
                 init_mode: str = "perturbed", noise: bool = True,
                 chunk: int = 32) -> SpectraBatch:
    """Simulate ``count`` observed spectra with item indices start..start+count-1."""
    P = shape.n_pix
    lam = wave_grid(shape)
    edges = _bin_edges(lam, shape.dlog10)
    xnode = -1.0 + 2.0 * np.arange(P) / P
    obs = np.empty((count, P), np.float32)
    ivar = np.empty((count, P), np.float32)
    init = np.empty((count, 5), np.float32)
    truth = np.empty((count, 5))
    snr_all = np.empty(count)
    scale_all = np.empty(count)
    nad = (lam >= 5880.0) & (lam <= 5905.0)
    arms = list(shape.arm_start) or [0]
    arm_sig = list(shape.arm_sigma_kms) or [0.0]
    arm_end = arms[1:] + [P]

    for c0 in range(0, count, chunk):
        n = min(chunk, count - c0)
        rngs = [_item_rng(config_id, start + c0 + i) for i in range(n)]
        th = np.empty((n, 5))
        for i, r in enumerate(rngs):
            teff = r.uniform(4000.0, 8000.0)
            th[i] = (math.log10(teff), r.uniform(1.0, 5.0), r.uniform(-2.5, 0.5),
                     r.uniform(-300.0, 300.0), r.uniform(50.0, 150.0))
        classes = lines if isinstance(lines, list) else [lines]
        cw = class_weights(10.0 ** th[:, 0]) if len(classes) > 1 else np.ones((n, 1))
        flux = np.zeros((n, P))
        for ci, cl in enumerate(classes):
            depth = _monomials(_normalise(th)[:, :3]) @ cl.coef.T     # [n, L]
            dop = np.exp(th[:, 3:4] / C_KMS)                            # [n, 1]
            cen = cl.centre[None, :] * dop
            sig_l = cl.sigma[None, :] * dop
            fc = np.empty((n, P))
            for a, (j0, j1) in enumerate(zip(arms, arm_end)):
                s_eff = np.sqrt(th[:, 4:5] ** 2 + arm_sig[a] ** 2)
                s_tot = np.sqrt(sig_l ** 2 + (cen * s_eff / C_KMS) ** 2)
                amp = depth * sig_l / s_tot
                prof = _binned_gaussians(edges[j0:j1 + 1], cen, s_tot, amp)
                fc[:, j0:j1] = 1.0 - prof
            flux += cw[:, ci:ci + 1] * fc
        for i, r in enumerate(rngs):
            s = 10.0 ** r.uniform(1.0, 3.0)
            while True:
                cpow = np.concatenate([[1.0], r.normal(0.0, 0.2 / np.arange(1, shape.degree + 1))])
                cont = s * np.polynomial.polynomial.polyval(xnode, cpow)
                if cont.min() >= 0.2 * s:
                    break
            clean = cont * flux[i]
            snr = r.uniform(10.0, 100.0)
            sig_n = float(np.median(clean)) / snr
            o = clean + (sig_n * r.standard_normal(P) if noise else 0.0)
            iv = np.full(P, 1.0 / sig_n ** 2)
            iv[nad] = 0.0
            bad = r.random(P) < 0.005
            iv[bad] = 0.0
            o[bad] *= 10.0
            pert = r.standard_normal(4)
            if init_mode == "perturbed":
                g = np.array([th[i, 0] + 0.02 * pert[0], th[i, 1] + 0.25 * pert[1],
                              th[i, 2] + 0.2 * pert[2], th[i, 3] + 15.0 * pert[3], 100.0])
            elif init_mode == "fixed7500":
                g = np.array([math.log10(7500.0), 3.0, -0.5, th[i, 3] + 50.0 * pert[3], 100.0])
            else:
                raise ValueError(init_mode)
            g = np.clip(g, BOX_LO, BOX_HI)
            k = c0 + i
            obs[k] = o
            ivar[k] = iv
            init[k] = (10.0 ** g[0], g[1], g[2], g[3], g[4])
            truth[k] = (10.0 ** th[i, 0], th[i, 1], th[i, 2], th[i, 3], th[i, 4])
            snr_all[k] = snr
            scale_all[k] = s
    return SpectraBatch(obs, ivar, init, truth, snr_all, scale_all)


def _chunk(args):
    shape, lines, config_id, start, count, init_mode, noise = args
    return make_spectra(shape, lines, config_id, start, count, init_mode, noise)


def make_spectra_parallel(shape: Shape, lines: LineList, config_id: int, start: int, count: int,
                          init_mode: str = "perturbed", noise: bool = True,
                          workers: int | None = None, chunk: int = 512) -> SpectraBatch:
    """make_spectra split over worker processes (identical result: every item
    has its own random stream).  Call before the process touches the GPU."""
    import multiprocessing as mp
    import os

    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or count <= chunk:
        return make_spectra(shape, lines, config_id, start, count, init_mode, noise)
    jobs = [(shape, lines, config_id, s, min(chunk, start + count - s), init_mode, noise)
            for s in range(start, start + count, chunk)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_chunk, jobs)
    return SpectraBatch(*(np.concatenate([getattr(p, f.name) for p in parts])
                          for f in dataclasses.fields(SpectraBatch)))


def poisson_requests(spectra_per_s: float, duration_s: float, seed: int,
                     lanes=("lamost3900", "desi7800"), weights=(0.5, 0.5),
                     size_min: int = 1, size_max: int = 4096):
    """Seeded request stream: exponential inter-arrival times at a request
    rate that carries ``spectra_per_s`` on average, group sizes log-uniform
    on [size_min, size_max], lanes drawn with ``weights``.  Returns a list of
    (arrival time s, lane, size)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([5, seed])))
    lo, hi = math.log(size_min), math.log(size_max + 1)
    mean_size = (math.exp(hi) - math.exp(lo)) / (hi - lo)
    rate = spectra_per_s / mean_size
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration_s:
            return out
        lane = lanes[int(rng.choice(len(lanes), p=np.asarray(weights) / np.sum(weights)))]
        n = int(min(max(math.floor(math.exp(rng.uniform(lo, hi))), size_min), size_max))
        out.append((t, lane, n))
