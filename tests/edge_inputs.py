"""Inputs for the edge paths of the method (test infrastructure).

Each builder returns seeded inputs that drive one edge of the model at a
known place: the 0.1 px floor of the broadening width and the window clamped
at the basis margin (Eq. 5 and the window size after it), a nonpositive
least-squares continuum (the failed-fit test of Section 4.2 on the
multiplicative correction of Step 5), and parameters outside the
normalisation box.  Observed spectra for constructed truths are the oracle's
noiseless model at that truth times a smooth continuum, plus seeded noise.
"""

from __future__ import annotations

import numpy as np

import oracle
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name

C_KMS = 299792.458
# evaluation bits shared by the HIP status word and the oracle's flags
GPU_SIGMA_FLOOR = 0x20
EVAL_MASK_ORACLE = (oracle.NONFINITE | oracle.NO_DATA | oracle.SINGULAR | oracle.CONT_NONPOS
                    | oracle.OUT_OF_BOX | oracle.SIGMA_FLOOR)


def gpu_flags_as_oracle(st: int) -> int:
    """The HIP status bits in the oracle's numbering (input and evaluation
    bits only)."""
    st = int(st)
    out = st & (oracle.NONFINITE | oracle.NO_DATA | oracle.SINGULAR | oracle.CONT_NONPOS
                | oracle.OUT_OF_BOX)
    if st & GPU_SIGMA_FLOOR:
        out |= oracle.SIGMA_FLOOR
    return out


def oracle_flags(res: dict) -> int:
    return int(res["flags"]) & EVAL_MASK_ORACLE


def min_continuum(res: dict) -> float:
    """Smallest continuum value over the pixels in an oracle evaluation."""
    return float(np.min(res["model"] / res["fpp"]))


def width_px(shape, sigma_kms):
    """Broadening width in pixels of the grid of ``shape``."""
    return sigma_kms / (C_KMS * np.log(10.0) * shape.dlog10)


def u_of_sigma(sigma_kms, box_lo=BOX_LO, box_hi=BOX_HI):
    return 2.0 * (sigma_kms - box_lo[4]) / (box_hi[4] - box_lo[4]) - 1.0


def model_obs(cfg, shape, basis, u_true, seed, snr=50.0, scale=50.0):
    """Noisy spectrum of the oracle's model at u_true times a smooth
    continuum scale * (1 + 0.1 x); ivar uniform."""
    ev = oracle.evaluate(cfg, np.ones(shape.n_pix, np.float32),
                         np.ones(shape.n_pix, np.float32), basis, u_true)
    x = -1.0 + 2.0 * np.arange(shape.n_pix) / shape.n_pix
    clean = scale * (1.0 + 0.1 * x) * ev["fpp"]
    sn = float(np.median(np.abs(clean))) / snr
    rng = np.random.default_rng(seed)
    obs = (clean + rng.normal(0.0, sn, clean.size)).astype(np.float32)
    ivar = np.full(clean.size, 1.0 / sn ** 2, np.float32)
    return obs, ivar


def negative_flux_case(n, name="lamost1550", config_id=21):
    """Spectra of the workload whose first fifth of the pixels has negative
    flux (as in spectra with a failed sky subtraction): the least-squares
    continuum is negative there at any parameters."""
    shape = shape_by_name(name)
    basis, lines = make_basis(shape)
    b = make_spectra(shape, lines, config_id, 0, n)
    obs = b.obs.copy()
    obs[:, : shape.n_pix // 5] *= -0.3
    return shape, basis, obs, b.ivar.copy(), b.init.copy(), b.truth.copy()


def bump_basis_case(n, name="lamost1550", config_id=21):
    """A fit whose continuum is nonpositive at the start only.

    The u1 row of the basis gets a narrow negative bump (centre at 20 % of
    the extended grid, width 1.5 %, depth 2): at u1 = 1 the model F' changes
    sign inside the bump, the least-squares continuum follows it below zero,
    and the model cannot match the data there; at the truth u1 = -0.5 the
    bump only deepens a feature.  Returns the shape, the modified basis,
    obs, ivar, the start u0 [n, 5] and the truth u [n, 5] (normalised)."""
    shape = shape_by_name(name)
    basis, lines = make_basis(shape)
    c = np.arange(shape.n_ext)
    bump = 2.0 * np.exp(-0.5 * ((c / shape.n_ext - 0.2) / 0.015) ** 2)
    basis = basis.copy()
    basis[1] -= bump.astype(np.float32)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    b = make_spectra(shape, lines, config_id, 0, n)
    u_true = cfg.normalise(b.truth)
    u_true[:, 0] = -0.5
    obs = np.empty((n, shape.n_pix), np.float32)
    ivar = np.empty_like(obs)
    for i in range(n):
        obs[i], ivar[i] = model_obs(cfg, shape, basis, u_true[i], seed=i)
    u0 = u_true.copy()
    u0[:, 0] = 1.0
    return shape, basis, obs, ivar, u0.astype(np.float32), u_true


def out_of_box_case(name="lamost1550", config_id=22):
    """Four fits around the normalisation box, as (truth u, start u) pairs
    sharing one basis: (0) truth and start outside the box (Teff near
    9,800 K, RV 510 km/s); (1) start outside (log g -0.2, sigma 185 km/s),
    truth inside; (2) start at sigma = 3 km/s, below the 0.1 px width floor
    and outside the box, where d chi2 / d sigma is zero so sigma stays;
    (3) an ordinary fit inside the box."""
    shape = shape_by_name(name)
    basis, lines = make_basis(shape)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    truth = np.array([[1.6, 0.2, -0.1, 1.7, 0.0],
                      [0.1, 0.5, 0.2, -0.2, 0.0],
                      [-0.3, -0.2, 0.4, 0.3, 0.1],
                      [0.2, -0.4, -0.3, 0.1, -0.2]])
    start = truth.copy()
    start[0] += np.array([0.03, -0.05, 0.04, 0.02, 0.0])
    start[1, 1] = -1.6
    start[1, 4] = 1.7
    start[2, 4] = u_of_sigma(3.0)
    start[3] += np.array([-0.05, 0.08, 0.05, 0.04, 0.0])
    obs = np.empty((4, shape.n_pix), np.float32)
    ivar = np.empty_like(obs)
    for i in range(4):
        obs[i], ivar[i] = model_obs(cfg, shape, basis, truth[i], seed=100 + i)
    return shape, basis, obs, ivar, start.astype(np.float32), truth
