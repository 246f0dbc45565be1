"""Levenberg-Marquardt polish on the GPU (damped Gauss-Newton with the
continuum profiled out) against the oracle's Levenberg-Marquardt fit over
(u, b): both reach the same minimiser of chi2, so the fitted values must
agree far inside the Adam tolerances."""

import numpy as np
import pytest
import torch

import oracle
import paper_2512_24840_amd as lasp
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name, wave_grid

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
DEV = torch.device("cuda:0")
FIT_TOL = np.array([2.0, 0.005, 0.005, 0.2])
TIGHT = FIT_TOL / 10


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def problem(name, n, cid):
    shape = shape_by_name(name)
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, cid, 0, n)
    return shape, basis, batch


def gpu_fit(shape, basis, batch, n_steps, polish, sl=slice(None)):
    arms = lasp.Arms(shape.arm_start, shape.arm_sigma_kms) if shape.arm_start else None
    res = lasp.fit_group(to_dev(batch.obs[sl]), to_dev(batch.ivar[sl]), wave_grid(shape),
                         to_dev(basis), to_dev(batch.init[sl]), n_steps, margin=shape.margin,
                         degree=shape.degree, arms=arms, polish_iters=polish)
    torch.cuda.synchronize()
    return res.params.cpu().numpy().astype(np.float64), res.status.cpu().numpy()


@pytest.mark.parametrize("name,n_steps,polish", [("lamost1550", 0, 30), ("lamost3900", 0, 30),
                                                 ("desi7800", 0, 30), ("lamost3900", 100, 12)])
def test_polish_reaches_the_oracle_lm_minimiser(name, n_steps, polish):
    print(f"[LM polish] {name} B=8 adam {n_steps} + polish {polish}", flush=True)
    shape, basis, batch = problem(name, 8, 61)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    p, st = gpu_fit(shape, basis, batch, n_steps, polish)
    ref = oracle.fit_many(cfg, batch.obs, batch.ivar, basis, batch.init)
    err = np.array([np.abs(p[i] - ref[i]["params"])[:4] for i in range(8)])
    print("  max |d| (Teff, logg, [Fe/H], RV):", err.max(axis=0), flush=True)
    assert not np.any(st & lasp.ST_POLISH_LIMIT), st
    assert np.all(err <= TIGHT), err


def test_polish_limit_is_flagged_and_fits_are_isolated():
    print("[LM polish] limit flag, alone == in group", flush=True)
    shape, basis, batch = problem("lamost1550", 6, 62)
    p1, st1 = gpu_fit(shape, basis, batch, 0, 1)
    assert np.all(st1 & lasp.ST_POLISH_LIMIT)
    p, st = gpu_fit(shape, basis, batch, 20, 8)
    for i in (0, 5):
        pa, sa = gpu_fit(shape, basis, batch, 20, 8, slice(i, i + 1))
        assert np.array_equal(pa[0], p[i]) and sa[0] == st[i], i


def test_plain_lm_with_200_iterations_alone_equals_in_group():
    """The plain method (no Adam steps, at most 200 LM iterations): the call
    stops enqueuing iterations once every spectrum has stopped, so a fit
    alone ends soon after its own stop while in the group the iterations
    run on until the slowest spectrum stops -- the results must agree bit
    for bit (a stopped spectrum's iterations change nothing), sit within a
    tenth of the fit tolerances of the oracle's LM, and none may reach the
    iteration limit."""
    print("[LM polish] plain LM, 200 iterations: alone == in group, vs the oracle", flush=True)
    shape, basis, batch = problem("lamost1550", 8, 61)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    p, st = gpu_fit(shape, basis, batch, 0, 200)
    assert not np.any(st & lasp.ST_POLISH_LIMIT), st
    for i in range(8):
        pa, sa = gpu_fit(shape, basis, batch, 0, 200, slice(i, i + 1))
        assert np.array_equal(pa[0], p[i]) and sa[0] == st[i], i
    ref = oracle.fit_many(cfg, batch.obs, batch.ivar, basis, batch.init)
    err = np.array([np.abs(p[i] - ref[i]["params"])[:4] for i in range(8)])
    assert np.all(err <= TIGHT), err
