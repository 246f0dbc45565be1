"""Pins of the oracle's optimisation stage (Section 2.2, stage 8): the
stopping rules on loss sequences whose stopping step has a closed form, the
Adam trajectory against torch.optim.Adam, a fixed point, and agreement of
the Adam endpoint with the Levenberg-Marquardt minimiser."""

import math

import numpy as np
import pytest
import torch

import oracle
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name

pytestmark = pytest.mark.usefixtures("oracle_lib")

W, TOL = 50, 1e-5


def test_constant_loss_stops_by_rule_2_after_one_window():
    assert oracle.stop_step(np.full(300, 0.7), 300, W, TOL) == (W, 2)


def test_strictly_rising_loss_stops_by_rule_3_after_one_window():
    ell = 1.0 + 0.01 * np.arange(300)
    assert oracle.stop_step(ell, 300, W, TOL) == (W, 3)


def test_one_fall_restarts_the_rising_count():
    ell = 1.0 + 0.01 * np.arange(300)
    ell[30:] -= 0.25                   # the loss falls at step 30 only
    assert oracle.stop_step(ell, 300, W, TOL) == (30 + W, 3)


@pytest.mark.parametrize("slope,expect", [(0.5 * TOL / W, (W, 2)), (2.0 * TOL / W, (400, 1))])
def test_linear_descent_stops_only_when_a_window_changes_less_than_tol(slope, expect):
    ell = 1.0 - slope * np.arange(400)
    assert oracle.stop_step(ell, 400, W, TOL) == expect


def test_geometric_approach_stops_at_the_closed_form_step():
    # ell_t = 1 + c r^t: the change over a window is c r^(t-W) (1 - r^W), below
    # tol from t = W + ceil(log(tol / (c (1 - r^W))) / log r) on
    c, r = 0.3, 0.97
    ell = 1.0 + c * r ** np.arange(2000)
    k = math.log(TOL / (c * (1 - r ** W))) / math.log(r)
    expect = W + math.floor(k) + 1 if k == math.floor(k) else W + math.ceil(k)
    assert oracle.stop_step(ell, 2000, W, TOL) == (expect, 2)


def test_window_zero_never_stops_early():
    assert oracle.stop_step(np.full(100, 1.0), 100, 0, TOL) == (100, 1)


def small_problem(n=3, seed=5):
    shape = shape_by_name("lamost1550")
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, seed, 0, n)
    return shape, basis, batch, oracle.Config.from_shape(shape, BOX_LO, BOX_HI)


def test_adam_trajectory_matches_torch_optim_adam_fed_the_oracle_gradient():
    shape, basis, batch, cfg = small_problem(2)
    for i in range(2):
        u0 = cfg.normalise(batch.init[i])
        ours = oracle.adam_fit(cfg, batch.obs[i], batch.ivar[i], basis, u0, n_max=40, window=0)
        assert ours["steps"] == 40 and ours["rule"] == 1
        p = torch.tensor(u0, dtype=torch.float64, requires_grad=True)
        opt = torch.optim.Adam([p], lr=1e-2)
        ell = []
        for _ in range(40):
            ev = oracle.evaluate(cfg, batch.obs[i], batch.ivar[i], basis, p.detach().numpy())
            ell.append(math.sqrt(ev["chi2"] / ev["n_eff"]))
            p.grad = torch.from_numpy(ev["grad"].copy())
            opt.step()
        np.testing.assert_allclose(ours["u"], p.detach().numpy(), rtol=0, atol=1e-12)
        np.testing.assert_allclose(ours["ell"][:40], ell, rtol=1e-13)


def test_fully_masked_spectrum_is_a_fixed_point_that_stops_after_one_window():
    shape, basis, batch, cfg = small_problem(1)
    u0 = cfg.normalise(batch.init[0])
    res = oracle.adam_fit(cfg, batch.obs[0], np.zeros_like(batch.ivar[0]), basis, u0,
                          n_max=500, window=W, tol=TOL)
    assert (res["steps"], res["rule"]) == (W, 2)
    np.testing.assert_array_equal(res["u"], u0)


def test_adam_with_stopping_rules_reaches_the_lm_minimiser():
    shape, basis, batch, cfg = small_problem(6, seed=9)
    ad = oracle.adam_fit_many(cfg, batch.obs, batch.ivar, basis, batch.init, n_max=500,
                              window=W, tol=TOL)
    lm = oracle.fit_many(cfg, batch.obs, batch.ivar, basis, batch.init)
    for a, l in zip(ad, lm):
        assert a["rule"] in (2, 3) and a["steps"] < 500
        d = np.abs(a["params"][:4] - l["params"][:4])
        assert d[0] <= 2.0 and d[1] <= 0.005 and d[2] <= 0.005 and d[3] <= 0.2, d
