"""The edge-path inputs do what they are built for, by the oracle alone.

The GPU edge tests compare status bits and values with the oracle at the
points the GPU returns; these checks make sure each constructed case really
reaches its edge (so that the GPU comparison is not vacuous).
"""

import numpy as np
import pytest

import oracle
from edge_inputs import (bump_basis_case, min_continuum, negative_flux_case, oracle_flags,
                         out_of_box_case)
from synth import BOX_HI, BOX_LO

pytestmark = pytest.mark.usefixtures("oracle_lib")


def test_negative_flux_case_has_nonpositive_continuum():
    shape, basis, obs, ivar, init, _ = negative_flux_case(4)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    for i in range(4):
        r = oracle.evaluate(cfg, obs[i], ivar[i], basis, cfg.normalise(init[i]))
        assert r["flags"] & oracle.CONT_NONPOS
        assert min_continuum(r) < -1.0


def test_bump_case_is_nonpositive_at_the_start_only():
    """Section 4.2's failed-fit test must look at the returned point: here
    the continuum is nonpositive where the fit starts and positive, by a wide
    margin, where the oracle's FP64 Adam (500 steps, lr 1e-2) ends."""
    n = 8
    shape, basis, obs, ivar, u0, u_true = bump_basis_case(n)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    for i in range(n):
        r0 = oracle.evaluate(cfg, obs[i], ivar[i], basis, u0[i].astype(np.float64))
        assert r0["flags"] & oracle.CONT_NONPOS, i
        ad = oracle.adam_fit(cfg, obs[i], ivar[i], basis, u0[i].astype(np.float64), n_max=500)
        r1 = oracle.evaluate(cfg, obs[i], ivar[i], basis, ad["u"])
        assert oracle_flags(r1) == 0, i
        assert min_continuum(r1) > 20.0, i
        assert abs(ad["u"][0] - u_true[i, 0]) < 0.1, i


def test_out_of_box_case_reaches_its_edges():
    shape, basis, obs, ivar, start, truth = out_of_box_case()
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    expect_start = [oracle.OUT_OF_BOX, oracle.OUT_OF_BOX, oracle.OUT_OF_BOX | oracle.SIGMA_FLOOR, 0]
    expect_end = [oracle.OUT_OF_BOX, 0, oracle.OUT_OF_BOX | oracle.SIGMA_FLOOR, 0]
    for i in range(4):
        r0 = oracle.evaluate(cfg, obs[i], ivar[i], basis, start[i].astype(np.float64))
        assert oracle_flags(r0) == expect_start[i], i
        ad = oracle.adam_fit(cfg, obs[i], ivar[i], basis, start[i].astype(np.float64), n_max=500)
        r1 = oracle.evaluate(cfg, obs[i], ivar[i], basis, ad["u"])
        assert oracle_flags(r1) == expect_end[i], i
    # below the floor the width does not move: its derivative is zero
    ad = oracle.adam_fit(cfg, obs[2], ivar[2], basis, start[2].astype(np.float64), n_max=500)
    assert ad["u"][4] == start[2, 4].astype(np.float64)
