"""Golden facts printed in the paper, checked against the generator and oracle."""

import json
import math
import os

import numpy as np
import pytest

import oracle
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name, wave_grid

pytestmark = pytest.mark.usefixtures("oracle_lib")
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def test_lamost_window_has_1327_pixels_at_1e4_dex():
    lo, hi = GOLDEN["lamost_window_angstrom"]["value"]
    step = GOLDEN["log10_step"]["value"]
    n = int(math.floor(math.log10(hi / lo) / step)) + 1
    assert n == GOLDEN["lamost_window_pixels"]["value"]
    shape = shape_by_name("lamost3900", lam0=lo, n_pix=n)
    lam = wave_grid(shape)
    assert lam[0] == lo and lam[-1] <= hi and lam[-1] * 10 ** step > hi


def test_kernel_taps_follow_eq5():
    for mu, sig, taps in GOLDEN["kernel_cases"]["value"]:
        H, G, _, _ = oracle.kernel(mu, sig, 64)
        assert G.size == taps == 2 * math.ceil(abs(mu) + 5 * sig) + 1


def test_legendre_nodes_as_printed():
    # x_j = -1 + 2(j-1)/p for j = 1..p: the first node is -1, the last
    # is -1 + 2(p-1)/p; the oracle's continuum at node j must use exactly that.
    P, D = 64, 3
    shape = shape_by_name("lamost3900", n_pix=P, margin=8, degree=D)
    basis, lines = make_basis(shape)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    u = np.zeros(5)
    ivar = np.ones(P, np.float32)
    fpp = oracle.evaluate(cfg, np.ones(P, np.float32), ivar, basis, u)["fpp"]
    x = np.array([-1 + 2 * (j - 1) / P for j in range(1, P + 1)])
    obs = ((1.0 + 0.3 * x ** 3) * fpp).astype(np.float32)   # cubic = P3-representable
    ev = oracle.evaluate(cfg, obs, ivar, basis, u)
    assert ev["chi2"] < 1e-10 * float((obs.astype(np.float64) ** 2).sum())
    assert x[0] == -1.0 and x[-1] == pytest.approx(1 - 2 / P)


@pytest.mark.parametrize("name,n", [("lamost3900", 24), ("desi7800", 8)])
def test_recovers_truth_of_analytic_simulator(name, n):
    """Noiseless spectra from the generator's closed-form line physics (shift
    by exp(v/c), analytic Gaussian broadening, bin averaging) are fitted back
    to their truths: this pins the pixel/km s^-1 conversions, the box
    mapping and the per-arm widths against an independent computation."""
    shape = shape_by_name(name)
    basis, lines = make_basis(shape)
    b = make_spectra(shape, lines, 41, 0, n, noise=False)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    res = oracle.fit_many(cfg, b.obs, b.ivar, basis, b.init)
    d = np.abs(np.array([r["params"] for r in res]) - b.truth)
    tol = np.array([1.0, 0.002, 0.002, 0.1, 0.5])
    assert np.all(d <= tol), d.max(axis=0)
