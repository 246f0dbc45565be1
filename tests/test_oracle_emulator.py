"""Pins of the oracle's emulator steps: the five Teff regimes of the
multi-class interpolator (Eq. 1) and the flux-conserving resampling
(Section 2.2, step 3), against closed forms and independent integrals."""

import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
from synth import BOX_HI, BOX_LO, class_weights, make_basis, make_spectra, shape_by_name

pytestmark = pytest.mark.usefixtures("oracle_lib")


def cfg3(name="lamost1550"):
    return oracle.Config.from_shape(shape_by_name(name), BOX_LO, BOX_HI, n_classes=3)


@pytest.mark.parametrize("teff,expect", [(3900.0, (1, 0, 0)), (4000.0, (1, 0, 0)),
                                         (4275.0, (0.5, 0.5, 0)), (4550.0, (0, 1, 0)),
                                         (6000.0, (0, 1, 0)), (7500.0, (0, 0.75, 0.25)),
                                         (9000.0, (0, 0, 1)), (9500.0, (0, 0, 1))])
def test_class_weights_follow_the_five_regimes(teff, expect):
    cfg = cfg3()
    u = cfg.normalise([teff, 3.0, -0.5, 0.0, 100.0])
    w, dw = oracle.class_weights(cfg, u)
    np.testing.assert_allclose(w, expect, atol=1e-12)
    assert abs(w.sum() - 1.0) < 1e-15


def test_class_weight_derivative_matches_finite_differences_inside_the_blends():
    cfg = cfg3()
    h = 1e-7
    for teff in (4100.0, 4400.0, 7300.0, 8500.0, 5500.0):
        u = cfg.normalise([teff, 3.0, -0.5, 0.0, 100.0])
        up, um = u.copy(), u.copy()
        up[0] += h
        um[0] -= h
        fd = (oracle.class_weights(cfg, up)[0] - oracle.class_weights(cfg, um)[0]) / (2 * h)
        np.testing.assert_allclose(oracle.class_weights(cfg, u)[1], fd, rtol=1e-6, atol=1e-9)


def test_three_class_model_is_the_blend_of_single_class_models():
    shape = shape_by_name("lamost1550")
    basis3, _ = make_basis(shape, n_classes=3)
    batch = make_spectra(shape, make_basis(shape)[1], 11, 0, 1)
    c1 = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    c3 = cfg3()
    for teff in (4300.0, 6000.0, 7600.0):
        u = c3.normalise([teff, 2.5, -1.0, 40.0, 90.0])
        w, _ = oracle.class_weights(c3, u)
        fp3 = oracle.evaluate(c3, batch.obs[0], batch.ivar[0], basis3, u)["fp"]
        fp1 = sum(w[c] * oracle.evaluate(c1, batch.obs[0], batch.ivar[0], basis3[20 * c:20 * c + 20], u)["fp"]
                  for c in range(3))
        np.testing.assert_allclose(fp3, fp1, rtol=1e-12, atol=1e-12)
        # and the weights are the generator's (an independent implementation)
        np.testing.assert_allclose(w, class_weights(np.array([teff]))[0], atol=1e-12)


def test_three_class_jacobian_matches_finite_differences():
    shape = shape_by_name("lamost1550")
    basis3, lines3 = make_basis(shape, n_classes=3)
    batch = make_spectra(shape, lines3, 12, 0, 1)
    cfg = cfg3()
    u = cfg.normalise([4400.0, 2.5, -1.0, 40.0, 90.0])       # inside the cool->warm blend
    ev = oracle.evaluate(cfg, batch.obs[0], batch.ivar[0], basis3, u)
    h = 1e-6
    for t in range(5):
        up, um = u.copy(), u.copy()
        up[t] += h
        um[t] -= h
        fd = (oracle.evaluate(cfg, batch.obs[0], batch.ivar[0], basis3, up)["chi2"]
              - oracle.evaluate(cfg, batch.obs[0], batch.ivar[0], basis3, um)["chi2"]) / (2 * h)
        g = ev["grad"][t] * ev["n_eff"]
        assert abs(g - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(ev["grad"]).max() * ev["n_eff"]), t


LAM0, DLAM = 3800.0, 0.2


def test_resampling_a_constant_gives_the_constant():
    src = np.ones((1, 6000), np.float32)
    out, ok = oracle.resample(src, LAM0, DLAM, 1000, math.log10(3850.0), 1e-4)
    assert ok
    np.testing.assert_allclose(out[0], 1.0, rtol=1e-12)


def test_resampling_conserves_the_integral_of_the_step_function():
    rng = np.random.default_rng(1)
    src = rng.uniform(0.5, 1.5, (1, 6000)).astype(np.float32)
    lg0, d, n = math.log10(3850.0), 1e-4, 1000
    out, ok = oracle.resample(src, LAM0, DLAM, n, lg0, d)
    e = 10.0 ** (lg0 + (np.arange(n + 1) - 0.5) * d)
    resampled = np.sum(out[0] * np.diff(e))
    # exact integral of the piecewise-constant source between e[0] and e[-1]
    e0 = LAM0 - DLAM / 2
    k0, k1 = int((e[0] - e0) // DLAM), int((e[-1] - e0) // DLAM)
    s = src[0].astype(np.float64)
    exact = (s[k0 + 1:k1].sum() * DLAM + s[k0] * (e0 + (k0 + 1) * DLAM - e[0])
             + s[k1] * (e[-1] - (e0 + k1 * DLAM)))
    assert abs(resampled - exact) <= 1e-9 * exact


def test_resampled_gaussian_line_matches_log_bin_averages():
    # a line averaged over the 0.2 A source bins (erf) resampled to log bins
    c, sig, amp = 4321.7, 0.8, 0.6
    n_src = 6000
    se = LAM0 - DLAM / 2 + DLAM * np.arange(n_src + 1)
    prof = amp * sig * math.sqrt(math.pi / 2) * np.diff(erf((se - c) / (math.sqrt(2) * sig))) / DLAM
    src = (1.0 - prof)[None, :].astype(np.float32)
    lg0, d, n = math.log10(3850.0), 1e-4, 1000
    out, _ = oracle.resample(src, LAM0, DLAM, n, lg0, d)
    e = 10.0 ** (lg0 + (np.arange(n + 1) - 0.5) * d)
    exact = 1.0 - amp * sig * math.sqrt(math.pi / 2) * np.diff(erf((e - c) / (math.sqrt(2) * sig))) / np.diff(e)
    # linear interpolation of the cumulative integral C errs by at most
    # max|C''| dlam^2 / 8 at each node, C'' being the flux slope (at most
    # amp / (sig sqrt(e)) for a Gaussian line); a bin value takes two nodes
    bound = 2 * (amp / (sig * math.sqrt(math.e))) * DLAM ** 2 / 8 / np.diff(e) + 1e-9
    assert np.all(np.abs(out[0] - exact) <= bound)
