"""Pins of the FP64 oracle against mathematics and library routines.

Each test checks one part of the oracle against something other than the
oracle itself: brute force on tiny inputs, closed forms, invariants, special
cases that reduce to numpy/scipy routines, and statistical properties.
"""

import itertools
import math

import numpy as np
import pytest
import scipy.optimize
import scipy.special

import oracle
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name

pytestmark = pytest.mark.usefixtures("oracle_lib")

C_KMS = 299792.458


def small_shape(P=240, M=24, D=6, **kw):
    return shape_by_name("lamost3900", n_pix=P, margin=M, degree=D, **kw)


def cfg_for(shape):
    return oracle.Config.from_shape(shape, BOX_LO, BOX_HI)


# ---------------------------------------------------------------- Eq. 1 ----

def test_features_are_all_cubic_monomials_in_graded_lex_order():
    rng = np.random.default_rng(0)
    x = rng.uniform(-1.2, 1.2, 3)
    phi, dphi = oracle.features(x)
    expect = []
    for deg in range(4):
        # graded, then lexicographic with x1 > x2 > x3
        exps = sorted((e for e in itertools.product(range(deg + 1), repeat=3) if sum(e) == deg),
                      reverse=True)
        expect += [x[0] ** a * x[1] ** b * x[2] ** c for a, b, c in exps]
    assert len(expect) == 20
    np.testing.assert_allclose(phi, expect, rtol=1e-15, atol=1e-15)
    h = 1e-6
    for t in range(3):
        e = np.zeros(3)
        e[t] = h
        fd = (oracle.features(x + e)[0] - oracle.features(x - e)[0]) / (2 * h)
        np.testing.assert_allclose(dphi[t], fd, rtol=1e-8, atol=1e-9)


# ------------------------------------------------------------- Legendre ----

def test_legendre_matches_scipy_eval_legendre_and_closed_forms():
    xs = np.linspace(-1, 1, 41)
    for n in range(0, 51):
        ours = np.array([oracle.legendre(n, x) for x in xs])
        np.testing.assert_allclose(ours, scipy.special.eval_legendre(n, xs), rtol=1e-12, atol=1e-13)
        assert oracle.legendre(n, 1.0) == pytest.approx(1.0, abs=1e-13)
        assert oracle.legendre(n, -1.0) == pytest.approx((-1.0) ** n, abs=1e-13)
    for x in xs:
        assert oracle.legendre(2, x) == pytest.approx(1.5 * x * x - 0.5, abs=1e-15)
        assert oracle.legendre(3, x) == pytest.approx(2.5 * x ** 3 - 1.5 * x, abs=1e-15)


def test_legendre_gauss_orthogonality():
    nodes, weights = np.polynomial.legendre.leggauss(40)
    D = 20
    V = np.array([[oracle.legendre(n, x) for n in range(D + 1)] for x in nodes])
    gram = V.T @ (weights[:, None] * V)
    np.testing.assert_allclose(gram, np.diag(2.0 / (2 * np.arange(D + 1) + 1)), atol=1e-13)


# --------------------------------------------------------------- Eq. 5 -----

@pytest.mark.parametrize("mu,sig", [(0.0, 1.0), (2.37, 1.3), (-4.1, 2.2), (0.49, 3.7)])
def test_kernel_shape_sum_and_moments(mu, sig):
    H, G, Gm, Gs = oracle.kernel(mu, sig, 64)
    assert H == math.ceil(abs(mu) + 5 * sig)
    assert G.size == 2 * H + 1
    assert G.sum() == pytest.approx(1.0, abs=1e-15)
    m = np.arange(-H, H + 1)
    # exact Gaussian ratios
    ratio = G / G[H]
    np.testing.assert_allclose(ratio, np.exp(-((m - mu) ** 2 - mu ** 2) / (2 * sig ** 2)), rtol=1e-13)
    # Poisson summation: aliasing exp(-2 pi^2 sig^2) < 3e-9 for sig >= 1, and
    # the two 5-sigma tails beyond the window hold < 1.6e-5 of the variance.
    mean = (G * m).sum()
    var = (G * (m - mean) ** 2).sum()
    assert abs(mean - mu) < 1e-5 * sig
    assert abs(var / sig ** 2 - 1) < 2e-5


def test_kernel_window_clamps_at_margin():
    H, G, _, _ = oracle.kernel(10.0, 5.0, 16)
    assert H == 16 and G.size == 33


def test_kernel_derivatives_by_central_differences():
    mu, sig, h = 1.234, 1.71, 1e-6
    H, G, Gm, Gs = oracle.kernel(mu, sig, 64)
    Gp = oracle.kernel(mu + h, sig, 64)[1]
    Gn = oracle.kernel(mu - h, sig, 64)[1]
    np.testing.assert_allclose(Gm, (Gp - Gn) / (2 * h), atol=1e-9)
    Gp = oracle.kernel(mu, sig + h, 64)[1]
    Gn = oracle.kernel(mu, sig - h, 64)[1]
    np.testing.assert_allclose(Gs, (Gp - Gn) / (2 * h), atol=1e-9)


def test_convolution_matches_numpy_convolve():
    rng = np.random.default_rng(1)
    P, M = 16, 8
    fp = rng.normal(size=P + 2 * M)
    H, G, _, _ = oracle.kernel(1.3, 1.1, M)
    ours = oracle.convolve(fp, G, M, P)
    full = np.convolve(fp, G)
    np.testing.assert_allclose(ours, full[H + M:H + M + P], rtol=1e-14, atol=1e-15)
    brute = [sum(G[m + H] * fp[j - m + M] for m in range(-H, H + 1)) for j in range(P)]
    np.testing.assert_allclose(ours, brute, rtol=1e-14, atol=1e-15)


def test_zero_velocity_floor_width_is_identity():
    rng = np.random.default_rng(2)
    P, M = 50, 8
    fp = rng.uniform(0.5, 1.5, P + 2 * M)
    H, G, _, _ = oracle.kernel(0.0, 0.1, M)
    np.testing.assert_allclose(oracle.convolve(fp, G, M, P), fp[M:M + P], rtol=1e-15)


@pytest.mark.parametrize("n", [-3, 1, 4])
def test_integer_shift_moves_spectrum(n):
    rng = np.random.default_rng(3)
    P, M = 40, 8
    fp = rng.uniform(0.5, 1.5, P + 2 * M)
    H, G, _, _ = oracle.kernel(float(n), 0.1, M)
    out = oracle.convolve(fp, G, M, P)
    np.testing.assert_allclose(out, fp[M - n:M - n + P], rtol=1e-15)


def test_line_centroid_moves_by_mu_pixels():
    P, M = 80, 30
    fp = np.zeros(P + 2 * M)
    c0 = 40 + M                       # rest pixel 40
    fp[c0] = 1.0
    for mu in (-3.3, 0.0, 2.7):
        H, G, _, _ = oracle.kernel(mu, 2.0, M)
        out = oracle.convolve(fp, G, M, P)
        cen = (np.arange(P) * out).sum() / out.sum()
        assert cen == pytest.approx(40 + mu, abs=1e-6)


# ----------------------------------------------- full model at fixed u ----

@pytest.fixture(scope="module")
def small_case():
    shape = small_shape()
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, 77, 0, 4)
    cfg = cfg_for(shape)
    return shape, cfg, basis, batch


def _legendre_design(P, D):
    x = -1.0 + 2.0 * np.arange(P) / P
    return np.stack([scipy.special.eval_legendre(n, x) for n in range(D + 1)], axis=1)


def test_interpolator_and_convolution_compose(small_case):
    shape, cfg, basis, batch = small_case
    u = cfg.normalise(batch.init[0])
    ev = oracle.evaluate(cfg, batch.obs[0], batch.ivar[0], basis, u)
    phi, _ = oracle.features(u[:3])
    np.testing.assert_allclose(ev["fp"], phi @ basis.astype(np.float64), rtol=1e-13, atol=1e-13)
    scale = C_KMS * math.log(10) * shape.dlog10
    th = cfg.box_lo + 0.5 * (u + 1) * (cfg.box_hi - cfg.box_lo)
    H, G, _, _ = oracle.kernel(th[3] / scale, th[4] / scale, shape.margin)
    full = np.convolve(ev["fp"], G)
    np.testing.assert_allclose(ev["fpp"], full[H + shape.margin:H + shape.margin + shape.n_pix],
                               rtol=1e-13)


def test_continuum_least_squares_matches_lstsq(small_case):
    shape, cfg, basis, batch = small_case
    obs, ivar = batch.obs[1].astype(np.float64), batch.ivar[1].astype(np.float64)
    u = cfg.normalise(batch.init[1])
    ev = oracle.evaluate(cfg, batch.obs[1], batch.ivar[1], basis, u)
    L = _legendre_design(shape.n_pix, shape.degree)
    w = np.where(ivar > 0, ivar, 0.0)
    o = np.where(ivar > 0, obs, 0.0)
    X = np.sqrt(w)[:, None] * ev["fpp"][:, None] * L
    b, *_ = np.linalg.lstsq(X, np.sqrt(w) * o, rcond=None)
    np.testing.assert_allclose(ev["b"], b, rtol=1e-9, atol=1e-12 * np.abs(b).max())
    model = (L @ b) * ev["fpp"]
    np.testing.assert_allclose(ev["model"], model, rtol=1e-9)
    assert ev["chi2"] == pytest.approx((w * (o - model) ** 2).sum(), rel=1e-10)
    assert ev["n_eff"] == int((ivar > 0).sum())


def test_noiseless_continuum_recovered_exactly(small_case):
    shape, cfg, basis, batch = small_case
    u = cfg.normalise(batch.init[2])
    ivar = np.ones(shape.n_pix, np.float32)
    fpp = oracle.evaluate(cfg, batch.obs[2], ivar, basis, u)["fpp"]
    L = _legendre_design(shape.n_pix, shape.degree)
    b_true = np.array([30.0, 2.0, -1.5, 0.7, 0.2, -0.1, 0.05])
    obs = ((L @ b_true) * fpp).astype(np.float32)
    ev = oracle.evaluate(cfg, obs, ivar, basis, u)
    # obs is rounded to float32, so b is exact to float32 resolution
    np.testing.assert_allclose(ev["b"], b_true, rtol=1e-5, atol=1e-5)
    assert ev["chi2"] / (obs.astype(np.float64) ** 2).sum() < 1e-13


def test_chi2_invariant_under_flux_weighting(small_case):
    shape, cfg, basis, batch = small_case
    u = cfg.normalise(batch.init[0])
    w = 123.456
    a = oracle.evaluate(cfg, batch.obs[0], batch.ivar[0], basis, u)
    # powers of two keep the float32 inputs exact under scaling
    w = 64.0
    b = oracle.evaluate(cfg, batch.obs[0] / np.float32(w), batch.ivar[0] * np.float32(w * w), basis, u)
    assert b["chi2"] == pytest.approx(a["chi2"], rel=1e-12)
    np.testing.assert_allclose(b["b"] * w, a["b"], rtol=1e-10)
    np.testing.assert_allclose(b["grad"], a["grad"], rtol=1e-9, atol=1e-12)


def _safe_point(cfg, shape, u):
    """Keep frac(|mu| + 5 sigma) away from integers so H is locally constant."""
    scale = C_KMS * math.log(10) * shape.dlog10
    u = u.copy()
    for _ in range(200):
        th = cfg.box_lo + 0.5 * (u + 1) * (cfg.box_hi - cfg.box_lo)
        f = (abs(th[3] / scale) + 5 * th[4] / scale) % 1.0
        if 0.05 < f < 0.95:
            return u
        u[4] += 0.003
    raise AssertionError


def test_residual_jacobian_by_central_differences(small_case):
    shape, cfg, basis, batch = small_case
    u = _safe_point(cfg, shape, cfg.normalise(batch.init[3]) + 0.03)
    b = oracle.evaluate(cfg, batch.obs[3], batch.ivar[3], basis, u)["b"]
    r, J = oracle.residual(cfg, batch.obs[3], batch.ivar[3], basis, u, b)
    x = np.concatenate([u, b])
    h = 1e-6
    for a in range(x.size):
        e = np.zeros(x.size)
        e[a] = h * max(1.0, abs(x[a]))
        rp = oracle.residual(cfg, batch.obs[3], batch.ivar[3], basis, (x + e)[:5], (x + e)[5:], False)
        rn = oracle.residual(cfg, batch.obs[3], batch.ivar[3], basis, (x - e)[:5], (x - e)[5:], False)
        fd = (rp - rn) / (2 * e[a])
        np.testing.assert_allclose(J[:, a], fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())


def test_envelope_gradient_by_central_differences(small_case):
    shape, cfg, basis, batch = small_case
    u = _safe_point(cfg, shape, cfg.normalise(batch.init[1]) + 0.05)
    ev = oracle.evaluate(cfg, batch.obs[1], batch.ivar[1], basis, u)
    h = 1e-6
    fd = np.empty(5)
    for t in range(5):
        e = np.zeros(5)
        e[t] = h
        jp = oracle.evaluate(cfg, batch.obs[1], batch.ivar[1], basis, u + e)["J"]
        jn = oracle.evaluate(cfg, batch.obs[1], batch.ivar[1], basis, u - e)["J"]
        fd[t] = (jp - jn) / (2 * h)
    np.testing.assert_allclose(ev["grad"], fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def test_model_jacobian_at_fixed_continuum(small_case):
    shape, cfg, basis, batch = small_case
    u = _safe_point(cfg, shape, cfg.normalise(batch.init[2]) - 0.04)
    ev = oracle.evaluate(cfg, batch.obs[2], batch.ivar[2], basis, u)
    sw = np.sqrt(np.where(batch.ivar[2] > 0, batch.ivar[2].astype(np.float64), 0.0))
    _, J = oracle.residual(cfg, batch.obs[2], batch.ivar[2], basis, u, ev["b"])
    keep = sw > 0
    np.testing.assert_allclose(ev["jac"].T[keep], -(J[keep, :5] / sw[keep, None]), rtol=1e-12,
                               atol=1e-12)


# --------------------------------------------------------- Arms (DESI) -----

def test_per_arm_kernel_uses_quadrature_sum_of_widths():
    shape = shape_by_name("desi7800", n_pix=300, margin=32, arm_start=(0, 100, 200),
                          arm_sigma_kms=(60.0, 35.0, 25.0))
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, 9, 0, 1)
    cfg = cfg_for(shape)
    u = cfg.normalise(batch.init[0])
    ev = oracle.evaluate(cfg, batch.obs[0], batch.ivar[0], basis, u)
    scale = C_KMS * math.log(10) * shape.dlog10
    th = cfg.box_lo + 0.5 * (u + 1) * (cfg.box_hi - cfg.box_lo)
    for a, (j0, j1) in enumerate([(0, 100), (100, 200), (200, 300)]):
        s_eff = math.hypot(th[4], shape.arm_sigma_kms[a])
        H, G, _, _ = oracle.kernel(th[3] / scale, s_eff / scale, shape.margin)
        full = np.convolve(ev["fp"], G)
        np.testing.assert_allclose(ev["fpp"][j0:j1],
                                   full[H + shape.margin:H + shape.margin + shape.n_pix][j0:j1],
                                   rtol=1e-13)


# ------------------------------------------------------------- LM fit ------

def _noiseless_obs(cfg, shape, basis, u_true, b_true, ivar):
    fpp = oracle.evaluate(cfg, np.ones(shape.n_pix, np.float32), ivar, basis, u_true)["fpp"]
    L = _legendre_design(shape.n_pix, shape.degree)
    return ((L @ b_true) * fpp).astype(np.float32)


def test_noiseless_injection_recovery():
    shape = small_shape(P=400, M=32, D=6)
    basis, lines = make_basis(shape)
    cfg = cfg_for(shape)
    rng = np.random.default_rng(5)
    for trial in range(4):
        u_true = rng.uniform(-0.7, 0.7, 5)
        b_true = np.concatenate([[50.0], rng.normal(0, 3.0, shape.degree)])
        ivar = np.ones(shape.n_pix, np.float32)
        obs = _noiseless_obs(cfg, shape, basis, u_true, b_true, ivar)
        u0 = u_true + rng.normal(0, 0.03, 5)
        res = oracle.fit(cfg, obs, ivar, basis, u0)
        # obs carries float32 rounding (~3e-8 relative), the only error left
        np.testing.assert_allclose(res["u"], u_true, atol=2e-6)
        assert res["flags"] & oracle.NOT_CONVERGED == 0


def test_lm_matches_scipy_minpack_lm(small_case):
    shape, cfg, basis, batch = small_case
    for i in range(3):
        obs, ivar = batch.obs[i], batch.ivar[i]
        u0 = cfg.normalise(batch.init[i])
        res = oracle.fit(cfg, obs, ivar, basis, u0)
        b0 = oracle.evaluate(cfg, obs, ivar, basis, u0)["b"]

        def fun(x):
            return oracle.residual(cfg, obs, ivar, basis, x[:5], x[5:], want_jac=False)

        sp = scipy.optimize.least_squares(fun, np.concatenate([u0, b0]), method="lm",
                                          xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=20000)
        chi_sp = float((sp.fun ** 2).sum())
        assert res["chi2"] <= chi_sp * (1 + 1e-9)
        np.testing.assert_allclose(res["u"], sp.x[:5], atol=1e-6)


def test_linear_problem_converges_in_one_step():
    # Continuum-only problem: at u fixed at the truth the residual is linear
    # in b, so Gauss-Newton lands on the answer in one accepted step; the
    # u part then has zero gradient and stays put.
    shape = small_shape(P=200, M=24, D=5)
    basis, _ = make_basis(shape)
    cfg = cfg_for(shape)
    u = np.array([0.1, -0.2, 0.3, 0.05, 0.4])
    b_true = np.array([20.0, 1.0, -0.5, 0.25, 0.1, -0.05])
    ivar = np.ones(shape.n_pix, np.float32)
    obs = _noiseless_obs(cfg, shape, basis, u, b_true, ivar)
    ev = oracle.evaluate(cfg, obs, ivar, basis, u)
    assert ev["chi2"] < 1e-9 * float((obs.astype(np.float64) ** 2).sum())
    res = oracle.fit(cfg, obs, ivar, basis, u)
    np.testing.assert_allclose(res["u"], u, atol=1e-7)


# ---------------------------------------------------------- covariance -----

def test_covariance_equals_schur_complement_inverse(small_case):
    shape, cfg, basis, batch = small_case
    res = oracle.fit(cfg, batch.obs[0], batch.ivar[0], basis, cfg.normalise(batch.init[0]))
    r, J = oracle.residual(cfg, batch.obs[0], batch.ivar[0], basis, res["u"], res["b"])
    Ju, Jb = J[:, :5], J[:, 5:]
    S = Ju.T @ Ju - Ju.T @ Jb @ np.linalg.solve(Jb.T @ Jb, Jb.T @ Ju)
    s2 = float(r @ r) / (res["n_eff"] - 5)
    np.testing.assert_allclose(res["cov_u"], s2 * np.linalg.inv(S), rtol=1e-8)
    # physical units: Teff via dT = T ln10 dlog10 T, the rest by box half-widths
    h = 0.5 * (cfg.box_hi - cfg.box_lo)
    jd = h.copy()
    jd[0] *= res["params"][0] * math.log(10)
    np.testing.assert_allclose(res["cov"], jd[:, None] * res["cov_u"] * jd[None, :], rtol=1e-12)



@pytest.fixture(scope="module")
def pull_draws():
    """400 noise realisations at one fixed truth, each fitted by the oracle."""
    shape = small_shape(P=300, M=32, D=4)
    basis, _ = make_basis(shape)
    cfg = cfg_for(shape)
    u_true = np.array([0.2, -0.1, 0.3, 0.1, 0.2])
    b_true = np.array([100.0, 5.0, -3.0, 1.0, 0.5])
    ivar = np.full(shape.n_pix, 1.0 / 2.0 ** 2, np.float32)
    clean = _noiseless_obs(cfg, shape, basis, u_true, b_true, ivar).astype(np.float64)
    rng = np.random.default_rng(11)
    fits = []
    for _ in range(400):
        obs = (clean + rng.normal(0, 2.0, shape.n_pix)).astype(np.float32)
        fits.append(oracle.fit(cfg, obs, ivar, basis, u_true))
    return cfg, u_true, fits


def test_covariance_pull_distribution(pull_draws):
    _, u_true, fits = pull_draws
    pulls = np.array([(r["u"] - u_true) / np.sqrt(np.diag(r["cov_u"])) for r in fits])
    std = pulls.std(axis=0)
    assert np.all(np.abs(std - 1.0) < 0.12), std
    assert np.all(np.abs(pulls.mean(axis=0)) < 0.2)


def test_covariance_pull_distribution_in_physical_units(pull_draws):
    """Section 2.2 stage 9 in the units the fit reports: the spread of the
    fitted Teff (K), log g, [Fe/H], RV (km/s) and sigma (km/s) around the
    truth over noise draws equals the covariance's standard deviations.  The
    physical parameters are the decoded fits, so a wrong Teff or ln 10
    factor in the covariance's mapping shifts the Teff spread away from 1."""
    cfg, u_true, fits = pull_draws
    theta_true = cfg.physical(u_true)
    pulls = np.array([(r["params"] - theta_true) / np.sqrt(np.diag(r["cov"])) for r in fits])
    std = pulls.std(axis=0)
    assert np.all(np.abs(std - 1.0) < 0.12), std
    assert np.all(np.abs(pulls.mean(axis=0)) < 0.2)
    # the Teff column differs from the u-space one by T ln 10 times the half
    # width: a factor of about 2000 here, so the check is not vacuous
    r = fits[0]
    assert r["cov"][0, 0] / r["cov_u"][0, 0] > 1e5


# ------------------------------------------------------ status flags ------

def test_width_floor_flag_and_zero_derivative():
    """Reading of Eq. 5 at small widths: sigma_px = max(sigma / (c ln10 dlog10),
    0.1), flagged, with d chi2 / d sigma = 0 below the floor; the model does
    not depend on sigma there."""
    shape = small_shape()
    basis, lines = make_basis(shape)
    cfg = cfg_for(shape)
    b = make_spectra(shape, lines, 31, 0, 1)
    scale = C_KMS * math.log(10.0) * shape.dlog10
    u = cfg.normalise(b.init[0])
    models = []
    for sigma in (2.0, 4.0, 0.1 * scale * 0.999, 0.1 * scale * 1.001, 60.0):
        uu = u.copy()
        uu[4] = 2.0 * (sigma - BOX_LO[4]) / (BOX_HI[4] - BOX_LO[4]) - 1.0
        r = oracle.evaluate(cfg, b.obs[0], b.ivar[0], basis, uu)
        floored = sigma / scale < 0.1
        assert bool(r["flags"] & oracle.SIGMA_FLOOR) == floored, sigma
        if floored:
            assert r["grad"][4] == 0.0
            models.append(r["model"])
        else:
            assert r["grad"][4] != 0.0
    np.testing.assert_array_equal(models[0], models[1])
    np.testing.assert_array_equal(models[0], models[2])


def test_width_floor_flag_per_arm():
    """With spectrograph arms each arm's width sqrt(sigma^2 + sigma_arm^2)
    is floored on its own; the flag marks any floored arm."""
    shape = small_shape(P=300, M=32, D=4, arm_start=(0, 100, 200),
                        arm_sigma_kms=(0.0, 40.0, 0.0))
    basis, lines = make_basis(shape)
    cfg = cfg_for(shape)
    b = make_spectra(shape, lines, 32, 0, 1)
    scale = C_KMS * math.log(10.0) * shape.dlog10
    u = cfg.normalise(b.init[0])
    for sigma, expect in ((3.0, True), (0.2 * scale, False)):
        uu = u.copy()
        uu[4] = 2.0 * (sigma - BOX_LO[4]) / (BOX_HI[4] - BOX_LO[4]) - 1.0
        r = oracle.evaluate(cfg, b.obs[0], b.ivar[0], basis, uu)
        assert bool(r["flags"] & oracle.SIGMA_FLOOR) == expect
        # the unfloored middle arm still depends on sigma
        assert r["grad"][4] != 0.0


def test_out_of_box_flag_threshold():
    shape = small_shape()
    basis, lines = make_basis(shape)
    cfg = cfg_for(shape)
    b = make_spectra(shape, lines, 33, 0, 1)
    u = np.array([0.1, -0.2, 0.3, 0.0, 0.1])
    for t in range(5):
        for val, expect in ((1.5, False), (-1.5, False), (1.5001, True), (-1.6, True)):
            uu = u.copy()
            uu[t] = val
            r = oracle.evaluate(cfg, b.obs[0], b.ivar[0], basis, uu)
            assert bool(r["flags"] & oracle.OUT_OF_BOX) == expect, (t, val)


def test_nonpositive_continuum_flag_matches_lstsq_sign():
    """CONT_NONPOS is set when the weighted least-squares continuum (numpy
    lstsq on the sqrt(W)-scaled Legendre design) is <= 0 at some pixel."""
    shape = small_shape(P=300, M=32, D=6)
    basis, lines = make_basis(shape)
    cfg = cfg_for(shape)
    b = make_spectra(shape, lines, 34, 0, 2)
    P = shape.n_pix
    x = -1.0 + 2.0 * np.arange(P) / P
    V = np.stack([scipy.special.eval_legendre(n, x) for n in range(shape.degree + 1)], axis=1)
    for i, negate in ((0, False), (1, True)):
        obs = b.obs[i].copy()
        if negate:
            obs[: P // 5] *= -0.3
        u = cfg.normalise(b.init[i])
        r = oracle.evaluate(cfg, obs, b.ivar[i], basis, u)
        w = b.ivar[i].astype(np.float64)
        A = np.sqrt(w)[:, None] * r["fpp"][:, None] * V
        coef = np.linalg.lstsq(A, np.sqrt(w) * obs.astype(np.float64), rcond=None)[0]
        cont = V @ coef
        assert bool(r["flags"] & oracle.CONT_NONPOS) == bool(cont.min() <= 0.0) == negate
