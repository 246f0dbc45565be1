"""HIP path vs the FP64 oracle, element by element, through the C ABI."""

import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2512_24840_amd as lasp
from paper_2512_24840_amd.lasp import ST_NO_DATA, ST_NONFINITE_INPUT, ST_SINGULAR
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name, wave_grid

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
DEV = torch.device("cuda:0")

# fitted-value tolerances (Teff K, log g, [Fe/H], RV km/s); sigma is not gated
FIT_TOL = np.array([2.0, 0.005, 0.005, 0.2])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def case(name, n, config_id=11, **overrides):
    shape = shape_by_name(name, **overrides)
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, config_id, 0, n)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    return shape, cfg, basis, batch


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def arms_of(shape):
    return lasp.Arms(shape.arm_start, shape.arm_sigma_kms) if shape.arm_start else None


FWD_CASES = [
    ("lamost1550", {}),
    ("lamost3900", {}),
    ("desi7800", {}),
    ("lamost3900", dict(n_pix=1001, margin=40, degree=6)),
    ("lamost3900", dict(n_pix=257, margin=17, degree=4)),
    # one arm over 7,800 px: the 512-thread workgroup of the one-arm pass
    ("desi7800", dict(arm_start=(), arm_sigma_kms=())),
]


@pytest.mark.parametrize("name,over", FWD_CASES)
def test_forward_model_chi2_gradient_match_oracle(name, over):
    say(f"[forward parity] shape={name} {over} B=7")
    shape, cfg, basis, batch = case(name, 7, **over)
    rng = np.random.default_rng(3)
    u = cfg.normalise(batch.init) + rng.normal(0, 0.03, (7, 5))
    res = lasp.forward(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis),
                       to_dev(u.astype(np.float32)), want_model=True, want_grad=True,
                       margin=shape.margin, degree=shape.degree, arms=arms_of(shape))
    torch.cuda.synchronize()
    model = res["model"].cpu().numpy()
    chi2 = res["chi2"].cpu().numpy()
    grad = res["grad"].cpu().numpy()
    neff = res["n_eff"].cpu().numpy()
    for i in range(7):
        # the oracle sees the same float32 u the GPU saw
        ref = oracle.evaluate(cfg, batch.obs[i], batch.ivar[i], basis,
                              u[i].astype(np.float32).astype(np.float64))
        rms = np.sqrt(np.mean(ref["model"] ** 2))
        assert np.max(np.abs(model[i] - ref["model"])) <= 1e-5 * rms, i
        assert chi2[i] == pytest.approx(ref["chi2"], rel=1e-5), i
        assert neff[i] == ref["n_eff"]
        g_ref = ref["grad"]
        assert np.linalg.norm(grad[i] - g_ref) <= 1e-5 * np.linalg.norm(g_ref) + 1e-9, \
            (i, grad[i], g_ref)


@pytest.mark.parametrize("k", [30, -30])
def test_results_do_not_depend_on_the_flux_scale_bit_for_bit(k):
    """The flux weight w is a power of two near the median flux, so scaling
    obs by 2^k and ivar by 2^-2k scales w by 2^k and leaves every step of the
    arithmetic unchanged: chi2, J, the gradient and the covariance must agree
    bit for bit, and the model scale by exactly 2^k.  The rows cover an odd
    and an even number of valid pixels and fluxes repeated at the median."""
    say(f"[flux scale] lamost1550 B=6, obs x 2^{k}, ivar x 2^{-2 * k}")
    shape, cfg, basis, batch = case("lamost1550", 6)
    obs, ivar = batch.obs.copy(), batch.ivar.copy()
    obs[0, 200:260] = np.median(obs[0])     # ties at the median
    ivar[1, :1] = 0.0                        # one pixel fewer: the other parity
    ivar[2, :3] = 0.0
    u = to_dev(cfg.normalise(batch.init).astype(np.float32))
    kw = dict(want_model=True, want_grad=True, want_cov=True, margin=shape.margin,
              degree=shape.degree)
    r0 = lasp.forward(to_dev(obs), to_dev(ivar), wave_grid(shape), to_dev(basis), u, **kw)
    r1 = lasp.forward(to_dev(np.ldexp(obs, k)), to_dev(np.ldexp(ivar, -2 * k)), wave_grid(shape),
                      to_dev(basis), u, **kw)
    torch.cuda.synchronize()
    for key in ("chi2", "J", "grad", "cov", "n_eff", "status"):
        assert np.array_equal(r0[key].cpu().numpy(), r1[key].cpu().numpy()), key
    assert np.array_equal(np.ldexp(r0["model"].cpu().numpy(), k), r1["model"].cpu().numpy())


def test_model_jacobian_matches_oracle():
    say("[jacobian parity] lamost3900 B=5")
    shape, cfg, basis, batch = case("lamost3900", 5)
    u = cfg.normalise(batch.init) + 0.02
    res = lasp.forward(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis),
                       to_dev(u.astype(np.float32)), want_jac=True, margin=shape.margin,
                       degree=shape.degree)
    torch.cuda.synchronize()
    jac = res["jac"].cpu().numpy()
    for i in range(5):
        ref = oracle.evaluate(cfg, batch.obs[i], batch.ivar[i], basis,
                              u[i].astype(np.float32).astype(np.float64))["jac"]
        for t in range(5):
            scale = np.sqrt(np.mean(ref[t] ** 2))
            assert np.max(np.abs(jac[i, t] - ref[t])) <= 1e-4 * scale, (i, t)


def test_fits_alone_match_oracle_lm():
    say("[fit parity] lamost1550, 64 spectra fitted alone (B=1), 500 Adam steps")
    shape, cfg, basis, batch = case("lamost1550", 64, config_id=1)
    ref = oracle.fit_many(cfg, batch.obs, batch.ivar, basis, batch.init)
    got = []
    for i in range(64):
        r = lasp.fit_group(to_dev(batch.obs[i:i + 1]), to_dev(batch.ivar[i:i + 1]),
                           wave_grid(shape), to_dev(basis), to_dev(batch.init[i:i + 1]), 500,
                           margin=shape.margin, degree=shape.degree)
        got.append(r.params.cpu().numpy()[0])
    got = np.array(got, dtype=np.float64)
    refp = np.array([r["params"] for r in ref])
    err = np.abs(got - refp)[:, :4]
    say("max |GPU - oracle|:", err.max(axis=0))
    assert np.all(err <= FIT_TOL), err.max(axis=0)


def test_covariance_matches_oracle():
    say("[covariance parity] lamost1550 B=8, at the oracle optimum")
    shape, cfg, basis, batch = case("lamost1550", 8, config_id=1)
    ref = oracle.fit_many(cfg, batch.obs, batch.ivar, basis, batch.init)
    start = np.array([r["params"] for r in ref], dtype=np.float32)
    r = lasp.fit_group(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis),
                       to_dev(start), 0, want_cov=True, margin=shape.margin, degree=shape.degree)
    torch.cuda.synchronize()
    cov = r.cov.cpu().numpy()
    for i in range(8):
        # reference covariance at exactly the float32 start the GPU used
        c_ref = oracle.covariance(cfg, batch.obs[i], batch.ivar[i], basis,
                                  cfg.normalise(start[i].astype(np.float64)))["cov"]
        rel = np.linalg.norm(cov[i] - c_ref) / np.linalg.norm(c_ref)
        sd_rel = np.abs(np.sqrt(np.diag(cov[i])) / np.sqrt(np.diag(c_ref)) - 1)
        assert rel < 1e-3 and sd_rel.max() < 1e-3, (i, rel, sd_rel)


def test_bad_spectra_are_flagged_and_isolated():
    say("[status/isolation] lamost1550 B=4 with a NaN pixel and an all-masked spectrum")
    shape, cfg, basis, batch = case("lamost1550", 4, config_id=1)
    obs, ivar = batch.obs.copy(), batch.ivar.copy()
    obs[1, 100] = np.nan
    ivar[2, :] = 0.0
    args = (wave_grid(shape), to_dev(basis))
    r = lasp.fit_group(to_dev(obs), to_dev(ivar), *args, to_dev(batch.init), 50,
                       margin=shape.margin, degree=shape.degree)
    clean = lasp.fit_group(to_dev(batch.obs[[0, 3]]), to_dev(batch.ivar[[0, 3]]), *args,
                           to_dev(batch.init[[0, 3]]), 50, margin=shape.margin,
                           degree=shape.degree)
    masked = obs[1:2].copy()
    iv1 = ivar[1:2].copy()
    iv1[0, 100] = 0.0
    masked[0, 100] = 0.0
    one = lasp.fit_group(to_dev(masked), to_dev(iv1), *args, to_dev(batch.init[1:2]), 50,
                         margin=shape.margin, degree=shape.degree)
    torch.cuda.synchronize()
    st = r.status.cpu().numpy()
    assert st[1] & ST_NONFINITE_INPUT and not st[0] & ST_NONFINITE_INPUT
    assert st[2] & ST_NO_DATA and st[2] & ST_SINGULAR
    p = r.params.cpu().numpy()
    assert np.array_equal(p[[0, 3]], clean.params.cpu().numpy())       # bitwise
    assert np.array_equal(p[1], one.params.cpu().numpy()[0])           # NaN == masked pixel
    np.testing.assert_allclose(p[2], batch.init[2], rtol=1e-6)          # no data: unmoved


def test_fit_is_deterministic_and_independent_of_batch_position():
    say("[determinism] lamost3900 B=19 twice, and spectrum 5 alone")
    shape, cfg, basis, batch = case("lamost3900", 19)
    args = (to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis),
            to_dev(batch.init), 100)
    a = lasp.fit_group(*args).params.cpu().numpy()
    b = lasp.fit_group(*args).params.cpu().numpy()
    alone = lasp.fit_group(to_dev(batch.obs[5:6]), to_dev(batch.ivar[5:6]), wave_grid(shape),
                           to_dev(basis), to_dev(batch.init[5:6]), 100).params.cpu().numpy()
    assert np.array_equal(a, b)
    assert np.array_equal(a[5], alone[0])
