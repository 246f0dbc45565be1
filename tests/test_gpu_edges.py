"""Edge paths of the model on the GPU against the FP64 oracle, through the C ABI.

Eq. 5 and the window size after it: the 0.1 px floor of the broadening width
(with its zero derivative) and the window clamped at the basis margin; the
failed-fit test of Section 4.2 (a nonpositive multiplicative continuum,
Step 5 of Section 2.2); parameters outside the normalisation box.  Values
are held to the forward bar (model 1e-5 of its rms, chi2 1e-5 relative,
gradient 1e-5 of its norm); status bits must equal the oracle's flags bit
for bit at the evaluated or returned parameters, whatever happened on the
way there.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2512_24840_amd as lasp
from edge_inputs import (bump_basis_case, gpu_flags_as_oracle, min_continuum, negative_flux_case,
                         oracle_flags, out_of_box_case, u_of_sigma)
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name, wave_grid

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def arms_of(shape):
    return lasp.Arms(shape.arm_start, shape.arm_sigma_kms) if shape.arm_start else None


def check_forward(shape, cfg, basis, obs, ivar, u, box=None, zero_sigma_grad=()):
    """lasp_forward at u vs oracle.evaluate: values and status bits."""
    n = obs.shape[0]
    res = lasp.forward(to_dev(obs), to_dev(ivar), wave_grid(shape), to_dev(basis),
                       to_dev(u.astype(np.float32)), want_model=True, want_grad=True,
                       margin=shape.margin, degree=shape.degree, arms=arms_of(shape), box=box)
    torch.cuda.synchronize()
    model = res["model"].cpu().numpy()
    chi2 = res["chi2"].cpu().numpy()
    grad = res["grad"].cpu().numpy()
    neff = res["n_eff"].cpu().numpy()
    status = res["status"].cpu().numpy()
    refs = []
    for i in range(n):
        ref = oracle.evaluate(cfg, obs[i], ivar[i], basis, u[i].astype(np.float32).astype(np.float64))
        refs.append(ref)
        rms = np.sqrt(np.mean(ref["model"] ** 2))
        assert np.max(np.abs(model[i] - ref["model"])) <= 1e-5 * rms, i
        assert chi2[i] == pytest.approx(ref["chi2"], rel=1e-5), i
        assert neff[i] == ref["n_eff"]
        g_ref = ref["grad"]
        assert np.linalg.norm(grad[i] - g_ref) <= 1e-5 * np.linalg.norm(g_ref) + 1e-9, \
            (i, grad[i], g_ref)
        assert gpu_flags_as_oracle(status[i]) == oracle_flags(ref), (i, status[i], ref["flags"])
    for i in zero_sigma_grad:
        assert grad[i, 4] == 0.0, i
    return status, refs


FLOOR_CASES = [
    # below the default box: sigma = 2.5 km/s is u5 = -1.95 (also OUT_OF_BOX)
    ("lamost1550", {}, "default"),
    # a box reaching down to sigma = 0 km/s: the floor inside the box
    ("lamost3900", {}, "to_zero"),
    # arms with no instrumental width in arms 0 and 2: those arms floored, arm 1 not
    ("desi7800", dict(arm_sigma_kms=(0.0, 36.4, 0.0)), "to_zero"),
]


@pytest.mark.parametrize("name,over,box", FLOOR_CASES)
def test_forward_at_the_width_floor(name, over, box):
    say(f"[edge: width floor] {name} {over} box={box} B=5")
    lo, hi = BOX_LO.copy(), BOX_HI.copy()
    if box == "to_zero":
        lo[4], hi[4] = 0.0, 100.0
    shape = shape_by_name(name, **over)
    basis, lines = make_basis(shape)
    b = make_spectra(shape, lines, 41, 0, 5)
    cfg = oracle.Config.from_shape(shape, lo, hi)
    u = cfg.normalise(b.init)
    # km/s: the first four below the floor on both grids (0.1 px is 6.9 km/s
    # at 1e-4 dex and 3.85 km/s on the three-arm grid), the last above it
    sig = np.array([2.5, 1.0, 3.0, 3.5, 60.0])
    u[:, 4] = u_of_sigma(sig, lo, hi)
    status, refs = check_forward(shape, cfg, basis, b.obs, b.ivar, u, box=(lo, hi),
                                 zero_sigma_grad=(0, 1, 2, 3) if not shape.arm_start else ())
    floored = status & 0x20
    assert floored[:4].all() and not floored[4]
    if shape.arm_start:  # the middle arm keeps a width derivative
        assert all(r["grad"][4] != 0.0 for r in refs)


CLAMP_CASES = [
    dict(margin=8, degree=8),
    dict(n_pix=1001, margin=8, degree=6),
]


@pytest.mark.parametrize("over", CLAMP_CASES)
def test_forward_with_the_window_clamped_at_the_margin(over):
    say(f"[edge: window clamp] lamost1550 {over} B=6")
    shape = shape_by_name("lamost1550", **over)
    basis, lines = make_basis(shape)
    b = make_spectra(shape, lines, 42, 0, 6)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    u = cfg.normalise(b.init)
    # (RV km/s, sigma km/s): ceil(|mu| + 5 sigma_px) = 15, 15, 11, 10 > M = 8; 6 and 4 fit
    rv_sig = [(250.0, 150.0), (-250.0, 150.0), (0.0, 150.0), (120.0, 110.0), (0.0, 80.0),
              (0.0, 50.0)]
    for i, (rv, sg) in enumerate(rv_sig):
        u[i, 3] = 2.0 * (rv - BOX_LO[3]) / (BOX_HI[3] - BOX_LO[3]) - 1.0
        u[i, 4] = u_of_sigma(sg)
    scale = 299792.458 * np.log(10.0) * shape.dlog10
    raw_h = [int(np.ceil(abs(rv) / scale + 5.0 * sg / scale)) for rv, sg in rv_sig]
    assert [h > shape.margin for h in raw_h] == [True, True, True, True, False, False], raw_h
    check_forward(shape, cfg, basis, b.obs, b.ivar, u)


def test_forward_flags_out_of_box_and_nonpositive_continuum():
    say("[edge: box and continuum flags] lamost1550 B=6")
    shape, basis, obs_neg, ivar, init, _ = negative_flux_case(6)
    b = make_spectra(shape, make_basis(shape)[1], 21, 0, 6)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    obs = b.obs.copy()
    obs[2:5] = obs_neg[2:5]  # rows 2-4: negative flux over the first fifth
    u = cfg.normalise(b.init)
    u[0, 0] = 1.7    # out of box in Teff
    u[1, 3] = -1.6   # out of box in RV
    u[4, 2] = 1.55   # out of box in [Fe/H], with the negative flux
    status, refs = check_forward(shape, cfg, basis, obs, b.ivar, u)
    flags = [gpu_flags_as_oracle(s) for s in status]
    assert [bool(f & oracle.OUT_OF_BOX) for f in flags] == [True, True, False, False, True, False]
    assert all(flags[i] & oracle.CONT_NONPOS for i in (2, 3, 4))


def fit_and_compare(shape, basis, obs, ivar, init_phys, n_steps, want_cov=False):
    """Grouped GPU fit, then the oracle evaluated at the returned parameters:
    status bits must equal the oracle's flags there."""
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    r = lasp.fit_group(to_dev(obs), to_dev(ivar), wave_grid(shape), to_dev(basis),
                       to_dev(init_phys.astype(np.float32)), n_steps, want_cov=want_cov,
                       margin=shape.margin, degree=shape.degree)
    torch.cuda.synchronize()
    params = r.params.cpu().numpy().astype(np.float64)
    status = r.status.cpu().numpy()
    u_end = cfg.normalise(params)
    refs = []
    for i in range(obs.shape[0]):
        ref = oracle.evaluate(cfg, obs[i], ivar[i], basis, u_end[i])
        refs.append(ref)
        got = gpu_flags_as_oracle(status[i])
        if want_cov:
            got &= ~oracle.SINGULAR  # the covariance's own test, checked by the caller
        assert got == oracle_flags(ref), (i, status[i], ref["flags"])
    return cfg, u_end, status, refs


def test_fit_with_nonpositive_continuum_at_the_end_is_flagged():
    say("[edge: fit, continuum <= 0 at the end] lamost1550 B=4, 300 steps")
    shape, basis, obs, ivar, init, _ = negative_flux_case(4)
    _, _, status, refs = fit_and_compare(shape, basis, obs, ivar, init, 300)
    assert all(s & lasp.ST_CONT_NONPOS for s in status)
    assert all(min_continuum(r) < -1.0 for r in refs)


def test_fit_with_nonpositive_continuum_only_on_the_way_is_not_flagged():
    say("[edge: fit, continuum <= 0 at the start only] lamost1550 bump basis B=8, 500 steps")
    shape, basis, obs, ivar, u0, u_true = bump_basis_case(8)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    init = cfg.physical(u0.astype(np.float64))
    _, u_end, status, refs = fit_and_compare(shape, basis, obs, ivar, init, 500)
    assert not np.any(status & (lasp.ST_CONT_NONPOS | lasp.ST_SINGULAR))
    assert all(min_continuum(r) > 20.0 for r in refs)
    np.testing.assert_allclose(u_end[:, 0], u_true[:, 0], atol=0.1)


def test_fit_out_of_box_and_width_floor_flags_at_the_end():
    say("[edge: fit, out of box / width floor] lamost1550 B=4, 500 steps, with covariance")
    shape, basis, obs, ivar, start, truth = out_of_box_case()
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    init = cfg.physical(start.astype(np.float64))
    _, u_end, status, _ = fit_and_compare(shape, basis, obs, ivar, init, 500, want_cov=True)
    flags = [gpu_flags_as_oracle(s) & ~oracle.SINGULAR for s in status]
    assert flags == [oracle.OUT_OF_BOX, 0, oracle.OUT_OF_BOX | oracle.SIGMA_FLOOR, 0]
    # the floored width has a zero Jacobian column, so the covariance is singular
    # there and only there (the oracle's full inverse fails the same way)
    for i in range(4):
        c = oracle.covariance(cfg, obs[i], ivar[i], basis, u_end[i])
        assert bool(status[i] & lasp.ST_SINGULAR) == (c["rc"] != 0), i
    assert u_end[2, 4] == pytest.approx(start[2, 4], abs=1e-6)


def test_pool_status_describes_the_point_of_each_finish():
    say("[edge: pool finish twice] lamost1550 bump basis + out-of-box fits, 8 slots")
    shape, basis, obs_b, ivar_b, u0, _ = bump_basis_case(4)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    pool = lasp.Pool(wave_grid(shape), to_dev(basis), 8, margin=shape.margin, degree=shape.degree)
    try:
        init = cfg.physical(u0.astype(np.float64)).astype(np.float32)
        pool.load(0, to_dev(obs_b), to_dev(ivar_b), to_dev(init), 500)
        params = torch.empty((4, 5), dtype=torch.float32, device=DEV)
        status = torch.empty(4, dtype=torch.int32, device=DEV)
        for k in (0, 500):
            for _ in range(k // 25):
                pool.step(4, 25)
            pool.finish(0, params, status=status)
            pool.stream.synchronize()
            p = params.cpu().numpy().astype(np.float64)
            st = status.cpu().numpy()
            u_now = cfg.normalise(p)
            for i in range(4):
                ref = oracle.evaluate(cfg, obs_b[i], ivar_b[i], basis, u_now[i])
                assert gpu_flags_as_oracle(st[i]) == oracle_flags(ref), (k, i, st[i], ref["flags"])
                assert bool(st[i] & lasp.ST_CONT_NONPOS) == (k == 0), (k, i)
    finally:
        pool.close()
