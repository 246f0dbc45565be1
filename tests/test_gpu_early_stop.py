"""Per-spectrum stopping rules of the optimisation stage (Section 2.2, stage
8) on the GPU: the stopping step and the fitted values against the oracle's
FP64 Adam with the same rules, the step limit, isolation between spectra,
and the resident slot pools."""

import numpy as np
import pytest
import torch

import oracle
import paper_2512_24840_amd as lasp
from loss_history import gpu_losses
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name, wave_grid

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
DEV = torch.device("cuda:0")
FIT_TOL = np.array([2.0, 0.005, 0.005, 0.2])
W, TOL, NMAX = 50, 1e-5, 500
RULE_BIT = {2: lasp.ST_STOP_FLAT, 3: lasp.ST_STOP_RISING,
            1: lasp.ST_NOT_CONVERGED}


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def problem(name, n, cid):
    shape = shape_by_name(name)
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, cid, 0, n)
    return shape, basis, batch


def gpu_fit(shape, basis, batch, sl=slice(None), **kw):
    res = lasp.fit_group(to_dev(batch.obs[sl]), to_dev(batch.ivar[sl]), wave_grid(shape),
                         to_dev(basis), to_dev(batch.init[sl]), kw.pop("n_steps", NMAX),
                         margin=shape.margin, degree=shape.degree, **kw)
    torch.cuda.synchronize()
    return (res.params.cpu().numpy().astype(np.float64), res.status.cpu().numpy(),
            res.steps.cpu().numpy())


@pytest.mark.parametrize("name", ["lamost1550", "lamost3900"])
def test_stopping_step_and_fit_match_oracle_adam(name):
    print(f"[early stop vs oracle Adam] {name} B=12", flush=True)
    shape, basis, batch = problem(name, 12, 41)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    p, st, steps = gpu_fit(shape, basis, batch, stop_window=W, stop_tol=TOL)
    ref = oracle.adam_fit_many(cfg, batch.obs, batch.ivar, basis, batch.init, n_max=NMAX,
                               window=W, tol=TOL)
    lm = oracle.fit_many(cfg, batch.obs, batch.ivar, basis, batch.init)
    for i in range(12):
        r = ref[i]
        print(f"  {i}: gpu {steps[i]} steps status {st[i]:#x}, oracle {r['steps']} rule {r['rule']}",
              flush=True)
        assert st[i] & RULE_BIT[r["rule"]], (i, st[i], r["rule"])
        assert abs(int(steps[i]) - r["steps"]) <= max(10, 0.1 * r["steps"]), (i, steps[i], r["steps"])
        assert np.all(np.abs(p[i] - r["params"])[:4] <= FIT_TOL), (i, p[i], r["params"])
        assert np.all(np.abs(p[i] - lm[i]["params"])[:4] <= FIT_TOL), (i, p[i], lm[i]["params"])


@pytest.mark.parametrize("name,w,tol,rule_seen", [
    ("lamost1550", W, TOL, 2), ("lamost3900", W, TOL, 2),
    ("lamost1550", 3, 1e-12, 3),     # a short window: the loss rises 3 steps running
    ("lamost1550", W, 1e-12, 1),     # no flat window: the step limit
])
def test_stopping_step_is_the_rule_on_the_gpu_own_losses(name, w, tol, rule_seen):
    """The stopping step is an integer decided on floating-point losses, so
    the decision is checked in the kernel's own arithmetic: the losses
    ell_t = sqrt(chi2 / n_eff) of the fixed-step fit after t = 0 .. T steps,
    scanned by the oracle's rules, give exactly the step and the rule at
    which the GPU stopped each fit; each case sees its rule (flat loss,
    rising loss, step limit) at least once."""
    print(f"[early stop: rules on the GPU's own losses] {name} B=12 W={w} tol={tol}", flush=True)
    shape, basis, batch = problem(name, 12, 41)
    p, st, steps = gpu_fit(shape, basis, batch, stop_window=w, stop_tol=tol)
    n, T = 12, int(steps.max())
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    ell, got, n_eff = gpu_losses(shape, to_dev(basis), to_dev(batch.obs), to_dev(batch.ivar),
                                 to_dev(batch.init),
                                 to_dev(cfg.normalise(batch.init).astype(np.float32)), T)
    # the rules are tested after t = 0 .. NMAX - 1 steps (none after the last)
    n_scan = min(T + 1, NMAX)
    rules = set()
    for i in range(n):
        assert n_eff[i] > 0
        t_ref, rule = oracle.stop_step(np.ascontiguousarray(ell[:n_scan, i]), n_scan, w, tol)
        rules.add(rule)
        print(f"  {i}: gpu {steps[i]} steps status {st[i]:#x}, rules on its losses: {t_ref} "
              f"rule {rule}", flush=True)
        assert t_ref == steps[i] and st[i] & RULE_BIT[rule], (i, steps[i], st[i], t_ref, rule)
        # the fit that stopped is the fixed-step fit's prefix, bitwise
        assert np.array_equal(got[steps[i], i].astype(np.float64), p[i]), i
    assert rule_seen in rules, rules


def test_rules_that_cannot_fire_give_the_fixed_step_fit_bitwise():
    print("[early stop] window beyond the step limit == fixed steps", flush=True)
    shape, basis, batch = problem("lamost1550", 9, 43)
    p0, st0, n0 = gpu_fit(shape, basis, batch, n_steps=120)
    p1, st1, n1 = gpu_fit(shape, basis, batch, n_steps=120, stop_window=200, stop_tol=0.0)
    assert np.array_equal(p0, p1)
    assert np.all(n0 == 120) and np.all(n1 == 120)
    assert np.all(st1 & lasp.ST_NOT_CONVERGED)
    assert np.array_equal(st1 & ~lasp.ST_NOT_CONVERGED, st0)


def test_masked_spectrum_stops_after_one_window_and_neighbours_are_unaffected():
    print("[early stop] isolation", flush=True)
    shape, basis, batch = problem("lamost1550", 7, 44)
    batch.ivar[3] = 0.0
    p, st, steps = gpu_fit(shape, basis, batch, stop_window=W, stop_tol=TOL)
    assert steps[3] == W and st[3] & lasp.ST_STOP_FLAT and st[3] & lasp.ST_NO_DATA
    np.testing.assert_allclose(p[3], batch.init[3], rtol=1e-6, atol=1e-4)
    for i in (0, 6):
        pa, sa, na = gpu_fit(shape, basis, batch, slice(i, i + 1), stop_window=W, stop_tol=TOL)
        assert np.array_equal(pa[0], p[i]) and na[0] == steps[i] and sa[0] == st[i], i


def test_pool_with_stopping_rules_equals_grouped_fit():
    print("[early stop] pools: progress query and results", flush=True)
    shape, basis, batch = problem("lamost1550", 24, 45)
    p_ref, st_ref, n_ref = gpu_fit(shape, basis, batch, stop_window=W, stop_tol=TOL)
    pool = lasp.Pool(wave_grid(shape), to_dev(basis), 64, margin=shape.margin,
                     degree=shape.degree, stop_window=W, stop_tol=TOL)
    with torch.cuda.stream(pool.stream):
        pool.load(5, to_dev(batch.obs[:10]), to_dev(batch.ivar[:10]), to_dev(batch.init[:10]), NMAX)
        pool.load(30, to_dev(batch.obs[10:]), to_dev(batch.ivar[10:]), to_dev(batch.init[10:]), NMAX)
        steps = torch.empty(64, dtype=torch.int32, device=DEV)
        done = torch.empty(64, dtype=torch.int32, device=DEV)
        for _ in range(NMAX // 25):
            pool.step(64, 25)
        pool.progress(0, steps, done)
        out = torch.empty((24, 5), dtype=torch.float32, device=DEV)
        status = torch.empty(24, dtype=torch.int32, device=DEV)
        pool.finish(5, out[:10], status=status[:10])
        pool.finish(30, out[10:], status=status[10:])
    pool.stream.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    sl = np.r_[5:15, 30:44]
    assert np.array_equal(got, p_ref)
    assert np.array_equal(steps.cpu().numpy()[sl], n_ref)
    assert np.all(done.cpu().numpy()[sl] == 1)
    assert np.array_equal(status.cpu().numpy(), st_ref)
    pool.close()
