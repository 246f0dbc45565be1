"""The emulator steps on the GPU: flux-conserving resampling (Section 2.2,
step 3, Eqs. 2-4) against the oracle's, and the interpolator of Eq. 1 over
the five Teff regimes (three temperature classes) -- model, gradient,
Jacobian and fits -- against the oracle's FP64 evaluation and fits."""

import math
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2512_24840_amd as lasp
from synth import (BOX_HI, BOX_LO, linear_grid_basis, make_basis, make_spectra, shape_by_name,
                   wave_grid)

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
DEV = torch.device("cuda:0")
FIT_TOL = np.array([2.0, 0.005, 0.005, 0.2])
EPS64 = np.finfo(np.float64).eps


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def arms_of(shape):
    return lasp.Arms(shape.arm_start, shape.arm_sigma_kms) if shape.arm_start else None


def ext_lg0(shape):
    """log10 of the centre of basis column 0 (pixel -margin)."""
    return math.log10(shape.lam0) - shape.margin * shape.dlog10


def resample_bound(src, lam0, dlam, n_out, lg0, d, ref):
    """Per-output bound on |GPU - oracle|: one FP32 rounding of the result,
    plus the rounding of the oracle's cumulative sums (a running sum of k
    terms errs by at most k eps sum|x| dlam; a bin value differences two
    of them and divides by the bin width) and of the GPU's local sums."""
    e = 10.0 ** (lg0 + (np.arange(n_out + 1) - 0.5) * d)
    width = np.diff(e)
    s_abs = np.abs(src.astype(np.float64)).sum(axis=1, keepdims=True) * dlam
    n = src.shape[1]
    return np.spacing(np.abs(ref.astype(np.float32))).astype(np.float64) + \
        4.0 * n * EPS64 * s_abs / width[None, :]


@pytest.mark.parametrize("name", ["lamost1550", "lamost3900", "desi7800"])
def test_resampled_basis_matches_oracle(name):
    shape = shape_by_name(name)
    lam0, dlam, rows = linear_grid_basis(shape, n_classes=3)
    say(f"[resample] {name}: {rows.shape[0]} rows x {rows.shape[1]} -> {shape.n_ext}")
    got = lasp.resample(to_dev(rows), lam0, dlam, shape.n_ext, ext_lg0(shape), shape.dlog10)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    ref, ok = oracle.resample(rows, lam0, dlam, shape.n_ext, ext_lg0(shape), shape.dlog10)
    assert ok
    err = np.abs(got.astype(np.float64) - ref)
    bound = resample_bound(rows, lam0, dlam, shape.n_ext, ext_lg0(shape), shape.dlog10, ref)
    exact = np.mean(got == ref.astype(np.float32))
    say(f"  equal to the rounded oracle value: {exact:.6f}, max err/bound {np.max(err / bound):.3g}")
    assert np.all(err <= bound)


def test_resample_many_rows_ragged_width_and_constant_rows():
    # more rows than the grid's row groups (1024), a width that is not a
    # multiple of the 256-thread block, constant rows that must stay constant
    rng = np.random.default_rng(7)
    lam0, dlam, n_src, n_out = 5000.0, 0.05, 4000, 333
    src = rng.uniform(0.2, 2.0, (1500, n_src)).astype(np.float32)
    src[::100] = 1.0
    lg0, d = math.log10(5010.0), 2e-5
    say(f"[resample] 1500 rows x {n_src} -> {n_out}")
    got = lasp.resample(to_dev(src), lam0, dlam, n_out, lg0, d)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    ref, ok = oracle.resample(src, lam0, dlam, n_out, lg0, d)
    assert ok
    bound = resample_bound(src, lam0, dlam, n_out, lg0, d, ref)
    assert np.all(np.abs(got - ref) <= bound)
    np.testing.assert_allclose(got[::100], 1.0, rtol=2 * np.finfo(np.float32).eps)


@pytest.mark.parametrize("ratio", [6, 12, 24, 34, 70])
def test_resample_every_staged_window_size(ratio):
    # target bins of about `ratio` source pixels: the 256-pixel blocks of the
    # tiled kernel stage windows of about 256 * ratio source pixels, which
    # selects each of its window sizes (2048, 4096, 8192, 12288 pixels) and,
    # at 70, the direct form; 700 target pixels leave a ragged last block
    rng = np.random.default_rng(100 + ratio)
    lam0, dlam, n_out = 4000.0, 0.05, 700
    lg0 = math.log10(4003.0)
    d = ratio * dlam / (4003.0 * math.log(10.0))
    n_src = int((10.0 ** (lg0 + (n_out - 0.5) * d) - (lam0 - dlam / 2)) / dlam) + 10
    src = rng.uniform(0.2, 2.0, (300, n_src)).astype(np.float32)
    say(f"[resample] 300 rows x {n_src} -> {n_out} (bins of ~{ratio} source pixels)")
    got = lasp.resample(to_dev(src), lam0, dlam, n_out, lg0, d)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    ref, ok = oracle.resample(src, lam0, dlam, n_out, lg0, d)
    assert ok
    bound = resample_bound(src, lam0, dlam, n_out, lg0, d, ref)
    assert np.all(np.abs(got - ref) <= bound)


def test_resample_16384_rows_at_the_resampling_leg_shape_on_sample():
    # the resampling leg's launch: 16,384 linear-grid rows of 28,054 pixels
    # (the three-class basis rows on their linear grid, each row with its
    # own scale and offset) onto the 4,028-column basis grid; 64 rows spread
    # over the launch against the oracle, the rest for finiteness
    shape = shape_by_name("lamost3900")
    lam0, dlam, rows = linear_grid_basis(shape, n_classes=3)
    B = 16384
    rng = np.random.default_rng(9)
    scale = rng.uniform(0.5, 1.5, (B, 1)).astype(np.float32)
    offset = rng.uniform(-0.2, 0.2, (B, 1)).astype(np.float32)
    src = rows[np.arange(B) % rows.shape[0]] * scale + offset
    lg0 = ext_lg0(shape)
    say(f"[resample] {B} rows x {src.shape[1]} -> {shape.n_ext}")
    got = lasp.resample(to_dev(src), lam0, dlam, shape.n_ext, lg0, shape.dlog10)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.all(np.isfinite(got))
    idx = np.linspace(0, B - 1, 64).astype(int)
    ref, ok = oracle.resample(src[idx], lam0, dlam, shape.n_ext, lg0, shape.dlog10)
    assert ok
    bound = resample_bound(src[idx], lam0, dlam, shape.n_ext, lg0, shape.dlog10, ref)
    err = np.abs(got[idx].astype(np.float64) - ref)
    say(f"  max err/bound on the sample {np.max(err / bound):.3g}")
    assert np.all(err <= bound)


def test_resample_coarse_target_bins_wider_than_the_staged_window():
    # target bins of about 920 source pixels: a chunk of target pixels spans
    # more source pixels than the tiled kernel stages in LDS, so the direct
    # form runs; results obey the same bound
    rng = np.random.default_rng(8)
    lam0, dlam, n_src, n_out = 4000.0, 0.01, 30000, 28
    src = rng.uniform(0.2, 2.0, (50, n_src)).astype(np.float32)
    lg0, d = math.log10(4006.0), 1e-3
    say(f"[resample] 50 rows x {n_src} -> {n_out} (coarse bins)")
    got = lasp.resample(to_dev(src), lam0, dlam, n_out, lg0, d)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    ref, ok = oracle.resample(src, lam0, dlam, n_out, lg0, d)
    assert ok
    bound = resample_bound(src, lam0, dlam, n_out, lg0, d, ref)
    assert np.all(np.abs(got - ref) <= bound)


def test_resample_strided_rows_through_the_c_abi():
    # lasp_resample takes row strides: source rows padded to 4,003 floats and
    # output rows to 341 (row starts off 16-byte boundaries), the padding
    # left untouched
    import ctypes
    rng = np.random.default_rng(11)
    lam0, dlam, n_src, n_out, rows = 5000.0, 0.05, 4000, 333, 300
    lds, ldo = n_src + 3, n_out + 8
    src = rng.uniform(0.2, 2.0, (rows, n_src)).astype(np.float32)
    lg0, d = math.log10(5010.0), 2e-5
    padded = np.full((rows, lds), np.nan, np.float32)
    padded[:, :n_src] = src
    src_dev = to_dev(padded)
    out_dev = torch.full((rows, ldo), -7.0, dtype=torch.float32, device=DEV)
    lib = lasp.lasp.load()
    rc = lib.lasp_resample(ctypes.c_void_p(src_dev.data_ptr()), rows, n_src, lds, lam0, dlam,
                           ctypes.c_void_p(out_dev.data_ptr()), n_out, ldo, lg0, d,
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    out = out_dev.cpu().numpy()
    assert np.all(out[:, n_out:] == -7.0)
    ref, ok = oracle.resample(src, lam0, dlam, n_out, lg0, d)
    assert ok
    bound = resample_bound(src, lam0, dlam, n_out, lg0, d, ref)
    assert np.all(np.abs(out[:, :n_out] - ref) <= bound)


def test_resample_rejects_a_target_outside_the_source():
    src = torch.ones((2, 100), dtype=torch.float32, device=DEV)
    with pytest.raises(lasp.LaspError) as e:
        lasp.resample(src, 4000.0, 0.2, 50, math.log10(3999.0), 1e-5)
    assert e.value.code == -2


def three_class_case(name, n, cid):
    shape = shape_by_name(name)
    basis3, lines3 = make_basis(shape, n_classes=3)
    batch = make_spectra(shape, lines3, cid, 0, n)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI, n_classes=3)
    return shape, cfg, basis3, batch


# Teff inside each regime the box reaches and inside both blends (away from
# the edges, where the class weights have a kink)
TEFFS = np.array([4150.0, 4420.0, 5200.0, 6600.0, 7300.0, 7650.0, 7950.0])


@pytest.mark.parametrize("name", ["lamost1550", "lamost3900", "desi7800"])
def test_three_class_forward_matches_oracle(name):
    n = TEFFS.size
    say(f"[3-class forward] {name} B={n}")
    shape, cfg, basis3, batch = three_class_case(name, n, 21)
    init = batch.init.astype(np.float64).copy()
    init[:, 0] = TEFFS
    rng = np.random.default_rng(4)
    u = (cfg.normalise(init) + rng.normal(0, 0.02, (n, 5))).astype(np.float32)
    res = lasp.forward(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis3),
                       to_dev(u), want_model=True, want_grad=True, want_jac=True,
                       margin=shape.margin, degree=shape.degree, arms=arms_of(shape), n_classes=3)
    torch.cuda.synchronize()
    model, chi2 = res["model"].cpu().numpy(), res["chi2"].cpu().numpy()
    grad, jac = res["grad"].cpu().numpy(), res["jac"].cpu().numpy()
    for i in range(n):
        ref = oracle.evaluate(cfg, batch.obs[i], batch.ivar[i], basis3, u[i].astype(np.float64))
        w, dw = oracle.class_weights(cfg, u[i].astype(np.float64))
        rms = np.sqrt(np.mean(ref["model"] ** 2))
        assert np.max(np.abs(model[i] - ref["model"])) <= 1e-5 * rms, i
        assert chi2[i] == pytest.approx(ref["chi2"], rel=1e-5), i
        assert np.linalg.norm(grad[i] - ref["grad"]) <= 1e-5 * np.linalg.norm(ref["grad"]) + 1e-9, \
            (i, w, grad[i], ref["grad"])
        for t in range(5):
            scale = np.sqrt(np.mean(ref["jac"][t] ** 2))
            assert np.max(np.abs(jac[i, t] - ref["jac"][t])) <= 1e-4 * scale, (i, t, w, dw)


EDGES = np.array([4000.0, 4550.0, 7000.0, 9000.0])


def check_fits(tag, cfg, batch, basis, got, ref, tol):
    """Fitted values against the oracle's LM fits.  The class blend is linear
    in Teff, so chi2 has a kink at each regime edge: where the oracle's fit
    ends within 30 K of an edge, a gradient method may stop at the kink or
    on either side of it, and the unique quantity is the minimum chi2 --
    the GPU's fit (evaluated by the oracle) must reach the oracle's chi2 to
    within 0.1 (a tenth of the one-sigma change).  Elsewhere the fitted
    values must agree to tol."""
    refp = np.array([r["params"] for r in ref])
    at_kink = np.min(np.abs(refp[:, :1] - EDGES[None, :]), axis=1) < 30.0
    for i in range(got.shape[0]):
        if at_kink[i]:
            c = oracle.evaluate(cfg, batch.obs[i], batch.ivar[i], basis, cfg.normalise(got[i]))["chi2"]
            say(f"  {tag} {i}: oracle fit at a regime edge (Teff {refp[i, 0]:.1f}); chi2 gpu {c:.4f} "
                f"oracle {ref[i]['chi2']:.4f}")
            assert c <= ref[i]["chi2"] + 0.1, (tag, i, c, ref[i]["chi2"])
        else:
            err = np.abs(got[i] - refp[i])[:4]
            assert np.all(err <= tol), (tag, i, err)
    far = ~at_kink
    if far.any():
        say(f"  {tag}: max |GPU - oracle| away from the edges {np.abs(got - refp)[far, :4].max(axis=0)}")


def test_three_class_fits_match_oracle_lm():
    say("[3-class fit] lamost1550 B=10: 500 Adam steps, and Adam 100 + LM polish")
    shape, cfg, basis3, batch = three_class_case("lamost1550", 10, 22)
    ref = oracle.fit_many(cfg, batch.obs, batch.ivar, basis3, batch.init)
    kw = dict(margin=shape.margin, degree=shape.degree, n_classes=3)
    a = lasp.fit_group(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis3),
                       to_dev(batch.init), 500, **kw)
    p = lasp.fit_group(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis3),
                       to_dev(batch.init), 100, polish_iters=15, **kw)
    torch.cuda.synchronize()
    check_fits("adam", cfg, batch, basis3, a.params.cpu().numpy().astype(np.float64), ref, FIT_TOL)
    check_fits("adam+lm", cfg, batch, basis3, p.params.cpu().numpy().astype(np.float64), ref,
               FIT_TOL / 10)
    st = p.status.cpu().numpy()
    assert not np.any(st & lasp.ST_POLISH_LIMIT), st


def test_fit_on_a_gpu_resampled_basis_matches_oracle_on_its_own_resampling():
    say("[resample + 3-class fit] lamost1550 B=6 from a linear-grid basis")
    shape = shape_by_name("lamost1550")
    lam0, dlam, rows = linear_grid_basis(shape, n_classes=3)
    basis_gpu = lasp.resample(to_dev(rows), lam0, dlam, shape.n_ext, ext_lg0(shape), shape.dlog10)
    ref_basis, ok = oracle.resample(rows, lam0, dlam, shape.n_ext, ext_lg0(shape), shape.dlog10)
    assert ok
    ref_basis = ref_basis.astype(np.float32)
    _, lines3 = make_basis(shape, n_classes=3)
    batch = make_spectra(shape, lines3, 23, 0, 6)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI, n_classes=3)
    res = lasp.fit_group(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), basis_gpu,
                         to_dev(batch.init), 100, margin=shape.margin, degree=shape.degree,
                         n_classes=3, polish_iters=15)
    torch.cuda.synchronize()
    ref = oracle.fit_many(cfg, batch.obs, batch.ivar, ref_basis, batch.init)
    check_fits("resampled", cfg, batch, ref_basis, res.params.cpu().numpy().astype(np.float64), ref,
               FIT_TOL / 10)


def test_three_class_pool_equals_grouped_fit():
    say("[3-class pool] lamost1550 B=8")
    shape, cfg, basis3, batch = three_class_case("lamost1550", 8, 24)
    ref = lasp.fit_group(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis3),
                         to_dev(batch.init), 150, margin=shape.margin, degree=shape.degree,
                         n_classes=3)
    pool = lasp.Pool(wave_grid(shape), to_dev(basis3), 16, margin=shape.margin,
                     degree=shape.degree, n_classes=3)
    with torch.cuda.stream(pool.stream):
        pool.load(3, to_dev(batch.obs), to_dev(batch.ivar), to_dev(batch.init), 150)
        for _ in range(6):
            pool.step(16, 25)
        out = torch.empty((8, 5), dtype=torch.float32, device=DEV)
        pool.finish(3, out)
    pool.stream.synchronize()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref.params.cpu().numpy())
    pool.close()


def test_three_class_fit_16384x3900_matches_oracle_adam_on_sample():
    # the three-class leg's launch: 16,384 spectra x 3,900 px, 500 Adam
    # steps on the regime-ordered work list; 32 fits spread over the group
    # against the oracle's FP64 Adam with the same settings
    from synth import make_spectra_parallel
    shape = shape_by_name("lamost3900")
    basis3, lines3 = make_basis(shape, n_classes=3)
    B = 16384
    batch = make_spectra_parallel(shape, lines3, 41, 0, B)
    say(f"[3-class full size] lamost3900 B={B}, 500 steps; oracle Adam on 32")
    res = lasp.fit_group(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis3),
                         to_dev(batch.init), 500, margin=shape.margin, degree=shape.degree,
                         n_classes=3)
    torch.cuda.synchronize()
    params = res.params.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(params))
    idx = np.linspace(0, B - 1, 32).astype(int)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI, n_classes=3)
    ref = oracle.adam_fit_many(cfg, batch.obs[idx], batch.ivar[idx], basis3, batch.init[idx],
                               n_max=500)
    err = np.abs(params[idx] - np.array([r["params"] for r in ref]))[:, :4]
    say(f"  max |GPU - oracle Adam| {err.max(axis=0)}")
    assert np.all(err <= FIT_TOL), err.max(axis=0)


@pytest.mark.parametrize("stop_window", [0, 20])
def test_three_class_fit_does_not_depend_on_the_order_of_the_batch(stop_window):
    # three-class fits go through a work list grouped by Teff regime, and
    # contraction tiles of one regime leave out the other classes' products
    # (which would add exact zeros): a fit's arithmetic must not depend on
    # the tile it lands in, so a shuffled batch gives bit-identical fits
    n = 150
    say(f"[3-class order] lamost1550 B={n} stop_window={stop_window}")
    shape, cfg, basis3, batch = three_class_case("lamost1550", n, 26)
    perm = np.random.default_rng(7).permutation(n)
    kw = dict(margin=shape.margin, degree=shape.degree, n_classes=3, want_cov=True,
              stop_window=stop_window)
    grid = wave_grid(shape)
    a = lasp.fit_group(to_dev(batch.obs), to_dev(batch.ivar), grid, to_dev(basis3),
                       to_dev(batch.init), 120, **kw)
    b = lasp.fit_group(to_dev(batch.obs[perm]), to_dev(batch.ivar[perm]), grid, to_dev(basis3),
                       to_dev(batch.init[perm]), 120, **kw)
    torch.cuda.synchronize()
    for f in ("params", "cov", "chi2", "steps"):
        x, y = getattr(a, f).cpu().numpy(), getattr(b, f).cpu().numpy()
        assert np.array_equal(x[perm], y), f
    # the batch spans the cool blend, the warm class and the hot blend
    teff = a.params.cpu().numpy()[:, 0]
    assert teff.min() < EDGES[1] and teff.max() > EDGES[2], (teff.min(), teff.max())


def test_bf16x3_with_three_classes_is_unsupported():
    shape, cfg, basis3, batch = three_class_case("lamost1550", 2, 25)
    with pytest.raises(lasp.LaspError) as e:
        lasp.fit_group(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis3),
                       to_dev(batch.init), 10, margin=shape.margin, degree=shape.degree,
                       n_classes=3, precision="bf16x3")
    assert e.value.code == -5
