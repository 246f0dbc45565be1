"""Clean outlier masking (Section 2.2, steps 6 and 8) on the GPU: the mask
kernel against the oracle's on identical residuals (integer work, bit
exact), and fits with mask updates against the oracle's FP64 Adam with the
same updates."""

import numpy as np
import pytest
import torch

import oracle
import paper_2512_24840_amd as lasp
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name, wave_grid

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
DEV = torch.device("cuda:0")
FIT_TOL = np.array([2.0, 0.005, 0.005, 0.2])


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def with_spikes(batch, n_spikes, seed):
    """Cosmic-ray-like outliers (30 noise sigma) and same-sign shoulders."""
    obs = batch.obs.copy()
    rng = np.random.default_rng(seed)
    where = []
    for i in range(obs.shape[0]):
        good = np.where(batch.ivar[i] > 0)[0]
        sp = rng.choice(good[10:-10], n_spikes, replace=False)
        sig = 1.0 / np.sqrt(batch.ivar[i][sp])
        obs[i, sp] += 30 * sig
        obs[i, sp + 1] += 4 * sig
        where.append(sp)
    return obs, where


@pytest.mark.parametrize("name", ["lamost3900", "desi7800", "lamost1550"])
@pytest.mark.parametrize("f_shift", [0.5, 0.2])
def test_clean_mask_equals_oracle_on_identical_residuals(name, f_shift):
    print(f"[clean mask] {name} f_shift {f_shift}", flush=True)
    shape = shape_by_name(name)
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, 81, 0, 6)
    obs, _ = with_spikes(batch, 12, 3)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    # a model that is close but not equal to the data (the start point's)
    model = np.stack([oracle.evaluate(cfg, obs[i], batch.ivar[i], basis,
                                      cfg.normalise(batch.init[i]))["model"]
                      for i in range(6)]).astype(np.float32)
    keep, nmask = lasp.clean_mask(to_dev(obs), to_dev(batch.ivar), to_dev(model), wave_grid(shape),
                                  f_shift, margin=shape.margin)
    torch.cuda.synchronize()
    keep, nmask = keep.cpu().numpy(), nmask.cpu().numpy()
    for i in range(6):
        ref = oracle.clean_mask(obs[i], batch.ivar[i], model[i].astype(np.float64), f_shift)
        assert np.array_equal(keep[i], ref["keep"]), (i, np.where(keep[i] != ref["keep"]))
        assert nmask[i] == ref["masked"]
        print(f"  {i}: clipped {ref['masked']} (k {ref['k']})", flush=True)


def test_fit_with_clean_updates_matches_oracle_adam_with_clean():
    print("[clean fit] lamost1550 B=6, 500 steps, updates every 30 (<= 11)", flush=True)
    shape = shape_by_name("lamost1550")
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, 82, 0, 6)
    obs, spikes = with_spikes(batch, 8, 4)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    res = lasp.fit_group(to_dev(obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis),
                         to_dev(batch.init), 500, margin=shape.margin, degree=shape.degree,
                         clean_every=30, clean_max=11, want_mask=True)
    torch.cuda.synchronize()
    p = res.params.cpu().numpy().astype(np.float64)
    mask = res.mask.cpu().numpy()
    for i in range(6):
        ref = oracle.adam_fit(cfg, obs[i], batch.ivar[i], basis, cfg.normalise(batch.init[i]),
                              n_max=500, clean_every=30, clean_max=11)
        agree = np.mean(mask[i] == ref["keep"])
        print(f"  {i}: clipped gpu {int((mask[i] == 0).sum())} oracle "
              f"{int((ref['keep'] == 0).sum())}, agreement {agree:.5f}", flush=True)
        assert np.all(mask[i][spikes[i]] == 0) and np.all(ref["keep"][spikes[i]] == 0)
        assert agree >= 0.998, i
        d = np.abs(p[i] - ref["params"])[:4]
        assert np.all(d <= FIT_TOL), (i, d)


def test_clean_does_not_touch_other_spectra():
    print("[clean fit] isolation", flush=True)
    shape = shape_by_name("lamost1550")
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, 83, 0, 5)
    obs, _ = with_spikes(batch, 6, 5)
    kw = dict(margin=shape.margin, degree=shape.degree, clean_every=30, clean_max=11)
    full = lasp.fit_group(to_dev(obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis),
                          to_dev(batch.init), 200, **kw)
    one = lasp.fit_group(to_dev(obs[2:3]), to_dev(batch.ivar[2:3]), wave_grid(shape),
                         to_dev(basis), to_dev(batch.init[2:3]), 200, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(full.params.cpu().numpy()[2], one.params.cpu().numpy()[0])
