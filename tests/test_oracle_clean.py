"""Pins of the oracle's Clean mask (Section 2.2, step 6): residual patterns
built so that each of the three clipping steps, the relaxation of k, the
flux-gradient allowance and the invalid-pixel rule decide known pixels."""

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.usefixtures("oracle_lib")

A = 0.01          # residual scale
N = 1000


def base(n=N):
    """Residual +-A alternating (sigma ~ A), flat model, every pixel valid."""
    eps = A * (-1.0) ** np.arange(n)
    return eps, np.ones(n), np.full(n, 1e4, dtype=np.float32)


def run(eps, model, ivar, f=0.5):
    obs = (model + eps).astype(np.float32)
    # the oracle sees the float32 flux; keep the designed residual exact
    model = obs.astype(np.float64) - eps
    r = oracle.clean_mask(obs, ivar, model, f)
    return set(np.where(r["keep"] == 0)[0].tolist()), r


def test_spike_b_neighbours_c_and_same_sign_shoulders_d():
    eps, m, iv = base()
    eps[500] = 20 * A                       # step B
    eps[499] = eps[501] = 3 * A             # step C (> 2 sigma, < 3 sigma)
    eps[498] = 1.5 * A                      # step D from 499 (same sign, smaller, > sigma')
    eps[502:506] = [1.5 * A, 1.4 * A, 1.3 * A, 1.2 * A]   # a D chain, one pixel per pass
    eps[497] = -A
    eps[506] = -A                           # sign change ends the chains
    masked, r = run(eps, m, iv)
    assert masked == set(range(498, 506)), sorted(masked)
    assert r["k"] == 3.0


def test_d_does_not_take_a_neighbour_larger_than_its_seed():
    eps, m, iv = base()
    eps[500] = 20 * A
    eps[499] = eps[501] = 3 * A
    eps[502] = 2.5 * A     # C masks it directly (> 2 sigma): a C outlier seeds D too
    eps[503] = 2.9 * A     # larger than its seed 502 -> not taken by D; < 3 sigma, not B
    eps[504] = -A
    masked, _ = run(eps, m, iv)
    assert 503 not in masked and {499, 500, 501, 502} <= masked


def test_k_relaxes_while_more_than_three_percent_would_be_clipped():
    eps, m, iv = base()
    eps[::20] = 4 * A      # 5 % of the pixels at ~3 sigma: clipped at k = 3, kept at k = 4
    masked, r = run(eps, m, iv)
    assert r["k"] == 4.0 and masked == set()


def test_flux_gradient_spares_residuals_at_steep_model_edges():
    eps, m, iv = base()
    m[600:] += 10 * A      # a model edge: G = 10 A at pixels 599 and 600
    eps[600] = 8 * A       # 8 A - 0.5 * 10 A = 3 A < 3 sigma: kept
    masked, _ = run(eps, m, iv, f=0.5)
    assert 600 not in masked
    masked, _ = run(eps, m, iv, f=0.2)  # 8 A - 2 A = 6 A > 3 sigma: clipped
    assert 600 in masked


def test_invalid_pixels_are_neither_masked_nor_seeds():
    eps, m, iv = base()
    eps[300] = 50 * A
    iv[300] = 0.0
    eps[299] = eps[301] = 3 * A
    masked, r = run(eps, m, iv)
    assert masked == set() and r["masked"] == 0


def test_adam_with_clean_masks_injected_spikes_and_recovers_the_masked_fit():
    from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name

    shape = shape_by_name("lamost1550")
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, 71, 0, 3)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    rng = np.random.default_rng(5)
    for i in range(3):
        obs = batch.obs[i].copy()
        iv = batch.ivar[i]
        good = np.where(iv > 0)[0]
        spikes = rng.choice(good[10:-10], 8, replace=False)
        obs[spikes] += 30.0 / np.sqrt(iv[spikes])          # cosmic-ray-like outliers
        u0 = cfg.normalise(batch.init[i])
        res = oracle.adam_fit(cfg, obs, iv, basis, u0, n_max=500, clean_every=30, clean_max=11)
        assert np.all(res["keep"][spikes] == 0), i          # every spike is clipped
        iv_m = iv.copy()
        iv_m[spikes] = 0.0
        ref = oracle.fit(cfg, batch.obs[i], iv_m, basis, u0)   # LM with the spikes masked a priori
        d = np.abs(res["params"] - ref["params"])[:4]
        assert d[0] <= 2.0 and d[1] <= 0.005 and d[2] <= 0.005 and d[3] <= 0.2, (i, d)
