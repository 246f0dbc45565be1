"""Continuous batching over resident slot pools: every request completes, each
result is the same alone and in the mix, and sampled results match the
oracle."""

import numpy as np
import pytest
import torch

import bench
import oracle
import paper_2512_24840_amd as lasp
from synth import BOX_HI, BOX_LO, wave_grid

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
FIT_TOL = np.array([2.0, 0.005, 0.005, 0.2])


def test_poisson_stream_alone_equals_mix_and_matches_oracle():
    print("[serving] 1.5 s Poisson stream, 10k spectra/s, LAMOST 3900 / DESI 7800 px", flush=True)
    banks = bench.serving_banks(n_lamost=8192, n_desi=4096)
    server, done, wall, where = bench.run_serving(banks, 10000.0, 1.5, seed=3,
                                                  capacity=(16384, 8192), size_max=2048)
    assert len(done) == len(where) and len(done) > 10
    lat = np.array([r.t_done - r.t_arrival for r in done])
    print(f"requests {len(done)}, spectra {sum(r.n for r in done)}, ticks {server.ticks}, "
          f"p50 {np.median(lat) * 1e3:.1f} ms, p99 {np.percentile(lat, 99) * 1e3:.1f} ms",
          flush=True)
    for r in done:
        assert np.isfinite(r.params.numpy()).all()
    dev = torch.device("cuda:0")
    checked = {"lamost3900": 0, "desi7800": 0}
    for r in sorted(done, key=lambda r: -r.n):
        lane, off, n = where[r.rid]
        if checked[lane] >= 3:
            continue
        checked[lane] += 1
        shape, basis, b = banks[lane]
        arms = lasp.Arms(shape.arm_start, shape.arm_sigma_kms) if shape.arm_start else None
        alone = lasp.fit_group(torch.from_numpy(b.obs[off:off + n]).to(dev),
                               torch.from_numpy(b.ivar[off:off + n]).to(dev), wave_grid(shape),
                               torch.from_numpy(basis).to(dev),
                               torch.from_numpy(b.init[off:off + n]).to(dev), 500,
                               margin=shape.margin, degree=shape.degree, arms=arms)
        torch.cuda.synchronize()
        assert np.array_equal(alone.params.cpu().numpy(), r.params.numpy()), (lane, r.rid)
    n_ok = n_chk = 0
    for r in done:
        if r.rid % 8:
            continue
        lane, off, n = where[r.rid]
        shape, basis, b = banks[lane]
        cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
        ref = oracle.fit(cfg, b.obs[off], b.ivar[off], basis, cfg.normalise(b.init[off]))
        err = np.abs(r.params[0].numpy().astype(np.float64) - ref["params"])[:4]
        n_chk += 1
        n_ok += int(np.all(err <= FIT_TOL))
        assert np.all(err <= FIT_TOL), (lane, r.rid, err)
    print(f"oracle parity {n_ok}/{n_chk}", flush=True)


def test_stream_with_stopping_rules_releases_requests_early_and_matches_grouped_fits():
    print("[serving, stopping rules] 1.0 s Poisson stream, 6k spectra/s", flush=True)
    banks = bench.serving_banks(n_lamost=4096, n_desi=2048)
    server, done, wall, where = bench.run_serving(banks, 6000.0, 1.0, seed=4,
                                                  capacity=(8192, 4096), size_max=1024,
                                                  stop_window=50, stop_tol=1e-5)
    assert len(done) == len(where) and len(done) > 5
    early = [r for r in done if r.steps < 500]
    print(f"requests {len(done)}, released before 500 steps: {len(early)}", flush=True)
    assert early, "no request was released by the stopping rules"
    dev = torch.device("cuda:0")
    for r in sorted(done, key=lambda r: -r.n)[:4]:
        lane, off, n = where[r.rid]
        shape, basis, b = banks[lane]
        arms = lasp.Arms(shape.arm_start, shape.arm_sigma_kms) if shape.arm_start else None
        alone = lasp.fit_group(torch.from_numpy(b.obs[off:off + n]).to(dev),
                               torch.from_numpy(b.ivar[off:off + n]).to(dev), wave_grid(shape),
                               torch.from_numpy(basis).to(dev),
                               torch.from_numpy(b.init[off:off + n]).to(dev), 500,
                               margin=shape.margin, degree=shape.degree, arms=arms,
                               stop_window=50, stop_tol=1e-5)
        torch.cuda.synchronize()
        assert np.array_equal(alone.params.cpu().numpy(), r.params.numpy()), (lane, r.rid)
        assert np.array_equal(alone.status.cpu().numpy(), r.status.numpy()), (lane, r.rid)
        cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
        ref = oracle.fit(cfg, b.obs[off], b.ivar[off], basis, cfg.normalise(b.init[off]))
        err = np.abs(r.params[0].numpy().astype(np.float64) - ref["params"])[:4]
        assert np.all(err <= FIT_TOL), (lane, r.rid, err)
