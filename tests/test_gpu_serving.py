"""The fit server (lasp_server_*) and pool resizing, through the C ABI.

Continuous batching over slot pools under one HBM budget: every request
completes; a request's results are bitwise the same alone (one grouped fit
of its spectra) and in the mix; sampled results match the oracle's fit
(Section 2.2 stages 2-9); the byte budget, not a slot count, holds requests
back; and a pool resized while its fits are resident continues them
unchanged.
"""

import sys
import time

import numpy as np
import pytest
import torch

import bench
import oracle
import paper_2512_24840_amd as lasp
from paper_2512_24840_amd.serving import Server
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name, wave_grid

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
FIT_TOL = np.array([2.0, 0.005, 0.005, 0.2])
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def arms_of(shape):
    return lasp.Arms(shape.arm_start, shape.arm_sigma_kms) if shape.arm_start else None


def alone(shape, basis, b, off, n, **kw):
    res = lasp.fit_group(to_dev(b.obs[off:off + n]), to_dev(b.ivar[off:off + n]), wave_grid(shape),
                         to_dev(basis), to_dev(b.init[off:off + n]), 500, margin=shape.margin,
                         degree=shape.degree, arms=arms_of(shape), **kw)
    torch.cuda.synchronize()
    return res


def check_oracle(shape, basis, b, off, params):
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    ref = oracle.fit(cfg, b.obs[off], b.ivar[off], basis, cfg.normalise(b.init[off]))
    return np.abs(params.astype(np.float64) - ref["params"])[:4]


def test_poisson_stream_alone_equals_mix_and_matches_oracle():
    say("[server] 1.5 s Poisson stream, 10k spectra/s, LAMOST 3900 / DESI 7800 px")
    banks = bench.serving_banks(n_lamost=8192, n_desi=4096)
    stats, done, wall, where = bench.run_serving(banks, 10000.0, 1.5, seed=3, size_max=2048)
    assert len(done) == len(where) and len(done) > 10
    lat = np.array([r.latency_s for r in done])
    say(f"requests {len(done)}, spectra {sum(r.n for r in done)}, ticks {stats['ticks']}, "
        f"resizes {stats['resizes']}, p50 {np.median(lat) * 1e3:.1f} ms, "
        f"p99 {np.percentile(lat, 99) * 1e3:.1f} ms")
    assert stats["completed"] == len(done) and stats["queued"] == 0
    for r in done:
        assert np.isfinite(r.params.cpu().numpy()).all()
    # alone = mix on 32 requests: the 16 largest of each shape
    for lane in ("lamost3900", "desi7800"):
        mine = sorted((r for r in done if where[r.rid][0] == lane), key=lambda r: -r.n)[:16]
        for r in mine:
            _, off, n, _ = where[r.rid]
            shape, basis, b = banks[lane]
            a = alone(shape, basis, b, off, n)
            assert np.array_equal(a.params.cpu().numpy(), r.params.cpu().numpy()), (lane, r.rid)
            assert np.array_equal(a.status.cpu().numpy(), r.status.cpu().numpy()), (lane, r.rid)
            assert np.array_equal(a.chi2.cpu().numpy(), r.chi2.cpu().numpy()), (lane, r.rid)
    n_ok = n_chk = 0
    for r in done:
        if r.rid % 8:
            continue
        lane, off, n, _ = where[r.rid]
        shape, basis, b = banks[lane]
        err = check_oracle(shape, basis, b, off, r.params[0].cpu().numpy())
        n_chk += 1
        n_ok += int(np.all(err <= FIT_TOL))
        assert np.all(err <= FIT_TOL), (lane, r.rid, err)
    say(f"oracle parity {n_ok}/{n_chk}")


def test_stream_with_stopping_rules_releases_requests_early_and_matches_grouped_fits():
    say("[server, stopping rules] 1.0 s Poisson stream, 6k spectra/s")
    banks = bench.serving_banks(n_lamost=4096, n_desi=2048)
    stats, done, wall, where = bench.run_serving(banks, 6000.0, 1.0, seed=4, size_max=1024,
                                                 stop_window=50, stop_tol=1e-5)
    assert len(done) == len(where) and len(done) > 5
    early = [r for r in done if r.info.stopped]
    say(f"requests {len(done)}, released before 500 steps: {len(early)}")
    assert early, "no request was released by the stopping rules"
    for r in early:
        assert r.info.max_steps < 500
    for r in sorted(done, key=lambda r: -r.n)[:4]:
        lane, off, n, _ = where[r.rid]
        shape, basis, b = banks[lane]
        a = alone(shape, basis, b, off, n, stop_window=50, stop_tol=1e-5)
        assert np.array_equal(a.params.cpu().numpy(), r.params.cpu().numpy()), (lane, r.rid)
        assert np.array_equal(a.status.cpu().numpy(), r.status.cpu().numpy()), (lane, r.rid)
        err = check_oracle(shape, basis, b, off, r.params[0].cpu().numpy())
        assert np.all(err <= FIT_TOL), (lane, r.rid, err)


def pool_sizes(shape, basis):
    """(bytes per slot, bytes independent of the capacity) of a pool of this shape."""
    p = lasp.Pool(wave_grid(shape), to_dev(basis), 16, margin=shape.margin, degree=shape.degree)
    slot, fixed = p.slot_bytes, p.bytes - 16 * p.slot_bytes
    p.close()
    return slot, fixed


def _one_shape_server(budget_slots, quantum):
    shape = shape_by_name("lamost1550")
    basis, lines = make_basis(shape)
    b = make_spectra(shape, lines, 61, 0, 96)
    slot, fixed = pool_sizes(shape, basis)
    srv = Server(hbm_budget=fixed + budget_slots * slot + 64, n_steps=500, steps_per_tick=50,
                 capacity_quantum=quantum)
    sid = srv.add_shape(wave_grid(shape), to_dev(basis), margin=shape.margin,
                        degree=shape.degree)
    return shape, basis, b, srv, sid


def test_byte_budget_holds_a_request_back_and_results_do_not_change():
    say("[server] a budget of 48 slots in quanta of 16: the third request waits for bytes")
    shape, basis, b, srv, sid = _one_shape_server(budget_slots=48, quantum=16)
    # 20 + 20 spectra take the pool to 48 slots; 30 more need 80 until both finish
    reqs = []
    for off, n in ((0, 20), (20, 20), (40, 30)):
        reqs.append(srv.submit(sid, to_dev(b.obs[off:off + n]), to_dev(b.ivar[off:off + n]),
                               to_dev(b.init[off:off + n])))
    seen_wait = False
    done = []
    deadline = time.time() + 60
    try:
        while len(done) < 3:
            assert time.time() < deadline, srv.stats()
            st = srv.stats()
            assert st["hbm_in_use"] <= st["hbm_budget"]
            if st["queued"] > 0 and st["active"] > 0:
                seen_wait = True
            done += srv.poll(timeout_ms=5)
    finally:
        srv.close()
    by = {r.rid: r for r in done}
    first, second, third = (by[q.rid] for q in reqs)
    assert seen_wait, "the budget never held the third request back"
    assert third.info.t_admit >= max(first.info.t_done, second.info.t_done) - 1e-3
    for q, (off, n) in zip((first, second, third), ((0, 20), (20, 20), (40, 30))):
        a = alone(shape, basis, b, off, n)
        assert np.array_equal(a.params.cpu().numpy(), q.params.cpu().numpy()), q.rid
        assert np.array_equal(a.chi2.cpu().numpy(), q.chi2.cpu().numpy()), q.rid


def test_request_beyond_the_budget_is_refused():
    say("[server] a request larger than the whole budget is refused at submit")
    shape, basis, b, srv, sid = _one_shape_server(budget_slots=32, quantum=16)
    try:
        with pytest.raises(lasp.LaspError) as e:
            srv.submit(sid, to_dev(b.obs[:40]), to_dev(b.ivar[:40]), to_dev(b.init[:40]))
        assert e.value.code == -4
        # a request that fits still runs
        srv.submit(sid, to_dev(b.obs[:10]), to_dev(b.ivar[:10]), to_dev(b.init[:10]))
        got = []
        deadline = time.time() + 60
        while not got:
            assert time.time() < deadline, srv.stats()
            got = srv.poll(timeout_ms=20)
    finally:
        srv.close()
    a = alone(shape, basis, b, 0, 10)
    assert np.array_equal(a.params.cpu().numpy(), got[0].params.cpu().numpy())


def test_two_shapes_share_one_budget():
    say("[server] two shapes under one budget: the second shape waits for the first's bytes")
    s1, s2 = shape_by_name("lamost1550"), shape_by_name("lamost3900")
    b1, l1 = make_basis(s1)
    b2, l2 = make_basis(s2)
    x1 = make_spectra(s1, l1, 62, 0, 64)
    x2 = make_spectra(s2, l2, 63, 0, 30)
    sl1, f1 = pool_sizes(s1, b1)
    sl2, f2 = pool_sizes(s2, b2)
    # shape 1 at 64 slots and shape 2 at its first 16 fill the budget; shape 2
    # at 32 slots fits only once shape 1 has shrunk back to 16
    budget = f1 + f2 + 64 * sl1 + 16 * sl2 + 64
    assert 48 * sl1 >= 16 * sl2
    srv = Server(hbm_budget=budget, steps_per_tick=50, capacity_quantum=16)
    i1 = srv.add_shape(wave_grid(s1), to_dev(b1), margin=s1.margin, degree=s1.degree)
    i2 = srv.add_shape(wave_grid(s2), to_dev(b2), margin=s2.margin, degree=s2.degree)
    done, peak = [], 0
    deadline = time.time() + 60
    try:
        r1 = srv.submit(i1, to_dev(x1.obs), to_dev(x1.ivar), to_dev(x1.init))
        r2 = srv.submit(i2, to_dev(x2.obs), to_dev(x2.ivar), to_dev(x2.init))
        while len(done) < 2:
            assert time.time() < deadline, srv.stats()
            st = srv.stats()
            assert st["hbm_in_use"] <= st["hbm_budget"]
            peak = max(peak, st["hbm_in_use"])
            done += srv.poll(timeout_ms=5)
        st = srv.stats()
    finally:
        srv.close()
    by = {r.rid: r for r in done}
    g1, g2 = by[r1.rid], by[r2.rid]
    say(f"budget {budget}, peak {peak}, resizes {st['resizes']}, "
        f"admit2 {g2.info.t_admit:.3f} done1 {g1.info.t_done:.3f}")
    assert st["resizes"] >= 3        # grow 1, shrink 1, grow 2
    assert g2.info.t_admit >= g1.info.t_done - 1e-3, "shape 2 was admitted beyond the budget"
    a1 = alone(s1, b1, x1, 0, 64)
    a2 = alone(s2, b2, x2, 0, 30)
    assert np.array_equal(a1.params.cpu().numpy(), g1.params.cpu().numpy())
    assert np.array_equal(a2.params.cpu().numpy(), g2.params.cpu().numpy())


def test_pool_resize_keeps_resident_fits():
    say("[pool] grow and shrink a pool between steps: fits continue unchanged")
    shape = shape_by_name("lamost1550")
    basis, lines = make_basis(shape)
    b = make_spectra(shape, lines, 64, 0, 24)
    pool = lasp.Pool(wave_grid(shape), to_dev(basis), 32, margin=shape.margin, degree=shape.degree)
    before = pool.bytes
    pool.load(0, to_dev(b.obs), to_dev(b.ivar), to_dev(b.init), 500)
    pool.step(24, 100)
    pool.resize(4096, 24)
    assert pool.capacity == 4096 and pool.bytes > before
    pool.step(24, 200)
    pool.resize(24, 24)
    assert pool.capacity == 24 and pool.bytes < before
    pool.step(24, 200)
    out = torch.empty((24, 5), dtype=torch.float32, device=DEV)
    pool.finish(0, out)
    torch.cuda.synchronize()
    pool.close()
    a = alone(shape, basis, b, 0, 24)
    assert np.array_equal(a.params.cpu().numpy(), out.cpu().numpy())
