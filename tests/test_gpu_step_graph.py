"""The Adam steps of lasp_fit_group replayed from the cached HIP graph of
25 steps (opts.step_graph, the default) against the same steps launched one
kernel at a time: the same kernels with the same arguments, so every output
must agree bit for bit -- over chunk counts with and without a remainder,
replays of one graph across calls with other work between them, argument
changes that need a new graph, BF16x3, a side stream, and against the
FP64 oracle."""

import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2512_24840_amd as lasp
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name, wave_grid

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
DEV = torch.device("cuda:0")
FIT_TOL = np.array([2.0, 0.005, 0.005, 0.2])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def prob():
    shape = shape_by_name("lamost1550")
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, 47, 0, 9)
    return shape, to_dev(basis), batch, dict(obs=to_dev(batch.obs), ivar=to_dev(batch.ivar),
                                             init=to_dev(batch.init))


def fit(prob, n_steps, graph, sl=slice(None), want_cov=True, **kw):
    shape, basis, _, d = prob
    r = lasp.fit_group(d["obs"][sl].contiguous(), d["ivar"][sl].contiguous(), wave_grid(shape),
                       basis, d["init"][sl].contiguous(), n_steps, margin=shape.margin,
                       degree=shape.degree, want_cov=want_cov, step_graph=graph, **kw)
    torch.cuda.current_stream().synchronize()
    return {k: getattr(r, k).cpu().numpy() for k in ("params", "status", "chi2", "steps", "cov")
            if getattr(r, k) is not None}


def same(a, b, tag):
    for k in a:
        assert np.array_equal(a[k], b[k]), (tag, k)


@pytest.mark.parametrize("n_steps", [0, 24, 25, 26, 60, 500])
def test_graph_replays_equal_kernel_by_kernel_launches(prob, n_steps):
    say(f"[step graph] lamost1550 B=9, {n_steps} steps: graph vs one launch per kernel")
    same(fit(prob, n_steps, True), fit(prob, n_steps, False), n_steps)


def test_graph_kept_across_calls_and_rebuilt_when_arguments_change(prob):
    say("[step graph] replays across calls with other work between; new B, lr, precision")
    ref = fit(prob, 75, False)
    x = torch.ones(1 << 20, device=DEV)
    for rep in range(3):
        same(fit(prob, 75, True), ref, ("replay", rep))
        x.mul_(1.5).add_(1.0)               # unrelated work on the same stream
        torch.cuda.synchronize()
    same(fit(prob, 50, True, slice(0, 5)), fit(prob, 50, False, slice(0, 5)), "B=5")
    same(fit(prob, 75, True), ref, "back to B=9")
    same(fit(prob, 50, True, lr=3e-3), fit(prob, 50, False, lr=3e-3), "lr")
    same(fit(prob, 50, True, precision="bf16x3"), fit(prob, 50, False, precision="bf16x3"),
         "bf16x3")
    same(fit(prob, 75, True), ref, "back to the first arguments")


def test_graph_on_a_side_stream(prob):
    say("[step graph] on a side stream")
    ref = fit(prob, 60, False)
    s = torch.cuda.Stream(device=DEV)
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        got = fit(prob, 60, True)
    same(got, ref, "side stream")


def test_graph_fit_matches_oracle_lm(prob):
    say("[step graph] 500 graph-replayed steps vs the oracle's LM fits")
    shape, _, batch, _ = prob
    got = fit(prob, 500, True, want_cov=False)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    ref = oracle.fit_many(cfg, batch.obs, batch.ivar, make_basis(shape)[0], batch.init)
    for i in range(batch.obs.shape[0]):
        err = np.abs(got["params"][i].astype(np.float64) - ref[i]["params"])[:4]
        assert np.all(err <= FIT_TOL), (i, err)


def test_kernel_timing_launches_every_step(prob):
    say("[step graph] kernel timing on: every step launched (and timed) on its own")
    ref = fit(prob, 60, False)
    lasp.profile_enable(["fused"])
    try:
        got = fit(prob, 60, True)
        n = lasp.profile_read()["fused"][1]
    finally:
        lasp.profile_enable([])
    assert n == 60, n
    same(got, ref, "timed")
