"""lasp_forward_noalloc (the fixed-scratch forward evaluation) against
lasp_forward, through the C ABI.

Both run the same kernels on the same inputs, and no kernel of the forward
evaluation reduces with floating-point atomics, so every output must agree
bit for bit.  Each test makes two calls in a row on the shared array, the
second with a smaller input, so that what the first call left in the array
cannot reach the second call's results.
"""

import sys

import numpy as np
import pytest
import torch

import paper_2512_24840_amd as lasp
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, shape_by_name, wave_grid

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
OUTS = ("model", "chi2", "J", "n_eff", "grad", "jac", "cov", "status")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def arms_of(shape):
    return lasp.Arms(shape.arm_start, shape.arm_sigma_kms) if shape.arm_start else None


def inputs(name, n, seed, **over):
    shape = shape_by_name(name, **over)
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, 41, 0, n)
    lo, hi = np.array(BOX_LO), np.array(BOX_HI)
    theta = batch.init.astype(np.float64).copy()
    theta[:, 0] = np.log10(theta[:, 0])
    u = 2.0 * (theta - lo) / (hi - lo) - 1.0
    u += np.random.default_rng(seed).normal(0.0, 0.03, u.shape)
    return shape, to_dev(basis), to_dev(batch.obs), to_dev(batch.ivar), to_dev(u.astype(np.float32))


def both(shape, basis, obs, ivar, u, **want):
    kw = dict(margin=shape.margin, degree=shape.degree, arms=arms_of(shape), **want)
    ref = lasp.forward(obs, ivar, wave_grid(shape), basis, u, **kw)
    got = lasp.forward(obs, ivar, wave_grid(shape), basis, u, noalloc=True, **kw)
    torch.cuda.synchronize()
    return ref, got


def assert_same(ref, got, tag):
    for k in OUTS:
        if ref[k] is None:
            assert got[k] is None, (tag, k)
            continue
        a, b = ref[k].cpu().numpy(), got[k].cpu().numpy()
        assert np.all(np.isfinite(a) | ~np.isfinite(b)), (tag, k)
        assert np.array_equal(a, b, equal_nan=True), \
            (tag, k, float(np.nanmax(np.abs(a.astype(np.float64) - b.astype(np.float64)))))


CASES = [
    # (shape, overrides, first B, second B, outputs)
    ("lamost3900", {}, 900, 130, dict(want_model=True, want_grad=True)),
    ("lamost3900", {}, 480, 57, dict(want_model=True, want_grad=True, want_jac=True,
                                     want_cov=True)),
    ("desi7800", {}, 200, 33, dict(want_model=True, want_grad=True, want_cov=True)),
    ("lamost1550", {}, 700, 9, dict(want_grad=True)),
]


@pytest.mark.parametrize("name,over,b1,b2,want", CASES)
def test_noalloc_matches_forward_twice(name, over, b1, b2, want):
    for call, n in enumerate((b1, b2)):
        say(f"[noalloc] shape={name} call={call} B={n} {sorted(want)}")
        shape, basis, obs, ivar, u = inputs(name, n, seed=call, **over)
        ref, got = both(shape, basis, obs, ivar, u, **want)
        assert_same(ref, got, (name, call, n))


def test_noalloc_bf16x3_matches_forward():
    for call, n in enumerate((300, 21)):
        say(f"[noalloc] shape=lamost3900 bf16x3 call={call} B={n}")
        shape, basis, obs, ivar, u = inputs("lamost3900", n, seed=7 + call)
        ref, got = both(shape, basis, obs, ivar, u, want_model=True, want_grad=True,
                        precision="bf16x3")
        assert_same(ref, got, ("bf16x3", call, n))


def test_noalloc_rejects_more_than_its_array():
    say("[noalloc] oversized request is refused before any work")
    shape, basis, obs, ivar, u = inputs("lamost3900", 1200, seed=3)
    with pytest.raises(lasp.LaspError) as e:
        lasp.forward(obs, ivar, wave_grid(shape), basis, u, want_grad=True,
                     margin=shape.margin, degree=shape.degree, noalloc=True)
    assert e.value.code == -4 and "scratch" in str(e.value)
    # a call that fits still works after the refusal
    shape, basis, obs, ivar, u = inputs("lamost3900", 64, seed=4)
    ref, got = both(shape, basis, obs, ivar, u, want_model=True, want_grad=True)
    assert_same(ref, got, ("after refusal", 64))
