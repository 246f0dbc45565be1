"""Adjoint behind torch.autograd.Function, Adam step, covariance at given u."""

import numpy as np
import pytest
import torch

import oracle
import paper_2512_24840_amd as lasp
from paper_2512_24840_amd.autograd import covariance, objective
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, make_spectra_parallel, shape_by_name
from synth import wave_grid

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
DEV = torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def setup(name="lamost3900", n=6, cid=44):
    shape = shape_by_name(name)
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, cid, 0, n)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    return shape, cfg, basis, batch


def test_autograd_gradient_matches_fp64_central_differences():
    print("[autograd] lamost3900 B=6 vs oracle FP64 central FD (h=1e-4)", flush=True)
    shape, cfg, basis, batch = setup()
    rng = np.random.default_rng(7)
    u32 = (cfg.normalise(batch.init) + rng.normal(0, 0.04, (6, 5))).astype(np.float32)
    u = to_dev(u32).requires_grad_(True)
    J = objective(u, to_dev(batch.obs), to_dev(batch.ivar), to_dev(basis), wave_grid(shape),
                  margin=shape.margin, degree=shape.degree)
    J.sum().backward()
    g = u.grad.cpu().numpy()
    Jc = J.detach().cpu().numpy()
    h = 1e-4
    for i in range(6):
        u0 = u32[i].astype(np.float64)
        ev = oracle.evaluate(cfg, batch.obs[i], batch.ivar[i], basis, u0)
        assert Jc[i] == pytest.approx(ev["J"], rel=1e-5)
        fd = np.empty(5)
        for t in range(5):
            e = np.zeros(5)
            e[t] = h
            fd[t] = (oracle.evaluate(cfg, batch.obs[i], batch.ivar[i], basis, u0 + e)["J"]
                     - oracle.evaluate(cfg, batch.obs[i], batch.ivar[i], basis, u0 - e)["J"]) / (2 * h)
        # FD of the profiled objective: O(h^2) truncation plus window-size jumps
        # are absent at these points (checked by the analytic gradient too)
        assert np.linalg.norm(g[i] - fd) <= 1e-3 * np.linalg.norm(fd), (i, g[i], fd)
        assert np.linalg.norm(g[i] - ev["grad"]) <= 1e-5 * np.linalg.norm(ev["grad"])


def test_autograd_gradient_matches_fp32_central_differences_on_gpu():
    print("[autograd] GPU FP32 central FD (h=1e-4) of the GPU objective", flush=True)
    shape, cfg, basis, batch = setup(n=4, cid=45)
    u32 = (cfg.normalise(batch.init) + 0.05).astype(np.float32)
    args = (to_dev(batch.obs), to_dev(batch.ivar), to_dev(basis), wave_grid(shape))
    kw = dict(margin=shape.margin, degree=shape.degree)
    u = to_dev(u32).requires_grad_(True)
    objective(u, *args, **kw).sum().backward()
    g = u.grad.cpu().numpy()
    h = 1e-4
    fd = np.empty((4, 5))
    for t in range(5):
        e = np.zeros((4, 5), np.float32)
        e[:, t] = h
        jp = objective(to_dev(u32 + e), *args, **kw).double().cpu().numpy()
        jn = objective(to_dev(u32 - e), *args, **kw).double().cpu().numpy()
        # the float32 u +- h is what the GPU evaluated
        step = ((u32 + e) - (u32 - e)).astype(np.float64)[:, t]
        fd[:, t] = (jp - jn) / step
    for i in range(4):
        assert np.linalg.norm(g[i] - fd[i]) <= 2e-2 * np.linalg.norm(fd[i]), (i, g[i], fd[i])


def test_adam_matches_torch_optim_adam_fed_the_same_gradients():
    print("[adam] 12 steps vs torch.optim.Adam (float64, CPU)", flush=True)
    shape, cfg, basis, batch = setup("lamost1550", 3, 46)
    args = (to_dev(batch.obs), to_dev(batch.ivar), to_dev(basis), wave_grid(shape))
    kw = dict(margin=shape.margin, degree=shape.degree)
    n = 12
    fit = lasp.fit_group(args[0], args[1], args[3], args[2], to_dev(batch.init), n, **kw)
    u_gpu = cfg.normalise(fit.params.cpu().numpy().astype(np.float64))
    # the library's own float32 start
    u_ref = torch.tensor(cfg.normalise(batch.init.astype(np.float64)).astype(np.float32),
                         dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([u_ref], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(n):
        res = lasp.forward(args[0], args[1], args[3], args[2],
                           to_dev(u_ref.detach().numpy().astype(np.float32)), want_grad=True, **kw)
        opt.zero_grad()
        u_ref.grad = res["grad"].cpu().double()
        opt.step()
    np.testing.assert_allclose(u_gpu, u_ref.detach().numpy(), atol=2e-5)


def test_covariance_at_given_u_matches_oracle():
    print("[covariance] lasp_forward(want_cov) vs oracle at a perturbed point", flush=True)
    shape, cfg, basis, batch = setup(n=5, cid=47)
    u32 = (cfg.normalise(batch.truth) + 0.01).astype(np.float32)
    cov = covariance(to_dev(u32), to_dev(batch.obs), to_dev(batch.ivar), to_dev(basis),
                     wave_grid(shape), margin=shape.margin, degree=shape.degree).cpu().numpy()
    for i in range(5):
        ref = oracle.covariance(cfg, batch.obs[i], batch.ivar[i], basis,
                                u32[i].astype(np.float64))["cov"]
        assert np.linalg.norm(cov[i] - ref) <= 1e-3 * np.linalg.norm(ref), i


def test_adjoint_and_covariance_65536x3900_on_sample():
    print("[adjoint + covariance] 65536 x 3900: gradient + covariance at fixed u, 64 sampled", flush=True)
    shape = shape_by_name("lamost3900")
    basis, lines = make_basis(shape)
    B = 65536
    batch = make_spectra_parallel(shape, lines, 4, 0, B)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    u32 = (cfg.normalise(batch.init)).astype(np.float32)
    res = lasp.forward(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis),
                       to_dev(u32), want_grad=True, want_cov=True, margin=shape.margin,
                       degree=shape.degree)
    torch.cuda.synchronize()
    g = res["grad"].cpu().numpy()
    cov = res["cov"].cpu().numpy()
    assert np.isfinite(g).all() and np.isfinite(cov).all()
    for i in np.arange(0, B, B // 64):
        ev = oracle.evaluate(cfg, batch.obs[i], batch.ivar[i], basis, u32[i].astype(np.float64))
        assert np.linalg.norm(g[i] - ev["grad"]) <= 1e-5 * np.linalg.norm(ev["grad"]), i
        ref = oracle.covariance(cfg, batch.obs[i], batch.ivar[i], basis,
                                u32[i].astype(np.float64))["cov"]
        assert np.linalg.norm(cov[i] - ref) <= 1e-3 * np.linalg.norm(ref), i
