"""BF16x3 interpolator contractions (hi/lo split, FP32 accumulate, exact FP32
constant row): error against the FP64 oracle, reported for every output."""

import numpy as np
import pytest
import torch

import oracle
import paper_2512_24840_amd as lasp
from synth import BOX_HI, BOX_LO, make_basis, make_spectra, make_spectra_parallel, shape_by_name
from synth import wave_grid

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]
DEV = torch.device("cuda:0")
FIT_TOL = np.array([2.0, 0.005, 0.005, 0.2])


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_bf16x3_forward_errors_vs_oracle():
    print("[bf16x3 forward] lamost3900 B=7", flush=True)
    shape = shape_by_name("lamost3900")
    basis, lines = make_basis(shape)
    batch = make_spectra(shape, lines, 31, 0, 7)
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    u = (cfg.normalise(batch.init) + 0.03).astype(np.float32)
    res = lasp.forward(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis),
                       to_dev(u), want_model=True, want_grad=True, precision="bf16x3",
                       margin=shape.margin, degree=shape.degree)
    torch.cuda.synchronize()
    m_err, c_err, g_err = [], [], []
    for i in range(7):
        ref = oracle.evaluate(cfg, batch.obs[i], batch.ivar[i], basis, u[i].astype(np.float64))
        rms = np.sqrt(np.mean(ref["model"] ** 2))
        m_err.append(np.max(np.abs(res["model"][i].cpu().numpy() - ref["model"])) / rms)
        c_err.append(abs(res["chi2"][i].item() / ref["chi2"] - 1))
        g = res["grad"][i].cpu().numpy()
        g_err.append(np.linalg.norm(g - ref["grad"]) / np.linalg.norm(ref["grad"]))
    print(f"bf16x3 max errors: model {max(m_err):.2e} (rms-relative), chi2 {max(c_err):.2e}, "
          f"gradient {max(g_err):.2e}", flush=True)
    # 2^-16 per product before cancellation, on the line-depth part only
    assert max(m_err) < 5e-5 and max(c_err) < 1e-3 and max(g_err) < 1e-3


def test_bf16x3_grouped_fit_262144x3900_errors_on_sample():
    print("[bf16x3 grouped fit] 262144 distinct spectra, 500 steps, 256 sampled", flush=True)
    shape = shape_by_name("lamost3900")
    basis, lines = make_basis(shape)
    n = 262144
    batch = make_spectra_parallel(shape, lines, 3, 0, n)
    res = lasp.fit_group(to_dev(batch.obs), to_dev(batch.ivar), wave_grid(shape), to_dev(basis),
                         to_dev(batch.init), 500, precision="bf16x3", margin=shape.margin,
                         degree=shape.degree)
    torch.cuda.synchronize()
    params = res.params.cpu().numpy().astype(np.float64)
    chi2 = res.chi2.cpu().numpy()
    assert np.isfinite(params).all()
    # 256 fits spread over the whole launch, the last spectrum included
    idx = np.unique(np.append(np.arange(0, n, n // 255), n - 1))
    cfg = oracle.Config.from_shape(shape, BOX_LO, BOX_HI)
    ref = oracle.fit_many(cfg, batch.obs[idx], batch.ivar[idx], basis, batch.init[idx])
    refp = np.array([r["params"] for r in ref])
    refc = np.array([r["chi2"] for r in ref])
    err = np.abs(params[idx] - refp)
    cerr = np.abs(chi2[idx] / refc - 1)
    names = ("Teff K", "logg", "[Fe/H]", "RV km/s", "sigma km/s")
    for k, nm in enumerate(names):
        print(f"  {nm:10s} max {err[:, k].max():.3e}  median {np.median(err[:, k]):.3e}  "
              f"p99 {np.percentile(err[:, k], 99):.3e}", flush=True)
    print(f"  chi2 rel   max {cerr.max():.3e}  median {np.median(cerr):.3e}", flush=True)
    assert np.all(err[:, :4] <= FIT_TOL), err.max(axis=0)
