"""The GPU's own loss sequence of a fixed-step fit, for checking the
stopping rules (Section 2.2, stage 8) in the kernels' arithmetic.

A pool holds the spectra T + 1 times: slot block t has a limit of t Adam
steps.  After T pool steps every block is evaluated at its returned point,
so block t gives chi2 and the parameters after exactly t steps of the same
fit (a fit's arithmetic does not depend on its slot)."""

import numpy as np
import torch

import paper_2512_24840_amd as lasp
from synth import wave_grid


def gpu_losses(shape, basis, obs, ivar, init, u0, T):
    """ell [T + 1, n] = sqrt(chi2 / n_eff) after t = 0 .. T steps, the
    returned parameters [T + 1, n, 5] and n_eff [n], for device tensors
    obs, ivar [n, P], init (physical) and u0 (normalised) [n, 5]."""
    n, dev = obs.shape[0], obs.device
    pool = lasp.Pool(wave_grid(shape), basis, n * (T + 1), margin=shape.margin,
                     degree=shape.degree)
    with torch.cuda.stream(pool.stream):
        for t in range(T + 1):
            pool.load(n * t, obs, ivar, init, t)
        pool.step(n * (T + 1), T)
        out = torch.empty((n * (T + 1), 5), dtype=torch.float32, device=dev)
        chi2 = torch.empty(n * (T + 1), dtype=torch.float64, device=dev)
        pool.finish(0, out, chi2=chi2)
    pool.stream.synchronize()
    pool.close()
    n_eff = lasp.forward(obs, ivar, wave_grid(shape), basis, u0, margin=shape.margin,
                         degree=shape.degree)["n_eff"]
    torch.cuda.synchronize()
    n_eff = n_eff.cpu().numpy()
    ell = np.sqrt(chi2.cpu().numpy().reshape(T + 1, n) / n_eff)
    return ell, out.cpu().numpy().reshape(T + 1, n, 5), n_eff
