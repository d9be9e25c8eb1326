"""Dipole of charged molecules (mu_r + Q e r_COM) on the GPU against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu

MASSES = [12.011, 1.008, 14.007, 15.999, 18.998]  # C, H, N, O, F
BOHR = 0.529177210903


def test_charged_molecules(gpu_lib):
    import torch

    ctx = gpu_lib.Context(0)
    m = synth.model("molecule_dipole")
    g = gpu_lib.Model(ctx, m)
    fr = synth.molecules(64, seed=61)
    # molecules far from the origin make the centre-of-mass term dominant
    fr = synth.Frames(fr.offsets, fr.positions + np.array([20.0, -35.0, 50.0]), fr.species, None, None)
    q = np.random.default_rng(62).integers(-2, 3, fr.n_frames).astype(np.float64)
    mu = gpu_lib.tnep_eval_dipole_charged(ctx, g, fr, q, MASSES, 1.0 / BOHR)
    ref = oracle.dipole_charged(m, fr, q, MASSES, 1.0 / BOHR)
    err = frame_errors(mu, ref)
    print("charged dipole error", err.max(), flush=True)
    assert np.all(err <= TENSOR_TOL)
    # neutral frames are the plain dipole, bit for bit
    neutral = q == 0
    plain = gpu_lib.tnep_eval_dipole(ctx, g, fr)
    assert np.array_equal(mu[neutral], plain[neutral])
    # device-resident frames and charges
    dfr = gpu_lib.DeviceFrames(fr)
    dmu = torch.zeros((fr.n_frames, 3), dtype=torch.float64, device="cuda")
    gpu_lib.tnep_eval_dipole_charged(ctx, g, dfr, torch.as_tensor(q).cuda(), MASSES, 1.0 / BOHR, mu_out=dmu)
    torch.cuda.synchronize()
    assert np.array_equal(dmu.cpu().numpy(), mu)
    ctx.close()


def test_charged_periodic_frame_is_an_error(gpu_lib):
    ctx = gpu_lib.Context(0)
    m = synth.model("water_dipole_small")
    g = gpu_lib.Model(ctx, m)
    fr = synth.water_small(2)
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_eval_dipole_charged(ctx, g, fr, np.array([0.0, 1.0]), [15.999, 1.008])
    assert e.value.code == -3
    mu = gpu_lib.tnep_eval_dipole_charged(ctx, g, fr, np.zeros(2), [15.999, 1.008])
    assert np.array_equal(mu, gpu_lib.tnep_eval_dipole(ctx, g, fr))
    ctx.close()
