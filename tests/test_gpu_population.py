"""Population loss (Sec. 2.4) on the GPU against the FP64 oracle.

Bound: every frame tensor meets the per-frame bound of tests/parity.py,
||T_gpu,f - T_ref,f|| <= 1e-5 d_f (d_f = max(||T_ref,f||, 1e-3 sum_i ||T_i||)),
so by the triangle inequality on the RMS
  |RMSE_gpu - RMSE_ref| <= RMS(T_gpu - T_ref) <= 1e-5 sqrt(sum_f d_f^2 / (F nt)).
The regularization terms are FP64 sums of the same parameters: 1e-12 relative.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _population(base, n, seed, scale=0.02):
    z0 = synth.pack_params(base)
    rng = np.random.default_rng(seed)
    return z0[None, :] * (1.0 + scale * rng.normal(size=(n, z0.size))) + 0.1 * scale * rng.normal(size=(n, z0.size))


def _rmse_bound(base, zs, fr):
    """1e-5 * sqrt(sum_f d_f^2 / (F nt)) for each individual."""
    out = []
    for z in zs:
        T, pa = oracle.eval_frames(synth.unpack_params(base, z), fr, per_atom=True)
        T = T.reshape(fr.n_frames, -1)
        pn = np.linalg.norm(pa.reshape(fr.n_atoms, -1), axis=1)
        d = np.array([max(np.linalg.norm(T[f]), 1e-3 * pn[fr.offsets[f]:fr.offsets[f + 1]].sum())
                      for f in range(fr.n_frames)])
        out.append(TENSOR_TOL * np.sqrt((d ** 2).sum() / T.size))
    return np.array(out)


def _check(gpu_lib, ctx, base, zs, fr, ref, l1, l2, label):
    loss, rmse = gpu_lib.tnep_population_loss(ctx, base, zs, fr, ref, l1, l2)
    loss_r, rmse_r = oracle.population_loss(base, zs, fr, ref, l1, l2)
    bound = _rmse_bound(base, zs, fr)
    reg_r = loss_r - rmse_r
    reg = loss - rmse
    print(f"{label}: rmse err {np.abs(rmse - rmse_r).max():.2e} (bound {bound.min():.2e}),"
          f" reg err {np.abs(reg - reg_r).max():.2e}", flush=True)
    assert np.all(np.abs(rmse - rmse_r) <= bound), label
    assert np.all(np.abs(reg - reg_r) <= 1e-12 * np.maximum(np.abs(reg_r), 1e-300)), label
    assert np.all(np.abs(loss - loss_r) <= bound + 1e-12 * np.abs(reg_r)), label
    return loss, rmse


@pytest.mark.parametrize("name", ["water_dipole_small", "water_polarizability"])
def test_water(gpu_lib, ctx, name):
    base = synth.model(name)
    fr = synth.water_small(3, seed=21)
    truth = synth.unpack_params(base, _population(base, 1, 22, 0.05)[0])
    ref = oracle.eval_frames(truth, fr).reshape(fr.n_frames, -1)
    zs = _population(base, 6, 23)
    _check(gpu_lib, ctx, base, zs, fr, ref, 0.05, 0.1, name)


def test_molecules_two_jobs(gpu_lib, ctx):
    """70 individuals: more than one job of models sharing a neighbour build."""
    base = synth.model("molecule_dipole")
    fr = synth.molecules(12, seed=24)
    ref = oracle.eval_frames(base, fr).reshape(fr.n_frames, -1) + 0.01
    zs = _population(base, 70, 25)
    zs[0] = synth.pack_params(base)
    loss, rmse = _check(gpu_lib, ctx, base, zs, fr, ref, 0.0, 0.02, "molecules x70")
    # the unperturbed individual is off by the constant 0.01 only
    assert abs(rmse[0] - 0.01) <= 1e-5 * np.sqrt((ref ** 2).mean())
    # the same individuals in another order give the same results
    perm = np.random.default_rng(26).permutation(len(zs))
    loss2, rmse2 = gpu_lib.tnep_population_loss(ctx, base, zs[perm], fr, ref, 0.0, 0.02)
    assert np.array_equal(loss2, loss[perm]) and np.array_equal(rmse2, rmse[perm])


def test_device_frames(gpu_lib, ctx):
    import torch

    base = synth.model("molecule_polarizability")
    fr = synth.molecules(10, seed=27)
    ref = oracle.eval_frames(base, fr).reshape(fr.n_frames, -1) * 1.01
    zs = _population(base, 4, 28)
    loss, rmse = _check(gpu_lib, ctx, base, zs, fr, ref, 0.01, 0.0, "molecules pol (host)")
    dfr = gpu_lib.DeviceFrames(fr)
    dl, dr = gpu_lib.tnep_population_loss(ctx, base, zs, dfr, torch.as_tensor(ref).cuda(), 0.01, 0.0)
    assert np.array_equal(dl, loss) and np.array_equal(dr, rmse)


def test_errors(gpu_lib, ctx):
    base = synth.model("water_dipole_small")
    fr = synth.water_small(1)
    ref = np.zeros((1, 3))
    zs = _population(base, 2, 29)
    with pytest.raises(gpu_lib.TnepError):
        gpu_lib.tnep_population_loss(ctx, base, zs, fr, ref, -1.0, 0.0)
    with pytest.raises(gpu_lib.TnepError):
        gpu_lib.tnep_population_loss(ctx, base, zs[:0], fr, ref)
    with pytest.raises(gpu_lib.TnepError):
        gpu_lib.tnep_population_loss(ctx, synth.model("water_pes"), zs, fr, ref)
    with pytest.raises(gpu_lib.TnepError):
        per = synth.per_species_model([base, synth.model("water_dipole")], [0, 1])
        gpu_lib.tnep_population_loss(ctx, per, zs, fr, ref)
