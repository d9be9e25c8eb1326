"""Models with the five-body descriptor term on the GPU against the FP64 oracle.

Bounds as for the other models (tests/parity.py): per-frame relative
Frobenius error <= 1e-5 for mu and alpha; for the potential-energy model
|dE| <= 1e-5 sum_i |U_i|, virial and forces 1e-5 relative per frame.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _cell_list_box():
    pos, spc, cell = synth.water_box(8, 24.84, seed=91)
    return synth.Frames(np.array([0, len(spc)], np.int64), pos, spc, cell[None], np.ones((1, 3), np.uint8))


@pytest.mark.parametrize("name", ["water_dipole_5b", "water_polarizability_5b"])
def test_tensors_small_and_cell_list(gpu_lib, ctx, name):
    m = synth.model(name)
    mdl = gpu_lib.Model(ctx, m)
    f = gpu_lib.tnep_eval_dipole if m.kind == synth.KIND_DIPOLE else gpu_lib.tnep_eval_polarizability
    for label, fr in (("192 atoms x 4", synth.water_small(4, seed=92)), ("1536-atom box", _cell_list_box())):
        nt = 3 if m.kind == synth.KIND_DIPOLE else 9
        pa = np.zeros((fr.n_atoms, nt))
        out = f(ctx, mdl, fr, per_atom=pa)
        ref, ref_pa = oracle.eval_frames(m, fr, per_atom=True)
        err = frame_errors(out, ref, ref_pa, fr.offsets)
        pa_err = np.linalg.norm(pa - ref_pa.reshape(fr.n_atoms, nt)) / np.linalg.norm(ref_pa)
        print(f"{name} {label}: frame {err.max():.2e}, per-atom {pa_err:.2e}", flush=True)
        assert np.all(err <= TENSOR_TOL) and pa_err <= TENSOR_TOL


def test_five_body_changes_the_result(gpu_lib, ctx):
    """The same weights on the first D - 5 inputs with the five-body inputs
    dropped give a different tensor (the term is really evaluated)."""
    m = synth.model("water_dipole_5b")
    d = m.dim - (m.n_max_angular + 1)
    m4 = synth.Model(m.kind, m.species, m.rc_radial, m.rc_angular, m.n_max_radial, m.n_max_angular,
                     m.basis_radial, m.basis_angular, m.l_max, m.four_body, m.n_hidden, m.c_radial, m.c_angular,
                     m.q_scaler[:d], [synth.Head(h.w0[:, :d], h.b0, h.w1, h.b1) for h in m.heads])
    fr = synth.water_small(2, seed=93)
    a = gpu_lib.tnep_eval_dipole(ctx, gpu_lib.Model(ctx, m), fr)
    b = gpu_lib.tnep_eval_dipole(ctx, gpu_lib.Model(ctx, m4), fr)
    rb = oracle.eval_frames(m4, fr)
    assert np.all(frame_errors(b, rb) <= TENSOR_TOL)
    assert frame_errors(a, b).min() > 1e-3


def test_potential_energy_surface(gpu_lib, ctx):
    m = synth.model("water_pes_5b")
    mdl = gpu_lib.Model(ctx, m)
    fr = synth.water_small(3, seed=94)
    E, W, F = gpu_lib.tnep_eval_pes(ctx, mdl, fr)
    Er, Wr, Fr, Ur = oracle.eval_pes(m, fr, per_atom=True)
    off = fr.offsets
    for f in range(fr.n_frames):
        assert abs(E[f] - Er[f]) <= TENSOR_TOL * np.abs(Ur[off[f]:off[f + 1]]).sum()
        Ff, Fref = F[off[f]:off[f + 1]], Fr[off[f]:off[f + 1]]
        assert np.linalg.norm(Ff - Fref) <= TENSOR_TOL * np.linalg.norm(Fref)
    assert np.all(frame_errors(W, Wr) <= TENSOR_TOL)


def test_population_loss_with_five_body(gpu_lib, ctx):
    base = synth.model("water_dipole_5b")
    fr = synth.water_small(2, seed=95)
    ref = oracle.eval_frames(base, fr) + 0.05
    z0 = synth.pack_params(base)
    zs = z0[None, :] * (1.0 + 0.01 * np.random.default_rng(96).normal(size=(3, z0.size)))
    loss, rmse = gpu_lib.tnep_population_loss(ctx, base, zs, fr, ref, 0.01, 0.01)
    loss_r, rmse_r = oracle.population_loss(base, zs, fr, ref, 0.01, 0.01)
    scale = np.sqrt((oracle.eval_frames(base, fr) ** 2).mean())
    assert np.all(np.abs(rmse - rmse_r) <= TENSOR_TOL * scale)
    assert np.all(np.abs((loss - rmse) - (loss_r - rmse_r)) <= 1e-12 * np.abs(loss_r - rmse_r))


def test_per_species_five_body(gpu_lib, ctx):
    """Per-species networks on a five-body descriptor."""
    a = synth.model("water_polarizability_5b")
    seed, kind, species, desc = synth.MODEL_SPECS["water_polarizability_5b"]
    b = synth.with_descriptor_of(synth.make_model(seed + 50, kind, species, **desc), a)
    m = synth.per_species_model([a, b], [1, 0])
    fr = synth.water_small(2, seed=97)
    out = gpu_lib.tnep_eval_polarizability(ctx, gpu_lib.Model(ctx, m), fr)
    ref, pa = oracle.eval_frames(m, fr, per_atom=True)
    err = frame_errors(out, ref, pa, fr.offsets)
    print("per-species five-body", err.max(), flush=True)
    assert np.all(err <= TENSOR_TOL)
