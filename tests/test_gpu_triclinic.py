"""Triclinic cells on the GPU against the oracle (which enumerates periodic
images itself)."""
import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu

SHEAR = np.array([[1, 0, 0], [1, 1, 0], [0, 1, 1]], np.float64)  # same lattice, other basis


def _frames(pos_list, spc, cells):
    n = len(spc)
    return synth.Frames(np.arange(len(pos_list) + 1, dtype=np.int64) * n, np.concatenate(pos_list),
                        np.tile(spc, len(pos_list)).astype(np.int32), np.asarray(cells, np.float64).reshape(-1, 9),
                        np.ones((len(pos_list), 3), np.uint8))


def _check(gpu, m, fr, label):
    ref, pa = oracle.eval_frames(m, fr, per_atom=True)
    err = frame_errors(gpu, ref, pa, fr.offsets)
    print(label, err.max(), flush=True)
    assert np.all(err <= TENSOR_TOL), label
    return ref


def test_sheared_and_rotated_boxes(gpu_lib):
    pos, spc, cell = synth.water_box(8, 24.84, seed=91)
    H = cell.reshape(3, 3)
    R, _ = np.linalg.qr(np.random.default_rng(92).normal(size=(3, 3)))
    ortho = _frames([pos], spc, [H])
    tri = _frames([pos, pos @ R.T], spc, [SHEAR @ H, H @ R.T])
    ctx = gpu_lib.Context(0)
    for name in ("water_dipole_small", "water_polarizability"):
        m = synth.model(name)
        g = gpu_lib.Model(ctx, m)
        f = gpu_lib.tnep_eval_dipole if m.kind == 1 else gpu_lib.tnep_eval_polarizability
        out = np.asarray(f(ctx, g, tri)).reshape(2, -1)
        _check(out, m, tri, name + " triclinic")
        # the sheared basis describes the same lattice: plain orthorhombic result up to summation order
        plain = np.asarray(f(ctx, g, ortho)).reshape(1, -1)
        assert frame_errors(out[:1], plain).max() <= 5e-6
    ctx.close()


def test_skewed_basis_of_orthorhombic_lattice_is_reduced(gpu_lib):
    """A skewed basis of a cubic lattice is reduced to the cubic one before the
    search (integer row operations keep the lattice): bitwise the result of
    the cubic description, for several skews."""
    pos, spc, cell = synth.water_box(8, 24.84, seed=95)
    H = cell.reshape(3, 3)
    skews = [SHEAR, np.array([[1, 0, 0], [0, 1, 0], [-1, 1, 1]], np.float64),
             np.array([[0, 1, 0], [1, 0, 1], [0, 0, -1]], np.float64)]
    ctx = gpu_lib.Context(0)
    g = gpu_lib.Model(ctx, synth.model("water_polarizability"))
    plain = gpu_lib.tnep_eval_polarizability(ctx, g, _frames([pos], spc, [H]))
    for U in skews:
        out = gpu_lib.tnep_eval_polarizability(ctx, g, _frames([pos], spc, [U @ H]))
        assert np.array_equal(out, plain), U
    ctx.close()


def test_small_sheared_box_all_pairs_and_pes(gpu_lib):
    """A 12.42 A water box with a 0.2 L shear: widths just above 2 r_c, fewer
    than three bins per axis, so the frame is searched all-pairs."""
    fr0 = synth.water_small(2, seed=93)
    L = 12.42
    cell = np.array([[L, 0, 0], [0.2 * L, L, 0], [0, 0, L]])
    fr = synth.Frames(fr0.offsets, fr0.positions, fr0.species, np.tile(cell.reshape(9), (2, 1)), fr0.pbc)
    ctx = gpu_lib.Context(0)
    m = synth.model("water_dipole_small")
    _check(gpu_lib.tnep_eval_dipole(ctx, gpu_lib.Model(ctx, m), fr), m, fr, "small sheared dipole")
    mp = synth.model("water_pes")
    E, W, F = gpu_lib.tnep_eval_pes(ctx, gpu_lib.Model(ctx, mp), fr)
    Er, Wr, Fr, Ur = oracle.eval_pes(mp, fr, per_atom=True)
    for k in range(2):
        sl = slice(fr.offsets[k], fr.offsets[k + 1])
        assert abs(E[k] - Er[k]) <= TENSOR_TOL * np.abs(Ur[sl]).sum()
        assert np.linalg.norm(F[sl] - Fr[sl]) <= TENSOR_TOL * np.linalg.norm(Fr[sl])
    assert np.all(frame_errors(W, Wr) <= TENSOR_TOL)
    ctx.close()


def test_triclinic_errors(gpu_lib):
    pos, spc, cell = synth.water_box(8, 24.84, seed=94)
    H = cell.reshape(3, 3)
    ctx = gpu_lib.Context(0)
    g = gpu_lib.Model(ctx, synth.model("water_dipole_small"))
    thin = _frames([pos], spc, [np.array([[1, 0, 0], [2, 1, 0], [0, 0, 1]], np.float64) @ H])
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_eval_dipole(ctx, g, thin)
    assert e.value.code == -3
    half = _frames([pos], spc, [SHEAR @ H])
    half.pbc[:] = [1, 1, 0]
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_eval_dipole(ctx, g, half)
    assert e.value.code == -3
    ctx.close()
