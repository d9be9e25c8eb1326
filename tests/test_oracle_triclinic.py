"""Pins of the oracle's triclinic cells: the same lattice described by
another basis (a unimodular transform of the cell rows) gives the same
results, a rigid rotation of positions and cell rotates the tensors, and the
neighbour sets match the orthorhombic description."""
import numpy as np
import pytest

import oracle
import synth


def _box(seed=3):
    pos, spc, cell = synth.water_box(8, 24.84, seed=seed)
    return pos, spc, cell


def _frame(pos, spc, cell):
    return synth.Frames(np.array([0, len(spc)], np.int64), pos, spc, np.asarray(cell, np.float64).reshape(1, 9),
                        np.ones((1, 3), np.uint8))


SHEAR = np.array([[1, 0, 0], [1, 1, 0], [0, 1, 1]], np.float64)  # rows a, a + b, b + c (det 1)


def test_same_lattice_other_basis():
    pos, spc, cell = _box()
    H = cell.reshape(3, 3)
    tri = (SHEAR @ H).reshape(9)
    for name in ("water_dipole_small", "water_polarizability"):
        m = synth.model(name)
        a = oracle.eval_frames(m, _frame(pos, spc, cell))
        b = oracle.eval_frames(m, _frame(pos, spc, tri))
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max(), name
    m = synth.model("water_pes")
    Ea, Wa, Fa = oracle.eval_pes(m, _frame(pos, spc, cell))
    Eb, Wb, Fb = oracle.eval_pes(m, _frame(pos, spc, tri))
    assert abs(Ea[0] - Eb[0]) <= 1e-12 * abs(Ea[0]) and np.abs(Fa - Fb).max() <= 1e-12 * np.abs(Fa).max()


def test_rotation_of_positions_and_cell():
    pos, spc, cell = _box(4)
    R, _ = np.linalg.qr(np.random.default_rng(9).normal(size=(3, 3)))
    H = cell.reshape(3, 3)
    m = synth.model("water_polarizability")
    a = oracle.eval_frames(m, _frame(pos, spc, cell))[0]
    b = oracle.eval_frames(m, _frame(pos @ R.T, spc, (H @ R.T).reshape(9)))[0]
    assert np.abs(b - R @ a @ R.T).max() <= 1e-11 * np.abs(a).max()
    md = synth.model("water_dipole_small")
    mu = oracle.eval_frames(md, _frame(pos, spc, cell))[0]
    mu_r = oracle.eval_frames(md, _frame(pos @ R.T, spc, (H @ R.T).reshape(9)))[0]
    assert np.abs(mu_r - R @ mu).max() <= 1e-11 * np.abs(mu).max()


def test_neighbour_sets_and_thin_cells():
    pos, spc, cell = _box(5)
    H = cell.reshape(3, 3)
    tri = (SHEAR @ H).reshape(9)
    a = oracle.neighbors(pos, cell, np.ones(3, np.uint8), 6.0)
    b = oracle.neighbors(pos, tri, np.ones(3, np.uint8), 6.0)
    assert len(a) == len(b) and all(np.array_equal(x, y) for x, y in zip(a, b))
    # a cell whose narrowest width is below 2 r_c is rejected
    thin = (np.array([[1, 0, 0], [2, 1, 0], [0, 0, 1]], np.float64) @ H).reshape(9)
    with pytest.raises(oracle.OracleError):
        oracle.eval_frames(synth.model("water_dipole_small"), _frame(pos, spc, thin))
