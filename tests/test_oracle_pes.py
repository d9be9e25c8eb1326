"""Pins of the oracle's potential-energy-surface evaluation (Sec. 2.1: energy
as a sum of site energies, the virial Eq., forces as the negative gradient).

Nothing here re-types the oracle's formulas: forces are checked against
central finite differences of the oracle's own total energy, the virial
against the derivative of the energy under a homogeneous strain, and both
against the symmetries that the definition implies.
"""
import numpy as np
import pytest

import oracle
import synth


def _frame(pos, spc, cell=None):
    n = len(spc)
    if cell is None:
        return synth.Frames(np.array([0, n], np.int64), np.asarray(pos, np.float64), np.asarray(spc, np.int32),
                            None, None)
    return synth.Frames(np.array([0, n], np.int64), np.asarray(pos, np.float64), np.asarray(spc, np.int32),
                        np.asarray(cell, np.float64)[None], np.ones((1, 3), np.uint8))


def _energy(m, pos, spc, cell=None):
    return oracle.eval_pes(m, _frame(pos, spc, cell))[0][0]


@pytest.fixture(scope="module")
def mol():
    fr = synth.molecules(4, seed=41)
    k = int(np.argmin(np.diff(fr.offsets)))  # the smallest molecule keeps the FD loop short
    sub = fr.subset([k])
    return sub.positions.copy(), sub.species.copy()


def test_forces_are_negative_energy_gradient_vacuum(mol):
    m = synth.model("molecule_pes")
    pos, spc = mol
    _, _, F = oracle.eval_pes(m, _frame(pos, spc))
    h = 1e-5
    fd = np.zeros_like(pos)
    for k in range(len(spc)):
        for d in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[k, d] += h
            p2[k, d] -= h
            fd[k, d] = -(_energy(m, p1, spc) - _energy(m, p2, spc)) / (2 * h)
    err = np.abs(F - fd).max() / np.abs(F).max()
    print("vacuum force vs -dU/dr FD:", err)
    assert err < 1e-7


def test_forces_are_negative_energy_gradient_periodic():
    """Periodic water box: forces of a few atoms (minimum-image pairs across
    the boundary included) against FD of the total energy."""
    m = synth.model("water_pes")
    fr = synth.water_small(1, seed=3)
    pos, spc, cell = fr.positions.copy(), fr.species.copy(), fr.cells[0]
    _, _, F = oracle.eval_pes(m, fr)
    L = cell[0]
    # atoms nearest the box faces: their neighbour lists use images
    edge = np.argsort(np.minimum(pos, L - pos).min(1))[:3]
    h = 1e-5
    for k in list(edge) + [0]:
        for d in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[k, d] += h
            p2[k, d] -= h
            fd = -(_energy(m, p1, spc, cell) - _energy(m, p2, spc, cell)) / (2 * h)
            assert abs(F[k, d] - fd) < 1e-7 * np.abs(F).max(), (k, d, F[k, d], fd)


def test_newton_third_law(mol):
    for name, fr in (("molecule_pes", _frame(*mol)), ("water_pes", synth.water_small(2, seed=4))):
        m = synth.model(name)
        _, _, F = oracle.eval_pes(m, fr)
        for f in range(fr.n_frames):
            Ff = F[fr.offsets[f]:fr.offsets[f + 1]]
            assert np.abs(Ff.sum(0)).max() < 1e-12 * np.abs(Ff).sum(), name


def test_virial_is_strain_derivative_vacuum(mol):
    """Positions r -> (I + eps) r change every pair vector the same way, so
    W^{nu ups} = -dU/d eps_{ups nu} (Sec. 2.1, Eq. virial)."""
    m = synth.model("molecule_pes")
    pos, spc = mol
    _, W, _ = oracle.eval_pes(m, _frame(pos, spc))
    h = 1e-6
    for u in range(3):
        for v in range(3):
            e = np.zeros((3, 3))
            e[u, v] = h
            up = _energy(m, pos @ (np.eye(3) + e).T, spc)
            dn = _energy(m, pos @ (np.eye(3) - e).T, spc)
            d = -(up - dn) / (2 * h)
            assert abs(W[0][v, u] - d) < 1e-7 * np.abs(W).max(), (u, v, W[0][v, u], d)


def test_virial_is_strain_derivative_periodic():
    """Diagonal strain of a periodic box: positions and box edge scale together."""
    m = synth.model("water_pes")
    fr = synth.water_small(1, seed=5)
    pos, spc, cell = fr.positions.copy(), fr.species.copy(), fr.cells[0].copy()
    _, W, _ = oracle.eval_pes(m, fr)
    h = 1e-6
    for u in range(3):
        s1, s2 = np.ones(3), np.ones(3)
        s1[u] += h
        s2[u] -= h
        c1, c2 = cell.copy(), cell.copy()
        c1[4 * u] *= 1 + h
        c2[4 * u] *= 1 - h
        d = -(_energy(m, pos * s1, spc, c1) - _energy(m, pos * s2, spc, c2)) / (2 * h)
        assert abs(W[0][u, u] - d) < 1e-7 * np.abs(W).max(), (u, W[0][u, u], d)


def test_rotation_translation_and_symmetry(mol):
    m = synth.model("molecule_pes")
    pos, spc = mol
    E, W, F = oracle.eval_pes(m, _frame(pos, spc))
    rng = np.random.default_rng(8)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    E2, W2, F2 = oracle.eval_pes(m, _frame(pos @ q.T + np.array([3.0, -1.0, 7.5]), spc))
    scale = np.abs(F).max()
    assert abs(E2[0] - E[0]) < 1e-12 * max(1.0, abs(E[0]))
    assert np.abs(F2 - F @ q.T).max() < 1e-11 * scale
    assert np.abs(W2[0] - q @ W[0] @ q.T).max() < 1e-11 * np.abs(W).max()
    # rotational invariance of U_i makes the virial symmetric
    assert np.abs(W[0] - W[0].T).max() < 1e-11 * np.abs(W).max()


def test_energy_is_sum_of_site_energies(mol):
    """The frame energy is the sum of the per-atom site energies (Sec. 2.1,
    Eq. site-energy); each site energy is unchanged when every other atom
    outside its cutoff sphere is removed."""
    m = synth.model("molecule_pes")
    pos, spc = mol
    E, _, _, U = oracle.eval_pes(m, _frame(pos, spc), per_atom=True)
    assert abs(E[0] - U.sum()) <= 1e-12 * np.abs(U).sum()
    i = 0
    keep = np.linalg.norm(pos - pos[i], axis=1) < m.rc_radial
    sub_index = int(np.nonzero(keep)[0].tolist().index(i))
    _, _, _, Us = oracle.eval_pes(m, _frame(pos[keep], spc[keep]), per_atom=True)
    assert abs(Us[sub_index] - U[i]) < 1e-13 * max(1.0, abs(U[i]))
