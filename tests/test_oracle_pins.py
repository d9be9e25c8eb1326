"""Pins of the FP64 oracle to facts fixed outside itself: closed forms,
library routines, invariants and finite differences.

Nothing here re-types an oracle formula: every expected value comes from
textbook identities (Chebyshev, Legendre addition theorem, Wigner 3j
tables via sympy), scipy/numpy routines, symmetry, or derivatives taken
numerically from the oracle's own forward values.
"""
import numpy as np
import pytest
import scipy.fft
from scipy.special import eval_legendre

import oracle
import synth

RNG = np.random.default_rng(12345)


def small_model(kind=synth.KIND_DIPOLE, species=synth.WATER_SPECIES, seed=7, four_body=True, **over):
    desc = dict(synth.WATER_DESCRIPTOR)
    desc["four_body"] = four_body
    desc.update(over)
    return synth.make_model(seed, kind, species, **desc)


def rand_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


# ---------------------------------------------------------------------------
# Cutoff and Chebyshev basis


def test_cutoff_closed_form():
    rc = 5.0
    fc, dfc = oracle.cutoff(0.0, rc)
    assert fc == pytest.approx(1.0, abs=1e-15) and dfc == pytest.approx(0.0, abs=1e-15)
    fc, dfc = oracle.cutoff(rc / 2, rc)
    assert fc == pytest.approx(0.5, abs=1e-15)
    # C^1 at the cutoff: value and slope go to zero from below
    fc, dfc = oracle.cutoff(rc * (1 - 1e-9), rc)
    assert abs(fc) < 1e-15 and abs(dfc) < 1e-8
    assert oracle.cutoff(rc, rc) == (0.0, 0.0)
    assert oracle.cutoff(rc + 1, rc) == (0.0, 0.0)


def test_chebyshev_is_cos_k_theta():
    rc, K = 6.0, 8
    for r in np.linspace(0.05, 5.95, 23):
        f, _ = oracle.basis(r, rc, K)
        fc, _ = oracle.cutoff(r, rc)
        x = 2.0 * (r / rc - 1.0) ** 2 - 1.0
        theta = np.arccos(np.clip(x, -1, 1))
        tk = 2.0 * f / fc - 1.0  # f_k = (T_k + 1)/2 f_c
        np.testing.assert_allclose(tk, np.cos(np.arange(K + 1) * theta), atol=1e-12)


def test_basis_derivative_fd():
    rc, K, h = 4.0, 8, 1e-6
    for r in np.linspace(0.3, 3.9, 13):
        _, df = oracle.basis(r, rc, K)
        fp, _ = oracle.basis(r + h, rc, K)
        fm, _ = oracle.basis(r - h, rc, K)
        np.testing.assert_allclose(df, (fp - fm) / (2 * h), atol=1e-8)


def test_basis_vanishes_beyond_cutoff():
    f, df = oracle.basis(6.0, 6.0, 8)
    assert np.all(f == 0) and np.all(df == 0)


# ---------------------------------------------------------------------------
# Spherical harmonics


def test_ylm_explicit_low_orders():
    v = np.array([0.3, -1.2, 0.7])
    x, y, z = v / np.linalg.norm(v)
    assert oracle.ylm(1, 0, v)[0] == pytest.approx(np.sqrt(3 / (4 * np.pi)) * z, abs=1e-14)
    assert oracle.ylm(1, 1, v)[0] == pytest.approx(np.sqrt(3 / (4 * np.pi)) * x, abs=1e-14)
    assert oracle.ylm(1, -1, v)[0] == pytest.approx(np.sqrt(3 / (4 * np.pi)) * y, abs=1e-14)
    assert oracle.ylm(2, 0, v)[0] == pytest.approx(0.25 * np.sqrt(5 / np.pi) * (3 * z * z - 1), abs=1e-14)
    assert oracle.ylm(2, -2, v)[0] == pytest.approx(0.5 * np.sqrt(15 / np.pi) * x * y, abs=1e-14)


def test_ylm_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) (6 nodes) x uniform phi (12 nodes) is exact
    # for the degree <= 8 products of l <= 4 harmonics.
    ct, wt = np.polynomial.legendre.leggauss(6)
    phis = np.arange(12) * 2 * np.pi / 12
    pts, wts = [], []
    for c, w in zip(ct, wt):
        s = np.sqrt(1 - c * c)
        for p in phis:
            pts.append([s * np.cos(p), s * np.sin(p), c])
            wts.append(w * 2 * np.pi / 12)
    lm = [(l, m) for l in range(0, 5) for m in range(-l, l + 1)]
    Y = np.array([[oracle.ylm(l, m, p)[0] for p in pts] for (l, m) in lm])
    G = (Y * np.array(wts)[None, :]) @ Y.T
    np.testing.assert_allclose(G, np.eye(len(lm)), atol=1e-13)


def test_ylm_addition_theorem():
    for _ in range(20):
        a = RNG.standard_normal(3)
        b = RNG.standard_normal(3)
        cosg = a @ b / np.linalg.norm(a) / np.linalg.norm(b)
        for l in range(1, 5):
            s = sum(oracle.ylm(l, m, a)[0] * oracle.ylm(l, m, b)[0] for m in range(-l, l + 1))
            assert s == pytest.approx((2 * l + 1) / (4 * np.pi) * eval_legendre(l, cosg), abs=1e-13)


def test_ylm_gradient_fd_and_homogeneity():
    h = 1e-6
    for _ in range(10):
        v = RNG.standard_normal(3) * 2
        for l in range(1, 5):
            for m in range(-l, l + 1):
                y, g = oracle.ylm(l, m, v)
                fd = np.array([(oracle.ylm(l, m, v + h * e)[0] - oracle.ylm(l, m, v - h * e)[0]) / (2 * h)
                               for e in np.eye(3)])
                np.testing.assert_allclose(g, fd, atol=1e-8)
                assert abs(g @ v) < 1e-12  # degree-0 homogeneous => radial derivative zero
                assert oracle.ylm(l, m, 3.7 * v)[0] == pytest.approx(y, abs=1e-14)


# ---------------------------------------------------------------------------
# 3j symbols and the 4-body invariant


def test_wigner3j_against_sympy():
    from sympy.physics.wigner import wigner_3j

    assert oracle.wigner3j(2, 2, 2, 0, 0, 0) == pytest.approx(-np.sqrt(2 / 35), abs=1e-15)
    for j1 in range(0, 4):
        for j2 in range(0, 4):
            for j3 in range(abs(j1 - j2), min(j1 + j2, 4) + 1):
                for m1 in range(-j1, j1 + 1):
                    for m2 in range(-j2, j2 + 1):
                        m3 = -m1 - m2
                        if abs(m3) > j3:
                            continue
                        ref = float(wigner_3j(j1, j2, j3, m1, m2, m3))
                        assert oracle.wigner3j(j1, j2, j3, m1, m2, m3) == pytest.approx(ref, abs=1e-14)


def test_four_body_real_and_derivative():
    h = 1e-6
    for _ in range(10):
        A = RNG.standard_normal(5)
        q, d, im = oracle.four_body(A)
        assert abs(im) < 1e-14
        fd = np.array([(oracle.four_body(A + h * e)[0] - oracle.four_body(A - h * e)[0]) / (2 * h) for e in np.eye(5)])
        np.testing.assert_allclose(d, fd, atol=1e-8)


def _single_neighbor_g(m, r, t_i, t_j, which):
    """g_n(r) from numpy's Chebyshev evaluation and the cutoff closed form."""
    if which == "R":
        rc, K, c = m.rc_radial, m.basis_radial, m.c_radial[t_i, t_j]
    else:
        rc, K, c = m.rc_angular, m.basis_angular, m.c_angular[t_i, t_j]
    x = 2 * (r / rc - 1) ** 2 - 1
    fc = 0.5 * (1 + np.cos(np.pi * r / rc))
    fk = np.array([0.5 * (np.polynomial.chebyshev.chebval(x, np.eye(K + 1)[k]) + 1) * fc for k in range(K + 1)])
    return c @ fk


def test_single_neighbor_descriptor_closed_form():
    m = small_model()
    r = 2.7
    for ti, tj in [(0, 0), (0, 1), (1, 0), (1, 1)]:
        res = oracle.atom_eval(m, 0, ti, [[0.0, 0.0, r]], [tj], forces=False)
        q = res["q"]
        gR = _single_neighbor_g(m, r, ti, tj, "R")
        gA = _single_neighbor_g(m, r, ti, tj, "A")
        nR, nA = m.n_max_radial + 1, m.n_max_angular + 1
        np.testing.assert_allclose(q[:nR], gR, atol=1e-14)
        for l in range(1, 5):
            np.testing.assert_allclose(q[nR + (l - 1) * nA: nR + l * nA], (2 * l + 1) / (4 * np.pi) * gA ** 2,
                                       atol=1e-14)
        # 4-body, neighbour along z: (2 2 2; 0 0 0) (5/4pi)^{3/2} g^3
        expect4 = -np.sqrt(2 / 35) * (5 / (4 * np.pi)) ** 1.5 * gA ** 3
        np.testing.assert_allclose(q[nR + 4 * nA:], expect4, atol=1e-14)


def test_three_body_brute_force_legendre():
    m = small_model()
    nR, nA = m.n_max_radial + 1, m.n_max_angular + 1
    for trial in range(3):
        n = 8
        vecs = RNG.standard_normal((n, 3))
        vecs *= (RNG.uniform(1.0, 3.9, n) / np.linalg.norm(vecs, axis=1))[:, None]
        tj = RNG.integers(0, 2, n)
        q = oracle.atom_eval(m, 0, 1, vecs, tj, forces=False)["q"]
        g = np.array([_single_neighbor_g(m, np.linalg.norm(v), 1, t, "A") for v, t in zip(vecs, tj)])  # [n, nA]
        u = vecs / np.linalg.norm(vecs, axis=1)[:, None]
        cos = np.clip(u @ u.T, -1, 1)
        for l in range(1, 5):
            P = eval_legendre(l, cos)
            brute = (2 * l + 1) / (4 * np.pi) * np.einsum("jn,kn,jk->n", g, g, P)
            np.testing.assert_allclose(q[nR + (l - 1) * nA: nR + l * nA], brute, rtol=1e-12, atol=1e-15)


def test_descriptor_rotation_invariant():
    m = small_model()
    vecs = RNG.standard_normal((12, 3)) * 1.6
    tj = RNG.integers(0, 2, 12)
    q0 = oracle.atom_eval(m, 0, 0, vecs, tj, forces=False)["q"]
    for _ in range(3):
        R = rand_rotation(RNG)
        q1 = oracle.atom_eval(m, 0, 0, vecs @ R.T, tj, forces=False)["q"]
        np.testing.assert_allclose(q1, q0, rtol=1e-11, atol=1e-14)
    # improper rotation (inversion) also leaves every invariant unchanged
    q2 = oracle.atom_eval(m, 0, 0, -vecs, tj, forces=False)["q"]
    np.testing.assert_allclose(q2, q0, rtol=1e-11, atol=1e-14)


# ---------------------------------------------------------------------------
# Network backward and partial forces


def test_dUdq_directional_fd():
    m = small_model()
    vecs = RNG.standard_normal((15, 3)) * 1.8
    tj = RNG.integers(0, 2, 15)
    base = oracle.atom_eval(m, 0, 1, vecs, tj, forces=False)
    h = 1e-6
    for _ in range(5):
        dv = RNG.standard_normal(vecs.shape)
        p = oracle.atom_eval(m, 0, 1, vecs + h * dv, tj, forces=False)
        mm = oracle.atom_eval(m, 0, 1, vecs - h * dv, tj, forces=False)
        dU = p["U"] - mm["U"]
        dq = p["q"] - mm["q"]
        assert dU == pytest.approx(base["dUdq"] @ dq, rel=1e-7, abs=1e-13)


@pytest.mark.parametrize("head,kind", [(0, synth.KIND_DIPOLE), (0, synth.KIND_POLARIZABILITY),
                                       (1, synth.KIND_POLARIZABILITY)])
def test_partial_force_fd(head, kind):
    m = small_model(kind=kind)
    n = 14
    vecs = RNG.standard_normal((n, 3))
    vecs *= (RNG.uniform(0.9, 5.9, n) / np.linalg.norm(vecs, axis=1))[:, None]
    tj = RNG.integers(0, 2, n)
    F = oracle.atom_eval(m, head, 0, vecs, tj)["dUdr"]
    h = 1e-5
    for j in range(n):
        for d in range(3):
            vp = vecs.copy()
            vp[j, d] += h
            vm = vecs.copy()
            vm[j, d] -= h
            fd = (oracle.atom_eval(m, head, 0, vp, tj, forces=False)["U"] -
                  oracle.atom_eval(m, head, 0, vm, tj, forces=False)["U"]) / (2 * h)
            assert F[j, d] == pytest.approx(fd, rel=1e-6, abs=1e-10)


# ---------------------------------------------------------------------------
# Whole-frame tensors


def _frame_pairs(m, fr, f=0):
    a0, a1 = int(fr.offsets[f]), int(fr.offsets[f + 1])
    pos = fr.positions[a0:a1]
    spc = fr.species[a0:a1]
    cell = None if fr.cells is None else fr.cells[f]
    pbc = None if fr.pbc is None else fr.pbc[f]
    nb = oracle.neighbors(pos, cell, pbc, m.rc_radial)
    box = np.zeros(3) if cell is None else np.array([cell[0], cell[4], cell[8]])
    per = np.zeros(3, bool) if pbc is None else np.asarray(pbc, bool)
    out = []
    for i in range(a1 - a0):
        v = pos[nb[i]] - pos[i]
        v[:, per] -= box[per] * np.round(v[:, per] / box[per])
        out.append((int(spc[i]), v, spc[nb[i]]))
    return out


def _total_U(m, head, pairs, deform):
    om = oracle.OracleModel(m)
    return sum(oracle.atom_eval(om, head, ti, deform(v), tj, forces=False)["U"] for ti, v, tj in pairs)


def test_dipole_equals_deformation_derivative():
    """mu^nu = -d/de sum_i U_i({r_ij + e r_ij^2 e_nu}) at e = 0 (forward values only)."""
    m = small_model(species=synth.MOLECULE_SPECIES)
    fr = synth.molecules(1, seed=11)
    pairs = _frame_pairs(m, fr)
    mu = oracle.eval_frames(m, fr)[0]
    h = 1e-6
    for nu in range(3):
        e = np.eye(3)[nu]
        up = _total_U(m, 0, pairs, lambda v: v + h * (v * v).sum(1)[:, None] * e[None])
        dn = _total_U(m, 0, pairs, lambda v: v - h * (v * v).sum(1)[:, None] * e[None])
        assert mu[nu] == pytest.approx(-(up - dn) / (2 * h), rel=1e-6, abs=1e-9)


def test_polarizability_equals_strain_derivative():
    """alpha = sum_i U^s_i I + W, W^{uv} = -d/de sum_i U^t_i({r_ij + e r_ij^u e_v})."""
    m = small_model(kind=synth.KIND_POLARIZABILITY, species=synth.MOLECULE_SPECIES)
    fr = synth.molecules(1, seed=12)
    pairs = _frame_pairs(m, fr)
    al = oracle.eval_frames(m, fr)[0]
    us = _total_U(m, 1, pairs, lambda v: v)
    h = 1e-6
    for u in range(3):
        for w in range(3):
            e = np.eye(3)[w]
            up = _total_U(m, 0, pairs, lambda v: v + h * v[:, u:u + 1] * e[None])
            dn = _total_U(m, 0, pairs, lambda v: v - h * v[:, u:u + 1] * e[None])
            expect = -(up - dn) / (2 * h) + (us if u == w else 0.0)
            assert al[u, w] == pytest.approx(expect, rel=1e-6, abs=1e-9)


def test_dimer_closed_form():
    """A-B dimer at distance r along e: mu = -r^2 (U_A'(r) - U_B'(r)) e,
    alpha = (U^s_A + U^s_B) I - r (U^t_A'(r) + U^t_B'(r)) e e^T, U' by 1-D FD."""
    md = small_model(kind=synth.KIND_DIPOLE, seed=21)
    mp = small_model(kind=synth.KIND_POLARIZABILITY, seed=22)
    e = np.array([0.36, -0.48, 0.8])
    r = 2.3
    fr = synth.Frames(np.array([0, 2], np.int64), np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0] + r * e]),
                      np.array([0, 1], np.int32))

    def U(m, head, t_self, t_other, dist):
        return oracle.atom_eval(m, head, t_self, [[0, 0, dist]], [t_other], forces=False)["U"]

    h = 1e-6

    def dU(m, head, a, b):
        return (U(m, head, a, b, r + h) - U(m, head, a, b, r - h)) / (2 * h)

    mu = oracle.eval_frames(md, fr)[0]
    np.testing.assert_allclose(mu, -r * r * (dU(md, 0, 0, 1) - dU(md, 0, 1, 0)) * e, rtol=1e-7, atol=1e-12)
    al = oracle.eval_frames(mp, fr)[0]
    expect = (U(mp, 1, 0, 1, r) + U(mp, 1, 1, 0, r)) * np.eye(3) - r * (dU(mp, 0, 0, 1) + dU(mp, 0, 1, 0)) * np.outer(e, e)
    np.testing.assert_allclose(al, expect, rtol=1e-7, atol=1e-12)
    # homonuclear dimer: no dipole
    fr.species[:] = 1
    np.testing.assert_allclose(oracle.eval_frames(md, fr)[0], 0.0, atol=1e-15)


def test_rotation_translation_permutation_vacuum():
    md = small_model(kind=synth.KIND_DIPOLE, species=synth.MOLECULE_SPECIES, seed=31)
    mp = small_model(kind=synth.KIND_POLARIZABILITY, species=synth.MOLECULE_SPECIES, seed=32)
    fr = synth.molecules(2, seed=13)
    mu0 = oracle.eval_frames(md, fr)
    al0 = oracle.eval_frames(mp, fr)
    R = rand_rotation(RNG)
    if np.linalg.det(R) > 0:
        R = -R  # include an improper rotation: mu -> R mu still (polar vector of the construction)
    fr2 = synth.Frames(fr.offsets, fr.positions @ R.T + np.array([3.0, -7.0, 11.0]), fr.species)
    mu1 = oracle.eval_frames(md, fr2)
    al1 = oracle.eval_frames(mp, fr2)
    np.testing.assert_allclose(mu1, mu0 @ R.T, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(al1, np.einsum("ab,fbc,dc->fad", R, al0, R), rtol=1e-10, atol=1e-12)
    # same-species permutation within each frame
    perm = []
    for f in range(fr.n_frames):
        idx = np.arange(fr.offsets[f], fr.offsets[f + 1])
        perm.append(RNG.permutation(idx))
    perm = np.concatenate(perm)
    fr3 = synth.Frames(fr.offsets, fr.positions[perm], fr.species[perm])
    np.testing.assert_allclose(oracle.eval_frames(md, fr3), mu0, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(oracle.eval_frames(mp, fr3), al0, rtol=1e-11, atol=1e-13)


def test_periodic_cubic_symmetry_and_translation():
    md = synth.model_raw("water_dipole_small")
    fr = synth.water_small(1, seed=5)
    L = fr.cells[0][0]
    mu0 = oracle.eval_frames(md, fr)[0]
    # 90 degree rotation about z followed by wrapping into the box
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    p = np.mod(fr.positions @ R.T, L)
    fr2 = synth.Frames(fr.offsets, p, fr.species, fr.cells, fr.pbc)
    np.testing.assert_allclose(oracle.eval_frames(md, fr2)[0], R @ mu0, rtol=1e-10, atol=1e-12)
    # translation through the periodic boundary
    fr3 = synth.Frames(fr.offsets, np.mod(fr.positions + np.array([5.1, -2.2, 9.9]), L), fr.species, fr.cells, fr.pbc)
    np.testing.assert_allclose(oracle.eval_frames(md, fr3)[0], mu0, rtol=1e-10, atol=1e-12)


def test_alpha_symmetric_per_atom():
    mp = synth.model_raw("water_polarizability")
    fr = synth.water_small(1, seed=6)
    al, pa = oracle.eval_frames(mp, fr, per_atom=True)
    np.testing.assert_allclose(pa, np.transpose(pa, (0, 2, 1)), atol=1e-12)
    np.testing.assert_allclose(al[0], pa.sum(0), rtol=1e-12, atol=1e-12)


def test_centrosymmetric_cubic_perovskite():
    """Ideal cubic ABO3: every site is an inversion centre, so mu = 0 (atom by
    atom); O_h symmetry makes alpha = a I while O sites alone are anisotropic."""
    desc = dict(synth.PEROVSKITE_DESCRIPTOR)
    md = synth.make_model(41, synth.KIND_DIPOLE, synth.PEROVSKITE_SPECIES, **desc)
    mp = synth.make_model(42, synth.KIND_POLARIZABILITY, synth.PEROVSKITE_SPECIES, **desc)
    fr = synth.perovskite(1, n_rep=4, sigma=0.0)
    hot = synth.perovskite(1, n_rep=4, sigma=0.08)
    scale = np.abs(oracle.eval_frames(md, hot, per_atom=True)[1]).sum()
    assert scale > 1e-3
    mu, mua = oracle.eval_frames(md, fr, per_atom=True)
    np.testing.assert_allclose(mua, 0.0, atol=1e-13 * scale)
    al, ala = oracle.eval_frames(mp, fr, per_atom=True)
    al = al[0]
    np.testing.assert_allclose(al - np.eye(3) * al[0, 0], 0.0, atol=1e-10 * abs(al[0, 0]))
    o_site = ala[2]  # an O atom: tetragonal (D4h) site, anisotropic
    assert abs(o_site[0, 0] - o_site[2, 2]) > 1e-6 * abs(o_site).max()


def test_neighbors_vs_numpy_all_pairs():
    fr = synth.water_small(1, seed=3)
    pos = fr.positions
    L = fr.cells[0][0]
    nb = oracle.neighbors(pos, fr.cells[0], fr.pbc[0], 6.0)
    d = pos[None, :, :] - pos[:, None, :]
    d -= L * np.round(d / L)
    r = np.linalg.norm(d, axis=2)
    for i in range(len(pos)):
        expect = np.nonzero((r[i] < 6.0) & (np.arange(len(pos)) != i))[0]
        np.testing.assert_array_equal(nb[i], expect)


def test_error_codes():
    m = synth.model_raw("water_dipole_small")
    fr = synth.water_small(1)
    small = synth.Frames(fr.offsets, fr.positions, fr.species, fr.cells * 0.9, fr.pbc)  # 11.2 A < 2 rc
    with pytest.raises(oracle.OracleError) as e:
        oracle.eval_frames(m, small)
    assert e.value.code == -3
    bad = synth.Frames(fr.offsets, fr.positions, fr.species.copy(), fr.cells, fr.pbc)
    bad.species[5] = 7
    with pytest.raises(oracle.OracleError) as e:
        oracle.eval_frames(m, bad)
    assert e.value.code == -2
    ov = synth.Frames(fr.offsets, fr.positions.copy(), fr.species, fr.cells, fr.pbc)
    ov.positions[4] = ov.positions[3]
    with pytest.raises(oracle.OracleError) as e:
        oracle.eval_frames(m, ov)
    assert e.value.code == -4


# ---------------------------------------------------------------------------
# Spectrum step


def test_acf_direct_vs_fft_routine():
    x = RNG.standard_normal(700)
    M = 300
    c = oracle.acf_direct(x, M)
    P = 2048
    X = np.fft.rfft(x, P)
    circ = np.fft.irfft(np.abs(X) ** 2, P)[:M]
    np.testing.assert_allclose(c, circ / (700 - np.arange(M)), rtol=1e-11, atol=1e-13)


def test_acf_sinusoid_closed_form():
    A, theta, n, M = 1.7, 0.21, 1000, 400
    x = A * np.cos(theta * np.arange(n))
    c = oracle.acf_direct(x, M)
    tau = np.arange(M)
    L = n - tau
    expect = A * A / 2 * (np.cos(theta * tau) + np.sin(L * theta) * np.cos(theta * (L - 1 + tau)) / (L * np.sin(theta)))
    np.testing.assert_allclose(c, expect, rtol=1e-12, atol=1e-12)


def test_spectrum_is_dct1_of_windowed_acf():
    """On the grid w_k = pi k / (M dt) the one-sided cosine sum is a type-I DCT."""
    s = RNG.standard_normal((600, 3))
    M, dt = 200, 0.5
    freq, S, C_ = oracle.spectrum([s], oracle.SPEC_IR, dt, M, omega2=False)
    w = 0.5 * (1 + np.cos(np.pi * np.arange(M) / M))
    y = scipy.fft.dct(np.append(w * C_, 0.0), type=1)
    np.testing.assert_allclose(S * 2 * np.pi / dt, y, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(freq[1], 1 / (2 * M * dt * oracle.SPEED_OF_LIGHT_CM_PER_FS), rtol=1e-15)


@pytest.mark.parametrize("kind", [oracle.SPEC_RAMAN_ISO, oracle.SPEC_RAMAN_ANISO, oracle.SPEC_RAMAN_PROJ])
def test_raman_peak_at_drive_frequency(kind):
    """alpha(t) = alpha0 + B cos(w0 t): the spectrum peaks at w0 (+- one bin)."""
    dt, n, M = 1.0, 4000, 1000
    k0 = 137
    w0 = np.pi * k0 / (M * dt)
    a0 = np.diag([3.0, 2.0, 2.5]).reshape(9)
    x = synth.sinusoid_series(n, w0 * dt, offset=a0, seed=8)
    x = (x.reshape(-1, 3, 3) + x.reshape(-1, 3, 3).transpose(0, 2, 1)).reshape(-1, 9) / 2
    freq, S, _ = oracle.spectrum([x], kind, dt, M, subtract_mean=True, n_hat=[1, 0, 0], e_hat=[0, 1, 0])
    assert abs(int(np.argmax(S)) - k0) <= 1


def test_ir_omega_squared_and_average():
    dt, n, M = 1.0, 2000, 500
    s1 = RNG.standard_normal((n, 3))
    s2 = RNG.standard_normal((n, 3))
    f, Sa, _ = oracle.spectrum([s1, s2], oracle.SPEC_IR, dt, M)
    _, S1, _ = oracle.spectrum([s1], oracle.SPEC_IR, dt, M)
    _, S2, _ = oracle.spectrum([s2], oracle.SPEC_IR, dt, M)
    np.testing.assert_allclose(Sa, (S1 + S2) / 2, rtol=1e-12, atol=1e-15)
    _, Sn, _ = oracle.spectrum([s1], oracle.SPEC_IR, dt, M, omega2=False)
    omega = np.pi * np.arange(M + 1) / (M * dt)
    np.testing.assert_allclose(S1, Sn * omega ** 2, rtol=1e-14, atol=1e-300)
