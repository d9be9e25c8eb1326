"""Pins of the optional five-body descriptor term (one degree-4 invariant of
the l = 1 angular sums per radial function n, appended after the four-body
block): q5_n equals the square of the three-body l = 1 invariant q_n1 of the
same atom (a wrong l block, a missing square or a wrong index fails), it is
unchanged by proper and improper rotations, and it is (g_n(r)^2 3 / (4 pi))^2
for a single neighbour (the l = 1 addition theorem); its backward passes the
same finite-difference checks as the rest of the descriptor.
"""
import numpy as np
import pytest

import oracle
import synth

RNG = np.random.default_rng(505)


def model5(kind=synth.KIND_DIPOLE, four_body=True, seed=11):
    desc = dict(synth.WATER_DESCRIPTOR, four_body=four_body, five_body=True)
    return synth.make_model(seed, kind, synth.WATER_SPECIES, **desc)


def blocks(m, q):
    nr, na = m.n_max_radial + 1, m.n_max_angular + 1
    q1 = q[nr:nr + na]
    q5 = q[m.dim - na:]
    return q1, q5


def _rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


@pytest.mark.parametrize("four_body", [True, False])
def test_square_of_l1_invariant_and_layout(four_body):
    m = model5(four_body=four_body)
    assert m.dim == 5 + 4 * 5 + (5 if four_body else 0) + 5
    vecs = RNG.standard_normal((13, 3)) * 1.5
    tj = RNG.integers(0, 2, 13)
    q = oracle.atom_eval(m, 0, 0, vecs, tj, forces=False)["q"]
    q1, q5 = blocks(m, q)
    np.testing.assert_allclose(q5, q1 ** 2, rtol=1e-13, atol=0)
    # the other blocks are those of the same model without the term
    m3 = synth.Model(m.kind, m.species, m.rc_radial, m.rc_angular, m.n_max_radial, m.n_max_angular,
                     m.basis_radial, m.basis_angular, m.l_max, m.four_body, m.n_hidden, m.c_radial, m.c_angular,
                     m.q_scaler[:m.dim - 5], [synth.Head(h.w0[:, :m.dim - 5], h.b0, h.w1, h.b1) for h in m.heads])
    q3 = oracle.atom_eval(m3, 0, 0, vecs, tj, forces=False)["q"]
    np.testing.assert_array_equal(q[:m.dim - 5], q3)


def test_rotation_and_inversion_invariant():
    m = model5()
    vecs = RNG.standard_normal((11, 3)) * 1.4
    tj = RNG.integers(0, 2, 11)
    q0 = oracle.atom_eval(m, 0, 1, vecs, tj, forces=False)["q"]
    for _ in range(3):
        R = _rotation(RNG)
        q1 = oracle.atom_eval(m, 0, 1, vecs @ R.T, tj, forces=False)["q"]
        np.testing.assert_allclose(q1, q0, rtol=1e-11, atol=1e-16)
    np.testing.assert_allclose(oracle.atom_eval(m, 0, 1, -vecs, tj, forces=False)["q"], q0, rtol=1e-11, atol=1e-16)


def test_single_neighbour_closed_form():
    m = model5()
    r = 2.3
    v = np.array([[0.3, -0.8, 0.52]])
    v *= r / np.linalg.norm(v)
    q = oracle.atom_eval(m, 0, 0, v, [1], forces=False)["q"]
    # g_n(r) = sum_k c_nk f_k(r) with f_k = (T_k(x) + 1) / 2 f_c, x = 2 (r/rc - 1)^2 - 1
    rc = m.rc_angular
    fc = 0.5 * (1.0 + np.cos(np.pi * r / rc))
    x = 2.0 * (r / rc - 1.0) ** 2 - 1.0
    f = (np.cos(np.arange(m.basis_angular + 1) * np.arccos(x)) + 1.0) / 2.0 * fc
    g = m.c_angular[0, 1] @ f
    _, q5 = blocks(m, q)
    np.testing.assert_allclose(q5, (g ** 2 * 3.0 / (4.0 * np.pi)) ** 2, rtol=1e-12, atol=0)


@pytest.mark.parametrize("head,kind", [(0, synth.KIND_DIPOLE), (1, synth.KIND_POLARIZABILITY),
                                       (0, synth.KIND_PES)])
def test_partial_force_fd(head, kind):
    m = model5(kind=kind)
    n = 12
    vecs = RNG.standard_normal((n, 3))
    vecs *= (RNG.uniform(0.9, 3.9, n) / np.linalg.norm(vecs, axis=1))[:, None]
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


def test_dUdq_of_five_body_block_fd():
    """dU/dq (five-body entries included) predicts the change of U under
    small random moves of the neighbours: dU = dU/dq . dq."""
    m = model5()
    vecs = RNG.standard_normal((10, 3)) * 1.7
    tj = RNG.integers(0, 2, 10)
    base = oracle.atom_eval(m, 0, 1, vecs, tj, forces=False)
    h = 1e-6
    for _ in range(4):
        dv = RNG.standard_normal(vecs.shape)
        p = oracle.atom_eval(m, 0, 1, vecs + h * dv, tj, forces=False)
        mm = oracle.atom_eval(m, 0, 1, vecs - h * dv, tj, forces=False)
        assert p["U"] - mm["U"] == pytest.approx(base["dUdq"] @ (p["q"] - mm["q"]), rel=1e-7, abs=1e-13)
