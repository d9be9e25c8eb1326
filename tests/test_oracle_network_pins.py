"""Pins of the oracle's network forward (Sec. 2.1, Eq. site-energy: one tanh
hidden layer on the scaled descriptor) with a hidden width H different from
the descriptor length D, so that a transposed W0, a mis-applied scaler, a
wrong bias sign or a swapped polarizability head changes a value that is
known without the oracle.

Every expected value is a special case of the definition that reduces to
numpy's tanh and the single-neighbour descriptor closed form:
  * W0 = 0: U = sum_m w1_m tanh(-b0_m) - b1 for any neighbourhood, dU/dq = 0;
  * W0 with one non-zero entry w at (row m*, column v*) and one neighbour:
    U = sum_{m != m*} w1_m tanh(-b0_m) + w1_m* tanh(w s_v* q_v* - b0_m*) - b1,
    q_v* from numpy's Chebyshev evaluation, the addition theorem
    ((2l+1)/4pi g^2) and the 3j value (2 2 2; 0 0 0) = -sqrt(2/35);
  * an A-B dimer with such networks: U'(r) from the analytic derivative of
    the same closed forms (numpy's chebder), mu = -r^2 (U_A' - U_B') e and
    alpha = (U^s_A + U^s_B) I - r (U^t_A' + U^t_B') e e^T (Sec. 2.2 Eq. mu,
    Sec. 2.3 Eq. polarizability-model) with the scalar and tensor heads given
    different one-hot networks.
"""
import numpy as np
import pytest

import oracle
import synth

RNG = np.random.default_rng(2024)
H = 7  # hidden width, != D = 30


def model_h7(kind, seed=41, species=synth.WATER_SPECIES):
    m = synth.make_model(seed, kind, species, **dict(synth.WATER_DESCRIPTOR, n_hidden=H))
    # a non-uniform descriptor scaler, so that a missing or doubled scaler shows
    m.q_scaler = RNG.uniform(0.5, 3.0, m.dim)
    return m


def one_hot(m, head, row, col, w):
    h = m.heads[head]
    h.w0 = np.zeros_like(h.w0)
    h.w0[row, col] = w


def blocks(m):
    """Descriptor index -> (block, n): block 'R', 1..4 (angular l) or '4b'."""
    nR, nA = m.n_max_radial + 1, m.n_max_angular + 1
    out = [("R", n) for n in range(nR)]
    for l in range(1, 5):
        out += [(l, n) for n in range(nA)]
    out += [("4b", n) for n in range(nA)]
    return out


def g_closed(m, r, ti, tj, which, deriv=False):
    """g_n(r) (or dg_n/dr) from numpy's Chebyshev routines and the cosine
    cutoff: f_k = (T_k(x) + 1)/2 f_c, x = 2 (r/rc - 1)^2 - 1."""
    if which == "R":
        rc, K, c = m.rc_radial, m.basis_radial, m.c_radial[ti, tj]
    else:
        rc, K, c = m.rc_angular, m.basis_angular, m.c_angular[ti, tj]
    cheb = np.polynomial.chebyshev
    x = 2 * (r / rc - 1) ** 2 - 1
    dx = 4 * (r / rc - 1) / rc
    fc = 0.5 * (1 + np.cos(np.pi * r / rc))
    dfc = -0.5 * np.pi / rc * np.sin(np.pi * r / rc)
    T = np.array([cheb.chebval(x, np.eye(K + 1)[k]) for k in range(K + 1)])
    if not deriv:
        return c @ (0.5 * (T + 1) * fc)
    dT = np.array([cheb.chebval(x, cheb.chebder(np.eye(K + 1)[k])) for k in range(K + 1)])
    return c @ (0.5 * dT * dx * fc + 0.5 * (T + 1) * dfc)


KAPPA4 = -np.sqrt(2 / 35) * (5 / (4 * np.pi)) ** 1.5


def q_closed(m, r, ti, tj, v, deriv=False):
    """Descriptor component v of an atom with one neighbour at distance r
    (or its derivative with respect to r)."""
    block, n = blocks(m)[v]
    if block == "R":
        return g_closed(m, r, ti, tj, "R", deriv)[n]
    g = g_closed(m, r, ti, tj, "A")[n]
    dg = g_closed(m, r, ti, tj, "A", True)[n]
    if block == "4b":
        return 3 * KAPPA4 * g * g * dg if deriv else KAPPA4 * g ** 3
    l = block
    return (2 * l + 1) / (4 * np.pi) * (2 * g * dg if deriv else g * g)


def rand_unit():
    v = RNG.standard_normal(3)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("kind,head", [(synth.KIND_DIPOLE, 0), (synth.KIND_POLARIZABILITY, 0),
                                       (synth.KIND_POLARIZABILITY, 1)])
def test_zero_first_layer_gives_bias_network(kind, head):
    m = model_h7(kind)
    one_hot(m, head, 0, 0, 0.0)
    hd = m.heads[head]
    expect = np.sum(hd.w1 * np.tanh(-hd.b0)) - hd.b1
    for trial in range(4):
        n = int(RNG.integers(0, 12))
        vecs = RNG.standard_normal((n, 3)) * 1.7
        tj = RNG.integers(0, 2, n)
        res = oracle.atom_eval(m, head, int(RNG.integers(0, 2)), vecs, tj)
        assert res["U"] == pytest.approx(expect, rel=1e-14, abs=1e-15)
        np.testing.assert_array_equal(res["dUdq"], 0.0)
        np.testing.assert_array_equal(res["dUdr"], 0.0)


@pytest.mark.parametrize("kind,head", [(synth.KIND_DIPOLE, 0), (synth.KIND_POLARIZABILITY, 0),
                                       (synth.KIND_POLARIZABILITY, 1)])
def test_one_hot_first_layer_single_neighbor(kind, head):
    m = model_h7(kind, seed=43)
    D = m.dim
    assert D == 30 and m.n_hidden == H
    hd = m.heads[head]
    # every descriptor block, rows spread over the hidden layer
    picks = [(0, 0), (6, 3), (2, 5), (5, 9), (1, 14), (4, 17), (3, 22), (6, 26), (0, 29)]
    for row, col in picks:
        w = float(RNG.uniform(-1.5, 1.5))
        one_hot(m, head, row, col, w)
        for _ in range(2):
            r = float(RNG.uniform(0.9, 3.9))
            ti, tj = int(RNG.integers(0, 2)), int(RNG.integers(0, 2))
            res = oracle.atom_eval(m, head, ti, [r * rand_unit()], [tj], forces=False)
            qv = q_closed(m, r, ti, tj, col)
            x = w * m.q_scaler[col] * qv - hd.b0[row]
            rest = np.delete(np.arange(H), row)
            expect = np.sum(hd.w1[rest] * np.tanh(-hd.b0[rest])) + hd.w1[row] * np.tanh(x) - hd.b1
            assert res["U"] == pytest.approx(expect, rel=1e-12, abs=1e-14), (row, col)
            dq = np.zeros(D)
            dq[col] = m.q_scaler[col] * w * hd.w1[row] * (1 - np.tanh(x) ** 2)
            np.testing.assert_allclose(res["dUdq"], dq, rtol=1e-12, atol=1e-15)


def _net(hd, s, qv, row, w):
    """(U, dU/dq_v) of a one-hot network on one descriptor component."""
    x = w * s * qv - hd.b0[row]
    rest = np.delete(np.arange(len(hd.b0)), row)
    U = np.sum(hd.w1[rest] * np.tanh(-hd.b0[rest])) + hd.w1[row] * np.tanh(x) - hd.b1
    return U, w * s * hd.w1[row] * (1 - np.tanh(x) ** 2)


def test_dimer_one_hot_dipole_and_distinct_polarizability_heads():
    """Closed-form dimer tensors; the polarizability model's scalar and tensor
    heads read different descriptor components with different weights, so a
    swap of the two heads (or of their roles) changes alpha."""
    e = np.array([0.36, -0.48, 0.8])
    r = 2.3
    fr = synth.Frames(np.array([0, 2], np.int64), np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0] + r * e]),
                      np.array([0, 1], np.int32))
    # dipole: one-hot on an l = 2 angular component
    md = model_h7(synth.KIND_DIPOLE, seed=47)
    row, col, w = 4, 5 + 5 + 2, 1.3
    one_hot(md, 0, row, col, w)

    def dU(m, head, row, col, w, ti, tj):
        hd = m.heads[head]
        s = m.q_scaler[col]
        _, dUdq = _net(hd, s, q_closed(m, r, ti, tj, col), row, w)
        return dUdq * q_closed(m, r, ti, tj, col, deriv=True)

    def U(m, head, row, col, w, ti, tj):
        return _net(m.heads[head], m.q_scaler[col], q_closed(m, r, ti, tj, col), row, w)[0]

    mu = oracle.eval_frames(md, fr)[0]
    expect_mu = -r * r * (dU(md, 0, row, col, w, 0, 1) - dU(md, 0, row, col, w, 1, 0)) * e
    np.testing.assert_allclose(mu, expect_mu, rtol=1e-10, atol=1e-14)
    assert np.linalg.norm(expect_mu) > 1e-6

    # polarizability: tensor head (0) one-hot on a radial component, scalar head
    # (1) one-hot on the four-body component of another n
    mp = model_h7(synth.KIND_POLARIZABILITY, seed=49)
    t_row, t_col, t_w = 2, 3, -0.9
    s_row, s_col, s_w = 6, 27, 1.7
    one_hot(mp, 0, t_row, t_col, t_w)
    one_hot(mp, 1, s_row, s_col, s_w)
    al = oracle.eval_frames(mp, fr)[0]
    us = U(mp, 1, s_row, s_col, s_w, 0, 1) + U(mp, 1, s_row, s_col, s_w, 1, 0)
    ut = dU(mp, 0, t_row, t_col, t_w, 0, 1) + dU(mp, 0, t_row, t_col, t_w, 1, 0)
    expect_al = us * np.eye(3) - r * ut * np.outer(e, e)
    np.testing.assert_allclose(al, expect_al, rtol=1e-10, atol=1e-14)
    # the heads' roles matter: the swapped reading differs
    us_sw = U(mp, 0, t_row, t_col, t_w, 0, 1) + U(mp, 0, t_row, t_col, t_w, 1, 0)
    ut_sw = dU(mp, 1, s_row, s_col, s_w, 0, 1) + dU(mp, 1, s_row, s_col, s_w, 1, 0)
    swapped = us_sw * np.eye(3) - r * ut_sw * np.outer(e, e)
    assert np.abs(swapped - expect_al).max() > 1e-3 * np.abs(expect_al).max()
