"""CPU self-check of the kernels' per-pair arithmetic (the inline functions of
csrc/tnep_math.h and csrc/radial_basis.h that the evaluation kernels call,
compiled for the host by csrc/host_check.cpp) against the FP64 oracle, through quantities that do
not depend on sign or basis conventions: the addition theorem, contracted
gradients, and the rotation invariants q_nl and the four-body term."""
import ctypes as C
import os

import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2312_05233_amd", "_host_check.so")
SRCS = [os.path.join(ROOT, "paper_2312_05233_amd", "csrc", f)
        for f in ("host_check.cpp", "tnep_math.h", "radial_basis.h")]
RNG = np.random.default_rng(99)
LRANGE = {1: (0, 3), 2: (3, 8), 3: (8, 15), 4: (15, 24)}


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(s) for s in SRCS):
        from paper_2312_05233_amd import build as b

        b.build_host_check(verbose=False)
    lib = C.CDLL(LIB)
    lib.tnep_hc_four_body.restype = C.c_float
    return lib


def fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def sh(hc, v):
    u = np.ascontiguousarray(v / np.linalg.norm(v), np.float32)
    P = np.zeros(24, np.float32)
    dP = np.zeros(72, np.float32)
    hc.tnep_hc_sh(fp(u), fp(P), fp(dP))
    return P.astype(np.float64), dP.reshape(24, 3).astype(np.float64)


def test_sh_addition_theorem(hc):
    for _ in range(30):
        a, b = RNG.standard_normal(3), RNG.standard_normal(3)
        Pa, _ = sh(hc, a)
        Pb, _ = sh(hc, b)
        c = a @ b / np.linalg.norm(a) / np.linalg.norm(b)
        for l, (lo, hi) in LRANGE.items():
            assert Pa[lo:hi] @ Pb[lo:hi] == pytest.approx((2 * l + 1) / (4 * np.pi) * eval_legendre(l, c), abs=2e-6)


def test_sh_gradient_contracted_with_oracle(hc):
    """sum_m grad_a Y_lm(a) Y_lm(b) is convention independent."""
    for _ in range(20):
        a, b = RNG.standard_normal(3) * 2, RNG.standard_normal(3)
        r = np.linalg.norm(a)
        u = a / r
        Pa, dPa = sh(hc, a)
        Pb, _ = sh(hc, b)
        for l, (lo, hi) in LRANGE.items():
            mine = sum(((dPa[c] - l * Pa[c] * u) / r) * Pb[c] for c in range(lo, hi))
            ref = sum(oracle.ylm(l, m, a)[1] * oracle.ylm(l, m, b)[0] for m in range(-l, l + 1))
            np.testing.assert_allclose(mine, ref, atol=5e-6)


def test_four_body_value_and_gradient(hc):
    for _ in range(10):
        vecs = RNG.standard_normal((6, 3))
        g = RNG.uniform(0.2, 1.0, 6)
        A_mine = sum(gi * sh(hc, v)[0][3:8] for gi, v in zip(g, vecs))
        A_ref = sum(gi * np.array([oracle.ylm(2, m, v)[0] for m in range(-2, 3)]) for gi, v in zip(g, vecs))
        a32 = np.ascontiguousarray(A_mine, np.float32)
        d = np.zeros(5, np.float32)
        q = hc.tnep_hc_four_body(fp(a32), fp(d))
        assert q == pytest.approx(oracle.four_body(A_ref)[0], rel=1e-5, abs=1e-7)
        h = 1e-2
        for k in range(5):
            e = np.zeros(5, np.float32)
            e[k] = h
            dd = np.zeros(5, np.float32)
            qp = hc.tnep_hc_four_body(fp(a32 + e), fp(dd))
            qm = hc.tnep_hc_four_body(fp(a32 - e), fp(dd))
            assert d[k] == pytest.approx((qp - qm) / (2 * h), rel=2e-3, abs=1e-5)


def test_basis_matches_oracle(hc):
    f = np.zeros(9, np.float32)
    df = np.zeros(9, np.float32)
    for r in np.linspace(0.5, 5.9, 17):
        hc.tnep_hc_basis9(C.c_float(r), C.c_float(6.0), fp(f), fp(df))
        fo, dfo = oracle.basis(r, 6.0, 8)
        np.testing.assert_allclose(f, fo, atol=2e-6)
        np.testing.assert_allclose(df, dfo, atol=2e-6)


def test_atom_descriptor_matches_oracle(hc):
    m = synth.model("water_dipole_small")
    fr = synth.water_small(1, seed=4)
    pos = fr.positions
    L = fr.cells[0][0]
    nb = oracle.neighbors(pos, fr.cells[0], fr.pbc[0], 6.0)
    for i in [0, 1, 2, 50, 191]:
        v = pos[nb[i]] - pos[i]
        v -= L * np.round(v / L)
        tj = fr.species[nb[i]]
        ti = fr.species[i]
        ref = oracle.atom_eval(m, 0, int(ti), v, tj, forces=False)["q"]
        cR = np.ascontiguousarray(m.c_radial[ti], np.float32)
        cA = np.ascontiguousarray(m.c_angular[ti], np.float32)
        q = np.zeros(30, np.float32)
        v32 = np.ascontiguousarray(v, np.float32)
        t32 = np.ascontiguousarray(tj, np.int32)
        hc.tnep_hc_descriptor(len(v), fp(v32), t32.ctypes.data_as(C.POINTER(C.c_int)), fp(cR), fp(cA),
                              C.c_float(6.0), C.c_float(4.0), fp(q))
        scale = np.abs(ref) + 1e-3 * np.abs(ref).max()
        assert np.max(np.abs(q - ref) / scale) < 1e-4
