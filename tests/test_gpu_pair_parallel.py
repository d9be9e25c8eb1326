"""The pair-parallel evaluation layout (TNEP_OPT_PAIR_PARALLEL: 16 lanes per
atom, the lanes' shares added by a fixed tree) against the FP64 oracle, the
default layout, and itself under rebatching.

Tensors: per-frame relative Frobenius error <= 1e-5 against the oracle
(tests/parity.py); the two layouts sum the same FP32 pair terms in another
order, so they agree to a few FP32 roundings of the atom terms.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctxs(gpu_lib):
    pp = gpu_lib.Context(0)
    pp.set_option(gpu_lib.OPT_PAIR_PARALLEL, 1)
    plain = gpu_lib.Context(0)
    yield pp, plain
    pp.close()
    plain.close()


def _eval(gpu_lib, ctx, m, fr, per_atom=None):
    mdl = gpu_lib.Model(ctx, m)
    f = gpu_lib.tnep_eval_dipole if m.kind == 1 else gpu_lib.tnep_eval_polarizability
    out = f(ctx, mdl, fr, per_atom=per_atom)
    mdl.close()
    return out


def _check(gpu, m, fr, label):
    ref, pa = oracle.eval_frames(m, fr, per_atom=True)
    err = frame_errors(gpu.reshape(len(ref), -1), ref.reshape(len(ref), -1), pa, fr.offsets)
    print(f"{label}: max frame error {err.max():.3e}", flush=True)
    assert np.all(err <= TENSOR_TOL), (label, err)


def _five_body_box():
    pos, spc, cell = synth.water_box(8, 24.84, seed=91)
    return synth.Frames(np.array([0, len(spc)], np.int64), pos, spc, cell[None], np.ones((1, 3), np.uint8))


CASES = [
    ("water_dipole_small", lambda: synth.water_small(10), "water 10 x 192"),
    ("water_polarizability", lambda: synth.water_small(3, seed=2), "water 3 x 192"),
    ("molecule_dipole", lambda: synth.molecules(96, seed=5), "96 molecules"),
    ("molecule_polarizability", lambda: synth.molecules(96, seed=6), "96 molecules"),
    ("perovskite_susceptibility", lambda: synth.perovskite(2, n_rep=4), "perovskite 4^3"),
    ("water_dipole_5b", _five_body_box, "water 1536, five-body"),
    ("water_polarizability_5b", lambda: synth.water_small(2, seed=3), "water 2 x 192, five-body"),
]


@pytest.mark.parametrize("name,make,label", CASES, ids=[c[0] for c in CASES])
def test_matches_oracle_and_default_layout(gpu_lib, ctxs, name, make, label):
    pp, plain = ctxs
    m = synth.model(name)
    fr = make()
    nt = 3 if m.kind == 1 else 9
    pa_pp, pa_plain = np.zeros((fr.n_atoms, nt)), np.zeros((fr.n_atoms, nt))
    a = _eval(gpu_lib, pp, m, fr, per_atom=pa_pp)
    b = _eval(gpu_lib, plain, m, fr, per_atom=pa_plain)
    _check(a, m, fr, label + " (pair-parallel)")
    # the same pair terms in another order: per-atom terms agree to FP32 rounding
    scale = np.abs(pa_plain).max()
    assert np.abs(pa_pp - pa_plain).max() <= 1e-5 * scale, np.abs(pa_pp - pa_plain).max() / scale


def test_per_species_networks(gpu_lib, ctxs):
    pp, _ = ctxs
    a = synth.model("molecule_polarizability")
    seed, kind, species, desc = synth.MODEL_SPECS["molecule_polarizability"]
    b = synth.with_descriptor_of(synth.make_model(seed + 50, kind, species, **desc), a)
    m = synth.per_species_model([a, b], [0, 1, 0, 1, 0])
    fr = synth.molecules(64, seed=82)
    _check(_eval(gpu_lib, pp, m, fr), m, fr, "per-species networks (pair-parallel)")


def test_deterministic_and_batch_invariant(gpu_lib, ctxs):
    pp, _ = ctxs
    m = synth.model("molecule_polarizability")
    fr = synth.molecules(120, seed=9)
    a = _eval(gpu_lib, pp, m, fr)
    assert np.array_equal(a, _eval(gpu_lib, pp, m, fr))
    c2 = gpu_lib.Context(0)
    c2.set_option(gpu_lib.OPT_PAIR_PARALLEL, 1)
    c2.set_option(gpu_lib.OPT_MAX_BATCH_ATOMS, 400)  # many small launch batches
    assert np.array_equal(a, _eval(gpu_lib, c2, m, fr))
    c2.close()
    assert np.array_equal(_eval(gpu_lib, pp, m, fr.subset([41]))[0], a[41])


def test_both_models_one_call_and_edge_cases(gpu_lib, ctxs):
    pp, _ = ctxs
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    mol = synth.molecules(3, seed=4)
    parts = [synth.Frames(np.array([0, 0], np.int64), np.zeros((0, 3)), np.zeros(0, np.int32)),
             mol.subset([0]),
             synth.Frames(np.array([0, 1], np.int64), np.zeros((1, 3)), np.array([2], np.int32)),
             synth.Frames(np.array([0, 2], np.int64), np.array([[0, 0, 0], [10.0, 0, 0]]), np.array([1, 3], np.int32)),
             mol.subset([1, 2])]
    fr = synth.Frames.concat(parts)
    gd, gp = gpu_lib.Model(pp, md), gpu_lib.Model(pp, mp)
    mu, al = gpu_lib.tnep_eval_dipole_polarizability(pp, gd, gp, fr)
    gd.close()
    gp.close()
    assert np.all(mu[[0, 2, 3]] == 0.0) and np.all(al[0] == 0.0)
    _check(mu, md, fr, "edge cases, dipole (pair-parallel)")
    _check(al, mp, fr, "edge cases, polarizability (pair-parallel)")


def test_potential_energy_keeps_default_layout(gpu_lib, ctxs):
    pp, plain = ctxs
    m = synth.model("water_pes")
    fr = synth.water_small(2, seed=5)
    outs = []
    for c in (pp, plain):
        mdl = gpu_lib.Model(c, m)
        outs.append(gpu_lib.tnep_eval_pes(c, mdl, fr))
        mdl.close()
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)


def test_grid_and_all_pairs_frames_in_one_call(gpu_lib, ctxs):
    """One call mixing frames searched on a cell grid (24.84 A box: the default
    search) and frames searched all-pairs (molecules, 12.42 A boxes: the
    pair-parallel search), both evaluated in the pair-parallel layout."""
    pp, _ = ctxs
    m = synth.model("water_polarizability")
    mp = synth.model("molecule_polarizability")
    pos, spc, cell = synth.water_box(8, 24.84, seed=93)
    big = synth.Frames(np.array([0, len(spc)], np.int64), pos, spc, cell[None], np.ones((1, 3), np.uint8))
    fr = synth.Frames.concat([synth.water_small(2, seed=11), big, synth.water_small(1, seed=12)])
    _check(_eval(gpu_lib, pp, m, fr), m, fr, "mixed grid / all-pairs water (pair-parallel)")
    mol = synth.molecules(40, seed=13)
    _check(_eval(gpu_lib, pp, mp, mol), mp, mol, "molecules (pair-parallel)")


def test_graph_replay_matches_plain_launches(gpu_lib):
    import torch

    plain = gpu_lib.Context(0)
    graph = gpu_lib.Context(0)
    for c in (plain, graph):
        c.set_option(gpu_lib.OPT_PAIR_PARALLEL, 1)
    graph.set_option(gpu_lib.OPT_GRAPHS, 1)
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    pd_, pp_ = gpu_lib.Model(plain, md), gpu_lib.Model(plain, mp)
    gd_, gp_ = gpu_lib.Model(graph, md), gpu_lib.Model(graph, mp)
    mols = synth.molecules(32, seed=33)
    for rep in range(3):
        for s, n in [(0, 5), (9, 6), (20, 7)]:
            fr = mols.subset(range(s, s + n))
            g = gpu_lib.tnep_eval_dipole_polarizability(graph, gd_, gp_, fr)
            torch.cuda.synchronize()
            p = gpu_lib.tnep_eval_dipole_polarizability(plain, pd_, pp_, fr)
            for a, b in zip(g, p):
                assert np.array_equal(a, b), (rep, s, n)
    captures, launches = graph.graph_counts()
    assert launches >= 9
    for x in (pd_, pp_, gd_, gp_):
        x.close()
    plain.close()
    graph.close()


def test_triclinic_and_trajectory_frames(gpu_lib):
    """Lists from the triclinic search and from trajectory candidate reuse
    (reference and follower frames) evaluated in the pair-parallel layout."""
    shear = np.array([[1, 0, 0], [1, 1, 0], [0, 1, 1]], np.float64)
    pos, spc, cell = synth.water_box(8, 24.84, seed=94)
    R, _ = np.linalg.qr(np.random.default_rng(95).normal(size=(3, 3)))
    H = cell.reshape(3, 3)
    n = len(spc)
    tri = synth.Frames(np.array([0, n, 2 * n], np.int64), np.concatenate([pos, pos @ R.T]),
                       np.tile(spc, 2).astype(np.int32), np.stack([shear @ H, H @ R.T]).reshape(2, 9),
                       np.ones((2, 3), np.uint8))
    traj = synth.ou_trajectory(pos, spc, cell, 6, seed=96)
    m = synth.model("water_polarizability")
    c = gpu_lib.Context(0)
    c.set_option(gpu_lib.OPT_PAIR_PARALLEL, 1)
    _check(_eval(gpu_lib, c, m, tri), m, tri, "triclinic (pair-parallel)")
    c.set_option(gpu_lib.OPT_TRAJECTORY_WINDOW, 3)
    _check(_eval(gpu_lib, c, m, traj), m, traj, "trajectory reuse (pair-parallel)")
    assert c.reuse_fallbacks() == 0
    c.close()


def test_edge_frames_with_host_layout(gpu_lib, ctxs):
    """Empty frames, a single atom and isolated atoms as device frames with the
    layout on the host, in both layouts: bitwise the host-frame results."""
    import torch

    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    mol = synth.molecules(3, seed=4)
    parts = [synth.Frames(np.array([0, 0], np.int64), np.zeros((0, 3)), np.zeros(0, np.int32)),
             mol.subset([0]),
             synth.Frames(np.array([0, 1], np.int64), np.zeros((1, 3)), np.array([2], np.int32)),
             synth.Frames(np.array([0, 0], np.int64), np.zeros((0, 3)), np.zeros(0, np.int32)),
             synth.Frames(np.array([0, 2], np.int64), np.array([[0, 0, 0], [10.0, 0, 0]]), np.array([1, 3], np.int32)),
             mol.subset([1, 2])]
    fr = synth.Frames.concat(parts)
    dfr = gpu_lib.DeviceFrames(fr, host_meta=True)
    for c in ctxs:
        gd, gp = gpu_lib.Model(c, md), gpu_lib.Model(c, mp)
        mu, al = gpu_lib.tnep_eval_dipole_polarizability(c, gd, gp, fr)
        dmu = torch.zeros((fr.n_frames, 3), dtype=torch.float64, device="cuda")
        dal = torch.zeros((fr.n_frames, 9), dtype=torch.float64, device="cuda")
        gpu_lib.tnep_eval_dipole_polarizability(c, gd, gp, dfr, dmu, dal)
        torch.cuda.synchronize()
        assert np.array_equal(dmu.cpu().numpy(), mu) and np.array_equal(dal.cpu().numpy(), al.reshape(-1, 9))
        assert np.all(mu[[0, 2, 3, 4]] == 0.0)
        gd.close()
        gp.close()
