"""Trajectory reuse of neighbour candidates (TNEP_OPT_TRAJECTORY_WINDOW).

With reuse the neighbour order of follower frames comes from their window's
reference frame and their pair vectors from FP64 positions (the plain search
forms them in FP32 from in-cell offsets), so results agree with plain searches
up to FP32 rounding: every frame of both paths is checked against the FP64
oracle at the 1e-5 bound (per-frame metric of tests/parity.py), and the two
paths against each other with the same metric.  A failed guard (an atom moved
more than skin / 2, or changed species) redoes the call with plain searches:
then results are bitwise those of plain searches.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu


def _traj(n_frames=40, seed=3):
    pos, spc, cell = synth.water_box(8, 24.84, seed=seed)
    return synth.ou_trajectory(pos, spc, cell, n_frames, seed=seed + 1)


def _ctx(gpu_lib, window=16, skin_ma=1000, **opts):
    c = gpu_lib.Context(0)
    if window:
        c.set_option(gpu_lib.OPT_TRAJECTORY_WINDOW, window)
        c.set_option(gpu_lib.OPT_SKIN_MA, skin_ma)
    for k, v in opts.items():
        c.set_option(getattr(gpu_lib, k), v)
    return c


def test_reuse_matches_plain_and_oracle(gpu_lib):
    fr = _traj()
    md, mp = synth.model("water_dipole_small"), synth.model("water_polarizability")
    plain, reuse = _ctx(gpu_lib, 0), _ctx(gpu_lib, 16)
    out = {}
    for name, c in (("plain", plain), ("reuse", reuse)):
        gd, gp = gpu_lib.Model(c, md), gpu_lib.Model(c, mp)
        out[name] = gpu_lib.tnep_eval_dipole_polarizability(c, gd, gp, fr)
    assert reuse.reuse_fallbacks() == 0
    refs = [oracle.eval_frames(m, fr, per_atom=True) for m in (md, mp)]
    for k, ((ref, pa), a, b) in enumerate(zip(refs, out["plain"], out["reuse"])):
        ref = ref.reshape(fr.n_frames, -1)
        e_plain = frame_errors(a, ref, pa, fr.offsets)
        e_reuse = frame_errors(b, ref, pa, fr.offsets)
        e_pair = frame_errors(b, np.asarray(a).reshape(fr.n_frames, -1), pa, fr.offsets)
        print(f"model {k}: plain {e_plain.max():.2e} reuse {e_reuse.max():.2e} reuse vs plain {e_pair.max():.2e}",
              flush=True)
        assert np.all(e_plain <= TENSOR_TOL) and np.all(e_reuse <= TENSOR_TOL)
        assert np.all(e_pair <= TENSOR_TOL)
    # deterministic
    gd, gp = gpu_lib.Model(reuse, md), gpu_lib.Model(reuse, mp)
    again = gpu_lib.tnep_eval_dipole_polarizability(reuse, gd, gp, fr)
    assert np.array_equal(again[0], out["reuse"][0]) and np.array_equal(again[1], out["reuse"][1])
    for c in (plain, reuse):
        c.close()


@pytest.mark.parametrize("breach", ["jump", "species"])
def test_guard_failure_redoes_plain(gpu_lib, breach):
    fr = _traj(20, seed=5)
    off = fr.offsets
    if breach == "jump":
        fr.positions[off[6] + 17] += np.array([0.6, 0.4, 0.3])  # 0.78 A > skin / 2 + the walk
    else:
        o = off[9] + 3 * 10  # swap the species of an O and its H in frame 9
        fr.species[o], fr.species[o + 1] = fr.species[o + 1], fr.species[o]
    m = synth.model("water_dipole_small")
    plain, reuse = _ctx(gpu_lib, 0), _ctx(gpu_lib, 8)
    a = gpu_lib.tnep_eval_dipole(plain, gpu_lib.Model(plain, m), fr)
    b = gpu_lib.tnep_eval_dipole(reuse, gpu_lib.Model(reuse, m), fr)
    assert reuse.reuse_fallbacks() == 1
    assert np.array_equal(a, b)
    for c in (plain, reuse):
        c.close()


def test_small_boxes_and_vacuum_stay_plain(gpu_lib):
    """Boxes shorter than 2 (r_c + skin) and vacuum frames are never reused."""
    m = synth.model("molecule_dipole")
    fr = synth.Frames.concat([synth.water_small(3, seed=8), synth.molecules(5, seed=9)])
    fr.species[: fr.offsets[3]] = np.where(fr.species[: fr.offsets[3]] == 0, 3, 1)  # O, H of the 5-species model
    plain, reuse = _ctx(gpu_lib, 0), _ctx(gpu_lib, 4)
    a = gpu_lib.tnep_eval_dipole(plain, gpu_lib.Model(plain, m), fr)
    b = gpu_lib.tnep_eval_dipole(reuse, gpu_lib.Model(reuse, m), fr)
    assert np.array_equal(a, b) and reuse.reuse_fallbacks() == 0
    for c in (plain, reuse):
        c.close()


def test_reuse_with_graphs_batches_and_pes(gpu_lib):
    fr = _traj(24, seed=11)
    m = synth.model("water_pes")
    base = _ctx(gpu_lib, 6)
    E, W, F = gpu_lib.tnep_eval_pes(base, gpu_lib.Model(base, m), fr)
    graph = _ctx(gpu_lib, 6, OPT_GRAPHS=1)
    gm = gpu_lib.Model(graph, m)
    for _ in range(3):
        Eg, Wg, Fg = gpu_lib.tnep_eval_pes(graph, gm, fr)
        assert np.array_equal(Eg, E) and np.array_equal(Wg, W) and np.array_equal(Fg, F)
    # windows cut by launch batches of 5 frames
    small = _ctx(gpu_lib, 6, OPT_MAX_BATCH_ATOMS=5 * 1536)
    Es, Ws, Fs = gpu_lib.tnep_eval_pes(small, gpu_lib.Model(small, m), fr)
    plain = _ctx(gpu_lib, 0)
    Up = np.zeros(fr.n_atoms)
    Ep, Wp, Fp = gpu_lib.tnep_eval_pes(plain, gpu_lib.Model(plain, m), fr, per_atom_energy=Up)
    for f in range(fr.n_frames):
        sl = slice(fr.offsets[f], fr.offsets[f + 1])
        for F_ in (F, Fs):
            assert np.linalg.norm(F_[sl] - Fp[sl]) <= 5e-6 * np.linalg.norm(Fp[sl])
    for f in range(fr.n_frames):
        scale = np.abs(Up[fr.offsets[f]:fr.offsets[f + 1]]).sum()
        assert abs(E[f] - Ep[f]) <= 5e-6 * scale and abs(Es[f] - Ep[f]) <= 5e-6 * scale
    assert base.reuse_fallbacks() == 0 and graph.reuse_fallbacks() == 0
    for c in (base, graph, small, plain):
        c.close()
