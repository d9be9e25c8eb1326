"""HIP-graph replay of launch batches (TNEP_OPT_GRAPHS) against plain launches.

Every replay is compared bit for bit with the plain-launch result of the same
input, with other eager GPU work and stream synchronisations between replays;
batches of different actual sizes share one graph when they fall into the same
power-of-two bucket of atoms, frames and cells.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu


def _ctx_pair(gpu_lib):
    plain = gpu_lib.Context(0)
    graph = gpu_lib.Context(0)
    graph.set_option(gpu_lib.OPT_GRAPHS, 1)
    return plain, graph


def _eager_noise(step):
    """Unrelated eager device work between replays, then a full sync."""
    x = torch.arange(4096, device="cuda:0", dtype=torch.int64) * (step + 1)
    y = torch.cumsum(x, 0)
    torch.cuda.synchronize()
    assert int(y[-1]) == int(x.sum()) == 4095 * 4096 // 2 * (step + 1)


def test_replays_match_plain_launches(gpu_lib):
    plain, graph = _ctx_pair(gpu_lib)
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    wd, wp = synth.model("water_dipole_small"), synth.model("water_polarizability")
    pd_, pp_ = gpu_lib.Model(plain, md), gpu_lib.Model(plain, mp)
    gd_, gp_ = gpu_lib.Model(graph, md), gpu_lib.Model(graph, mp)
    pwd, pwp = gpu_lib.Model(plain, wd), gpu_lib.Model(plain, wp)
    gwd, gwp = gpu_lib.Model(graph, wd), gpu_lib.Model(graph, wp)
    mols = synth.molecules(64, seed=31)
    # molecule batches of 5..7 frames (same frame bucket, different atom counts)
    inputs = [("mol", mols.subset(range(s, s + n))) for s, n in [(0, 5), (9, 6), (20, 7), (40, 5)]]
    inputs += [("water", synth.water_small(k, seed=40 + k)) for k in (2, 3)]
    for rep in range(4):
        for label, fr in inputs:
            if label == "mol":
                g = gpu_lib.tnep_eval_dipole_polarizability(graph, gd_, gp_, fr)
                _eager_noise(rep)
                p = gpu_lib.tnep_eval_dipole_polarizability(plain, pd_, pp_, fr)
            else:
                g = gpu_lib.tnep_eval_dipole_polarizability(graph, gwd, gwp, fr)
                _eager_noise(rep)
                p = gpu_lib.tnep_eval_dipole_polarizability(plain, pwd, pwp, fr)
            for a, b in zip(g, p):
                assert np.array_equal(a, b), (rep, label, fr.n_frames)
    captures, launches = graph.graph_counts()
    print("graph captures", captures, "launches", launches, flush=True)
    assert launches >= 4 * len(inputs)
    assert 1 <= captures < launches
    assert plain.graph_counts() == (0, 0)
    # and the replayed results are right, not only equal to each other
    fr = inputs[1][1]
    mu, al = gpu_lib.tnep_eval_dipole_polarizability(graph, gd_, gp_, fr)
    for out, m in ((mu, md), (al, mp)):
        ref, pa = oracle.eval_frames(m, fr, per_atom=True)
        assert np.all(frame_errors(out, ref, pa, fr.offsets) <= TENSOR_TOL)
    for c in (plain, graph):
        c.close()


def test_replays_with_per_atom_and_batches(gpu_lib):
    """Per-atom outputs and calls split into several launch batches."""
    plain, graph = _ctx_pair(gpu_lib)
    for c in (plain, graph):
        c.set_option(gpu_lib.OPT_MAX_BATCH_ATOMS, 700)
    m = synth.model("molecule_polarizability")
    pm, gm = gpu_lib.Model(plain, m), gpu_lib.Model(graph, m)
    mols = synth.molecules(120, seed=32)
    for rep in range(3):
        for lo, hi in [(0, 40), (40, 100), (100, 120)]:
            fr = mols.subset(range(lo, hi))
            pa_g = np.zeros((fr.n_atoms, 9))
            pa_p = np.zeros((fr.n_atoms, 9))
            g = gpu_lib.tnep_eval_polarizability(graph, gm, fr, per_atom=pa_g)
            _eager_noise(rep)
            p = gpu_lib.tnep_eval_polarizability(plain, pm, fr, per_atom=pa_p)
            assert np.array_equal(g, p)
            assert np.array_equal(pa_g, pa_p)
    captures, launches = graph.graph_counts()
    assert launches > captures >= 1
    for c in (plain, graph):
        c.close()


def test_capacity_growth_recaptures(gpu_lib):
    """A denser input grows the neighbour capacities: graphs are recaptured."""
    plain, graph = _ctx_pair(gpu_lib)
    m = synth.model("perovskite_susceptibility")
    pm, gm = gpu_lib.Model(plain, m), gpu_lib.Model(graph, m)
    small = synth.perovskite(2, n_rep=4, seed=6)
    dense = synth.perovskite(2, n_rep=4, seed=7, sigma=0.3)
    for rep in range(2):
        for fr in (small, dense, small):
            g = gpu_lib.tnep_eval_polarizability(graph, gm, fr)
            _eager_noise(rep)
            p = gpu_lib.tnep_eval_polarizability(plain, pm, fr)
            assert np.array_equal(g, p)
    captures, launches = graph.graph_counts()
    assert captures >= 1 and launches >= 6
    for c in (plain, graph):
        c.close()


def test_server_slots_use_graphs(gpu_lib):
    """Server slot contexts inherit graphs; results equal the plain path."""
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    plain = gpu_lib.Context(0)
    pm = {1: gpu_lib.Model(plain, md), 2: gpu_lib.Model(plain, mp)}
    ctx = gpu_lib.Context(0)
    ctx.set_option(gpu_lib.OPT_GRAPHS, 1)
    sm = {1: gpu_lib.Model(ctx, md), 2: gpu_lib.Model(ctx, mp)}
    mols = synth.molecules(300, seed=33)
    rng = np.random.default_rng(5)
    reqs = []
    for k in range(40):
        s = int(rng.integers(0, 290))
        reqs.append((1 + k % 2, mols.subset(range(s, s + 1 + int(rng.integers(0, 8))))))
    srv = gpu_lib.Server(ctx, max_batch_atoms=1500, max_inflight=2)
    results = []
    for wave in range(2):
        tickets = [srv.submit(sm[kind], fr) for kind, fr in reqs]
        for t in tickets:
            st, _, out = srv.wait(t)
            assert st == 0
            results.append(out.copy())
        _eager_noise(wave)
    captures, launches = ctx.graph_counts()
    srv.stop()
    assert launches > captures >= 1
    for i, (kind, fr) in enumerate(reqs + reqs):
        f = gpu_lib.tnep_eval_dipole if kind == 1 else gpu_lib.tnep_eval_polarizability
        ref = np.asarray(f(plain, pm[kind], fr)).reshape(fr.n_frames, -1)
        assert np.array_equal(ref, results[i]), i
    for c in (plain, ctx):
        c.close()


def test_pes_outputs_switch_between_replays(gpu_lib):
    """Energy-only, forces and site-energy calls alternate on one graph context:
    each call's graph matches the outputs it asks for (the forces and site
    energies of a call are those of the plain launches, never left over from
    a graph captured for another output set)."""
    plain, graph = _ctx_pair(gpu_lib)
    m = synth.model("water_pes")
    pm, gm = gpu_lib.Model(plain, m), gpu_lib.Model(graph, m)
    fr = synth.water_small(2, seed=21)
    Er, Wr, Fr, Ur = oracle.eval_pes(m, fr, per_atom=True)
    A = fr.n_atoms
    for rep in range(2):
        for want_forces, want_sites in ((False, False), (True, False), (False, True), (True, True), (False, False)):
            Fg = np.full((A, 3), np.nan) if want_forces else None
            Ug = np.full(A, np.nan) if want_sites else None
            Fp = np.full((A, 3), np.nan) if want_forces else None
            Up = np.full(A, np.nan) if want_sites else None
            Eg, Wg, _ = gpu_lib.tnep_eval_pes(graph, gm, fr, forces=Fg, per_atom_energy=Ug, want_forces=want_forces)
            _eager_noise(rep)
            Ep, Wp, _ = gpu_lib.tnep_eval_pes(plain, pm, fr, forces=Fp, per_atom_energy=Up, want_forces=want_forces)
            assert np.array_equal(Eg, Ep) and np.array_equal(Wg, Wp)
            if want_forces:
                assert np.array_equal(Fg, Fp), (rep, want_forces, want_sites)
                assert np.linalg.norm(Fg - Fr) <= TENSOR_TOL * np.linalg.norm(Fr)
            if want_sites:
                assert np.array_equal(Ug, Up), (rep, want_forces, want_sites)
                assert np.abs(Ug - Ur).max() <= TENSOR_TOL * np.abs(Ur).max()
    captures, launches = graph.graph_counts()
    assert captures >= 4 and launches >= 10
    for c in (plain, graph):
        c.close()


def test_skin_change_between_trajectory_replays(gpu_lib):
    """Trajectory candidate reuse under graphs: changing the skin between two
    calls uses the new search radius and displacement guard (results equal to
    plain launches with the same options)."""
    pos, spc, cell = synth.water_box(8, 24.84, seed=3)
    fr = synth.ou_trajectory(pos, spc, cell, 12, seed=4)
    md = synth.model("water_dipole_small")
    plain, graph = _ctx_pair(gpu_lib)
    for c in (plain, graph):
        c.set_option(gpu_lib.OPT_TRAJECTORY_WINDOW, 6)
    pm, gm = gpu_lib.Model(plain, md), gpu_lib.Model(graph, md)
    for rep, skin_ma in enumerate((1000, 200, 1000, 600)):
        for c in (plain, graph):
            c.set_option(gpu_lib.OPT_SKIN_MA, skin_ma)
        g = gpu_lib.tnep_eval_dipole(graph, gm, fr)
        _eager_noise(rep)
        p = gpu_lib.tnep_eval_dipole(plain, pm, fr)
        assert np.array_equal(g, p), skin_ma
        assert graph.reuse_fallbacks() == plain.reuse_fallbacks()
    ref, pa = oracle.eval_frames(md, fr, per_atom=True)
    assert np.all(frame_errors(g, ref, pa, fr.offsets) <= TENSOR_TOL)
    captures, _ = graph.graph_counts()
    assert captures >= 3
    for c in (plain, graph):
        c.close()


def test_device_frames_replay_and_buffer_switch(gpu_lib):
    """Device-resident frames replay a graph keyed by the call's device
    addresses: the same buffers replay it (bitwise equal to plain launches);
    other output tensors, other input tensors and a per-atom output each get a
    graph of their own, the earlier buffers untouched."""
    plain, graph = _ctx_pair(gpu_lib)
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    pd_, pp_ = gpu_lib.Model(plain, md), gpu_lib.Model(plain, mp)
    gd_, gp_ = gpu_lib.Model(graph, md), gpu_lib.Model(graph, mp)
    mols = synth.molecules(40, seed=61)
    other = synth.molecules(40, seed=62)
    dev, dev2 = gpu_lib.DeviceFrames(mols), gpu_lib.DeviceFrames(other)
    F = mols.n_frames

    def outs():
        return (torch.zeros((F, 3), dtype=torch.float64, device="cuda"),
                torch.zeros((F, 9), dtype=torch.float64, device="cuda"))

    ref_mu, ref_al = outs()
    gpu_lib.tnep_eval_dipole_polarizability(plain, pd_, pp_, dev, ref_mu, ref_al)
    ref2_mu, ref2_al = outs()
    gpu_lib.tnep_eval_dipole_polarizability(plain, pd_, pp_, dev2, ref2_mu, ref2_al)
    a_mu, a_al = outs()
    for rep in range(3):
        a_mu.zero_()
        a_al.zero_()
        gpu_lib.tnep_eval_dipole_polarizability(graph, gd_, gp_, dev, a_mu, a_al)
        _eager_noise(rep)
        assert torch.equal(a_mu, ref_mu) and torch.equal(a_al, ref_al), rep
    captures, launches = graph.graph_counts()
    assert captures == 1 and launches == 3, (captures, launches)
    # other outputs: a new graph; the first outputs keep what they hold
    a_mu.zero_()
    a_al.zero_()
    b_mu, b_al = outs()
    gpu_lib.tnep_eval_dipole_polarizability(graph, gd_, gp_, dev, b_mu, b_al)
    torch.cuda.synchronize()
    assert torch.equal(b_mu, ref_mu) and torch.equal(b_al, ref_al)
    assert not a_mu.any() and not a_al.any()
    # other inputs (same sizes): a new graph with the new positions
    c_mu, c_al = outs()
    gpu_lib.tnep_eval_dipole_polarizability(graph, gd_, gp_, dev2, c_mu, c_al)
    assert torch.equal(c_mu, ref2_mu) and torch.equal(c_al, ref2_al)
    assert graph.graph_counts()[0] == 3
    # per-atom device output (single-model call)
    pa_ref = torch.zeros((mols.n_atoms, 3), dtype=torch.float64, device="cuda")
    mu_p, _ = outs()
    gpu_lib.tnep_eval_dipole(plain, pd_, dev, mu_p, pa_ref)
    for rep in range(2):
        pa = torch.zeros_like(pa_ref)
        mu_g, _ = outs()
        gpu_lib.tnep_eval_dipole(graph, gd_, dev, mu_g, pa)
        assert torch.equal(pa, pa_ref) and torch.equal(mu_g, mu_p), rep
    # and the replayed values are right
    ref, pa_o = oracle.eval_frames(mp, mols, per_atom=True)
    assert np.all(frame_errors(b_al.cpu().numpy(), ref, pa_o, mols.offsets) <= TENSOR_TOL)
    for c in (plain, graph):
        c.close()
