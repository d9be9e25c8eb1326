"""Parity at the workloads' full sizes, in one call each (the launch batches,
frame counts and cell grids of the benchmark runs):

* perovskite susceptibility: 2 frames of the 12 x 12 x 12 supercell (8,640
  atoms each), FP32 vector and FP32 matrix-core hidden layers;
* all 8,192 ragged vacuum molecules in one dipole + polarizability call,
  every frame against the oracle;
* a serving mix whose largest request is a 24,576-atom water box of 64 OU
  frames: every request alone == in the mix (bitwise), sampled frames against
  the oracle.

Tolerance: 1e-5 per frame (tests/parity.py metric)."""
import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["MLP_FP32_VALU", "MLP_FP32_MFMA"])
def test_perovskite_full_supercell(gpu_lib, mode):
    m = synth.model("perovskite_susceptibility")
    fr = synth.perovskite(2, seed=21)
    assert fr.n_atoms == 2 * 8640
    ctx = gpu_lib.Context(0)
    ctx.set_option(gpu_lib.OPT_MLP, getattr(gpu_lib, mode))
    gm = gpu_lib.Model(ctx, m)
    al = np.asarray(gpu_lib.tnep_eval_polarizability(ctx, gm, fr)).reshape(2, 9)
    ref, pa = oracle.eval_frames(m, fr, per_atom=True)
    err = frame_errors(al, ref.reshape(2, 9), pa, fr.offsets)
    print(f"perovskite 2 x 8640 {mode}: {err.max():.2e}", flush=True)
    assert np.all(err <= TENSOR_TOL)
    ctx.close()


def test_all_molecules_one_call(gpu_lib):
    fr = synth.molecules(8192)
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    ctx = gpu_lib.Context(0)
    gd, gp = gpu_lib.Model(ctx, md), gpu_lib.Model(ctx, mp)
    mu, al = gpu_lib.tnep_eval_dipole_polarizability(ctx, gd, gp, fr)
    ref_mu, pa_mu = oracle.eval_frames(md, fr, per_atom=True)
    ref_al, pa_al = oracle.eval_frames(mp, fr, per_atom=True)
    e_mu = frame_errors(mu, ref_mu, pa_mu, fr.offsets)
    e_al = frame_errors(np.asarray(al).reshape(-1, 9), ref_al.reshape(-1, 9), pa_al, fr.offsets)
    w = int(np.argmax(e_mu))
    pa_norm = np.linalg.norm(pa_mu[fr.offsets[w]:fr.offsets[w + 1]], axis=1).sum()
    print(f"8192 molecules ({fr.n_atoms} atoms): dipole {e_mu.max():.2e} (frame {w}, |mu| / sum |mu_i| = "
          f"{np.linalg.norm(ref_mu[w]) / pa_norm:.2e}) polarizability {e_al.max():.2e}", flush=True)
    assert e_mu.shape == (8192,) and np.all(e_mu <= TENSOR_TOL)
    assert np.all(e_al <= TENSOR_TOL)
    ctx.close()


def test_serving_mix_with_largest_box(gpu_lib):
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    pos, spc, cell = synth.water_box_orthorhombic((16, 16, 32), 3.105, seed=31, o_species=3, h_species=1)
    assert len(spc) == 24576
    big = synth.ou_trajectory(pos, spc, cell, 64, seed=32)
    rng = np.random.default_rng(33)
    mols = synth.molecules(600, seed=34)
    reqs = [(2, big), (1, big.subset(range(0, 64, 9)))]
    for k in range(10):
        if k % 2:
            n = int(rng.choice([4, 8, 16]))
            p, sp, c = synth.water_box(n, 3.105 * n, seed=40 + k, o_species=3, h_species=1)
            reqs.append((1 + k % 2, synth.ou_trajectory(p, sp, c, int(rng.integers(1, 65)), seed=k)))
        else:
            s0 = int(rng.integers(0, 500))
            reqs.append((1 + (k // 2) % 2, mols.subset(range(s0, s0 + int(rng.integers(1, 65))))))
    ctx = gpu_lib.Context(0, budget_bytes=32 << 30)
    gm = {1: gpu_lib.Model(ctx, md), 2: gpu_lib.Model(ctx, mp)}
    alone = []
    for kind, fr in reqs:
        f = gpu_lib.tnep_eval_dipole if kind == 1 else gpu_lib.tnep_eval_polarizability
        alone.append(np.asarray(f(ctx, gm[kind], fr)).reshape(fr.n_frames, -1))
    srv = gpu_lib.Server(ctx, budget_bytes=32 << 30, max_batch_atoms=1 << 19, max_inflight=3)
    tickets = [srv.submit(gm[kind], fr) for kind, fr in reqs]
    for i, t in enumerate(tickets):
        st, _, out = srv.wait(t)
        assert st == 0
        assert np.array_equal(out, alone[i]), i
    srv.stop()
    # oracle on the largest box (first and last frame) and one frame of each other request
    sub = big.subset([0, 63])
    ref, pa = oracle.eval_frames(mp, sub, per_atom=True)
    err = frame_errors(alone[0][[0, 63]], ref.reshape(2, 9), pa, sub.offsets)
    print(f"24576-atom box x 64 frames, polarizability: {err.max():.2e}", flush=True)
    assert np.all(err <= TENSOR_TOL)
    for (kind, fr), a in list(zip(reqs, alone))[2:]:
        one = fr.subset([fr.n_frames - 1])
        ref, pa = oracle.eval_frames(md if kind == 1 else mp, one, per_atom=True)
        assert frame_errors(a[-1:], ref.reshape(1, -1), pa, one.offsets).max() <= TENSOR_TOL
    ctx.close()
