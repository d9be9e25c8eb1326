"""Potential-energy surface (Sec. 2.1) on the GPU against the FP64 oracle.

Tolerances (FP32 arithmetic, FP64 sums):
  energy: |E_gpu - E_ref| <= 1e-5 * sum_i |U_i,ref| per frame (the site
          energies' size, since their sum can cancel);
  virial: per-frame relative Frobenius error <= 1e-5 (tests/parity.py metric);
  forces: per-frame ||F_gpu - F_ref||_F / ||F_ref||_F <= 1e-5.
Forces are summed in each atom's fixed neighbour-list order (no atomics), so
they are bitwise reproducible whatever the batching.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _check(gpu_lib, ctx, mdl, m, fr, label):
    E, W, F = gpu_lib.tnep_eval_pes(ctx, mdl, fr)
    Er, Wr, Fr, Ur = oracle.eval_pes(m, fr, per_atom=True)
    off = fr.offsets
    for f in range(fr.n_frames):
        scale = np.abs(Ur[off[f]:off[f + 1]]).sum()
        assert abs(E[f] - Er[f]) <= TENSOR_TOL * max(scale, 1e-300), (label, f, E[f], Er[f])
    werr = frame_errors(W, Wr)
    ferr = np.array([np.linalg.norm(F[off[f]:off[f + 1]] - Fr[off[f]:off[f + 1]]) /
                     max(np.linalg.norm(Fr[off[f]:off[f + 1]]), 1e-300) for f in range(fr.n_frames)
                     if off[f + 1] > off[f]])
    print(f"{label}: virial {werr.max():.2e} forces {ferr.max() if len(ferr) else 0:.2e}", flush=True)
    assert np.all(werr <= TENSOR_TOL), (label, werr)
    assert np.all(ferr <= TENSOR_TOL), (label, ferr)
    return E, W, F


def test_water_small(gpu_lib, ctx):
    m = synth.model("water_pes")
    mdl = gpu_lib.Model(ctx, m)
    fr = synth.water_small(6, seed=11)
    _, _, F = _check(gpu_lib, ctx, mdl, m, fr, "water 192 PES")
    # Newton's third law up to the FP32 rounding of each atom's own sum
    for f in range(fr.n_frames):
        Ff = F[fr.offsets[f]:fr.offsets[f + 1]]
        assert np.abs(Ff.sum(0)).max() <= 1e-6 * np.abs(Ff).sum()


def test_per_atom_energies(gpu_lib, ctx):
    m = synth.model("water_pes")
    mdl = gpu_lib.Model(ctx, m)
    fr = synth.water_small(2, seed=12)
    U = np.zeros(fr.n_atoms)
    E, _, _ = gpu_lib.tnep_eval_pes(ctx, mdl, fr, per_atom_energy=U)
    _, _, _, Ur = oracle.eval_pes(m, fr, per_atom=True)
    assert np.abs(U - Ur).max() <= 1e-5 * np.abs(Ur).max()
    # skipping the optional outputs changes nothing
    E2, W2, F2 = gpu_lib.tnep_eval_pes(ctx, mdl, fr, want_virial=False, want_forces=False)
    assert W2 is None and F2 is None and np.array_equal(E, E2)


def test_cell_list_and_full_size(gpu_lib, ctx):
    m = synth.model("water_pes")
    mdl = gpu_lib.Model(ctx, m)
    pos, spc, cell = synth.water_box(8, 24.84, seed=78)
    fr = synth.Frames(np.array([0, len(spc)], np.int64), pos, spc, cell[None], np.ones((1, 3), np.uint8))
    _check(gpu_lib, ctx, mdl, m, fr, "water 1536 PES")
    big = synth.water_trajectory(2).subset([1])
    _check(gpu_lib, ctx, mdl, m, big, "water 12288 PES")


def test_molecules_ragged(gpu_lib, ctx):
    m = synth.model("molecule_pes")
    mdl = gpu_lib.Model(ctx, m)
    fr = synth.molecules(80, seed=13)
    _check(gpu_lib, ctx, mdl, m, fr, "molecules PES")


def test_deterministic_batches_graphs_and_device(gpu_lib, ctx):
    import torch

    m = synth.model("molecule_pes")
    fr = synth.molecules(150, seed=14)
    mdl = gpu_lib.Model(ctx, m)
    E, W, F = gpu_lib.tnep_eval_pes(ctx, mdl, fr)
    E1, W1, F1 = gpu_lib.tnep_eval_pes(ctx, mdl, fr)
    assert np.array_equal(E, E1) and np.array_equal(W, W1) and np.array_equal(F, F1)
    small = gpu_lib.Context(0)
    small.set_option(gpu_lib.OPT_MAX_BATCH_ATOMS, 600)
    graph = gpu_lib.Context(0)
    graph.set_option(gpu_lib.OPT_GRAPHS, 1)
    ms, mg = gpu_lib.Model(small, m), gpu_lib.Model(graph, m)
    for rep in range(3):
        Es, Ws, Fs = gpu_lib.tnep_eval_pes(small, ms, fr)
        Eg, Wg, Fg = gpu_lib.tnep_eval_pes(graph, mg, fr)
        torch.cuda.synchronize()
        for a, b in ((Es, E), (Ws, W), (Fs, F), (Eg, E), (Wg, W), (Fg, F)):
            assert np.array_equal(a, b), rep
    assert graph.graph_counts()[1] >= 2
    # device-resident frames and outputs
    dfr = gpu_lib.DeviceFrames(fr)
    dE = torch.zeros(fr.n_frames, dtype=torch.float64, device="cuda")
    dW = torch.zeros((fr.n_frames, 9), dtype=torch.float64, device="cuda")
    dF = torch.zeros((fr.n_atoms, 3), dtype=torch.float64, device="cuda")
    dU = torch.zeros(fr.n_atoms, dtype=torch.float64, device="cuda")
    gpu_lib.tnep_eval_pes(ctx, mdl, dfr, dE, dW, dF, dU)
    torch.cuda.synchronize()
    assert np.array_equal(dE.cpu().numpy(), E)
    assert np.array_equal(dW.cpu().numpy(), W.reshape(-1, 9))
    assert np.array_equal(dF.cpu().numpy(), F)
    U = np.zeros(fr.n_atoms)
    gpu_lib.tnep_eval_pes(ctx, mdl, fr, per_atom_energy=U)
    assert np.array_equal(dU.cpu().numpy(), U)
    for c in (small, graph):
        c.close()


def test_pes_errors(gpu_lib, ctx):
    m = synth.model("water_pes")
    mdl = gpu_lib.Model(ctx, m)
    md = gpu_lib.Model(ctx, synth.model("water_dipole_small"))
    fr = synth.water_small(1)
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_eval_dipole(ctx, mdl, fr)
    assert e.value.code == -1
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_eval_pes(ctx, md, fr)
    assert e.value.code == -1
