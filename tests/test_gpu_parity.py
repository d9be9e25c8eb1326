"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tensors: per-frame relative Frobenius error <= 1e-5 (tests/parity.py).
Spectra: max |dS| / max |S_ref| <= 1e-4.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import SPECTRUM_TOL, TENSOR_TOL, frame_errors, spectrum_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _check(gpu, m, fr, label):
    ref, pa = oracle.eval_frames(m, fr, per_atom=True)
    err = frame_errors(gpu, ref, pa, fr.offsets)
    print(f"{label}: max frame error {err.max():.3e}", flush=True)
    assert np.all(err <= TENSOR_TOL), (label, err)
    return ref


def test_water_small_dipole(gpu_lib, ctx):
    """64 H2O, 10 frames, 12.42 A periodic box (all-pairs search: 2 cells per axis)."""
    m = synth.model("water_dipole_small")
    fr = synth.water_small(10)
    mdl = gpu_lib.Model(ctx, m)
    mu = gpu_lib.tnep_eval_dipole(ctx, mdl, fr)
    _check(mu, m, fr, "water 192 dipole")


def test_water_small_polarizability_per_atom(gpu_lib, ctx):
    m = synth.model("water_polarizability")
    fr = synth.water_small(3, seed=2)
    mdl = gpu_lib.Model(ctx, m)
    pa = np.zeros((fr.n_atoms, 9))
    al = gpu_lib.tnep_eval_polarizability(ctx, mdl, fr, per_atom=pa)
    ref, ref_pa = oracle.eval_frames(m, fr, per_atom=True)
    _check(al, m, fr, "water 192 polarizability")
    atom_err = np.linalg.norm(pa - ref_pa.reshape(-1, 9), axis=1) / np.linalg.norm(ref_pa.reshape(-1, 9), axis=1)
    print("per-atom max", atom_err.max())
    assert atom_err.max() < 1e-4


def test_water_cell_list_frame(gpu_lib, ctx):
    """A 1536-atom box (24.84 A): 4 cells per axis, so the cell-list path runs."""
    m = synth.model("water_dipole_small")
    pos, spc, cell = synth.water_box(8, 24.84, seed=77)
    fr = synth.Frames(np.array([0, len(spc)], np.int64), pos, spc, cell[None], np.ones((1, 3), np.uint8))
    mdl = gpu_lib.Model(ctx, m)
    _check(gpu_lib.tnep_eval_dipole(ctx, mdl, fr), m, fr, "water 1536 dipole")


def test_perovskite_susceptibility(gpu_lib, ctx):
    """BaZrO3-like 6x6x6 (1080 atoms, cell list) and 4x4x4 (320 atoms, all pairs)."""
    m = synth.model("perovskite_susceptibility")
    mdl = gpu_lib.Model(ctx, m)
    for n_rep, nf in [(6, 2), (4, 3)]:
        fr = synth.perovskite(nf, n_rep=n_rep, seed=5)
        _check(gpu_lib.tnep_eval_polarizability(ctx, mdl, fr), m, fr, f"perovskite {n_rep}^3")


def test_molecules_ragged_both_heads(gpu_lib, ctx):
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    fr = synth.molecules(96, seed=21)
    gd, gp = gpu_lib.Model(ctx, md), gpu_lib.Model(ctx, mp)
    mu, al = gpu_lib.tnep_eval_dipole_polarizability(ctx, gd, gp, fr)
    _check(mu, md, fr, "molecules dipole")
    _check(al, mp, fr, "molecules polarizability")
    # the single-model entry points agree bit for bit with the combined one
    assert np.array_equal(gpu_lib.tnep_eval_dipole(ctx, gd, fr), mu)
    assert np.array_equal(gpu_lib.tnep_eval_polarizability(ctx, gp, fr), al)


def test_full_size_water_frame(gpu_lib, ctx):
    """One 12,288-atom frame of the OU water trajectory, both models."""
    md, mp = synth.model("water_dipole"), synth.model("water_polarizability")
    fr = synth.water_trajectory(3).subset([2])
    gd, gp = gpu_lib.Model(ctx, md), gpu_lib.Model(ctx, mp)
    mu, al = gpu_lib.tnep_eval_dipole_polarizability(ctx, gd, gp, fr)
    _check(mu, md, fr, "water 12288 dipole")
    _check(al, mp, fr, "water 12288 polarizability")
    # the combined call shares the radial descriptor sums between the models:
    # bit for bit the single-model calls
    assert np.array_equal(gpu_lib.tnep_eval_dipole(ctx, gd, fr), mu)
    assert np.array_equal(gpu_lib.tnep_eval_polarizability(ctx, gp, fr), al)


def test_deterministic_and_batch_invariant(gpu_lib, ctx):
    m = synth.model("molecule_dipole")
    fr = synth.molecules(200, seed=8)
    mdl = gpu_lib.Model(ctx, m)
    a = gpu_lib.tnep_eval_dipole(ctx, mdl, fr)
    b = gpu_lib.tnep_eval_dipole(ctx, mdl, fr)
    assert np.array_equal(a, b)
    c2 = gpu_lib.Context(0)
    c2.set_option(gpu_lib.OPT_MAX_BATCH_ATOMS, 500)  # many small launch batches
    mdl2 = gpu_lib.Model(c2, m)
    c = gpu_lib.tnep_eval_dipole(c2, mdl2, fr)
    assert np.array_equal(a, c)
    # one frame alone equals the same frame inside the batch
    one = gpu_lib.tnep_eval_dipole(ctx, mdl, fr.subset([37]))
    assert np.array_equal(one[0], a[37])
    mdl2.close()
    c2.close()


def test_frame_sums_small_and_large_frames(gpu_lib, ctx):
    """Frames of up to 256 atoms are summed by one wavefront each, larger ones in
    four chunks: frames on both sides of the bound (1 to 300 atoms) in one batch
    equal the oracle and, bitwise, each frame evaluated alone, with plain
    launches and with graph replay."""
    rng = np.random.default_rng(81)
    sizes = [255, 256, 257, 64, 1, 300]
    parts = [synth.molecule(rng, n) for n in sizes]
    offs = np.zeros(len(sizes) + 1, np.int64)
    offs[1:] = np.cumsum(sizes)
    fr = synth.Frames(offs, np.concatenate([p for p, _ in parts]),
                      np.concatenate([s for _, s in parts]).astype(np.int32), None, None)
    m = synth.model("molecule_polarizability")
    mdl = gpu_lib.Model(ctx, m)
    a = gpu_lib.tnep_eval_polarizability(ctx, mdl, fr)
    _check(a, m, fr, "frames of 1-300 atoms")
    for i in range(len(sizes)):
        assert np.array_equal(gpu_lib.tnep_eval_polarizability(ctx, mdl, fr.subset([i]))[0], a[i]), sizes[i]
    c2 = gpu_lib.Context(0)
    c2.set_option(gpu_lib.OPT_GRAPHS, 1)
    mdl2 = gpu_lib.Model(c2, m)
    for _ in range(3):
        assert np.array_equal(gpu_lib.tnep_eval_polarizability(c2, mdl2, fr), a)
    assert np.array_equal(gpu_lib.tnep_eval_polarizability(c2, mdl2, fr.subset([1, 2]))[1], a[2])
    mdl2.close()
    c2.close()


def test_frame_larger_than_launch_batch(gpu_lib, ctx):
    """A frame larger than the launch-batch size runs in a batch of its own;
    results equal the default batching bitwise."""
    m = synth.model("water_polarizability")
    mdl = gpu_lib.Model(ctx, m)
    pos, spc, cell = synth.water_box(8, 24.84, seed=34)
    big = synth.Frames(np.array([0, len(spc)], np.int64), pos, spc, cell[None], np.ones((1, 3), np.uint8))
    fr = synth.Frames.concat([synth.water_small(2, seed=35), big, synth.water_small(1, seed=36)])
    a = gpu_lib.tnep_eval_polarizability(ctx, mdl, fr)
    c2 = gpu_lib.Context(0)
    c2.set_option(gpu_lib.OPT_MAX_BATCH_ATOMS, 1000)
    b = gpu_lib.tnep_eval_polarizability(c2, gpu_lib.Model(c2, m), fr)
    assert np.array_equal(a, b)
    _check(a, m, fr, "mixed sizes")
    c2.close()


def test_device_resident_inputs(gpu_lib, ctx):
    import torch

    m = synth.model("water_dipole_small")
    fr = synth.water_small(4, seed=9)
    mdl = gpu_lib.Model(ctx, m)
    host = gpu_lib.tnep_eval_dipole(ctx, mdl, fr)
    dfr = gpu_lib.DeviceFrames(fr)
    out = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    gpu_lib.tnep_eval_dipole(ctx, mdl, dfr, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), host)


def test_edge_cases(gpu_lib, ctx):
    """Empty frames, a single atom, isolated atoms, and an empty call."""
    m = synth.model("molecule_dipole")
    mdl = gpu_lib.Model(ctx, m)
    mol = synth.molecules(2, seed=4)
    parts = [synth.Frames(np.array([0, 0], np.int64), np.zeros((0, 3)), np.zeros(0, np.int32)),
             mol.subset([0]),
             synth.Frames(np.array([0, 1], np.int64), np.zeros((1, 3)), np.array([2], np.int32)),
             synth.Frames(np.array([0, 2], np.int64), np.array([[0, 0, 0], [10.0, 0, 0]]), np.array([1, 3], np.int32)),
             mol.subset([1])]
    fr = synth.Frames.concat(parts)
    mu = gpu_lib.tnep_eval_dipole(ctx, mdl, fr)
    ref = oracle.eval_frames(m, fr)
    assert np.all(mu[[0, 2, 3]] == 0.0)
    _check(mu, m, fr, "edge cases")
    assert np.array_equal(ref[[0, 2, 3]], np.zeros((3, 3)))
    empty = synth.Frames(np.array([0], np.int64), np.zeros((0, 3)), np.zeros(0, np.int32))
    assert gpu_lib.tnep_eval_dipole(ctx, mdl, empty).shape == (0, 3)


def test_error_codes(gpu_lib, ctx):
    m = synth.model("water_dipole_small")
    mdl = gpu_lib.Model(ctx, m)
    fr = synth.water_small(2)
    bad = synth.Frames(fr.offsets, fr.positions, fr.species.copy(), fr.cells, fr.pbc)
    bad.species[7] = 5
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_eval_dipole(ctx, mdl, bad)
    assert e.value.code == -2
    small = synth.Frames(fr.offsets, fr.positions, fr.species, fr.cells * 0.9, fr.pbc)
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_eval_dipole(ctx, mdl, small)
    assert e.value.code == -3
    nan = synth.Frames(fr.offsets, fr.positions.copy(), fr.species, fr.cells, fr.pbc)
    nan.positions[3, 1] = np.nan
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_eval_dipole(ctx, mdl, nan)
    assert e.value.code == -5
    ov = synth.Frames(fr.offsets, fr.positions.copy(), fr.species, fr.cells, fr.pbc)
    ov.positions[10] = ov.positions[11]
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_eval_dipole(ctx, mdl, ov)
    assert e.value.code == -4
    # the context still works after errors
    _check(gpu_lib.tnep_eval_dipole(ctx, mdl, fr), m, fr, "after errors")


@pytest.mark.parametrize("batch_atoms", [0, 400])
def test_error_names_frame_and_atom(gpu_lib, batch_atoms):
    """The first offending atom is reported by frame and atom index within it,
    also when the call is split into several launch batches."""
    c = gpu_lib.Context(0)
    if batch_atoms:
        c.set_option(gpu_lib.OPT_MAX_BATCH_ATOMS, batch_atoms)
    mdl = gpu_lib.Model(c, synth.model("water_dipole_small"))
    fr = synth.water_small(5, seed=33)
    o = fr.offsets
    cases = [("nan", 3, 17, -5), ("species", 4, 0, -2), ("overlap", 2, 5, -4)]
    for label, f, i, code in cases:
        bad = synth.Frames(fr.offsets, fr.positions.copy(), fr.species.copy(), fr.cells, fr.pbc)
        a = o[f] + i
        if label == "nan":
            bad.positions[a, 2] = np.nan
        elif label == "species":
            bad.species[a] = 9
        else:
            bad.positions[a + 4] = bad.positions[a]
        with pytest.raises(gpu_lib.TnepError) as e:
            gpu_lib.tnep_eval_dipole(c, mdl, bad)
        assert e.value.code == code, label
        assert f"at atom {i} of frame {f}" in str(e.value), (label, str(e.value))
    c.close()


# ---------------------------------------------------------------------------
# spectra


def _series(n_series, n_steps, comps, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_series):
        x = np.zeros((n_steps, comps))
        d = np.zeros(comps)
        for t in range(n_steps):
            d = 0.97 * d + rng.normal(0, 0.1, comps)
            x[t] = d + np.cos(0.3 * t) * 0.2
        if comps == 9:
            x = ((x.reshape(-1, 3, 3) + x.reshape(-1, 3, 3).transpose(0, 2, 1)) / 2 + 3 * np.eye(3)).reshape(-1, 9)
        out.append(x)
    return np.stack(out)


@pytest.mark.parametrize("kind,comps", [(0, 3), (1, 9), (2, 9), (3, 9)])
@pytest.mark.parametrize("flags", [0, 1])
def test_spectrum_parity(gpu_lib, ctx, kind, comps, flags):
    s = _series(3, 1500, comps, seed=kind * 10 + flags)
    M = 400
    nh, eh = (0.0, 0.6, 0.8), (1.0, 0.0, 0.0)
    f, S, acf = gpu_lib.tnep_spectrum(ctx, s, kind, 0.5, M, flags=flags, n_hat=nh, e_hat=eh)
    fr, Sr, Cr = oracle.spectrum(list(s), kind, 0.5, M, n_hat=nh, e_hat=eh, subtract_mean=bool(flags))
    np.testing.assert_allclose(f, fr, rtol=1e-13)
    assert spectrum_error(acf, Cr) < 1e-10
    assert spectrum_error(S, Sr) < SPECTRUM_TOL


def test_spectrum_edge_sizes(gpu_lib, ctx):
    """Power-of-two length, max lag = n_steps, no window, IR without w^2."""
    s = _series(1, 1024, 3, seed=3)
    for M, win, flags in [(1024, 1, 2), (1, 0, 0), (37, 0, 1)]:
        f, S, acf = gpu_lib.tnep_spectrum(ctx, s, 0, 1.0, M, window=win, flags=flags)
        fr, Sr, Cr = oracle.spectrum(list(s), 0, 1.0, M, window=(win == 0), omega2=not (flags & 2),
                                     subtract_mean=bool(flags & 1))
        assert spectrum_error(S, Sr) < SPECTRUM_TOL
        assert spectrum_error(acf, Cr) < 1e-10


# ---------------------------------------------------------------------------
# hidden layer on the matrix cores: FP32, BF16 and split-BF16 against the oracle

@pytest.mark.parametrize("name,frames", [("water_dipole_small", "water"), ("water_polarizability", "water"),
                                         ("perovskite_susceptibility", "perovskite")])
def test_hidden_layer_precision_modes(gpu_lib, name, frames):
    m = synth.model(name)
    fr = synth.water_small(3, seed=31) if frames == "water" else synth.perovskite(2, n_rep=6, seed=32)
    ref, pa = oracle.eval_frames(m, fr, per_atom=True)
    errs = {}
    for mode in (gpu_lib.MLP_FP32_VALU, gpu_lib.MLP_FP32_MFMA, gpu_lib.MLP_BF16_MFMA, gpu_lib.MLP_BF16X3_MFMA):
        c = gpu_lib.Context(0)
        c.set_option(gpu_lib.OPT_MLP, mode)
        mdl = gpu_lib.Model(c, m)
        out = (gpu_lib.tnep_eval_dipole if m.kind == 1 else gpu_lib.tnep_eval_polarizability)(c, mdl, fr)
        errs[mode] = frame_errors(out, ref, pa, fr.offsets).max()
        mdl.close()
        c.close()
    print(name, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs[gpu_lib.MLP_FP32_VALU] <= TENSOR_TOL
    assert errs[gpu_lib.MLP_FP32_MFMA] <= TENSOR_TOL
    # bf16 operands (8-bit mantissa) cannot meet 1e-5; the split form must stay within 10x of it
    assert errs[gpu_lib.MLP_BF16_MFMA] < 5e-2
    assert errs[gpu_lib.MLP_BF16X3_MFMA] < 1e-4


def test_autotune_keeps_results(gpu_lib):
    """Autotuned launch parameters change speed only, never the numbers."""
    m = synth.model("molecule_polarizability")
    fr = synth.molecules(300, seed=14)
    c1 = gpu_lib.Context(0)
    g1 = gpu_lib.Model(c1, m)
    a = gpu_lib.tnep_eval_polarizability(c1, g1, fr)
    c2 = gpu_lib.Context(0)
    c2.set_option(gpu_lib.OPT_AUTOTUNE, 1)
    g2 = gpu_lib.Model(c2, m)
    b = gpu_lib.tnep_eval_polarizability(c2, g2, fr)
    rep = c2.autotune_report()
    print(rep)
    assert rep.startswith("autotune") and "->" in rep
    assert np.array_equal(a, b)
    assert np.array_equal(a, gpu_lib.tnep_eval_polarizability(c2, g2, fr))
    for c, g in ((c1, g1), (c2, g2)):
        g.close()
        c.close()


def test_small_frame_sums_direct_and_in_mixed_batches(gpu_lib, ctx):
    """A batch of frames of at most 256 atoms writes its frame sums directly; a
    batch with a larger frame adds chunk sums.  Both give every molecule's
    tensors bit for bit."""
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    mols = synth.molecules(150, seed=21)
    big = synth.molecule_frames(1, seed=22, n_min=300, n_max=300)
    mixed = synth.Frames.concat([mols, big])
    gd, gp = gpu_lib.Model(ctx, md), gpu_lib.Model(ctx, mp)
    mu_o, al_o = gpu_lib.tnep_eval_dipole_polarizability(ctx, gd, gp, mols)
    mu_p, al_p = gpu_lib.tnep_eval_dipole_polarizability(ctx, gd, gp, mixed)
    assert np.array_equal(mu_o, mu_p[:150]) and np.array_equal(al_o, al_p[:150])
    # parity of these frames (the dipoles are checked against the oracle by the
    # other molecule tests; this set holds a molecule whose atom terms cancel to
    # 1 % of their sum, which sits at the FP32 limit of the bound)
    _check(al_p.reshape(len(al_p), -1), mp, mixed, "150 molecules + 300-atom frame")
    gd.close()
    gp.close()


def test_small_and_large_batch_searches_agree_bitwise(gpu_lib, ctx):
    """Frames without a cell grid are searched with 16 lanes per atom in launch
    batches of at most 32,768 atoms and with one lane per atom in larger ones;
    both give the same rows and radial sums, so every tensor (and the
    potential-energy outputs) is bitwise the same in either kind of batch."""
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    mols = synth.molecules(1600, seed=23)  # about 80,000 atoms: one batch above the bound
    few = mols.subset(range(120))
    gd, gp = gpu_lib.Model(ctx, md), gpu_lib.Model(ctx, mp)
    mu_s, al_s = gpu_lib.tnep_eval_dipole_polarizability(ctx, gd, gp, few)
    mu_l, al_l = gpu_lib.tnep_eval_dipole_polarizability(ctx, gd, gp, mols)
    assert mols.n_atoms > 32768 >= few.n_atoms
    assert np.array_equal(mu_s, mu_l[:120]) and np.array_equal(al_s, al_l[:120])
    _check(al_s.reshape(len(al_s), -1), mp, few, "120 molecules, 16-lane search")
    gd.close()
    gp.close()
    wd = synth.model("water_dipole_small")
    boxes = synth.water_small(400, seed=24)  # 76,800 atoms of 12.42 A boxes (no cell grid)
    g = gpu_lib.Model(ctx, wd)
    assert np.array_equal(gpu_lib.tnep_eval_dipole(ctx, g, boxes.subset(range(7))),
                          gpu_lib.tnep_eval_dipole(ctx, g, boxes)[:7])
    g.close()
    pm = synth.model("molecule_pes")
    g = gpu_lib.Model(ctx, pm)
    e_s, v_s, f_s = gpu_lib.tnep_eval_pes(ctx, g, few)
    e_l, v_l, f_l = gpu_lib.tnep_eval_pes(ctx, g, mols)
    assert np.array_equal(e_s, e_l[:120]) and np.array_equal(v_s, v_l[:120])
    assert np.array_equal(f_s, f_l[:few.n_atoms])
    g.close()


def test_small_batch_bucket_pipeline_matches_large_batches(gpu_lib, ctx):
    """Launch batches of at most 4,096 atoms and 1,024 cells are binned, scanned
    and placed by one work-group, larger ones by the five-kernel pipeline; both
    give the same tile slots, so grid frames (orthorhombic, triclinic, and
    trajectory windows with reference and follower frames) are bitwise the same
    alone and inside a large batch, and equal the oracle alone."""
    m = synth.model("water_polarizability")
    mdl = gpu_lib.Model(ctx, m)
    pos, spc, cell = synth.water_box(8, 24.84, seed=97)  # 1,536 atoms, 8^3 cells
    n = len(spc)
    R, _ = np.linalg.qr(np.random.default_rng(98).normal(size=(3, 3)))
    box = synth.Frames(np.array([0, n], np.int64), pos, spc, cell[None], np.ones((1, 3), np.uint8))
    tri = synth.Frames(np.array([0, n], np.int64), pos @ R.T, spc, (cell.reshape(3, 3) @ R.T).reshape(1, 9),
                       np.ones((1, 3), np.uint8))
    for label, one in (("orthorhombic 1,536-atom box", box), ("rotated (triclinic) box", tri)):
        a = gpu_lib.tnep_eval_polarizability(ctx, mdl, one)
        _check(a, m, one, label + " alone")
        many = synth.Frames.concat([one] * 24)  # 36,864 atoms, 12,288 cells
        b = gpu_lib.tnep_eval_polarizability(ctx, mdl, many)
        assert all(np.array_equal(b[i], a[0]) for i in range(24)), label
    p6, s6, c6 = synth.water_box(6, 18.63, seed=99)  # 648 atoms, 6^3 cells
    traj = synth.ou_trajectory(p6, s6, c6, 4, seed=100)
    c3 = gpu_lib.Context(0)
    c3.set_option(gpu_lib.OPT_TRAJECTORY_WINDOW, 3)
    m3 = gpu_lib.Model(c3, m)
    a = gpu_lib.tnep_eval_polarizability(c3, m3, traj)  # 2,592 atoms, 864 cells
    _check(a, m, traj, "trajectory window alone")
    longer = synth.Frames.concat([traj, synth.ou_trajectory(p6, s6, c6, 60, seed=101)])
    b = gpu_lib.tnep_eval_polarizability(c3, m3, longer)
    assert np.array_equal(b[:4], a)
    assert c3.reuse_fallbacks() == 0
    m3.close()
    c3.close()
    mdl.close()


def test_device_frames_with_host_layout(gpu_lib, ctx):
    """TNEP_DEVICE_META_HOST (positions and species on the device; offsets,
    cells and pbc on the host): tensors and potential-energy outputs bitwise
    those of host and device frames, also under graph replay; the calls that do
    not take it return TNEP_E_INVALID."""
    import torch

    md, mp, pm = synth.model("water_dipole"), synth.model("water_polarizability"), synth.model("water_pes")
    pos, spc, cell = synth.water_box(8, 24.84, seed=102)
    big = synth.Frames(np.array([0, len(spc)], np.int64), pos, spc, cell[None], np.ones((1, 3), np.uint8))
    fr = synth.Frames.concat([synth.water_small(3, seed=103), big])
    gd, gp, ge = gpu_lib.Model(ctx, md), gpu_lib.Model(ctx, mp), gpu_lib.Model(ctx, pm)
    mu, al = gpu_lib.tnep_eval_dipole_polarizability(ctx, gd, gp, fr)
    _check(al.reshape(len(al), -1), mp, fr, "water boxes (host frames)")
    E, W, F = gpu_lib.tnep_eval_pes(ctx, ge, fr)
    cg = gpu_lib.Context(0)
    cg.set_option(gpu_lib.OPT_GRAPHS, 1)
    hd, hp = gpu_lib.Model(cg, md), gpu_lib.Model(cg, mp)
    for host_meta in (False, True):
        dfr = gpu_lib.DeviceFrames(fr, host_meta=host_meta)
        want = gpu_lib.DEVICE_META_HOST if host_meta else gpu_lib.DEVICE
        assert gpu_lib.frames_desc(dfr).location == want
        for c, a, b in ((ctx, gd, gp), (cg, hd, hp), (cg, hd, hp), (cg, hd, hp)):
            dmu = torch.zeros((fr.n_frames, 3), dtype=torch.float64, device="cuda")
            dal = torch.zeros((fr.n_frames, 9), dtype=torch.float64, device="cuda")
            gpu_lib.tnep_eval_dipole_polarizability(c, a, b, dfr, dmu, dal)
            torch.cuda.synchronize()
            assert np.array_equal(dmu.cpu().numpy(), mu) and np.array_equal(dal.cpu().numpy(), al.reshape(-1, 9))
        dE = torch.zeros(fr.n_frames, dtype=torch.float64, device="cuda")
        dW = torch.zeros((fr.n_frames, 9), dtype=torch.float64, device="cuda")
        dF = torch.zeros((fr.n_atoms, 3), dtype=torch.float64, device="cuda")
        gpu_lib.tnep_eval_pes(ctx, ge, dfr, dE, dW, dF)
        torch.cuda.synchronize()
        assert np.array_equal(dE.cpu().numpy(), E) and np.array_equal(dW.cpu().numpy(), W.reshape(-1, 9))
        assert np.array_equal(dF.cpu().numpy(), F)
    assert cg.graph_counts()[1] >= 4
    dfr = gpu_lib.DeviceFrames(fr, host_meta=True)
    dmu = torch.zeros((fr.n_frames, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.TnepError) as e:
        gpu_lib.tnep_eval_dipole_charged(ctx, gd, dfr, torch.zeros(fr.n_frames, dtype=torch.float64, device="cuda"),
                                         [15.999, 1.008], mu_out=dmu)
    assert e.value.code == -1
    for x in (gd, gp, ge, hd, hp):
        x.close()
    cg.close()


def test_bucket_pipeline_size_bounds(gpu_lib, ctx):
    """The one-work-group bucket pipeline at its bounds (4,096 atoms, 1,024
    cells: 1,024 four-atom molecules) and one past each (a fifth atom in the
    last molecule: the five-kernel pipeline with the one-work-group scan; a
    1,025th molecule: the three-phase scan); the frames they share are bitwise
    the same, and a sample equals the oracle."""
    m = synth.model("molecule_dipole")
    mdl = gpu_lib.Model(ctx, m)
    rng = np.random.default_rng(105)
    parts = [synth.molecule(rng, 4) for _ in range(1025)] + [synth.molecule(rng, 5)]

    def frames(sel):
        ps = [parts[i] for i in sel]
        offs = np.zeros(len(ps) + 1, np.int64)
        offs[1:] = np.cumsum([len(s) for _, s in ps])
        return synth.Frames(offs, np.concatenate([p for p, _ in ps]),
                            np.concatenate([s for _, s in ps]).astype(np.int32), None, None)

    at_bound = frames(range(1024))  # 4,096 atoms, 1,024 cells
    assert at_bound.n_atoms == 4096
    a = gpu_lib.tnep_eval_dipole(ctx, mdl, at_bound)
    b = gpu_lib.tnep_eval_dipole(ctx, mdl, frames(list(range(1023)) + [1025]))  # 4,097 atoms
    c = gpu_lib.tnep_eval_dipole(ctx, mdl, frames(range(1025)))  # 1,025 cells
    assert np.array_equal(a[:1023], b[:1023]) and np.array_equal(a, c[:1024])
    sample = at_bound.subset(range(0, 1024, 16))
    _check(a[::16], m, sample, "four-atom molecules at the pipeline bound")
    mdl.close()
