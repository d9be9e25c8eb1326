#!/usr/bin/env python3
"""Benchmark: TNEP atom-frames/s for dipole + polarizability on one MI355X.

Workload (one step = the whole hot path over one synthetic job):
  liquid-water box of 4096 H2O (12,288 atoms, 49.7 A, periodic), 2000-frame
  Ornstein-Uhlenbeck displacement trajectory (sigma 0.02 A, tau 50 steps),
  dipole model + polarizability model (scalar + tensor heads), NEP
  descriptor r_c 6/4 A, n_max 4/4, basis 8/8, l_max 4 + four-body, 30 tanh
  neurons; then the IR spectrum of mu(t) and the isotropic / anisotropic
  Raman spectra of alpha(t) (dt = 1 fs, max lag 500).
Inputs (positions, species, frame offsets, cells) are resident in HBM when
the timed region starts; outputs stay in HBM.

Printed: one JSON line with the metric, a roofline record for the dominant
kernel (the polarizability evaluation kernel, FP32 VALU bound) measured with
HIP events inside the library, and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X, published FP32 vector peak
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "eval_polarizability_water12288_traffic.md")


RADIAL_TERMS_SEARCHED = 9  # radial basis size whose sums the neighbour search forms


def radial_forward_flops(model):
    """Forward share of f_R: basis and accumulation of the radial sums, which
    the neighbour search forms for models of RADIAL_TERMS_SEARCHED radial
    terms, so that their evaluation kernels load them."""
    nR, KR = model.n_max_radial + 1, model.basis_radial + 1
    return 2 * nR * KR + 4 * KR + nR + 20


def flops_per_atom_frame(model, n_rad_mean, n_ang_mean, radial_forward=None):
    """Algorithmic FP32 work per atom-frame of the evaluation kernel (FMA = 2
    flops), no recomputation: f_R per radial pair, f_A per angular pair, f_atom
    per atom; without the forward radial share when the kernel loads the
    radial sums that the neighbour search formed (by default: when the model
    has RADIAL_TERMS_SEARCHED radial terms)."""
    if radial_forward is None:
        radial_forward = model.basis_radial + 1 != RADIAL_TERMS_SEARCHED
    nR, nA = model.n_max_radial + 1, model.n_max_angular + 1
    KR, KA = model.basis_radial + 1, model.basis_angular + 1
    L = (model.l_max + 1) ** 2 - 1
    D, H = model.dim, model.n_hidden
    f_R = 4 * nR * KR + 12 * KR + 3 * nR + 40
    f_A = 4 * nA * KA + 12 * KA + 6 * nA * L + 8 * L + 180
    heads = len(model.heads)
    f_atom = 4 * D * H + (2 * D * H if heads == 2 else 0) + 10 * H * heads + 4 * nA * L + \
        (120 * nA if model.four_body else 0) + 4 * D
    total = n_rad_mean * f_R + n_ang_mean * f_A + f_atom
    return total if radial_forward else total - n_rad_mean * radial_forward_flops(model)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels_eval.hip", "tnep_math.h", "radial_basis.h"):
        with open(os.path.join(ROOT, "paper_2312_05233_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(atoms_per_launch):
    """HBM bytes per launch of the evaluation kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_RECORD):
        return None
    txt = open(TRAFFIC_RECORD).read()
    m_hash = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", txt)
    m_bpa = re.search(r"hbm_bytes_per_atom:\s*([0-9.eE+-]+)", txt)
    if not m_hash or not m_bpa or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bpa.group(1)) * atoms_per_launch


def cpu_baseline(frames, md, mp, n_sample, gpu_mu, gpu_alpha):
    """The FP64 oracle on frames 0..n_sample-1 with all its threads, then on
    frame 0 with one thread (the per-core rate)."""
    import oracle

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import frame_errors

    idx = list(range(n_sample))
    sub = frames.subset(idx)
    cores = oracle.max_threads()
    t0 = time.perf_counter()
    mu_ref, mu_pa = oracle.eval_frames(md, sub, per_atom=True)
    al_ref, al_pa = oracle.eval_frames(mp, sub, per_atom=True)
    dt = time.perf_counter() - t0
    atoms = sub.n_atoms
    err_mu = frame_errors(gpu_mu[idx], mu_ref, mu_pa, sub.offsets).max()
    err_al = frame_errors(gpu_alpha[idx], al_ref.reshape(-1, 9), al_pa, sub.offsets).max()
    one = frames.subset([0])
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.eval_frames(md, one)
        oracle.eval_frames(mp, one)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    return {
        "value": atoms / dt, "unit": "atom-frames/s", "cores": cores, "kind": "oracle",
        "sample": f"frames 0..{n_sample - 1} of the trajectory ({atoms} atom-frames), dipole + polarizability "
                  f"models, FP64, {dt:.1f} s wall",
        "single_thread": {"value": one.n_atoms / dt1, "unit": "atom-frames/s", "cores": 1,
                          "sample": f"frame 0 ({one.n_atoms} atom-frames), dipole + polarizability models, FP64, "
                                    f"{dt1:.1f} s wall"},
    }, float(err_mu), float(err_al)


def _timed(fn, steps, warmup):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_perovskite(args):
    """BaZrO3-like 12x12x12 supercell (8,640 atoms), batches of 64 frames,
    susceptibility model (H = 50); FP32 vs matrix-core hidden layers, with the
    error of each against the FP64 oracle on two frames."""
    import torch

    import oracle
    from paper_2312_05233_amd import tnep

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import frame_errors

    frames = synth.perovskite(64)
    m = synth.model("perovskite_susceptibility")
    dfr = tnep.DeviceFrames(frames)
    out = torch.zeros((frames.n_frames, 9), dtype=torch.float64, device="cuda")
    ref, pa = oracle.eval_frames(m, frames.subset([0, 1]), per_atom=True)
    modes = {}
    for mode, name in ((tnep.MLP_FP32_VALU, "fp32_valu"), (tnep.MLP_FP32_MFMA, "fp32_mfma"),
                       (tnep.MLP_BF16_MFMA, "bf16_mfma"), (tnep.MLP_BF16X3_MFMA, "bf16x3_mfma")):
        ctx = tnep.Context(0)
        ctx.set_option(tnep.OPT_MLP, mode)
        gm = tnep.Model(ctx, m)
        t = _timed(lambda: tnep.tnep_eval_polarizability(ctx, gm, dfr, out), args.steps, args.warmup)
        err = frame_errors(out[:2].cpu().numpy(), ref.reshape(2, 9), pa, frames.subset([0, 1]).offsets).max()
        modes[name] = {"atom_frames_per_s": frames.n_atoms / t, "ms_per_batch": 1e3 * t, "max_frame_error": float(err)}
        gm.close()
        ctx.close()
    print(json.dumps({"metric": "TNEP atom-frames/s (susceptibility) at FP32 tol", "value": modes["fp32_valu"][
        "atom_frames_per_s"], "unit": "atom-frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "dtype": "f32", "data": "synthetic", "config": {
            "workload": "perovskite Ba/Zr/O 12x12x12 (8640 atoms, a=4.19 A, sigma 0.08 A), batch of 64 frames, "
                        "susceptibility model rc 7/5 A, n_max 6/4, H=50"}, "hidden_layer_modes": modes}), flush=True)


def bench_molecules(args):
    """8192 ragged vacuum molecules (20-80 atoms, C/H/N/O/F), dipole +
    polarizability heads in one call (one launch per model per batch)."""
    import torch

    from paper_2312_05233_amd import tnep

    frames = synth.molecules(8192)
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    ctx = tnep.Context(0)
    gd, gp = tnep.Model(ctx, md), tnep.Model(ctx, mp)
    dfr = tnep.DeviceFrames(frames)
    mu = torch.zeros((frames.n_frames, 3), dtype=torch.float64, device="cuda")
    al = torch.zeros((frames.n_frames, 9), dtype=torch.float64, device="cuda")
    step = lambda: tnep.tnep_eval_dipole_polarizability(ctx, gd, gp, dfr, mu, al)  # noqa: E731
    t = _timed(step, args.steps, args.warmup)
    # the same call with its launch batch replayed as a HIP graph (TNEP_OPT_GRAPHS)
    gctx = tnep.Context(0)
    gctx.set_option(tnep.OPT_GRAPHS, 1)
    ggd, ggp = tnep.Model(gctx, md), tnep.Model(gctx, mp)
    gmu, gal = torch.zeros_like(mu), torch.zeros_like(al)
    t_graph = _timed(lambda: tnep.tnep_eval_dipole_polarizability(gctx, ggd, ggp, dfr, gmu, gal), args.steps,
                     args.warmup)
    torch.cuda.synchronize()
    graph_equal = bool(torch.equal(gmu, mu) and torch.equal(gal, al))
    gctx.close()
    # kernel times and pair counts from an instrumented pass
    ctx.set_option(tnep.OPT_TIMING, 1)
    ctx.reset_timing()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kt = {name: ctx.kernel_time(k)[0] / args.steps for name, k in (
        ("neighbors", tnep.KERNEL_NEIGHBORS), ("eval_dipole", tnep.KERNEL_EVAL_DIPOLE),
        ("eval_polarizability", tnep.KERNEL_EVAL_POLARIZABILITY), ("frame_reduce", tnep.KERNEL_FRAME_REDUCE))}
    atoms, rad, ang = ctx.pair_counts()
    print(json.dumps({"metric": "TNEP atom-frames/s (dipole+polarizability) at FP32 tol", "value": frames.n_atoms / t,
                      "unit": "atom-frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": 1e3 * t, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "8192 vacuum molecules, 20-80 atoms (%d atoms), C/H/N/O/F, dipole + "
                                             "polarizability" % frames.n_atoms},
                      "kernels_ms_per_step": kt, "mean_radial_neighbors": rad / atoms,
                      "mean_angular_neighbors": ang / atoms,
                      "graph_replay": {"atom_frames_per_s": frames.n_atoms / t_graph, "ms_per_step": 1e3 * t_graph,
                                       "bitwise_equal_to_plain": graph_equal}}), flush=True)


def bench_pes(args):
    """Potential-energy surface (Sec. 2.1) on the 12,288-atom water box: energy,
    virial and forces of every frame, device-resident inputs and outputs; the
    evaluation kernel's time from HIP events and its FP32 roofline; errors of
    one frame against the FP64 oracle."""
    import torch

    import oracle
    from paper_2312_05233_amd import tnep

    n_frames = min(args.frames, 340)
    frames = synth.water_trajectory(n_frames)
    m = synth.model("water_pes")
    ctx = tnep.Context(0)
    gm = tnep.Model(ctx, m)
    dfr = tnep.DeviceFrames(frames)
    E = torch.zeros(frames.n_frames, dtype=torch.float64, device="cuda")
    W = torch.zeros((frames.n_frames, 9), dtype=torch.float64, device="cuda")
    F = torch.zeros((frames.n_atoms, 3), dtype=torch.float64, device="cuda")
    step = lambda: tnep.tnep_eval_pes(ctx, gm, dfr, E, W, F)  # noqa: E731
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_option(tnep.OPT_TIMING, 1)
    ctx.reset_timing()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    ms_e, n = ctx.kernel_time(tnep.KERNEL_EVAL_PES)
    ms_f, _ = ctx.kernel_time(tnep.KERNEL_PES_FORCES)
    ms = ms_e + ms_f  # the two kernels that evaluate the model, per launch batch
    atoms, rad, ang = ctx.pair_counts()
    kt = {name: ctx.kernel_time(k)[0] / args.steps for name, k in (
        ("neighbors", tnep.KERNEL_NEIGHBORS), ("eval_pes", tnep.KERNEL_EVAL_PES),
        ("pes_forces", tnep.KERNEL_PES_FORCES), ("frame_reduce", tnep.KERNEL_FRAME_REDUCE))}
    flop = flops_per_atom_frame(m, rad / atoms, ang / atoms)
    atoms_per_launch = frames.n_atoms / (n / args.steps)
    achieved = flop * atoms_per_launch / (ms / n * 1e-3) / 1e12
    # errors of one frame against the oracle
    sub = frames.subset([0])
    Er, Wr, Fr, Ur = oracle.eval_pes(m, sub, per_atom=True)
    n0 = sub.n_atoms
    errs = {"energy_vs_sum_abs_site_energies": float(abs(E[0].item() - Er[0]) / np.abs(Ur).sum()),
            "virial_frobenius": float(np.linalg.norm(W[0].cpu().numpy() - Wr[0].reshape(9)) / np.linalg.norm(Wr[0])),
            "forces_frobenius": float(np.linalg.norm(F[:n0].cpu().numpy() - Fr) / np.linalg.norm(Fr))}
    print(json.dumps({
        "metric": "NEP PES atom-frames/s (energy + virial + forces) at FP32 tol", "value": frames.n_atoms / t,
        "unit": "atom-frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "water 4096 H2O (12288 atoms, 49.7 A PBC) x %d-frame OU trajectory, potential-energy "
                               "model rc 6/4 A, n_max 4/4, basis 8/8, l_max 4 + 4-body, H=30" % n_frames},
        "roofline": {"kernel": "k_eval<5,5,9,9,4-body,potential> + k_pes_forces", "bound": "alu",
                     "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s", "frac": achieved / 157.3,
                     "flop_per_atom_frame": flop, "atoms_per_launch": atoms_per_launch,
                     "avg_launch_ms": ms / n, "avg_launch_ms_eval": ms_e / n, "avg_launch_ms_forces": ms_f / n,
                     "mean_radial_neighbors": rad / atoms, "mean_angular_neighbors": ang / atoms,
                     "note": "flops counted once per pair; the force kernel re-evaluates each pair term from "
                             "the neighbour's side"},
        "kernels_ms_per_step": kt, "errors_vs_oracle_frame0": errs}), flush=True)


def bench_population(args):
    """Loss of an evolution-strategy population (Sec. 2.4): 50 individuals of
    the susceptibility model over a training set of 800 perovskite structures
    (4x4x4 supercells, 320 atoms), against synthetic reference tensors; all
    inputs device-resident.  Errors against the oracle and the oracle's own
    rate on a sample of individuals and structures."""
    import torch

    import oracle
    from paper_2312_05233_amd import tnep

    n_pop, n_struct = 50, 800
    frames = synth.perovskite_frames(4, 4.19, n_struct, 5)
    base = synth.model("perovskite_susceptibility")
    z0 = synth.pack_params(base)
    rng = np.random.default_rng(6)
    zs = z0[None, :] * (1.0 + 0.02 * rng.normal(size=(n_pop, z0.size)))
    ref = rng.normal(size=(n_struct, 9))
    ctx = tnep.Context(0)
    dfr = tnep.DeviceFrames(frames)
    dref = torch.as_tensor(ref).cuda()
    step = lambda: tnep.tnep_population_loss(ctx, base, zs, dfr, dref, 0.05, 0.05)  # noqa: E731
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_option(tnep.OPT_TIMING, 1)
    ctx.reset_timing()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    ms, n = ctx.kernel_time(tnep.KERNEL_EVAL_POLARIZABILITY)
    atoms, rad, ang = ctx.pair_counts()
    kt = {name: ctx.kernel_time(k)[0] / args.steps for name, k in (
        ("neighbors", tnep.KERNEL_NEIGHBORS), ("eval_polarizability", tnep.KERNEL_EVAL_POLARIZABILITY),
        ("frame_reduce", tnep.KERNEL_FRAME_REDUCE))}
    flop = flops_per_atom_frame(base, rad / atoms, ang / atoms)
    atoms_per_launch = frames.n_atoms * n_pop / (n / args.steps)
    achieved = flop * atoms_per_launch / (ms / n * 1e-3) / 1e12
    evals = frames.n_atoms * n_pop
    # oracle on a sample: 4 individuals x 160 structures (also the error check)
    sub = frames.subset(list(range(160)))
    t1 = time.perf_counter()
    loss_r, rmse_r = oracle.population_loss(base, zs[:4], sub, ref[:160], 0.05, 0.05)
    t_cpu = time.perf_counter() - t1
    loss_g, rmse_g = tnep.tnep_population_loss(ctx, base, zs[:4], sub, ref[:160], 0.05, 0.05)
    print(json.dumps({
        "metric": "population loss: atom-evaluations/s (individuals x atoms) at FP32 tol", "value": evals / t,
        "unit": "atom-evaluations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * t, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "population of %d susceptibility models (rc 7/5 A, n_max 6/4, H=50) x %d perovskite "
                               "structures (4x4x4 Ba/Zr/O, 320 atoms, sigma 0.08 A), synthetic reference tensors"
                               % (n_pop, n_struct)},
        "generations_per_s": 1.0 / t,
        "roofline": {"kernel": "k_eval (polarizability)", "bound": "alu", "achieved": achieved, "peak": 157.3,
                     "unit": "TFLOP/s", "frac": achieved / 157.3, "flop_per_atom_frame": flop,
                     "atoms_per_launch": atoms_per_launch, "avg_launch_ms": ms / n},
        "kernels_ms_per_step": kt,
        "errors_vs_oracle_sample": {"rmse_abs_max": float(np.abs(rmse_g - rmse_r).max()),
                                    "loss_abs_max": float(np.abs(loss_g - loss_r).max()),
                                    "rmse_ref_min": float(rmse_r.min())},
        "cpu_baseline": {"value": 4 * sub.n_atoms / t_cpu, "unit": "atom-evaluations/s",
                         "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                         "kind": "oracle", "sample": "4 individuals x 160 structures (51,200 atoms)"}}), flush=True)


def bench_variants(args):
    """Model and cell variants on the water trajectory (340 frames x 12,288
    atoms, dipole + polarizability in one call): the shared four-body models
    (reference), per-species networks, the five-body term, and the same
    lattice described by a skewed basis, and a rotated copy (a triclinic cell in
    every basis); then charged molecules (8192
    ragged molecules, mu_r + Q e r_COM) against the plain dipole call.  Each
    with its largest frame error against the FP64 oracle on a sample."""
    import torch

    import oracle
    from paper_2312_05233_amd import tnep

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import frame_errors

    n_frames = min(args.frames, 340)
    base = synth.water_trajectory(n_frames)
    shear = np.array([[1, 0, 0], [1, 1, 0], [0, 1, 1]], np.float64)  # same lattice, skewed basis
    tri_cells = np.stack([(shear @ c.reshape(3, 3)).reshape(9) for c in base.cells])
    tric = synth.Frames(base.offsets, base.positions, base.species, tri_cells, base.pbc)
    # a rotated copy: the lattice vectors are not along the axes in any basis
    rot, _ = np.linalg.qr(np.random.default_rng(8).normal(size=(3, 3)))
    rot_cells = np.stack([(c.reshape(3, 3) @ rot.T).reshape(9) for c in base.cells])
    rotated = synth.Frames(base.offsets, base.positions @ rot.T, base.species, rot_cells, base.pbc)

    def second(name):
        seed, kind, species, desc = synth.MODEL_SPECS[name]
        return synth.with_descriptor_of(synth.make_model(seed + 50, kind, species, **desc), synth.model(name))

    variants = {
        "shared_4body": (synth.model("water_dipole"), synth.model("water_polarizability"), base),
        "per_species": (synth.per_species_model([synth.model("water_dipole"), second("water_dipole")], [0, 1]),
                        synth.per_species_model([synth.model("water_polarizability"),
                                                 second("water_polarizability")], [1, 0]), base),
        "five_body": (synth.model("water_dipole_5b"), synth.model("water_polarizability_5b"), base),
        "skewed_basis": (synth.model("water_dipole"), synth.model("water_polarizability"), tric),
        "triclinic_rotated": (synth.model("water_dipole"), synth.model("water_polarizability"), rotated),
    }
    results = {}
    ctx = tnep.Context(0)
    for name, (md, mp, fr) in variants.items():
        gd, gp = tnep.Model(ctx, md), tnep.Model(ctx, mp)
        dfr = tnep.DeviceFrames(fr)
        mu = torch.zeros((fr.n_frames, 3), dtype=torch.float64, device="cuda")
        al = torch.zeros((fr.n_frames, 9), dtype=torch.float64, device="cuda")
        t = _timed(lambda: tnep.tnep_eval_dipole_polarizability(ctx, gd, gp, dfr, mu, al), args.steps, args.warmup)
        sub = fr.subset([0])
        rm, pm = oracle.eval_frames(md, sub, per_atom=True)
        ra, pa = oracle.eval_frames(mp, sub, per_atom=True)
        err = max(frame_errors(mu[:1].cpu().numpy(), rm, pm, sub.offsets).max(),
                  frame_errors(al[:1].cpu().numpy(), ra.reshape(1, 9), pa, sub.offsets).max())
        results[name] = {"atom_frames_per_s": fr.n_atoms / t, "ms_per_call": 1e3 * t,
                         "max_frame_error_vs_oracle": float(err)}
        gd.close()
        gp.close()
    # charged molecules
    masses = [12.011, 1.008, 14.007, 15.999, 18.998]
    mol = synth.molecules(8192)
    q = np.random.default_rng(7).integers(-2, 3, mol.n_frames).astype(np.float64)
    md = synth.model("molecule_dipole")
    gd = tnep.Model(ctx, md)
    dmol = tnep.DeviceFrames(mol)
    dq = torch.as_tensor(q).cuda()
    mu = torch.zeros((mol.n_frames, 3), dtype=torch.float64, device="cuda")
    t_plain = _timed(lambda: tnep.tnep_eval_dipole(ctx, gd, dmol, mu), args.steps, args.warmup)
    t_ch = _timed(lambda: tnep.tnep_eval_dipole_charged(ctx, gd, dmol, dq, masses, 1.0, mu), args.steps, args.warmup)
    sub = mol.subset(list(range(32)))
    ref = oracle.dipole_charged(md, sub, q[:32], masses, 1.0)
    results["charged_molecules"] = {"atom_frames_per_s": mol.n_atoms / t_ch, "ms_per_call": 1e3 * t_ch,
                                    "plain_dipole_ms_per_call": 1e3 * t_plain,
                                    "max_frame_error_vs_oracle": float(frame_errors(mu[:32].cpu().numpy(), ref).max())}
    print(json.dumps({
        "metric": "TNEP atom-frames/s of model and cell variants at FP32 tol",
        "value": results["shared_4body"]["atom_frames_per_s"], "unit": "atom-frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "water 4096 H2O (12288 atoms, 49.7 A) x %d-frame OU trajectory, dipole + "
                               "polarizability per call; variants: per-species networks, five-body term, a skewed "
                               "basis of the same lattice, a rotated (triclinic) copy; 8192 charged vacuum molecules"
                               % n_frames},
        "variants": results}), flush=True)


def bench_latency(args):
    """Calls of few atoms on device-resident frames, one synchronous call at a
    time, in the default layout (one lane per atom) and the pair-parallel
    layout (TNEP_OPT_PAIR_PARALLEL: 16 lanes per atom): mean wall time per call
    and the evaluation kernels' mean time per call (HIP events); then both
    layouts with the frames' layout (offsets, cells, pbc) in host memory
    (TNEP_DEVICE_META_HOST: no metadata read back from the device), and both
    on host frames (inputs copied in and tensors returned within the call)."""
    import torch

    from paper_2312_05233_amd import tnep

    mol = synth.molecules(64, seed=3)
    water = synth.water_small(10)
    mu_m, al_m = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    cases = [("10 x 192 water atoms, dipole", water, [synth.model("water_dipole_small")]),
             ("1 x 192 water atoms, dipole + polarizability", water.subset([0]),
              [synth.model("water_dipole"), synth.model("water_polarizability")]),
             ("1 molecule, dipole + polarizability", mol.subset([0]), [mu_m, al_m]),
             ("64 molecules, dipole + polarizability", mol, [mu_m, al_m])]
    n = max(args.steps, 50)
    out = []
    for label, frames, models in cases:
        rec = {"workload": label, "atoms": frames.n_atoms}
        for pp, where in ((0, "device"), (1, "device"), (0, "host_layout"), (1, "host_layout"), (0, "host"),
                          (1, "host")):
            ctx = tnep.Context(0)
            ctx.set_option(tnep.OPT_PAIR_PARALLEL, pp)
            gm = [tnep.Model(ctx, m) for m in models]
            if where == "host":
                dfr, mu, al = frames, np.zeros((frames.n_frames, 3)), np.zeros((frames.n_frames, 3, 3))
            else:
                dfr = tnep.DeviceFrames(frames, host_meta=where == "host_layout")
                mu = torch.zeros((frames.n_frames, 3), dtype=torch.float64, device="cuda")
                al = torch.zeros((frames.n_frames, 9), dtype=torch.float64, device="cuda")
            if len(gm) == 2:
                step = lambda: tnep.tnep_eval_dipole_polarizability(ctx, gm[0], gm[1], dfr, mu, al)  # noqa: E731
            else:
                step = lambda: tnep.tnep_eval_dipole(ctx, gm[0], dfr, mu)  # noqa: E731

            def one_call():
                step()
                torch.cuda.synchronize()

            t = _timed(one_call, n, 5)
            ctx.set_option(tnep.OPT_TIMING, 1)
            ctx.reset_timing()
            for _ in range(n):
                one_call()
            ev = sum(ctx.kernel_time(k)[0] for k in (tnep.KERNEL_EVAL_DIPOLE, tnep.KERNEL_EVAL_POLARIZABILITY)) / n
            name = ("pair_parallel" if pp else "default") + ("" if where == "device" else "_" + where)
            rec[name] = {"us_per_call": 1e6 * t, "eval_kernels_us_per_call": 1e3 * ev}
            for g in gm:
                g.close()
            ctx.close()
        out.append(rec)
    print(json.dumps({"metric": "latency of one synchronous call", "unit": "us", "n_gpus": 1, "calls": n,
                      "data": "synthetic", "cases": out}), flush=True)


def bench_spectra(args):
    """Paper-scale Raman spectra of a recorded susceptibility: 20 runs of
    10^5 samples (500 ps at 5 fs), pushed through the streaming accumulator in
    device-resident chunks, then Z(XX)Z-bar, Z(XY)Z-bar and a 180-point
    crystal-rotation map; the whole-run map call on the same data; the FP64
    oracle (direct lag sums) on a bounded sample for the CPU baseline."""
    import torch

    import oracle
    from paper_2312_05233_amd import tnep

    runs = synth.susceptibility_runs(20, 100000)
    M, dt, chunk = 2000, 5.0, 10000
    ctx = tnep.Context(0)
    dev = torch.as_tensor(runs).cuda()
    phis = np.linspace(0.0, np.pi, 90, endpoint=False)
    nh = np.concatenate([np.stack([np.cos(phis), np.sin(phis), 0 * phis], 1)] * 2)
    eh = np.concatenate([np.stack([np.cos(phis), np.sin(phis), 0 * phis], 1),
                         np.stack([-np.sin(phis), np.cos(phis), 0 * phis], 1)])

    def stream_all():
        st = tnep.AcfStream(ctx, tnep.RAMAN_MAP, M)
        for r in range(dev.shape[0]):
            for pos in range(0, dev.shape[1], chunk):
                st.push(dev[r, pos:pos + chunk])
            st.end_run()
        f, S = st.raman_map(dt, nh, eh)
        st.close()
        return f, S

    stream_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f, S = stream_all()
    t_stream = (time.perf_counter() - t0) / args.steps
    fw = torch.zeros(M + 1, dtype=torch.float64, device="cuda")
    Sw = torch.zeros((len(nh), M + 1), dtype=torch.float64, device="cuda")
    tnep.tnep_raman_map(ctx, dev, dt, M, nh, eh, freq=fw, intensity=Sw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tnep.tnep_raman_map(ctx, dev, dt, M, nh, eh, freq=fw, intensity=Sw)
    torch.cuda.synchronize()
    t_whole = (time.perf_counter() - t0) / args.steps
    agree = float(np.abs(Sw.cpu().numpy() - S).max() / np.abs(S).max())
    # oracle: the two Porto geometries of one run, truncated to 20,000 samples
    sample = [runs[0, :20000]]
    t0 = time.perf_counter()
    _, Sr = oracle.raman_map(sample, dt, M, nh[[0, 90]], eh[[0, 90]])
    t_cpu = time.perf_counter() - t0
    st = tnep.AcfStream(ctx, tnep.RAMAN_MAP, M)
    st.push(sample[0])
    st.end_run()
    _, Sg = st.raman_map(dt, nh[[0, 90]], eh[[0, 90]])
    st.close()
    err = float(max(np.abs(Sg[o] - Sr[o]).max() / np.abs(Sr[o]).max() for o in range(2)))
    samples = runs.shape[0] * runs.shape[1]
    print(json.dumps({
        "metric": "Raman-map correlation samples/s (streaming, 180 polarisation pairs)", "value": samples / t_stream,
        "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": 1e3 * t_stream,
        "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "susceptibility tensor series, 20 runs x 100,000 samples (5 fs), max lag 2000, "
                               "streamed in 10,000-sample device chunks; map over 90 crystal rotations x "
                               "(parallel, crossed)"},
        "whole_run_map_call": {"samples_per_s": samples / t_whole, "ms": 1e3 * t_whole,
                               "max_rel_diff_vs_stream": agree},
        "input_GB_per_s": samples * 72 / t_stream / 1e9,
        "cpu_baseline": {"value": 20000 / t_cpu, "unit": "samples/s", "cores": 1, "kind": "oracle",
                         "sample": "one run truncated to 20,000 samples, Z(XX)Z-bar and Z(XY)Z-bar by direct lag "
                                   "sums (numpy)"},
        "max_rel_error_vs_oracle": err}), flush=True)


def _serving_requests(n_requests, seed=4):
    """Request mix: half water boxes of 64..8000 H2O (consecutive OU frames,
    species O=3, H=1 of the five-species models), half batches of vacuum
    molecules; each a dipole or polarizability evaluation of 1-64 frames."""
    rng = np.random.default_rng(seed)
    mols = synth.molecules(4096, seed=seed + 1)
    sides = [4, 6, 8, 10, 16, 20]
    reqs = []
    for k in range(n_requests):
        kind = 1 + int(rng.integers(0, 2))
        nf = int(rng.integers(1, 65))
        if k % 2 == 0:
            n = int(rng.choice(sides))
            pos, spc, cell = synth.water_box(n, 3.105 * n, seed=seed * 1000 + k, o_species=3, h_species=1)
            fr = synth.ou_trajectory(pos, spc, cell, nf, seed=k)
        else:
            start = int(rng.integers(0, 4096 - nf))
            fr = mols.subset(range(start, start + nf))
        reqs.append((kind, fr))
    return reqs


def bench_serving(args):
    """Poisson request stream through the continuous-batching server versus
    the plain per-frame path (one synchronous call per frame, FIFO)."""
    import threading

    from paper_2312_05233_amd import tnep

    reqs = _serving_requests(args.requests)
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    total_af = sum(fr.n_atoms for _, fr in reqs)

    def run_server(qps, seed, graphs=False):
        ctx = tnep.Context(0, budget_bytes=32 << 30)
        ctx.set_option(tnep.OPT_GRAPHS, int(graphs))
        gm = {1: tnep.Model(ctx, md), 2: tnep.Model(ctx, mp)}
        srv = tnep.Server(ctx, budget_bytes=32 << 30, max_batch_atoms=1 << 19, max_inflight=3)
        # warm-up: one request of each kind
        for kind, fr in reqs[:4]:
            srv.wait(srv.submit(gm[kind], fr))
        rng = np.random.default_rng(seed)
        lat = [None] * len(reqs)
        tickets = [None] * len(reqs)
        ready = threading.Semaphore(0)

        def waiter():
            for i in range(len(reqs)):
                ready.acquire()
                st, l, _ = srv.wait(tickets[i])
                lat[i] = l if st == 0 else float("nan")

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        t_next = t0
        for i, (kind, fr) in enumerate(reqs):
            if qps:
                t_next += rng.exponential(1.0 / qps)
                dt = t_next - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            tickets[i] = srv.submit(gm[kind], fr)
            ready.release()
        th.join()
        wall = time.perf_counter() - t0
        stats = srv.stats()
        srv.stop()
        ctx.close()
        lat = np.array(lat) * 1e3
        return {"qps": qps, "atom_frames_per_s": total_af / wall, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "launches": stats["launches"],
                "peak_device_bytes": stats["peak_bytes"], "graphs": graphs}

    def run_plain(qps, seed, graphs=False):
        """Single FIFO worker, one synchronous evaluation call per frame."""
        ctx = tnep.Context(0)
        ctx.set_option(tnep.OPT_GRAPHS, int(graphs))
        gm = {1: tnep.Model(ctx, md), 2: tnep.Model(ctx, mp)}
        for kind, fr in reqs[:4]:
            (tnep.tnep_eval_dipole if kind == 1 else tnep.tnep_eval_polarizability)(ctx, gm[kind], fr)
        rng = np.random.default_rng(seed)
        arrivals = np.cumsum(rng.exponential(1.0 / qps, len(reqs))) if qps else np.zeros(len(reqs))
        t0 = time.perf_counter()
        lat = []
        for (kind, fr), ta in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if now < ta:
                time.sleep(ta - now)
            f = tnep.tnep_eval_dipole if kind == 1 else tnep.tnep_eval_polarizability
            for k in range(fr.n_frames):
                f(ctx, gm[kind], fr.subset([k]))
            lat.append(time.perf_counter() - t0 - ta)
        wall = time.perf_counter() - t0
        ctx.close()
        lat = np.array(lat) * 1e3
        return {"qps": qps, "atom_frames_per_s": total_af / wall, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "graphs": graphs}

    def call_latency(graphs, n_calls=300):
        """Wall time of one synchronous host-to-host call on a small input."""
        ctx = tnep.Context(0)
        ctx.set_option(tnep.OPT_GRAPHS, int(graphs))
        gm = {1: tnep.Model(ctx, md), 2: tnep.Model(ctx, mp)}
        mol = synth.molecules(4, seed=9)
        res = {}
        for label, fr in (("1 molecule frame", mol.subset([0])), ("4 molecule frames", mol)):
            for kind in (1, 2):
                f = tnep.tnep_eval_dipole if kind == 1 else tnep.tnep_eval_polarizability
                for _ in range(10):
                    f(ctx, gm[kind], fr)
                ts = []
                for _ in range(n_calls):
                    t0 = time.perf_counter()
                    f(ctx, gm[kind], fr)
                    ts.append(time.perf_counter() - t0)
                ts = np.array(ts) * 1e3
                res["%s %s" % (label, "dipole" if kind == 1 else "polarizability")] = {
                    "p50_ms": float(np.percentile(ts, 50)), "p99_ms": float(np.percentile(ts, 99))}
        res["graph_captures_launches"] = list(ctx.graph_counts())
        ctx.close()
        return res

    sat = run_server(0, 1)
    sat_g = run_server(0, 1, graphs=True)
    sat_qps = len(reqs) / (total_af / sat["atom_frames_per_s"])
    plain_sat = run_plain(0, 1)
    plain_sat_g = run_plain(0, 1, graphs=True)
    loads = []
    for frac in (0.25, 0.5, 0.8, 0.95):
        loads.append(dict(run_server(frac * sat_qps, 10 + int(100 * frac)), load=frac))
        loads.append(dict(run_server(frac * sat_qps, 10 + int(100 * frac), graphs=True), load=frac))
    plain_qps = len(reqs) / (total_af / plain_sat["atom_frames_per_s"])
    plain_half = dict(run_plain(0.5 * plain_qps, 60), load=0.5)
    plain_half_g = dict(run_plain(0.5 * plain_qps, 60, graphs=True), load=0.5)
    small_calls = {"plain launches": call_latency(False), "graph replay": call_latency(True)}
    print(json.dumps({
        "metric": "TNEP atom-frames/s (dipole+polarizability) at FP32 tol; p50/p99 request latency",
        "value": sat["atom_frames_per_s"], "unit": "atom-frames/s", "n_gpus": 1, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals, %d requests (water boxes 192-24000 atoms / vacuum "
                               "molecules, 1-64 frames each, dipole or polarizability), 32 GB budget" % len(reqs),
                   "atom_frames": total_af},
        "saturation": sat, "saturation_with_graphs": sat_g, "saturation_qps": sat_qps, "poisson_loads": loads,
        "plain_per_frame_path": {"saturation": plain_sat, "saturation_with_graphs": plain_sat_g,
                                 "at_half_load": plain_half, "at_half_load_with_graphs": plain_half_g},
        "small_call_latency": small_calls}), flush=True)


def extra_legs(args, ctx, gd, gp, frames, dfr, md, mp, M, ms_step):
    """Legs that complete the metric beside the headline (a few seconds):
    host_inputs_value  the same step with host-resident positions and host
                       outputs (host-to-device copies inside the timed region);
    plain_path         one synchronous call per frame on a subset of frames
                       (the per-frame path the batched calls are compared with);
    serving            a short Poisson request stream through the
                       continuous-batching server at half of its measured
                       saturation: p50/p99 request latency."""
    import torch

    from paper_2312_05233_amd import tnep

    out = {}
    F = frames.n_frames

    def host_step():
        mu_h, al_h = tnep.tnep_eval_dipole_polarizability(ctx, gd, gp, frames)
        tnep.tnep_spectrum(ctx, mu_h.reshape(1, F, 3), tnep.IR, 1.0, M)
        tnep.tnep_spectrum(ctx, al_h.reshape(1, F, 9), tnep.RAMAN_ISO, 1.0, M)
        tnep.tnep_spectrum(ctx, al_h.reshape(1, F, 9), tnep.RAMAN_ANISO, 1.0, M)

    host_step()
    n_host = 2
    t0 = time.perf_counter()
    for _ in range(n_host):
        host_step()
    t_host = (time.perf_counter() - t0) / n_host
    out["host_inputs_value"] = frames.n_atoms / t_host
    out["host_inputs"] = {"ms_per_step": 1e3 * t_host, "steps": n_host,
                          "h2d_bytes_per_step": frames.n_atoms * 28,
                          "note": "positions, species and offsets in host memory, outputs back to host; "
                                  "the copies are inside the timed steps"}

    # plain per-frame path: one dipole+polarizability call per frame, device inputs
    n_plain = min(40, F)
    subs = [tnep.DeviceFrames(frames.subset([f])) for f in range(n_plain)]
    mu1 = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    al1 = torch.zeros((1, 9), dtype=torch.float64, device="cuda")
    for d in subs[:2]:
        tnep.tnep_eval_dipole_polarizability(ctx, gd, gp, d, mu1, al1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in subs:
        tnep.tnep_eval_dipole_polarizability(ctx, gd, gp, d, mu1, al1)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    af_plain = n_plain * (frames.n_atoms // F)
    out["plain_path"] = {"atom_frames_per_s": af_plain / t_plain, "frames": n_plain,
                         "ms_per_frame": 1e3 * t_plain / n_plain,
                         "batched_ms_per_frame_eval_and_spectra": ms_step / F}

    # serving: saturation, then Poisson arrivals at half of it
    reqs = _serving_requests(args.serving_requests, seed=14)
    sm_d, sm_p = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    total_af = sum(fr.n_atoms for _, fr in reqs)
    sctx = tnep.Context(0, budget_bytes=32 << 30)
    sctx.set_option(tnep.OPT_GRAPHS, 1)
    gm = {1: tnep.Model(sctx, sm_d), 2: tnep.Model(sctx, sm_p)}

    def run(qps, seed):
        srv = tnep.Server(sctx, budget_bytes=32 << 30, max_batch_atoms=1 << 19, max_inflight=3)
        for kind, fr in reqs[:2]:
            srv.wait(srv.submit(gm[kind], fr))
        rng = np.random.default_rng(seed)
        t0 = time.perf_counter()
        t_next = t0
        tickets = []
        for kind, fr in reqs:
            if qps:
                t_next += rng.exponential(1.0 / qps)
                dt = t_next - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            tickets.append(srv.submit(gm[kind], fr))
        lat = []
        for t in tickets:
            st, l, _ = srv.wait(t)
            lat.append(l if st == 0 else float("nan"))
        wall = time.perf_counter() - t0
        srv.stop()
        lat = np.array(lat) * 1e3
        return total_af / wall, lat, wall

    sat_rate, _, sat_wall = run(0, 1)
    sat_qps = len(reqs) / sat_wall
    rate, lat, _ = run(0.5 * sat_qps, 2)
    sctx.close()
    out["serving"] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                      "qps": 0.5 * sat_qps, "load": 0.5, "atom_frames_per_s_at_load": rate,
                      "saturation_atom_frames_per_s": sat_rate, "requests": len(reqs),
                      "workload": "water boxes 192-24000 atoms (OU frames) and vacuum molecules, 1-64 frames per "
                                  "request, dipole or polarizability, HIP-graph replay, 32 GB pool, 3 slots"}
    return out


def _eval_roofline(ctx, model, step, steps, kernel):
    """Average launch time of one evaluation kernel (HIP events around its
    launches on the context's stream) and its FP32 rate from the flop model."""
    import torch

    from paper_2312_05233_amd import tnep

    ctx.set_option(tnep.OPT_TIMING, 1)
    ctx.reset_timing()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms, launches = ctx.kernel_time(kernel)
    atoms, rad, ang = ctx.pair_counts()
    ctx.set_option(tnep.OPT_TIMING, 0)
    flop_af = flops_per_atom_frame(model, rad / atoms, ang / atoms)
    per_launch = atoms / launches
    achieved = flop_af * per_launch / (ms / launches * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None, "flop_per_atom_frame": flop_af,
            "atoms_per_launch": per_launch, "avg_launch_ms": ms / launches,
            "mean_radial_neighbors": rad / atoms, "mean_angular_neighbors": ang / atoms}


def config_legs(args):
    """The other frame workloads beside the headline, one record each: the
    throughput of one call over device-resident frames, the roofline of its
    dominant evaluation kernel, and the largest per-frame error against the
    FP64 oracle on the frames named in the record."""
    import torch

    import oracle
    from paper_2312_05233_amd import tnep

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import frame_errors

    legs = {}
    steps = max(args.steps, 5)

    # small periodic water, dipole model
    frames = synth.water_small(10)
    m = synth.model("water_dipole_small")
    ctx = tnep.Context(0)
    gm = tnep.Model(ctx, m)
    dfr = tnep.DeviceFrames(frames)
    mu = torch.zeros((frames.n_frames, 3), dtype=torch.float64, device="cuda")
    step = lambda: tnep.tnep_eval_dipole(ctx, gm, dfr, mu)  # noqa: E731
    t = _timed(step, 4 * steps, args.warmup + 1)
    ref, pa = oracle.eval_frames(m, frames, per_atom=True)
    err = frame_errors(mu.cpu().numpy(), ref, pa, frames.offsets).max()
    rl = _eval_roofline(ctx, m, step, steps, tnep.KERNEL_EVAL_DIPOLE)
    rl["kernel"] = "k_eval<dipole>"
    # the same call in the pair-parallel layout (16 lanes per atom, for calls of few atoms)
    pctx = tnep.Context(0)
    pctx.set_option(tnep.OPT_PAIR_PARALLEL, 1)
    pgm = tnep.Model(pctx, m)
    pmu = torch.zeros_like(mu)
    pstep = lambda: tnep.tnep_eval_dipole(pctx, pgm, dfr, pmu)  # noqa: E731
    tp = _timed(pstep, 4 * steps, args.warmup + 1)
    perr = frame_errors(pmu.cpu().numpy(), ref, pa, frames.offsets).max()
    prl = _eval_roofline(pctx, m, pstep, steps, tnep.KERNEL_EVAL_DIPOLE)
    prl["kernel"] = "k_eval<dipole>, 16 lanes per atom"
    legs["water_small_dipole"] = {
        "workload": "64 H2O (192 atoms), 12.42 A periodic box, 10 independent frames, dipole model",
        "value": frames.n_atoms / t, "unit": "atom-frames/s", "ms_per_call": 1e3 * t, "dtype": "f32",
        "max_frame_error_vs_oracle": float(err), "error_frames": "all 10", "roofline": rl,
        "pair_parallel": {"value": frames.n_atoms / tp, "ms_per_call": 1e3 * tp,
                          "max_frame_error_vs_oracle": float(perr), "roofline": prl}}
    pgm.close()
    pctx.close()
    gm.close()
    ctx.close()

    # perovskite 12^3 supercell, susceptibility model, one batch of 64 frames
    frames = synth.perovskite(64)
    m = synth.model("perovskite_susceptibility")
    ctx = tnep.Context(0)
    gm = tnep.Model(ctx, m)
    dfr = tnep.DeviceFrames(frames)
    out = torch.zeros((frames.n_frames, 9), dtype=torch.float64, device="cuda")
    step = lambda: tnep.tnep_eval_polarizability(ctx, gm, dfr, out)  # noqa: E731
    t = _timed(step, steps, args.warmup)
    two = frames.subset([0, 1])
    ref, pa = oracle.eval_frames(m, two, per_atom=True)
    err = frame_errors(out[:2].cpu().numpy(), ref.reshape(2, 9), pa, two.offsets).max()
    rl = _eval_roofline(ctx, m, step, steps, tnep.KERNEL_EVAL_POLARIZABILITY)
    rl["kernel"] = "k_eval<7,5,9,9,polarizability>"
    legs["perovskite_susceptibility"] = {
        "workload": "Ba/Zr/O 12x12x12 supercell (8640 atoms, a = 4.19 A, sigma 0.08 A), batch of 64 frames, "
                    "susceptibility model rc 7/5 A, n_max 6/4, H = 50, FP32 hidden layer",
        "value": frames.n_atoms / t, "unit": "atom-frames/s", "ms_per_call": 1e3 * t, "dtype": "f32",
        "max_frame_error_vs_oracle": float(err), "error_frames": "0 and 1", "roofline": rl}
    gm.close()
    ctx.close()

    # ragged vacuum molecules, dipole + polarizability in one call
    frames = synth.molecules(8192)
    md, mp = synth.model("molecule_dipole"), synth.model("molecule_polarizability")
    ctx = tnep.Context(0)
    gd, gp = tnep.Model(ctx, md), tnep.Model(ctx, mp)
    dfr = tnep.DeviceFrames(frames)
    mu = torch.zeros((frames.n_frames, 3), dtype=torch.float64, device="cuda")
    al = torch.zeros((frames.n_frames, 9), dtype=torch.float64, device="cuda")
    step = lambda: tnep.tnep_eval_dipole_polarizability(ctx, gd, gp, dfr, mu, al)  # noqa: E731
    t = _timed(step, steps, args.warmup)
    idx = list(range(256))
    sub = frames.subset(idx)
    ref_mu, pa_mu = oracle.eval_frames(md, sub, per_atom=True)
    ref_al, pa_al = oracle.eval_frames(mp, sub, per_atom=True)
    err = max(frame_errors(mu[:256].cpu().numpy(), ref_mu, pa_mu, sub.offsets).max(),
              frame_errors(al[:256].cpu().numpy(), ref_al.reshape(-1, 9), pa_al, sub.offsets).max())
    rl = _eval_roofline(ctx, mp, step, steps, tnep.KERNEL_EVAL_POLARIZABILITY)
    rl["kernel"] = "k_eval<5,5,9,9,4-body,polarizability>"
    legs["molecules"] = {
        "workload": "8192 vacuum molecules of 20-80 atoms (%d atoms), C/H/N/O/F, dipole + polarizability in one "
                    "call" % frames.n_atoms,
        "value": frames.n_atoms / t, "unit": "atom-frames/s", "ms_per_call": 1e3 * t, "dtype": "f32",
        "max_frame_error_vs_oracle": float(err), "error_frames": "molecules 0..255, both models", "roofline": rl}
    gd.close()
    gp.close()
    ctx.close()
    return legs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=2000)
    ap.add_argument("--max-lag", type=int, default=500)
    ap.add_argument("--cpu-frames", type=int, default=32)
    ap.add_argument("--requests", type=int, default=200, help="serving workload: number of requests")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="skip the host-input, plain per-frame, serving and other-workload legs of the headline run")
    ap.add_argument("--serving-requests", type=int, default=60, help="requests of the headline run's serving leg")
    ap.add_argument("--mlp", type=int, default=None, help="TNEP_MLP_* mode of the hidden layer")
    ap.add_argument("--atoms-per-block", type=int, default=None)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch parameters")
    ap.add_argument("--trajectory-window", type=int, default=0,
                    help="frames per neighbour-candidate window of the trajectory (0 = plain searches)")
    ap.add_argument("--skin", type=float, default=1.0, help="candidate skin in Angstrom")
    ap.add_argument("--workload", default="water", choices=["water", "perovskite", "molecules", "serving", "pes", "spectra",
                                                              "population", "variants", "latency"],
                    help="water: the headline line; the others print their own JSON line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (frames shard trivially "
              "across GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4}))
        return

    from paper_2312_05233_amd import tnep

    if args.workload != "water":
        {"perovskite": bench_perovskite, "molecules": bench_molecules, "serving": bench_serving,
         "pes": bench_pes, "spectra": bench_spectra, "population": bench_population,
         "variants": bench_variants, "latency": bench_latency}[args.workload](args)
        return

    dev = torch.device("cuda:0")
    frames = synth.water_trajectory(args.frames)
    md, mp = synth.model("water_dipole"), synth.model("water_polarizability")
    F, A = frames.n_frames, frames.n_atoms
    stream = torch.cuda.Stream(device=dev)
    ctx = tnep.Context(0, stream=stream)
    if args.mlp is not None:
        ctx.set_option(tnep.OPT_MLP, args.mlp)
    if args.atoms_per_block is not None:
        ctx.set_option(tnep.OPT_ATOMS_PER_BLOCK, args.atoms_per_block)
    if not args.no_autotune:
        ctx.set_option(tnep.OPT_AUTOTUNE, 1)  # tuned during the warm-up step
    if args.trajectory_window > 1:
        ctx.set_option(tnep.OPT_TRAJECTORY_WINDOW, args.trajectory_window)
        ctx.set_option(tnep.OPT_SKIN_MA, int(round(args.skin * 1000)))
    gd, gp = tnep.Model(ctx, md), tnep.Model(ctx, mp)
    dfr = tnep.DeviceFrames(frames)
    mu = torch.zeros((F, 3), dtype=torch.float64, device=dev)
    alpha = torch.zeros((F, 9), dtype=torch.float64, device=dev)
    M = min(args.max_lag, F)
    spec = {k: [torch.zeros(M + 1, dtype=torch.float64, device=dev) for _ in range(2)] + [
        torch.zeros(M, dtype=torch.float64, device=dev)] for k in ("ir", "iso", "aniso")}
    torch.cuda.synchronize()

    def step():
        tnep.tnep_eval_dipole_polarizability(ctx, gd, gp, dfr, mu, alpha)
        for name, kind, ser in (("ir", tnep.IR, mu.view(1, F, 3)), ("iso", tnep.RAMAN_ISO, alpha.view(1, F, 9)),
                                ("aniso", tnep.RAMAN_ANISO, alpha.view(1, F, 9))):
            f, s, c = spec[name]
            tnep.tnep_spectrum(ctx, ser, kind, 1.0, M, freq=f, intensity=s, acf=c)

    for _ in range(max(args.warmup, 0 if args.no_autotune else 1)):
        step()
    # timed region: the production path (no per-launch events, no pair counting)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps

    # instrumented pass over the same steps: HIP events around every launch on
    # the context's stream, and the neighbour-pair counts of the flop model
    ctx.set_option(tnep.OPT_TIMING, 1)
    ctx.reset_timing()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step_timed = 1e3 * (time.perf_counter() - t1) / args.steps
    ctx.set_option(tnep.OPT_TIMING, 0)

    kt = {name: ctx.kernel_time(k) for name, k in (
        ("neighbors", tnep.KERNEL_NEIGHBORS), ("eval_dipole", tnep.KERNEL_EVAL_DIPOLE),
        ("eval_polarizability", tnep.KERNEL_EVAL_POLARIZABILITY), ("frame_reduce", tnep.KERNEL_FRAME_REDUCE),
        ("spectrum", tnep.KERNEL_SPECTRUM))}
    atoms, rad_pairs, ang_pairs = ctx.pair_counts()
    n_rad = rad_pairs / atoms
    n_ang = ang_pairs / atoms
    pol_ms, pol_launches = kt["eval_polarizability"]
    atoms_per_launch = atoms / pol_launches
    # the kernel loads the radial descriptor sums that the neighbour search
    # formed: their forward flops are not its work
    flop_af = flops_per_atom_frame(mp, n_rad, n_ang)
    achieved = flop_af * atoms_per_launch / (pol_ms / pol_launches * 1e-3) / 1e12
    traffic = read_traffic(atoms_per_launch)

    mu_h = mu.cpu().numpy()
    al_h = alpha.cpu().numpy()
    result = {
        "metric": "TNEP atom-frames/s (dipole+polarizability) at FP32 tol",
        "value": A / (ms_step * 1e-3),
        "unit": "atom-frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "water 4096 H2O (12288 atoms, 49.7 A PBC) x 2000-frame OU trajectory; dipole + "
                        "polarizability models; IR + Raman iso/aniso spectra (M=500)",
            "frames": F, "atoms_per_frame": A // F, "atom_frames_per_step": A,
            "descriptor": "rc 6/4 A, n_max 4/4, basis 8/8, l_max 4 + 4-body, H=30",
            "precision": "FP32 descriptor/network/partial forces, FP64 frame sums and spectra",
            "neighbour_reuse": {"window": args.trajectory_window, "skin_A": args.skin,
                                "fallbacks": ctx.reuse_fallbacks()},
        },
        "roofline": {
            "kernel": "k_eval<5,5,9,9,4-body,polarizability>",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_VECTOR_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
            "traffic": traffic,
            "flop_per_atom_frame": flop_af,
            "atoms_per_launch": atoms_per_launch,
            "avg_launch_ms": pol_ms / pol_launches,
            "mean_radial_neighbors": n_rad,
            "mean_angular_neighbors": n_ang,
            "note": "radial descriptor sums formed by the neighbour search; their forward flops are not counted "
                    "for this kernel",
        },
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
        "ms_per_step_instrumented": ms_step_timed,
        "autotune": ctx.autotune_report(),
    }
    if not args.no_extra_legs:
        result.update(extra_legs(args, ctx, gd, gp, frames, dfr, md, mp, M, ms_step))
        result["other_configs"] = config_legs(args)
    if not args.no_cpu_baseline:
        cb, e_mu, e_al = cpu_baseline(frames, md, mp, min(args.cpu_frames, F), mu_h, al_h)
        result["cpu_baseline"] = cb
        result["max_frame_error_vs_oracle"] = {"dipole": e_mu, "polarizability": e_al}
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
