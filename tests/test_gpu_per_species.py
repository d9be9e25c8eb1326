"""Per-species networks on the GPU against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu


def _pair(name):
    a = synth.model(name)
    seed, kind, species, desc = synth.MODEL_SPECS[name]
    b = synth.with_descriptor_of(synth.make_model(seed + 50, kind, species, **desc), a)
    return a, b


@pytest.mark.parametrize("name", ["molecule_dipole", "molecule_polarizability"])
def test_per_species_matches_oracle_and_shared_networks(gpu_lib, name):
    a, b = _pair(name)
    p = synth.per_species_model([a, b], [0, 1, 0, 1, 0])
    fr = synth.molecules(96, seed=81)
    ctx = gpu_lib.Context(0)
    f = gpu_lib.tnep_eval_dipole if a.kind == 1 else gpu_lib.tnep_eval_polarizability
    nt = 3 if a.kind == 1 else 9
    gp, ga, gb = gpu_lib.Model(ctx, p), gpu_lib.Model(ctx, a), gpu_lib.Model(ctx, b)
    pa_p, pa_a, pa_b = (np.zeros((fr.n_atoms, nt)) for _ in range(3))
    out = f(ctx, gp, fr, per_atom=pa_p)
    f(ctx, ga, fr, per_atom=pa_a)
    f(ctx, gb, fr, per_atom=pa_b)
    ref, ref_pa = oracle.eval_frames(p, fr, per_atom=True)
    err = frame_errors(out, ref, ref_pa, fr.offsets)
    print(name, "per-species error", err.max(), flush=True)
    assert np.all(err <= TENSOR_TOL)
    # every atom is evaluated exactly as by the shared model its species uses
    use_b = np.isin(fr.species, [1, 3])[:, None]
    assert np.array_equal(pa_p, np.where(use_b, pa_b, pa_a))
    # the matrix-core setting keeps the vector hidden layer for per-species networks
    ctx.set_option(gpu_lib.OPT_MLP, gpu_lib.MLP_FP32_MFMA)
    assert np.array_equal(f(ctx, gp, fr), out)
    ctx.close()


def test_per_species_pes(gpu_lib):
    a, b = _pair("water_pes")
    p = synth.per_species_model([a, b], [1, 0])
    fr = synth.water_small(3, seed=82)
    ctx = gpu_lib.Context(0)
    E, W, F = gpu_lib.tnep_eval_pes(ctx, gpu_lib.Model(ctx, p), fr)
    Er, Wr, Fr, Ur = oracle.eval_pes(p, fr, per_atom=True)
    for k in range(fr.n_frames):
        sl = slice(fr.offsets[k], fr.offsets[k + 1])
        assert abs(E[k] - Er[k]) <= TENSOR_TOL * np.abs(Ur[sl]).sum()
        assert np.linalg.norm(F[sl] - Fr[sl]) <= TENSOR_TOL * np.linalg.norm(Fr[sl])
    assert np.all(frame_errors(W, Wr) <= TENSOR_TOL)
    ctx.close()
