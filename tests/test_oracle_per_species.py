"""Pins of per-species networks in the oracle: a per-species model assembled
from two shared-network models gives, atom by atom, the terms of the model
whose network the atom's species uses."""
import numpy as np

import oracle
import synth


def _pair(kind_name):
    a = synth.model(kind_name)
    seed, kind, species, desc = synth.MODEL_SPECS[kind_name]
    b = synth.with_descriptor_of(synth.make_model(seed + 50, kind, species, **desc), a)
    return a, b


def test_atoms_follow_their_species_network():
    for name in ("molecule_dipole", "molecule_polarizability"):
        a, b = _pair(name)
        choice = [0, 1, 0, 1, 0]  # C, N, F on network a; H, O on network b
        p = synth.per_species_model([a, b], choice)
        fr = synth.molecules(12, seed=71)
        _, pa_a = oracle.eval_frames(a, fr, per_atom=True)
        _, pa_b = oracle.eval_frames(b, fr, per_atom=True)
        out, pa_p = oracle.eval_frames(p, fr, per_atom=True)
        use_b = np.isin(fr.species, [1, 3])
        expect = np.where(use_b.reshape((-1,) + (1,) * (pa_a.ndim - 1)), pa_b, pa_a)
        assert np.abs(pa_p - expect).max() <= 1e-14 * np.abs(expect).max(), name
        sums = np.array([expect[fr.offsets[f]:fr.offsets[f + 1]].sum(0) for f in range(fr.n_frames)])
        assert np.abs(out - sums).max() <= 1e-12 * np.abs(sums).max()


def test_identical_networks_equal_the_shared_model():
    a, _ = _pair("molecule_dipole")
    p = synth.per_species_model([a], [0] * 5)
    fr = synth.molecules(6, seed=72)
    assert np.array_equal(oracle.eval_frames(p, fr), oracle.eval_frames(a, fr))
