"""Pins of the population loss (Sec. 2.4): parameter packing round trip, a
zero error when the reference is the individual's own prediction (the loss is
then the regularization, in closed form), and a constant offset of the
reference giving exactly that offset as RMSE."""
import numpy as np

import oracle
import synth


def test_pack_round_trip():
    m = synth.model("molecule_polarizability")
    z = synth.pack_params(m)
    m2 = synth.unpack_params(m, z)
    fr = synth.molecules(5, seed=101)
    assert np.array_equal(oracle.eval_frames(m, fr), oracle.eval_frames(m2, fr))


def test_loss_closed_forms():
    base = synth.model("molecule_dipole")
    fr = synth.molecules(8, seed=102)
    z0 = synth.pack_params(base)
    z1 = z0 + np.random.default_rng(3).normal(0.0, 0.01, z0.size)
    own = oracle.eval_frames(base, fr)
    loss, rmse = oracle.population_loss(base, [z0, z1], fr, own, lambda1=0.05, lambda2=0.1)
    assert rmse[0] == 0.0
    n = z0.size
    assert abs(loss[0] - (0.05 * np.abs(z0).sum() / n + 0.1 * np.sqrt((z0 ** 2).sum() / n))) < 1e-15
    assert rmse[1] > 0.0
    _, r2 = oracle.population_loss(base, [z0], fr, own + 0.25)
    assert abs(r2[0] - 0.25) < 1e-14
