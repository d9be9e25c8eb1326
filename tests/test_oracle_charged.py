"""Pins of the charged-molecule dipole (Sec. 3, charged molecules):
mu = mu_r + Q e r_COM."""
import numpy as np

import oracle
import synth

MASSES = [12.011, 1.008, 14.007, 15.999, 18.998]  # C, H, N, O, F


def test_translation_moves_dipole_by_charge_times_shift():
    """mu_r does not change under a translation t (a sum of relative vectors),
    so mu(r + t) - mu(r) = Q * unit * t exactly."""
    m = synth.model("molecule_dipole")
    fr = synth.molecules(6, seed=51)
    q = np.array([1.0, -1.0, 2.0, 0.0, -3.0, 1.0])
    unit = 1.0 / 0.529177210903
    a = oracle.dipole_charged(m, fr, q, MASSES, unit)
    t = np.array([3.0, -7.5, 11.25])
    moved = synth.Frames(fr.offsets, fr.positions + t, fr.species, None, None)
    b = oracle.dipole_charged(m, moved, q, MASSES, unit)
    assert np.abs(b - a - q[:, None] * unit * t[None]).max() < 1e-10 * np.abs(a).max()


def test_neutral_frames_and_com_closed_form():
    m = synth.model("molecule_dipole")
    fr = synth.molecules(3, seed=52)
    assert np.array_equal(oracle.dipole_charged(m, fr, np.zeros(3), MASSES), oracle.eval_frames(m, fr))
    # two atoms of one species: the centre of mass is the midpoint
    pos = np.array([[0.3, -1.0, 2.0], [1.7, 0.4, 2.6]])
    two = synth.Frames(np.array([0, 2], np.int64), pos, np.array([3, 3], np.int32), None, None)
    d = oracle.dipole_charged(m, two, [1.0], MASSES) - oracle.eval_frames(m, two)
    assert np.abs(d[0] - pos.mean(0)).max() < 1e-15
