"""Pins of the oracle's orientation-resolved Raman map and the Raman
prefactor (Sec. 2.7, Eqs. raman-cross-section, raman-lineshape,
raman-lineshape-isotropic-anisotropic).

The map is evaluated orientation by orientation from the projected signal
n^T alpha e; it is pinned against the isotropic / anisotropic channels
through the exact spherical average of quartic polynomials, and against a
pure oscillation whose projected amplitude is known in closed form.
"""
import numpy as np

import oracle


def _icosahedron():
    phi = (1 + 5 ** 0.5) / 2
    v = []
    for a in (-1, 1):
        for b in (-1, 1):
            v += [(0, a, b * phi), (a, b * phi, 0), (b * phi, 0, a)]
    v = np.array(v, np.float64)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _symmetric_series(n_steps, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n_steps, 3, 3))
    # a smooth, correlated series: running sums of noise, symmetrised
    a = np.cumsum(a, axis=0) * 0.1 + rng.normal(size=(1, 3, 3))
    a = 0.5 * (a + a.transpose(0, 2, 1))
    return a.reshape(n_steps, 9)


def test_orientation_average_is_iso_plus_two_fifteenths_aniso():
    """For symmetric alpha and unit n uniform on the sphere,
    <(n^T A n)(n^T B n)> = Tr A Tr B / 15 + 2 Tr(AB) / 15 = g_A g_B + (2/15) Tr(b_A b_B);
    the 12 icosahedron vertices average every polynomial of degree <= 5
    exactly, so the mean of the parallel-polarised map equals
    S_iso + (2/15) S_aniso."""
    series = [_symmetric_series(300, 1), _symmetric_series(300, 2)]
    n = _icosahedron()
    for window in (True, False):
        f, S = oracle.raman_map(series, 1.0, 120, n, n, window=window)
        _, Si, _ = oracle.spectrum(series, oracle.SPEC_RAMAN_ISO, 1.0, 120, window=window)
        _, Sa, _ = oracle.spectrum(series, oracle.SPEC_RAMAN_ANISO, 1.0, 120, window=window)
        target = Si + (2.0 / 15.0) * Sa
        assert np.abs(S.mean(0) - target).max() < 1e-12 * np.abs(target).max()


def test_pure_oscillation_scales_with_projected_amplitude():
    """alpha(t) = B cos(theta t) with a non-symmetric B: every orientation's
    spectrum is (n^T B e)^2 times that of cos(theta t) (an n/e swap or a
    transpose changes the factor for this B)."""
    rng = np.random.default_rng(3)
    B = rng.normal(size=(3, 3))
    t = np.arange(400)
    c = np.cos(0.37 * t)
    series = [(c[:, None, None] * B[None]).reshape(400, 9)]
    unit = np.zeros((400, 9))
    unit[:, 0] = c
    _, S1, _ = oracle.spectrum([unit], oracle.SPEC_RAMAN_PROJ, 2.0, 150, n_hat=[1, 0, 0], e_hat=[1, 0, 0])
    nh = rng.normal(size=(5, 3))
    eh = rng.normal(size=(5, 3))
    nh /= np.linalg.norm(nh, axis=1, keepdims=True)
    eh /= np.linalg.norm(eh, axis=1, keepdims=True)
    _, S = oracle.raman_map(series, 2.0, 150, nh, eh)
    for o in range(5):
        amp = nh[o] @ B @ eh[o]
        assert np.abs(S[o] - amp ** 2 * S1).max() < 1e-12 * np.abs(S1).max()
    # Z(XY)Z-bar differs from Z(YX)Z-bar for this B
    _, Sxy = oracle.raman_map(series, 2.0, 150, [[1, 0, 0]], [[0, 1, 0]])
    _, Syx = oracle.raman_map(series, 2.0, 150, [[0, 1, 0]], [[1, 0, 0]])
    assert abs(Sxy.max() / Syx.max() - (B[0, 1] / B[1, 0]) ** 2) < 1e-10


def test_laser_prefactor_endpoints():
    """The (w_in - w)^4 factor of Eq. raman-cross-section: (2 pi nu_in)^4 at
    zero shift, zero at nu = nu_in; IR is unaffected."""
    series = [_symmetric_series(200, 4)]
    f, S0, _ = oracle.spectrum(series, oracle.SPEC_RAMAN_ISO, 1.0, 80)
    nu_in = float(f[40])
    _, S1, _ = oracle.spectrum(series, oracle.SPEC_RAMAN_ISO, 1.0, 80, laser_cm1=nu_in)
    assert abs(S1[0] - S0[0] * (2 * np.pi * nu_in) ** 4) <= 1e-12 * abs(S1[0])
    assert S1[40] == 0.0
    mu = [np.random.default_rng(5).normal(size=(200, 3))]
    _, I0, _ = oracle.spectrum(mu, oracle.SPEC_IR, 1.0, 80)
    _, I1, _ = oracle.spectrum(mu, oracle.SPEC_IR, 1.0, 80, laser_cm1=nu_in)
    assert np.array_equal(I0, I1)
