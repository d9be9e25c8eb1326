"""FP64 CPU oracle for TNEP (arXiv:2312.05233): test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library.

* tensor evaluation (Eqs. virial, mu, polarizability-model) and the
  potential-energy surface of Sec. 2.1 (energy, virial, forces) live in
  ``tnep_oracle.c`` and are reached through ctypes;
* the spectrum step (Sec. 2.6 The IR intensity, Sec. 2.7 The Raman
  intensity: time-origin-averaged correlation
  functions, their Fourier transform, the omega^2 IR prefactor and the
  isotropic/anisotropic Raman split) is written here in numpy as plain
  lag sums and cosine sums.

Pins: the paper prints no numerical example of either stage, so no pin is a
value from the paper; every part is pinned instead by facts outside this
package (closed forms, library routines of the special cases, invariants and
finite differences: tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tnep_oracle.c")
_LIB = os.path.join(_HERE, "_tnep_oracle.so")
_lock = threading.Lock()
_lib = None

ERRORS = {0: "ok", -1: "invalid", -2: "species", -3: "box", -4: "overlap", -5: "nonfinite", -9: "capacity"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code} ({ERRORS.get(code, '?')})")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP) into oracle/_tnep_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("n_species", C.c_int32),
        ("rc_radial", C.c_double), ("rc_angular", C.c_double),
        ("n_max_radial", C.c_int32), ("n_max_angular", C.c_int32),
        ("basis_radial", C.c_int32), ("basis_angular", C.c_int32),
        ("l_max", C.c_int32), ("four_body", C.c_int32), ("n_hidden", C.c_int32),
        ("c_radial", C.POINTER(C.c_double)), ("c_angular", C.POINTER(C.c_double)),
        ("q_scaler", C.POINTER(C.c_double)),
        ("w0", C.POINTER(C.c_double) * 2), ("b0", C.POINTER(C.c_double) * 2),
        ("w1", C.POINTER(C.c_double) * 2), ("b1", C.c_double * 2),
        ("per_species", C.c_int32), ("b1_species", C.POINTER(C.c_double) * 2),
        ("five_body", C.c_int32),
    ]


def _lib_handle():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = C.CDLL(_LIB)
            P = C.POINTER
            lib.or_set_threads.argtypes = [C.c_int]
            lib.or_max_threads.restype = C.c_int
            lib.or_ylm.restype = C.c_double
            lib.or_ylm.argtypes = [C.c_int, C.c_int, P(C.c_double), P(C.c_double)]
            lib.or_wigner3j.restype = C.c_double
            lib.or_wigner3j.argtypes = [C.c_int] * 6
            lib.or_cutoff.argtypes = [C.c_double, C.c_double, P(C.c_double), P(C.c_double)]
            lib.or_basis.argtypes = [C.c_double, C.c_double, C.c_int, P(C.c_double), P(C.c_double)]
            lib.or_four_body.restype = C.c_double
            lib.or_four_body.argtypes = [P(C.c_double), P(C.c_double)]
            lib.or_four_body_imag.restype = C.c_double
            lib.or_four_body_imag.argtypes = [P(C.c_double)]
            lib.or_descriptor_size.restype = C.c_int
            lib.or_atom_eval.restype = C.c_int
            lib.or_atom_eval.argtypes = [P(_Model), C.c_int, C.c_int, C.c_int, P(C.c_double), P(C.c_int32),
                                         P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_double)]
            lib.or_neighbors.restype = C.c_int
            lib.or_neighbors.argtypes = [C.c_int, P(C.c_double), P(C.c_double), P(C.c_uint8), C.c_double,
                                         C.c_int, P(C.c_int32), P(C.c_int32)]
            lib.or_eval_frames.restype = C.c_int
            lib.or_eval_frames.argtypes = [P(_Model), C.c_int, P(C.c_int64), P(C.c_double), P(C.c_int32),
                                           P(C.c_double), P(C.c_uint8), P(C.c_double), P(C.c_double)]
            lib.or_eval_pes.restype = C.c_int
            lib.or_eval_pes.argtypes = [P(_Model), C.c_int, P(C.c_int64), P(C.c_double), P(C.c_int32),
                                        P(C.c_double), P(C.c_uint8), P(C.c_double), P(C.c_double),
                                        P(C.c_double), P(C.c_double)]
            lib.or_init()
            _lib = lib
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


class OracleModel:
    """Keeps the numpy buffers alive for the ctypes struct."""

    def __init__(self, m):
        self.m = m
        self._keep = []

        def arr(x):
            a = np.ascontiguousarray(np.asarray(x, np.float64))
            self._keep.append(a)
            return _dp(a)

        s = _Model()
        s.kind = m.kind
        s.n_species = m.n_species
        s.rc_radial = m.rc_radial
        s.rc_angular = m.rc_angular
        s.n_max_radial = m.n_max_radial
        s.n_max_angular = m.n_max_angular
        s.basis_radial = m.basis_radial
        s.basis_angular = m.basis_angular
        s.l_max = m.l_max
        s.four_body = int(bool(m.four_body))
        s.n_hidden = m.n_hidden
        s.c_radial = arr(m.c_radial)
        s.c_angular = arr(m.c_angular)
        s.q_scaler = arr(m.q_scaler)
        for h, head in enumerate(m.heads):
            s.w0[h] = arr(head.w0)
            s.b0[h] = arr(head.b0)
            s.w1[h] = arr(head.w1)
            if getattr(m, "per_species", False):
                s.b1_species[h] = arr(head.b1)
            else:
                s.b1[h] = head.b1
        s.per_species = int(bool(getattr(m, "per_species", False)))
        s.five_body = int(bool(getattr(m, "five_body", False)))
        self.s = s


def _model(m):
    return m if isinstance(m, OracleModel) else OracleModel(m)


# -------------------------------------------------------------------------
# Building blocks exposed for the pins


def set_threads(n):
    """Threads of the oracle's frame loops (OpenMP) from now on."""
    _lib_handle().or_set_threads(int(n))


def max_threads():
    """Threads the oracle's frame loops use."""
    return int(_lib_handle().or_max_threads())


def ylm(l, m, v):
    """Real orthonormal Y_lm(v/|v|) and its gradient with respect to v."""
    lib = _lib_handle()
    v = np.ascontiguousarray(np.asarray(v, np.float64))
    g = np.zeros(3)
    y = lib.or_ylm(l, m, _dp(v), _dp(g))
    return y, g


def wigner3j(j1, j2, j3, m1, m2, m3):
    return _lib_handle().or_wigner3j(j1, j2, j3, m1, m2, m3)


def cutoff(r, rc):
    a, b = C.c_double(), C.c_double()
    _lib_handle().or_cutoff(r, rc, C.byref(a), C.byref(b))
    return a.value, b.value


def basis(r, rc, K):
    f = np.zeros(K + 1)
    df = np.zeros(K + 1)
    _lib_handle().or_basis(r, rc, K, _dp(f), _dp(df))
    return f, df


def four_body(A2):
    """(q4, dq4/dA, imaginary part) for the five real l=2 sums A2[m+2]."""
    a = np.ascontiguousarray(np.asarray(A2, np.float64))
    d = np.zeros(5)
    lib = _lib_handle()
    q = lib.or_four_body(_dp(a), _dp(d))
    return q, d, lib.or_four_body_imag(_dp(a))


def atom_eval(m, head, ti, vecs, tj, forces=True):
    """One atom: returns dict(U, q, dUdq, dUdr) for neighbour vectors vecs [n,3]."""
    om = _model(m)
    lib = _lib_handle()
    vecs = np.ascontiguousarray(np.asarray(vecs, np.float64).reshape(-1, 3))
    tj = np.ascontiguousarray(np.asarray(tj, np.int32))
    n = vecs.shape[0]
    D = om.m.dim
    U = C.c_double()
    q = np.zeros(D)
    dq = np.zeros(D)
    F = np.zeros((max(n, 1), 3))
    e = lib.or_atom_eval(C.byref(om.s), head, ti, n, _dp(vecs), tj.ctypes.data_as(C.POINTER(C.c_int32)),
                         C.byref(U), _dp(q), _dp(dq), _dp(F) if forces else None)
    if e:
        raise OracleError(e)
    return {"U": U.value, "q": q, "dUdq": dq, "dUdr": F[:n]}


def neighbors(pos, cell, pbc, rc, cap=512):
    """Brute-force neighbour lists: list of index arrays (increasing j)."""
    lib = _lib_handle()
    pos = np.ascontiguousarray(np.asarray(pos, np.float64))
    n = pos.shape[0]
    cnt = np.zeros(n, np.int32)
    lst = np.zeros((n, cap), np.int32)
    cell = None if cell is None else np.ascontiguousarray(np.asarray(cell, np.float64))
    pbc = None if pbc is None else np.ascontiguousarray(np.asarray(pbc, np.uint8))
    e = lib.or_neighbors(n, _dp(pos), _dp(cell), None if pbc is None else pbc.ctypes.data_as(C.POINTER(C.c_uint8)),
                         rc, cap, cnt.ctypes.data_as(C.POINTER(C.c_int32)), lst.ctypes.data_as(C.POINTER(C.c_int32)))
    if e:
        raise OracleError(e)
    return [lst[i, : cnt[i]].copy() for i in range(n)]


def frame_descriptors(m, frames, f, head=0, forces=False):
    """Per-atom descriptor q [n,D], U [n] (and optionally dU/dr per pair) of
    frame f, neighbours by brute force within rc_radial."""
    a0, a1 = int(frames.offsets[f]), int(frames.offsets[f + 1])
    pos = frames.positions[a0:a1]
    spc = frames.species[a0:a1]
    cell = None if frames.cells is None else frames.cells[f]
    pbc = None if frames.pbc is None else frames.pbc[f]
    nb = neighbors(pos, cell, pbc, m.rc_radial)
    per = np.zeros(3, bool) if pbc is None else np.asarray(pbc, bool)
    if cell is not None and np.any(np.asarray(cell, np.float64).reshape(3, 3)[~np.eye(3, dtype=bool)] != 0):
        raise ValueError("frame_descriptors takes orthorhombic cells only (use eval_frames)")
    box = np.zeros(3) if cell is None else np.array([cell[0], cell[4], cell[8]])
    om = _model(m)
    qs, us, frc = [], [], []
    for i in range(a1 - a0):
        v = pos[nb[i]] - pos[i]
        v[:, per] -= box[per] * np.round(v[:, per] / box[per])
        r = atom_eval(om, head, int(spc[i]), v, spc[nb[i]], forces=forces)
        qs.append(r["q"])
        us.append(r["U"])
        if forces:
            frc.append((nb[i], v, r["dUdr"]))
    out = (np.array(qs), np.array(us))
    return out + (frc,) if forces else out


def eval_frames(m, frames, per_atom=False):
    """mu [F,3] (dipole model) or alpha [F,3,3] (polarizability model), FP64.
    With per_atom=True also returns the per-atom terms [A,3] / [A,3,3]."""
    om = _model(m)
    lib = _lib_handle()
    nt = 3 if om.m.kind == 1 else 9
    F = frames.n_frames
    out = np.zeros((F, nt))
    pa = np.zeros((frames.n_atoms, nt)) if per_atom else None
    offs = np.ascontiguousarray(frames.offsets.astype(np.int64))
    pos = np.ascontiguousarray(frames.positions.astype(np.float64))
    spc = np.ascontiguousarray(frames.species.astype(np.int32))
    cells = None if frames.cells is None else np.ascontiguousarray(frames.cells.astype(np.float64))
    pbc = None if frames.pbc is None else np.ascontiguousarray(frames.pbc.astype(np.uint8))
    e = lib.or_eval_frames(C.byref(om.s), F, offs.ctypes.data_as(C.POINTER(C.c_int64)), _dp(pos),
                           spc.ctypes.data_as(C.POINTER(C.c_int32)), _dp(cells),
                           None if pbc is None else pbc.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(out), _dp(pa))
    if e:
        raise OracleError(e)
    if nt == 9:
        out = out.reshape(F, 3, 3)
        if pa is not None:
            pa = pa.reshape(-1, 3, 3)
    return (out, pa) if per_atom else out


def population_loss(base, params, frames, reference, lambda1=0.0, lambda2=0.0):
    """Loss of every individual z_p of a population (Sec. 2.4): the RMSE of the
    model's tensors over all frames and components against reference, plus
    regularization lambda1 * sum|z| / N + lambda2 * sqrt(sum z^2 / N), N the
    number of parameters.  params [P, N] in the layout of synth.pack_params.
    Returns (loss [P], rmse [P])."""
    import synth

    params = np.asarray(params, np.float64)
    ref = np.asarray(reference, np.float64).reshape(frames.n_frames, -1)
    loss, rmse = [], []
    for z in params:
        pred = np.asarray(eval_frames(synth.unpack_params(base, z), frames)).reshape(frames.n_frames, -1)
        e = float(np.sqrt(np.mean((pred - ref) ** 2)))
        n = z.size
        rmse.append(e)
        loss.append(e + lambda1 * np.abs(z).sum() / n + lambda2 * np.sqrt((z * z).sum() / n))
    return np.array(loss), np.array(rmse)


def dipole_charged(m, frames, charges, species_masses, length_unit=1.0):
    """Dipole of charged molecules (Sec. 3, charged molecules): the model gives
    mu_r, the permanent dipole relative to the centre of mass, and the absolute
    dipole is mu = mu_r + Q e r_COM, r_COM = sum_i m_i r_i / sum_i m_i, with Q the
    frame's net charge in units of e and length_unit the model's dipole units
    per (e * Angstrom).  Frames without atoms get no shift.  [F, 3], FP64."""
    mu = eval_frames(m, frames)
    masses = np.asarray(species_masses, np.float64)
    out = mu.copy()
    for f in range(frames.n_frames):
        a0, a1 = frames.offsets[f], frames.offsets[f + 1]
        if a1 == a0:
            continue
        w = masses[frames.species[a0:a1]]
        com = (w[:, None] * frames.positions[a0:a1]).sum(0) / w.sum()
        out[f] += float(charges[f]) * length_unit * com
    return out


def eval_pes(m, frames, per_atom=False):
    """Potential-energy surface model (kind 3, Sec. 2.1): per frame the energy
    U = sum_i U_i [F], the virial W = -sum_i sum_j r_ij (x) dU_i/dr_ij [F,3,3]
    and the forces F_k = -dU/dr_k [A,3], FP64.  per_atom=True adds U_i [A]."""
    om = _model(m)
    lib = _lib_handle()
    F = frames.n_frames
    energy = np.zeros(F)
    virial = np.zeros((F, 9))
    forces = np.zeros((frames.n_atoms, 3))
    pa = np.zeros(frames.n_atoms) if per_atom else None
    offs = np.ascontiguousarray(frames.offsets.astype(np.int64))
    pos = np.ascontiguousarray(frames.positions.astype(np.float64))
    spc = np.ascontiguousarray(frames.species.astype(np.int32))
    cells = None if frames.cells is None else np.ascontiguousarray(frames.cells.astype(np.float64))
    pbc = None if frames.pbc is None else np.ascontiguousarray(frames.pbc.astype(np.uint8))
    e = lib.or_eval_pes(C.byref(om.s), F, offs.ctypes.data_as(C.POINTER(C.c_int64)), _dp(pos),
                        spc.ctypes.data_as(C.POINTER(C.c_int32)), _dp(cells),
                        None if pbc is None else pbc.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(energy),
                        _dp(virial), _dp(forces), _dp(pa))
    if e:
        raise OracleError(e)
    out = (energy, virial.reshape(F, 3, 3), forces)
    return out + (pa,) if per_atom else out


# -------------------------------------------------------------------------
# Spectrum step (Secs. 2.6-2.7), numpy.

SPEED_OF_LIGHT_CM_PER_FS = 2.99792458e-5

SPEC_IR, SPEC_RAMAN_ISO, SPEC_RAMAN_ANISO, SPEC_RAMAN_PROJ = 0, 1, 2, 3


def acf_direct(x, max_lag, y=None):
    """Time-origin average C(tau) = 1/(N-tau) sum_t x(t) y(t+tau), tau < max_lag,
    by the direct lag sum (1-D series; y defaults to x)."""
    x = np.asarray(x, np.float64)
    y = x if y is None else np.asarray(y, np.float64)
    n = x.shape[0]
    out = np.zeros(max_lag)
    for tau in range(max_lag):
        out[tau] = np.dot(x[: n - tau], y[tau:]) / (n - tau)
    return out


def channel_acf(series, kind, max_lag, n_hat=None, e_hat=None, subtract_mean=False):
    """Correlation function of one series [N_t, 3] (IR) or [N_t, 9] (Raman):
    IR     (1/3) sum_a <mu_a mu_a>                        (isotropic sample)
    iso    <gamma gamma>, gamma = Tr(alpha)/3
    aniso  <Tr beta(0) beta(t)> = sum_ab <beta_ab(0) beta_ba(t)>, beta = alpha - gamma I
    proj   <s s>, s = n^T alpha e"""
    s = np.asarray(series, np.float64)
    if subtract_mean:
        s = s - s.mean(axis=0, keepdims=True)
    if kind == SPEC_IR:
        return sum(acf_direct(s[:, a], max_lag) for a in range(3)) / 3.0
    al = s.reshape(-1, 3, 3)
    if kind == SPEC_RAMAN_ISO:
        g = np.trace(al, axis1=1, axis2=2) / 3.0
        if subtract_mean:
            g = g - g.mean()
        return acf_direct(g, max_lag)
    if kind == SPEC_RAMAN_ANISO:
        g = np.trace(al, axis1=1, axis2=2) / 3.0
        beta = al - g[:, None, None] * np.eye(3)[None]
        return sum(acf_direct(beta[:, a, b], max_lag, beta[:, b, a]) for a in range(3) for b in range(3))
    if kind == SPEC_RAMAN_PROJ:
        n_hat = np.asarray(n_hat, np.float64)
        e_hat = np.asarray(e_hat, np.float64)
        proj = np.einsum("a,tab,b->t", n_hat, al, e_hat)
        return acf_direct(proj, max_lag)
    raise ValueError(kind)


def spectrum(series_list, kind, dt_fs, max_lag, window=True, omega2=None, n_hat=None, e_hat=None,
             subtract_mean=False, acf_fn=None, laser_cm1=None):
    """One-sided windowed cosine transform of the averaged correlation function.

    S(w_k) = dt/(2 pi) [w(0) C(0) + 2 sum_{tau=1}^{M-1} w(tau) C(tau) cos(w_k tau dt)],
    w_k = pi k / (M dt), k = 0..M, Hann lag window w(tau) = (1 + cos(pi tau / M)) / 2.
    IR multiplies by w_k^2 (classical prefactor).  Frequencies in cm^-1.
    Raman kinds with laser_cm1 (incoming wavenumber) multiply by the
    ((w_in - w) / c)^4 factor of Eq. raman-cross-section, (2 pi (laser - nu_k))^4
    in cm^-4.
    Returns (freq_cm1 [M+1], intensity [M+1], acf [M])."""
    M = int(max_lag)
    fn = acf_fn or channel_acf
    C_ = np.mean([fn(s, kind, M, n_hat, e_hat, subtract_mean) for s in series_list], axis=0)
    tau = np.arange(M)
    w = 0.5 * (1.0 + np.cos(np.pi * tau / M)) if window else np.ones(M)
    k = np.arange(M + 1)
    omega = np.pi * k / (M * dt_fs)  # rad / fs
    S = np.zeros(M + 1)
    for kk in range(M + 1):
        S[kk] = w[0] * C_[0] + 2.0 * np.sum(w[1:] * C_[1:] * np.cos(omega[kk] * tau[1:] * dt_fs))
    S *= dt_fs / (2.0 * np.pi)
    if omega2 is None:
        omega2 = kind == SPEC_IR
    if omega2:
        S = S * omega ** 2
    freq = k / (2.0 * M * dt_fs * SPEED_OF_LIGHT_CM_PER_FS)
    if laser_cm1 is not None and kind != SPEC_IR:
        S = S * (2.0 * np.pi * (laser_cm1 - freq)) ** 4
    return freq, S, C_


def raman_map(series_list, dt_fs, max_lag, n_hats, e_hats, window=True, subtract_mean=False, laser_cm1=None):
    """Orientation-resolved Raman lineshapes (Eq. raman-cross-section with the
    lineshape of Eq. raman-lineshape): for each polarisation pair (n, e),
    sum n_g n_m L_gdmn e_d e_n, which is the spectrum of s(t) = n^T alpha(t) e.
    Evaluated per orientation by the direct lag sums of the projected signal.
    Returns (freq_cm1 [M+1], intensity [n_orient, M+1])."""
    out = []
    freq = None
    for n_hat, e_hat in zip(n_hats, e_hats):
        freq, S, _ = spectrum(series_list, SPEC_RAMAN_PROJ, dt_fs, max_lag, window=window, n_hat=n_hat,
                              e_hat=e_hat, subtract_mean=subtract_mean, laser_cm1=laser_cm1)
        out.append(S)
    return freq, np.array(out)
