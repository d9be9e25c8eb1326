"""Python binding of libtnep (include/tnep.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
(host memory) or torch CUDA tensors (device memory) into the C structs and
calls the entry points of the same names.  Importing it raises if the
compiled library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnep.so")

TNEP_OK = 0
ERRORS = {0: "TNEP_OK", -1: "TNEP_E_INVALID", -2: "TNEP_E_SPECIES", -3: "TNEP_E_BOX", -4: "TNEP_E_OVERLAP",
          -5: "TNEP_E_NONFINITE", -6: "TNEP_E_BUDGET", -7: "TNEP_E_MODEL", -8: "TNEP_E_HIP",
          -9: "TNEP_E_NEIGH_OVERFLOW", -10: "TNEP_E_CANCELLED"}
HOST, DEVICE, DEVICE_META_HOST = 0, 1, 2
KIND_DIPOLE, KIND_POLARIZABILITY, KIND_PES = 1, 2, 3
MLP_FP32_VALU, MLP_FP32_MFMA, MLP_BF16_MFMA, MLP_BF16X3_MFMA = 0, 1, 2, 3
OPT_MLP, OPT_ATOMS_PER_BLOCK, OPT_AUTOTUNE, OPT_DETERMINISTIC, OPT_MAX_BATCH_ATOMS, OPT_TIMING = 1, 2, 3, 4, 5, 6
OPT_NEIGH_BLOCK = 7
OPT_GRAPHS = 8
OPT_TRAJECTORY_WINDOW, OPT_SKIN_MA = 9, 10
OPT_PAIR_PARALLEL = 11
KERNEL_NEIGHBORS, KERNEL_EVAL_DIPOLE, KERNEL_EVAL_POLARIZABILITY, KERNEL_FRAME_REDUCE, KERNEL_SPECTRUM = 0, 1, 2, 3, 4
KERNEL_EVAL_PES, KERNEL_PES_FORCES = 5, 6
IR, RAMAN_ISO, RAMAN_ANISO, RAMAN_PROJ, RAMAN_MAP = 0, 1, 2, 3, 4
WIN_HANN, WIN_NONE = 0, 1
SUBTRACT_MEAN, NO_OMEGA2 = 1, 2

EXPORTED = ["tnep_ctx_create", "tnep_ctx_destroy", "tnep_last_error", "tnep_set_option", "tnep_ctx_memory_in_use",
            "tnep_model_create", "tnep_model_free", "tnep_eval_dipole", "tnep_eval_polarizability",
            "tnep_eval_dipole_polarizability", "tnep_spectrum", "tnep_server_start", "tnep_submit", "tnep_wait",
            "tnep_server_stop", "tnep_server_stats", "tnep_server_memory", "tnep_ctx_kernel_time", "tnep_ctx_pair_counts",
            "tnep_ctx_reset_timing", "tnep_autotune_report", "tnep_ctx_graph_counts", "tnep_eval_pes",
            "tnep_raman_map", "tnep_acf_stream_create", "tnep_acf_stream_push", "tnep_acf_stream_end_run",
            "tnep_acf_stream_spectrum", "tnep_acf_stream_raman_map", "tnep_acf_stream_free",
            "tnep_ctx_reuse_fallbacks", "tnep_eval_dipole_charged", "tnep_population_loss", "tnep_model_save",
            "tnep_model_load", "tnep_model_info", "tnep_spectrum_noalloc"]


class TnepError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


P = C.POINTER


class ModelDesc(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("n_species", C.c_int32), ("rc_radial", C.c_double), ("rc_angular", C.c_double),
        ("n_max_radial", C.c_int32), ("n_max_angular", C.c_int32), ("basis_radial", C.c_int32),
        ("basis_angular", C.c_int32), ("l_max", C.c_int32), ("four_body", C.c_int32), ("n_hidden", C.c_int32),
        ("c_radial", P(C.c_double)), ("c_angular", P(C.c_double)), ("q_scaler", P(C.c_double)),
        ("w0", P(C.c_double) * 2), ("b0", P(C.c_double) * 2), ("w1", P(C.c_double) * 2), ("b1", C.c_double * 2),
        ("per_species", C.c_int32), ("b1_species", P(C.c_double) * 2), ("five_body", C.c_int32),
    ]


class FramesDesc(C.Structure):
    _fields_ = [("n_frames", C.c_int32), ("atom_offsets", C.c_void_p), ("positions", C.c_void_p),
                ("species", C.c_void_p), ("cells", C.c_void_p), ("pbc", C.c_void_p), ("location", C.c_int32)]


class SpectrumArgs(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_series", C.c_int32), ("n_steps", C.c_int64), ("series", C.c_void_p),
                ("dt_fs", C.c_double), ("max_lag", C.c_int64), ("window", C.c_int32), ("flags", C.c_int32),
                ("n_hat", C.c_double * 3), ("e_hat", C.c_double * 3), ("location", C.c_int32),
                ("laser_cm1", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_uint64), ("max_batch_atoms", C.c_int32), ("max_inflight", C.c_int32)]


def _load():
    # torch and libtnep must share one HIP runtime in the process: torch's
    # libraries ask for "libamdhip64.so", libtnep for "libamdhip64.so.7"; once
    # torch's copy (soname libamdhip64.so.7) is loaded, libtnep binds to it.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtnep.so is not built ({LIB_PATH}); run `python -m paper_2312_05233_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.tnep_ctx_create.argtypes = [C.c_int, vp, C.c_uint64, P(vp)]
    lib.tnep_ctx_destroy.argtypes = [vp]
    lib.tnep_ctx_destroy.restype = None
    lib.tnep_last_error.argtypes = [vp]
    lib.tnep_last_error.restype = C.c_char_p
    lib.tnep_set_option.argtypes = [vp, C.c_int32, C.c_int64]
    lib.tnep_ctx_memory_in_use.argtypes = [vp]
    lib.tnep_ctx_memory_in_use.restype = C.c_uint64
    lib.tnep_model_create.argtypes = [vp, P(ModelDesc), P(vp)]
    lib.tnep_model_free.argtypes = [vp]
    lib.tnep_model_free.restype = None
    lib.tnep_eval_dipole.argtypes = [vp, vp, P(FramesDesc), vp, vp]
    lib.tnep_eval_polarizability.argtypes = [vp, vp, P(FramesDesc), vp, vp]
    lib.tnep_eval_dipole_polarizability.argtypes = [vp, vp, vp, P(FramesDesc), vp, vp]
    lib.tnep_eval_pes.argtypes = [vp, vp, P(FramesDesc), vp, vp, vp, vp]
    lib.tnep_eval_dipole_charged.argtypes = [vp, vp, P(FramesDesc), vp, vp, C.c_double, vp, vp]
    lib.tnep_model_save.argtypes = [P(ModelDesc), C.c_char_p]
    lib.tnep_model_load.argtypes = [vp, C.c_char_p, P(vp)]
    lib.tnep_model_info.argtypes = [vp, P(C.c_int32), P(C.c_int32), P(C.c_int32)]
    lib.tnep_population_loss.argtypes = [vp, P(ModelDesc), C.c_int32, vp, P(FramesDesc), vp, C.c_double, C.c_double,
                                         vp, vp]
    lib.tnep_raman_map.argtypes = [vp, P(SpectrumArgs), C.c_int32, vp, vp, vp, vp]
    lib.tnep_acf_stream_create.argtypes = [vp, C.c_int32, C.c_int64, C.c_int32, vp, vp, P(vp)]
    lib.tnep_acf_stream_push.argtypes = [vp, vp, C.c_int64, C.c_int32]
    lib.tnep_acf_stream_end_run.argtypes = [vp]
    lib.tnep_acf_stream_spectrum.argtypes = [vp, C.c_double, C.c_int32, C.c_double, vp, vp, vp]
    lib.tnep_acf_stream_raman_map.argtypes = [vp, C.c_double, C.c_int32, C.c_double, C.c_int32, vp, vp, vp, vp]
    lib.tnep_acf_stream_free.argtypes = [vp]
    lib.tnep_acf_stream_free.restype = None
    lib.tnep_spectrum.argtypes = [vp, P(SpectrumArgs), vp, vp, vp]
    lib.tnep_spectrum_noalloc.argtypes = [vp, P(SpectrumArgs), vp, vp, vp]
    lib.tnep_server_start.argtypes = [vp, P(ServerOpts)]
    lib.tnep_submit.argtypes = [vp, vp, C.c_int32, P(FramesDesc), vp, P(C.c_uint64)]
    lib.tnep_wait.argtypes = [vp, C.c_uint64, P(C.c_int32), P(C.c_double)]
    lib.tnep_server_stop.argtypes = [vp]
    lib.tnep_server_stats.argtypes = [vp, P(C.c_uint64), P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
    lib.tnep_server_memory.argtypes = [vp, P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
    lib.tnep_ctx_kernel_time.argtypes = [vp, C.c_int32, P(C.c_double), P(C.c_uint64)]
    lib.tnep_ctx_pair_counts.argtypes = [vp, P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
    lib.tnep_ctx_reset_timing.argtypes = [vp]
    lib.tnep_ctx_graph_counts.argtypes = [vp, P(C.c_uint64), P(C.c_uint64)]
    lib.tnep_ctx_reuse_fallbacks.argtypes = [vp, P(C.c_uint64)]
    lib.tnep_autotune_report.argtypes = [vp]
    lib.tnep_autotune_report.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("tnep_ctx_destroy", "tnep_last_error", "tnep_model_free", "tnep_ctx_memory_in_use",
                        "tnep_autotune_report", "tnep_acf_stream_free"):
            getattr(lib, name).restype = C.c_int
    return lib


lib = _load()


def _ptr(x):
    """Address of a numpy array (host) or torch tensor (device), or None."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


class Context:
    """tnep_ctx: one GPU, one stream (hip_stream: torch.cuda.Stream or raw handle)."""

    def __init__(self, device: int = 0, stream=None, budget_bytes: int = 0):
        h = C.c_void_p()
        raw = None
        if stream is not None:
            raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        e = lib.tnep_ctx_create(device, raw, budget_bytes, C.byref(h))
        if e:
            raise TnepError(e, lib.tnep_last_error(None).decode())
        self.h = h
        self.stream = stream

    def check(self, e):
        if e:
            raise TnepError(e, lib.tnep_last_error(self.h).decode())

    def set_option(self, key, value):
        self.check(lib.tnep_set_option(self.h, key, int(value)))

    def memory_in_use(self):
        return lib.tnep_ctx_memory_in_use(self.h)

    def kernel_time(self, kernel_class):
        """(total ms, launches) of one kernel class since the last reset."""
        ms, n = C.c_double(), C.c_uint64()
        self.check(lib.tnep_ctx_kernel_time(self.h, kernel_class, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def pair_counts(self):
        """(atoms, radial pairs, angular pairs) processed since the last reset."""
        a, r, g = C.c_uint64(), C.c_uint64(), C.c_uint64()
        self.check(lib.tnep_ctx_pair_counts(self.h, C.byref(a), C.byref(r), C.byref(g)))
        return a.value, r.value, g.value

    def graph_counts(self):
        """(graphs captured, graph launches) since the context was created."""
        n, k = C.c_uint64(), C.c_uint64()
        self.check(lib.tnep_ctx_graph_counts(self.h, C.byref(n), C.byref(k)))
        return n.value, k.value

    def reuse_fallbacks(self):
        """Calls redone with plain neighbour searches (trajectory guard failed)."""
        n = C.c_uint64()
        self.check(lib.tnep_ctx_reuse_fallbacks(self.h, C.byref(n)))
        return n.value

    def reset_timing(self):
        self.check(lib.tnep_ctx_reset_timing(self.h))

    def autotune_report(self):
        return lib.tnep_autotune_report(self.h).decode()

    def close(self):
        if self.h:
            lib.tnep_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """tnep_model created from any object with the tnep_model_desc fields
    (e.g. synth.Model); heads[0] tensor head, heads[1] scalar head."""

    def __init__(self, ctx: Context, m):
        self.ctx = ctx
        self.kind = m.kind
        d, keep = model_desc(m)
        h = C.c_void_p()
        ctx.check(lib.tnep_model_create(ctx.h, C.byref(d), C.byref(h)))
        self.h = h

    @classmethod
    def load(cls, ctx: Context, path):
        """tnep_model_load: a model from a model file."""
        self = cls.__new__(cls)
        self.ctx, self.h = ctx, None
        h = C.c_void_p()
        ctx.check(lib.tnep_model_load(ctx.h, os.fsencode(path), C.byref(h)))
        self.h = h
        kind = C.c_int32()
        ctx.check(lib.tnep_model_info(h, C.byref(kind), None, None))
        self.kind = kind.value
        return self

    def close(self):
        if self.h:
            lib.tnep_model_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def model_desc(m):
    """tnep_model_desc of a model object, and the arrays it points into (keep
    them alive while the descriptor is used)."""
    keep = []

    def arr(x):
        a = np.ascontiguousarray(np.asarray(x, np.float64))
        keep.append(a)
        return a.ctypes.data_as(P(C.c_double))

    d = ModelDesc()
    d.kind = m.kind
    d.n_species = len(m.species) if hasattr(m, "species") else m.n_species
    d.rc_radial, d.rc_angular = m.rc_radial, m.rc_angular
    d.n_max_radial, d.n_max_angular = m.n_max_radial, m.n_max_angular
    d.basis_radial, d.basis_angular = m.basis_radial, m.basis_angular
    d.l_max, d.four_body, d.n_hidden = m.l_max, int(bool(m.four_body)), m.n_hidden
    d.c_radial, d.c_angular, d.q_scaler = arr(m.c_radial), arr(m.c_angular), arr(m.q_scaler)
    per_species = bool(getattr(m, "per_species", False))
    d.per_species = int(per_species)
    d.five_body = int(bool(getattr(m, "five_body", False)))
    for k, head in enumerate(m.heads):
        d.w0[k], d.b0[k], d.w1[k] = arr(head.w0), arr(head.b0), arr(head.w1)
        if per_species:
            d.b1_species[k] = arr(head.b1)
        else:
            d.b1[k] = head.b1
    return d, keep


def tnep_model_save(m, path):
    """Write a model object (tnep_model_desc fields, e.g. synth.Model) as a model file."""
    d, keep = model_desc(m)
    r = lib.tnep_model_save(C.byref(d), os.fsencode(path))
    del keep
    if r != TNEP_OK:
        raise TnepError(r, (lib.tnep_last_error(None) or b"").decode())


def frames_desc(frames, location=None):
    """Build a tnep_frames from host numpy arrays (synth.Frames) or from an
    object whose fields are torch CUDA tensors (DeviceFrames; with host_meta,
    its offsets, cells and pbc are numpy arrays: TNEP_DEVICE_META_HOST)."""
    d = FramesDesc()
    d.n_frames = int(frames.offsets.shape[0] - 1)
    if location is None:
        if isinstance(frames.positions, np.ndarray):
            location = HOST
        else:
            location = DEVICE_META_HOST if isinstance(frames.offsets, np.ndarray) else DEVICE
    if location == HOST:
        keep = (np.ascontiguousarray(frames.offsets, np.int64), np.ascontiguousarray(frames.positions, np.float64),
                np.ascontiguousarray(frames.species, np.int32),
                None if frames.cells is None else np.ascontiguousarray(frames.cells, np.float64),
                None if frames.pbc is None else np.ascontiguousarray(frames.pbc, np.uint8))
    else:
        keep = (frames.offsets, frames.positions, frames.species, frames.cells, frames.pbc)
    d.atom_offsets, d.positions, d.species, d.cells, d.pbc = [_ptr(x) for x in keep]
    d.location = location
    d._keep = keep
    return d


class DeviceFrames:
    """Frames resident in device memory as torch tensors.  host_meta: keep the
    layout (offsets, cells, pbc) as host numpy arrays (TNEP_DEVICE_META_HOST)."""

    def __init__(self, frames, device="cuda", host_meta=False):
        import torch

        def meta(x, dtype):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype)
            return a if host_meta else torch.as_tensor(a).to(device)

        self.offsets = meta(frames.offsets, np.int64)
        self.positions = torch.as_tensor(np.asarray(frames.positions, np.float64)).to(device).contiguous()
        self.species = torch.as_tensor(np.asarray(frames.species, np.int32)).to(device)
        self.cells = meta(frames.cells, np.float64)
        self.pbc = meta(frames.pbc, np.uint8)
        self.n_frames = int(frames.offsets.shape[0] - 1)
        self.n_atoms = int(frames.offsets[-1])


def tnep_eval_dipole(ctx: Context, model: Model, frames, mu_out=None, per_atom=None):
    """mu [F,3]; host arrays in -> numpy out, device tensors in -> caller's device tensors."""
    fd = frames_desc(frames)
    F = fd.n_frames
    if fd.location == HOST:
        mu_out = np.zeros((F, 3)) if mu_out is None else mu_out
    ctx.check(lib.tnep_eval_dipole(ctx.h, model.h, C.byref(fd), _ptr(mu_out), _ptr(per_atom)))
    return mu_out


def tnep_eval_polarizability(ctx: Context, model: Model, frames, alpha_out=None, per_atom=None):
    """alpha [F,3,3] (host) or the caller's [F,9] device tensor."""
    fd = frames_desc(frames)
    F = fd.n_frames
    if fd.location == HOST:
        alpha_out = np.zeros((F, 3, 3)) if alpha_out is None else alpha_out
    ctx.check(lib.tnep_eval_polarizability(ctx.h, model.h, C.byref(fd), _ptr(alpha_out), _ptr(per_atom)))
    return alpha_out


def tnep_eval_dipole_polarizability(ctx: Context, dipole_model: Model, pol_model: Model, frames, mu_out=None,
                                    alpha_out=None):
    fd = frames_desc(frames)
    F = fd.n_frames
    if fd.location == HOST:
        mu_out = np.zeros((F, 3)) if mu_out is None else mu_out
        alpha_out = np.zeros((F, 3, 3)) if alpha_out is None else alpha_out
    ctx.check(lib.tnep_eval_dipole_polarizability(ctx.h, dipole_model.h, pol_model.h, C.byref(fd), _ptr(mu_out),
                                                  _ptr(alpha_out)))
    return mu_out, alpha_out


def tnep_eval_dipole_charged(ctx: Context, model: Model, frames, charges, species_masses, length_unit=1.0,
                             mu_out=None, per_atom=None):
    """mu = mu_r + Q e r_COM: charges [F] (numpy for host frames, device tensor
    for device frames), species_masses [n_species] host."""
    fd = frames_desc(frames)
    F = fd.n_frames
    if fd.location == HOST:
        mu_out = np.zeros((F, 3)) if mu_out is None else mu_out
        charges = np.ascontiguousarray(charges, np.float64)
    masses = np.ascontiguousarray(species_masses, np.float64)
    ctx.check(lib.tnep_eval_dipole_charged(ctx.h, model.h, C.byref(fd), _ptr(charges), _ptr(masses),
                                           float(length_unit), _ptr(mu_out), _ptr(per_atom)))
    return mu_out


def tnep_population_loss(ctx: Context, base, params, frames, reference, lambda1=0.0, lambda2=0.0):
    """Loss and RMSE [P] of each parameter vector params [P, N] (layout of
    synth.pack_params) with base's hyperparameters, over frames against
    reference [F, nt] (numpy for host frames, device tensor for device frames)."""
    d, keep = model_desc(base)
    params = np.ascontiguousarray(params, np.float64)
    fd = frames_desc(frames)
    if fd.location == HOST:
        reference = np.ascontiguousarray(reference, np.float64)
    n = params.shape[0]
    loss, rmse = np.zeros(n), np.zeros(n)
    ctx.check(lib.tnep_population_loss(ctx.h, C.byref(d), n, _ptr(params), C.byref(fd), _ptr(reference),
                                       float(lambda1), float(lambda2), _ptr(loss), _ptr(rmse)))
    del keep
    return loss, rmse


def tnep_eval_pes(ctx: Context, model: Model, frames, energy=None, virial=None, forces=None, per_atom_energy=None,
                  want_virial=True, want_forces=True):
    """Potential-energy surface: (energy [F], virial [F,3,3] or None, forces [A,3] or None).
    Host frames -> numpy outputs (allocated unless given); device frames ->
    the caller's device tensors (pass None to skip virial / forces)."""
    fd = frames_desc(frames)
    F = fd.n_frames
    if fd.location == HOST:
        energy = np.zeros(F) if energy is None else energy
        if want_virial and virial is None:
            virial = np.zeros((F, 3, 3))
        if want_forces and forces is None:
            forces = np.zeros((int(np.asarray(frames.offsets)[-1]), 3))
    ctx.check(lib.tnep_eval_pes(ctx.h, model.h, C.byref(fd), _ptr(energy), _ptr(virial), _ptr(forces),
                                _ptr(per_atom_energy)))
    return energy, virial, forces


def tnep_spectrum(ctx: Context, series, kind, dt_fs, max_lag, window=WIN_HANN, flags=0, n_hat=(0, 0, 0),
                  e_hat=(0, 0, 0), freq=None, intensity=None, acf=None, want_acf=True, laser_cm1=0.0):
    """series [S, N_t, 3|9] (numpy: host; torch CUDA: device, outputs must be given)."""
    a = SpectrumArgs()
    a.kind = kind
    a.n_series, a.n_steps = int(series.shape[0]), int(series.shape[1])
    a.dt_fs, a.max_lag, a.window, a.flags = dt_fs, int(max_lag), window, flags
    a.laser_cm1 = float(laser_cm1)
    for k in range(3):
        a.n_hat[k], a.e_hat[k] = n_hat[k], e_hat[k]
    if isinstance(series, np.ndarray):
        series = np.ascontiguousarray(series, np.float64)
        a.location = HOST
        M = int(max_lag)
        freq = np.zeros(M + 1) if freq is None else freq
        intensity = np.zeros(M + 1) if intensity is None else intensity
        if want_acf and acf is None:
            acf = np.zeros(M)
    else:
        a.location = DEVICE
    a.series = _ptr(series)
    ctx.check(lib.tnep_spectrum(ctx.h, C.byref(a), _ptr(freq), _ptr(intensity), _ptr(acf)))
    return freq, intensity, acf


def tnep_spectrum_noalloc(ctx: Context, series, kind, dt_fs, max_lag, freq, intensity, acf=None, window=WIN_HANN,
                          flags=0, n_hat=(0, 0, 0), e_hat=(0, 0, 0), laser_cm1=0.0):
    """tnep_spectrum on device tensors with the library's fixed workspace (no
    device allocation); enqueued on the context's stream, not waited for.
    series [S, N_t, 3|9], freq and intensity [M+1], acf [M] or None: torch
    CUDA tensors."""
    a = SpectrumArgs()
    a.kind = kind
    a.n_series, a.n_steps = int(series.shape[0]), int(series.shape[1])
    a.dt_fs, a.max_lag, a.window, a.flags = dt_fs, int(max_lag), window, flags
    a.laser_cm1 = float(laser_cm1)
    for k in range(3):
        a.n_hat[k], a.e_hat[k] = n_hat[k], e_hat[k]
    # numpy input is reported as host memory, which the library rejects
    a.location = HOST if isinstance(series, np.ndarray) else DEVICE
    a.series = _ptr(series)
    ctx.check(lib.tnep_spectrum_noalloc(ctx.h, C.byref(a), _ptr(freq), _ptr(intensity), _ptr(acf)))
    return freq, intensity, acf


def tnep_raman_map(ctx: Context, series, dt_fs, max_lag, n_hats, e_hats, window=WIN_HANN, flags=0, laser_cm1=0.0,
                   freq=None, intensity=None):
    """Orientation map: series [S, N_t, 9]; n_hats, e_hats [n_orient, 3] (host).
    Returns (freq [M+1], intensity [n_orient, M+1])."""
    n_hats = np.ascontiguousarray(n_hats, np.float64).reshape(-1, 3)
    e_hats = np.ascontiguousarray(e_hats, np.float64).reshape(-1, 3)
    a = SpectrumArgs()
    a.kind = RAMAN_PROJ
    a.n_series, a.n_steps = int(series.shape[0]), int(series.shape[1])
    a.dt_fs, a.max_lag, a.window, a.flags, a.laser_cm1 = dt_fs, int(max_lag), window, flags, float(laser_cm1)
    M = int(max_lag)
    if isinstance(series, np.ndarray):
        series = np.ascontiguousarray(series, np.float64)
        a.location = HOST
        freq = np.zeros(M + 1) if freq is None else freq
        intensity = np.zeros((len(n_hats), M + 1)) if intensity is None else intensity
    else:
        a.location = DEVICE
    a.series = _ptr(series)
    ctx.check(lib.tnep_raman_map(ctx.h, C.byref(a), len(n_hats), _ptr(n_hats), _ptr(e_hats), _ptr(freq),
                                 _ptr(intensity)))
    return freq, intensity


class AcfStream:
    """Streaming correlation accumulator (tnep_acf_stream_*)."""

    def __init__(self, ctx: Context, kind, max_lag, flags=0, n_hat=None, e_hat=None):
        self.ctx, self.kind, self.M = ctx, kind, int(max_lag)
        nh = None if n_hat is None else np.ascontiguousarray(n_hat, np.float64)
        eh = None if e_hat is None else np.ascontiguousarray(e_hat, np.float64)
        h = C.c_void_p()
        ctx.check(lib.tnep_acf_stream_create(ctx.h, kind, self.M, flags, _ptr(nh), _ptr(eh), C.byref(h)))
        self.h = h

    def push(self, samples):
        if isinstance(samples, np.ndarray):
            samples = np.ascontiguousarray(samples, np.float64)
            loc = HOST
        else:
            loc = DEVICE
        self.ctx.check(lib.tnep_acf_stream_push(self.h, _ptr(samples), int(samples.shape[0]), loc))

    def end_run(self):
        self.ctx.check(lib.tnep_acf_stream_end_run(self.h))

    def spectrum(self, dt_fs, window=WIN_HANN, laser_cm1=0.0):
        f, s, a = np.zeros(self.M + 1), np.zeros(self.M + 1), np.zeros(self.M)
        self.ctx.check(lib.tnep_acf_stream_spectrum(self.h, dt_fs, window, float(laser_cm1), _ptr(f), _ptr(s), _ptr(a)))
        return f, s, a

    def raman_map(self, dt_fs, n_hats, e_hats, window=WIN_HANN, laser_cm1=0.0):
        n_hats = np.ascontiguousarray(n_hats, np.float64).reshape(-1, 3)
        e_hats = np.ascontiguousarray(e_hats, np.float64).reshape(-1, 3)
        f, s = np.zeros(self.M + 1), np.zeros((len(n_hats), self.M + 1))
        self.ctx.check(lib.tnep_acf_stream_raman_map(self.h, dt_fs, window, float(laser_cm1), len(n_hats),
                                                     _ptr(n_hats), _ptr(e_hats), _ptr(f), _ptr(s)))
        return f, s

    def close(self):
        if self.h:
            lib.tnep_acf_stream_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server on a context (tnep_server_*).  Requests are
    host numpy frames; their buffers stay referenced until wait()."""

    def __init__(self, ctx: Context, budget_bytes: int = 0, max_batch_atoms: int = 0, max_inflight: int = 0):
        self.ctx = ctx
        o = ServerOpts()
        o.mem_budget_bytes, o.max_batch_atoms, o.max_inflight = budget_bytes, max_batch_atoms, max_inflight
        ctx.check(lib.tnep_server_start(ctx.h, C.byref(o)))
        self._live = {}

    def submit(self, model: Model, frames, out=None):
        fd = frames_desc(frames, HOST)
        nt = 3 if model.kind == KIND_DIPOLE else 9
        if out is None:
            out = np.zeros((fd.n_frames, nt))
        t = C.c_uint64()
        e = lib.tnep_submit(self.ctx.h, model.h, model.kind, C.byref(fd), _ptr(out), C.byref(t))
        if e:
            raise TnepError(e, "submit rejected")
        self._live[t.value] = (fd, out)
        return t.value

    def wait(self, ticket):
        """(status, latency_s, output array)."""
        st, lat = C.c_int32(), C.c_double()
        self.ctx.check(lib.tnep_wait(self.ctx.h, ticket, C.byref(st), C.byref(lat)))
        fd, out = self._live.pop(ticket)
        return st.value, lat.value, out

    def stats(self):
        r, l, a, p = C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_uint64()
        self.ctx.check(lib.tnep_server_stats(self.ctx.h, C.byref(r), C.byref(l), C.byref(a), C.byref(p)))
        return {"requests": r.value, "launches": l.value, "atom_frames": a.value, "peak_bytes": p.value}

    def memory(self):
        """(pool bytes, bytes granted to slots now, times a slot waited for pool memory)."""
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        self.ctx.check(lib.tnep_server_memory(self.ctx.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def stop(self):
        self.ctx.check(lib.tnep_server_stop(self.ctx.h))
