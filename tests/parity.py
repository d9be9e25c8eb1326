"""Tolerance metric shared by the GPU parity tests, the smoke check and the
benchmark: per-frame relative Frobenius error of a tensor.

err_f = ||T_gpu - T_ref||_F / max(||T_ref||_F, 1e-3 sum_i ||T_i,ref||_F)

The second term guards frames whose atom terms cancel almost exactly
(e.g. a near-centrosymmetric lattice dipole): there the error is measured
against the size of the atom terms instead.  Bound: 1e-5 for tensors.
"""
import numpy as np

TENSOR_TOL = 1e-5
SPECTRUM_TOL = 1e-4


def frame_errors(gpu, ref, ref_per_atom=None, offsets=None):
    gpu = np.asarray(gpu, np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, np.float64).reshape(len(ref), -1)
    num = np.linalg.norm(gpu - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    if ref_per_atom is not None and offsets is not None:
        pa = np.linalg.norm(np.asarray(ref_per_atom).reshape(int(offsets[-1]), -1), axis=1)
        sums = np.array([pa[offsets[f]:offsets[f + 1]].sum() for f in range(len(ref))])
        den = np.maximum(den, 1e-3 * sums)
    den = np.where(den > 0, den, 1.0)
    return num / den


def spectrum_error(gpu, ref):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(gpu - ref)) / max(np.max(np.abs(ref)), 1e-300))
