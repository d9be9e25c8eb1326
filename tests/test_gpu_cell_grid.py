"""Cell grids of orthorhombic frames on the GPU against the FP64 oracle.

The search bins fully periodic orthorhombic frames into cells of edge >=
r_c / 2 (at least five per axis), walks 5 x 5 columns of cells trimmed to
the z-cells in reach, and forms pair vectors from fixed-point offsets within
the cells.  These cases exercise the grid shapes that the water benchmark
does not: exactly five cells per axis (edges between 2.5 and 3 r_c, which a
grid of r_c cells could not serve), unequal cell counts per axis, a sparse
frame whose grid is coarsened, atoms given far outside the box, trajectory
reuse on such a grid, and all of them in one call; and the same shapes for
the fractional bins of skewed cells.  Bound: per-frame
relative Frobenius error <= 1e-5 (tests/parity.py).
"""
import numpy as np
import pytest

import oracle
import synth
from parity import TENSOR_TOL, frame_errors

pytestmark = pytest.mark.gpu

def _lattice_frame(L, spacing, seed, jitter=0.25, unwrap=0):
    """Jittered simple-cubic lattice filling an L[0] x L[1] x L[2] box (no two
    atoms closer than spacing - 2 jitter), species 0/1 at random; `unwrap`
    atoms are moved by random whole box vectors."""
    rng = np.random.default_rng(seed)
    n = [max(1, int(np.floor(l / spacing))) for l in L]
    h = [l / k for l, k in zip(L, n)]
    g = np.stack(np.meshgrid(*[np.arange(k) * s for k, s in zip(n, h)], indexing="ij"), -1).reshape(-1, 3)
    pos = g + rng.uniform(-jitter, jitter, g.shape)
    spc = rng.integers(0, 2, len(pos)).astype(np.int32)
    if unwrap:
        idx = rng.choice(len(pos), unwrap, replace=False)
        pos[idx] += rng.integers(-3, 4, (unwrap, 3)) * np.asarray(L)
    return pos, spc, np.diag(np.asarray(L, np.float64)).reshape(9)


def _sparse_frame(L, n_clusters, per_cluster, seed, min_sep=1.3):
    """A few clusters of atoms (radius 3 A) in a large box, the first one at
    the box corner so that its pairs cross the faces."""
    rng = np.random.default_rng(seed)
    centres = np.vstack([np.zeros((1, 3)), rng.uniform(0, L, (n_clusters - 1, 3))])
    pts = []
    for c in centres:
        k = 0
        while k < per_cluster:
            p = c + rng.uniform(-3.0, 3.0, 3)
            if all(np.linalg.norm((p - q) - L * np.rint((p - q) / L)) >= min_sep for q in pts):
                pts.append(p)
                k += 1
    n = len(pts)
    return np.array(pts), rng.integers(0, 2, n).astype(np.int32), np.diag([L, L, L]).reshape(9).astype(np.float64)


def _frames(items):
    offs = np.cumsum([0] + [len(s) for _, s, _ in items]).astype(np.int64)
    return synth.Frames(offs, np.concatenate([p for p, _, _ in items]), np.concatenate([s for _, s, _ in items]),
                        np.stack([c for _, _, c in items]), np.ones((len(items), 3), np.uint8))


CASES = {
    # edges (15.5, 18.3, 30.2): 5, 6 and 10 cells
    "unequal_5_6_10": ((15.5, 18.3, 30.2), 1.9, 11, 40),
    # 16 A cube: 5 cells of 3.2 A per axis, every column wraps in z
    "five_cells": ((16.0, 16.0, 16.0), 1.9, 12, 25),
    # 15 A cube: exactly 2.5 r_c
    "edge_2p5_rc": ((15.0, 15.0, 15.0), 1.8, 13, 0),
}


def _items():
    items = [_lattice_frame(L, sp, seed, unwrap=u) for L, sp, seed, u in CASES.values()]
    items.append(_sparse_frame(60.0, 6, 6, 14))  # 36 atoms: 20^3 cells coarsened to 5^3
    return items


def _check(gpu, m, fr, label):
    ref, pa = oracle.eval_frames(m, fr, per_atom=True)
    err = frame_errors(gpu, ref, pa, fr.offsets)
    print(label, np.array2string(err, precision=2), flush=True)
    assert np.all(err <= TENSOR_TOL), label


@pytest.mark.parametrize("name", ["water_dipole_small", "water_polarizability"])
def test_grids_one_frame_per_call(gpu_lib, name):
    m = synth.model(name)
    ctx = gpu_lib.Context(0)
    g = gpu_lib.Model(ctx, m)
    f = gpu_lib.tnep_eval_dipole if m.kind == synth.KIND_DIPOLE else gpu_lib.tnep_eval_polarizability
    for label, item in zip(list(CASES) + ["sparse_coarsened"], _items()):
        fr = _frames([item])
        _check(f(ctx, g, fr), m, fr, f"{name} {label}")
    ctx.close()


def test_grids_batched_match_single_calls(gpu_lib):
    """All grids in one call: per-frame results bitwise those of one call per
    frame (frame sums depend only on the frame), and within the oracle bound."""
    m = synth.model("water_polarizability")
    items = _items()
    fr = _frames(items)
    ctx = gpu_lib.Context(0)
    g = gpu_lib.Model(ctx, m)
    batched = gpu_lib.tnep_eval_polarizability(ctx, g, fr)
    _check(batched, m, fr, "batched")
    for k, item in enumerate(items):
        single = gpu_lib.tnep_eval_polarizability(ctx, g, _frames([item]))
        assert np.array_equal(single[0], batched[k]), k
    ctx.close()


def test_trajectory_reuse_on_unequal_grid(gpu_lib):
    """Reference frames search out to r_c + skin = 7 A on their own grid (5 x 6
    x 8 cells here, against 6 x 7 x 10 for r_c); followers reuse their
    candidates."""
    L = (18.0, 21.0, 30.2)
    pos, spc, cell = _lattice_frame(L, 1.9, 21)
    traj = synth.ou_trajectory(pos, spc, cell, 12, seed=22)
    m = synth.model("water_dipole_small")
    plain, reuse = gpu_lib.Context(0), gpu_lib.Context(0)
    reuse.set_option(gpu_lib.OPT_TRAJECTORY_WINDOW, 6)
    reuse.set_option(gpu_lib.OPT_SKIN_MA, 1000)
    a = gpu_lib.tnep_eval_dipole(plain, gpu_lib.Model(plain, m), traj)
    b = gpu_lib.tnep_eval_dipole(reuse, gpu_lib.Model(reuse, m), traj)
    assert reuse.reuse_fallbacks() == 0
    assert frame_errors(b, a).max() <= 5e-6
    sub = traj.subset([0, 5, 11])
    _check(b[[0, 5, 11]], m, sub, "reuse")
    for c in (plain, reuse):
        c.close()


def _skewed_frame(L, shear, n, seed, min_sep=1.3):
    """Random atoms (no two closer than min_sep under the minimum image) in a
    skewed, rotated cell; fractional coordinates drawn from [-0.5, 1.5) so that
    many atoms lie outside the cell as given."""
    rng = np.random.default_rng(seed)
    R, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    H = np.array([[L, 0, 0], [shear * L, L, 0], [0.1 * L, -shear * L, 1.1 * L]]) @ R.T
    Hinv = np.linalg.inv(H)
    pts = []
    while len(pts) < n:
        r = rng.uniform(-0.5, 1.5, 3) @ H
        if all(np.linalg.norm(((((r - q) @ Hinv) + 0.5) % 1.0 - 0.5) @ H) >= min_sep for q in pts):
            pts.append(r)
    return np.array(pts), rng.integers(0, 2, n).astype(np.int32), H.reshape(9)


SKEWED = {
    # perpendicular widths ~15.1, 15.4, 17.6 A: 5 bins of >= r_c / 2 per axis
    "skewed_five_bins": (16.0, 0.3, 200, 31),
    # widths ~17.2, 18.2, 22.0 A: 5, 6 and 7 bins
    "skewed_5_6_7": (20.0, 0.5, 300, 32),
    # widths ~29-33 A with 120 atoms: the grid is coarsened to about two bins per atom
    "skewed_coarsened": (30.0, 0.2, 120, 33),
}


@pytest.mark.parametrize("name", ["water_dipole_small", "water_polarizability"])
def test_triclinic_bins(gpu_lib, name):
    m = synth.model(name)
    ctx = gpu_lib.Context(0)
    g = gpu_lib.Model(ctx, m)
    f = gpu_lib.tnep_eval_dipole if m.kind == synth.KIND_DIPOLE else gpu_lib.tnep_eval_polarizability
    items = [_skewed_frame(*args) for args in SKEWED.values()]
    for label, item in zip(SKEWED, items):
        fr = _frames([item])
        _check(f(ctx, g, fr), m, fr, f"{name} {label}")
    batched = f(ctx, g, _frames(items))
    for k, item in enumerate(items):
        assert np.array_equal(batched[k], f(ctx, g, _frames([item]))[0]), k
    ctx.close()


def test_pes_forces_on_grids(gpu_lib):
    """Potential-energy model on the grid shapes above, orthorhombic and
    skewed: energy, virial and forces against the oracle, and the forces of a
    frame summing to zero.  The force kernel reads each pair force that the
    neighbour's evaluation stored at its own entry for the atom, so it relies
    on both atoms of a pair sorting it into the same (angular or radial-only)
    segment."""
    m = synth.model("water_pes")
    ctx = gpu_lib.Context(0)
    g = gpu_lib.Model(ctx, m)
    items = [_lattice_frame(*CASES["five_cells"][:3], unwrap=10), _skewed_frame(*SKEWED["skewed_5_6_7"]),
             _skewed_frame(*SKEWED["skewed_five_bins"])]
    fr = _frames(items)
    E, W, F = gpu_lib.tnep_eval_pes(ctx, g, fr)
    Er, Wr, Fr, Ur = oracle.eval_pes(m, fr, per_atom=True)
    off = fr.offsets
    for f in range(fr.n_frames):
        sl = slice(off[f], off[f + 1])
        assert abs(E[f] - Er[f]) <= TENSOR_TOL * np.abs(Ur[sl]).sum(), f
        ferr = np.linalg.norm(F[sl] - Fr[sl]) / np.linalg.norm(Fr[sl])
        net = np.linalg.norm(F[sl].sum(0)) / np.abs(F[sl]).sum()
        print(f"pes frame {f}: forces {ferr:.2e}, net force / sum |F| {net:.1e}", flush=True)
        assert ferr <= TENSOR_TOL and net <= 1e-6, f
    assert np.all(frame_errors(W, Wr) <= TENSOR_TOL)
    ctx.close()
