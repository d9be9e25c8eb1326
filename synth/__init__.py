"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds random numbers and data layout only: it performs none of
the method's arithmetic.  It builds

* frames: liquid-water boxes, Ornstein-Uhlenbeck displacement trajectories,
  a cubic ABO3 (Ba/Zr/O) perovskite supercell with thermal displacements,
  and ragged bonded-chain molecules in vacuum;
* models: TNEP dipole / polarizability parameter sets drawn from a seed.

The workloads are stand-ins for the paper's water, BaZrO3 and molecular
data sets (Sec. 3 Performance evaluation and Sec. 4 Applications), which are
not available here.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import List, Optional

import numpy as np

KIND_DIPOLE = 1
KIND_POLARIZABILITY = 2
KIND_PES = 3  # potential-energy surface: one head, the site energy

WATER_SPECIES = ("O", "H")
PEROVSKITE_SPECIES = ("Ba", "Zr", "O")
MOLECULE_SPECIES = ("C", "H", "N", "O", "F")

_GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")


# --------------------------------------------------------------------------
# Frames


@dataclasses.dataclass
class Frames:
    """A batch of ragged frames, CSR by atom.

    offsets   int64 [F+1]   atoms of frame f are offsets[f]:offsets[f+1]
    positions float64 [A,3] Angstrom
    species   int32 [A]     index into the model's species list
    cells     float64 [F,9] row-major lattice vectors, or None (vacuum)
    pbc       uint8 [F,3]   periodic flags, or None (vacuum)
    """

    offsets: np.ndarray
    positions: np.ndarray
    species: np.ndarray
    cells: Optional[np.ndarray] = None
    pbc: Optional[np.ndarray] = None

    @property
    def n_frames(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_atoms(self) -> int:
        return int(self.offsets[-1])

    def subset(self, frames) -> "Frames":
        frames = list(frames)
        sizes = [int(self.offsets[f + 1] - self.offsets[f]) for f in frames]
        offs = np.zeros(len(frames) + 1, np.int64)
        offs[1:] = np.cumsum(sizes)
        idx = np.concatenate([np.arange(self.offsets[f], self.offsets[f + 1]) for f in frames]) if frames else np.zeros(0, np.int64)
        return Frames(
            offs,
            np.ascontiguousarray(self.positions[idx]),
            np.ascontiguousarray(self.species[idx]),
            None if self.cells is None else np.ascontiguousarray(self.cells[frames]),
            None if self.pbc is None else np.ascontiguousarray(self.pbc[frames]),
        )

    @staticmethod
    def concat(parts: List["Frames"]) -> "Frames":
        offs = [np.zeros(1, np.int64)]
        base = 0
        for p in parts:
            offs.append(p.offsets[1:] + base)
            base += p.n_atoms
        periodic = any(p.cells is not None for p in parts)
        cells = pbc = None
        if periodic:
            cells = np.concatenate([p.cells if p.cells is not None else np.zeros((p.n_frames, 9)) for p in parts])
            pbc = np.concatenate([p.pbc if p.pbc is not None else np.zeros((p.n_frames, 3), np.uint8) for p in parts])
        return Frames(
            np.concatenate(offs),
            np.ascontiguousarray(np.concatenate([p.positions for p in parts])),
            np.ascontiguousarray(np.concatenate([p.species for p in parts]).astype(np.int32)),
            cells,
            pbc,
        )


def _random_rotations(rng, n):
    """Uniform random rotation matrices (QR of Gaussian matrices, sign-fixed)."""
    g = rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diagonal(r, axis1=1, axis2=2))
    q = q * d[:, None, :]
    det = np.linalg.det(q)
    q[det < 0, :, 0] *= -1.0
    return q


def water_box(n_side: int, box: float, seed: int, jitter: float = 0.3, oh: float = 0.96,
              angle_deg: float = 104.5, o_species: int = 0, h_species: int = 1):
    """One periodic liquid-water-like frame: n_side^3 molecules.

    O on a cubic lattice of spacing box/n_side plus N(0, jitter^2) per
    coordinate; two H at `oh` Angstrom with the H-O-H angle `angle_deg`,
    molecule orientation uniformly random.  Atom order O, H, H per molecule.
    Returns (positions [3 n_side^3, 3], species [.], cell [9]).
    """
    rng = np.random.default_rng(seed)
    n_mol = n_side ** 3
    a = box / n_side
    grid = np.stack(np.meshgrid(np.arange(n_side), np.arange(n_side), np.arange(n_side), indexing="ij"), -1)
    o = (grid.reshape(-1, 3) + 0.5) * a + rng.normal(0.0, jitter, (n_mol, 3))
    half = np.deg2rad(angle_deg) / 2.0
    local = np.array([[np.sin(half), 0.0, np.cos(half)], [-np.sin(half), 0.0, np.cos(half)]]) * oh
    rot = _random_rotations(rng, n_mol)
    h = o[:, None, :] + np.einsum("mij,hj->mhi", rot, local)
    pos = np.concatenate([o[:, None, :], h], axis=1).reshape(-1, 3)
    pos = np.mod(pos, box)
    spc = np.tile(np.array([o_species, h_species, h_species], np.int32), n_mol)
    cell = np.diag([box, box, box]).reshape(9).astype(np.float64)
    return pos, spc, cell


def water_box_orthorhombic(counts, spacing: float, seed: int, jitter: float = 0.3, oh: float = 0.96,
                           angle_deg: float = 104.5, o_species: int = 0, h_species: int = 1):
    """Like water_box on an orthorhombic lattice of counts = (nx, ny, nz)
    molecules with the given O spacing (e.g. 16 x 16 x 32 = 8192 H2O, 24,576
    atoms, in a 49.7 x 49.7 x 99.4 A box at the 3.105 A spacing of the water
    workloads).  Returns (positions, species, cell [9])."""
    rng = np.random.default_rng(seed)
    counts = np.asarray(counts, np.int64)
    n_mol = int(np.prod(counts))
    box = counts * spacing
    grid = np.stack(np.meshgrid(*[np.arange(c) for c in counts], indexing="ij"), -1)
    o = (grid.reshape(-1, 3) + 0.5) * spacing + rng.normal(0.0, jitter, (n_mol, 3))
    half = np.deg2rad(angle_deg) / 2.0
    local = np.array([[np.sin(half), 0.0, np.cos(half)], [-np.sin(half), 0.0, np.cos(half)]]) * oh
    rot = _random_rotations(rng, n_mol)
    h = o[:, None, :] + np.einsum("mij,hj->mhi", rot, local)
    pos = np.mod(np.concatenate([o[:, None, :], h], axis=1).reshape(-1, 3), box)
    spc = np.tile(np.array([o_species, h_species, h_species], np.int32), n_mol)
    return pos, spc, np.diag(box.astype(np.float64)).reshape(9)


def water_frames(n_side: int, box: float, n_frames: int, seed: int, **kw) -> Frames:
    """n_frames independent water boxes (seeds seed*1000 + f)."""
    parts = []
    for f in range(n_frames):
        pos, spc, cell = water_box(n_side, box, seed * 1000 + f, **kw)
        parts.append(Frames(np.array([0, len(spc)], np.int64), pos, spc, cell[None, :], np.ones((1, 3), np.uint8)))
    return Frames.concat(parts)


def ou_trajectory(pos0: np.ndarray, spc: np.ndarray, cell: np.ndarray, n_frames: int, seed: int,
                  sigma: float = 0.02, tau: float = 50.0, wrap: bool = True) -> Frames:
    """Ornstein-Uhlenbeck displacement walk d_{t+1} = e^{-1/tau} d_t + sigma xi,
    d_0 = 0, applied per atom and coordinate to the reference frame pos0."""
    rng = np.random.default_rng(seed)
    n = pos0.shape[0]
    decay = np.exp(-1.0 / tau)
    out = np.empty((n_frames, n, 3), np.float64)
    d = np.zeros((n, 3))
    box = np.array([cell[0], cell[4], cell[8]])
    for t in range(n_frames):
        p = pos0 + d
        out[t] = np.mod(p, box) if wrap else p
        d = decay * d + sigma * rng.standard_normal((n, 3))
    offs = np.arange(n_frames + 1, dtype=np.int64) * n
    return Frames(offs, out.reshape(-1, 3), np.tile(spc, n_frames).astype(np.int32),
                  np.tile(cell, (n_frames, 1)), np.ones((n_frames, 3), np.uint8))


def perovskite_frames(n_rep: int, a: float, n_frames: int, seed: int, sigma: float = 0.08) -> Frames:
    """Cubic ABO3 supercell (A = Ba at 0, B = Zr at body centre, O at face
    centres), n_rep^3 cells of edge a, with N(0, sigma^2) displacements
    drawn independently per frame.  sigma = 0 gives the ideal lattice."""
    rng = np.random.default_rng(seed)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0.5], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    bsp = np.array([0, 1, 2, 2, 2], np.int32)
    grid = np.stack(np.meshgrid(np.arange(n_rep), np.arange(n_rep), np.arange(n_rep), indexing="ij"), -1).reshape(-1, 3)
    ideal = ((grid[:, None, :] + basis[None, :, :]) * a).reshape(-1, 3)
    spc = np.tile(bsp, grid.shape[0])
    box = n_rep * a
    n = ideal.shape[0]
    pos = np.empty((n_frames, n, 3))
    for f in range(n_frames):
        pos[f] = np.mod(ideal + (rng.normal(0.0, sigma, (n, 3)) if sigma > 0 else 0.0), box)
    cell = np.diag([box, box, box]).reshape(9)
    return Frames(np.arange(n_frames + 1, dtype=np.int64) * n, pos.reshape(-1, 3),
                  np.tile(spc, n_frames).astype(np.int32), np.tile(cell, (n_frames, 1)),
                  np.ones((n_frames, 3), np.uint8))


def molecule(rng, n_atoms: int, n_species: int = 5, bond=(1.0, 1.5), min_sep: float = 1.0,
             noise: float = 0.05):
    """Random-walk bonded chain: bond lengths U(bond), isotropic directions;
    a step is redrawn if the new atom comes closer than min_sep to any atom
    other than its bonded predecessor; then N(0, noise^2) per coordinate."""
    pos = np.zeros((n_atoms, 3))
    for i in range(1, n_atoms):
        for _attempt in range(1000):
            v = rng.standard_normal(3)
            v /= np.linalg.norm(v)
            cand = pos[i - 1] + v * rng.uniform(*bond)
            if i < 2 or np.min(np.linalg.norm(pos[: i - 1] - cand, axis=1)) >= min_sep:
                break
        pos[i] = cand
    pos += rng.normal(0.0, noise, pos.shape)
    spc = rng.integers(0, n_species, n_atoms).astype(np.int32)
    return pos, spc


def molecule_frames(n_frames: int, seed: int, n_min: int = 20, n_max: int = 80) -> Frames:
    """n_frames vacuum molecules of U{n_min..n_max} atoms, species uniform."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_min, n_max + 1, n_frames)
    pos, spc = [], []
    for n in sizes:
        p, s = molecule(rng, int(n))
        pos.append(p)
        spc.append(s)
    offs = np.zeros(n_frames + 1, np.int64)
    offs[1:] = np.cumsum(sizes)
    return Frames(offs, np.concatenate(pos), np.concatenate(spc).astype(np.int32), None, None)


# --------------------------------------------------------------------------
# Models


@dataclasses.dataclass
class Head:
    w0: np.ndarray  # [H, D]  ([T, H, D] for per-species networks)
    b0: np.ndarray  # [H]     ([T, H])
    w1: np.ndarray  # [H]     ([T, H])
    b1: float       # scalar  ([T] array)


@dataclasses.dataclass
class Model:
    """TNEP parameter set.  heads[0] is the tensor head (virial term; for a
    potential-energy model, the site energy); heads[1], polarizability only,
    is the scalar head (the U_i delta term)."""

    kind: int
    species: tuple
    rc_radial: float
    rc_angular: float
    n_max_radial: int
    n_max_angular: int
    basis_radial: int
    basis_angular: int
    l_max: int
    four_body: bool
    n_hidden: int
    c_radial: np.ndarray  # [T, T, n_R+1, K_R+1]
    c_angular: np.ndarray  # [T, T, n_A+1, K_A+1]
    q_scaler: np.ndarray  # [D]
    heads: List[Head]
    per_species: bool = False  # one network per centre species
    five_body: bool = False  # l = 1 five-body invariants (after the four-body block)

    @property
    def n_species(self) -> int:
        return len(self.species)

    @property
    def dim(self) -> int:
        """Descriptor length: radial, then l = 1..l_max angular blocks, then 4-body, then 5-body."""
        na = self.n_max_angular + 1
        return self.n_max_radial + 1 + na * self.l_max + (na if self.four_body else 0) + \
            (na if self.five_body else 0)

    def to_json(self) -> dict:
        return {
            "kind": self.kind, "species": list(self.species), "rc_radial": self.rc_radial,
            "rc_angular": self.rc_angular, "n_max_radial": self.n_max_radial,
            "n_max_angular": self.n_max_angular, "basis_radial": self.basis_radial,
            "basis_angular": self.basis_angular, "l_max": self.l_max, "four_body": bool(self.four_body),
            "n_hidden": self.n_hidden, "c_radial": self.c_radial.tolist(), "c_angular": self.c_angular.tolist(),
            "q_scaler": self.q_scaler.tolist(),
            "heads": [{"w0": np.asarray(h.w0).tolist(), "b0": np.asarray(h.b0).tolist(),
                       "w1": np.asarray(h.w1).tolist(), "b1": np.asarray(h.b1).tolist()} for h in self.heads],
            "per_species": bool(self.per_species), "five_body": bool(self.five_body),
        }

    @staticmethod
    def from_json(d: dict) -> "Model":
        return Model(
            d["kind"], tuple(d["species"]), d["rc_radial"], d["rc_angular"], d["n_max_radial"],
            d["n_max_angular"], d["basis_radial"], d["basis_angular"], d["l_max"], d["four_body"],
            d["n_hidden"], np.array(d["c_radial"], np.float64), np.array(d["c_angular"], np.float64),
            np.array(d["q_scaler"], np.float64),
            [Head(np.array(h["w0"], np.float64), np.array(h["b0"], np.float64), np.array(h["w1"], np.float64),
                  np.array(h["b1"], np.float64) if d.get("per_species") else float(h["b1"])) for h in d["heads"]],
            bool(d.get("per_species", False)), bool(d.get("five_body", False)),
        )


def make_model(seed: int, kind: int, species, rc_radial: float, rc_angular: float, n_max_radial: int,
               n_max_angular: int, basis_radial: int, basis_angular: int, l_max: int, four_body: bool,
               n_hidden: int, scale: float = 0.1, q_scaler=None, five_body: bool = False) -> Model:
    """All parameters ~ N(0, scale^2) from `seed`; q_scaler defaults to ones."""
    rng = np.random.default_rng(seed)
    T = len(species)
    cr = rng.normal(0.0, scale, (T, T, n_max_radial + 1, basis_radial + 1))
    ca = rng.normal(0.0, scale, (T, T, n_max_angular + 1, basis_angular + 1))
    na = n_max_angular + 1
    D = n_max_radial + 1 + na * l_max + (na if four_body else 0) + (na if five_body else 0)
    heads = []
    for _ in range(2 if kind == KIND_POLARIZABILITY else 1):
        heads.append(Head(rng.normal(0.0, scale, (n_hidden, D)), rng.normal(0.0, scale, n_hidden),
                          rng.normal(0.0, scale, n_hidden), float(rng.normal(0.0, scale))))
    qs = np.ones(D) if q_scaler is None else np.asarray(q_scaler, np.float64)
    return Model(kind, tuple(species), rc_radial, rc_angular, n_max_radial, n_max_angular, basis_radial,
                 basis_angular, l_max, four_body, n_hidden, cr, ca, qs, heads, five_body=five_body)


# --------------------------------------------------------------------------
# The workloads (sizes, seeds) used by tests and the benchmark.

WATER_DESCRIPTOR = dict(rc_radial=6.0, rc_angular=4.0, n_max_radial=4, n_max_angular=4, basis_radial=8,
                        basis_angular=8, l_max=4, four_body=True, n_hidden=30)
WATER5_DESCRIPTOR = dict(WATER_DESCRIPTOR, five_body=True)
PEROVSKITE_DESCRIPTOR = dict(rc_radial=7.0, rc_angular=5.0, n_max_radial=6, n_max_angular=4, basis_radial=8,
                             basis_angular=8, l_max=4, four_body=False, n_hidden=50)

# name -> (seed, kind, species, descriptor)
def per_species_model(networks: List["Model"], species_network: List[int]) -> "Model":
    """A per-species-network model: the descriptor (coefficients, scaler) of
    networks[0], and for centre species t the heads of networks[species_network[t]]
    (all networks of one kind, descriptor shape and width)."""
    base = networks[species_network[0]]
    heads = []
    for h in range(len(base.heads)):
        src = [networks[species_network[t]].heads[h] for t in range(len(base.species))]
        heads.append(Head(np.stack([x.w0 for x in src]), np.stack([x.b0 for x in src]),
                          np.stack([x.w1 for x in src]), np.array([x.b1 for x in src], np.float64)))
    d = networks[0]
    return Model(d.kind, d.species, d.rc_radial, d.rc_angular, d.n_max_radial, d.n_max_angular, d.basis_radial,
                 d.basis_angular, d.l_max, d.four_body, d.n_hidden, d.c_radial, d.c_angular, d.q_scaler, heads,
                 True, d.five_body)


def with_descriptor_of(m: "Model", ref: "Model") -> "Model":
    """m's network heads on ref's descriptor coefficients and scaler."""
    return Model(m.kind, ref.species, ref.rc_radial, ref.rc_angular, ref.n_max_radial, ref.n_max_angular,
                 ref.basis_radial, ref.basis_angular, ref.l_max, ref.four_body, ref.n_hidden, ref.c_radial,
                 ref.c_angular, ref.q_scaler, m.heads, m.per_species, ref.five_body)


def pack_params(m: "Model") -> np.ndarray:
    """Trainable parameters of a shared-network model as one vector:
    c_radial, c_angular, then per head w0 [H, D], b0 [H], w1 [H], b1."""
    parts = [np.ravel(m.c_radial), np.ravel(m.c_angular)]
    for h in m.heads:
        parts += [np.ravel(h.w0), np.ravel(h.b0), np.ravel(h.w1), np.array([h.b1], np.float64)]
    return np.concatenate(parts).astype(np.float64)


def unpack_params(base: "Model", z) -> "Model":
    """The model with base's hyperparameters and descriptor scaler and the
    trainable parameters z (layout of pack_params)."""
    z = np.asarray(z, np.float64)
    o = 0

    def take(shape):
        nonlocal o
        n = int(np.prod(shape))
        out = z[o:o + n].reshape(shape)
        o += n
        return out

    cr = take(base.c_radial.shape)
    ca = take(base.c_angular.shape)
    heads = []
    for h in base.heads:
        heads.append(Head(take(h.w0.shape), take(h.b0.shape), take(h.w1.shape), float(take((1,))[0])))
    assert o == z.size, "parameter vector of the wrong length"
    return Model(base.kind, base.species, base.rc_radial, base.rc_angular, base.n_max_radial, base.n_max_angular,
                 base.basis_radial, base.basis_angular, base.l_max, base.four_body, base.n_hidden, cr, ca,
                 base.q_scaler, heads, five_body=base.five_body)


MODEL_SPECS = {
    "water_dipole_small": (100, KIND_DIPOLE, WATER_SPECIES, WATER_DESCRIPTOR),
    "water_dipole": (101, KIND_DIPOLE, WATER_SPECIES, WATER_DESCRIPTOR),
    "water_polarizability": (102, KIND_POLARIZABILITY, WATER_SPECIES, WATER_DESCRIPTOR),
    "perovskite_susceptibility": (103, KIND_POLARIZABILITY, PEROVSKITE_SPECIES, PEROVSKITE_DESCRIPTOR),
    "molecule_dipole": (104, KIND_DIPOLE, MOLECULE_SPECIES, WATER_DESCRIPTOR),
    "molecule_polarizability": (105, KIND_POLARIZABILITY, MOLECULE_SPECIES, WATER_DESCRIPTOR),
    "water_pes": (106, KIND_PES, WATER_SPECIES, WATER_DESCRIPTOR),
    "molecule_pes": (107, KIND_PES, MOLECULE_SPECIES, WATER_DESCRIPTOR),
    "water_dipole_5b": (108, KIND_DIPOLE, WATER_SPECIES, WATER5_DESCRIPTOR),
    "water_polarizability_5b": (109, KIND_POLARIZABILITY, WATER_SPECIES, WATER5_DESCRIPTOR),
    "water_pes_5b": (110, KIND_PES, WATER_SPECIES, WATER5_DESCRIPTOR),
}


def model_raw(name: str) -> Model:
    """The seeded model before descriptor scaling (q_scaler = 1)."""
    seed, kind, species, desc = MODEL_SPECS[name]
    return make_model(seed, kind, species, **desc)


def model(name: str) -> Model:
    """The seeded model with its stored descriptor scaler
    (tests/golden/model_scaling.json, written by the script beside it)."""
    m = model_raw(name)
    path = os.path.join(_GOLDEN, "model_scaling.json")
    with open(path) as fh:
        table = json.load(fh)
    m.q_scaler = np.array(table[name]["q_scaler"], np.float64)
    return m


# Frame workloads ---------------------------------------------------------

def water_small(n_frames: int = 10, seed: int = 0) -> Frames:
    """64 H2O (192 atoms), cubic periodic box 12.42 A, independent frames."""
    return water_frames(4, 12.42, n_frames, seed)


def water_large_reference(seed: int = 1):
    """4096 H2O (12,288 atoms), box 49.7 A: the trajectory's starting frame."""
    return water_box(16, 49.7, seed)


def water_trajectory(n_frames: int = 2000, seed: int = 1) -> Frames:
    """12,288-atom water box + OU displacement walk (sigma 0.02 A, tau 50)."""
    pos, spc, cell = water_large_reference(seed)
    return ou_trajectory(pos, spc, cell, n_frames, seed + 10)


def perovskite(n_frames: int = 64, seed: int = 2, n_rep: int = 12, sigma: float = 0.08) -> Frames:
    """BaZrO3-like 12x12x12 cubic supercell (8,640 atoms), a = 4.19 A."""
    return perovskite_frames(n_rep, 4.19, n_frames, seed, sigma)


def molecules(n_frames: int = 8192, seed: int = 3) -> Frames:
    """Ragged vacuum molecules of 20-80 atoms over C/H/N/O/F."""
    return molecule_frames(n_frames, seed)


# Spectrum inputs ------------------------------------------------------------

def sinusoid_series(n_steps: int, omega_per_step: float, amp: float = 1.0, offset=None, comps: int = 9,
                    seed: int = 7, noise: float = 0.0):
    """Tensor time series x(t) = offset + B cos(omega t) (+ noise), [n_steps, comps]."""
    rng = np.random.default_rng(seed)
    b = rng.normal(0.0, amp, comps)
    base = np.zeros(comps) if offset is None else np.asarray(offset, np.float64)
    t = np.arange(n_steps)
    x = base[None, :] + b[None, :] * np.cos(omega_per_step * t)[:, None]
    if noise:
        x = x + rng.normal(0.0, noise, x.shape)
    return x


def susceptibility_runs(n_runs: int = 20, n_steps: int = 100000, seed: int = 5, n_modes: int = 6,
                        dt_fs: float = 5.0) -> np.ndarray:
    """Stand-in for the recorded chi(t) of the perovskite runs (20 runs of
    500 ps at 5 fs): per run a symmetric tensor series = a static part, a sum
    of damped-random-phase modes (wavenumbers 50-800 cm^-1, random symmetric
    mode tensors) and white noise.  [n_runs, n_steps, 9]."""
    rng = np.random.default_rng(seed)
    c_cm_per_fs = 2.99792458e-5
    t = np.arange(n_steps) * dt_fs
    out = np.empty((n_runs, n_steps, 9))
    base = rng.normal(size=(3, 3))
    base = 0.5 * (base + base.T) + 5.0 * np.eye(3)
    for r in range(n_runs):
        x = np.broadcast_to(base, (n_steps, 3, 3)).copy()
        for _ in range(n_modes):
            nu = rng.uniform(50.0, 800.0)
            w = 2.0 * np.pi * nu * c_cm_per_fs
            phase = np.cumsum(rng.normal(0.0, 0.02, n_steps))  # slow phase diffusion: finite line width
            T = rng.normal(size=(3, 3))
            T = 0.5 * (T + T.T)
            x += (0.3 * np.cos(w * t + phase))[:, None, None] * T[None]
        x += rng.normal(0.0, 0.05, x.shape)
        out[r] = x.reshape(n_steps, 9)
    return out
