// Neighbour search for a batch of ragged frames on gfx950.
//
// The sums over j != i of the method (Sec. 2.1, Eq. virial; Sec. 2.2, Eq. mu;
// Sec. 2.3, Eq. polarizability-model) run over the atoms inside the radial
// cutoff, with the minimum-image convention.  On orthorhombic cell grids a
// pair vector is formed in FP32 from the two atoms' FP32 offsets within their
// cells and the cells' offset (a few 1e-7 A from the exact vector, about the
// FP32 rounding of the stored entry); triclinic bins use fixed-point
// fractional offsets and FP64, frames without a grid FP64 positions.  Entries
// are stored as FP32.
//
// Pipeline (all on the device):
//   1. bin every atom into a bucket (cell, species).  Fully periodic
//      orthorhombic frames use a cell grid of edge >= rc_radial / 2 (at least
//      5 cells per axis), triclinic ones
//      a grid of >= 3 bins of width >= rc_radial per axis; every other frame
//      (vacuum molecules, small boxes) is one cell;
//   2. scan the bucket counts twice: in (cell, species) order for the
//      scatter and in (species, cell) order for the atom tiles;
//   3. scatter atoms into buckets; each atom's place in its bucket is its rank
//      by atom index, which makes the whole result independent of thread
//      scheduling;
//   4. build the tile permutation: atoms ordered by (species, cell, index),
//      each species padded to whole 64-atom tiles (species-pure wavefronts),
//      and store the positions in the same (slot) order, so that the atoms of
//      one species in consecutive cells of a frame are one contiguous range;
//   5. one lane per tile slot walks the cells within reach (or its frame) once
//      per neighbour species t and writes the neighbours of species t into
//      that species' angular (r < rc_angular) and radial-only segments.
//      Orthorhombic grids are walked as 25 columns of cells along z, each
//      trimmed to the z-cells within reach of the atom: one contiguous range of
//      candidates per column (two where the column crosses the box face).
// Entries are grouped four to a lane (64 contiguous bytes), so every store and
// load of a wavefront covers one contiguous 4 KB block.
#include <algorithm>

#include "internal.h"
#include "radial_basis.h"

namespace tnep {

namespace {

constexpr int kBlock = 256;

// Set-up of a launch batch in one launch: work-group f < (frames) writes the
// frame index of frame f's atoms; thread i clears bucket count i and marks tile
// slot i as padding.
__global__ void k_batch_setup(const FrameInfo* __restrict__ frames, const int32_t* __restrict__ meta,
                              int32_t* __restrict__ frame_of, int32_t* __restrict__ bucket_count, int64_t n_buckets,
                              int32_t* __restrict__ perm, int64_t n_pad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_buckets) bucket_count[i] = 0;
    if (i < n_pad) perm[i] = -1;
    const int f = blockIdx.x;
    if (f >= meta[kMetaNFrames]) return;
    const FrameInfo fi = frames[f];
    for (int64_t a = threadIdx.x; a < fi.n_atoms; a += blockDim.x) frame_of[fi.atom_begin + a] = f;
}

// Index of batch atom a in the whole call (for error reports), saturated.
__device__ __forceinline__ int call_atom(const int32_t* meta, int64_t a) {
    const int64_t g = (int64_t)meta[kMetaAtomBase] + a;
    return g > INT32_MAX ? INT32_MAX : (int)g;
}

__device__ __forceinline__ int cell_coord(double p, double L, int nc) {
    const double s = p - L * floor(p / L);
    const int c = (int)(s * (double)nc / L);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// key = (frame cell) * T + species; invalid atoms get key -1.  An atom of a
// follower frame is binned where its reference atom is (the reference frame's
// position), so the follower frame's slots mirror the reference frame's: the
// same rank within each species range (CandLists).
__device__ __forceinline__ int bin_key(const FrameInfo& fi, const FrameTric* __restrict__ tric, int f, int64_t a,
                                       const double* __restrict__ pos, const int32_t* __restrict__ species,
                                       const int32_t* __restrict__ meta, int T, int32_t* __restrict__ flags) {
    const double x = pos[3 * a], y = pos[3 * a + 1], z = pos[3 * a + 2];
    const int t = species[a];
    int err = 0;
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) err |= kErrNonFinite;
    if (t < 0 || t >= T) err |= kErrSpecies;
    if (err) {
        atomicOr(&flags[kFlagError], err);
        atomicMin(&flags[kFlagBadAtom], call_atom(meta, a));
        return -1;
    }
    int c = fi.cell_base;
    if (fi.mode == 1 && fi.tric) {
        // triclinic: bins of the wrapped fractional coordinates s = r Hinv
        int b[3];
        for (int k = 0; k < 3; ++k) {
            double sk = x * tric[f].Hinv[k] + y * tric[f].Hinv[3 + k] + z * tric[f].Hinv[6 + k];
            sk -= floor(sk);
            const int q = (int)(sk * (double)fi.nc[k]);
            b[k] = q < 0 ? 0 : (q >= fi.nc[k] ? fi.nc[k] - 1 : q);
        }
        c += (b[0] * fi.nc[1] + b[1]) * fi.nc[2] + b[2];
    } else if (fi.mode == 1) {
        double bx = x, by = y, bz = z;
        if (fi.role == kRoleFollower) {
            const int64_t ar = fi.ref_begin + (a - fi.atom_begin);
            bx = pos[3 * ar];
            by = pos[3 * ar + 1];
            bz = pos[3 * ar + 2];
        }
        const int ix = cell_coord(bx, fi.L[0], fi.nc[0]);
        const int iy = cell_coord(by, fi.L[1], fi.nc[1]);
        const int iz = cell_coord(bz, fi.L[2], fi.nc[2]);
        c += (ix * fi.nc[1] + iy) * fi.nc[2] + iz;
    }
    return c * T + t;
}

__global__ void k_bin(const FrameInfo* __restrict__ frames, const FrameTric* __restrict__ tric,
                      const int32_t* __restrict__ frame_of,
                      const double* __restrict__ pos, const int32_t* __restrict__ species,
                      const int32_t* __restrict__ meta, int T, int32_t* __restrict__ key_of,
                      int32_t* __restrict__ bucket_count, int32_t* __restrict__ flags) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= meta[kMetaNAtoms]) return;
    const int f = frame_of[a];
    const int key = bin_key(frames[f], tric, f, a, pos, species, meta, T, flags);
    key_of[a] = key;
    if (key >= 0) atomicAdd(&bucket_count[key], 1);
}

// Bucket scans in three phases over chunks of kScanCells cells (all T species
// of a cell are adjacent in key order):
//   phase 1: per chunk, the total count and the per-species totals;
//   phase 2 (one work-group): chunk offsets in key order and, per species, in
//            (species, cell) order; species totals give the tile bases;
//   phase 3: per chunk, bucket_start (key order) and perm_start (first tile
//            slot of the bucket in (species, cell) order).
constexpr int kScanCells = 1024;  // cells per chunk; 256 threads x 4 cells

template <int NT>
__device__ int32_t block_exclusive(int32_t v, int32_t* part) {
    const int tid = threadIdx.x;
    part[tid] = v;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        const int32_t u = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += u;
        __syncthreads();
    }
    const int32_t incl = part[tid];
    __syncthreads();
    return incl - v;
}
__device__ int32_t block_exclusive_256(int32_t v, int32_t* part) { return block_exclusive<256>(v, part); }

__global__ void __launch_bounds__(256) k_scan_partials(const int32_t* __restrict__ count,
                                                       const int32_t* __restrict__ meta, int T,
                                                       int32_t* __restrict__ chunk_sums) {
    __shared__ int32_t red[256];
    const int n_cells = meta[kMetaNCells];
    if ((int)blockIdx.x * kScanCells >= n_cells) return;
    const int c0 = blockIdx.x * kScanCells + threadIdx.x * 4;
    for (int t = 0; t <= T; ++t) {
        int32_t s = 0;
        for (int c = c0; c < min(c0 + 4, n_cells); ++c) {
            if (t < T)
                s += count[c * T + t];
            else
                for (int u = 0; u < T; ++u) s += count[c * T + u];
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) chunk_sums[blockIdx.x * 9 + t] = red[0];
        __syncthreads();
    }
}

// chunk_sums[k*9 + t] (t < T: species t, t = T: all) -> chunk_off[k*9 + t]:
// species t: slot offset in (species, cell) order incl. tile padding; T: key order.
__global__ void __launch_bounds__(256) k_scan_chunks(const int32_t* __restrict__ chunk_sums, int T,
                                                     int32_t* __restrict__ chunk_off, int32_t* __restrict__ meta,
                                                     int32_t* __restrict__ bucket_start) {
    __shared__ int32_t part[256];
    const int n_cells = meta[kMetaNCells];
    const int n_chunks = (n_cells + kScanCells - 1) / kScanCells;
    const int n_buckets = n_cells * T;
    int32_t* bucket_start_end = bucket_start;
    __shared__ int32_t s_carry;
    int32_t tiles = 0;
    for (int t = 0; t <= T; ++t) {
        if (threadIdx.x == 0) s_carry = 0;
        __syncthreads();
        for (int base = 0; base < n_chunks; base += 256) {
            const int k = base + threadIdx.x;
            const int32_t v = k < n_chunks ? chunk_sums[k * 9 + t] : 0;
            const int32_t ex = block_exclusive_256(v, part);
            const int32_t carry = s_carry;
            if (k < n_chunks) chunk_off[k * 9 + t] = carry + ex + (t < T ? tiles * 64 : 0);
            __syncthreads();
            if (threadIdx.x == 255) s_carry = carry + ex + v;
            __syncthreads();
        }
        const int32_t total = s_carry;
        if (t < T) {
            if (threadIdx.x == 0) meta[kMetaTileBase + t] = tiles;
            tiles += (total + 63) / 64;
        } else if (threadIdx.x == 0) {
            bucket_start_end[n_buckets] = total;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) meta[kMetaTileBase + T] = tiles;
}

__global__ void __launch_bounds__(256) k_scan_final(const int32_t* __restrict__ count,
                                                    const int32_t* __restrict__ meta, int T,
                                                    const int32_t* __restrict__ chunk_off,
                                                    int32_t* __restrict__ bucket_start,
                                                    int32_t* __restrict__ bucket_fill,
                                                    int32_t* __restrict__ perm_start) {
    __shared__ int32_t part[256];
    const int n_cells = meta[kMetaNCells];
    const int k = blockIdx.x;
    if (k * kScanCells >= n_cells) return;
    const int c0 = k * kScanCells + threadIdx.x * 4;
    const int c1 = min(c0 + 4, n_cells);
    // key order (cell-major, species-minor)
    {
        int32_t s = 0;
        for (int c = c0; c < c1; ++c)
            for (int u = 0; u < T; ++u) s += count[c * T + u];
        int32_t run = block_exclusive_256(s, part) + chunk_off[k * 9 + T];
        for (int c = c0; c < c1; ++c)
            for (int u = 0; u < T; ++u) {
                bucket_start[c * T + u] = run;
                bucket_fill[c * T + u] = 0;
                run += count[c * T + u];
            }
    }
    // species-major order; perm_start[n_cells * T + t] closes species t, so
    // perm_start[(c + 1) * T + t] always ends the bucket (c, t)
    for (int t = 0; t < T; ++t) {
        int32_t s = 0;
        for (int c = c0; c < c1; ++c) s += count[c * T + t];
        int32_t run = block_exclusive_256(s, part) + chunk_off[k * 9 + t];
        for (int c = c0; c < c1; ++c) {
            perm_start[c * T + t] = run;
            run += count[c * T + t];
        }
        if (c0 < c1 && c1 == n_cells) perm_start[n_cells * T + t] = run;
    }
}

// Exclusive prefix sums of M values per thread over the NT threads of a
// work-group, all M at once: a shuffle scan within each wavefront, then the
// wavefronts' totals through LDS (wave_tot: NT / 64 x M ints), two barriers.
// total[m]: the sum over all threads.
template <int NT, int M>
__device__ __forceinline__ void block_exclusive_multi(int32_t (&v)[M], int32_t (&total)[M], int32_t* wave_tot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t x[M];
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] = v[m];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1)
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int32_t u = __shfl_up(x[m], off, 64);
            if (lane >= off) x[m] += u;
        }
    if (lane == 63)
#pragma unroll
        for (int m = 0; m < M; ++m) wave_tot[wave * M + m] = x[m];
    __syncthreads();
    int32_t before[M] = {}, all[M] = {};
#pragma unroll 1
    for (int w = 0; w < NT / 64; ++w)
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int32_t y = wave_tot[w * M + m];
            before[m] += w < wave ? y : 0;
            all[m] += y;
        }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        v[m] = before[m] + x[m] - v[m];
        total[m] = all[m];
    }
    __syncthreads();
}

constexpr int kScanMaxSpecies = 8;

// All three scan phases in one work-group of NT threads, for batches of at
// most kScanCells cells (one chunk): the same offsets as k_scan_partials,
// k_scan_chunks and k_scan_final give for a single chunk.  One scan of T + 1
// sums per thread: its cells' buckets in key order and, per species, in
// (species, cell) order; species t's tiles follow those of species < t, each
// species padded to whole 64-slot tiles.  bucket_fill (if given) is cleared for
// k_scatter.  wave_tot: NT / 64 x (kScanMaxSpecies + 1) ints of LDS.
template <int NT>
__device__ void scan_one_chunk(const int32_t* count, int32_t* __restrict__ meta, int T,
                               int32_t* __restrict__ bucket_start, int32_t* __restrict__ bucket_fill,
                               int32_t* __restrict__ perm_start, int32_t* wave_tot) {
    constexpr int kPer = kScanCells / NT;  // cells per thread
    constexpr int M = kScanMaxSpecies + 1;
    const int n_cells = meta[kMetaNCells];
    const int c0 = threadIdx.x * kPer;
    const int c1 = min(c0 + kPer, n_cells);
    int32_t v[M] = {}, tot[M];
    for (int c = c0; c < c1; ++c)
#pragma unroll
        for (int u = 0; u < kScanMaxSpecies; ++u) {
            const int32_t k = u < T ? count[c * T + u] : 0;
            v[0] += k;
            v[1 + u] += k;
        }
    block_exclusive_multi<NT, M>(v, tot, wave_tot);
    // key order (cell-major, species-minor)
    int32_t run = v[0];
    for (int c = c0; c < c1; ++c)
        for (int u = 0; u < T; ++u) {
            bucket_start[c * T + u] = run;
            if (bucket_fill) bucket_fill[c * T + u] = 0;
            run += count[c * T + u];
        }
    // species-major order
    int32_t tiles = 0;
#pragma unroll
    for (int t = 0; t < kScanMaxSpecies; ++t) {
        if (t < T) {
            int32_t r = v[1 + t] + tiles * 64;
            for (int c = c0; c < c1; ++c) {
                perm_start[c * T + t] = r;
                r += count[c * T + t];
            }
            if (threadIdx.x == 0) {
                perm_start[n_cells * T + t] = tot[1 + t] + tiles * 64;
                meta[kMetaTileBase + t] = tiles;
            }
            tiles += (tot[1 + t] + 63) / 64;
        }
    }
    if (threadIdx.x == 0) {
        bucket_start[n_cells * T] = tot[0];
        meta[kMetaTileBase + T] = tiles;
    }
}

__global__ void __launch_bounds__(256) k_scan_one(const int32_t* __restrict__ count, int32_t* __restrict__ meta,
                                                  int T, int32_t* __restrict__ bucket_start,
                                                  int32_t* __restrict__ bucket_fill, int32_t* __restrict__ perm_start) {
    __shared__ int32_t wave_tot[256 / 64 * (kScanMaxSpecies + 1)];
    scan_one_chunk<256>(count, meta, T, bucket_start, bucket_fill, perm_start, wave_tot);
}

__global__ void k_scatter(const int32_t* __restrict__ key_of, const int32_t* __restrict__ bucket_start,
                          int32_t* __restrict__ bucket_fill, int32_t* __restrict__ bucket_atoms,
                          const int32_t* __restrict__ meta) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= meta[kMetaNAtoms]) return;
    const int k = key_of[a];
    if (k < 0) return;
    const int slot = atomicAdd(&bucket_fill[k], 1);
    bucket_atoms[bucket_start[k] + slot] = (int32_t)a;
}

// Place every atom into the tile permutation at (first slot of its bucket) +
// (number of smaller atom indices in its bucket) and store its position at
// that slot.  One thread per atom: buckets hold a few atoms on cell grids and
// a whole frame otherwise, so the rank loop is never longer than the frame's
// own neighbour loop.  Cell grids get a 16-byte record: the offsets of the
// wrapped position from its cell's centre (orthorhombic grids: FP32, in A) or
// origin (triclinic bins: fractional, as integers in units of q_unit, a power
// of two so the scaling is exact), and the cell's index along the third axis
// (z, or the third lattice vector).  Frames without a grid keep the FP64 position
// (triclinic ones: wrapped fractional coordinates).
// Atom a (bucket k >= 0, frame f) of k_sort_place at tile slot `slot` (the
// first slot of its bucket plus the number of smaller atom indices in it).
__device__ __forceinline__ void place_atom(int64_t a, int k, int f, int slot, const FrameInfo* __restrict__ frames,
                                           const FrameTric* __restrict__ tric, int32_t* __restrict__ perm,
                                           int32_t* __restrict__ slot_of, const double* __restrict__ pos,
                                           double4* __restrict__ bucket_pos, int4* __restrict__ cell_rec, int T) {
    perm[slot] = (int32_t)a;
    slot_of[a] = slot;
    double x = pos[3 * a], y = pos[3 * a + 1], z = pos[3 * a + 2];
    const FrameInfo& fi = frames[f];
    if (fi.mode == 1) {
        const int local = k / T - fi.cell_base;
        const int ny = fi.nc[1], nz = fi.nc[2];
        const int c[3] = {local / (nz * ny), (local / nz) % ny, local % nz};
        const double r[3] = {x, y, z};
        int q[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double s, h;
            if (fi.tric) {
                // wrapped fractional coordinate, as k_bin bins it
                s = x * tric[f].Hinv[d] + y * tric[f].Hinv[3 + d] + z * tric[f].Hinv[6 + d];
                s -= floor(s);
                h = 1.0 / fi.nc[d];
            } else {
                s = r[d] - fi.L[d] * floor(r[d] * fi.Linv[d]);
                h = fi.L[d] / fi.nc[d];
            }
            // triclinic: fixed point in units of q_unit from the bin origin;
            // orthorhombic: FP32 offset (A) from the cell centre, the minimum image
            // (|offset| <= h / 2 for an atom in its own cell; a follower frame's atom
            // is in its reference atom's cell, at most skin / 2 beyond it)
            double o = s - (c[d] + 0.5) * h;
            if (!fi.tric) o -= fi.L[d] * rint(o * fi.Linv[d]);
            q[d] = fi.tric ? (int)rint((s - c[d] * h) / fi.q_unit) : __float_as_int((float)o);
        }
        cell_rec[slot] = make_int4(q[0], q[1], q[2], c[2]);
        return;
    }
    if (fi.tric) {
        // triclinic frames: the wrapped fractional coordinates (as k_bin bins them)
        double sf[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            sf[q] = x * tric[f].Hinv[q] + y * tric[f].Hinv[3 + q] + z * tric[f].Hinv[6 + q];
            sf[q] -= floor(sf[q]);
        }
        x = sf[0];
        y = sf[1];
        z = sf[2];
    }
    bucket_pos[slot] = make_double4(x, y, z, 0.0);
}

__global__ void k_sort_place(const FrameInfo* __restrict__ frames, const FrameTric* __restrict__ tric,
                             const int32_t* __restrict__ frame_of,
                             const int32_t* __restrict__ key_of, const int32_t* __restrict__ bucket_start,
                             const int32_t* __restrict__ bucket_atoms, const int32_t* __restrict__ perm_start,
                             int32_t* __restrict__ perm, int32_t* __restrict__ slot_of, const double* __restrict__ pos,
                             double4* __restrict__ bucket_pos, int4* __restrict__ cell_rec,
                             const int32_t* __restrict__ meta, int T) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= meta[kMetaNAtoms]) return;
    const int k = key_of[a];
    if (k < 0) return;
    const int b = bucket_start[k], n = bucket_start[k + 1] - b;
    int rank = 0;
    for (int i = 0; i < n; ++i) rank += bucket_atoms[b + i] < (int32_t)a ? 1 : 0;
    place_atom(a, k, frame_of[a], perm_start[k] + rank, frames, tric, perm, slot_of, pos, bucket_pos, cell_rec, T);
}

// The bucket pipeline of a small launch batch in one work-group: set-up,
// binning, the one-chunk scan, scatter and placement as k_batch_setup, k_bin,
// k_scan_one, k_scatter and k_sort_place do them (the same key, scan and
// placement functions), with the bucket counts and members in LDS and barriers
// in place of four launch boundaries.  The outputs are the same integers, so
// every later kernel sees the same slots.  For batches of at most
// kBucketSmallAtoms atoms and kScanCells cells, hence at most kScanCells frames
// (a frame has at least one cell) and kScanCells x 8 buckets (at most 8 species).
constexpr int kBucketSmallBlock = 1024;
constexpr int kBucketSmallAtoms = 4096;
constexpr int kBucketSmallBuckets = kScanCells * kScanMaxSpecies;
__global__ void __launch_bounds__(kBucketSmallBlock) k_bucket_small(const FrameInfo* __restrict__ frames,
                                                                    const FrameTric* __restrict__ tric,
                                                                    const double* __restrict__ pos,
                                                                    const int32_t* __restrict__ species, int T,
                                                                    NeighborWork w, int64_t n_pad,
                                                                    int32_t* __restrict__ flags) {
    __shared__ int32_t s_begin[kScanCells];            // first atom of every frame
    __shared__ int32_t s_count[kBucketSmallBuckets];   // bucket counts, then fill levels
    __shared__ int32_t s_atoms[kBucketSmallAtoms];     // bucket members (bucket_atoms)
    __shared__ int32_t s_wave[kBucketSmallBlock / 64 * (kScanMaxSpecies + 1)];
    const int n_atoms = w.meta[kMetaNAtoms], n_frames = w.meta[kMetaNFrames];
    const int n_buckets = w.meta[kMetaNCells] * T;
    for (int i = threadIdx.x; i < n_buckets; i += kBucketSmallBlock) s_count[i] = 0;
    for (int64_t i = threadIdx.x; i < n_pad; i += kBucketSmallBlock) w.perm[i] = -1;
    for (int f = threadIdx.x; f < n_frames; f += kBucketSmallBlock) s_begin[f] = (int)frames[f].atom_begin;
    __syncthreads();
    // frames are consecutive atom ranges (an empty frame begins where the next
    // one does): atom a is in the last frame that begins at or before it
    for (int a = threadIdx.x; a < n_atoms; a += kBucketSmallBlock) {
        int lo = 0, hi = n_frames - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_begin[mid] <= a)
                lo = mid;
            else
                hi = mid - 1;
        }
        w.frame_of[a] = lo;
        const int key = bin_key(frames[lo], tric, lo, a, pos, species, w.meta, T, flags);
        w.key_of[a] = key;
        if (key >= 0) atomicAdd(&s_count[key], 1);
    }
    __syncthreads();
    scan_one_chunk<kBucketSmallBlock>(s_count, w.meta, T, w.bucket_start, nullptr, w.perm_start, s_wave);
    __syncthreads();  // every thread's reads of the counts are done
    for (int i = threadIdx.x; i < n_buckets; i += kBucketSmallBlock) s_count[i] = 0;
    __syncthreads();
    for (int a = threadIdx.x; a < n_atoms; a += kBucketSmallBlock) {
        const int k = w.key_of[a];
        if (k >= 0) s_atoms[w.bucket_start[k] + atomicAdd(&s_count[k], 1)] = a;
    }
    __syncthreads();
    for (int a = threadIdx.x; a < n_atoms; a += kBucketSmallBlock) {
        const int k = w.key_of[a];
        if (k < 0) continue;
        const int b = w.bucket_start[k], n = w.bucket_start[k + 1] - b;
        int rank = 0;
#pragma unroll 8
        for (int i = 0; i < n; ++i) rank += s_atoms[b + i] < a ? 1 : 0;
        place_atom(a, k, w.frame_of[a], w.perm_start[k] + rank, frames, tric, w.perm, w.slot_of, pos, w.bucket_pos,
                   w.cell_rec, T);
    }
}

// Minimum image along one axis; Linv = 1/L on periodic axes, 0 otherwise.
__device__ __forceinline__ double min_image(double d, double L, double Linv) { return d - L * rint(d * Linv); }

// Distance along one axis from an atom to the cell o steps away (|o| <= 2),
// given its distances lo, hi to its own cell's faces and the cell edge h.
static_assert(kCellReachXY == 2, "the column walk visits the 5 x 5 columns within two cells");
__device__ __forceinline__ float cell_gap(int o, float lo, float hi, float h) {
    return o == 0 ? 0.f : (o < 0 ? lo + (o == -2 ? h : 0.f) : hi + (o == 2 ? h : 0.f));
}

__device__ __forceinline__ int wrap_cell(int u, int n) { return u < 0 ? u + n : (u >= n ? u - n : u); }

// The entries of one (atom, neighbour species) pass: angular segment (r <
// r_c^A) and radial-only segment.  Each lane stages four entries per segment
// in LDS; a completed 64-byte group is stored by the whole wave (coop_flush),
// the partial groups at the end by the lane (flush).  Staging in LDS instead
// of registers keeps a push to one store and one address, where a register
// buffer costs a shift of four entries per push and copies of both buffers at
// every divergent branch.  Slot (segment s, entry k) of a lane is
// stage[(4 s + k) * stride] (consecutive lanes at consecutive 16-byte words).
struct PairSink {
    float4* stage;
    int stride;
    float4* ga;
    float4* gr;
    int capA, capR;
    int na, nr;
    __device__ __forceinline__ void flush_one(int n, int cap, float4* base, const float4* src) {
        const int k = n & 3;
        if (k == 0 || n > cap) return;
        float4* g = base + (int64_t)((n - k) >> 2) * 256;
        for (int i = 0; i < k; ++i) g[i] = src[i * stride];
    }
    __device__ __forceinline__ void flush() {
        flush_one(na, capA, ga, stage);
        flush_one(nr, capR, gr, stage + 4 * stride);
    }

    // A completed group is not stored by its lane but left for the wave's
    // next coop_flush (pend_src = LDS index of its first entry relative to
    // lds, pend_dst = its destination).
    int pend_src;
    float4* pend_dst;
    __device__ __forceinline__ void push_deferred(const float4& e, bool ang, const float4* lds) {
        const int n = ang ? na : nr;
        const int s4 = ang ? 0 : 4;
        stage[(s4 + (n & 3)) * stride] = e;
        const int m = n + 1;
        if (ang)
            na = m;
        else
            nr = m;
        if ((m & 3) == 0 && m <= (ang ? capA : capR)) {
            pend_dst = (ang ? ga : gr) + (int64_t)((m - 4) >> 2) * 256;
            pend_src = (int)(stage + s4 * stride - lds);
        }
    }
};

__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Cooperative store of the groups that lanes completed since the last call
// (every active lane calls it): each completing lane posts (destination, LDS
// source) to the wave's list, then the active lanes store one 16-byte quarter
// of a group each, so a 64-byte group leaves as one coalesced request and one
// store instruction carries up to 16 groups (instead of four sparse store
// instructions per completing lane).  LDS accesses of one wave complete in
// order, so the list and the staged entries are read after they are written.
__device__ __forceinline__ void coop_flush(PairSink& ps, const float4* lds, int4* list) {
    const bool mine = ps.pend_src >= 0;
    const uint64_t pend = __ballot(mine);
    if (pend == 0) return;
    const uint64_t act = __ballot(1);
    if (mine) {
        const uint64_t d = (uint64_t)ps.pend_dst;
        list[lanes_below(pend)] = make_int4((int)(uint32_t)d, (int)(uint32_t)(d >> 32), ps.pend_src, 0);
        ps.pend_src = -1;
    }
    __builtin_amdgcn_wave_barrier();
    const int rank = lanes_below(act), n_act = __popcll(act), pieces = 4 * __popcll(pend);
    for (int pb = 0; pb < pieces; pb += n_act) {
        const int piece = pb + rank;
        if (piece < pieces) {
            const int4 L = list[piece >> 2];
            const int part = piece & 3;
            float4* dst = (float4*)(((uint64_t)(uint32_t)L.y << 32) | (uint32_t)L.x) + part;
            *dst = lds[L.z + part * ps.stride];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Radial descriptor sums of one (atom, neighbour species) pass: over the
// accepted pairs, sum f_c T_k(x) and sum f_c (Sec. 2.1, radial functions
// f_k = (T_k(x) + 1) / 2 f_c), from the FP32 pair vector that the entry
// stores.  They depend on the lists, r_c^R and the basis size only, so every
// model evaluated on the lists loads them instead of forming them again.
struct RadialSums {
    float FT[kRadialTerms];
    float Fs;
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int k = 0; k < kRadialTerms; ++k) FT[k] = 0.f;
        Fs = 0.f;
    }
    // The terms of one pair from its FP32 entry: sf with f_c = sf^2, and T_k(x).
    // Every step is an explicit product or fused multiply-add, so the sums come
    // out bit for bit the same in every kernel that forms them (the compiler
    // would otherwise fuse f_c = sf^2 into some of the additions and not others).
    static __device__ __forceinline__ void terms(float x, float y, float z, float rcR_inv, float& sf,
                                                 float (&Tk)[kRadialTerms]) {
        const float r = pair_sqrt(__builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x)));
        sf = sin_half_pi(1.57079632679489662f * __builtin_fmaf(-r, rcR_inv, 1.f));
        const float tt = __builtin_fmaf(r, rcR_inv, -1.f);
        const float xc = __builtin_fmaf(tt + tt, tt, -1.f);
        Tk[0] = 1.f;
        Tk[1] = xc;
#pragma unroll
        for (int k = 2; k < kRadialTerms; ++k) Tk[k] = __builtin_fmaf(xc + xc, Tk[k - 1], -Tk[k - 2]);
    }
    __device__ __forceinline__ void accumulate(float sf, const float (&Tk)[kRadialTerms]) {
        Fs = __builtin_fmaf(sf, sf, Fs);
        FT[0] = __builtin_fmaf(sf, sf, FT[0]);
        const float fc = sf * sf;
#pragma unroll
        for (int k = 1; k < kRadialTerms; ++k) FT[k] = __builtin_fmaf(fc, Tk[k], FT[k]);
    }
    __device__ __forceinline__ void add(float x, float y, float z, float rcR_inv) {
        float sf, Tk[kRadialTerms];
        terms(x, y, z, rcR_inv, sf, Tk);
        accumulate(sf, Tk);
    }
    // sum_j f_k(r_ij) for species t of slot p
    __device__ __forceinline__ void store(float* __restrict__ v, int t, int64_t n_pad, int64_t p) const {
        if (!v) return;
#pragma unroll
        for (int k = 0; k < kRadialTerms; ++k) v[(int64_t)(t * kRadialTerms + k) * n_pad + p] = 0.5f * (FT[k] + Fs);
    }
};

// One candidate of k_neighbors: pair vector d = r_j - r_i, in = a real
// candidate other than the atom itself within the search radius.  Reference
// frames also keep the candidate, packed (CandLists), in the lane's list.
template <bool REF, typename R>
__device__ __forceinline__ void take_candidate(PairSink& ps, RadialSums& rs, float rcR_inv, const float4* lds, bool in,
                                               R dx, R dy, R dz, R r2, int j, R rc2r, R rc2a, bool& overlap,
                                               int& n_cand, int32_t* cand, int cand_cap, int packed) {
    if (in) {
        if constexpr (REF) {
            if (n_cand < cand_cap) cand[(n_cand >> 2) * 256 + (n_cand & 3)] = packed;
            ++n_cand;
        }
        if (!REF || r2 < rc2r) {
            overlap |= r2 < (R)1e-8;
            const float4 e = make_float4((float)dx, (float)dy, (float)dz, __int_as_float(j));
            ps.push_deferred(e, r2 < rc2a, lds);
            rs.add(e.x, e.y, e.z, rcR_inv);
        }
    }
}

// Candidates per iteration of the cell-grid walk (their record loads are
// issued together): four for plain searches, two for reference frames, whose
// candidate-list bookkeeping leaves no registers for four.
template <bool REF>
constexpr int cand_per_iter() { return REF ? 2 : 4; }

// Four waves per SIMD (<= 128 VGPRs): the candidate loop is bound by load
// latency, so occupancy matters more than anything the registers could buy.
// REF = false: plain frames and padding slots; REF = true: reference frames,
// which also keep their candidates out to r_c + skin.
template <bool REF>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_neighbors(const FrameInfo* __restrict__ frames,
                                                      const int32_t* __restrict__ frame_of,
                                                      const double* __restrict__ pos,
                                                      const int32_t* __restrict__ species,
                                                      const int32_t* __restrict__ slot_of,
                                                      const int32_t* __restrict__ key_of,
                                                      const int32_t* __restrict__ perm_start,
                                                      const double4* __restrict__ bucket_pos,
                                                      const int4* __restrict__ cell_rec, float rc_radial,
                                                      float rc_angular, NeighborLists nl, CandLists cl,
                                                      int32_t* __restrict__ flags, float* __restrict__ rad_v,
                                                      bool pair_search) {
    // 8 staged entries per lane (PairSink), then a 64-entry list per wave (coop_flush)
    extern __shared__ float4 nb_stage[];
    float4* stage = nb_stage + threadIdx.x;
    int4* list = reinterpret_cast<int4*>(nb_stage + 8 * blockDim.x) + (threadIdx.x & ~63u);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nl.n_pad) return;
    const int T = nl.T;
    const int a = nl.perm[p];
    const int tile = (int)(p >> 6), lane = (int)(p & 63);
    if (a < 0) {
        if (REF) return;
        RadialSums none;
        none.clear();
        for (int t = 0; t < T; ++t) {
            nl.counts[(int64_t)(2 * t) * nl.n_pad + p] = 0;
            nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p] = 0;
            none.store(rad_v, t, nl.n_pad, p);
        }
        return;
    }
    const FrameInfo fi = frames[frame_of[a]];  // by value: kept in registers across the stores below
    // followers: k_neighbors_follow, after the reference lists are complete;
    // triclinic frames: k_neighbors_tri; with pair_search, frames without a
    // cell grid: k_neighbors_pp
    if (fi.role != (REF ? kRoleReference : kRolePlain) || fi.tric || (pair_search && fi.mode == 0)) return;
    const double xi = pos[3 * a], yi = pos[3 * a + 1], zi = pos[3 * a + 2];
    const double rc2r = (double)rc_radial * rc_radial, rc2a = (double)rc_angular * rc_angular;
    const float rcR_inv = 1.f / rc_radial;
    // references collect candidates out to r_c + skin
    const float rs = REF ? cl.rc_search : rc_radial;
    const float rc2rf = rc_radial * rc_radial, rc2af = rc_angular * rc_angular, rcs2f = rs * rs;
    // cell pruning in FP32 with a 1e-3 A margin: a cell is skipped only when surely beyond the radius
    const float prune2 = (rs + 1e-3f) * (rs + 1e-3f);
    // entry (row r) of this lane: lane_base + (r / 4) * 256 + r % 4
    float4* lane_base = nl.entries + ((int64_t)tile * (nl.slots >> 2) * 64 + lane) * 4;
    int ix = 0, iy = 0, iz = 0;
    const int nx = fi.nc[0], ny = fi.nc[1], nz = fi.nc[2];
    // distances from the atom to the lower / upper faces of its cell (cell list)
    float lo_x = 0, hi_x = 0, lo_y = 0, hi_y = 0, lo_z = 0, hi_z = 0;
    float hxf = 0, hyf = 0, hz_inv = 0;
    double hx = 0, hy = 0, hz = 0;
    int4 own = make_int4(0, 0, 0, 0);  // the atom's own cell record
    if (fi.mode == 1) {
        own = cell_rec[p];
        const int local = key_of[a] / T - fi.cell_base;
        iz = local % nz;
        iy = (local / nz) % ny;
        ix = local / (nz * ny);
        hx = fi.L[0] / nx;
        hy = fi.L[1] / ny;
        hz = fi.L[2] / nz;
        const double wx = xi - fi.L[0] * floor(xi * fi.Linv[0]);
        const double wy = yi - fi.L[1] * floor(yi * fi.Linv[1]);
        const double wz = zi - fi.L[2] * floor(zi * fi.Linv[2]);
        lo_x = (float)fmax(wx - ix * hx, 0.0);
        hi_x = (float)fmax((ix + 1) * hx - wx, 0.0);
        lo_y = (float)fmax(wy - iy * hy, 0.0);
        hi_y = (float)fmax((iy + 1) * hy - wy, 0.0);
        lo_z = (float)fmax(wz - iz * hz, 0.0);
        hi_z = (float)fmax((iz + 1) * hz - wz, 0.0);
        hxf = (float)hx;
        hyf = (float)hy;
        hz_inv = (float)(1.0 / hz);
    }
    bool overlap = false;
    // reference frames: the atom's candidate-list index (CandLists)
    int64_t R = 0;
    if constexpr (REF) {
        const int ti = species[a];
        R = fi.cl_base + (int64_t)ti * ((fi.n_atoms + 63) & ~63) + ((int)p - perm_start[fi.cell_base * T + ti]);
    }
    for (int t = 0; t < T; ++t) {
        PairSink ps{stage, (int)blockDim.x,
                    lane_base + (int64_t)(nl.meta[kMetaSegA + t] >> 2) * 256,
                    lane_base + (int64_t)(nl.meta[kMetaSegR + t] >> 2) * 256,
                    nl.meta[kMetaCapA + t], nl.meta[kMetaCapR + t], 0, 0, -1, nullptr};
        RadialSums rsum;
        rsum.clear();
        int n_cand = 0;
        int32_t* cand = nullptr;
        int base_t = 0;  // first slot of the frame's species-t atoms
        if constexpr (REF) {
            cand = cl.idx + (((R >> 6) * T + t) * (cl.cap >> 2)) * 256 + (R & 63) * 4;
            base_t = perm_start[fi.cell_base * T + t];
        }
        // cell grids: every candidate within rs is at most kCellReachXY cells
        // away along x, y and kCellReachZ along z; visited as 25 z-columns
        const int n_col = fi.mode == 1 ? 25 : 1;
        for (int col = 0; col < n_col; ++col) {
            // slot ranges [b0, e0) and [b1, e1) of species t
            int b0, e0, b1 = 0, e1 = 0;
            int ox = 0, oy = 0, z0 = 0, z1 = 0;
            if (fi.mode == 1) {
                ox = col / 5 - 2;
                oy = col % 5 - 2;
                // skip columns whose nearest point is beyond the search radius
                const float gx = cell_gap(ox, lo_x, hi_x, hxf), gy = cell_gap(oy, lo_y, hi_y, hyf);
                const float gxy = gx * gx + gy * gy;
                if (gxy >= prune2) continue;
                // the z-cells of the column within reach, iz - below .. iz + above:
                // cell iz - k is in reach when lo_z + (k - 1) hz < dz = sqrt(prune2 - gxy)
                const float dz_left = __builtin_amdgcn_sqrtf(prune2 - gxy);
                const int below = min(kCellReachZ, max(0, (int)floorf((dz_left - lo_z) * hz_inv) + 1));
                const int above = min(kCellReachZ, max(0, (int)floorf((dz_left - hi_z) * hz_inv) + 1));
                z0 = iz - below;
                z1 = iz + above;
                const int col0 = (fi.cell_base + (wrap_cell(ix + ox, nx) * ny + wrap_cell(iy + oy, ny)) * nz) * T + t;
                if (z0 >= 0 && z1 < nz) {
                    b0 = perm_start[col0 + z0 * T];
                    e0 = perm_start[col0 + (z1 + 1) * T];
                } else {
                    // across the box face in z (nz >= 2 kCellReachZ + 1 keeps the two parts apart)
                    b0 = perm_start[col0 + (z0 < 0 ? z0 + nz : z0) * T];
                    e0 = perm_start[col0 + nz * T];
                    b1 = perm_start[col0];
                    e1 = perm_start[col0 + ((z1 >= nz ? z1 - nz : z1) + 1) * T];
                }
            } else {
                b0 = perm_start[fi.cell_base * T + t];
                e0 = perm_start[(fi.cell_base + 1) * T + t];
            }
            // one loop over both ranges (candidate q is slot b0 + q for q < n0,
            // else b1 + q - n0), so a wavefront runs as long as its longest lane
            const int n0 = e0 - b0, n = n0 + (e1 - b1), d1 = b1 - n0;
            if (fi.mode == 1) {
                // pair vector from the cell records (FP32 offsets from the cell centres):
                // (q_j + column offset - q_i) in x and y, (q_j - q_i) + oz h_z in z
                auto slot_at = [&](int q) { return q < n0 ? b0 + q : d1 + q; };
                const float bxf = (float)(ox * hx - (double)__int_as_float(own.x));
                const float byf = (float)(oy * hy - (double)__int_as_float(own.y));
                const float ozf = __int_as_float(own.z), hzf = (float)hz;
                // z-cell offset = record's z index + shift of the column part (below / above the box face)
                const int zadd0 = (z0 < 0 ? -nz : 0) - iz, zadd1 = (z1 >= nz ? nz : 0) - iz;
                constexpr int kCand = cand_per_iter<REF>();
                for (int q = 0; q < n; q += kCand) {
                    // candidates past the end re-read the last one (never taken: q + u >= n)
                    int4 cur[kCand];
#pragma unroll
                    for (int u = 0; u < kCand; ++u) cur[u] = cell_rec[slot_at(min(q + u, n - 1))];
                    // all loads issued before the first use (else the compiler waits on
                    // the first two before it issues the others)
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < kCand; ++u) {
                        const int4 cr = cur[u];
                        const int j = slot_at(q + u);  // tile slot of the candidate
                        const int oz = cr.w + (q + u < n0 ? zadd0 : zadd1);
                        const float dx = __int_as_float(cr.x) + bxf;
                        const float dy = __int_as_float(cr.y) + byf;
                        const float dz = fmaf((float)oz, hzf, __int_as_float(cr.z) - ozf);
                        const float r2 = dx * dx + dy * dy + dz * dz;
                        const int packed = REF ? (int)(((unsigned)(j - base_t) << 9) | (unsigned)((ox + 3) << 6) |
                                                       (unsigned)((oy + 3) << 3) | (unsigned)(oz + 3))
                                               : 0;
                        take_candidate<REF, float>(ps, rsum, rcR_inv, nb_stage, (q + u < n) & (j != (int)p) & (r2 < rcs2f),
                                                   dx, dy, dz, r2, j, rc2rf, rc2af, overlap, n_cand, cand, cl.cap,
                                                   packed);
                        coop_flush(ps, nb_stage, list);
                    }
                }
            } else {
                // one cell per frame: FP64 positions and the rounding minimum image
                for (int q = 0; q < n; q += 2) {
                    const int k0 = b0 + q, k1 = b0 + q + 1;
                    const double4 q0 = bucket_pos[k0];
                    const double4 q1 = q + 1 < n ? bucket_pos[k1] : make_double4(0.0, 0.0, 0.0, 0.0);
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const double4 cur = u == 0 ? q0 : q1;
                        const int j = u == 0 ? k0 : k1;
                        const double dx = min_image(cur.x - xi, fi.L[0], fi.Linv[0]);
                        const double dy = min_image(cur.y - yi, fi.L[1], fi.Linv[1]);
                        const double dz = min_image(cur.z - zi, fi.L[2], fi.Linv[2]);
                        const double r2 = dx * dx + dy * dy + dz * dz;
                        // (reference frames always have a cell grid: no candidates kept here)
                        take_candidate<false, double>(ps, rsum, rcR_inv, nb_stage, (q + u < n) & (j != (int)p) & (r2 < rc2r),
                                                      dx, dy, dz, r2, j, rc2r, rc2a, overlap, n_cand, cand, cl.cap, 0);
                        coop_flush(ps, nb_stage, list);
                    }
                }
            }
        }
        if constexpr (REF) {
            cl.count[((R >> 6) * T + t) * 64 + (R & 63)] = n_cand;
            if (n_cand > cl.cap) atomicMax(&flags[kFlagCapCand], n_cand);
        }
        rsum.store(rad_v, t, nl.n_pad, p);
        ps.flush();
        nl.counts[(int64_t)(2 * t) * nl.n_pad + p] = min(ps.na, ps.capA);
        nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p] = min(ps.nr, ps.capR);
        if (ps.na > ps.capA) atomicMax(&flags[kFlagCapAng + t], ps.na);
        if (ps.nr > ps.capR) atomicMax(&flags[kFlagCapRad + t], ps.nr);
    }
    if (overlap) {
        atomicOr(&flags[kFlagError], kErrOverlap);
        atomicMin(&flags[kFlagBadAtom], call_atom(nl.meta, a));
    }
}

// Frames without a cell grid (vacuum frames and boxes narrower than 2.5 r_c,
// where every atom of the frame is a candidate, with the rounding minimum
// image), for the pair-parallel evaluation layout: kPairLanes lanes per atom,
// lane g testing the candidates g, g + G, ... of each species range, two per
// iteration.  Accepted pairs keep the candidates' order: a pair's row is the
// number of pairs accepted before it, counted over the group's lanes with a
// ballot, and each lane stores its rows itself.  These are the rows k_neighbors
// writes for such frames, in the same order.  RAD = true forms the radial
// descriptor sums as k_neighbors forms them, bit for bit: every lane computes
// its accepted candidates' terms and puts them in LDS, then lane k of the group
// adds term k of the accepted candidates in candidate order (the same fused
// multiply-adds), so a call's results do not depend on which of the two
// searches ran; RAD = false (the pair-parallel evaluation layout, which forms
// them itself) leaves them out.
constexpr int kPpTermStride = kRadialTerms + 1;  // floats per candidate in k_neighbors_pp's LDS
template <bool RAD>
__global__ void __launch_bounds__(kBlock) k_neighbors_pp(const FrameInfo* __restrict__ frames,
                                                         const int32_t* __restrict__ frame_of,
                                                         const double* __restrict__ pos,
                                                         const int32_t* __restrict__ perm_start,
                                                         const double4* __restrict__ bucket_pos, float rc_radial,
                                                         float rc_angular, NeighborLists nl,
                                                         int32_t* __restrict__ flags, float* __restrict__ rad_v) {
    constexpr int G = kPairLanes;
    __shared__ float pp_terms[RAD ? kBlock : 1][2 * kPpTermStride];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = tid / G;  // tile slot (the whole group takes the same branches below)
    const int g = (int)(tid % G);
    if (p >= nl.n_pad) return;
    const int a = nl.perm[p];
    const int T = nl.T;
    if (a < 0) {  // padding slot (k_neighbors writes the same zeros when it runs)
        if (g == 0) {
            RadialSums none;
            none.clear();
            for (int t = 0; t < T; ++t) {
                nl.counts[(int64_t)(2 * t) * nl.n_pad + p] = 0;
                nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p] = 0;
                none.store(rad_v, t, nl.n_pad, p);
            }
        }
        return;
    }
    const FrameInfo fi = frames[frame_of[a]];
    if (fi.mode != 0 || fi.tric || fi.role != kRolePlain) return;
    const double xi = pos[3 * a], yi = pos[3 * a + 1], zi = pos[3 * a + 2];
    const double rc2r = (double)rc_radial * rc_radial, rc2a = (double)rc_angular * rc_angular;
    const float rcR_inv = 1.f / rc_radial;
    float4* lane_base = nl.entries + ((int64_t)(p >> 6) * (nl.slots >> 2) * 64 + (p & 63)) * 4;
    const int first = (int)(threadIdx.x & 63) & ~(G - 1);  // first lane of the group in the wave
    const uint32_t before = (1u << g) - 1;                  // lanes of the group below this one
    bool overlap = false;
    for (int t = 0; t < T; ++t) {
        const int b0 = perm_start[fi.cell_base * T + t];
        const int n = perm_start[(fi.cell_base + 1) * T + t] - b0;
        float4* ga = lane_base + (int64_t)(nl.meta[kMetaSegA + t] >> 2) * 256;
        float4* gr = lane_base + (int64_t)(nl.meta[kMetaSegR + t] >> 2) * 256;
        const int capA = nl.meta[kMetaCapA + t], capR = nl.meta[kMetaCapR + t];
        int na = 0, nr = 0;  // rows so far (equal in the group's lanes)
        // lane g < kRadialTerms: sum over accepted pairs of f_c T_g (g = 0: of f_c)
        float rsum = 0.f;
        for (int q0 = 0; q0 < n; q0 += 2 * G) {
            float sf[2] = {0.f, 0.f}, Tk[2][kRadialTerms] = {};
            uint32_t acc[2];
            double4 cur[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int q = q0 + u * G + g;
                cur[u] = q < n ? bucket_pos[b0 + q] : make_double4(0.0, 0.0, 0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int q = q0 + u * G + g;
                const int j = b0 + q;
                const double dx = min_image(cur[u].x - xi, fi.L[0], fi.Linv[0]);
                const double dy = min_image(cur[u].y - yi, fi.L[1], fi.Linv[1]);
                const double dz = min_image(cur[u].z - zi, fi.L[2], fi.Linv[2]);
                const double r2 = dx * dx + dy * dy + dz * dz;
                const bool in = (q < n) & (j != (int)p) & (r2 < rc2r);
                const bool ang = in && r2 < rc2a, rad = in && !(r2 < rc2a);
                overlap |= in && r2 < 1e-8;
                const uint32_t ma = (uint32_t)(__ballot(ang) >> first) & 0xFFFFu;
                const uint32_t mr = (uint32_t)(__ballot(rad) >> first) & 0xFFFFu;
                const float4 e = make_float4((float)dx, (float)dy, (float)dz, __int_as_float(j));
                if (ang) {
                    const int row = na + __popc(ma & before);
                    if (row < capA) ga[(int64_t)(row >> 2) * 256 + (row & 3)] = e;
                }
                if (rad) {
                    const int row = nr + __popc(mr & before);
                    if (row < capR) gr[(int64_t)(row >> 2) * 256 + (row & 3)] = e;
                }
                na += __popc(ma);
                nr += __popc(mr);
                acc[u] = ma | mr;
                if (RAD && in) RadialSums::terms(e.x, e.y, e.z, rcR_inv, sf[u], Tk[u]);
            }
            if constexpr (RAD) {
                // each lane's terms (sf, f_c = sf^2, T_1..T_8 per candidate half) in LDS;
                // the wave's LDS accesses complete in order, so the reads below see
                // these writes and the next iteration's writes follow the reads
                float* mine = pp_terms[threadIdx.x];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    mine[u * kPpTermStride] = sf[u];
                    mine[u * kPpTermStride + 1] = sf[u] * sf[u];
#pragma unroll
                    for (int k = 1; k < kRadialTerms; ++k) mine[u * kPpTermStride + 1 + k] = Tk[u][k];
                }
                // candidate order: u = 0 (lanes 0..15), then u = 1; the mask is the
                // same in the group's lanes, so they run the loop together
                const float(*wave_terms)[2 * kPpTermStride] = pp_terms + (threadIdx.x & ~63u);
                if (g < kRadialTerms) {
                    // up to four accepted candidates per step: their terms are read
                    // together, then added one after another in candidate order
                    const int a = g == 0 ? 0 : 1, b = g == 0 ? 0 : 1 + g;  // rsum += t[a] * t[b]
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        uint32_t m = acc[u];
                        while (m != 0u) {
                            float x[4], y[4];
                            int n_take = 0;
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                x[i] = 0.f;
                                y[i] = 0.f;
                                if (m != 0u) {
                                    const float* ts = wave_terms[first + __builtin_ctz(m)] + u * kPpTermStride;
                                    x[i] = ts[a];
                                    y[i] = ts[b];
                                    m &= m - 1u;
                                    n_take = i + 1;
                                }
                            }
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                if (i < n_take) rsum = __builtin_fmaf(x[i], y[i], rsum);
                        }
                    }
                }
            }
        }
        if constexpr (RAD) {
            // sum_j f_k(r_ij) = (sum f_c T_k + sum f_c) / 2, as RadialSums::store forms it
            const float fs = __shfl(rsum, first, 64);
            if (g < kRadialTerms) rad_v[(int64_t)(t * kRadialTerms + g) * nl.n_pad + p] = 0.5f * (rsum + fs);
        }
        if (g == 0) {
            nl.counts[(int64_t)(2 * t) * nl.n_pad + p] = min(na, capA);
            nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p] = min(nr, capR);
            if (na > capA) atomicMax(&flags[kFlagCapAng + t], na);
            if (nr > capR) atomicMax(&flags[kFlagCapRad + t], nr);
        }
    }
    if (overlap) {
        atomicOr(&flags[kFlagError], kErrOverlap);
        atomicMin(&flags[kFlagBadAtom], call_atom(nl.meta, a));
    }
}

// Frames that follow a reference frame of their trajectory window.  Their
// atoms were binned where their reference atoms are (k_bin), so an atom has its
// reference atom's rank in its species range and takes that atom's candidate
// list (CandLists, read four candidates per 16-byte load, the lists of a
// wavefront's lanes side by side).  A packed candidate gives the neighbour's
// rank and the offset between the two atoms' cells; the pair vector is
// (q_j - q_i) + offset x cell edge from the FP32 offsets of this frame's atoms
// to those cell centres (k_sort_place), tested with the exact r < r_c.  Lists
// are complete while no atom is more than skin / 2 from its reference
// position (and species match), which the kernel checks in FP64.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_neighbors_follow(
    const FrameInfo* __restrict__ frames, const int32_t* __restrict__ frame_of, const double* __restrict__ pos,
    const int32_t* __restrict__ species, const int32_t* __restrict__ perm_start, const int4* __restrict__ cell_rec,
    float rc_radial, float rc_angular, NeighborLists nl, CandLists cl, int32_t* __restrict__ flags,
    float* __restrict__ rad_v) {
    // 8 staged entries per lane (PairSink), then a 64-entry list per wave (coop_flush)
    extern __shared__ float4 nb_stage[];
    float4* stage = nb_stage + threadIdx.x;
    int4* wlist = reinterpret_cast<int4*>(nb_stage + 8 * blockDim.x) + (threadIdx.x & ~63u);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nl.n_pad) return;
    const int T = nl.T;
    const int a = nl.perm[p];
    if (a < 0) return;
    const FrameInfo fi = frames[frame_of[a]];
    if (fi.role != kRoleFollower) return;
    const int tile = (int)(p >> 6), lane = (int)(p & 63);
    const int ti = species[a];
    const int64_t aref = fi.ref_begin + (a - fi.atom_begin);
    const double mx = min_image(pos[3 * a] - pos[3 * aref], fi.L[0], fi.Linv[0]);
    const double my = min_image(pos[3 * a + 1] - pos[3 * aref + 1], fi.L[1], fi.Linv[1]);
    const double mz = min_image(pos[3 * a + 2] - pos[3 * aref + 2], fi.L[2], fi.Linv[2]);
    if (!(mx * mx + my * my + mz * mz <= (double)cl.half_skin2) || ti != species[aref])
        atomicOr(&flags[kFlagReuse], 1);
    const float rcR_inv = 1.f / rc_radial;
    const float rc2rf = rc_radial * rc_radial, rc2af = rc_angular * rc_angular;
    const float hx = (float)(fi.L[0] / fi.nc[0]), hy = (float)(fi.L[1] / fi.nc[1]), hz = (float)(fi.L[2] / fi.nc[2]);
    const int4 own = cell_rec[p];
    const float qx = __int_as_float(own.x), qy = __int_as_float(own.y), qz = __int_as_float(own.z);
    float4* lane_base = nl.entries + ((int64_t)tile * (nl.slots >> 2) * 64 + lane) * 4;
    const int64_t R = fi.cl_base + (int64_t)ti * ((fi.n_atoms + 63) & ~63) + ((int)p - perm_start[fi.cell_base * T + ti]);
    bool overlap = false;
    int no_cand = 0;
    for (int t = 0; t < T; ++t) {
        PairSink ps{stage, (int)blockDim.x,
                    lane_base + (int64_t)(nl.meta[kMetaSegA + t] >> 2) * 256,
                    lane_base + (int64_t)(nl.meta[kMetaSegR + t] >> 2) * 256,
                    nl.meta[kMetaCapA + t], nl.meta[kMetaCapR + t], 0, 0, -1, nullptr};
        RadialSums rsum;
        rsum.clear();
        const int64_t li = (R >> 6) * T + t;
        const int n = min(cl.count[li * 64 + (R & 63)], cl.cap);
        const int4* c4 = reinterpret_cast<const int4*>(cl.idx) + li * (cl.cap >> 2) * 64 + (R & 63);
        const int base_t = perm_start[fi.cell_base * T + t];
        for (int q = 0; q < n; q += 4) {
            const int4 cc = c4[(q >> 2) * 64];
            // rows past the list's end hold no candidate: read slot base_t instead
            const unsigned pk[4] = {q < n ? (unsigned)cc.x : 0u, q + 1 < n ? (unsigned)cc.y : 0u,
                                    q + 2 < n ? (unsigned)cc.z : 0u, q + 3 < n ? (unsigned)cc.w : 0u};
            int4 rec[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) rec[u] = cell_rec[base_t + (int)(pk[u] >> 9)];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = base_t + (int)(pk[u] >> 9);
                const float dx = (__int_as_float(rec[u].x) - qx) + (float)((int)((pk[u] >> 6) & 7u) - 3) * hx;
                const float dy = (__int_as_float(rec[u].y) - qy) + (float)((int)((pk[u] >> 3) & 7u) - 3) * hy;
                const float dz = (__int_as_float(rec[u].z) - qz) + (float)((int)(pk[u] & 7u) - 3) * hz;
                const float r2 = dx * dx + dy * dy + dz * dz;
                take_candidate<false, float>(ps, rsum, rcR_inv, nb_stage, (q + u < n) & (r2 < rc2rf), dx, dy, dz, r2,
                                             j, rc2rf, rc2af, overlap, no_cand, nullptr, 0, 0);
                coop_flush(ps, nb_stage, wlist);
            }
        }
        rsum.store(rad_v, t, nl.n_pad, p);
        ps.flush();
        nl.counts[(int64_t)(2 * t) * nl.n_pad + p] = min(ps.na, ps.capA);
        nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p] = min(ps.nr, ps.capR);
        if (ps.na > ps.capA) atomicMax(&flags[kFlagCapAng + t], ps.na);
        if (ps.nr > ps.capR) atomicMax(&flags[kFlagCapRad + t], ps.nr);
    }
    if (overlap) {
        atomicOr(&flags[kFlagError], kErrOverlap);
        atomicMin(&flags[kFlagBadAtom], call_atom(nl.meta, a));
    }
}

// Triclinic frames: one lane per tile slot.  Bins in fractional coordinates
// s = r Hinv of perpendicular width w_k / nc_k >= r_c / 2, so a neighbour
// within r_c is at most two bins away along each lattice vector (the distance
// between two lattice planes bounds the pair distance from below).  As for
// orthorhombic grids, the bins are walked as 25 columns along the third
// lattice vector, each trimmed to the bins within reach; a column or bin is
// skipped when the perpendicular distance to it along one axis reaches r_c
// (the sum of squares would not be a lower bound on skewed cells).  The
// fractional difference of a pair is (bin offset) / nc + (q_j - q_i) q_unit
// from the cell records, and d = f H.  Frames without bins (cells narrower
// than 2.5 r_c) take the minimum image by rounding, f -= rint(f): with every
// width >= 2 r_c an image within r_c has all |f_k| < 1/2.
__global__ void __launch_bounds__(kBlock) k_neighbors_tri(const FrameInfo* __restrict__ frames,
                                                          const FrameTric* __restrict__ tric,
                                                          const int32_t* __restrict__ frame_of,
                                                          const double* __restrict__ pos,
                                                          const int32_t* __restrict__ key_of,
                                                          const int32_t* __restrict__ perm_start,
                                                          const double4* __restrict__ bucket_pos,
                                                          const int4* __restrict__ cell_rec, float rc_radial,
                                                          float rc_angular, NeighborLists nl,
                                                          int32_t* __restrict__ flags, float* __restrict__ rad_v) {
    // 8 staged entries per lane (PairSink), then a 64-entry list per wave (coop_flush)
    extern __shared__ float4 nb_stage[];
    float4* stage = nb_stage + threadIdx.x;
    int4* list = reinterpret_cast<int4*>(nb_stage + 8 * blockDim.x) + (threadIdx.x & ~63u);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nl.n_pad) return;
    const int T = nl.T;
    const int a = nl.perm[p];
    if (a < 0) return;
    const int fidx = frame_of[a];
    if (!frames[fidx].tric) return;
    const FrameInfo& fi = frames[fidx];
    const FrameTric& ft = tric[fidx];
    const int tile = (int)(p >> 6), lane = (int)(p & 63);
    const double xi = pos[3 * a], yi = pos[3 * a + 1], zi = pos[3 * a + 2];
    const double rc2r = (double)rc_radial * rc_radial, rc2a = (double)rc_angular * rc_angular;
    const float prune = rc_radial + 1e-3f;
    float4* lane_base = nl.entries + ((int64_t)tile * (nl.slots >> 2) * 64 + lane) * 4;
    const int mode = fi.mode, cell_base = fi.cell_base;
    const int nx = fi.nc[0], ny = fi.nc[1], nz = fi.nc[2];
    double H[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) H[q] = ft.H[q];
    // wrapped fractional coordinates of the atom
    double si[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        si[q] = xi * ft.Hinv[q] + yi * ft.Hinv[3 + q] + zi * ft.Hinv[6 + q];
        si[q] -= floor(si[q]);
    }
    int ib[3] = {0, 0, 0};
    float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f}, hb[3] = {0.f, 0.f, 0.f};
    int4 own = make_int4(0, 0, 0, 0);  // the atom's own cell record
    if (mode == 1) {
        own = cell_rec[p];
        const int local = key_of[a] / T - cell_base;
        ib[2] = local % nz;
        ib[1] = (local / nz) % ny;
        ib[0] = local / (nz * ny);
        // perpendicular distances (A) to the faces of the atom's bin, and bin widths
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double inv = 1.0 / (double)fi.nc[k];
            lo[k] = (float)fmax((si[k] - ib[k] * inv) * ft.w[k], 0.0);
            hi[k] = (float)fmax(((ib[k] + 1) * inv - si[k]) * ft.w[k], 0.0);
            hb[k] = (float)(ft.w[k] * inv);
        }
    }
    const float hb2_inv = mode == 1 ? 1.f / hb[2] : 0.f;
    const float rcR_inv = 1.f / rc_radial;
    bool overlap = false;
    for (int t = 0; t < T; ++t) {
        PairSink ps{stage, (int)blockDim.x,
                    lane_base + (int64_t)(nl.meta[kMetaSegA + t] >> 2) * 256,
                    lane_base + (int64_t)(nl.meta[kMetaSegR + t] >> 2) * 256,
                    nl.meta[kMetaCapA + t], nl.meta[kMetaCapR + t], 0, 0, -1, nullptr};
        RadialSums rsum;
        rsum.clear();
        if (mode == 1) {
            for (int col = 0; col < 25; ++col) {
                const int o0 = col / 5 - 2, o1 = col % 5 - 2;
                if (fmaxf(cell_gap(o0, lo[0], hi[0], hb[0]), cell_gap(o1, lo[1], hi[1], hb[1])) >= prune) continue;
                // bins ib2 - below .. ib2 + above: bin ib2 - k is in reach when lo_2 + (k - 1) hb_2 < prune
                const int below = min(kCellReachZ, max(0, (int)floorf((prune - lo[2]) * hb2_inv) + 1));
                const int above = min(kCellReachZ, max(0, (int)floorf((prune - hi[2]) * hb2_inv) + 1));
                const int z0 = ib[2] - below, z1 = ib[2] + above;
                const int col0 = (cell_base + (wrap_cell(ib[0] + o0, nx) * ny + wrap_cell(ib[1] + o1, ny)) * nz) * T + t;
                int b0, e0, b1 = 0, e1 = 0;
                if (z0 >= 0 && z1 < nz) {
                    b0 = perm_start[col0 + z0 * T];
                    e0 = perm_start[col0 + (z1 + 1) * T];
                } else {
                    b0 = perm_start[col0 + (z0 < 0 ? z0 + nz : z0) * T];
                    e0 = perm_start[col0 + nz * T];
                    b1 = perm_start[col0];
                    e1 = perm_start[col0 + ((z1 >= nz ? z1 - nz : z1) + 1) * T];
                }
                const int n0 = e0 - b0, n = n0 + (e1 - b1), d1 = b1 - n0;
                const double f0_off = (double)o0 / nx, f1_off = (double)o1 / ny, inv_nz = 1.0 / nz, qu = fi.q_unit;
                for (int q = 0; q < n; q += 2) {
                    const int k0 = q < n0 ? b0 + q : d1 + q;
                    const int k1 = q + 1 < n0 ? b0 + q + 1 : d1 + q + 1;
                    const int4 c0 = cell_rec[k0];
                    const int4 c1 = q + 1 < n ? cell_rec[k1] : make_int4(0, 0, 0, 0);
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int4 cr = u == 0 ? c0 : c1;
                        const int j = u == 0 ? k0 : k1;  // tile slot of the candidate
                        int oz = cr.w - ib[2];
                        oz = oz > kCellReachZ ? oz - nz : (oz < -kCellReachZ ? oz + nz : oz);
                        const double f0 = fma((double)(cr.x - own.x), qu, f0_off);
                        const double f1 = fma((double)(cr.y - own.y), qu, f1_off);
                        const double f2 = fma((double)(cr.z - own.z), qu, oz * inv_nz);
                        const double dx = f0 * H[0] + f1 * H[3] + f2 * H[6];
                        const double dy = f0 * H[1] + f1 * H[4] + f2 * H[7];
                        const double dz = f0 * H[2] + f1 * H[5] + f2 * H[8];
                        const double r2 = dx * dx + dy * dy + dz * dz;
                        // one branch per candidate: a real candidate, not the atom itself, within r_c
                        if ((q + u < n) & (j != (int)p) & (r2 < rc2r)) {
                            overlap |= r2 < 1e-8;
                            const float4 ent = make_float4((float)dx, (float)dy, (float)dz, __int_as_float(j));
                            ps.push_deferred(ent, r2 < rc2a, nb_stage);
                            rsum.add(ent.x, ent.y, ent.z, rcR_inv);
                        }
                        coop_flush(ps, nb_stage, list);
                    }
                }
            }
        } else {
            // one bin per frame: wrapped fractional positions, minimum image by rounding
            const int b = perm_start[cell_base * T + t], e = perm_start[(cell_base + 1) * T + t];
            for (int k0 = b; k0 < e; k0 += 2) {
                const double4 q0 = bucket_pos[k0];
                const double4 q1 = k0 + 1 < e ? bucket_pos[k0 + 1] : make_double4(0.0, 0.0, 0.0, 0.0);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const double4 cur = u == 0 ? q0 : q1;
                    const int j = k0 + u;  // tile slot of the candidate
                    double f0 = cur.x - si[0], f1 = cur.y - si[1], f2 = cur.z - si[2];
                    f0 -= rint(f0);
                    f1 -= rint(f1);
                    f2 -= rint(f2);
                    const double dx = f0 * H[0] + f1 * H[3] + f2 * H[6];
                    const double dy = f0 * H[1] + f1 * H[4] + f2 * H[7];
                    const double dz = f0 * H[2] + f1 * H[5] + f2 * H[8];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if ((k0 + u < e) & (j != (int)p) & (r2 < rc2r)) {
                        overlap |= r2 < 1e-8;
                        const float4 ent = make_float4((float)dx, (float)dy, (float)dz, __int_as_float(j));
                        ps.push_deferred(ent, r2 < rc2a, nb_stage);
                        rsum.add(ent.x, ent.y, ent.z, rcR_inv);
                    }
                    coop_flush(ps, nb_stage, list);
                }
            }
        }
        rsum.store(rad_v, t, nl.n_pad, p);
        ps.flush();
        nl.counts[(int64_t)(2 * t) * nl.n_pad + p] = min(ps.na, ps.capA);
        nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p] = min(ps.nr, ps.capR);
        if (ps.na > ps.capA) atomicMax(&flags[kFlagCapAng + t], ps.na);
        if (ps.nr > ps.capR) atomicMax(&flags[kFlagCapRad + t], ps.nr);
    }
    if (overlap) {
        atomicOr(&flags[kFlagError], kErrOverlap);
        atomicMin(&flags[kFlagBadAtom], call_atom(nl.meta, a));
    }
}

// Grid-stride over the tile slots with a bounded grid: the block totals are
// added with three atomics per block on the same three counters, which
// serialise (one block per 256 slots spent ~0.15 ms per million atoms there).
constexpr int kCountBlocks = 512;
__global__ void k_count_pairs(const NeighborLists nl, unsigned long long* __restrict__ counters) {
    __shared__ unsigned long long s_ang[kBlock], s_rad[kBlock], s_at[kBlock];
    unsigned long long na = 0, nr = 0, at = 0;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nl.n_pad; p += (int64_t)gridDim.x * kBlock) {
        if (nl.perm[p] < 0) continue;
        at += 1;
        for (int t = 0; t < nl.T; ++t) {
            na += (unsigned long long)nl.counts[(int64_t)(2 * t) * nl.n_pad + p];
            nr += (unsigned long long)nl.counts[(int64_t)(2 * t + 1) * nl.n_pad + p];
        }
    }
    s_ang[threadIdx.x] = na;
    s_rad[threadIdx.x] = nr;
    s_at[threadIdx.x] = at;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s_ang[threadIdx.x] += s_ang[threadIdx.x + off];
            s_rad[threadIdx.x] += s_rad[threadIdx.x + off];
            s_at[threadIdx.x] += s_at[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&counters[0], s_at[0]);
        atomicAdd(&counters[1], s_ang[0] + s_rad[0]);
        atomicAdd(&counters[2], s_ang[0]);
    }
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_neighbors(const FrameInfo* d_frames, const FrameTric* d_tric, int cap_frames, const double* pos,
                            const int32_t* species,
                            int64_t cap_atoms, int cap_cells, float rc_radial, float rc_angular, const NeighborWork& w,
                            const NeighborLists& nl, const CandLists& cl, bool references, bool followers,
                            bool triclinic, bool pair_search, bool pair_radial, bool plain_grid, int32_t* d_flags,
                            int neigh_block, float* rad_sums, hipStream_t s) {
    if (cap_atoms == 0 || cap_frames == 0) return hipSuccess;
    const int nb = (neigh_block == 64 || neigh_block == 128) ? neigh_block : kBlock;
    const int T = nl.T;
    const int cap_buckets = cap_cells * T;
    const int cap_chunks = (cap_cells + kScanCells - 1) / kScanCells;
    if (cap_atoms <= kBucketSmallAtoms && cap_cells <= kScanCells && cap_frames <= kScanCells &&
        cap_buckets <= kBucketSmallBuckets) {
        k_bucket_small<<<1, kBucketSmallBlock, 0, s>>>(d_frames, d_tric, pos, species, T, w, nl.n_pad, d_flags);
    } else {
        const int64_t setup_threads = std::max<int64_t>({(int64_t)cap_frames * kBlock, (int64_t)cap_buckets, nl.n_pad});
        k_batch_setup<<<blocks_for(setup_threads, kBlock), kBlock, 0, s>>>(d_frames, nl.meta, w.frame_of, w.bucket_count,
                                                                          cap_buckets, w.perm, nl.n_pad);
        k_bin<<<blocks_for(cap_atoms, kBlock), kBlock, 0, s>>>(d_frames, d_tric, w.frame_of, pos, species, nl.meta, T,
                                                              w.key_of, w.bucket_count, d_flags);
        if (cap_chunks == 1) {
            k_scan_one<<<1, 256, 0, s>>>(w.bucket_count, w.meta, T, w.bucket_start, w.bucket_fill, w.perm_start);
        } else {
            k_scan_partials<<<cap_chunks, 256, 0, s>>>(w.bucket_count, nl.meta, T, w.chunk);
            k_scan_chunks<<<1, 256, 0, s>>>(w.chunk, T, w.chunk + 9 * cap_chunks, w.meta, w.bucket_start);
            k_scan_final<<<cap_chunks, 256, 0, s>>>(w.bucket_count, nl.meta, T, w.chunk + 9 * cap_chunks, w.bucket_start,
                                                   w.bucket_fill, w.perm_start);
        }
        k_scatter<<<blocks_for(cap_atoms, kBlock), kBlock, 0, s>>>(w.key_of, w.bucket_start, w.bucket_fill,
                                                                  w.bucket_atoms, nl.meta);
        k_sort_place<<<blocks_for(cap_atoms, kBlock), kBlock, 0, s>>>(d_frames, d_tric, w.frame_of, w.key_of,
                                                                     w.bucket_start, w.bucket_atoms, w.perm_start, w.perm,
                                                                     w.slot_of, pos, w.bucket_pos, w.cell_rec, nl.meta, T);
    }
    const size_t list_bytes = sizeof(float4) * 9 * nb;  // staging + per-wave flush lists
    // with pair_search and no plain cell-grid frame, k_neighbors_pp covers every
    // slot k_neighbors would (frames without a grid and the padding)
    if (!pair_search || plain_grid)
        k_neighbors<false><<<blocks_for(nl.n_pad, nb), nb, list_bytes, s>>>(d_frames, w.frame_of, pos, species, w.slot_of,
                                                              w.key_of, w.perm_start, w.bucket_pos, w.cell_rec,
                                                              rc_radial, rc_angular, nl, cl, d_flags, rad_sums,
                                                              pair_search);
    if (pair_search) {  // n_pad is a multiple of 64: whole work-groups
        const unsigned grid = (unsigned)(nl.n_pad * kPairLanes / kBlock);
        if (pair_radial)
            k_neighbors_pp<true><<<grid, kBlock, 0, s>>>(d_frames, w.frame_of, pos, w.perm_start, w.bucket_pos, rc_radial,
                                                         rc_angular, nl, d_flags, rad_sums);
        else
            k_neighbors_pp<false><<<grid, kBlock, 0, s>>>(d_frames, w.frame_of, pos, w.perm_start, w.bucket_pos, rc_radial,
                                                          rc_angular, nl, d_flags, nullptr);
    }
    if (references)
        k_neighbors<true><<<blocks_for(nl.n_pad, nb), nb, list_bytes, s>>>(d_frames, w.frame_of, pos, species, w.slot_of,
                                                                 w.key_of, w.perm_start, w.bucket_pos, w.cell_rec,
                                                                 rc_radial, rc_angular, nl, cl, d_flags, rad_sums, false);
    if (triclinic)
        k_neighbors_tri<<<blocks_for(nl.n_pad, nb), nb, list_bytes, s>>>(d_frames, d_tric, w.frame_of, pos, w.key_of, w.perm_start,
                                                               w.bucket_pos, w.cell_rec, rc_radial, rc_angular, nl,
                                                               d_flags, rad_sums);
    if (followers)
        k_neighbors_follow<<<blocks_for(nl.n_pad, nb), nb, list_bytes, s>>>(d_frames, w.frame_of, pos, species,
                                                                  w.perm_start, w.cell_rec, rc_radial, rc_angular,
                                                                  nl, cl, d_flags, rad_sums);
    return hipGetLastError();
}

hipError_t launch_count_pairs(const NeighborLists& nl, unsigned long long* counters, hipStream_t s) {
    if (nl.n_pad == 0) return hipSuccess;
    k_count_pairs<<<std::min<unsigned>(blocks_for(nl.n_pad, kBlock), kCountBlocks), kBlock, 0, s>>>(nl, counters);
    return hipGetLastError();
}

}  // namespace tnep
