// Neighbour search for a batch of ragged frames on gfx950.
//
// The sums over j != i of the method (Sec. 2.1, Eq. virial; Sec. 2.2, Eq. mu;
// Sec. 2.3, Eq. polarizability-model) run over the atoms inside the radial
// cutoff.  Fully periodic orthorhombic frames with at least three cells of
// edge >= rc_radial per axis use a cell list (counting sort of atoms into
// cells, then the 27-cell stencil); every other frame (vacuum molecules,
// small boxes) uses an all-pairs scan inside the frame.  Pair vectors are
// formed in FP64 with the minimum-image convention and stored as FP32.
//
// Results are independent of thread scheduling: atoms inside a cell are
// sorted by index after the atomic scatter, and neighbours are written in
// stencil order, then index order.
#include "internal.h"

namespace tnep {

namespace {

constexpr int kBlock = 256;

__global__ void k_frame_of(const FrameInfo* __restrict__ frames, int32_t* __restrict__ frame_of) {
    const int f = blockIdx.x;
    const FrameInfo fi = frames[f];
    for (int64_t a = threadIdx.x; a < fi.n_atoms; a += blockDim.x) frame_of[fi.atom_begin + a] = f;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__device__ __forceinline__ int cell_coord(double p, double L, int nc) {
    double s = p - L * floor(p / L);
    int c = (int)(s * (double)nc / L);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_bin(const FrameInfo* __restrict__ frames, const int32_t* __restrict__ frame_of,
                      const double* __restrict__ pos, const int32_t* __restrict__ species, int64_t n_atoms,
                      int n_species, int32_t* __restrict__ cell_of, int32_t* __restrict__ cell_count,
                      int32_t* __restrict__ flags) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_atoms) return;
    const FrameInfo& fi = frames[frame_of[a]];
    const double x = pos[3 * a], y = pos[3 * a + 1], z = pos[3 * a + 2];
    const int t = species[a];
    int err = 0;
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) err |= kErrNonFinite;
    if (t < 0 || t >= n_species) err |= kErrSpecies;
    if (err) {
        atomicOr(&flags[kFlagError], err);
        atomicMin(&flags[kFlagBadAtom], (int)a);
        cell_of[a] = -1;
        return;
    }
    if (fi.mode != 1) {
        cell_of[a] = -1;
        return;
    }
    const int ix = cell_coord(x, fi.L[0], fi.nc[0]);
    const int iy = cell_coord(y, fi.L[1], fi.nc[1]);
    const int iz = cell_coord(z, fi.L[2], fi.nc[2]);
    const int c = fi.cell_base + (ix * fi.nc[1] + iy) * fi.nc[2] + iz;
    cell_of[a] = c;
    atomicAdd(&cell_count[c], 1);
}

// Exclusive scan of cell_count into cell_start (n + 1 entries); one work-group.
__global__ void __launch_bounds__(1024) k_scan(const int32_t* __restrict__ count, int32_t* __restrict__ start,
                                               int32_t* __restrict__ fill, int n) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int b = tid * chunk;
    const int e = min(b + chunk, n);
    int32_t s = 0;
    for (int i = b; i < e; ++i) s += count[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = part[tid] - s;  // exclusive prefix of this chunk
    for (int i = b; i < e; ++i) {
        start[i] = run;
        fill[i] = 0;
        run += count[i];
    }
    if (tid == 1023) start[n] = part[1023];
}

__global__ void k_scatter(const int32_t* __restrict__ cell_of, const int32_t* __restrict__ cell_start,
                          int32_t* __restrict__ cell_fill, int32_t* __restrict__ cell_atoms, int64_t n_atoms) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n_atoms) return;
    const int c = cell_of[a];
    if (c < 0) return;
    const int slot = atomicAdd(&cell_fill[c], 1);
    cell_atoms[cell_start[c] + slot] = (int32_t)a;
}

__global__ void k_sort_cells(const int32_t* __restrict__ cell_start, int32_t* __restrict__ cell_atoms, int n_cells) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int b = cell_start[c], e = cell_start[c + 1];
    for (int i = b + 1; i < e; ++i) {
        const int32_t v = cell_atoms[i];
        int j = i - 1;
        while (j >= b && cell_atoms[j] > v) {
            cell_atoms[j + 1] = cell_atoms[j];
            --j;
        }
        cell_atoms[j + 1] = v;
    }
}

struct PairSink {
    float4* entries;
    int64_t n_atoms;
    int64_t i;
    int cap_ang, cap_rad;
    int n_ang, n_rad;
    float rc2_ang, rc2_rad;
    bool overlap;

    __device__ __forceinline__ void add(double dx, double dy, double dz, int tj) {
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= (double)rc2_rad) return;
        if (r2 < 1e-8) overlap = true;
        const float4 e = make_float4((float)dx, (float)dy, (float)dz, __int_as_float(tj));
        if (r2 < (double)rc2_ang) {
            if (n_ang < cap_ang) entries[(int64_t)n_ang * n_atoms + i] = e;
            ++n_ang;
        } else {
            if (n_rad < cap_rad) entries[(int64_t)(cap_ang + n_rad) * n_atoms + i] = e;
            ++n_rad;
        }
    }
};

__device__ __forceinline__ double min_image(double d, double L, int per) {
    return per ? d - L * rint(d / L) : d;
}

__global__ void __launch_bounds__(kBlock) k_neighbors(const FrameInfo* __restrict__ frames,
                                                      const int32_t* __restrict__ frame_of,
                                                      const double* __restrict__ pos,
                                                      const int32_t* __restrict__ species,
                                                      const int32_t* __restrict__ cell_of,
                                                      const int32_t* __restrict__ cell_start,
                                                      const int32_t* __restrict__ cell_atoms, int64_t n_atoms,
                                                      float rc_radial, float rc_angular, NeighborLists nl,
                                                      int32_t* __restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_atoms) return;
    const FrameInfo& fi = frames[frame_of[i]];
    PairSink sink{nl.entries, n_atoms, i, nl.cap_ang, nl.cap_rad, 0, 0,
                  rc_angular * rc_angular, rc_radial * rc_radial, false};
    const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    if (fi.mode == 1) {
        const int c = cell_of[i];
        if (c < 0) {
            nl.n_ang[i] = 0;
            nl.n_rad[i] = 0;
            return;
        }
        const int local = c - fi.cell_base;
        const int nz = fi.nc[2], ny = fi.nc[1], nx = fi.nc[0];
        const int iz = local % nz, iy = (local / nz) % ny, ix = local / (nz * ny);
        for (int ddx = -1; ddx <= 1; ++ddx) {
            const int cx = (ix + ddx + nx) % nx;
            for (int ddy = -1; ddy <= 1; ++ddy) {
                const int cy = (iy + ddy + ny) % ny;
                for (int ddz = -1; ddz <= 1; ++ddz) {
                    const int cz = (iz + ddz + nz) % nz;
                    const int cc = fi.cell_base + (cx * ny + cy) * nz + cz;
                    const int b = cell_start[cc], e = cell_start[cc + 1];
                    for (int k = b; k < e; ++k) {
                        const int j = cell_atoms[k];
                        if (j == i) continue;
                        const double dx = min_image(pos[3 * j] - xi, fi.L[0], 1);
                        const double dy = min_image(pos[3 * j + 1] - yi, fi.L[1], 1);
                        const double dz = min_image(pos[3 * j + 2] - zi, fi.L[2], 1);
                        sink.add(dx, dy, dz, species[j]);
                    }
                }
            }
        }
    } else {
        const int64_t b = fi.atom_begin, e = fi.atom_begin + fi.n_atoms;
        for (int64_t j = b; j < e; ++j) {
            if (j == i) continue;
            const double dx = min_image(pos[3 * j] - xi, fi.L[0], fi.per[0]);
            const double dy = min_image(pos[3 * j + 1] - yi, fi.L[1], fi.per[1]);
            const double dz = min_image(pos[3 * j + 2] - zi, fi.L[2], fi.per[2]);
            sink.add(dx, dy, dz, species[j]);
        }
    }
    nl.n_ang[i] = min(sink.n_ang, nl.cap_ang);
    nl.n_rad[i] = min(sink.n_rad, nl.cap_rad);
    if (sink.n_ang > nl.cap_ang) atomicMax(&flags[kFlagMaxAng], sink.n_ang);
    if (sink.n_rad > nl.cap_rad) atomicMax(&flags[kFlagMaxRad], sink.n_rad);
    if (sink.overlap) {
        atomicOr(&flags[kFlagError], kErrOverlap);
        atomicMin(&flags[kFlagBadAtom], (int)i);
    }
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void k_count_pairs(const int32_t* __restrict__ n_ang, const int32_t* __restrict__ n_rad, int64_t n,
                              unsigned long long* __restrict__ counters) {
    __shared__ unsigned long long s_ang[kBlock], s_rad[kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    s_ang[threadIdx.x] = i < n ? (unsigned long long)n_ang[i] : 0ull;
    s_rad[threadIdx.x] = i < n ? (unsigned long long)n_rad[i] : 0ull;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s_ang[threadIdx.x] += s_ang[threadIdx.x + off];
            s_rad[threadIdx.x] += s_rad[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long na = (unsigned long long)min<int64_t>(kBlock, n - (int64_t)blockIdx.x * kBlock);
        atomicAdd(&counters[0], na);
        atomicAdd(&counters[1], s_ang[0] + s_rad[0]);
        atomicAdd(&counters[2], s_ang[0]);
    }
}

}  // namespace

hipError_t launch_count_pairs(const NeighborLists& nl, unsigned long long* counters, hipStream_t s) {
    if (nl.n_atoms == 0) return hipSuccess;
    k_count_pairs<<<blocks_for(nl.n_atoms, kBlock), kBlock, 0, s>>>(nl.n_ang, nl.n_rad, nl.n_atoms, counters);
    return hipGetLastError();
}

hipError_t launch_neighbors(const FrameInfo* d_frames, int n_frames, const double* pos, const int32_t* species,
                            int64_t n_atoms, int n_species, int n_cells, float rc_radial, float rc_angular,
                            const NeighborWork& w, const NeighborLists& nl, int32_t* d_flags, hipStream_t s) {
    if (n_atoms == 0 || n_frames == 0) return hipSuccess;
    k_frame_of<<<n_frames, kBlock, 0, s>>>(d_frames, w.frame_of);
    if (n_cells > 0) k_fill_i32<<<blocks_for(n_cells, kBlock), kBlock, 0, s>>>(w.cell_count, n_cells, 0);
    k_bin<<<blocks_for(n_atoms, kBlock), kBlock, 0, s>>>(d_frames, w.frame_of, pos, species, n_atoms, n_species,
                                                        w.cell_of, w.cell_count, d_flags);
    if (n_cells > 0) {
        k_scan<<<1, 1024, 0, s>>>(w.cell_count, w.cell_start, w.cell_fill, n_cells);
        k_scatter<<<blocks_for(n_atoms, kBlock), kBlock, 0, s>>>(w.cell_of, w.cell_start, w.cell_fill, w.cell_atoms,
                                                                n_atoms);
        k_sort_cells<<<blocks_for(n_cells, kBlock), kBlock, 0, s>>>(w.cell_start, w.cell_atoms, n_cells);
    }
    k_neighbors<<<blocks_for(n_atoms, kBlock), kBlock, 0, s>>>(d_frames, w.frame_of, pos, species, w.cell_of,
                                                              w.cell_start, w.cell_atoms, n_atoms, rc_radial,
                                                              rc_angular, nl, d_flags);
    return hipGetLastError();
}

}  // namespace tnep
