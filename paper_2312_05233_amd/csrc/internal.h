// Internal interfaces between the C-ABI layer and the gfx950 kernels of libtnep.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tnep {

// Per-frame geometry of one launch batch (built on the host).
// Trajectory reuse of neighbour candidates (TNEP_OPT_TRAJECTORY_WINDOW): a
// reference frame (role 1) searches its cells out to r_c + skin and keeps,
// per atom and neighbour species, the frame-local indices of the candidates;
// the following frames of its window (role 2: same atom count, species and
// box) test only those candidates against the exact r < r_c.  Every follower
// atom checks that it moved at most skin / 2 from the reference (minimum
// image) and kept its species, else the call is redone with plain searches.
enum FrameRole { kRolePlain = 0, kRoleReference = 1, kRoleFollower = 2 };

// Orthorhombic cell grids: cells of edge >= r / kCellReachXY along x, y and
// >= r / kCellReachZ along z for the search radius r, so every neighbour lies
// within that many cells of the atom's own cell along each axis.
constexpr int kCellReachXY = 2;
constexpr int kCellReachZ = 2;

// Radial basis terms (K_R + 1) of every compiled descriptor shape: the
// neighbour search accumulates the radial descriptor sums for this size.
constexpr int kRadialTerms = 9;

struct FrameInfo {
    int64_t atom_begin;  // first atom, batch-local index
    int32_t n_atoms;
    int32_t mode;        // 0: all-pairs search inside the frame, 1: cell list
    int32_t nc[3];       // cells per axis (mode 1)
    int32_t cell_base;   // first cell of this frame in the batch's cell arrays
    int32_t per[3];      // periodic axes
    int32_t role;        // FrameRole
    double L[3];         // box edges (periodic axes)
    double Linv[3];      // 1 / L (periodic axes), else 0
    int64_t ref_begin;   // follower: atom_begin of its reference frame
    int64_t cl_base;     // reference / follower: first candidate list of the reference's atoms
    // tric = 1: triclinic cell (all axes periodic), its lattice in the batch's
    // FrameTric array at the frame's index; 0: orthorhombic or non-periodic.
    int32_t tric;
    int32_t pad_;
    // Triclinic bins: unit (a power of two, fractional units) of the fixed-point
    // offsets from the bin origin in the candidate records.
    double q_unit;
};

// Lattice of a triclinic frame, kept apart from FrameInfo so that the frame
// records of other frames stay small (they are copied to the device for every
// launch batch): lattice vectors as the rows of H, fractional coordinates
// s = r Hinv, cells binned in s, widths w[k] between opposite faces (>= 2 r_c).
struct FrameTric {
    double H[9], Hinv[9], w[3];
};

// Device-resident FP32 model parameters.
struct DevModel {
    const float* c_radial;   // [T][T][NR][KR]
    const float* c_angular;  // [T][T][NA][KA]
    const float* c_angular_d;  // [T][T][NA][KA]: Chebyshev coefficients of d/dx sum_k c_nk T_k(x)
                               // (last one 0), so sum_k c_nk T_k'(x) = sum_k c_angular_d[n][k] T_k(x)
    const float* scaler;     // [D]
    const float* w0[2];      // [H][D]
    const float* b0[2];      // [H]
    const float* w1[2];      // [H]
    const float* w0t[2];     // [D][H] transposed copy (backward GEMM operand)
    // Matrix-core operand fragments, one element (or 8 bf16) per lane:
    //   f32_fwd[h]  [Hp/16][Dp4/4][64]   W0[16 nt + l%16][4 ks + l/16]
    //   f32_bwd     [Dp16/16][Hp/4][64]  W0[4 ns + l/16][16 kt + l%16]   (tensor head)
    //   bf_fwd_*[h] [Hp/16][Dp32/32][64] W0[16 nt + l%16][32 kc + 8 (l/16) + j], j < 8
    //   bf_bwd_*    [Dp16/16][Hp/32][64] W0[32 nc + 8 (l/16) + j][16 kt + l%16]
    // with Hp = H rounded up to 32, hi/lo = the bf16 rounding and its remainder.
    const float* f32_fwd[2];
    const float* f32_bwd;
    const uint4* bf_fwd_hi[2];
    const uint4* bf_fwd_lo[2];
    const uint4* bf_bwd_hi;
    const uint4* bf_bwd_lo;
    float b1[2];
    // per-species networks: head h of centre species t at w0[h] + t * sp_w0,
    // b0[h] / w1[h] + t * sp_h, output bias b1s[h][t]; sp_w0 = sp_h = 0 and
    // b1s = null for one shared network
    int32_t sp_w0, sp_h;
    const float* b1s[2];
    float rc_radial, rc_angular;
    int32_t n_species, n_hidden;
};

// Shape key of a compiled evaluation kernel.
struct Shape {
    int nr, na, kr, ka, four_body, kind, five_body;
};

// Neighbour lists of a batch.
// Atoms are processed in 64-atom tiles of one species: tile slot p = 64 * tile
// + lane holds atom perm[p] (-1 = padding).  The neighbours of that atom are
// stored by neighbour species t in two segments: rows [segA[t], segA[t] +
// capA[t]) for r < rc_angular (used by the radial and the angular terms) and
// rows [segR[t], segR[t] + capR[t]) for rc_angular <= r < rc_radial (radial
// terms only).  Entry (row r) of slot p is the float4 (dx, dy, dz, 0) with
// r_ij = r_j - r_i (x, y, z; w holds the tile slot of j as int bits),
// stored at entries[((tile * slots/4 + r/4) * 64 + lane) * 4
// + r % 4]: four consecutive rows of one lane are 64 contiguous bytes.
// Per-species segment tables live in device memory (meta) so that kernels
// index them with scalar loads.
// The batch's actual sizes are read from meta too, so that one captured graph
// (launched with grids sized for a capacity bucket) serves every batch that
// fits the bucket; blocks beyond the actual sizes return at once.
enum Meta {
    kMetaTileBase = 0,
    kMetaSegA = 16,
    kMetaSegR = 24,
    kMetaCapA = 32,
    kMetaCapR = 40,
    kMetaNAtoms = 48,
    kMetaNFrames = 49,
    kMetaNCells = 50,
    kMetaAtomBase = 51,  // index of the batch's first atom in the call (saturated at INT32_MAX)
    kMetaInts = 56
};
// Device header of a launch batch: the kMetaInts meta ints, then the batch's
// FrameInfo records from this byte offset on (one host-to-device copy fills
// both, from kMetaSegA on).
constexpr size_t kHeaderFrames = sizeof(int32_t) * kMetaInts;

struct NeighborLists {
    float4* entries;
    int32_t* counts;      // [2T][n_pad]: row 2t angular count, 2t+1 radial-only count
    const int32_t* perm;  // [n_pad]
    const int32_t* meta;  // [kMetaInts]: tile_base[T + 1] (first tile of species t, tiles in use at
                          // T), segA[t], segR[t], capA[t], capR[t]
    int64_t n_pad;        // tile slots (multiple of 64)
    int32_t T;
    int32_t slots;        // rows per slot (multiple of 4)
};

// Error / overflow flags written by the kernels (device int32[32]).
enum Flag { kFlagError = 0, kFlagBadAtom = 1, kFlagCapAng = 8, kFlagCapRad = 16, kFlagCapCand = 24, kFlagReuse = 25 };
enum ErrBits { kErrSpecies = 1, kErrNonFinite = 2, kErrOverlap = 4 };

// ---- neighbour search (kernels_neighbors.hip) ----
// Candidate lists of reference-frame atoms: list (cl_base + i) * T + t holds
// up to cap frame-local indices of species-t candidates of atom i.
// Candidate lists of trajectory reuse.  A reference frame's atom of species
// t_i with rank k in the frame's species-t_i slot range has the list index
// R = cl_base + t_i * A64 + k (A64: the frame's atom count rounded up to 64;
// cl_base: the frame's first index, a multiple of 64); a follower frame's atom
// has its reference atom's R.  Candidate q of neighbour species t of R is at
// idx[(((R / 64) * T + t) * cap / 4 + q / 4) * 256 + (R % 64) * 4 + q % 4], so
// four candidates are one 16-byte word and the lists of 64 consecutive R lie
// side by side; count at [((R / 64) * T + t) * 64 + R % 64].  A candidate is
// packed as (rank of the neighbour in its frame's species-t range) << 9 |
// (ox + 3) << 6 | (oy + 3) << 3 | (oz + 3), o the offset of the neighbour's cell
// from the atom's cell (|o| <= 2 on the grid for r_c + skin).
struct CandLists {
    int32_t* idx;      // [lists / 64][T][cap / 4][64][4]
    int32_t* count;    // [lists / 64][T][64]
    int32_t cap;       // multiple of 4
    float rc_search;   // r_c + skin
    float half_skin2;  // (skin / 2)^2
};

struct NeighborWork {
    int32_t* frame_of;      // [n_atoms]
    int32_t* key_of;        // [n_atoms] bucket (cell * T + species)
    int32_t* bucket_count;  // [n_buckets]
    int32_t* bucket_start;  // [n_buckets + 1]
    int32_t* bucket_fill;   // [n_buckets]
    int32_t* bucket_atoms;  // [n_atoms]
    double4* bucket_pos;    // [n_pad] FP64 positions by tile slot (frames without an orthorhombic cell grid)
    int4* cell_rec;         // [n_pad] cell grids: (q_0, q_1, q_2, cell index along axis 2) by tile slot
    int32_t* perm_start;    // [n_buckets]
    int32_t* perm;          // [n_pad]
    int32_t* meta;          // [kMetaInts], tile_base part written on the device
    int32_t* chunk;         // [2 * 9 * n_chunks] scan partials (n_chunks = ceil(n_cells / 1024))
    int32_t* slot_of;       // [n_atoms] tile slot of every atom
};

// Sizes: the actual atoms, frames and cells of the batch are in meta
// (kMetaNAtoms, kMetaNFrames, kMetaNCells); cap_* are the launch capacities
// (>= the actual sizes) that size the grids.
// references / followers: the batch has frames of role 1 / role 2 (each
// role has a pass over the slots of its own; followers run after the
// reference frames' lists are complete).
// triclinic: the batch has triclinic frames (a pass of their own).
// pair_search: frames without a cell grid are searched with kPairLanes lanes
// per atom (the same rows in the same order); pair_radial: that search also
// forms their radial sums, bit for bit as the one-lane search does (else they
// are not written: the pair-parallel evaluation layout forms them itself).
// plain_grid: the batch has plain (not trajectory, not triclinic) frames on an
// orthorhombic cell grid.
hipError_t launch_neighbors(const FrameInfo* d_frames, const FrameTric* d_tric, int cap_frames, const double* pos,
                            const int32_t* species,
                            int64_t cap_atoms, int cap_cells, float rc_radial, float rc_angular, const NeighborWork& w,
                            const NeighborLists& nl, const CandLists& cl, bool references, bool followers,
                            bool triclinic, bool pair_search, bool pair_radial, bool plain_grid, int32_t* d_flags,
                            int neigh_block, float* rad_sums, hipStream_t s);

// ---- evaluation (kernels_eval.hip) ----
struct EvalLaunch {
    int mlp_mode;         // TNEP_MLP_*
    int atoms_per_block;  // work-group size of the FP32-VALU evaluation kernel: 64, 128, 256
    int neigh_block;      // work-group size of the neighbour kernel: 64, 128, 256
    int pair_parallel;    // 1: kPairLanes lanes per atom in the evaluation of the tensor models
};

// Lanes per atom of the pair-parallel evaluation layout (one 16-lane DPP row).
constexpr int kPairLanes = 16;
// Launch batches of at most this many atoms search frames without a cell grid
// with kPairLanes lanes per atom in every layout.  Below it the one-lane search
// takes as long as one atom's walk over its frame; above it (vacuum molecules of
// 20-80 atoms and 192-atom boxes alike: crossing near 35k atoms) the sixteen
// times as many lanes cost more than they save.
constexpr int64_t kPairSearchAtoms = 32768;

// Potential-energy models: the evaluation kernel leaves, per atom a in tile
// slot p, a record of rec_stride floats at rec + p * rec_stride (slots keep
// atoms of one cell together, so the records of a lane's neighbours are close):
//   [t * KRP + k]   sum_n dU_a/dq^R_n c^R_{t_a t}[n][k]   (t < T, KRP = KR rounded up to 4)
//   [T * KRP + d]   sum_j dU_a/dr_aj, component d < 3
// and, for every entry of an angular segment (r_aj < r_c^A), the pair force
// dU_a/dr_aj at the entry's place in `pair` (same layout as the neighbour
// entries) and the neighbour's slot at the same index of `slot` (four rows of
// a lane in one 16-byte word, so that a lookup reads four rows at once).  From
// these the second kernel forms, for every pair (k, j), the term that U_j
// contributes to the force on k.
struct PesOut {
    float* rec;
    int32_t rec_stride;
    float4* pair;
    int32_t* slot;
};
inline int pes_rec_stride(const Shape& s, int T) { return T * ((s.kr + 3) / 4 * 4) + 4; }

// Per-atom records (FP64, batch atom order) of one model: dipole [n][3],
// polarizability [n][9], potential energy [n][10] = (U_i, W_i row-major).
bool eval_shape_supported(const Shape& s);
// Whether the matrix-core hidden layer is compiled for this shape (else the
// FP32 vector path runs whatever TNEP_OPT_MLP says).
bool eval_matrix_supported(const Shape& s, int n_hidden);
// Radial descriptor sums: per slot, the sums over the neighbours of species t
// of f_k(r_ij) (T * kRadialTerms floats at v[(t * kRadialTerms + k) * n_pad +
// p]), which depend only on the lists, r_c^R and KR, not on a model's
// coefficients; the neighbour search accumulates them.  mode 0: the
// evaluation forms them itself; 2: v holds them, and the FP32 vector kernel of
// a model with KR = kRadialTerms loads them (the matrix-core kernels, which
// also serve other basis sizes, form them).
struct RadSums {
    float* v;
    int32_t mode;
};
hipError_t launch_eval(const Shape& shape, const DevModel& m, const NeighborLists& nl, double* per_atom,
                       const PesOut& pes, const RadSums& rs, const EvalLaunch& cfg, hipStream_t s);

// Potential-energy models, after launch_eval over the same lists: forces[a]
// (FP64, NULL to skip) = sum_j dU_a/dr_aj - sum_j dU_j/dr_ja, summed in a fixed
// order, and energies[a] = U_a (column 0 of the per-atom records, NULL to skip).
hipError_t launch_pes_forces(const Shape& shape, const DevModel& m, const NeighborLists& nl, const PesOut& pes,
                             const double* per_atom, double* forces, double* energies, int block, hipStream_t s);

// Charged molecules: mu[f] += charges[f] * unit * (mass-weighted mean of the
// frame's positions); frames without atoms unchanged.  All device pointers.
hipError_t launch_com_shift(const int64_t* offsets, int n_frames, const double* pos, const int32_t* species,
                            const double* masses, const double* charges, double unit, double* mu, hipStream_t s);

// Add the batch's atom count and neighbour-pair counts to counters[0..2].
hipError_t launch_count_pairs(const NeighborLists& nl, unsigned long long* counters, hipStream_t s);

// Per-frame sums of per-atom records (nt <= 10 values) in a fixed order:
// values 0..na-1 go to out_a[f][na], values na..nt-1 to out_b[f][nt - na]
// (out_b may be NULL).  Frames beyond meta[kMetaNFrames] are skipped
// (cap_frames sizes the grid).  part: scratch of kReduceChunks * 10 doubles
// per frame.  Frames of at most kSmallFrame atoms are summed by one wavefront
// each, larger ones in kReduceChunks chunks; small / large: whether the batch
// holds frames of that class (the other kernel is not launched).
constexpr int kReduceChunks = 4;
constexpr int kSmallFrame = 256;
hipError_t launch_frame_reduce(const FrameInfo* d_frames, int cap_frames, const int32_t* meta, const double* per_atom,
                               int nt, int na, double* part, double* out_a, double* out_b, bool small, bool large,
                               hipStream_t s);

// ---- spectra (kernels_spectrum.hip) ----
struct SpectrumPlan {
    int kind, window, flags;
    int n_series;
    int64_t n_steps, max_lag, fft_len;
    double dt_fs;
    double n_hat[3], e_hat[3];
    double laser_cm1;  // > 0: Raman (w_in - w)^4 factor
};
size_t spectrum_workspace_bytes(const SpectrumPlan& p);
hipError_t launch_spectrum(const SpectrumPlan& p, const double* d_series, double* d_freq, double* d_intensity,
                           double* d_acf, void* d_work, hipStream_t s);

// Orientation map: h_weights [n_orient][45] host array (v_P v_Q, doubled off
// the diagonal, v = n (x) e flattened), intensity [n_orient][M+1].
size_t raman_map_workspace_bytes(const SpectrumPlan& p, int n_orient);
hipError_t launch_raman_map(const SpectrumPlan& p, const double* d_series, const double* h_weights, int n_orient,
                            double* d_freq, double* d_intensity, void* d_work, hipStream_t s);

// Streaming correlation accumulators (device pointers; host-side sizes).
struct StreamState {
    int kind, nsig, nch;
    int64_t M;
    double n_hat[3], e_hat[3];
    const int32_t *chx, *chy, *chsym;  // [nch] channel signal pairs, symmetric flag
    const double* chw;                 // [nch] channel weights (kinds 0-3)
    double* carry;                     // [nsig][carry_cap] last samples of the run
    double* carry_next;                // same size: written by a push, then swapped
    int64_t carry_cap, carry_len;      // carry_cap = M - 1 (at least 1)
    double* head;                      // [nsig][M] first samples of the run
    double* totals;                    // [nsig] sums over the run
    double* S;                         // [nch][M] pair sums of the run
    double* run_sum;                   // [nch][M] sum over finished runs of C(tau)
    int64_t run_len;                   // samples in the current run
    int64_t n_runs;                    // finished runs
    const void* blk_tw;                // [kBlkN / 2] twiddles of the blocked path (max lag <= kBlkMaxLag)
};
// Blocked streaming path: a chunk is split into blocks of kBlkN - (M - 1) new
// samples whose kBlkN-point transforms run inside one work-group (LDS), at most
// kBlkRound blocks per launch round; used when M <= kBlkMaxLag.
constexpr int kBlkN = 4096;
constexpr int64_t kBlkMaxLag = kBlkN / 2;
constexpr int kBlkRound = 32;
size_t stream_blk_workspace_bytes(int nsig, int nch, int64_t M, int64_t n);
size_t stream_blk_twiddle_bytes();
hipError_t launch_stream_twiddles(void* tw, hipStream_t s);
hipError_t launch_stream_push_blocked(const StreamState& st, const double* d_chunk, int64_t n, void* d_work,
                                      hipStream_t s);
size_t stream_push_workspace_bytes(int nsig, int nch, int64_t P);
hipError_t launch_stream_push(const StreamState& st, const double* d_chunk, int64_t n, int64_t P, void* d_work,
                              hipStream_t s);
hipError_t launch_stream_end_run(const StreamState& st, int subtract, hipStream_t s);
hipError_t launch_stream_spectrum(const StreamState& st, double dt_fs, int window, int omega2, double laser_cm1,
                                  double* d_tab, double* d_acf, double* d_freq, double* d_intensity, hipStream_t s);
hipError_t launch_stream_map(const StreamState& st, double dt_fs, int window, double laser_cm1, const double* d_w,
                             int n_orient, double* d_tab, double* d_acf, double* d_L, double* d_freq,
                             double* d_intensity, hipStream_t s);
hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t s);

}  // namespace tnep
