/*
 * tnep.h -- C ABI of libtnep: TNEP tensor evaluation and spectra on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: tensorial neuroevolution potential, arXiv:2312.05233.
 *   - tnep_eval_dipole          : Sec. 2.2, Eq. (mu)
 *       mu = - sum_i sum_{j != i} r_ij^2 dU_i/dr_ij,   r_ij = r_j - r_i
 *   - tnep_eval_polarizability  : Sec. 2.3, Eq. (polarizability-model)
 *       alpha^{uv} = sum_i U_i delta^{uv} - sum_i sum_{j != i} r_ij^u dU_i/dr_ij^v
 *     (the same form serves the susceptibility chi)
 *   - tnep_spectrum             : Secs. 2.6-2.7, IR lineshape M(w) with the
 *     classical w^2 prefactor (Eq. ir-intensity) and the Raman lineshape
 *     L(w) (Eq. raman-lineshape) with its isotropic / anisotropic split
 *     (Eq. raman-lineshape-isotropic-anisotropic) or a polarisation
 *     projection n^T alpha e (Eq. raman-cross-section).
 * U_i is the output of a single-hidden-layer tanh network acting on the NEP
 * descriptor of atom i (Sec. 2.1, Eq. site-energy); the descriptor is the
 * NEP radial/angular form with Chebyshev radial functions, a cosine cutoff,
 * angular invariants l = 1..4, the l = 2 four-body term and optionally the
 * l = 1 five-body term.
 *
 * Conventions
 *   - Every call returns TNEP_OK (0) or a negative error code; nothing is
 *     thrown across the ABI.  tnep_last_error() gives a message.
 *   - Ownership: the caller owns every input and output buffer; calls borrow
 *     them for their duration (tnep_submit: until tnep_wait returns for that
 *     ticket).  Contexts, models and servers are library-owned and are freed
 *     explicitly.
 *   - Memory location: tnep_frames.location says whether the pointers in
 *     that struct AND the output pointers of the call are host memory
 *     (TNEP_HOST) or device memory of the context's GPU (TNEP_DEVICE).
 *     TNEP_DEVICE_META_HOST: positions, species and the outputs in device
 *     memory, atom_offsets, cells and pbc in host memory, for callers that keep
 *     the frame layout on the host (the call then reads no metadata back from
 *     the device and does not synchronize with the legacy default stream before
 *     it starts: order the work that writes the positions before the call on the
 *     context's stream).  Accepted by tnep_eval_dipole, tnep_eval_polarizability,
 *     tnep_eval_dipole_polarizability and tnep_eval_pes; TNEP_E_INVALID elsewhere.
 *   - Threading: a context is used by one host thread at a time, except the
 *     tnep_submit / tnep_wait pair, which is thread-safe.
 *   - Units: positions in Angstrom; tensors are returned in the model's own
 *     units (no conversion).
 *   - Synchronous calls return after their results are complete.
 */
#ifndef TNEP_H
#define TNEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define TNEP_OK 0
#define TNEP_E_INVALID (-1)        /* bad argument, null pointer, bad size      */
#define TNEP_E_SPECIES (-2)        /* species index outside [0, n_species)     */
#define TNEP_E_BOX (-3)            /* periodic box shorter than 2 r_c^R, or a  */
                                   /* non-orthorhombic cell                    */
#define TNEP_E_OVERLAP (-4)        /* two atoms closer than 1e-4 Angstrom      */
#define TNEP_E_NONFINITE (-5)      /* NaN / Inf in positions or cell           */
#define TNEP_E_BUDGET (-6)         /* request exceeds the context's budget     */
#define TNEP_E_MODEL (-7)          /* model shape not supported / bad model    */
#define TNEP_E_HIP (-8)            /* HIP runtime failure                      */
#define TNEP_E_NEIGH_OVERFLOW (-9) /* neighbour capacity exceeded (internal)   */
#define TNEP_E_CANCELLED (-10)     /* request cancelled or server stopped      */

/* ---- enums ------------------------------------------------------------- */
#define TNEP_HOST 0
#define TNEP_DEVICE 1
#define TNEP_DEVICE_META_HOST 2   /* tnep_frames only: data on the device, layout on the host */

#define TNEP_KIND_DIPOLE 1         /* rank-1: one tensor head               */
#define TNEP_KIND_POLARIZABILITY 2 /* rank-2: tensor head + scalar head     */
#define TNEP_KIND_PES 3            /* potential-energy surface (Sec. 2.1): one head, the site
                                      energy U_i; hidden layer always FP32 vector ALU */

/* precision of the hidden layer (option TNEP_OPT_MLP) */
#define TNEP_MLP_FP32_VALU 0  /* FP32 vector ALU                           */
#define TNEP_MLP_FP32_MFMA 1  /* FP32 matrix cores                          */
#define TNEP_MLP_BF16_MFMA 2  /* BF16 inputs, FP32 accumulation             */
#define TNEP_MLP_BF16X3_MFMA 3 /* split-BF16 (hi/lo, 3 products), FP32 acc */

/* options for tnep_set_option */
#define TNEP_OPT_MLP 1            /* one of TNEP_MLP_*                          */
#define TNEP_OPT_ATOMS_PER_BLOCK 2 /* work-group size of the fused kernel: 64, 128, 256 */
#define TNEP_OPT_AUTOTUNE 3       /* 1 = time candidate work-group and batch sizes on the first
                                     call of each (model shape, frame size class, location) and
                                     keep the fastest; results do not depend on the choice  */
#define TNEP_OPT_DETERMINISTIC 4  /* 1 (default) = fixed reduction order        */
#define TNEP_OPT_MAX_BATCH_ATOMS 5 /* atoms per launch batch (default 2^20)       */
#define TNEP_OPT_TIMING 6         /* 1 = time every launch with HIP events and count pairs */
#define TNEP_OPT_NEIGH_BLOCK 7    /* work-group size of the neighbour kernel: 64, 128, 256 */
#define TNEP_OPT_GRAPHS 8         /* 1 = (timing off) capture each launch batch's kernels once
                                     per signature (models, neighbour capacities, launch sizes,
                                     power-of-two bucket of atoms, frames and cells; for
                                     TNEP_DEVICE frames also the device addresses of the call's
                                     inputs and outputs, so a call on other buffers captures a
                                     graph of its own) as a HIP graph and replay it; results are
                                     bitwise those of the plain launches.  Needs a non-null
                                     stream.  A call on a context must not overlap another
                                     call on the same context (as for every entry point). */
#define TNEP_OPT_TRAJECTORY_WINDOW 9 /* W >= 2: consecutive frames of a call with equal atom counts
                                     and boxes (all axes periodic, edges >= 2 (r_c + skin)) are
                                     taken as frames of one trajectory: in each window of W
                                     frames the first searches its cells out to r_c + skin and
                                     the others test only those candidates (exact r < r_c
                                     test).  If any atom moved more than skin/2 from the
                                     window's first frame or changed species, the call is
                                     redone with plain searches.  Results agree with plain
                                     searches up to FP32 summation order (the neighbour order
                                     differs).  0 (default) = off */
#define TNEP_OPT_SKIN_MA 10       /* skin for TNEP_OPT_TRAJECTORY_WINDOW in 1e-3 Angstrom
                                     (1..5000, default 1000) */
#define TNEP_OPT_PAIR_PARALLEL 11 /* 1 = evaluation of the dipole and polarizability models with
                                     16 lanes per atom (each takes every 16th neighbour row and
                                     hidden neuron; the lanes' shares are added by a fixed tree)
                                     and the FP32 vector hidden layer: for calls of few atoms,
                                     whose time one lane per atom sets by its serial work per
                                     atom; large calls take more device time per atom.  Results
                                     agree with the default layout to FP32 summation order, and
                                     within the layout they do not depend on batching.
                                     Potential-energy models keep the default layout.
                                     0 (default) = one lane per atom */

/* kernel classes for tnep_ctx_kernel_time */
#define TNEP_KERNEL_NEIGHBORS 0
#define TNEP_KERNEL_EVAL_DIPOLE 1
#define TNEP_KERNEL_EVAL_POLARIZABILITY 2
#define TNEP_KERNEL_FRAME_REDUCE 3
#define TNEP_KERNEL_SPECTRUM 4
#define TNEP_KERNEL_EVAL_PES 5
#define TNEP_KERNEL_PES_FORCES 6

/* ---- opaque handles ---------------------------------------------------- */
typedef struct tnep_ctx tnep_ctx;
typedef struct tnep_model tnep_model;

/* ---- model ------------------------------------------------------------- */
/* Parameters of one TNEP model, FP64, host memory (copied at creation).
 * Descriptor length D = (n_max_radial+1) + l_max*(n_max_angular+1)
 *                       + (four_body ? n_max_angular+1 : 0) + (five_body ? n_max_angular+1 : 0),
 * ordered [q^R_0..q^R_nR | l=1: q_{0,1}..q_{nA,1} | ... | l=l_max | q4_0..q4_nA | q5_0..q5_nA],
 * q5_n = (sum_m A_n1m^2)^2 (the degree-4 invariant of the l = 1 sums).
 * Network (per head): U = sum_m w1[m] tanh(sum_n w0[m][n] q_scaler[n] q[n] - b0[m]) - b1. */
typedef struct {
    int32_t kind;          /* TNEP_KIND_DIPOLE, TNEP_KIND_POLARIZABILITY or TNEP_KIND_PES */
    int32_t n_species;     /* T                                                      */
    double rc_radial;      /* radial cutoff r_c^R, Angstrom                          */
    double rc_angular;     /* angular cutoff r_c^A <= r_c^R                          */
    int32_t n_max_radial;  /* nR: nR+1 radial functions                              */
    int32_t n_max_angular; /* nA: nA+1 angular radial functions                      */
    int32_t basis_radial;  /* KR: KR+1 Chebyshev terms                               */
    int32_t basis_angular; /* KA                                                     */
    int32_t l_max;         /* must be 4                                              */
    int32_t four_body;     /* 0 / 1: l = 2 four-body invariant                       */
    int32_t n_hidden;      /* H, 1..128                                              */
    const double* c_radial;  /* [T][T][nR+1][KR+1], block (t_i, t_j)                 */
    const double* c_angular; /* [T][T][nA+1][KA+1]                                   */
    const double* q_scaler;  /* [D]                                                  */
    const double* w0[2];     /* head 0 tensor, head 1 scalar (polarizability): [H][D] */
    const double* b0[2];     /* [H]                                                  */
    const double* w1[2];     /* [H]                                                  */
    double b1[2];
    int32_t per_species;     /* 1: one network per centre species: w0 [T][H][D], b0 and w1
                                [T][H], output biases b1_species[head] [T] (b1 unused); the
                                hidden layer then always runs on the FP32 vector ALU      */
    const double* b1_species[2];
    int32_t five_body;       /* 0 / 1: the l = 1 five-body invariants q5 (after q4; compiled for
                                nR = nA = 4, KR = KA = 8 with the four-body term)            */
} tnep_model_desc;

/* ---- frames ------------------------------------------------------------ */
/* A batch of ragged frames, CSR by atom.  Periodic axes use the minimum-image
 * convention and need an orthorhombic cell with edge >= 2 r_c^R. */
typedef struct {
    int32_t n_frames;
    const int64_t* atom_offsets; /* [n_frames+1], offsets[0] = 0, non-decreasing   */
    const double* positions;     /* [total_atoms][3], Angstrom                     */
    const int32_t* species;      /* [total_atoms], 0..n_species-1                  */
    const double* cells;         /* [n_frames][9] row-major lattice vectors or NULL */
    const uint8_t* pbc;          /* [n_frames][3] periodic flags or NULL (vacuum)   */
    int32_t location;            /* TNEP_HOST, TNEP_DEVICE or TNEP_DEVICE_META_HOST */
} tnep_frames;

/* ---- context ----------------------------------------------------------- */
/* Create a context on `device`.  hip_stream: a hipStream_t to run on, or NULL
 * for a context-owned stream.  mem_budget_bytes: device-memory ceiling for the
 * context's work buffers (0 = 32 GiB).  Returns TNEP_E_HIP if the device is
 * unusable. */
int tnep_ctx_create(int device, void* hip_stream, uint64_t mem_budget_bytes, tnep_ctx** out);
void tnep_ctx_destroy(tnep_ctx* ctx);
/* Message of the last failing call on ctx (library-owned, valid until the next
 * call on ctx).  ctx may be NULL for errors of tnep_ctx_create. */
const char* tnep_last_error(const tnep_ctx* ctx);
/* Set an integer option (TNEP_OPT_*).  TNEP_E_INVALID for unknown keys/values. */
int tnep_set_option(tnep_ctx* ctx, int32_t key, int64_t value);
/* Text of the last autotuning decision (candidates and their times), library-owned,
 * empty if none was made. */
const char* tnep_autotune_report(const tnep_ctx* ctx);
/* Device bytes currently held by the context's work buffers. */
uint64_t tnep_ctx_memory_in_use(const tnep_ctx* ctx);
/* With TNEP_OPT_TIMING on: summed device time (ms, HIP events on the context's
 * stream, one pair per launch) and number of launches of one kernel class
 * (TNEP_KERNEL_*) since the last reset; atoms and neighbour pairs processed by
 * the evaluation kernels (radial pairs r < rc_radial, angular pairs r < rc_angular).
 * Any output pointer may be NULL. */
int tnep_ctx_kernel_time(const tnep_ctx* ctx, int32_t kernel_class, double* total_ms, uint64_t* launches);
int tnep_ctx_pair_counts(const tnep_ctx* ctx, uint64_t* atoms, uint64_t* radial_pairs, uint64_t* angular_pairs);
int tnep_ctx_reset_timing(tnep_ctx* ctx);
/* With TNEP_OPT_GRAPHS on: graphs captured and graph launches since the
 * context was created (with a running server: its slots' counts added).
 * Either pointer may be NULL. */
int tnep_ctx_graph_counts(const tnep_ctx* ctx, uint64_t* captures, uint64_t* launches);
/* Calls redone with plain searches because a trajectory window's guard
 * failed (TNEP_OPT_TRAJECTORY_WINDOW). */
int tnep_ctx_reuse_fallbacks(const tnep_ctx* ctx, uint64_t* count);

/* ---- model ------------------------------------------------------------- */
/* Copy a model to the device (resident until tnep_model_free). TNEP_E_MODEL if
 * the shape is unsupported (l_max != 4, rc_angular > rc_radial, sizes out of
 * range). */
int tnep_model_create(tnep_ctx* ctx, const tnep_model_desc* desc, tnep_model** out);
/* Free a model (waits for the device first); valid before or after its
 * context is destroyed. */
void tnep_model_free(tnep_model* model);
/* Model files: a plain-text form of tnep_model_desc (Sec. 2.1: the descriptor
 * hyperparameters and coefficients, the descriptor scaler and the networks),
 * FP64 values written with 17 significant digits (exact round trip).  Layout,
 * one keyword per item, '#' comments allowed:
 *   tnep_model 1 / kind dipole|polarizability|pes / n_species T / rc rR rA /
 *   n_max nR nA / basis KR KA / l_max 4 / four_body 0|1 / five_body 0|1 /
 *   n_hidden H / per_species 0|1 / c_radial ... / c_angular ... / q_scaler ... /
 *   head 0 w0 ... b0 ... w1 ... b1 ... [head 1 ... for polarizability] / end
 * with each array's values in the order of tnep_model_desc.
 * tnep_model_save: writes desc (host arrays) to path; no context or GPU needed;
 *   TNEP_E_INVALID if the file cannot be written, TNEP_E_MODEL for a bad
 *   desc; the message is tnep_last_error(NULL).
 * tnep_model_load: parses path and creates the model as tnep_model_create
 *   does; TNEP_E_INVALID if the file cannot be read, TNEP_E_MODEL (with the
 *   line number in tnep_last_error) if it is malformed or the shape is not
 *   supported. */
int tnep_model_save(const tnep_model_desc* desc, const char* path);
int tnep_model_load(tnep_ctx* ctx, const char* path, tnep_model** out);
/* Kind (TNEP_KIND_*), species count and descriptor length D of a model;
 * any output pointer may be NULL.  TNEP_E_INVALID for a NULL model. */
int tnep_model_info(const tnep_model* model, int32_t* kind, int32_t* n_species, int32_t* descriptor_length);

/* ---- evaluation -------------------------------------------------------- */
/* Dipole of every frame (Sec. 2.2, Eq. mu).  mu_out: [n_frames][3] FP64.
 * per_atom: NULL or [total_atoms][3] FP64, the atom terms
 * -sum_j r_ij^2 dU_i/dr_ij whose frame sums are mu_out.  The model must be
 * a dipole model.  Frame sums are FP64 in a fixed order: results do not
 * depend on how frames are batched. */
int tnep_eval_dipole(tnep_ctx* ctx, const tnep_model* model, const tnep_frames* frames,
                     double* mu_out, double* per_atom);

/* Polarizability / susceptibility of every frame (Sec. 2.3, Eq.
 * polarizability-model).  alpha_out: [n_frames][9] FP64 row-major (u, v).
 * per_atom: NULL or [total_atoms][9] FP64 (U^s_i delta - sum_j r_ij (x) dU^t_i/dr_ij).
 * The model must be a polarizability model (scalar head for the delta term,
 * tensor head for the virial term). */
int tnep_eval_polarizability(tnep_ctx* ctx, const tnep_model* model, const tnep_frames* frames,
                             double* alpha_out, double* per_atom);

/* Dipole with one model and polarizability with another over the same frames
 * (Secs. 2.2-2.3), sharing one neighbour search when the two models have the
 * same cutoffs.  mu_out [n_frames][3], alpha_out [n_frames][9], FP64. */
int tnep_eval_dipole_polarizability(tnep_ctx* ctx, const tnep_model* dipole_model,
                                    const tnep_model* polarizability_model, const tnep_frames* frames,
                                    double* mu_out, double* alpha_out);

/* Dipole of charged molecules (Sec. 3, charged molecules): a model trained on
 * mu_r, the permanent dipole relative to the centre of mass, gives the
 * absolute dipole mu = mu_r + Q e r_COM, r_COM = sum_i m_i r_i / sum_i m_i.
 *   charges [n_frames]: net charge of each frame in units of e (location of
 *     the frames); species_masses [n_species]: host; length_unit: the model's
 *     dipole unit per (e * Angstrom), e.g. 1/0.529177210903 for e*bohr;
 *   mu_out, per_atom as for tnep_eval_dipole (per_atom holds the mu_r terms).
 * A charged frame with a periodic axis is TNEP_E_BOX (its centre of mass is
 * not defined); frames without atoms get no shift. */
int tnep_eval_dipole_charged(tnep_ctx* ctx, const tnep_model* model, const tnep_frames* frames,
                             const double* charges, const double* species_masses, double length_unit,
                             double* mu_out, double* per_atom);

/* Potential-energy surface of every frame (Sec. 2.1) with a TNEP_KIND_PES
 * model, whose one head gives the site energies U_i:
 *   energy  [n_frames]        U = sum_i U_i (Eq. site-energy), FP64;
 *   virial  [n_frames][9]     W = -sum_i sum_j r_ij (x) dU_i/dr_ij (Eq. virial),
 *                             row-major (u, v); NULL to skip;
 *   forces  [total_atoms][3]  F_k = -dU/dr_k = sum_j dU_k/dr_kj - sum_i dU_i/dr_ik
 *                             (r_ij = r_j - r_i), input atom order; NULL to skip;
 *   per_atom_energy [total_atoms] U_i; NULL to skip.
 * Forces: a first kernel leaves every atom's own pair terms and its network
 * derivatives; a second evaluates, for each atom k and neighbour j, the term
 * -dU_j/dr_jk from j's derivatives, and sums all terms in a fixed order, so
 * results do not depend on scheduling or batching.  Location, ownership and
 * errors as for tnep_eval_dipole. */
int tnep_eval_pes(tnep_ctx* ctx, const tnep_model* model, const tnep_frames* frames, double* energy,
                  double* virial, double* forces, double* per_atom_energy);

/* ---- spectra ----------------------------------------------------------- */
#define TNEP_IR 0          /* series rank 1 [.][3]: (1/3) sum_a <mu_a(0) mu_a(t)>, x w^2      */
#define TNEP_RAMAN_ISO 1   /* rank 2 [.][9]: <gamma(0) gamma(t)>, gamma = Tr(alpha)/3         */
#define TNEP_RAMAN_ANISO 2 /* rank 2: <Tr beta(0) beta(t)>, beta = alpha - gamma I           */
#define TNEP_RAMAN_PROJ 3  /* rank 2: <s(0) s(t)>, s = n^T alpha e                           */
#define TNEP_RAMAN_MAP 4   /* streams only: all nine components, for orientation maps       */

#define TNEP_WIN_HANN 0    /* lag window w(tau) = (1 + cos(pi tau / M)) / 2 */
#define TNEP_WIN_NONE 1

#define TNEP_SUBTRACT_MEAN 1 /* flags: remove each series' time mean first   */
#define TNEP_NO_OMEGA2 2     /* flags: IR without the w^2 prefactor           */

typedef struct {
    int32_t kind;          /* TNEP_IR / TNEP_RAMAN_*                                  */
    int32_t n_series;      /* independent runs; spectra are averaged over them         */
    int64_t n_steps;       /* N_t samples per run (>= 2)                               */
    const double* series;  /* [n_series][n_steps][3 or 9], FP64                        */
    double dt_fs;          /* sample spacing, fs                                       */
    int64_t max_lag;       /* M, 1 <= M <= n_steps                                     */
    int32_t window;        /* TNEP_WIN_*                                               */
    int32_t flags;         /* TNEP_SUBTRACT_MEAN | TNEP_NO_OMEGA2                      */
    double n_hat[3];       /* TNEP_RAMAN_PROJ only                                     */
    double e_hat[3];
    int32_t location;      /* TNEP_HOST / TNEP_DEVICE for series and the outputs       */
    double laser_cm1;      /* > 0: Raman kinds times ((w_in - w)/c)^4 = (2 pi (laser_cm1 - nu_k))^4,
                              cm^-4 (Eq. raman-cross-section); 0 = off; ignored for IR     */
} tnep_spectrum_args;

/* Correlation function of the series (time-origin average, 1/(N_t - tau)
 * normalisation, tau = 0..M-1), its one-sided windowed cosine transform
 *   S(w_k) = dt/(2 pi) [w(0) C(0) + 2 sum_{tau=1}^{M-1} w(tau) C(tau) cos(w_k tau dt)],
 *   w_k = pi k / (M dt), k = 0..M,
 * times w_k^2 for TNEP_IR (unless TNEP_NO_OMEGA2), averaged over the series.
 * freq_cm1: [M+1] wavenumbers k / (2 M dt c); intensity: [M+1]; acf: NULL or [M].
 * All FP64. */
int tnep_spectrum(tnep_ctx* ctx, const tnep_spectrum_args* args, double* freq_cm1, double* intensity,
                  double* acf);

/* tnep_spectrum for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and results as tnep_spectrum, with two differences:
 *   - args->location must be TNEP_DEVICE (series and outputs in device memory
 *     of the context's GPU); TNEP_HOST is TNEP_E_INVALID;
 *   - the call enqueues its kernels on the context's stream and returns
 *     without waiting: results are complete when the stream reaches that
 *     point.
 * The workspace (the signals, their FFTs and the cosine table:
 * 32 n_series s P + 72 n_series + 24 M + 1040 bytes plus alignment, s = 3
 * (IR), 1 (iso, proj) or 9 (aniso) signals, P the FFT length, the power of
 * two >= 2 n_steps) lives
 * in one fixed 64 MiB device array per GPU, held by the library until the
 * process ends; larger requests are TNEP_E_BUDGET with a message.  The call
 * allocates nothing (no hipMalloc / hipFree, no events).  All calls on one
 * GPU share that array: calls that overlap in time on one GPU (other streams,
 * contexts or threads) race and must be serialised by the caller. */
int tnep_spectrum_noalloc(tnep_ctx* ctx, const tnep_spectrum_args* args, double* freq_cm1, double* intensity,
                          double* acf);

/* Orientation-resolved Raman lineshapes (Sec. 2.7, Eqs. raman-cross-section
 * and raman-lineshape; Sec. 4 maps the crystal-orientation dependence): for
 * each polarisation pair o, sum_{g d m n} n_g n_m L_{g d m n}(w) e_d e_n, i.e.
 * the spectrum of s(t) = n_o^T alpha(t) e_o, for all n_orient pairs from one
 * pass over the series (the 45 symmetrised cross-correlations of alpha's nine
 * components are transformed once, then contracted).  args as for
 * tnep_spectrum with series [n_series][n_steps][9]; args->kind, n_hat, e_hat
 * are ignored; TNEP_SUBTRACT_MEAN and laser_cm1 apply.  n_hat, e_hat:
 * [n_orient][3] host memory (used as given, not normalised); intensity:
 * [n_orient][M+1]; freq_cm1 [M+1]; location of series and outputs from args. */
int tnep_raman_map(tnep_ctx* ctx, const tnep_spectrum_args* args, int32_t n_orient, const double* n_hat,
                   const double* e_hat, double* freq_cm1, double* intensity);

/* ---- streaming correlation accumulators --------------------------------- */
/* For series too long (or arriving too late) to hold whole: samples are
 * pushed in chunks of any size; each run's pair sums
 * S(tau) = sum_{t + tau < N} x(t) y(t + tau) are accumulated in FP64 on the
 * device (a chunk's contribution by zero-padded FFT against the run's last
 * M - 1 samples), and at the end of a run C(tau) = S(tau) / (N - tau) (with the
 * run means removed under TNEP_SUBTRACT_MEAN) joins the average over runs.
 * The results equal tnep_spectrum / tnep_raman_map on the whole runs (up to
 * rounding).  A stream belongs to its context, which must outlive it; calls
 * on a stream are synchronous (device pushes excepted, see below) and not
 * thread-safe. */
typedef struct tnep_acf_stream tnep_acf_stream;
/* kind: TNEP_IR (samples [.][3]), TNEP_RAMAN_ISO / ANISO / PROJ (with n_hat,
 * e_hat) or TNEP_RAMAN_MAP (samples [.][9]); max_lag M >= 1; flags:
 * TNEP_SUBTRACT_MEAN | TNEP_NO_OMEGA2. */
int tnep_acf_stream_create(tnep_ctx* ctx, int32_t kind, int64_t max_lag, int32_t flags, const double* n_hat,
                           const double* e_hat, tnep_acf_stream** out);
/* Append n_samples samples ([n_samples][3 or 9] FP64, host or device) to the current run.
 * Host samples are consumed before the call returns.  Device samples
 * (TNEP_DEVICE, with TNEP_OPT_TIMING off) are only enqueued on the context's
 * stream: the call returns without waiting, so consecutive pushes run back to
 * back on the GPU, and the caller keeps the chunk unchanged until the next
 * tnep_acf_stream_end_run / _spectrum / _raman_map call on the stream (these
 * wait) or until the stream is otherwise synchronised. */
int tnep_acf_stream_push(tnep_acf_stream* s, const double* samples, int64_t n_samples, int32_t location);
/* Close the current run (it needs at least max_lag samples). */
int tnep_acf_stream_end_run(tnep_acf_stream* s);
/* Spectrum over the finished runs (as tnep_spectrum; host outputs freq [M+1],
 * intensity [M+1], acf NULL or [M]).  Not for TNEP_RAMAN_MAP streams. */
int tnep_acf_stream_spectrum(tnep_acf_stream* s, double dt_fs, int32_t window, double laser_cm1, double* freq_cm1,
                             double* intensity, double* acf);
/* Orientation map over the finished runs of a TNEP_RAMAN_MAP stream (as
 * tnep_raman_map; host arrays). */
int tnep_acf_stream_raman_map(tnep_acf_stream* s, double dt_fs, int32_t window, double laser_cm1, int32_t n_orient,
                              const double* n_hat, const double* e_hat, double* freq_cm1, double* intensity);
void tnep_acf_stream_free(tnep_acf_stream* s);

/* ---- training loss of a population ------------------------------------- */
/* Loss of each individual of an evolution-strategy population (Sec. 2.4, loss
 * function of the training; the optimiser draws the individuals):
 *   L(z) = RMSE(z) + lambda1 * sum_i |z_i| / N + lambda2 * sqrt(sum_i z_i^2 / N),
 * RMSE over all F * nt predicted frame-tensor components (nt = 3 dipole, 9
 * polarizability) against reference [F][nt] (same units as the predictions).
 * base: hyperparameters (kind, species, cutoffs, basis sizes, hidden width,
 * four-body flag; shared networks only), its parameter pointers are ignored.
 * params: [n_individuals][N] FP64 host array, each row in the order
 * c_radial [T][T][nr][kr], c_angular [T][T][na][ka], then per output head
 * (one dipole, two polarizability: anisotropic, scalar) w0 [H][D], b0 [H],
 * w1 [H], b1.  frames: host or device; reference in the frames' location.
 * loss_out, rmse_out (may be NULL): [n_individuals] host.  Up to 64
 * individuals share one neighbour build.  Errors: TNEP_E_INVALID on bad
 * arguments, TNEP_E_BUDGET / TNEP_E_HIP as for the evaluators. */
int tnep_population_loss(tnep_ctx* ctx, const tnep_model_desc* base, int32_t n_individuals, const double* params,
                         const tnep_frames* frames, const double* reference, double lambda1, double lambda2,
                         double* loss_out, double* rmse_out);

/* ---- serving (continuous batching) ------------------------------------- */
typedef struct {
    uint64_t mem_budget_bytes; /* admission budget for in-flight requests (0 = ctx budget) */
    int32_t max_batch_atoms;   /* atoms per fused launch (0 = 262144)                       */
    int32_t max_inflight;      /* launches in flight on the device (0 = 2)                  */
} tnep_server_opts;

/* Start the server thread of ctx.  After this, only tnep_submit / tnep_wait /
 * tnep_server_stop / tnep_server_stats / tnep_server_memory /
 * tnep_ctx_graph_counts may be used on ctx.  Slot contexts inherit the launch
 * options of ctx, TNEP_OPT_GRAPHS included.
 * Memory: the slots draw their device work buffers from one pool of
 * mem_budget_bytes.  A slot about to evaluate a batch makes its grant cover
 * that batch; if the pool cannot give even what the batch's largest frame
 * needs, the slot returns its buffers and waits until other slots return
 * theirs (they do so after their current batch), so such requests are queued
 * until memory frees up instead of failing. */
int tnep_server_start(tnep_ctx* ctx, const tnep_server_opts* opts);
/* Queue one request: `kind` selects dipole (out [n_frames][3]) or
 * polarizability (out [n_frames][9]); potential-energy models are not served
 * (TNEP_E_INVALID).  frames and out must be host memory and
 * stay valid until tnep_wait returns for the ticket.  Returns TNEP_E_BUDGET
 * if the request's largest frame alone needs more device memory than the
 * whole pool (it could never run); every other request is queued. */
int tnep_submit(tnep_ctx* ctx, const tnep_model* model, int32_t kind, const tnep_frames* frames, double* out,
                uint64_t* ticket);
/* Block until the request is done.  status: the request's own TNEP_* code
 * (TNEP_E_CANCELLED if the server stopped first); latency_s:
 * submit-to-completion time in seconds.  Each ticket is waited for once: a
 * second call for the same ticket, also while the first still waits, returns
 * TNEP_E_INVALID.  tnep_server_stop waits for wait calls in progress to
 * return before it frees the server. */
int tnep_wait(tnep_ctx* ctx, uint64_t ticket, int32_t* status, double* latency_s);
/* Drain and stop the server thread. */
int tnep_server_stop(tnep_ctx* ctx);
/* Counters since start: requests done, fused launches, atom-frames done,
 * peak bytes granted to the slots from the pool (an upper bound of the
 * device memory their work buffers held at any time). */
int tnep_server_stats(tnep_ctx* ctx, uint64_t* requests, uint64_t* launches, uint64_t* atom_frames,
                      uint64_t* peak_bytes);
/* The memory pool: its size, the bytes granted to slots now, and how many
 * times a slot had to wait for pool memory.  Any pointer may be NULL. */
int tnep_server_memory(tnep_ctx* ctx, uint64_t* pool_bytes, uint64_t* granted_bytes, uint64_t* memory_waits);

#ifdef __cplusplus
}
#endif
#endif /* TNEP_H */
