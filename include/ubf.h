/*
 * ubf.h -- far-zone matrix-vector product of the uniform-basis,
 * group-by-group integral-equation method (arXiv 2501.04684,
 * Koc, Kalfa, Dogan, Erturk), on one AMD Instinct MI355X (gfx950).
 *
 * The product evaluated is y = T * G_far * S * x, the far part Z^F I of
 * Eq. (2), in three stages (Algorithm 5):
 *   1. aggregate:    P_i = S_i x_i              (Sec. 2.1, Eq. 11, Algorithm 1)
 *   2. translate:    E_j = sum_{i in F_j} G_{c_j - c_i} P_i
 *                                              (Sec. 2.2, Eq. 13-14, Algorithm 2)
 *   3. disaggregate: y_j = T_j E_j              (Sec. 2.3, Eq. 15-17, Algorithm 3)
 *
 * Geometry (Sec. 2, box partition; Sec. 2.2, translation vectors): the
 * caller gives the integer coordinates c of the occupied child boxes of
 * side a. Box c has its centre at a*(c + 1/2). Each box carries n_d^3
 * Hertzian dipoles on a cell-centred uniform lattice, site m in
 * {0..n_d-1}^3 at a*((m + 1/2)/n_d - 1/2) from the box centre, site index
 * s = (m_x*n_d + m_y)*n_d + m_z, and three components per site, so
 * N_u = 3*n_d^3 coefficients per box with index u = 3*s + alpha
 * (alpha = x, y, z).
 *
 * Far set: UBF_FAR_FULL takes every pair with Chebyshev offset >= 2
 * (Algorithm 2's ||w|| >= 2a on the box lattice); UBF_FAR_ILIST further
 * keeps only pairs whose parent boxes floor(c/2) are Chebyshev-adjacent
 * (the one-box-buffer interaction list of a two-level tree; its 316
 * distinct offsets are the translation vectors counted in Sec. 2.2).
 *
 * Operators: G_w[(l,alpha),(s,beta)] = D(a*w + r_l - r_s)[alpha][beta],
 * D the free-space dyadic Green's function of Eq. (5)-(6) with time
 * convention exp(+j omega t). They are generated on the host in FP64 at
 * plan creation and stored once per distinct offset in FP32.
 *
 * Conventions shared by every entry point:
 *   - Status codes: UBF_OK (0) or a negative UBF_E* value. No exception
 *     crosses this interface and nothing aborts. ubf_last_error() returns
 *     a thread-local message describing the last failure on this thread.
 *   - All argument checks finish before any HIP call, so an invalid
 *     argument never leaves work queued. Errors of kernels already queued
 *     surface at a later call (as from any asynchronous HIP work).
 *   - Device memory is owned by the caller. The library never allocates
 *     device memory; it works in the caller's workspace (ubf_plan_bind).
 *   - "d_" arguments are device pointers; all others are host pointers.
 *   - Complex vectors are complex64, interleaved (re, im) float pairs, the
 *     layout of torch.complex64, laid out [nrhs][length] row-major.
 *   - hip_stream is a hipStream_t (NULL = the null stream). Compute entry
 *     points only enqueue work on it and return. A plan may be used by one
 *     stream at a time: two calls on one plan that overlap in time race on
 *     its workspace.
 */
#ifndef UBF_H
#define UBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum ubf_status {
  UBF_OK = 0,
  UBF_EINVAL = -1,   /* invalid argument */
  UBF_ENOMEM = -2,   /* workspace too small, or a host allocation failed */
  UBF_EDEVICE = -3,  /* a HIP runtime call failed */
  UBF_ESTATE = -4    /* plan not bound to a workspace / wrong state */
};

enum ubf_far_mode {
  UBF_FAR_ILIST = 0, /* parent-adjacent pairs with Chebyshev offset >= 2 */
  UBF_FAR_FULL = 1   /* every pair with Chebyshev offset >= 2 (Algorithm 2) */
};

enum ubf_precision {
  UBF_FP32 = 0,        /* FP32 operands, FP32 accumulation */
  UBF_SPLIT_BF16 = 1,  /* stage 2 with operators and coefficients each split
                          into a BF16 high part and a BF16 remainder,
                          G P ~ Gh Ph + Gh Pl + Gl Ph on the BF16 matrix cores
                          with FP32 accumulation (stages 1 and 3 stay FP32);
                          n_d 1..4 (at n_d = 4 the operator is stored in
                          matrix-core fragment order and the item's box
                          vectors are staged in LDS) */
  UBF_SPLIT_FP16 = 2,  /* as UBF_SPLIT_BF16 with FP16 parts: each operator is
                          stored divided by a power of two (per offset) and
                          each box vector by a power of two (per box and
                          RHS) so both fit the FP16 range; the scales are
                          multiplied back into the FP32 result (exact) */
  UBF_FP16 = 3         /* one FP16 product Gh Ph per pair (scaled as in
                          UBF_SPLIT_FP16): about 2^-11 relative error per
                          product, for tolerances near 1e-3 */
};

/* Where the translation operators of Eq. (12)-(13) come from. */
enum ubf_operator_source {
  UBF_OPERATORS_TABLE = 0,     /* evaluated once on the host in FP64 at plan
                                  creation and kept in the workspace (one
                                  image per distinct offset) */
  UBF_OPERATORS_GENERATED = 1  /* evaluated by the stage-2 kernel from the
                                  offset each time it stages an operator:
                                  the Green's function of Eq. (5)-(6) in FP64
                                  once per lattice difference of the dipole
                                  sites, rounded as the table would be; no
                                  table is built or stored (FULL far sets of
                                  large scatterers, ~10^5 offsets). 16-bit
                                  forms with n_d 1..3 only; the round kernels
                                  of enum ubf_translate_kernel need a table */
};

/* Problem statement (Sec. 2: box grid, dipoles per box, wavenumber). */
typedef struct ubf_problem {
  int64_t n_boxes;         /* number of occupied boxes, >= 1 */
  const int32_t* box_ijk;  /* host, 3*n_boxes: (x, y, z) per box, each in
                              0..2^31-1 (any int32 >= 0; the box index is
                              keyed on the exact triple), no duplicates;
                              copied at creation */
  double a;                /* box side, > 0 */
  double k;                /* free-space wavenumber, > 0, per unit of a */
  double eta;              /* intrinsic impedance; 0 selects 376.730313668 */
  int32_t n_d;             /* dipoles per box edge, 1..4 */
  int32_t far_mode;        /* enum ubf_far_mode */
  int32_t precision;       /* enum ubf_precision */
  int32_t operators;       /* enum ubf_operator_source; 0 = table */
} ubf_problem;

/* Sizes and work counts of a plan, for benchmarks and tests. */
typedef struct ubf_info {
  int64_t n_boxes;
  int64_t n_pairs;          /* far-zone (test, source) box pairs */
  int32_t n_offsets;        /* distinct translation vectors */
  int32_t n_orbits;         /* classes under the 48 cube symmetries */
  int32_t n_u;              /* uniform-basis coefficients per box, 3*n_d^3 */
  int32_t n_d;
  int64_t n_chunks;         /* translation work units (per RHS) */
  int64_t table_bytes;      /* device operator table */
  double translate_flops;   /* real flops per RHS: 8 * n_u^2 * n_pairs */
  int32_t mfma;             /* 1 if stage 2 runs on the matrix cores */
  int32_t precision;        /* enum ubf_precision of the plan */
  int32_t n_scatterers;     /* independent scatterers in the plan (>= 1) */
  int32_t translate_groups; /* persistent stage-2 workgroups per RHS */
  int64_t n_items;          /* work items of the kernels that stage box vectors
                               in LDS (N_u = 192, networks) and of the round
                               kernels: up to 32 pairs of one offset each,
                               per RHS */
  int32_t translate_kernel; /* stage-2 kernel of the 16-bit forms: a value of
                               enum ubf_translate_kernel, 0 for the FP32 form */
  int32_t operators;        /* enum ubf_operator_source */
} ubf_info;

/* Stage-2 kernels of the 16-bit forms (ubf_plan_schedule, ubf_plan_tune).
 * All compute each column with the same products in the same order, so
 * they agree bit for bit; they differ in how the work is scheduled. */
enum ubf_translate_kernel {
  UBF_TRANSLATE_CHUNKS = 0,       /* persistent workgroups over chunks of up to
                                     128 pairs of one offset, one right-hand
                                     side per grid row (the FP32 form's only
                                     schedule) */
  UBF_TRANSLATE_CHUNKS_WALK = 1,  /* the same, each workgroup taking every
                                     right-hand side of a chunk in turn (one
                                     operator staging for all of them) */
  UBF_TRANSLATE_ROUNDS = 2,       /* rounds of four 32-pair items per
                                     workgroup, two workgroups per compute unit,
                                     partial rows stored while the next rows
                                     compute */
  UBF_TRANSLATE_ROUNDS_DOUBLE = 3 /* the same at one workgroup per compute unit
                                     with two operator buffers, the next
                                     segment's operator copied ahead */
};

typedef struct ubf_plan ubf_plan;

/* Build a plan on the host (no device work): validate the problem, build
 * the far set (Algorithm 2), its distinct offsets and their symmetry
 * orbits (Sec. 2.2), the work partition, and (UBF_OPERATORS_TABLE) the
 * operator table of the plan's form from FP64 evaluations of Eq. (5)-(6)
 * and (13).
 * Errors: UBF_EINVAL for a null pointer, n_boxes < 1, a negative or
 * duplicate coordinate, a <= 0, k <= 0, eta < 0, n_d outside 1..4, an
 * unknown far_mode, precision or operator source, generated operators
 * with the FP32 form or n_d = 4, a far set beyond 2^31-1 pairs, or an
 * operator table beyond 16 GiB;
 * UBF_ENOMEM if host memory runs out. *out is set only on success. */
int ubf_plan_create(const ubf_problem* problem, ubf_plan** out);

/* One plan over many independent scatterers, run together by every compute
 * entry point (batching). problem->box_ijk holds the boxes of all
 * scatterers concatenated (problem->n_boxes in total); boxes
 * [scatterer_ptr[s], scatterer_ptr[s+1]) form scatterer s. All scatterers
 * share a, k, eta, n_d, far_mode and precision, hence one operator table
 * over the union of their offsets (an operator depends only on the
 * integer offset, Sec. 2.2). The far set (Algorithm 2) is built within
 * each scatterer: no pair joins two scatterers, and coordinates may repeat
 * across scatterers (each has its own origin, which the ILIST parent rule
 * floor(c/2) uses). Box vectors and x, y follow the concatenated box
 * order, so y restricted to scatterer s equals the product of a plan made
 * from scatterer s alone.
 * scatterer_ptr: host, n_scatterers+1 values, scatterer_ptr[0] = 0,
 * strictly increasing, scatterer_ptr[n_scatterers] = n_boxes; copied.
 * Errors: those of ubf_plan_create, plus UBF_EINVAL for a null
 * scatterer_ptr, n_scatterers < 1, an empty scatterer or a last value
 * other than n_boxes; duplicate coordinates are rejected within a
 * scatterer only. */
int ubf_plan_create_batch(const ubf_problem* problem, int32_t n_scatterers,
                          const int64_t* scatterer_ptr, ubf_plan** out);

/* Device workspace bytes needed to run up to max_nrhs right-hand sides
 * per call (operator table, index tables, internal vectors). Returns 0 for
 * a null plan or max_nrhs < 1. */
size_t ubf_workspace_bytes(const ubf_plan* plan, int32_t max_nrhs);

/* Attach a caller-owned device workspace of `bytes` bytes (>= the size
 * ubf_workspace_bytes(plan, max_nrhs) returns; 256-byte aligned) and copy
 * the plan's tables into it on hip_stream, waiting for the copy to end.
 * The workspace must stay allocated until the plan is destroyed or bound
 * again. Errors: UBF_EINVAL (null, misaligned, max_nrhs < 1), UBF_ENOMEM
 * (too small), UBF_EDEVICE (copy failed). */
int ubf_plan_bind(ubf_plan* plan, void* d_workspace, size_t bytes,
                  int32_t max_nrhs, void* hip_stream);

/* Set the subdomain basis (Algorithm 1 and 3 preprocessing results).
 * nb_ptr: host, n_boxes+1 prefix sums of the per-box function counts N_b,i
 *   (nb_ptr[0] = 0, non-decreasing); copied.
 * d_S: per box, S_i = A^dagger [B_1..B_Nb] of size N_u x N_b,i, complex64,
 *   column-major, the boxes' blocks concatenated in box order.
 * d_T: per box, T_i of size N_b,i x N_u, complex64, column-major,
 *   concatenated; NULL means T_i = S_i^T (Galerkin point testing).
 * Passing nb_ptr = NULL and d_S = NULL restores the identity basis, in
 * which x holds the N_u uniform-basis coefficients of every box.
 * The matrices stay owned by the caller and must outlive their use.
 * Needs a bound plan (it copies nb_ptr into the workspace, synchronously).
 * Errors: UBF_EINVAL (bad prefix sums, d_S NULL with nb_ptr given),
 * UBF_ESTATE (unbound), UBF_EDEVICE. */
int ubf_plan_set_basis(ubf_plan* plan, const int64_t* nb_ptr,
                       const void* d_S, const void* d_T);

/* Bytes of the device image that ubf_plan_set_networks fills for networks
 * of `hidden` units; 0 if the plan's box size or the width has no network
 * kernel (n_d must be 2, 3 or 4; 1 <= hidden <= 64). */
size_t ubf_network_bytes(const ubf_plan* plan, int32_t hidden);

/* Let trained networks stand in for the translation operators (Sec. 3,
 * Fig. 5): stage 2 then adds, for each far-zone pair (i -> j) with offset
 * w, the network output ||P_i|| (W2_w CReLU(W1_w P_i/||P_i|| + b1_w) +
 * b2_w) to E_j, where ||.|| is the largest modulus (l-infinity norm) of the
 * box vector, CReLU(z) = max(Re z, 0) + j max(Im z, 0) per component, and
 * a zero box vector contributes zero. Stages 1 and 3 are unchanged.
 * Weights, complex64 on the device, one network per distinct offset in the
 * order of ubf_plan_offsets: d_W1 [n_offsets][hidden][N_u] (row-major),
 * d_b1 [n_offsets][hidden], d_W2 [n_offsets][N_u][hidden], d_b2
 * [n_offsets][N_u]. They are converted on hip_stream into d_net (caller
 * owned, 16-byte aligned, at least ubf_network_bytes(plan, hidden) bytes),
 * which must stay allocated while the plan uses it; the weight arrays may
 * be freed once the stream has passed this call (and may be NULL when the
 * plan has no offsets). hidden = 0 (pointers ignored) returns stage 2 to
 * the operator table. Needs a bound plan of
 * the FP32 form (precision 0). Any captured graph is discarded.
 * Errors: UBF_EINVAL (null, precision, n_d or hidden out of range,
 * misaligned image), UBF_ENOMEM (image too small), UBF_ESTATE (unbound),
 * UBF_EDEVICE. */
int ubf_plan_set_networks(ubf_plan* plan, int32_t hidden, const void* d_W1, const void* d_b1,
                          const void* d_W2, const void* d_b2, void* d_net, size_t net_bytes,
                          void* hip_stream);

/* The whole far-zone product y = T G S x (Algorithm 5) for nrhs vectors.
 * d_x, d_y: [nrhs][sum N_b] complex64 (identity basis: sum N_b =
 * n_boxes*N_u); y is overwritten. 1 <= nrhs <= the bound max_nrhs.
 * x and y must not overlap. Errors: UBF_EINVAL (null, aliasing, nrhs out
 * of range), UBF_ESTATE (unbound), UBF_EDEVICE (launch failed). */
int ubf_far_mvm(ubf_plan* plan, const void* d_x, void* d_y, int32_t nrhs,
                void* hip_stream);

/* Size of the static device array behind ubf_far_mvm_noalloc (96 MiB). */
#define UBF_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as ubf_far_mvm, same arguments, kernels and results bit for bit,
 * but its per-call intermediates (box vectors, partial rows, FP16 box
 * scales) live in one static device array of UBF_NOALLOC_SCRATCH_BYTES
 * inside the library instead of the plan's bound workspace (which still
 * holds the plan's tables). Nothing is allocated on any call; each GPU the
 * library runs on holds its own copy of the array until the process ends.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (any plan, any stream) race, so
 * order them on one stream or synchronize between them. The first call on
 * a device looks the array's address up once.
 * Errors: those of ubf_far_mvm, plus UBF_EINVAL when one call of nrhs
 * vectors needs more than UBF_NOALLOC_SCRATCH_BYTES (the 3,338-box shell
 * with 108,888 far pairs needs 75.6 MB per right-hand side), checked
 * before any device work. */
int ubf_far_mvm_noalloc(ubf_plan* plan, const void* d_x, void* d_y, int32_t nrhs,
                        void* hip_stream);

/* Record the whole product y = T G S x for these d_x, d_y and nrhs as a
 * HIP graph owned by the plan (the three stage launches, no memory
 * operations), replacing any earlier one. Nothing runs at capture; the
 * capture uses a stream of the plan's own. The graph holds the pointers it
 * was captured with and the plan's workspace addresses: ubf_plan_bind,
 * ubf_plan_set_basis and ubf_plan_tune discard it.
 * Errors: those of ubf_far_mvm; UBF_EDEVICE if capture or instantiation
 * fails. */
int ubf_plan_capture(ubf_plan* plan, const void* d_x, void* d_y, int32_t nrhs);

/* Launch the captured product on hip_stream (asynchronous, one graph
 * launch for the three stages). Errors: UBF_EINVAL (null plan),
 * UBF_ESTATE (nothing captured), UBF_EDEVICE. */
int ubf_plan_replay(ubf_plan* plan, void* hip_stream);

/* Autotune stage 2 of a bound plan, the counterpart of the paper's
 * scheduling of translations by translation vector (Sec. 4): time `reps`
 * translation launches for nrhs right-hand sides under each candidate
 * schedule and keep the fastest. Candidates: the persistent chunk kernel at
 * 256, 512, 1024, 2048 and 4096 workgroups (capped by the number of
 * chunks); for the 16-bit forms also the walk over right-hand sides at the
 * same grids (nrhs > 1), the rounds kernel at 512, 1024 and 2048 workgroups
 * and the double-buffered rounds kernel at 256. The chosen workgroup count
 * goes to *groups_out (may be NULL), the kernel to ubf_info's
 * translate_kernel. If the environment variable UBF_TUNE_CACHE names a
 * file, a schedule recorded there for the same plan statistics (form, N_u,
 * nrhs, boxes, scatterers, pairs, offsets, chunks, items) is applied
 * without timing, and a new choice is appended to it with every
 * candidate's time. Runs and waits on hip_stream; overwrites the
 * workspace's internal vectors (never x or y). Results of later products
 * do not depend on the choice (bit for bit). Plans whose stage 2 has no
 * persistent grid (networks set, or 192 coefficients per box in FP32) are
 * left as they are. Any captured graph is discarded. Errors: UBF_EINVAL
 * (null plan, nrhs out of 1..max_nrhs, reps out of 1..1000), UBF_ESTATE
 * (unbound), UBF_EDEVICE. */
int ubf_plan_tune(ubf_plan* plan, int32_t nrhs, int32_t reps, void* hip_stream,
                  int32_t* groups_out);

/* Set stage 2 of a bound plan to a given schedule (what ubf_plan_tune
 * would choose): kernel is an enum ubf_translate_kernel value (only 0 for
 * the FP32 form), groups the persistent workgroup count (1..4096, rounded
 * up to a multiple of 8 and capped by the work units). Uploads the work
 * partition on hip_stream and waits. Results do not depend on the choice.
 * Any captured graph is discarded. Errors: UBF_EINVAL (null plan, unknown
 * kernel, a 16-bit kernel on an FP32 plan, a round kernel on a plan with
 * generated operators, groups out of range, or a plan whose stage 2 runs
 * one workgroup per item: networks set, or 192 coefficients per box),
 * UBF_ESTATE (unbound), UBF_EDEVICE. */
int ubf_plan_schedule(ubf_plan* plan, int32_t kernel, int32_t groups, void* hip_stream);

/* Stage 1 alone: d_P[nrhs][n_boxes][N_u] = S_i x_i (complex64). */
int ubf_aggregate(ubf_plan* plan, const void* d_x, void* d_P, int32_t nrhs,
                  void* hip_stream);

/* Stage 2 alone: d_E[nrhs][n_boxes][N_u] = sum_{i in F_j} G P_i
 * (complex64 in and out; d_E overwritten; must not overlap d_P). */
int ubf_translate(ubf_plan* plan, const void* d_P, void* d_E, int32_t nrhs,
                  void* hip_stream);

/* Stage 3 alone: d_y[nrhs][sum N_b] = T_j E_j (complex64). */
int ubf_disaggregate(ubf_plan* plan, const void* d_E, void* d_y,
                     int32_t nrhs, void* hip_stream);

/* ------------------------------------------------------------------ */
/* Iterative solution (Algorithm 5's solver loop): restarted GMRES for
 * (sigma I + Z^F) x = b, Z^F = T G S the far-zone product of a bound plan
 * (the near-field part Z^N needs meshes, so a complex shift sigma stands in
 * for it). nrhs right-hand sides run as independent Krylov processes whose
 * products share each ubf_far_mvm launch. Krylov vectors are complex64 (the
 * product's input); every inner product, norm and Gram-Schmidt update is
 * accumulated in FP64 (two classical passes), and the Hessenberg matrix,
 * Givens rotations and least-squares solve are FP64, all on the device.
 * Sums use a fixed block count and order, so runs repeat bit for bit.
 * A right-hand side stops updating once its residual estimate
 * ||b - A x|| / ||b|| (the rotated least-squares residual) reaches tol. */
typedef struct ubf_gmres ubf_gmres;

typedef struct ubf_gmres_status {
  int32_t ready;       /* 1 if the last enqueued step has completed */
  int32_t done;        /* every right-hand side converged, or max_steps reached */
  int32_t converged;   /* every right-hand side within tol */
  int32_t steps;       /* Arnoldi steps enqueued (one product each) */
  int32_t restarts;    /* restarts enqueued (one extra product each) */
  int32_t reserved;
  double max_rel_res;  /* largest residual estimate over the right-hand sides */
} ubf_gmres_status;

/* Device workspace bytes of a solver for nrhs (1..64) right-hand sides and
 * restart length 1..128 on this plan (0 if out of range): the restart+1
 * Krylov blocks [nrhs][sum N_b] complex64 dominate. */
size_t ubf_gmres_workspace_bytes(const ubf_plan* plan, int32_t nrhs, int32_t restart);

/* Create a solver on a bound plan (whose max_nrhs >= nrhs) in a caller-owned
 * 256-byte aligned device workspace. sigma = sigma_re + j sigma_im; tol in
 * (0, 1) bounds the relative residual; max_steps caps the Arnoldi steps.
 * The solver allocates only a small pinned host block for its status. While
 * it runs, the plan is in use on the solver's stream. Errors: UBF_EINVAL,
 * UBF_ESTATE (unbound plan), UBF_ENOMEM (workspace too small), UBF_EDEVICE. */
int ubf_gmres_create(ubf_plan* plan, int32_t nrhs, int32_t restart, double sigma_re,
                     double sigma_im, double tol, int32_t max_steps, void* d_workspace,
                     size_t bytes, ubf_gmres** out);

/* Begin a solve from x_0 = 0: d_b and d_x are [nrhs][sum N_b] complex64,
 * not overlapping; x is written by ubf_gmres_finish (and at restarts).
 * Enqueued on hip_stream. Errors: UBF_EINVAL, UBF_ESTATE, UBF_EDEVICE. */
int ubf_gmres_start(ubf_gmres* solver, const void* d_b, void* d_x, void* hip_stream);

/* Enqueue one Arnoldi step (one product, orthogonalisation, rotation); when
 * the cycle is full, also the restart (x += V y, one more product for the
 * new residual). Never waits. Errors: UBF_ESTATE (not started, finished,
 * plan unbound, basis changed, or the plan bound again with a max_nrhs
 * below the solver's nrhs), UBF_EDEVICE. All checks finish before any
 * device work is enqueued. */
int ubf_gmres_step(ubf_gmres* solver, void* hip_stream);

/* Status of the last enqueued step: with wait = 0 it returns at once
 * (out->ready = 0 while that step is still running), else it waits for it.
 * rel_res (may be NULL) receives nrhs residual estimates.
 * Errors: UBF_EINVAL (null), UBF_ESTATE (not started), UBF_EDEVICE. */
int ubf_gmres_poll(ubf_gmres* solver, int32_t wait, ubf_gmres_status* out,
                   double* rel_res);

/* Complete the solution: x += V y over the current cycle. The solver must be
 * started again before further steps. Errors: as ubf_gmres_step. */
int ubf_gmres_finish(ubf_gmres* solver, void* hip_stream);

/* Estimate ||Z^F||_2 (the plan's far-zone product) by `iters` (1..100)
 * rounds of power iteration on Z^H Z, using Z^H u = conj(Z^F conj(u)):
 * Z^F is complex symmetric by the reciprocity of the dyadic Green's
 * function (Eq. 5-6), for the identity basis and for T = S^T. The start
 * vector comes from a counter hash of `seed` on the device. Each round is
 * two products on the first right-hand-side row plus FP64 norms; *out
 * (host) receives the square root of the last Rayleigh quotient, which
 * approaches the norm from below. Uses the solver's Krylov blocks, so a
 * solve in progress is abandoned (start again afterwards). Waits for the
 * stream. Errors: UBF_EINVAL (null, iters out of range, or a plan whose
 * product is not complex symmetric: an explicit T, or networks standing in
 * for the operators), UBF_ESTATE, UBF_EDEVICE. */
int ubf_gmres_norm_estimate(ubf_gmres* solver, int32_t iters, uint64_t seed,
                            void* hip_stream, double* out);

/* Replace the shift sigma of the system (takes effect at the next start or
 * step). Errors: UBF_EINVAL (null). */
int ubf_gmres_set_shift(ubf_gmres* solver, double sigma_re, double sigma_im);

/* Release the solver (its pinned status block; the workspace stays the
 * caller's). */
void ubf_gmres_destroy(ubf_gmres* solver);

/* Plan sizes and work counts. Errors: UBF_EINVAL for null pointers. */
int ubf_plan_info(const ubf_plan* plan, ubf_info* out);

/* Host copy of the distinct offsets w (3*n_offsets int32, in the plan's
 * offset order). Errors: UBF_EINVAL for null pointers. */
int ubf_plan_offsets(const ubf_plan* plan, int32_t* out);

/* Host copy of the far set, grouped by offset: for each pair its test box,
 * source box and offset index (n_pairs int32 each; any may be NULL). */
int ubf_plan_far_pairs(const ubf_plan* plan, int32_t* test, int32_t* src,
                       int32_t* offset_index);

/* G_w for offset index `o`, evaluated in FP64 by the plan's generator:
 * out is N_u*N_u complex values as interleaved doubles, row-major
 * (row = (l, alpha) test coefficient, column = (s, beta) source).
 * Errors: UBF_EINVAL (null, o out of range). */
int ubf_plan_operator(const ubf_plan* plan, int32_t o, double* out);

/* Measurement support (not part of the method). Time the kernel of each
 * of the three stages of products on this plan, whether issued by
 * ubf_far_mvm or by a GMRES solver on the plan: the kernel's dispatch
 * itself records a HIP event when it starts and one when it ends
 * (hipExtLaunchKernel), so a stage's time is its kernel's execution time
 * alone. Products recorded: the 1st, (every+1)-th, (2*every+1)-th ...
 * after this call, up to max_calls of them. A recorded dispatch costs
 * more device time than a plain one, so every > 1 keeps the recording's
 * cost off a throughput measurement.
 * Errors: UBF_EINVAL (max_calls < 1, every < 1), UBF_EDEVICE. */
int ubf_profile_begin(ubf_plan* plan, int32_t max_calls, int32_t every);

/* Wait for the recorded calls and release their events. stage_ms (3
 * doubles, may be NULL) receives the summed kernel milliseconds of stage
 * 1, 2 and 3; call_ms (may be NULL, room for max_calls floats) receives
 * each call's time from the start of stage 1 to the end of stage 3;
 * *n_calls (may be NULL) the number of calls recorded.
 * Errors: UBF_ESTATE (no profile begun), UBF_EDEVICE. */
int ubf_profile_end(ubf_plan* plan, double* stage_ms, float* call_ms,
                    int32_t* n_calls);

/* Release the plan (host memory only; the workspace stays the caller's). */
void ubf_plan_destroy(ubf_plan* plan);

/* Static text for a status code. */
const char* ubf_status_string(int status);

/* Thread-local description of the last error on this thread ("" if none). */
const char* ubf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* UBF_H */
