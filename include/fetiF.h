/*
 * fetiF — explicit FETI local dual operators on AMD Instinct MI355X (gfx950).
 *
 * The library assembles, for every subdomain i of a torn (Total-FETI)
 * problem, the explicit local dual operator
 *
 *     F~_i = B~_i K_i^+ B~_i^T,   K_i^+ = K_reg,i^{-1} = L_i^{-T} L_i^{-1}
 *
 * (paper Sec. II-A, eq. localdualoperator; Sec. III, eq.
 * localdualoperatorwithU with the symmetric factor K_reg,i = L_i L_i^T), by
 * the SYRK path of Sec. IV-C: X_i = L_i^{-1} P_i B~_i^T, F~_i = X_i^T X_i,
 * and applies the cluster operator q = sum_i D_i^T F~_i D_i lambda
 * (eq. dualop_apply_expl with the scatter/gather of Alg. 2).
 *
 * Lifecycle (Alg. 2): fetiF_create (preparation: ordering, symbolic
 * factorisation, device structures) -> per step fetiF_factor_upload for all
 * subdomains (numeric factorisation on host threads + copy of the factor
 * values) and fetiF_assemble -> per solver iteration fetiF_apply.
 *
 * Conventions for every entry point:
 *  - Pointers named *_d are device pointers on the context's device; all
 *    other pointers are host pointers, read during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Device work is enqueued on it; the calls do not synchronise the host
 *    unless stated.  Caller-owned device buffers must stay valid until the
 *    enqueued work completes.
 *  - Errors: argument errors return FETIF_EINVAL synchronously and change
 *    nothing; FETIF_ESTATE reports a call out of lifecycle order; HIP
 *    failures return FETIF_EDEVICE and are sticky for the context.  The
 *    message of the last error is fetiF_last_error(ctx).
 *  - One context is used by one host thread at a time.
 *  - Calls on one context share its device work buffers (solve vectors,
 *    apply partials, solver scalars): enqueue them on one stream, or order
 *    them across streams yourself (events).  Assembly and the solves with
 *    the factors wait for the last factor copy also when it was enqueued on
 *    another stream; fetiF_apply waits for nothing (it must stay capturable
 *    in a graph), so order it after fetiF_assemble when they use different
 *    streams.
 */
#ifndef FETIF_H
#define FETIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fetiF_ctx_s* fetiF_ctx;

typedef enum {
    FETIF_OK = 0,
    FETIF_EINVAL = 1,  /* invalid argument; nothing changed */
    FETIF_ENOMEM = 2,  /* host or device allocation failed */
    FETIF_ESTATE = 3,  /* call not valid in the current lifecycle state */
    FETIF_EDEVICE = 4, /* HIP runtime error or no usable device (sticky) */
    FETIF_ENOTSPD = 5, /* numeric factorisation met a non-positive pivot */
    FETIF_ENOTSUP = 6, /* option not supported */
    FETIF_ENONFINITE = 7 /* debug checks (fetiF_options.debug_checks) found a NaN or Inf */
} fetiF_status;

/* Storage precision of the assembled F~_i.  Assembly always computes in
 * FP64; FP32/BF16 are rounded to nearest-even when stored and are applied
 * with FP32 accumulation (FP64 accumulation for FP64 storage). */
typedef enum { FETIF_F64 = 0, FETIF_F32 = 1, FETIF_BF16 = 2 } fetiF_prec;

/* One subdomain, as given to fetiF_create (all arrays are copied).
 *  n            DOFs of K_reg,i.
 *  dofs_per_node  dof = dofs_per_node*node + component; DOFs of one node
 *               stay together in the ordering.
 *  k_ptr,k_idx  CSR of the FULL symmetric pattern of K_reg,i (both
 *               triangles, diagonal present, column indices ascending);
 *               fetiF_factor_upload takes values in this same order.
 *  dim,coords   optional node coordinates (n/dofs_per_node x dim, row-major)
 *               for geometric nested dissection; dim=0/coords=NULL selects
 *               graph nested dissection.
 *  m            rows of B~_i (local Lagrange multipliers), m >= 1 (a
 *               subdomain with none is not coupled: FETIF_EINVAL).
 *  b_dof,b_sign row j of B~_i has the single entry b_sign[j] (+1 or -1) in
 *               column b_dof[j] (Sec. II: one gluing/Dirichlet entry per row).
 *  dual_map     D_i: global multiplier of local row j, strictly increasing,
 *               in [0, n_lambda).
 *  nelem,edofs,elem_dofs,dK   optional element data for the theta-adjoint
 *               of fetiF_apply_backward: element e couples the local DOFs
 *               elem_dofs[e*edofs .. +edofs) and dK (edofs x edofs,
 *               row-major) is dK_reg,i/dtheta_e, the same for every element
 *               of the subdomain.  nelem=0 disables the adjoint.
 *  nkernel,R    optional kernel basis R_i of K_i (n x nkernel, row-major,
 *               nkernel <= 6; Sec. II) defining G = B R for the solver entry
 *               points; nkernel=0 in any subdomain disables them. */
typedef struct {
    int32_t n;
    int32_t dofs_per_node;
    const int32_t* k_ptr;
    const int32_t* k_idx;
    int32_t dim;
    const double* coords;
    int32_t m;
    const int32_t* b_dof;
    const int8_t* b_sign;
    const int32_t* dual_map;
    int32_t nelem;
    int32_t edofs;
    const int32_t* elem_dofs;
    const double* dK;
    int32_t nkernel;
    const double* R;
} fetiF_subdomain;

/* Options; zero-initialised fields select defaults. */
typedef struct {
    fetiF_prec f_storage; /* storage precision of F~_i (default FP64) */
    int32_t leaf_nodes;   /* nested-dissection leaf size in nodes (default 24) */
    int32_t nthreads;     /* host threads for analysis/factorisation (default: the CPUs of
                             the process's affinity mask) */
    int32_t apply_band;   /* stored elements of F~ per apply work-group (default 131072) */
    int32_t trsm_chunk;   /* most RHS columns per TRSM work-group: 16, 32 or 64 (default 64) */
    int32_t apply_rows;   /* rows of F~ per pass of a wavefront pair in apply, 2 or 4 (default 4) */
    int32_t apply_nontemporal; /* 1: stream F~ with non-temporal loads (default), 0: cached */
    int32_t apply_split;  /* apply work split: 0 bands per triangle, largest first (default);
                             1 equal shares of all stored elements, one per work-group */
    int32_t trsm_panel;   /* most supernode columns per TRSM panel, a multiple of 16 up to 96 (default 48) */
    int32_t apply_seg;    /* apply kernel: 0 whole rows per wavefront pair (m <= 4096); 2, 3, 4
                             or 8 column segments of that many 1 KiB chunks (default 4; with 8
                             the rows per pass are 2 whatever apply_rows says) */
    int32_t assembly_groups; /* contiguous subdomain groups of about equal factor size, each
                                with its own assembly schedule (default 1; fewer when a group
                                would hold fewer subdomains than there are host threads):
                                fetiF_factor_assemble factors group g+1 on the host while the
                                device copies and assembles group g */
    int32_t schur_order;  /* 1: Schur-complement route (Sec. III, eq. matrix_for_sc): the nodes
                             that carry Lagrange multipliers are ordered after all others, so
                             the factorisation of K_reg,i is a partial factorisation of the
                             interior followed by the Cholesky factor of its Schur complement
                             on those nodes, and X_i = L^{-1} P B~^T lives in that trailing
                             block only; the same kernels then assemble F~_i = -S of the
                             augmented matrix [K_reg B~^T; B~ 0].  0 (default): nested
                             dissection of all nodes (the SYRK path with a sparse RHS) */
    int32_t debug_checks; /* 1: fetiF_assemble, fetiF_apply, fetiF_apply_static,
                             fetiF_apply_implicit and fetiF_apply_backward wait for their
                             work and scan their device inputs and outputs (lambda, g, q,
                             dlambda, dtheta, the stored F~) for NaN or Inf, returning
                             FETIF_ENONFINITE with the vector and the first bad index in
                             fetiF_last_error.  These calls then synchronise their stream
                             and must not be captured in a graph.  0 (default): no scans;
                             non-finite values propagate */
} fetiF_options;

/* Preparation (Alg. 2, "preparation"; Sec. IV-B "Preparation"): nested
 * dissection and supernodal symbolic analysis of every K_reg,i on host
 * threads, the work schedules of assembly and application, and the device
 * memory for factors, X_i, F~_i and the dual-vector maps, with the constant
 * structures copied to the device.  `device` is the HIP ordinal.  On success
 * *out owns all of it until fetiF_destroy.  Synchronous.  FETIF_ENOTSUP if a
 * supernode's TRSM panel (up to 96 columns of ncols + nrows entries) spans
 * more than 2^31 bytes: the kernels address a panel with 32-bit offsets. */
fetiF_status fetiF_create(fetiF_ctx* out, int device, int64_t n_lambda, int32_t nsub,
                          const fetiF_subdomain* subs, const fetiF_options* opt);

/* Numeric factorisation K_reg,i = L_i L_i^T (Sec. III; Alg. 2 "FETI
 * preprocessing, num. fact.") of subdomains [first, first+count) on host
 * threads, then an asynchronous copy of the factor values to the device on
 * `stream` (Sec. IV-B "copy the factors' non-zero values to the GPU").
 * k_vals[k] holds the CSR values of K_reg of subdomain first+k in the
 * pattern given at create.  Returns FETIF_ENOTSPD (naming the subdomain and
 * pivot in fetiF_last_error) if a pivot is not positive.  The host arrays
 * may be freed on return; invalidates a previous assembly. */
fetiF_status fetiF_factor_upload(fetiF_ctx ctx, int32_t first, int32_t count,
                                 const double* const* k_vals, void* stream);

/* Assembly of every F~_i from the uploaded factors (Sec. IV-C, SYRK path):
 * RHS initialisation X_i = P_i B~_i^T, supernodal forward TRSM
 * X_i <- L_i^{-1} X_i, and F~_i = X_i^T X_i stored as one triangle in the
 * chosen precision.  Requires every subdomain uploaded since the last
 * assembly (else FETIF_ESTATE).  Asynchronous on `stream`. */
fetiF_status fetiF_assemble(fetiF_ctx ctx, void* stream);

/* Factorisation, copy and assembly of every subdomain, pipelined by the
 * assembly groups (Sec. IV-B "Preprocessing": the host factors the next
 * subdomains while the device assembles the previous ones): for each group,
 * host factorisation of its subdomains, then on `stream` the copy of their
 * factor values and their assembly, while the host goes on to the next
 * group.  k_vals[i] holds the CSR values of K_reg of subdomain i (all nsub).
 * The result is the one of fetiF_factor_upload over all subdomains followed
 * by fetiF_assemble (bitwise).  Returns when the last group is enqueued (the
 * host arrays may be freed then); FETIF_ENOTSPD as fetiF_factor_upload, after
 * which no subdomain counts as uploaded and F~ as not assembled. */
fetiF_status fetiF_factor_assemble(fetiF_ctx ctx, const double* const* k_vals, void* stream);

/* q_d[0..n_lambda) = sum_i D_i^T F~_i D_i lambda_d (Alg. 2 scatter, apply,
 * gather; eq. dualop_apply_expl).  FP64 vectors.  Each q entry is summed in
 * a fixed order (bitwise reproducible).  Allocates nothing and does no host
 * copy; capturable in a HIP graph.  lambda_d and q_d must not overlap. */
fetiF_status fetiF_apply(fetiF_ctx ctx, const double* lambda_d, double* q_d, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * application as fetiF_apply (same kernels, same summation order, bitwise
 * the same q), but the partial vectors of the band kernels live in a
 * file-scope device array of the library, 64 MiB per device (its address is
 * looked up once per device at fetiF_create), instead of the context's own
 * buffer.  Allocates nothing and does no host copy.  Nothing in the array
 * needs to start at zero: every partial the gather reads is written by the
 * band kernels of the same call.  All contexts on one device share that
 * array, so calls of fetiF_apply_static that overlap on one device (other
 * streams, other contexts, other host threads) race on it: order them.
 * FETIF_ENOTSUP (nothing enqueued) when the current apply plan's partial
 * vectors need more than 64 MiB (sum over bands of their last row, times 8
 * bytes for FP64 storage, 4 otherwise): larger bands (fetiF_set_apply) or
 * fetiF_apply serve such problems. */
fetiF_status fetiF_apply_static(fetiF_ctx ctx, const double* lambda_d, double* q_d, void* stream);

/* Assembly path (Sec. IV-C; the paper's "path" parameter, Sec. IV-D):
 * 0 (default) the SYRK path, F~_i = X_i^T X_i with X_i = L_i^{-1} P_i B~_i^T;
 * 1 the TRSM path: the same forward solve, then the backward solve
 * Z_i = L_i^{-T} X_i (dense, n_i x m_i, every column of every supernode
 * panel; FP64 MFMA) and the SpMM F~_i = B~_i P_i^T Z_i (a signed row gather)
 * into the stored triangle.  Path 1 allocates Z for all subdomains (sum n_i
 * m_i FP64 values; FETIF_ENOMEM if that fails, and path 0 stays) and frees
 * it when path 0 is set again.  Synchronises the device; the next
 * fetiF_assemble uses the path (fetiF_factor_assemble supports path 0 only:
 * FETIF_ENOTSUP).  Both paths give the same F~_i up to rounding. */
fetiF_status fetiF_set_assembly_path(fetiF_ctx ctx, int32_t path);

/* The application with host-resident cluster vectors, the setting of the
 * paper's "scatter and gather" parameter (Sec. IV-D, Table 1): lambda_h and
 * q_h are host arrays of n_lambda FP64 values.
 *  cpu_scatter_gather = 0: lambda is copied to the device, scattered, applied
 *    and gathered there (fetiF_apply), and q is copied back;
 *  cpu_scatter_gather = 1: host threads scatter lambda into the subdomain
 *    vectors p~_i = D_i lambda (all subdomains in one buffer, so one copy
 *    instead of one per subdomain), the band kernels apply F~_i to them, the
 *    band partials are copied back and host threads gather them into q in
 *    the same fixed order as the gather kernel.
 * Both give the fetiF_apply result bitwise.  Enqueued on `stream`; returns
 * when q_h holds the result.  The first call allocates device buffers
 * (2 n_lambda + sum m_i values) and pinned host staging (the same plus the
 * band partials); a later apply plan with more partials grows the staging. */
fetiF_status fetiF_apply_host(fetiF_ctx ctx, const double* lambda_h, double* q_h, int32_t cpu_scatter_gather,
                              void* stream);

/* Re-plan the application (tuning hook): band_elems > 0 sets the stored
 * elements of F~ per work-group (the band/gather tables are rebuilt, which
 * synchronises the device), rows (2 or 4; 0 keeps) the rows per pass of a
 * wavefront pair, nontemporal (0/1; -1 keeps) the load policy for F~, split
 * (0/1; -1 keeps) the work split of fetiF_options.apply_split, seg (0, 2, 3,
 * 4 or 8; -1 keeps) the kernel of fetiF_options.apply_seg.  The result of
 * fetiF_apply does not depend on these up to summation order.  A new band
 * size or split frees the previous apply tables: HIP graphs the caller
 * captured around fetiF_apply must be captured again (the library's own
 * captured solver iterations are discarded here). */
fetiF_status fetiF_set_apply(fetiF_ctx ctx, int32_t band_elems, int32_t rows, int32_t nontemporal,
                             int32_t split, int32_t seg);

/* Re-plan the assembly TRSM (tuning hook): trsm_panel (a multiple of 16 in
 * [16, 96]; 0 keeps) the most supernode columns per panel, trsm_chunk
 * (16, 32 or 64; 0 keeps) the most RHS columns per work-group.  Synchronises
 * the device; the assembled operator stays valid (the next fetiF_assemble
 * uses the new schedule).  The result of fetiF_assemble does not depend on
 * these up to summation order. */
fetiF_status fetiF_set_assembly(fetiF_ctx ctx, int32_t trsm_panel, int32_t trsm_chunk);

/* Reverse mode of J = g^T F(theta) lambda for the applied operator:
 *   dlambda_d = F g_d   (F is symmetric),
 *   dtheta_d[e] = -u_g|_e^T dK_e u_lambda|_e  for every element of every
 *   subdomain (concatenated in subdomain order), with u_x = K_reg,i^{-1}
 *   B~_i^T D_i x by forward and backward substitution with L_i.
 * dtheta_d may be NULL (then only dlambda is formed); requires element data
 * at create for a non-NULL dtheta_d.  Asynchronous on `stream`. */
fetiF_status fetiF_apply_backward(fetiF_ctx ctx, const double* g_d, const double* lambda_d,
                                  double* dlambda_d, double* dtheta_d, void* stream);

/* Implicit application (eq. dualop_apply_impl): q_d = sum_i D_i^T B~_i
 * L_i^{-T} L_i^{-1} B~_i^T D_i lambda_d by batched supernodal forward and
 * backward substitution with the uploaded factors (no assembled F needed).
 * Requires every subdomain factored.  Deterministic.  Asynchronous. */
fetiF_status fetiF_apply_implicit(fetiF_ctx ctx, const double* lambda_d, double* q_d, void* stream);

/* Dual right-hand side d = B K^+ f - c (Sec. II, below eq. alphaconstraint):
 * f_d is the concatenation of the subdomain load vectors f_i (local DOF
 * order, sum n_i entries), c_d the n_lambda constraint values (may be NULL
 * for c = 0).  Requires every subdomain factored.  Asynchronous. */
fetiF_status fetiF_dual_rhs(fetiF_ctx ctx, const double* f_d, const double* c_d, double* d_d, void* stream);

/* ---------------------------------------------------------------------
 * Dual solver (paper Sec. II and Alg. 1), all in FP64 on the device.
 * Needs the kernel bases R_i at create.  G = B R, e = R^T f,
 * P = I - G (G^T G)^{-1} G^T with (G^T G)^{-1} formed densely at create.
 * --------------------------------------------------------------------- */

/* e_d = R^T f: f_d concatenated subdomain loads (sum n_i), e_d one entry per
 * kernel vector (subdomain order).  Asynchronous. */
fetiF_status fetiF_coarse_rhs(fetiF_ctx ctx, const double* f_d, double* e_d, void* stream);

typedef struct {
    double tol;          /* stop when ||w_k|| <= tol ||w_0|| (default 1e-9) */
    int32_t max_iters;   /* default 1000 */
    int32_t fixed_iters; /* > 0: run exactly this many iterations */
    int32_t implicit;    /* 1: apply F implicitly with the factors; 0: assembled F~ */
    int32_t check_every; /* iterations between convergence checks (default 10);
                            a check also stops the solve when w^T y is not
                            finite or exceeds 1e8 times its start value */
    int32_t refine;      /* 1: FP64 iterative refinement around the assembled
                            (FP32/BF16) operator: outer true residual
                            P(d - F lambda) with the implicit FP64 operator,
                            inner PCPG on the correction to inner_tol (at most
                            2000 iterations each); a correction that does not
                            lower the true residual is taken back and the
                            refinement stops (rel_residual then says how far
                            it got) */
    double inner_tol;    /* relative tolerance of each inner solve (default 1e-4) */
    int32_t use_graph;   /* 1: replay captured iterations (needs a non-NULL stream) */
    int32_t precond;     /* M of Alg. 1: 0 identity; 1 lumped,
                            M = sum_i D_i^T B~_i K_i B~_i^T D_i; 2 lumped with the
                            scaled jump operator, M = B_D K B_D^T with
                            B_D = (B W B^T)^{-1} B W and W_i = diag(K_i)^{-1} on
                            the multiplier DOFs (stiffness scaling; B W B^T is
                            block diagonal over the multipliers that share a
                            DOF of some subdomain, inverted on the host when
                            the values change).  K_i: the values given by
                            fetiF_precond_values, else the K_reg,i values of
                            the last fetiF_factor_upload */
} fetiF_pcpg_options;

typedef struct {
    int32_t iters;        /* operator applications in PCPG iterations (all inner solves) */
    int32_t outer;        /* refinement steps (0 without refinement) */
    double rel_residual;  /* ||w|| / ||w_0|| at exit: recursive (no refinement) or
                             true FP64 projected residual (refinement); NaN when a
                             residual was not finite (NaN or Inf in d, e or the initial
                             lambda, or an operator that broke down), never 0 */
    double w0;            /* ||w_0|| (NaN when not finite) */
} fetiF_pcpg_result;

/* Stiffness values for the lumped preconditioners (fetiF_pcpg_options
 * precond 1 and 2) of subdomains [first, first+count): k_vals[k] holds the
 * values of K_i (normally the unregularised stiffness; the rows and columns
 * that carry multipliers are used) in the CSR pattern of K_reg,i given at
 * create (zero where K_i has no entry).  They are used instead of the K_reg
 * values of later factor uploads until given again.  Synchronises the
 * device.  FETIF_ESTATE without kernel bases (no solver). */
fetiF_status fetiF_precond_values(fetiF_ctx ctx, int32_t first, int32_t count, const double* const* k_vals);

/* Solve the dual problem (eq. tfetidualproblem) for lambda by PCPG with
 * M = I or a lumped preconditioner (options.precond) and
 * lambda_0 = G (G^T G)^{-1} e (Alg. 1).  d_d (n_lambda) from
 * fetiF_dual_rhs, e_d from fetiF_coarse_rhs; lambda_d receives the result.
 * Enqueued on `stream`; the call waits for the stream to report the
 * iteration count (every check_every iterations, and at the end). */
fetiF_status fetiF_pcpg(fetiF_ctx ctx, const double* d_d, const double* e_d, double* lambda_d,
                        const fetiF_pcpg_options* opt, fetiF_pcpg_result* res, void* stream);

/* Primal recovery: alpha = -(G^T G)^{-1} G^T (d - F lambda) (eq.
 * alphacompute, F applied implicitly in FP64) and u_i = K_reg,i^{-1} (f_i -
 * B~_i^T lambda_i) + R_i alpha_i (eq. solutionUeval).  u_d has sum n_i
 * entries (local DOF order per subdomain), alpha_d one per kernel vector.
 * Asynchronous. */
fetiF_status fetiF_primal(fetiF_ctx ctx, const double* f_d, const double* d_d, const double* lambda_d,
                          double* alpha_d, double* u_d, void* stream);

/* Copy F~_i of one subdomain to host_out as a full m_i x m_i row-major
 * matrix in the local multiplier order of create (test/debug hook).
 * Synchronises the device. */
fetiF_status fetiF_download_F(fetiF_ctx ctx, int32_t sub, double* host_out);

/* Sizes and work counts of a context (for reporting). */
typedef struct {
    int32_t nsub;
    int64_t n_lambda;
    int64_t sum_m;          /* sum of m_i */
    int64_t factor_values;  /* FP64 values of all supernodal panels */
    int64_t x_values;       /* FP64 values of the compact X_i */
    int64_t f_elements;     /* stored triangle elements (incl. row padding) */
    int64_t f_tri_elements; /* sum m_i (m_i+1)/2 */
    double trsm_flops;      /* algorithmic flops of the sparse-RHS TRSM */
    double syrk_flops;      /* algorithmic flops of the row-sparse SYRK */
    double factor_flops;    /* host numeric factorisation flops */
    int32_t trsm_levels;    /* launches of the level-scheduled TRSM */
    int32_t apply_groups;   /* work-groups of one apply */
    int64_t apply_elements; /* stored elements the apply streams (sum of packed triangles) */
    int32_t assembly_groups; /* groups of fetiF_factor_assemble (see fetiF_options) */
    double trsm_bwd_flops;  /* algorithmic flops of the TRSM path's backward solve (dense RHS:
                               sum over panels of (ns^2 + 2 ns nr) m_i); 0 on the SYRK path */
} fetiF_info;

fetiF_status fetiF_query(fetiF_ctx ctx, fetiF_info* info);

/* Phase timing with HIP events recorded on the caller's stream around each
 * device phase: 0 factor copy (H2D), 1 RHS initialisation, 2 forward TRSM
 * (all levels), 3 SYRK, 4 apply band kernel, 5 apply gather kernel,
 * 6 solves with the factors (implicit apply, dual RHS, adjoint), 7 backward
 * TRSM and 8 SpMM of the TRSM path (fetiF_set_assembly_path).  fetiF_profile_enable(ctx, 1) starts
 * recording (it inserts event records, so keep it off inside captured
 * graphs); fetiF_profile_read waits for the recorded events and adds their
 * elapsed times into ms[phase] / counts[phase] for phase < nphases, then
 * forgets them when reset != 0. */
#define FETIF_NPHASES 9
fetiF_status fetiF_profile_enable(fetiF_ctx ctx, int on);
fetiF_status fetiF_profile_read(fetiF_ctx ctx, int reset, double* ms, int64_t* counts, int32_t nphases);

/* Measurement aid, no part of the method: a streaming read of buf_d (bytes,
 * a multiple of 16) in which work-group g reads the contiguous region
 * [g region_bytes, (g+1) region_bytes) with 16-byte non-temporal loads and
 * writes the sum of its FP64 values to out_d[g] (ceil(bytes / region_bytes)
 * entries, caller-owned).  It gives the read rate of the access pattern of
 * the apply's bands (each work-group streams one contiguous stretch of a
 * packed triangle).  region_bytes: a multiple of 16384.  Asynchronous on the
 * current device; errors via fetiF_last_error(NULL). */
fetiF_status fetiF_read_probe(const void* buf_d, int64_t bytes, int64_t region_bytes, double* out_d, void* stream);

/* Release everything owned by the context (synchronises its device). */
fetiF_status fetiF_destroy(fetiF_ctx ctx);

/* Message of the last error of ctx (or of the last failed create when ctx is
 * NULL).  Valid until the next call on the same context. */
const char* fetiF_last_error(fetiF_ctx ctx);

/* ---------------------------------------------------------------------
 * Host-only analysis (no device needed): the ordering, symbolic analysis
 * and numeric factorisation of one K_reg that feed the device path
 * (Sec. III, symbolic and numeric stages).  For inspection and tests.
 * --------------------------------------------------------------------- */
typedef struct fetiF_hfactor_s* fetiF_hfactor;

/* Order, analyse and factor one subdomain's K_reg (values in CSR order). */
fetiF_status fetiF_host_factor(const fetiF_subdomain* sub, const double* k_vals,
                               const fetiF_options* opt, fetiF_hfactor* out);

/* n, number of stored factor entries (lower part of the supernodal panels,
 * explicit zeros included), supernodes and elimination-tree levels. */
fetiF_status fetiF_hfactor_info(fetiF_hfactor h, int32_t* n, int64_t* nnz, int32_t* nsuper,
                                int32_t* nlevels);

/* perm[k] = original DOF at position k; L as CSC (colptr[n+1], rowidx[nnz],
 * vals[nnz]) in the permuted order, so that L L^T = P K_reg P^T.
 * Any output pointer may be NULL. */
fetiF_status fetiF_hfactor_export(fetiF_hfactor h, int32_t* perm, int64_t* colptr,
                                  int32_t* rowidx, double* vals);

/* Supernode table: first column, columns, rows below the diagonal block,
 * parent supernode (-1 root) and height level, each [nsuper]. */
fetiF_status fetiF_hfactor_supernodes(fetiF_hfactor h, int32_t* first, int32_t* ncols,
                                      int32_t* nrows, int32_t* parent, int32_t* level);

void fetiF_hfactor_free(fetiF_hfactor h);

#ifdef __cplusplus
}
#endif
#endif /* FETIF_H */
