/*
 * mar.h - C ABI of the multiple-Arnoldi (mArnoldi) per-seed hot path, gfx950.
 *
 * The method (Sec. 2 of the paper): for the generalized shifted equations
 * (zS - H) x = b of Eq. (1), with H and S sparse, real symmetric and S
 * positive definite, the problem is reduced to one small nu x nu *standard*
 * eigenproblem per basis index j, posed in a Krylov subspace L_nu^(j) that
 * contains the unit vector e_j; the subspace eigen levels eps_alpha and
 * vectors v_alpha determine the Green's function and from it the energy.
 *
 * This library computes, for each requested seed j (0-based here; the paper
 * counts j = 1..M):
 *   1. the S-orthonormal basis K = [u_1 .. u_nu] of span{e_j, He_j, ...,
 *      H^(nu-1) e_j}, u_1 = e_j / sqrt(S_jj), by classical Gram-Schmidt with
 *      two passes (CGS2) in the S-inner product, and A = K^T H K from the dot
 *      products u_k . (H u_n) (k <= n), mirrored from its upper triangle;
 *   2. the eigenpairs (eps_alpha, y_alpha) of A in FP64, v_alpha = K y_alpha;
 *   3. the spin-summed density-matrix column on the pattern P(j) of H's row j,
 *        rho_ij = 2 sum_alpha f((eps_alpha - mu)/kT) (e_i.v_alpha)(e_j.v_alpha),
 *      f(x) = 1/(1+e^x) (kT = 0: step, 1/2 at eps = mu); the band-energy and
 *      electron-count contributions E_j = sum_{i in P(j)} rho_ij H_ij and
 *      N_j = sum_{i in P(j)} rho_ij S_ij; the weights
 *      w_alpha = (e_j^T S v_alpha)(v_alpha^T e_j); E_band = sum_j E_j.
 * Breakdown: when the S-norm beta of the new residual satisfies
 * beta <= tau * eta (eta^2 = |c1|^2 + |c2|^2 + beta^2 from the two projection
 * passes; tau = 1e-12 in FP64, 1e-5 in FP32) the subspace stops at
 * nu_eff = n vectors. Breakdown is not an error.
 *
 * Precision forms: MAR_FP64 runs everything in FP64. MAR_FP32 stores the
 * Krylov basis and runs the sparse products and the CGS2 projections/updates
 * in FP32 with FP32 accumulation; the norms and breakdown test, the subspace
 * eigensolve, the Fermi weighting and all energy sums stay FP64.
 *
 * Errors: every entry point returns a mar_status. Arguments are validated
 * before any device work; on error the outputs are unspecified and
 * mar_last_error() gives a message. No exception crosses this boundary.
 * A context serves one solve at a time and is not thread-safe.
 */
#ifndef MAR_H
#define MAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mar_ctx mar_ctx;

typedef enum {
    MAR_OK = 0,
    MAR_ERR_ARG = -1,      /* bad argument (sizes, nu, kT, seeds, NULL outputs) */
    MAR_ERR_PATTERN = -2,  /* malformed CSR, asymmetric H or S, pattern(S) not in pattern(H) */
    MAR_ERR_NOT_SPD = -3,  /* S_jj <= 0 at create, or w^T S w < 0 during a solve */
    MAR_ERR_NOMEM = -4,    /* device allocation failed */
    MAR_ERR_HIP = -5,      /* HIP runtime error (message in mar_last_error) */
    MAR_ERR_STATE = -6,    /* NULL context or use after an unrecoverable error */
    MAR_ERR_NOCONV = -7    /* the subspace eigensolve of some seed did not converge (nu_eff = -3) */
} mar_status;

/* MAR_FP64: every step in FP64.
 * MAR_FP32: the Krylov basis is stored in FP32, and the sparse products and both Gram-Schmidt sweeps run in
 * FP32 with FP32 sums in registers and FP64 partial sums across workgroups; in the delayed schedule with
 * nu > 128 the update sweep keeps its running sums over the slabs in FP64 and rounds them once when stored.
 * Coefficients, norms, breakdown tests, the subspace eigensolve, the Fermi weighting and the energy sums
 * are FP64 in both. */
typedef enum { MAR_FP64 = 0, MAR_FP32 = 1 } mar_precision;

/* MAR_FORM_PLAIN: one seed at a time (B = 1), one kernel launch per phase.
 * MAR_FORM_BATCHED: B seeds per block with seed-interleaved vectors. */
typedef enum { MAR_FORM_BATCHED = 0, MAR_FORM_PLAIN = 1 } mar_form;

/* CGS2 schedules. Both run two classical Gram-Schmidt passes per new vector
 * in the S-inner product and give the same subspace and A = K^T H K up to
 * rounding.
 * TEXTBOOK: per step w = H u_n, h = K^T w and c1 = (S K)^T w in one pass,
 *   w -= K c1, c2 = (S K)^T w, w -= K c2, then S w; K and S K are stored
 *   (five basis passes per step).
 * DELAYED: the second pass of a vector is merged with the first pass of the
 *   next one. The SpMMs act on the once-orthogonalized vector u~ (y = H u~);
 *   one sweep over K gives K^T S u~, K^T S y and K^T y; one update sweep
 *   finishes u_n = (u~ - K c2)/gamma and the first-pass residual of y. The
 *   relation H K = K R (R: the Gram-Schmidt coefficients) carries the change
 *   from H u~ to H u_n into A and the coefficients; only K is stored (two basis
 *   passes per step). The breakdown test on the two-pass norm runs one step
 *   later, plus a first-pass test. The products of the unnormalized residual
 *   with itself are cubic in the scale of H, so this schedule needs the
 *   entries of H within about 2^-300 ... 2^300 in magnitude (the textbook
 *   schedule, whose vectors are normalized every step, about 2^-480 ... 2^480).
 * AUTO: TEXTBOOK for the plain form, DELAYED for the batched form. */
typedef enum { MAR_SCHED_AUTO = 0, MAR_SCHED_TEXTBOOK = 1, MAR_SCHED_DELAYED = 2 } mar_schedule;

typedef struct {
    int32_t seed_block;    /* B for the batched form: power of two, 1..256 (FP32) or 1..128
                              (FP64); 0 = choose from the problem size */
    int32_t schedule;      /* mar_schedule */
    int32_t proj_wgs;      /* workgroup cap of a delayed-schedule projection sweep (0 = as many as
                              the device holds at once) */
    int32_t slab_pad_kb;   /* extra KiB between consecutive basis slabs (0 = 1 KiB) */
    int32_t proj_variant;  /* delayed-schedule projection, slabs x 16-byte vectors per thread and row
                              tile: 0 = 4 x 4, or, when the solve's widest sweep of nu + 3 slabs
                              exceeds 512 MB (outside local regions), variant 7 (variant 2 at nu <= 64
                              and for the FP32 form at nu > 128); 1 = 8 x 4, 2 = 4 x 4 with
                              non-temporal basis loads, 3 = 4 x 2, 4 = 8 x 2, 5 = 6 x 4, 6 = 6 x 2,
                              7 = 8 x 4 with non-temporal basis loads */
    int32_t upd_q;         /* delayed-schedule update: 16-byte vectors per thread, 2/4/8 (0 = 4) */
    int32_t support_off;   /* 1 = stream every row of every slab; 0 (default) = skip, in the batched
                              delayed schedule on a 4x4-block H, the row tiles where all vectors of the
                              seed block are exactly zero (farther from each seed than the step, in hops
                              of H's pattern). The results differ only in the order of partial sums. */
    int32_t two_streams;   /* with two or more seed blocks: 3 = one block at a time on the caller's
                              stream, each block's subspace eigensolve on the context's second
                              stream, overlapping the next block's sweeps (two copies of the subspace
                              matrices); 1 = alternate whole blocks between two workspaces and the two
                              streams, so that one block's short FP64 kernels overlap the other's
                              sweeps (only when both workspaces fit in 160 GB); 2 = everything on the
                              caller's stream; 0 (default) = 1 for local regions of 6 hops or more
                              (3 when the two workspaces do not fit in 160 GB or in the
                              device's free memory), else 3. Neither overlap is used
                              while profiling, for the
                              eigen-state passes or inside mar_solve_many's graphs; the caller's stream
                              waits for the second one before the solve's last kernel. The results do
                              not depend on it. */
    int32_t eig_max_sweeps; /* Jacobi sweeps allowed to the nu x nu subspace eigensolve (0 = 40; about
                              ten are needed at nu = 100). A seed whose eigensolve has not converged
                              after them gets nu_eff = -3 (see mar_solve). */
} mar_tuning;

/* Create a context from host CSR arrays of H and S (M x M, 0-based, columns
 * sorted and unique in each row, rowptr[0] = 0). The arrays are copied to the
 * device; the caller keeps ownership. Validation (MAR_ERR_PATTERN unless
 * noted): rowptr monotone, columns in range, values finite (MAR_ERR_ARG), H and
 * S symmetric in pattern and value (exact equality), every stored entry of S
 * also stored in H, S_jj > 0 (MAR_ERR_NOT_SPD), at most 63 stored entries per
 * row of H (MAR_ERR_ARG). Full positive definiteness of S is not checked here.
 * A 4x4 block structure (identical patterns in rows 4I..4I+3 made of aligned
 * 4-column groups) is detected and stored as BSR; otherwise CSR is used.
 * Returns MAR_ERR_HIP if no GPU is usable. */
mar_status mar_create(int64_t M,
                      const int64_t* H_rowptr, const int32_t* H_col, const double* H_val,
                      const int64_t* S_rowptr, const int32_t* S_col, const double* S_val,
                      mar_ctx** out);

void mar_destroy(mar_ctx* ctx);

/* Host-side solve (blocking). seeds: n_seeds distinct indices in [0, M)
 * (MAR_ERR_ARG otherwise); 1 <= nu <= M; mu finite; kT >= 0 and finite.
 * The subspace eigensolve (Sec. 2: the nu x nu standard eigenproblem) is the
 * parallel cyclic Jacobi method; a seed whose eigensolve has not converged
 * after eig_max_sweeps sweeps (mar_tuning) gets nu_eff = -3, NaN in its rho
 * slots, E_j, N_j, eps and weight entries (so e_band is NaN), and the call
 * returns MAR_ERR_NOCONV naming the seed.
 * Outputs (host, caller-allocated):
 *   rho     [nnz(H)]   CSR row j slots of each listed seed j receive rho_ij for
 *                      i in P(j) (slot (j,i) holds rho_ij); all other slots keep
 *                      the caller's values. Required.
 *   e_band  [1]        sum of E_j over the listed seeds (fixed-order FP64). Required.
 *   e_seed  [n_seeds]  E_j, or NULL.
 *   n_seed  [n_seeds]  N_j, or NULL.
 *   nu_eff  [n_seeds]  subspace dimension reached, or NULL.
 *   eps     [n_seeds * nu] subspace eigen levels of seed s at eps[s*nu + a],
 *                      a < nu_eff (unsorted; remaining entries 0), or NULL.
 *   weight  [n_seeds * nu] w_alpha in the same layout, or NULL.
 * Returns MAR_ERR_NOT_SPD if some seed met w^T S w < 0. */
mar_status mar_solve(mar_ctx* ctx, const int32_t* seeds, int64_t n_seeds, int32_t nu,
                     double mu, double kT, mar_precision prec, mar_form form,
                     double* rho, double* e_band, double* e_seed, double* n_seed,
                     int32_t* nu_eff, double* eps, double* weight);

/* Device-side solve, enqueued on hip_stream (a hipStream_t; NULL = the null
 * stream) without host synchronization. All pointers are device pointers with
 * the same meaning and layout as in mar_solve; d_seeds is read on the device,
 * so range and uniqueness are not validated on the host: a seed outside
 * [0, M) gets d_nu_eff = -2 and no other output, a seed that met w^T S w < 0
 * gets d_nu_eff = -1, a seed whose subspace eigensolve did not converge
 * d_nu_eff = -3 and NaN outputs (d_nu_eff must be non-NULL to see these). Scalar
 * arguments are validated as in mar_solve. The device workspace is owned by
 * the context and may be reallocated (hipMalloc) when nu, B, or the precision
 * grows; call once with the largest shapes before capturing. */
mar_status mar_solve_async(mar_ctx* ctx, const int32_t* d_seeds, int64_t n_seeds, int32_t nu,
                           double mu, double kT, mar_precision prec, mar_form form,
                           double* d_rho, double* d_e_band, double* d_e_seed, double* d_n_seed,
                           int32_t* d_nu_eff, double* d_eps, double* d_weight, void* hip_stream);

/* ---- the solve without device allocation ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * arguments, outputs and errors as mar_solve_async, but the solve runs on a
 * static device array of MAR_NOALLOC_SCRATCH_BYTES instead of the context's
 * workspace, and the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine; per-kernel timing is suspended for the call).
 * Every GPU the library runs on holds the array until the process ends; its
 * address is looked up at the first call on each device. With the batched
 * form and no seed block fixed by mar_set_tuning, the planned block is halved
 * until the solve's workspace fits the array; a solve that does not fit even
 * then (or with the block fixed) is refused with MAR_ERR_ARG and the needed
 * size in mar_last_error (about nu * M * B * 4 bytes of FP32 basis for blocks
 * of B seeds: M = 16384, nu = 30 runs FP32 blocks of up to 16-32 seeds). All
 * calls on one GPU share the array and it keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other threads, other
 * contexts) race and must be serialized by the caller. */
#define MAR_NOALLOC_SCRATCH_BYTES (64ull << 20)
mar_status mar_solve_async_noalloc(mar_ctx* ctx, const int32_t* d_seeds, int64_t n_seeds, int32_t nu, double mu,
                                   double kT, mar_precision prec, mar_form form, double* d_rho, double* d_e_band,
                                   double* d_e_seed, double* d_n_seed, int32_t* d_nu_eff, double* d_eps,
                                   double* d_weight, void* hip_stream);

/* ---- Fermi level found on the device ----
 * The method takes the chemical potential mu as given (Sec. 2: the subspace
 * levels give the Green's function, and from it the energy at mu). These
 * entry points find it instead: the subspace eigenpairs of every listed seed
 * are computed first (levels, weights and the rows e_i.v_alpha, i in P(j),
 * kept on the device), then mu is bisected on the device, 200 halvings of
 * [min eps - 40 kT, max eps + 40 kT] over all kept levels, so that
 *     N(mu) = sum_j 2 sum_alpha f((eps_alpha^(j) - mu)/kT) w_alpha^(j) = n_target
 * (half filling of a seed sample: n_target = n_seeds), and rho, E_j, N_j and
 * E_band are assembled at that mu. No second Krylov pass. Where N(mu) is not
 * monotone (some w_alpha < 0 when S != I) the bisection returns a root inside
 * the bracket. Arguments and outputs as in mar_solve_async / mar_solve, plus
 * n_target (finite, >= 0) and mu (one double, device or host) receiving the
 * level. The kept rows take n_seeds * nu * (max row length of H) * 8 bytes of
 * device memory, owned by the context. */
mar_status mar_solve_fermi_async(mar_ctx* ctx, const int32_t* d_seeds, int64_t n_seeds, int32_t nu,
                                 double n_target, double kT, mar_precision prec, mar_form form,
                                 double* d_rho, double* d_e_band, double* d_e_seed, double* d_n_seed,
                                 int32_t* d_nu_eff, double* d_eps, double* d_weight, double* d_mu,
                                 void* hip_stream);
mar_status mar_solve_fermi(mar_ctx* ctx, const int32_t* seeds, int64_t n_seeds, int32_t nu, double n_target,
                           double kT, mar_precision prec, mar_form form, double* rho, double* e_band,
                           double* mu, double* e_seed, double* n_seed, int32_t* nu_eff, double* eps,
                           double* weight);

/* ---- eigen states (Sec. 3, Eq. 3; Appendix) ----
 * The k-th eigen level and the components of its eigenvector over the listed
 * seeds, from the same subspaces. With the weights w_alpha^(j) of every listed
 * seed, the integrated density of states is
 *     n(eta) = sum_j sum_alpha w_alpha^(j) F((eta - eps_alpha^(j)) / sigma)
 * (F the logistic step 1/(1+e^-x); sigma = 0: the unit step, 1/2 at 0), so that
 * n(+inf) = n_seeds; eta(n) is its inverse, found by 200 halvings of
 * [min eps - 1, max eps + 1]. The level is eps_k = eta(k - 1/2), and (Eq. 3,
 * with the delta smoothed to the derivative of F(x/sigma))
 *     e_j^T phi_k = sum_alpha s_alpha^(j) (e_j^T v_alpha^(j))
 *                   [F((eta(k) - eps_alpha^(j))/sigma) - F((eta(k-1) - eps_alpha^(j))/sigma)],
 * where s_alpha^(j) = +1 or -1 makes v_ref . v_alpha^(j) >= 0 (inner-product
 * method), v_ref being the subspace eigenvector with the largest
 * |(e_j^T v_alpha^(j)) x window| over all listed seeds. Cost: every listed seed
 * is solved twice (levels and reference first, signs second) plus the
 * reference seed alone in the plain form. With all M seeds listed and
 * nu = M the result is the exact S-normalized generalized eigenvector up to one
 * global sign. Arguments: 1 <= k <= n_seeds, sigma finite and >= 0, the rest as
 * in mar_solve_async. Outputs: phi [n_seeds] (component of each listed seed, in
 * list order), levels [3] = {eps_k, eta(k-1), eta(k)}, ref [3] = {position in
 * the list, alpha, seed} of the reference (or NULL). Host variant: host arrays. */
mar_status mar_eigen_state_async(mar_ctx* ctx, const int32_t* d_seeds, int64_t n_seeds, int32_t nu, int32_t k,
                                 double sigma, mar_precision prec, mar_form form, double* d_phi,
                                 double* d_levels, int32_t* d_ref, void* hip_stream);
mar_status mar_eigen_state(mar_ctx* ctx, const int32_t* seeds, int64_t n_seeds, int32_t nu, int32_t k,
                           double sigma, mar_precision prec, mar_form form, double* phi, double* levels,
                           int32_t* ref);

/* ---- several independent systems in one launch ----
 * One request per context: the same arguments as mar_solve_async (device
 * pointers, validated the same way). */
typedef struct {
    const int32_t* d_seeds;
    int64_t n_seeds;
    int32_t nu;
    double mu, kT;
    mar_precision prec;
    mar_form form;
    double* d_rho;
    double* d_e_band;
    double* d_e_seed;     /* or NULL */
    double* d_n_seed;     /* or NULL */
    int32_t* d_nu_eff;    /* or NULL */
    double* d_eps;        /* or NULL */
    double* d_weight;     /* or NULL */
} mar_request;

/* Solve n_sys independent systems (the Sec. 2 per-seed problem of each system,
 * as in mar_solve_async) with one graph launch on hip_stream: the launch
 * sequences of all systems are captured into one HIP graph as parallel
 * branches, so systems of uneven size and nu overlap on the device. Contexts
 * must be distinct and on the current device. The instantiated graph is cached
 * under the exact request set (contexts, pointers, sizes, scalars and the
 * resolved block sizes): calling again with identical requests replays it
 * without capture, so a caller that refills the same seed buffers pays one
 * capture. Workspaces are sized (and allocated) before the capture. Errors are
 * reported on the context of the failing request (on ctx[0] for errors of the
 * call itself). Cached graphs of a context are released by mar_destroy.
 * A context that has run any solve with two seed blocks in flight (two_streams
 * 1, or the default for local regions of 6 hops or more) is refused with
 * MAR_ERR_STATE for the rest of its life: host crashes followed a capture
 * after such solves, and their cause is not known. Contexts meant for graphs
 * keep two_streams 3 or 2 from their creation on. */
mar_status mar_solve_many(int32_t n_sys, mar_ctx* const* ctx, const mar_request* req, void* hip_stream);

/* Autotuner: time the batched form on the first min(n_seeds, 256) of d_seeds
 * (device) for every block size B (powers of two allowed by the precision and
 * the 128 GB basis budget) and, for the delayed schedule, the projection tile
 * variants 0 and 3; keep the fastest (B, variant) for (nu, prec) in the context.
 * Later batched solves with seed_block = 0 and proj_variant = 0 in the tuning
 * use it. Outputs of the probe solves go to a context-owned scratch buffer;
 * the call synchronizes hip_stream. best_block (or NULL) receives B;
 * best_rate (or NULL) the probe throughput in seed-subspaces/s. */
mar_status mar_autotune(mar_ctx* ctx, int32_t nu, mar_precision prec, const int32_t* d_seeds, int64_t n_seeds,
                        double mu, double kT, void* hip_stream, int32_t* best_block, int32_t* best_variant,
                        double* best_rate);

/* Local flipping refinement of one eigenvector (Appendix). The signs of the
 * components a_l of phi (level eps) are flipped one at a time when that lowers
 *     R = |r|^2 (+ c (phi_ref^T S phi)^2),   r = (H - eps S) phi,
 * the penalty acting as an orthogonality constraint to an earlier state
 * phi_ref (the paper uses c = 5 atomic units, 5 x 27.211386^2 eV^2 for
 * matrices in eV). A flip changes r only on the rows of P(l), so no matrix
 * product is needed after the first residual. Rows are visited by colour of a
 * greedy distance-2 colouring of H's pattern (row l takes the smallest colour
 * unused by earlier rows within two hops; built on the first call and kept),
 * and in index order within a colour. Row l flips when its single-flip change
 *     dR_l = sum_{i in P(l)} A_il (4 a_l^2 A_il - 4 a_l r_i)
 *            + c (4 a_l^2 s_l^2 - 4 a_l s_l p) < 0,   A = H - eps S, s = S phi_ref,
 * is negative, on the current r and p: every accepted flip lowers R. Rows of
 * one colour have disjoint supports, so the first sum does not depend on the
 * colour's other flips; without the penalty the colour's rows decide at once,
 * with it they decide one after the other on the p left by the flips before
 * (p drops by 2 a_l s_l at each flip). A sweep visits every colour; sweeps
 * repeat until one flips nothing or max_sweeps have run. Sums run in fixed
 * orders with separately rounded products, so the decisions are reproducible.
 *   d_phi     [M] device, FP64, in/out.
 *   d_phi_ref [M] device or NULL (no penalty when NULL or c == 0).
 *   d_R       [max_sweeps + 1] device or NULL: R before the first sweep and after
 *             each sweep run (later entries untouched).
 *   d_info    [2] device or NULL: sweeps run, flips made.
 * One workgroup on the caller's stream; asynchronous. The context keeps a
 * workspace of 25 M bytes for it (allocated at the first call). MAR_ERR_ARG for
 * a NULL phi, eps or c not finite, c < 0 or max_sweeps < 0. */
mar_status mar_local_flip(mar_ctx* ctx, double* d_phi, double eps, const double* d_phi_ref, double c,
                          int32_t max_sweeps, double* d_R, int32_t* d_info, void* hip_stream);
/* Number of colours of that colouring (built if needed; synchronous); -1 on error. */
int32_t mar_flip_colours(mar_ctx* ctx);

/* Local regions: the order-N form of the method (Sec. 1 gives its cost as
 * proportional to the number of atoms, so the work of one seed may not grow
 * with the system; how the subspace is kept local is left to the cited mArnoldi
 * paper). hops >= 0: later solves of ctx generate the Krylov subspace of seed j
 * inside its local region R_j, the rows whose 4-row block lies within `hops`
 * hops of j's block in the graph of H's 4x4 block pattern (0 = j's block
 * alone): the method runs on the principal submatrices H[R_j, R_j] and
 * S[R_j, R_j], and rho_ij for i in P(j) outside R_j is 0. The regions are per
 * seed, so results do not depend on the seed order or the block size (up to
 * the order of partial sums). hops < 0 (the default) restores the full system.
 * Needs H with 4x4 block structure (MAR_ERR_ARG here otherwise); solves then
 * need the batched delayed form with blocks of at least 4 (FP32) / 2 (FP64)
 * seeds, and the eigen-state entry points refuse a local region (MAR_ERR_ARG). */
mar_status mar_set_local_region(mar_ctx* ctx, int32_t hops);
/* Current local-region hops of ctx (-1: the full system, or ctx NULL). */
int32_t mar_local_region(const mar_ctx* ctx);

/* Set the tuning used by later solves. NULL restores the defaults (every
 * field 0): later batched solves then use the (B, projection variant) that
 * mar_autotune kept for their (nu, precision) on this context, when it ran,
 * else the widest block whose basis fits in 128 GB. A nonzero seed_block or
 * proj_variant overrides the autotuned choice. */
mar_status mar_set_tuning(mar_ctx* ctx, const mar_tuning* t);
mar_status mar_get_tuning(const mar_ctx* ctx, mar_tuning* t);

/* Seeds per block the batched form would use for (nu, prec) with the current tuning. */
int32_t mar_seed_block(const mar_ctx* ctx, int32_t nu, mar_precision prec);

/* Last error message of ctx, or of the calling thread's last mar_create when
 * ctx is NULL. Never NULL; valid until the next call on the same context. */
const char* mar_last_error(const mar_ctx* ctx);

/* ---- per-kernel timing (HIP events on the solve stream) ----
 * While enabled, each kernel launch of a solve is bracketed by a pair of HIP
 * events on the launch stream. mar_profile_collect synchronizes those events
 * and accumulates, per kernel class, the launch count, the summed event time
 * and the algorithmic bytes and flops (bytes: every operand read once and
 * every result written once, as the method requires). */
enum { MAR_PROF_CLASSES = 16 };
typedef struct {
    char name[24];
    int64_t launches;
    double ms;        /* summed launch durations */
    double bytes;     /* summed algorithmic bytes */
    double flops;     /* summed algorithmic flops */
} mar_prof_entry;

mar_status mar_profile_enable(mar_ctx* ctx, int32_t on);
mar_status mar_profile_reset(mar_ctx* ctx);
mar_status mar_profile_collect(mar_ctx* ctx, mar_prof_entry* out /* [MAR_PROF_CLASSES] */,
                               int32_t* n_out);

/* Identity of the build: the first 16 hex digits of the SHA-256 over the
 * library's source files and this header, as the build script computed them
 * (static string, never NULL). */
const char* mar_build_id(void);

/* Library description: matrix storage actually used (1 = BSR 4x4 for H, 2 = for S). */
int32_t mar_ctx_info(const mar_ctx* ctx, int64_t* M, int64_t* nnz_H, int64_t* nnz_S);

#ifdef __cplusplus
}
#endif
#endif /* MAR_H */
