/*
 * bfc.h -- C ABI of the MI355X butterfly-completion library (libbfc.so).
 *
 * The library completes an n x n complex matrix T from a set of observed
 * entries (i, j, t_ij) in the tensorized butterfly format of Singh,
 * Solomonik, Li and Liu, "Efficient Tensor Completion Algorithms for Highly
 * Oscillatory Operators":
 *
 *   n = c * 2^L; row i has digits i_l = floor(i / (c 2^(L-l-1))) mod 2 for
 *   l < L (i_0 most significant) and i_L = i mod c (Sec. 4.1, eq. (indices));
 *   same for columns j.
 *
 *   Cores (App. A.2, eq. (reshaped_tensors), psi^{-1} most-significant first):
 *     core 0       Z^1     n x r              row i
 *     core m=1..L  Z^(m+1) 2^(L+1) x r x r    slice k = psi^{-1}(i_0..i_(L-m), j_0..j_(m-1))
 *                                             = ((ib >> (m-1)) << m) | (jb >> (L-m)),
 *                                             ib = i / c, jb = j / c
 *     core L+1     Z^(L+2) n x r              column j
 *
 *   Entry (Sec. 4.1, eq. (BF_tensor_rep)):
 *     x_ij = Z^1[i] Z^2[k_2] ... Z^(L+1)[k_(L+1)] Z^(L+2)[j]^T
 *
 *   Objective (Sec. 5, eq. (BF_objective)): 1/2 ||P_Omega(T - X)||_F^2.
 *
 * bfc_sweep_core performs one core update of the ALS method (Sec. 5.1.1,
 * Alg. "ALS for Butterfly Completion"): every fiber of Z^1 / Z^(L+2) or slice
 * of an inner core is the solution of the regularized normal equations of
 * the observed entries it touches,
 *     (K + lam I) s = y + lam s_old        (proximal, default)
 *     (K + lam I) s = y                    (ridge)
 * with K = sum conj(a) a^T, y = sum conj(a) t and
 * lam = max(reg_rel, d * u) * trace(K) / d, u the rounding level described
 * at bfc_init_cores (the regularization floor).
 * A fiber or slice with no observed entry keeps its values.  Inner-core
 * slices are stored row-major: s[a*r + b] = Z[k][a][b].
 *
 * Memory and layout conventions (all calls):
 *   - Complex numbers are interleaved (re, im) pairs of doubles (complex128)
 *     at the ABI, whatever the internal precision.
 *   - Index arrays are int32, values in [0, n).
 *   - Pointers named d_* are DEVICE pointers (HIP device memory of the
 *     current device); the caller owns them.  The library copies what it
 *     needs during bfc_init_cores and keeps no caller pointer afterwards.
 *   - Every call takes a hipStream_t (as void*, NULL = default stream) and
 *     enqueues its work there.  bfc_init_cores, bfc_residual and
 *     bfc_sync_status synchronize that stream before returning; the others
 *     return as soon as the work is enqueued.
 *   - Cores layout for get/set/init: core 0 (n*r values, row-major), then
 *     cores 1..L (2^(L+1)*r*r each, slice-major then row-major), then core
 *     L+1 (n*r) -- bfc_num_params(n, L, r) complex values in total.
 *
 * Errors: every function returns a bfc_status; nothing throws or aborts
 * across the ABI.  A message for the last error of the calling thread is
 * returned by bfc_last_error().  Solve failures inside enqueued work (a
 * block whose regularized K is not positive definite) leave that block's
 * old values in place and are reported by the next bfc_sync_status or
 * bfc_residual call on the problem.
 */
#ifndef BFC_H
#define BFC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bfc_status;
#define BFC_OK 0
#define BFC_EINVAL 1      /* bad argument: sizes, ranges, null pointers       */
#define BFC_ENOMEM 2      /* device allocation failed                         */
#define BFC_EHIP 3        /* a HIP runtime call failed                        */
#define BFC_ENOTSPD 4     /* a regularized normal-equation matrix was not SPD */
#define BFC_ENONFINITE 5  /* NaN or Inf in an input value                     */

/* arithmetic modes */
#define BFC_C128 0        /* complex128 cores and contractions, FP64 Gram, FP64 solves        */
#define BFC_C64 1         /* complex64 cores and contractions, FP32 Gram, FP64 solves          */
#define BFC_C64_BF16GRAM 2 /* as BFC_C64 but the inner cores' Gram/right-hand-side products
                             take bf16 inputs (FP32 accumulation on the BF16 matrix cores):
                             every FP32 row value x is split as x = h + m + l with h, m, l
                             bf16 (h = bf16(x), m = bf16(x - h), l = bf16(x - h - m)) and the
                             products h h' + h m' + m h' + h l' + m m' + l h' are summed, so
                             the Gram keeps FP32-level accuracy; each inner FP64 solve is
                             followed by one refinement step whose residual
                             sum conj(a_e)(t_e - a_e.s) is recomputed from the entries in
                             FP32, solved with the same factor and regularization (the outer
                             cores' Grams stay FP32)                                            */

/* regularization forms (the paper leaves the regularization unspecified) */
#define BFC_REG_PROXIMAL 0
#define BFC_REG_RIDGE 1

/* Ranks: the ALS sweep (bfc_sweep_core, bfc_sweep), reconstruction and the
 * residual calls take 1 <= r <= BFC_MAX_RANK.  Every other call (ADAM, ADF,
 * the loss gradient, batches, work-item sizes, the low-rank conversion) and
 * the BFC_C64_BF16GRAM mode need r <= BFC_MAX_RANK_FULL and return EINVAL
 * above it.  From r = BFC_MAX_RANK_FULL + 1 (the ranks 10 - 12 of the c = 4
 * examples of Sec. 6.1 and 6.3) an inner slice's system (d = r^2 unknowns)
 * is built and solved by one fused kernel per slice, with a region of
 * device memory of its own for the real Gram and the factor.             */
#define BFC_MAX_RANK 12
#define BFC_MAX_RANK_FULL 8
#define BFC_MAX_LEVELS 24

typedef struct bfc_config {
    int64_t n;          /* matrix size; n = c * 2^L with c >= 1 an integer          */
    int32_t L;          /* butterfly levels, 0 <= L <= BFC_MAX_LEVELS                */
    int32_t r;          /* rank, 1 <= r <= BFC_MAX_RANK                              */
    int32_t precision;  /* BFC_C128, BFC_C64 or BFC_C64_BF16GRAM                     */
    int32_t reg_mode;   /* BFC_REG_PROXIMAL or BFC_REG_RIDGE                         */
    double reg_rel;     /* relative regularization, >= 0: lam = max(reg_rel, d u) trace(K)/d */
    uint64_t seed;      /* random start when bfc_init_cores gets no initial cores    */
    double reg_floor;   /* lower bound on u, in [0, 2^-4]; 0 keeps the mode's own u_K.
                           An FP64 run with reg_floor = 2^-20 uses exactly the
                           regularization of the complex64 modes, so the two
                           differ only in their arithmetic                           */
} bfc_config;

typedef struct bfc_problem bfc_problem;

/* Number of complex parameters 2 n r + L 2^(L+1) r^2 (Sec. 3.2). */
int64_t bfc_num_params(int64_t n, int32_t L, int32_t r);

/*
 * Build a completion problem from nnz observed entries (d_rows[e], d_cols[e],
 * d_vals[e]) (Sec. 5, the set Omega of eq. (BF_objective)).  Duplicated
 * pairs are kept and count as separate least-squares rows.  The library
 * computes every entry's block keys, sorts a private copy of the entries per
 * core by block (and, inside inner-core slices, by row or column), and sets
 * the starting cores: d_cores_init (bfc_num_params complex128 values, layout
 * above) or, when NULL, i.i.d. complex Gaussian values CN(0, 1/r) drawn from
 * a counter-based generator keyed by cfg->seed.
 *
 * Regularization used by every later core update: with tau = trace(K)/d,
 * lam = max(reg_rel, d * u) * tau, u = max(u_K, cfg->reg_floor), where u_K
 * is the rounding level of the Gram accumulation (0 in BFC_C128; 2^-20 for
 * the FP32-accumulated Grams of the complex64 modes: the FP32 unit roundoff
 * 2^-24 times the sqrt(256) growth of the sums forming them; the same 2^-20
 * for the inner Grams of BFC_C64_BF16GRAM, whose bf16 inputs are split in
 * three bf16 parts; 0 again for BFC_C64 at r > BFC_MAX_RANK_FULL, where the
 * Grams are accumulated in FP64 from the complex64 values), so that
 * rounding cannot make K + lam I indefinite.  If
 * the FP64 Cholesky factorization still fails while lam > 0, lam is raised to
 * max(100 lam, d max(u, 2^-53) tau), at most three times.
 * Returns EINVAL for nnz < 1, a bad config (n not c*2^L, r or L out of
 * range, negative reg_rel) or an index outside [0, n); ENONFINITE for a
 * non-finite value; ENOMEM when device memory runs out.  On success *out
 * owns all device memory of the problem until bfc_destroy.
 */
bfc_status bfc_init_cores(const bfc_config* cfg, int64_t nnz,
                          const int32_t* d_rows, const int32_t* d_cols,
                          const void* d_vals, const void* d_cores_init,
                          void* hip_stream, bfc_problem** out);

/*
 * One ALS core update (Alg. "ALS for Butterfly Completion", one value of its
 * core loop): core = 0 .. L+1 (the paper's S^(core+1)).  All other cores are
 * read at their current values.  Asynchronous on hip_stream.
 */
bfc_status bfc_sweep_core(bfc_problem* p, int32_t core, void* hip_stream);

/*
 * One full ALS iteration: cores 0, 1, ..., L+1 in that order.  Asynchronous.
 * On a non-default stream, with graphs enabled (the default) and per-kernel
 * profiling off, the sweep's kernels are captured once into a HIP graph and
 * replayed on later calls; the results are the same as issuing the core
 * updates one by one.
 */
bfc_status bfc_sweep(bfc_problem* p, void* hip_stream);

/* Enable (default) or disable the graph replay of bfc_sweep. */
bfc_status bfc_use_graphs(bfc_problem* p, int32_t enable);

/*
 * x_ij for m listed pairs (eq. (BF_tensor_rep)), written to d_out as m
 * complex128 values.  m = 0 is allowed (no work).  A pair with an index
 * outside [0, n) gets NaN (nothing outside the cores is read).  Asynchronous.
 */
bfc_status bfc_predict_entries(const bfc_problem* p, int64_t m,
                               const int32_t* d_rows, const int32_t* d_cols,
                               void* d_out, void* hip_stream);

/*
 * out_sq[0] = sum |t - x|^2 and out_sq[1] = sum |t|^2 over m listed entries
 * (the two norms of eq. (BF_convergence)), accumulated in FP64 in a fixed
 * order (bitwise reproducible); an index outside [0, n) makes out_sq[0] NaN.
 * out_sq is HOST memory.  Synchronizes.
 * Also reports (and clears) pending solve failures: returns ENOTSPD after
 * filling out_sq if any block failed since the last report.
 */
bfc_status bfc_residual(const bfc_problem* p, int64_t m, const int32_t* d_rows,
                        const int32_t* d_cols, const void* d_vals, double out_sq[2],
                        void* hip_stream);

/*
 * The same two norms over the problem's own observed entries (the training
 * error of eq. (BF_convergence)), from the environments the sweep keeps:
 * x = (left environment of the last core) . Z^(L+2)[j].  The observed values
 * are taken in the problem's compute precision.  Synchronizes; reports
 * pending solve failures like bfc_residual.
 */
bfc_status bfc_residual_observed(bfc_problem* p, double out_sq[2], void* hip_stream);

/*
 * The relative error of eq. (BF_convergence), ||P(T - X)|| / ||P T||, over
 * the listed entries (bfc_relative_error, arguments as bfc_residual) or over
 * the problem's own observed entries (bfc_relative_error_observed, the
 * training error, as bfc_residual_observed): sqrt(out_sq[0] / out_sq[1])
 * from the two FP64 norms (sqrt(out_sq[0]) when ||P T|| = 0), written to
 * *out (HOST).  Synchronizes; returns ENOTSPD, after writing *out, when solve
 * failures were pending (and clears them), like the residual calls.
 */
bfc_status bfc_relative_error(const bfc_problem* p, int64_t m, const int32_t* d_rows,
                              const int32_t* d_cols, const void* d_vals, double* out,
                              void* hip_stream);
bfc_status bfc_relative_error_observed(bfc_problem* p, double* out, void* hip_stream);

/* Copy the cores out to / in from d_cores (bfc_num_params complex128 values). */
bfc_status bfc_get_cores(const bfc_problem* p, void* d_cores, void* hip_stream);
bfc_status bfc_set_cores(bfc_problem* p, const void* d_cores, void* hip_stream);

/*
 * The same as bfc_set_cores from FP32 values: d_cores holds
 * bfc_num_params(n, L, r) complex values as interleaved (re, im) floats in
 * the bfc_get_cores layout (device, caller owned), e.g. the output of a
 * network that proposes starting cores.  Asynchronous.
 */
bfc_status bfc_set_cores_f32(bfc_problem* p, const float* d_cores, void* hip_stream);

/*
 * Replace the observed values t_e, keeping the observed index pairs (and so
 * every sorted layout built by bfc_init_cores): d_vals is device complex128,
 * nnz values in the order the pairs were given to bfc_init_cores.  Used to
 * fit the same sample of positions to another matrix.  Synchronizes
 * hip_stream; BFC_ENONFINITE if a value is NaN or Inf (the layout then holds
 * the given values, the caller should replace them).
 */
bfc_status bfc_set_values(bfc_problem* p, const void* d_vals, void* hip_stream);

/*
 * Gradient of phi = 1/2 ||P_Omega(X - T)||^2 (Sec. 5.1.2: eq.
 * (grad_butterfly_1), (grad_butterfly_l), (grad_butterfly_last)) with respect
 * to every core at the current cores, none of which moves: per core the
 * Wirtinger gradient g = sum_e conj(a_e)(x_e - t_e) from the cached
 * environments (phi(s + d) = phi(s) + Re<g, d> + O(|d|^2), so (Re g, Im g) is
 * the gradient with respect to the real and imaginary parts).  Writes
 * scale * g to d_grad in the bfc_get_cores layout as interleaved (re, im)
 * floats (grad_fp64 = 0) or doubles (grad_fp64 != 0); device, caller owned.
 * If loss is not NULL, *loss = scale * phi (host; synchronizes hip_stream;
 * solve-failure counts of earlier sweeps stay pending for bfc_sync_status).
 * Sums run in the compute precision.  BFC_EINVAL for a NULL d_grad or a NaN
 * scale.
 */
bfc_status bfc_loss_gradient(bfc_problem* p, float scale, void* d_grad, int32_t grad_fp64,
                             double* loss, void* hip_stream);

/*
 * The loss gradients of `count` matrices observed on this problem's positions
 * (the instances of a training batch), one after another on hip_stream with
 * one synchronization at the end: for b = 0 .. count-1 the problem takes the
 * values d_vals[b] (as bfc_set_values) and the cores d_cores[b] (as
 * bfc_set_cores_f32), then scales[b] * g is written to d_grads[b] (as
 * bfc_loss_gradient, FP32 or FP64 by grad_fp64) and losses[b] =
 * scales[b] * phi.  d_vals, d_cores and d_grads are host arrays of count
 * device pointers (caller owned, each d_grads[b] distinct), scales and
 * losses host arrays of count values.  The problem keeps the last instance's
 * values and cores.  Results equal count calls of the three single-instance
 * functions bit for bit.  BFC_EINVAL for count < 1 or a NULL pointer,
 * BFC_ENONFINITE if any instance's values hold a NaN or Inf (every gradient
 * is still written; none of them should be used).
 */
bfc_status bfc_loss_gradient_batch(bfc_problem* p, int32_t count, const void* const* d_vals,
                                   const float* const* d_cores, const float* scales,
                                   void* const* d_grads, int32_t grad_fp64, double* losses,
                                   void* hip_stream);

/* Synchronize hip_stream and report (and clear) pending solve failures. */
bfc_status bfc_sync_status(bfc_problem* p, void* hip_stream);

/*
 * Solve counters since the problem was created or last reset: out[0] =
 * blocks whose system stayed not positive definite (they kept their old
 * values; bfc_sync_status / bfc_residual report and clear this count), out[1]
 * = blocks solved only after the regularization was raised (see
 * bfc_init_cores for the ladder).  Synchronizes hip_stream; reset != 0 clears
 * both counts.
 */
bfc_status bfc_solve_counters(bfc_problem* p, int32_t reset, int64_t out[2], void* hip_stream);

/*
 * Per-kernel timing with HIP events, for benchmarks and profiling.  When
 * enabled, every launch of the kinds below is bracketed by two events on the
 * launch's stream.  bfc_profile_enable synchronizes the device and resets the
 * counters; bfc_profile_read waits for the recorded events and returns the
 * summed elapsed time (ms) and the launch count of one kind since the reset.
 */
#define BFC_KERNEL_OUTER 0        /* outer-core fiber update (Gram, RHS and solve fused) */
#define BFC_KERNEL_INNER_GRAM 1   /* inner-core Gram / right-hand-side partial products   */
#define BFC_KERNEL_INNER_SOLVE 2  /* inner-core slice solves                              */
#define BFC_KERNEL_RESIDUAL 3     /* residual norms                                       */
#define BFC_KERNEL_PREDICT 4      /* entry reconstruction                                 */
#define BFC_KERNEL_ENV 5          /* environment-trie levels (shared partial products)    */
#define BFC_KERNEL_INNER_IR 6     /* BF16-Gram mode: refinement residual from the entries */
bfc_status bfc_profile_enable(bfc_problem* p, int32_t enable);
bfc_status bfc_profile_read(bfc_problem* p, int32_t kind, double* total_ms, int64_t* launches);

/*
 * Layout figures of one core, for work accounting: out[0] = blocks (fibers
 * or slices); for an inner core out[1] = runs (distinct (slice, row) pairs,
 * or (slice, column) pairs, holding entries), out[2] = subgroups (runs cut
 * into pieces of at most 8 entries), out[3] = Gram work items (wavefronts),
 * out[4] = 1 if the core groups by row, 0 by column; for an outer core
 * out[1..3] = 0 and out[4] = -1.  out[5] / out[6] = distinct right / left
 * environments of the core that the sweep computes and caches (0 where the
 * environment is a row of Z^(L+2) / Z^1 or absent).
 */
bfc_status bfc_core_stats(const bfc_problem* p, int32_t core, int64_t out[7]);

/*
 * Debug checks: every invariant the kernels rely on when they index the
 * problem's layout, recomputed on the host from the stored entries -- each
 * core's sorted copy a permutation of core 0's (same index pairs and
 * values), every entry in the block its key names (row, slice key
 * ((ib >> (m-1)) << m) | (jb >> (L-m)), column), block offsets spanning the
 * entries, inner slices sorted by their grouping index, subgroups of 1 to 8
 * entries sharing a row (or column) inside one slice, work items tiling each
 * slice's subgroups, and the environment trie (node tables strictly
 * increasing, every entry pointing at the node of its own (ib >> p, j) or
 * (jb >> (L-p+1), i), every node at its parent on the adjacent level).
 * Synchronizes the device and copies the arrays to the host (O(nnz L) host
 * work); launches no kernel.  BFC_OK, or BFC_EINVAL with bfc_last_error()
 * naming the first violation (core and position).
 */
bfc_status bfc_validate(const bfc_problem* p);

/*
 * Test hook for the out-of-memory paths: after `count` more device
 * allocations by the library succeed, the next one fails as if the device
 * were out of memory (the call making it returns BFC_ENOMEM and releases what
 * it had allocated), and allocations then behave normally again.  count < 0
 * turns the hook off (the default).  Returns the previous setting.  Process
 * wide; not for concurrent use.
 */
int64_t bfc_debug_fail_allocation_after(int64_t count);

/* Release every device allocation of the problem.  NULL is ignored. */
void bfc_destroy(bfc_problem* p);

/* Message describing the calling thread's last error ("" if none). */
const char* bfc_last_error(void);

/*
 * Batched sweeps of independent problems (many completion instances of uneven
 * n, L and r advanced together).  Each problem's sweep is Alg. "ALS for
 * Butterfly Completion" (Sec. 5.1.1) exactly as bfc_sweep runs it; the batch
 * only shares the launches: every launch covers one kernel kind of every
 * problem that needs it at that step of the sweep (problems of one rank per
 * launch), and results are bit-identical to sweeping the problems one by one.
 *
 * bfc_batch_create: problems[0..count-1] (count >= 1, distinct, all BFC_C128
 *   or all BFC_C64; BFC_C64_BF16GRAM is rejected with BFC_EINVAL) stay owned
 *   by the caller and must outlive the batch.  Builds the launch plan in
 *   device memory (synchronous).  *out receives the batch, NULL on error.
 * bfc_batch_sweep: one sweep of every problem on hip_stream (asynchronous);
 *   on a non-null stream the launch list is captured once into a HIP graph
 *   and replayed.
 * bfc_batch_residuals: out_sq[2k], out_sq[2k+1] = ||P(T - X)||^2, ||P T||^2 of
 *   problem k over its own observed entries, FP64 (host array of 2*count;
 *   synchronizes hip_stream).  Returns BFC_ENOTSPD, after filling out_sq,
 *   when any problem's slices were kept since the last report.
 * bfc_batch_destroy: releases the plan (not the problems); NULL is ignored.
 */
typedef struct bfc_batch bfc_batch;
/* (bfc_batch_create etc. below.)  A batch re-plans itself when a problem's
 * work items change (bfc_set_item_size / bfc_autotune_item_size). */
bfc_status bfc_batch_create(bfc_problem* const* problems, int32_t count, bfc_batch** out);
bfc_status bfc_batch_sweep(bfc_batch* b, void* hip_stream);
bfc_status bfc_batch_residuals(bfc_batch* b, double* out_sq, void* hip_stream);
bfc_status bfc_batch_destroy(bfc_batch* b);

/*
 * Tile shape of the inner-core Gram (the subgroup work items of a1, each one
 * wavefront): subgroups per work item, 0 for the automatic rule (at least 128,
 * and enough that a core has about 16384 items), else a multiple of 64 in
 * [64, 65536].  Larger items mean fewer partial products for the slice solve
 * to sum, smaller ones more wavefronts in flight.  Rebuilds every inner core's
 * items (synchronizes hip_stream), grows the partial-product buffers when
 * needed and drops the captured sweep graph.  Results change only by the
 * order of the FP partial sums.
 */
bfc_status bfc_set_item_size(bfc_problem* p, int32_t subgroups, void* hip_stream);

/*
 * Autotuner for the tile shape above: for each candidate (NULL: 64, 128, 256,
 * 512) sets it on every problem, runs one warm-up sweep and `sweeps` timed
 * sweeps (batched when count > 1, HIP events on hip_stream), and keeps the
 * fastest.  Every problem's cores are restored bit-exactly after each trial
 * and at the end (its solve-failure counters are cleared); *chosen receives
 * the selected size, ms_per_sweep[c] (optional, ncand entries) the measured
 * time of candidate c.  Synchronous.
 */
bfc_status bfc_autotune_item_size(bfc_problem* const* problems, int32_t count, int32_t sweeps,
                                  const int32_t* candidates, int32_t ncand, int32_t* chosen,
                                  double* ms_per_sweep, void* hip_stream);

/*
 * One iteration t (1-based) of Alg. "ADAM for Butterfly Completion"
 * (Sec. 5.1.2): cores 0..L+1 in order, each moved by one Alg. "ADAM_Update"
 * step on the gradient of phi = 1/2 ||P(X - T)||^2 at the current cores
 * (the core before it already moved), from the same environments as the ALS
 * update (eq. (grad_butterfly_1), (grad_butterfly_l), (grad_butterfly_last)).
 * For complex data the gradient is sum_e conj(a_e)(x_e - t_e) and the second
 * moment accumulates |g|^2: m <- beta1 m + (1 - beta1) g,
 * v <- beta2 v + (1 - beta2) |g|^2, s <- s - alpha m_hat / (sqrt(v_hat) + sigma)
 * with m_hat = m / (1 - beta1^t), v_hat = v / (1 - beta2^t).  Gradients are
 * accumulated in the compute precision (FP32 in the complex64 modes), the
 * step in FP64.  The moments live in the problem (zero at the first call;
 * bfc_adam_reset zeroes them for a new run); the caller passes t.
 * Asynchronous on hip_stream.  BFC_EINVAL unless t >= 1, alpha > 0,
 * 0 <= beta1, beta2 < 1, sigma >= 0.
 */
bfc_status bfc_adam_sweep(bfc_problem* p, int32_t t, double alpha, double beta1, double beta2,
                          double sigma, void* hip_stream);
bfc_status bfc_adam_reset(bfc_problem* p, void* hip_stream);

/*
 * One iteration of Alg. "ADF for Butterfly Completion" (Sec. 5.1.3) with the
 * orthogonalization sweeps of App. A.3.  First a right-to-left sweep makes
 * cores L+1 .. 1 right-orthogonal: each leaf block of Z^(L+2) (c x r) and
 * each pair of inner slices that differ in the last column digit (an LQ of
 * the r x 2r pair) keeps the orthonormal factor, the triangular one is
 * multiplied into the previous core.  Then for p = 0..L+1: the direction
 * N = sum_e conj(a_e)(t_e - x_e) per block (a fiber of an outer core, a
 * slice of an inner core), the exact line-search step
 * alpha = ||N||^2 / ||A N||^2 and Z <- Z + alpha N per block (a block whose
 * A N vanishes keeps its values), and for p <= L the left orthogonalization
 * of core p (leaf blocks of Z^1; inner slices paired over the row digit they
 * consume, stacked 2r x r) with R multiplied into core p+1.  Every QR runs
 * in FP64 (Householder, reflector sign exp(i arg x_1)); the sums over the
 * observed entries run in the compute precision.  The factors' phases
 * differ from other QR routines' by a diagonal unitary, which leaves the
 * represented tensor and every step unchanged.  Asynchronous on hip_stream;
 * uses the problem's ADAM work buffers (allocated at the first call).
 * BFC_EINVAL unless r <= c = n / 2^L <= 64.
 */
bfc_status bfc_adf_sweep(bfc_problem* p, void* hip_stream);

/*
 * Initial guess of Sec. 5.2: low-rank completion is a problem with L = 0
 * (x_ij = Z^1[i] . Z^2[j], rank R), run with the calls above; this call turns
 * its result X = A B^T into butterfly cores by Alg.
 * "Randomized_LR_to_Butterfly": per row leaf block the first r columns of a
 * column-pivoted QR of the Gaussian sketch A_block (B^T O_0); per inner level
 * the two child blocks' projected factors stacked (2r x R), sketched with
 * B restricted to the current column block, the pivoted QR's first r
 * columns giving the two children's r x r slices; the same from the column
 * side; the middle core (core ceil(L/2)) absorbs V W^T.  Rows take
 * ceil(L/2) inner levels, columns floor(L/2).  Exact (up to rounding) when
 * R <= r.
 *
 * d_A, d_B: device, n x R complex128 (interleaved re/im), row-major, caller
 *   owned; A = Z^1 and B = Z^2 of the L = 0 problem (bfc_get_cores layout).
 * d_sketches: device complex128, the Gaussian matrices the algorithm draws,
 *   concatenated row-major: row-side levels l = 0..ceil(L/2), each
 *   (n >> l) x (r + p), then column-side levels l = 0..floor(L/2), same
 *   shapes.  The caller draws them (any distribution the caller chooses;
 *   the algorithm calls for Gaussian).
 * d_cores_out: device complex128, bfc_num_params(n, L, r) values in the
 *   bfc_get_cores layout; pass it to bfc_init_cores or bfc_set_cores.
 * Requires L >= 1, n = c 2^L with r <= c <= 64, 1 <= r <= 8, 1 <= R <= 16,
 * p >= 0, r + p <= 32; else BFC_EINVAL.  Allocates a scratch buffer of
 * 2^L (4 r R + R (r + p)) complex values for the call and synchronizes
 * hip_stream before returning.
 */
bfc_status bfc_lowrank_to_butterfly(int64_t n, int32_t L, int32_t r, int32_t R, int32_t p,
                                    const void* d_A, const void* d_B, const void* d_sketches,
                                    void* d_cores_out, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * conversion as bfc_lowrank_to_butterfly, with the same arguments, checks and
 * results (bit-identical: the same kernels in the same order), but it calls
 * no hipMalloc, hipFree or other allocating routine and does not synchronize:
 * the work is only enqueued on hip_stream.  Its scratch is a fixed 16 MiB
 * device array per GPU (held from the first call on that GPU until the
 * process ends), so it accepts only sizes with
 * 16 * 2^L (4 r R + R (r + p)) <= 16 MiB (e.g. L <= 11 at r = R = 8, p = 4);
 * larger sizes return BFC_EINVAL with a message naming the limit.  Every
 * call on one GPU shares that array, which keeps the last call's values (the
 * conversion writes every scratch value before reading it, so nothing needs
 * clearing): calls that overlap on one GPU (other streams, other threads)
 * race and must be ordered by the caller.
 */
bfc_status bfc_lowrank_to_butterfly_noalloc(int64_t n, int32_t L, int32_t r, int32_t R, int32_t p,
                                            const void* d_A, const void* d_B,
                                            const void* d_sketches, void* d_cores_out,
                                            void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* BFC_H */
