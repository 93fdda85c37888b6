/*
 * idp.h -- C-ABI of the MI355X library for the second-order
 * invariant-domain-preserving (IDP) Q1 finite-element scheme for the
 * compressible Euler equations (Maier & Kronbichler, arXiv:2007.00094).
 *
 * The problem (Section 3): given admissible conserved states U^n on the
 * nodes of a Q1 mesh (rho > 0, internal energy > 0), compute the time step
 * tau_n (Section 3.3) and U^{n+1} by SSP-RK3 (eq. ssprk3) over the limited
 * forward-Euler update of Alg. 1 (low-order graph-viscosity update, high-
 * order update with the entropy-viscosity indicator of Section 3.8, convex
 * limiting of Section 3.9 with Alg. 2/3, two limiter passes).  The mesh
 * matrices m_ij, c_ij, m_i (eq. matrices) are computed once, at create time.
 *
 * Conventions shared by every call:
 *  - dim is 2 or 3; nc = dim + 2 conserved components per node, in the
 *    order (rho, m_1..m_dim, E).
 *  - State arrays are FP64, array-of-struct [n_nodes][nc], row-major,
 *    contiguous, in the caller's node numbering, and live in DEVICE memory
 *    of the device that was current at idp_create.  The library never keeps
 *    a state pointer beyond the call and never aliases it.
 *  - Mesh arrays given to idp_create are HOST memory, read during the call.
 *  - Every device call is ordered on the HIP stream given at idp_create.
 *    idp_step synchronises that stream at its end unless IDP_FLAG_ASYNC is
 *    set; idp_max_dt always synchronises.
 *  - A context is not thread-safe: one caller at a time.
 *  - Return codes: 0 success, +1 warning (the step completed but tau
 *    exceeded the stability bound m_i/(-2 d_ii) of stage 2 or 3), negative
 *    values are errors (see IDP_E*); idp_strerror names them.
 */
#ifndef IDP_H
#define IDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IDP_OK 0
#define IDP_WARN_CFL 1          /* stage-2/3 tau exceeded m_i/(-2 d_ii)     */
#define IDP_EINVAL (-1)         /* bad argument (null pointer, size, index)  */
#define IDP_EMESH (-2)          /* det J <= 0 at a quadrature point          */
#define IDP_ENOMEM (-3)         /* device or host allocation failed          */
#define IDP_EHIP (-4)           /* HIP runtime error                         */
#define IDP_ESTATE (-5)         /* input state not admissible (rho<=0, eps<=0, NaN) */
#define IDP_EDT (-6)            /* given dt > min_i m_i/(-2 d_ii) at stage 1 */
#define IDP_ENOTSUP (-7)        /* option not supported by this build        */
#define IDP_EWAIT (-8)          /* a persistent batch launch gave up waiting
                                   on a dependency (its results are void)  */
#define IDP_ESCRATCH (-9)       /* the call needs more than the static scratch
                                   of idp_batch_steps_noalloc              */

/* flags for idp_params.flags */
#define IDP_FLAG_ASYNC 1        /* idp_step does not synchronise; errors are
                                   sticky and read with idp_get_status     */
#define IDP_FLAG_NO_STAGING 2   /* row sweeps gather every neighbour record
                                   from memory instead of staging each row
                                   block's neighbourhood in LDS (same results,
                                   bit for bit; for tests and measurement)  */
#define IDP_FLAG_RENUMBER 4     /* the library numbers the nodes along a
                                   Morton curve of their coordinates (every
                                   row keeps the caller's column order, so
                                   results are bit for bit those without);
                                   U and every export stay in the caller's
                                   order.  For meshes numbered without
                                   locality.  Single meshes only
                                   (idp_create_batch returns IDP_ENOTSUP)  */
#define IDP_FLAG_SPLIT_P 8      /* the paper's variant 3 of Section 5: the
                                   low-order sweep stores the viscous part
                                   (d^H_ij - d^L_ij)(U_j - U_i) of P_ij per
                                   entry (nc doubles) and the limiter sweeps
                                   and passes read it instead of forming it
                                   (same results, bit for bit; more memory
                                   traffic).  Single meshes only, no adjoint
                                   (IDP_ENOTSUP)                           */

/* Parameters of the scheme.  gamma: ratio of specific heats (Section 2);
 * cfl: c_cfl of Section 3.3 (0 < cfl <= 1); limiter_passes: 1 or 2
 * (Section 3.5 asks for at least two); newton_max_iter, newton_tol: the
 * iteration cap and the tolerance TOL of Alg. 2 (the paper gives no
 * values; defaults 2 and 1e-10); relax_bounds: 0 (default) keeps the
 * bounds of Section 3.9, 1 widens them as the remark of Section 3.9
 * suggests, by r_i = (m_i/|Omega|)^(1.5/d) with |Omega| = sum_i m_i:
 * rho_min (1 - r_i), rho_max (1 + r_i), phi_min (1 - r_i) (the paper gives
 * no formula; this one restores second order at smooth extrema); single
 * meshes only (idp_create_batch returns IDP_ENOTSUP) and no adjoint (the
 * adjoint entry points return IDP_ENOTSUP); other values: IDP_EINVAL.
 * sell_sigma:
 * the sorting window sigma of the SELL-C-sigma row layout (Section 4.3;
 * C = 64): rows are sorted by length, longest first and stable, within
 * consecutive windows of sell_sigma rows (a positive multiple of 64), or
 * across all rows (0, the default).  Results do not depend on it.       */
typedef struct {
    int dim;
    double gamma;
    double cfl;
    int limiter_passes;
    int newton_max_iter;
    double newton_tol;
    int relax_bounds;
    int flags;
    int sell_sigma;
} idp_params;

typedef struct idp_ctx idp_ctx;

/* Fill p with the defaults for dimension dim (gamma 1.4, cfl 0.5, two
 * passes, 2 Newton steps, TOL 1e-10, no relaxation, synchronous, rows
 * sorted across the whole mesh).
 * Returns IDP_EINVAL if dim is not 2 or 3.                               */
int idp_default_params(idp_params *p, int dim);

/* Build the solver for a Q1 mesh (Section 3.1-3.2).
 *  coords    host [n_nodes][dim] node coordinates;
 *  cells     host [n_cells][2^dim] node ids of each cell, vertex
 *            b = bx + 2 by (+ 4 bz) at the reference corner (bx, by, bz);
 *  dirichlet host [n_nodes] or NULL: 1 = the node keeps its step-initial
 *            state after every stage (boundary values held);
 *  hip_stream hipStream_t (may be NULL = default stream) used by every call.
 * Builds the stencil graph I(i) (nodes sharing a cell, diagonal included),
 * m_ij and c_ij by 3-point Gauss quadrature per direction, m_i = sum_j m_ij,
 * and the device work buffers.  On success *out owns all of it; destroy
 * with idp_destroy.  Errors: IDP_EINVAL (n_nodes or n_cells below 1, ids
 * out of range, bad params; the first and the last before any device call),
 * IDP_EMESH (an inverted or degenerate cell), IDP_ENOMEM, IDP_EHIP.      */
int idp_create(idp_ctx **out, const idp_params *p, int64_t n_nodes,
               const double *coords, int64_t n_cells, const int64_t *cells,
               const uint8_t *dirichlet, void *hip_stream);

/* tau = cfl * min_i m_i/(-2 d_ii(U)) (Section 3.3) for the device state
 * U_dev; synchronises the stream.  IDP_ESTATE if U is not admissible.    */
int idp_max_dt(idp_ctx *ctx, const double *U_dev, double *dt_out);

/* One SSP-RK3 step (eq. ssprk3, increment form U^n + theta (E(U) - U^n))
 * of the limited forward-Euler update E (Alg. 1), in place on U_dev.
 * dt <= 0: tau = cfl * (stage-1 bound), computed on the device;
 * dt > 0: tau = dt, IDP_EDT if dt exceeds the stage-1 bound (U untouched).
 * dt_used (host, may be NULL) receives tau.  Returns IDP_OK, IDP_WARN_CFL,
 * IDP_ESTATE (U untouched), IDP_EDT, or IDP_EHIP.  With IDP_FLAG_ASYNC the
 * call returns IDP_OK after enqueueing and dt_used is not written.       */
int idp_step(idp_ctx *ctx, double *U_dev, double dt, double *dt_used);

/* One limited forward-Euler update Uout = E(U) with step tau (> 0), no
 * boundary hold (the building block of idp_step, Alg. 1).  U_dev and
 * Uout_dev must not overlap.  Synchronises.  Returns IDP_OK or
 * IDP_WARN_CFL (tau > min_i m_i/(-2 d_ii)), IDP_ESTATE, IDP_EINVAL.      */
int idp_euler_stage(idp_ctx *ctx, const double *U_dev, double tau,
                    double *Uout_dev);

/* Sticky status of asynchronous steps (synchronises, then clears it).    */
int idp_get_status(idp_ctx *ctx);

/* Sizes: nodes, stencil entries (CSR nonzeros incl. diagonal), bytes of
 * device memory the context holds.  Any pointer may be NULL.            */
int idp_info(const idp_ctx *ctx, int64_t *n_nodes, int64_t *nnz,
             size_t *device_bytes);

/* Host copies of the graph and matrices in CSR form (rows in the caller's
 * node order, columns ascending): row_ptr [n+1], col [nnz], m_i [n],
 * m_ij [nnz], c_ij [nnz][dim].  Any pointer may be NULL.  Synchronises.  */
int idp_export_matrices(const idp_ctx *ctx, int64_t *row_ptr, int32_t *col,
                        double *m_i, double *m_ij, double *c_ij);

/* Host copy of an intermediate of the last forward-Euler stage run
 * (idp_euler_stage, or the last stage of idp_step), CSR / node order:
 *  IDP_DBG_D      d^L_ij [nnz] (diagonal: d_ii)
 *  IDP_DBG_ALPHA  alpha_i [n]          IDP_DBG_R      R_i [n][nc]
 *  IDP_DBG_UL     U^L_i [n][nc]        IDP_DBG_BOUNDS (rho_min, rho_max,
 *                                                      phi_min) [n][3]
 *  IDP_DBG_L1     min(l_ij, l_ji) of pass 1 [nnz]  (diagonal: 1)
 *  IDP_DBG_L2     min(l_ij, l_ji) of pass 2 [nnz]  (diagonal: 1)
 *  IDP_DBG_UPASS  state after pass 1 [n][nc]
 *  IDP_DBG_TAUI   m_i/(-2 d_ii) [n]
 *  IDP_DBG_P      P_ij of eq. def-p, before pass 1 [nnz][nc] (diagonal: 0)
 *  IDP_DBG_L1RAW  row candidate l_ij of pass 1 (Alg. 2 on U^L_i, P_ij and
 *                 the bounds of row i) [nnz]  (diagonal: 1)
 *  IDP_DBG_L2RAW  row candidate of pass 2 (on the pass-1 state of i and
 *                 (1 - min(l_ij, l_ji)) P_ij) [nnz]  (diagonal: 1)
 * The last three are recomputed from the stage's buffers with the sweeps'
 * own device functions (the sweeps keep only the pair minima); they
 * allocate a temporary device array of one double per entry (IDP_ENOMEM if
 * that fails).  Synchronises.  IDP_EINVAL for an unknown code.           */
#define IDP_DBG_D 0
#define IDP_DBG_ALPHA 1
#define IDP_DBG_R 2
#define IDP_DBG_UL 3
#define IDP_DBG_BOUNDS 4
#define IDP_DBG_L1 5
#define IDP_DBG_L2 6
#define IDP_DBG_UPASS 7
#define IDP_DBG_TAUI 8
#define IDP_DBG_P 9
#define IDP_DBG_L1RAW 10
#define IDP_DBG_L2RAW 11
int idp_debug_export(idp_ctx *ctx, int what, double *host_out);

/* Per-kernel timing with HIP events on the context's stream: on = 1 starts
 * recording every kernel launch (and clears the totals), 0 stops.        */
int idp_set_timing(idp_ctx *ctx, int on);

/* Kernel names and accumulated event-timed milliseconds / launch counts.
 * Fills at most max entries; returns the number of kernels, or < 0.      */
int idp_kernel_times(idp_ctx *ctx, int max, const char **names,
                     double *total_ms, int64_t *launches);

/* Evaluate the device arithmetic on n values (device arrays): kind 0
 * x^y (the library's fixed-method power), 1 sqrt(x), 2 x / y.  Used to
 * check that device and host arithmetic agree bit for bit.  Synchronises. */
int idp_device_math(idp_ctx *ctx, int kind, int64_t n, const double *x_dev,
                    const double *y_dev, double *out_dev);

/* ------------------------------------------------------------ batches
 * Many independent meshes of uneven sizes advanced together, each with its
 * own tau (the same scheme per instance, Section 3).  Instance k owns the
 * nodes [off[k], off[k+1]) of one concatenated state U_dev [N][nc]
 * (off from idp_batch_info); its results are bit-identical to a context
 * created for that mesh alone.  idp_step, idp_euler_stage and idp_max_dt
 * answer IDP_ENOTSUP on a context with more than one instance; the batch
 * calls below answer IDP_ENOTSUP on a context created with
 * IDP_FLAG_RENUMBER (its state is in the caller's order: use idp_step).  */

/* Build a batch context: n_inst meshes, each given like idp_create's
 * (host arrays n_nodes[k], coords[k], n_cells[k], cells[k], dirichlet[k]
 * or dirichlet == NULL / dirichlet[k] == NULL for none).  Node ids inside
 * cells[k] are local to instance k.  Errors as idp_create.                */
int idp_create_batch(idp_ctx **out, const idp_params *p, int n_inst,
                     const int64_t *n_nodes, const double *const *coords,
                     const int64_t *n_cells, const int64_t *const *cells,
                     const uint8_t *const *dirichlet, void *hip_stream);

/* Number of instances and host [n_inst + 1] node offsets (may be NULL).  */
int idp_batch_info(const idp_ctx *ctx, int *n_inst, int64_t *node_offsets);

/* How idp_batch_steps runs: IDP_SCHED_LAUNCHES, one kernel launch per
 * sweep covering every instance; IDP_SCHED_PERSISTENT, one persistent
 * launch for all n_steps steps in which every wavefront pops work items of
 * `tile` units (a unit: 64 nodes, 64 pairs or one 64-row stencil slice of
 * one instance) from a queue, each item waiting only on the earlier sweeps
 * of its own instance.  Both give the same bits.                         */
#define IDP_SCHED_LAUNCHES 1
#define IDP_SCHED_PERSISTENT 2
typedef struct {
    int kind;
    int tile;     /* persistent: units per work item, 1..1024; or -1..-256:
                     each sweep of each instance in at most -tile items of
                     equal size (coarse items for large instances)        */
} idp_schedule;

/* n_steps SSP-RK3 steps of every instance, in place on U_dev.
 * dt: host [n_inst] fixed per-instance tau (IDP_EDT if one exceeds its
 * stage-1 bound), or NULL for tau_k = cfl * (stage-1 bound of instance k)
 * at every step.  dt_used: host [n_steps][n_inst] or NULL.  sched: NULL =
 * the schedule chosen by idp_batch_tune (else IDP_SCHED_LAUNCHES).
 * Synchronises.  Returns IDP_OK, IDP_WARN_CFL, IDP_ESTATE, IDP_EDT,
 * IDP_EWAIT, IDP_EINVAL or IDP_EHIP; after an error U_dev is undefined.  */
int idp_batch_steps(idp_ctx *ctx, double *U_dev, int n_steps, const double *dt,
                    double *dt_used, const idp_schedule *sched);

/* For callers that cannot allocate device memory during the call (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): idp_batch_steps with the launch schedule (IDP_SCHED_LAUNCHES),
 * same arguments and same bits, that calls no hipMalloc, hipFree or other
 * allocating routine.  idp_batch_steps allocates, on first need, the
 * per-instance dt and the tau record of n_steps x n_inst; here those and the
 * status word and per-instance tau scalars live in one static device array
 * of 1 MiB per device (held by each device the library runs on until the
 * process ends), so 16 + 32 n_inst + 8 n_steps n_inst bytes must fit in
 * 1 MiB, else IDP_ESCRATCH before any device work.  The context's device
 * must be current (IDP_EINVAL otherwise).  Every call on a device shares its
 * array (kernels clear what must start at zero): calls that overlap on one
 * device, from several threads or on several streams, race.  Returns as
 * idp_batch_steps; IDP_ENOTSUP on a renumbered context.                  */
int idp_batch_steps_noalloc(idp_ctx *ctx, double *U_dev, int n_steps, const double *dt,
                            double *dt_used);

/* tau_k = cfl * min_{i in instance k} m_i/(-2 d_ii(U)) for every instance:
 * host dt_out [n_inst].  Synchronises.                                   */
int idp_batch_max_dt(idp_ctx *ctx, const double *U_dev, double *dt_out);

/* Autotuner: times n_steps steps from U_dev (left unchanged: the runs use
 * a scratch copy) under each candidate schedule (one launch per sweep;
 * persistent with tile 4, 16, 32, 64, 128, 256), keeps the fastest for
 * idp_batch_steps(sched = NULL) and returns it in *best (may be NULL).
 * ms_out (host, may be NULL) receives the time of each candidate, in that
 * order, and *n_candidates their number.  Synchronises.                  */
int idp_batch_tune(idp_ctx *ctx, const double *U_dev, int n_steps, idp_schedule *best,
                   double *ms_out, int *n_candidates);

/* ------------------------------------------------------------ adjoint
 * Reverse mode of the scheme with a fixed time step (the tau of every stage
 * given), for one mesh (IDP_ENOTSUP on a batch context, with
 * newton_max_iter > 8 or with relaxed bounds).  Every max, min, clamp and branch of the forward is
 * differentiated on the branch the forward took (at an exact tie, the
 * branch its comparison picks); the limiter's Newton iterations (Alg. 2/3)
 * are differentiated as unrolled.  Cotangent arrays are device [n][nc],
 * like states.  All calls synchronise; they return IDP_OK, IDP_WARN_CFL
 * (some tau exceeded a stage's bound), IDP_ESTATE, IDP_EINVAL, IDP_ENOMEM
 * or IDP_EHIP.                                                           */

/* Ubar = (dE/dU)^T Ebar for the forward-Euler update E with step tau
 * (Alg. 1; idp_euler_stage's map).  U_dev, Ebar_dev, Ubar_dev distinct.  */
int idp_euler_stage_vjp(idp_ctx *ctx, const double *U_dev, double tau,
                        const double *Ebar_dev, double *Ubar_dev);

/* Ubar = (dS/dU)^T Ubar_next for one SSP-RK3 step S (eq. ssprk3, held
 * nodes included) from U_dev with step dt > 0.  Arrays distinct.        */
int idp_step_vjp(idp_ctx *ctx, const double *U_dev, double dt,
                 const double *Ubar_next_dev, double *Ubar_dev);

/* n_steps SSP-RK3 steps in place on U_dev with the steps dt[s] (host
 * [n_steps], each > 0), keeping the state before steps 0, every,
 * 2 every, ... in device memory owned by the context (checkpoints).     */
int idp_forward_checkpoints(idp_ctx *ctx, double *U_dev, int n_steps,
                            const double *dt, int every);

/* Decision trace, for tests of the adjoint (its callers are finite-
 * difference checks that need to know whether two nearby forward runs
 * took the same branches): n_steps SSP-RK3 steps in place on U_dev with the
 * steps dt[s] (as idp_forward_checkpoints, no checkpoints kept), and after
 * every stage its decisions written to the device buffer trace_dev, stage
 * k (0-based, three per step) at byte offset k * (*stage_bytes):
 *   [npairs] uint64: per unordered pair {i < j}: bits 0-13 the branches of
 *     the graph viscosity (which state holds p_max; for each orientation
 *     evaluated: psi(p_max) < 0, p_max < p~, the two-rarefaction
 *     numerator > 0, p* > p_i, p* > p_j, which wave speed is larger; which
 *     orientation set the max), bits 16-23 / 24-31 the limiter of (i,j) /
 *     (j,i) in pass 1 (density cut at rho_max, at rho_min, clamped;
 *     enclosure steps taken; how the search ended; a safeguard acted),
 *     bits 32-39 / 40-47 the same in pass 2, bits 48 / 49 which side set
 *     min(l_ij, l_ji) in pass 1 / 2;
 *   then (256-byte aligned) [n] uint32: per node the signs of the terms of
 *     the smoothness indicator (Section 3.8);
 *   then (256-byte aligned) [n] int32: per node the row positions of the
 *     entries that set rho_min, rho_max and phi_min (bits 0-7, 8-15,
 *     16-23; 255: the node itself).
 * Node and pair indices are the library's; two traces of one context
 * compare element by element.  n_steps = 0 only returns *stage_bytes.
 * trace_bytes must hold 3 n_steps stages.  Returns IDP_OK, IDP_WARN_CFL,
 * IDP_EINVAL, IDP_ENOTSUP (batch or renumbered context, relaxed bounds,
 * newton_max_iter > 8), IDP_ENOMEM or IDP_EHIP; synchronises.           */
int idp_trace_decisions(idp_ctx *ctx, double *U_dev, int n_steps, const double *dt,
                        void *trace_dev, int64_t trace_bytes, int64_t *stage_bytes);

/* Ubar0 = (d U_final / d U_0)^T Ubar_final for the steps of the last
 * idp_forward_checkpoints call (same n_steps, dt, every): each segment of
 * `every` steps is recomputed from its checkpoint, then stepped backwards
 * with idp_step_vjp.  IDP_EINVAL if the arguments differ from that call. */
int idp_adjoint_checkpoints(idp_ctx *ctx, int n_steps, const double *dt, int every,
                            const double *Ubar_final_dev, double *Ubar0_dev);

/* Host copy of a total cotangent of the last stage VJP run (for tests):
 *  IDP_ADJ_UL     U^L_i's [n][nc]      IDP_ADJ_R      R_i's [n][nc]
 *  IDP_ADJ_BOUNDS (rho_min, rho_max, phi_min)'s [n][3]
 *  IDP_ADJ_ALPHA  alpha_i's [n]
 *  IDP_ADJ_D      d_ij's [nnz] in CSR order, at the entry (i, j) with
 *                 i < j of each pair (the symmetric entry and the
 *                 diagonal hold 0)
 *  IDP_ADJ_P      P_ij's [nnz][nc] in CSR order (diagonal: 0).
 * Synchronises.                                                          */
#define IDP_ADJ_UL 0
#define IDP_ADJ_R 1
#define IDP_ADJ_BOUNDS 2
#define IDP_ADJ_ALPHA 3
#define IDP_ADJ_D 4
#define IDP_ADJ_P 5
int idp_debug_adjoint(idp_ctx *ctx, int what, double *host_out);

/* Text of a return code.                                                 */
const char *idp_strerror(int code);

/* Free the context and its device memory (NULL is allowed).              */
void idp_destroy(idp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* IDP_H */
