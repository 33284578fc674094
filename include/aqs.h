/*
 * aqs.h -- C ABI of the MI355X (gfx950) batched athermal quasistatic engine.
 *
 * Method: M. Reihn, F. Bamer, B. Stamm, "Parallel athermal quasistatic
 * deformation stepping of molecular systems", arXiv 2507.20802.
 *
 * One context holds a batch of independent replicas ("slots") of a binary
 * Lennard-Jones system in a periodic, simply sheared box (or, per slot, a
 * pure-sheared one, Eq. 17).  The calls below
 * are the operators of the paper, applied to any subset of slots at once:
 *
 *   aqs_affine_shear     F_N^(dk * dgamma), Eqs. (2), (3), (16)
 *   aqs_minimize_batch   the minimisation operator of Eq. (10) (FIRE 2.0),
 *                        optionally followed on the device by n fine AQS
 *                        steps (F o F_N^(dgamma))^n, Eqs. (11)-(12), (19)
 *   aqs_compare_configs  the equality test of Eq. (20)
 *   aqs_stress           the Cauchy stress; tau = sigma_12 of Fig. 2
 *
 * Conventions (every call):
 *   - Host pointers are plain host memory, read or written during the call
 *     only; the caller keeps ownership.  The device workspace given to
 *     aqs_create belongs to the caller, must stay allocated until
 *     aqs_destroy, and is never freed by the library.
 *   - Positions cross the ABI atom-major (pos[i*dim + a]) and in atom-id
 *     order; the device keeps its own cell-sorted order internally.
 *   - Box: the unstrained box of slot r is diag(L_r); at strain index k the
 *     box is H = F^(gamma) diag(L_r) with gamma = k * dgamma_r computed in one
 *     product, columns (Lx,0,0), (gamma*Ly, Ly, 0), (0,0,Lz) (Eq. 1); for a
 *     slot set to the pure shear of Eq. (17) (aqs_set_pure_shear) it is
 *     F^k diag(L_r) with F acting on (x, y); aqs_get_box returns it.
 *   - Calls that return values to the host synchronise the context's stream;
 *     the others are stream-ordered on it.
 *   - No call throws.  A return value < 0 is an error; aqs_last_error()
 *     describes it.  Per-slot minimiser outcomes are data (AQS_CONVERGED ...),
 *     not errors.
 *   - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef AQS_H
#define AQS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aqs_ctx aqs_ctx;
typedef int32_t aqs_status;

/* return codes */
#define AQS_OK 0
#define AQS_EINVAL (-1)     /* bad argument */
#define AQS_EHIP (-2)       /* HIP runtime error */
#define AQS_ENOMEM (-3)     /* workspace smaller than aqs_workspace_bytes() */
#define AQS_ECAPACITY (-4)  /* neighbour list or log capacity exceeded */
#define AQS_ESTATE (-5)     /* call not valid in the current state */

/* per-slot outcome of one minimisation */
#define AQS_CONVERGED 0  /* max_i |F_i| < ftol */
#define AQS_MAXITER 1    /* max_iter updates done */
#define AQS_STALLED 2    /* FIRE: more than n_neg_max consecutive P <= 0;
                            CG: more than n_fail_max failed line searches in a row */
#define AQS_NONFINITE 3  /* energy or a force not finite */
#define AQS_CANCELLED 4  /* record only: not run, the chain was stopped after a
                            failed check of aqs_run_round */

/* minimiser of the minimisation operator of Eq. (10) (aqs_set_minimizer) */
#define AQS_MIN_FIRE 0  /* FIRE 2.0, aqs_fire_params (the default) */
#define AQS_MIN_CG 1    /* nonlinear conjugate gradients, aqs_cg_params */

/* start of the minimisation after each fine affine step */
#define AQS_START_PLAIN 0    /* the affine image F r (Eq. 12) */
#define AQS_START_LEARNED 1  /* F r + predicted non-affine displacement */
#define AQS_START_FALLBACK 2 /* record only: learned, extrapolated or
                                linear-response start rejected, F r used */
#define AQS_START_EXTRAPOLATED 3 /* F r + the previous step's non-affine
                                    displacement (see aqs_minimize_batch) */
#define AQS_START_LINEAR 4   /* F r + u, H u = f(F r): the linear response of
                                Eqs. (7)-(8) (see aqs_minimize_batch) */

/* Binary truncated-and-shifted Lennard-Jones pair potential, Eq. (13):
 * U_ab(r) = 4 eps_ab [(sigma_ab/r)^12 - (sigma_ab/r)^6] - U_ab(rc_ab) for
 * r < rc_ab = rc_factor * sigma_ab, else 0.  Types are 0 (A) and 1 (B). */
typedef struct {
  int32_t dim;  /* 2 or 3 */
  int32_t pad_;
  double eps[2][2];
  double sigma[2][2];
  double rc_factor;
} aqs_potential;

/* FIRE 2.0 (Guenole et al. 2020), unit mass; the step order is documented
 * at aqs_minimize_batch. */
typedef struct {
  double dt0, dt_max, dt_min, f_inc, f_dec, alpha0, f_alpha;
  double dmax;  /* per-atom cap on one step's displacement */
  double ftol;  /* convergence: max_i |F_i| < ftol */
  int32_t n_delay, n_neg_max, initial_delay, pad_;
  int64_t max_iter;
} aqs_fire_params;

/* Nonlinear conjugate gradients, the paper's own minimiser (Sec. 2.1); the
 * step order is documented at aqs_set_minimizer. */
typedef struct {
  double a_init;      /* first trial step of the first line search (x += a F) */
  double sigma;       /* line search ends at |phi'(a)| <= sigma |phi'(0)|, in (0, 1) */
  double grow;        /* largest extrapolation factor of a trial step, > 1.1 */
  double dmax;        /* largest displacement of an atom within one line search */
  double ftol;        /* convergence: max_i |F_i| < ftol */
  int32_t ls_max;     /* evaluations per line search before it counts as failed */
  int32_t n_fail_max; /* consecutive failed line searches before STALLED */
  int64_t max_iter;
} aqs_cg_params;

/* Performance knobs.  None changes what is computed beyond the rounding of
 * one atom's force sum (its order depends on skin and threads_per_atom);
 * results are bitwise repeatable for fixed knobs. */
typedef struct {
  double skin;              /* Verlet skin added to each pair cutoff; 0 = 0.3 */
  int32_t max_neighbors;    /* list capacity per atom; 0 = 64 (2D) / 192 (3D) */
  int32_t block_iters;      /* FIRE iterations launched between host polls, rounded up to
                               an even number; 0 = 32 */
  int32_t use_graph;        /* 1: replay each block of iterations as a hipGraph */
  int32_t max_chain_steps;  /* largest n_steps accepted by aqs_minimize_batch; 0 = 1024 */
  int32_t threads_per_atom; /* force kernel: 1, 2, 4 or 8 lanes per atom; 0 = 2 */
  int32_t live_batch_blocks;/* aqs_run_round with live = 1: while a chain runs alone on
                               the second stream, the batch's force launches hold at
                               most this many blocks per compute unit, so that every
                               compute unit keeps room for a block of the critical
                               chain (1-4; 0 = 3; < 0 = no limit).  Changes no result. */
  int32_t live_xcds;        /* aqs_run_round with live = 1: the critical chain's blocks run
                               on the last live_xcds of the 8 XCDs (accelerator dies; a
                               launch deals block b to XCD b mod 8) and the batch's on
                               the others, so that each keeps its own compute units and
                               L2 (0-7; 0 = no partition).  Changes no result. */
  int32_t force_waves;      /* occupancy target of the force kernel: 4 or 5 wavefronts per
                               SIMD (4 leaves it up to 128 VGPRs, 5 up to 102); 0 = 5 */
  double tile_fill;         /* force tiles (cell-row segments) hold about tile_fill times
                               the atoms a block's lanes take at once (256 /
                               threads_per_atom); clamped to [0.5, 2]; 0 = 0.9 */
} aqs_tuning;

/* One record per minimisation of a chain (index 0 = the first minimisation,
 * s = the minimisation after fine step s). */
typedef struct {
  int64_t iters;      /* FIRE updates performed */
  double energy;      /* E at the last force evaluation */
  double max_f;       /* max_i |F_i| at the last force evaluation */
  double sigma_xy;    /* shear stress at the last force evaluation */
  int32_t status;     /* AQS_CONVERGED ... */
  int32_t start;      /* start used: AQS_START_PLAIN, AQS_START_LEARNED,
                         AQS_START_EXTRAPOLATED, AQS_START_LINEAR, or
                         AQS_START_FALLBACK (a predicted start asked for and
                         rejected) */
} aqs_step_record;

/* Bytes of device workspace a context with these slots needs.  n_atoms:
 * host array of n_rep atom counts; box_len: host array n_rep x dim of
 * unstrained edge lengths (needed to size the cell grids).  Returns 0 on
 * invalid input. */
size_t aqs_workspace_bytes(const aqs_potential* pot, const aqs_tuning* tune,
                           int32_t n_rep, const int32_t* n_atoms,
                           const double* box_len);

/* Create a context over the caller's device workspace (>= 256-byte
 * aligned, >= aqs_workspace_bytes) and HIP stream (hipStream_t; NULL = the
 * null stream).  dgamma: host array of n_rep fine strain increments.  Slots
 * start empty; fill them with aqs_set_replica.  AQS_ECAPACITY if a slot's
 * neighbour list (atoms rounded up to 256, times max_neighbors) reaches 2^30
 * entries. */
aqs_status aqs_create(const aqs_potential* pot, const aqs_fire_params* fire,
                      const aqs_tuning* tune, int32_t n_rep,
                      const int32_t* n_atoms, const double* box_len,
                      const double* dgamma, void* workspace,
                      size_t workspace_bytes, void* stream, aqs_ctx** out);

aqs_status aqs_destroy(aqs_ctx* ctx);

/* Load slot rep: types[n] (0/1), positions pos[n*dim] in atom-id order, at
 * strain index k (the positions must belong to that box).  Velocities are
 * cleared.  Synchronises. */
aqs_status aqs_set_replica(aqs_ctx* ctx, int32_t rep, const uint8_t* types,
                           const double* pos, int64_t strain_index);

/* Replace the positions of slot rep (atom-id order, current box).
 * Synchronises. */
aqs_status aqs_set_positions(aqs_ctx* ctx, int32_t rep, const double* pos);

/* Positions of slot rep in atom-id order (wrapped into the box at the last
 * neighbour-list build, so compare them by minimum image).  Synchronises. */
aqs_status aqs_get_positions(aqs_ctx* ctx, int32_t rep, double* pos);

aqs_status aqs_get_strain_index(aqs_ctx* ctx, int32_t rep, int64_t* k);

/* Bravais tensor of slot rep at its current strain index (Eq. 1; columns are
 * the box vectors), dim x dim row-major into the host array H: simple shear
 * (Eq. 16) or the slot's pure shear (Eq. 17, aqs_set_pure_shear). */
aqs_status aqs_get_box(aqs_ctx* ctx, int32_t rep, double* H);

/* Copy slot src into slot dst (same atom count, shear mode and dgamma):
 * positions, types, order, strain index and last energy.  Level I anchors
 * and snapshots.  AQS_EINVAL if the slots differ in any of these. */
aqs_status aqs_copy_replica(aqs_ctx* ctx, int32_t src, int32_t dst);

/* Affine simple shear of the selected slots, Eqs. (2)-(3) with Eq. (16):
 * x_i += (dk_r * dgamma_r) y_i in one multiplication (level I uses
 * dk = i K, Eq. 18), and k_r += dk_r so the box follows (Eq. 1).  A slot set
 * to pure shear (aqs_set_pure_shear) takes (x_i, y_i) <- F^dk (x_i, y_i)
 * instead, dk >= 0 only.  rep[n_sel], dk[n_sel] are host arrays of distinct
 * slots (AQS_EINVAL, nothing changed, if a slot is listed twice or a pure
 * shear would go backwards).  Stream-ordered. */
aqs_status aqs_affine_shear(aqs_ctx* ctx, int32_t n_sel, const int32_t* rep,
                            const int64_t* dk);

/* Minimise the selected slots to their inherent structures (Eq. 10) with
 * FIRE 2.0 (or the minimiser set by aqs_set_minimizer), all in one batched
 * launch sequence, then -- per slot, on the
 * device, without returning to the host -- run n_steps[r] fine AQS steps
 * (affine map by dgamma_r, Eq. 16, then minimise again; Eq. 12).  A slot
 * stops early if a minimisation does not converge.
 *
 * FIRE, per slot, unit mass, global norms over the slot:
 *   1 evaluate E, F;  2 non-finite -> NONFINITE; max_i |F_i| < ftol ->
 *   CONVERGED (before any update: an inherent structure takes 0 iterations);
 *   3 P = F.v;  4 P > 0: n_pos++, n_neg = 0, if n_pos > n_delay:
 *   dt = min(dt f_inc, dt_max), alpha *= f_alpha;  5 P <= 0: n_pos = 0,
 *   n_neg++, n_neg > n_neg_max -> STALLED; unless (initial_delay and
 *   it < n_delay): {if dt f_dec >= dt_min: dt *= f_dec; alpha = alpha0};
 *   x -= dt v / 2; v = 0;  6 v += dt F;  7 v = (1-alpha) v +
 *   alpha |v|/|F| F (skipped if |F| = 0);  8 per atom, dt |v_i| > dmax ->
 *   v_i scaled to dmax / dt;  9 x += dt v; it++; it >= max_iter -> MAXITER.
 *
 * rep[n_sel]      host, distinct slots
 * start_mode      AQS_START_PLAIN, AQS_START_LEARNED (needs aqs_learned_load)
 *                 or AQS_START_EXTRAPOLATED; with AQS_START_LEARNED the fine
 *                 steps start as documented at aqs_learned_load (the first
 *                 minimisation starts as given).  AQS_START_EXTRAPOLATED (the
 *                 extrapolation the paper's conclusion, Sec. 5, proposes to
 *                 cut the minimiser's iterations): fine step s >= 2 of the call
 *                 starts from F r + dgamma (u_hat - mean u_hat), u_hat =
 *                 (r(IS_(s-1)) - F r(IS_(s-2))) / dgamma, the non-affine
 *                 displacement of the step before, with the acceptance rules
 *                 of the learned start; step 1 has no history and starts from
 *                 F r (record AQS_START_FALLBACK).  AQS_START_LINEAR (the
 *                 equilibrium condition of Sec. 2.1, Eqs. 7-8, as a start):
 *                 every fine step starts from x0 + u, x0 = F r, where u
 *                 solves H u = f(x0), H the Hessian at x0, by conjugate
 *                 gradients from u = 0 (residual r = f(x0) - H u, direction
 *                 p; H p by central differences of the forces,
 *                 (f(x0 - s p) - f(x0 + s p)) / (2 h) max_i |p_i| with
 *                 s = h / max_i |p_i|; stop at |r|^2 <= tol^2 |f(x0)|^2, at
 *                 p.Hp <= 0 before the update, or after max_cg updates;
 *                 aqs_set_linear_start), with the acceptance rules of the
 *                 learned start (max_i |u_i| <= 0.1 sigma_AA, E and max_i
 *                 |F_i| no worse than at x0; else x0, record
 *                 AQS_START_FALLBACK).  Each update costs two force
 *                 evaluations, counted in aqs_counters.atom_evals.
 * n_steps[n_sel]  host, fine steps after the first minimisation; NULL = all 0
 * snap_dst[n_sel] host, slot that receives a copy of the first inherent
 *                 structure (the "outgoing" configuration of Sec. 3.3), or -1;
 *                 NULL = none.  Must have the same atom count, shear mode and
 *                 dgamma.
 * records         host, n_sel x (max_s n_steps + 1) records, row r for
 *                 rep[r]; entries past a slot's last minimisation are left
 *                 untouched.  May be NULL.
 * Synchronises. */
aqs_status aqs_minimize_batch(aqs_ctx* ctx, int32_t n_sel, const int32_t* rep,
                              int32_t start_mode, const int32_t* n_steps,
                              const int32_t* snap_dst, aqs_step_record* records);

/* Minimiser of the later aqs_minimize_batch and aqs_run_round calls of ctx:
 * AQS_MIN_FIRE (cg may be NULL) or AQS_MIN_CG with cg (copied).  The paper
 * minimises with conjugate gradients (Sec. 2.1) and names no variant; this
 * one is Polak-Ribiere with beta >= 0 and a line search on the directional
 * derivative phi'(a) = -F(x0 + a d).d only, which stops at the nearest
 * minimum along d.  Per slot, one force evaluation per iteration:
 *   1 evaluate F;  2 non-finite -> NONFINITE; max_i |F_i| < ftol ->
 *   CONVERGED (before any update);  3 with a direction d: p = phi'(a),
 *   the search ends if |p| <= sigma |p0| or if p < 0 and a >= dmax /
 *   max_i |d_i|; then beta = max(0, (|F|^2 - F.F0) / |F0|^2);  4 after
 *   ls_max evaluations it has failed: beta = 0, and more than n_fail_max
 *   failures in a row -> STALLED;  5 else the next trial: a secant step from
 *   the last two descending points, kept in [1.1 a, grow a] and under
 *   dmax / max_i |d_i|, or, once a point past the minimum exists, the secant
 *   root of the bracket kept in its middle 80 %; x += (a' - a) d;
 *   6 new direction: beta = 0 unless |F|^2 - beta p > 0; d = F + beta d;
 *   p0 = -F.d; first trial a1 = a_prev p0_prev / p0 (a_init for the first
 *   search and after a failed one), at most dmax / (max_i |F_i| + beta
 *   max_i |d_old,i|); F0 = F; x += a1 d;  7 it++; it >= max_iter -> MAXITER.
 * Records count iterations (= force evaluations before convergence) as for
 * FIRE.  AQS_EINVAL for an unknown minimiser or parameters out of range. */
aqs_status aqs_set_minimizer(aqs_ctx* ctx, int32_t minimizer, const aqs_cg_params* cg);

/* Change the tuning field live_batch_blocks of ctx (same meaning, same
 * default for 0) for later live rounds, e.g. from how often earlier checks
 * passed.  Changes no result. */
aqs_status aqs_set_live_batch_blocks(aqs_ctx* ctx, int32_t blocks);

/* Change the tuning field live_xcds of ctx for later live rounds (0-7,
 * AQS_EINVAL otherwise).  Changes no result. */
aqs_status aqs_set_live_xcds(aqs_ctx* ctx, int32_t xcds);

/* New fine strain increments dgamma[i] for the selected slots (dynamic step
 * sizing, Sec. 5): a slot's strain k dgamma is kept exactly, so its strain
 * index becomes k' = k dgamma_old / dgamma_new, which must be an integer
 * whose strain k' dgamma_new equals k dgamma_old bit for bit (a dyadic ladder
 * dgamma_0 / 2^m always converts forward; AQS_EINVAL otherwise, nothing
 * changed).  Simple-shear slots only (a pure shear's box depends on dgamma);
 * the slots must not be running (AQS_ESTATE).  Lists are rebuilt at the next
 * call.  Synchronises. */
aqs_status aqs_set_dgamma(aqs_ctx* ctx, int32_t n_sel, const int32_t* rep, const double* dgamma);

/* Parameters of the linear-response start (AQS_START_LINEAR): at most
 * max_cg updates of the conjugate-gradient solve, stop at |r| <= tol
 * |f(x0)|, probe length h (sigma_AA, max norm) of the Hessian-vector
 * products.  Defaults 50, 1e-3, 1e-5.  AQS_EINVAL for max_cg outside
 * [1, 100000], tol outside (0, 1) or h outside (0, 0.1). */
aqs_status aqs_set_linear_start(aqs_ctx* ctx, int32_t max_cg, double tol, double probe);

/* Duty cycle of the speculative batch in later live rounds (aqs_run_round
 * with live = 1 or 2): while a chain runs alone on the second stream, after
 * each block of iterations of the batch that took wall time T the batch
 * waits (duty - 1) T, so that the critical chain runs alone that share of the
 * time (1 = the batch runs whenever it can, the default; at most 64,
 * AQS_EINVAL otherwise).  Changes no result, only when the speculative
 * chains get their work done. */
aqs_status aqs_set_live_duty(aqs_ctx* ctx, int32_t duty);

/* The deformation of the selected slots: dgamma_y[i] = 0 keeps the simple
 * shear of Eq. (16); otherwise the pure (pull-push) shear of Eq. (17),
 * F = [[1, dgamma_r], [dgamma_y, 1]] acting on (x, y) (z unchanged, also in
 * 3D), dgamma_r the slot's increment from aqs_create.  The box at strain
 * index k is then H_k = F^k diag(Lx, Ly[, Lz]), F^k formed by square and
 * multiply over the bits of k (from the lowest bit: R <- R B if set, then
 * B <- B B) without fused multiply-adds, so that any plain FP64 evaluation in
 * that order gives the same box; the fine affine step of a chain is
 * (x, y) <- F (x, y), the level-I step F^dk (aqs_affine_shear), the learned
 * and extrapolated starts use the same map and take dgamma_r as the strain of
 * a step, and the stress divides by the deformed volume |det H_k|.  The
 * strain index of a pure-shear slot stays >= 0.  Positions given to
 * aqs_set_replica or aqs_set_positions afterwards are read in the box of the
 * slot's mode at its strain index.  Copies, comparisons, snapshots and
 * learned targets need slots of the same mode.  rep[n_sel], dgamma_y[n_sel]:
 * host arrays; the slots must not be running (AQS_ESTATE otherwise);
 * AQS_EINVAL for a slot out of range or a non-finite dgamma_y or
 * |dgamma_r dgamma_y| >= 1 (F would not be invertible).  Synchronises. */
aqs_status aqs_set_pure_shear(aqs_ctx* ctx, int32_t n_sel, const int32_t* rep,
                              const double* dgamma_y);

/* Outcome of check i of a round (Algorithm 1, Sec. 3.5): the end of chain
 * i-1 against the first inherent structure of chain i, Eq. (20). */
typedef struct {
  int32_t decided;     /* 1: evaluated; 0: not reached (a check before it failed);
                          2: not evaluated, predicted to fail (live = 2) */
  int32_t equal;       /* max_disp < delta_eq */
  double max_disp;     /* max over atom ids of the minimum-image distance */
  double de_per_atom;  /* (E_end(i-1) - E_first(i)) / N */
} aqs_check;

/* Level II and the sequential checks of one round of Algorithm 1 (Sec. 3.5):
 * chain i (slot chain[i], already at its level-I start) gets its first
 * minimisation, then n_steps[i] fine AQS steps, as in aqs_minimize_batch;
 * the first inherent structure of chain i >= 1 is copied into snap[i].
 * Check i = 1 .. P-1 compares the end of chain i-1 with snap[i] (Eq. 20);
 * the first check that fails rejects chains i .. P-1.
 *
 * live = 0: every chain runs to completion in one batched launch sequence on
 * the context stream, then the checks are taken in order.
 * live = 1: the checks are taken as soon as both of their configurations
 * exist, and after a failed check the rejected chains are stopped at their
 * next read-back (the live check the paper proposes in its discussion of
 * load balance, Sec. 4).  The chain whose end the next check needs runs on a
 * second stream of its own, the other chains in one batch on the context
 * stream, so the critical chain does not wait on the batch; the batch's
 * force launches leave room for it on every compute unit
 * (aqs_tuning.live_batch_blocks, aqs_set_live_batch_blocks).  Decisions,
 * accepted steps and every kept inherent structure are those of live = 0
 * (the minimisations do not depend on which slots share a launch).
 * live = 2: as live = 1, and a fine step of the critical chain whose
 * inherent structure carries less shear stress sigma_xy than the step before
 * (a plastic event: an elastic branch under growing shear only gains stress)
 * predicts that the check on that chain's end fails, as the paper's
 * conclusion asks to recognise mispredictions beforehand: the chains after it
 * are stopped at once (check decided = 2, equal = 0) and the critical chain
 * runs on alone.  Every accepted step is still a step of sequential AQS from
 * the verified structure; the round may accept fewer steps than with live =
 * 1 (when the predicted check would have passed).
 *
 * chain[P], snap[P] (snap[0] unused), n_steps[P]: host arrays; distinct slots
 * of equal atom count.  records: host, P x (max n_steps + 1), as in
 * aqs_minimize_batch; entries of a stopped chain after its last finished
 * minimisation read AQS_CANCELLED.  checks: host, P entries (entry 0 unused).
 * Synchronises. */
aqs_status aqs_run_round(aqs_ctx* ctx, int32_t P, const int32_t* chain, const int32_t* snap,
                         const int32_t* n_steps, int32_t start_mode, double delta_eq,
                         int32_t live, aqs_step_record* records, aqs_check* checks);

/* Equality test of Eq. (20) between two slots at the same strain index:
 * max_disp = max over atom ids of |minimum image (r_a,i - r_b,i)|,
 * de_per_atom = (E_a - E_b) / N from the last force evaluations,
 * equal = (max_disp < delta_eq).  Synchronises. */
aqs_status aqs_compare_configs(aqs_ctx* ctx, int32_t rep_a, int32_t rep_b,
                               double delta_eq, int32_t* equal,
                               double* max_disp, double* de_per_atom);

/* Stress of slot rep at its current positions: sigma[a*dim + b] =
 * (1/V) sum_{i<j} U'(r) d_a d_b / r (so sigma_xy V = dE/dgamma), and the
 * energy.  Synchronises. */
aqs_status aqs_stress(aqs_ctx* ctx, int32_t rep, double* sigma, double* energy);

/* Energy and forces (atom-id order, n*dim; may be NULL) of slot rep at its
 * current positions.  Synchronises. */
aqs_status aqs_energy_forces(aqs_ctx* ctx, int32_t rep, double* energy,
                             double* forces);

/* Work counters of a context, accumulated since creation or the last reset.
 * Kernel times are measured with HIP events on the context stream around
 * sampled launches (see aqs_set_profiling); launches counts all. */
typedef struct {
  double force_ms;          /* summed duration of the timed force launches */
  int64_t force_timed;      /* force launches timed */
  double update_ms;         /* summed duration of the timed update launches */
  int64_t update_timed;
  int64_t force_launches;   /* force launches issued */
  int64_t rebuilds;         /* neighbour-list rebuild passes */
  int64_t host_polls;       /* state read-backs of the minimisation loop */
  int64_t atom_evals;       /* atoms whose force was evaluated, summed over launches */
  int64_t timed_atom_evals; /* ... over the force launches timed (force_timed) */
} aqs_counters;

/* Time every n-th block of FIRE iterations (0 = no timing), on every
 * driver lane's stream (aqs_run_round with live = 1 has two). */
aqs_status aqs_set_profiling(aqs_ctx* ctx, int32_t every_nth_block);

aqs_status aqs_get_counters(aqs_ctx* ctx, aqs_counters* out, int32_t reset);

/* ------------------------------------------------------------------------
 * Learned start (the paper starts every minimisation at F r, Eq. 12, and
 * names better starting points as an outlook, Sec. 5).
 *
 * Descriptors of atom i at an inherent structure (64, FP64 sums, minimum
 * image in the current box, neighbours j within the pair cutoff r_d =
 * rc_ab of the potential, f_c(r) = (cos(pi r / r_d) + 1) / 2):
 *   f[24 s + b] = sum over neighbours of species s of
 *                 exp(-(r - mu_b)^2 / (2 w^2)) f_c(r),
 *                 mu_b = 0.6 + b w, w = (2.5 - 0.6) / 23, b = 0..23;
 *   f[48 + k]   = sum_j f_c(r) max(0, n_k . r_ij / r)^2, k = 0..15, n_k at
 *                 angles 2 pi k / 16 (2D) or the 16 points
 *                 (sqrt(1-z^2) cos phi, sqrt(1-z^2) sin phi, z),
 *                 z = 1 - (2k+1)/16, phi = k pi (3 - sqrt 5) (3D).
 * Network: z = bf16((f - feat_mean) / feat_std) (FP32 arithmetic, round to
 * nearest even); h1 = bf16(silu(z W1 + b1)); h2 = bf16(silu(h1 W2 + b2));
 * y = h2 W3 + b3 (BF16 operands, FP32 sums); u_hat = y tgt_std + tgt_mean,
 * the non-affine displacement per unit strain.  silu(a) = a / (1 + e^-a).
 * Learned start of a fine step from inherent structure r: F r + dgamma
 * (u_hat - mean u_hat), kept only if every u_hat is finite, max_i dgamma
 * |u_hat_i| <= 0.1, and E and max_i |F_i| there do not exceed their values at
 * F r; otherwise F r (record start AQS_START_FALLBACK). */

typedef struct {
  int32_t dim;               /* outputs d = 2 or 3 (the context's dim) */
  int32_t pad_;
  float w1[64 * 128];        /* [in][out] */
  float b1[128];
  float w2[128 * 128];
  float b2[128];
  float w3[128 * 3];         /* [in][out]; column 2 unused when d = 2 */
  float b3[3];
  float feat_mean[64], feat_std[64];
  float tgt_mean[3], tgt_std[3];
} aqs_mlp;

typedef struct {
  float lr, beta1, beta2, eps;  /* Adam (Kingma and Ba) */
  float huber_delta;            /* Huber loss threshold, standardised units */
  int32_t batch;                /* samples per Adam step (the last one may be short) */
  int32_t epochs;
  int32_t pad_;
} aqs_train_params;

/* Load a trained network into the context (copied; the caller keeps m). */
aqs_status aqs_learned_load(aqs_ctx* ctx, const aqs_mlp* m);

/* Descriptors of slot rep at its current positions: feat is a DEVICE
 * pointer to n x 64 floats, atom-id order.  Rebuilds the slot's cell lists.
 * Synchronises. */
aqs_status aqs_learned_features(aqs_ctx* ctx, int32_t rep, float* feat);

/* u_hat of the loaded network for slot rep: DEVICE pointer, n x dim
 * floats, atom-id order.  Synchronises. */
aqs_status aqs_learned_predict(aqs_ctx* ctx, int32_t rep, float* u_hat);

/* Training targets from two inherent structures of one system: slot
 * rep_next at strain index k_b > k_a of slot rep_prev, same dgamma.
 * target (DEVICE, n x dim floats, atom-id order) = u / (s dgamma),
 * u = minimum image of (r_next - F^(s dgamma) r_prev) in the box of
 * rep_next, s = k_b - k_a.  Synchronises. */
aqs_status aqs_learned_targets(aqs_ctx* ctx, int32_t rep_prev, int32_t rep_next,
                               float* target);

/* Train a network on the GPU.  feat (n x 64), target (n x dim) and order
 * (epochs x n sample indices, one permutation per epoch) are DEVICE
 * pointers.  model: in, the initial weights (dim set); out, the trained
 * weights and the standardisation: mean and population std per column of
 * feat (FP64 sums); for target the same statistics trimmed three times to
 * the samples whose every component lies within 5 std of the mean (the
 * samples outside the final window -- plastic jumps -- are left out of the
 * loss).  Each epoch takes the samples in its order, cut into consecutive
 * batches; each batch is one Adam step on the Huber loss summed over its
 * kept samples and outputs, divided by (batch size x dim).  loss_hist (host, epochs, may be
 * NULL): mean batch loss per epoch.  stream: hipStream_t or NULL.
 * Allocates and frees its own device buffers.  Synchronises. */
aqs_status aqs_mlp_train(const aqs_train_params* p, int64_t n, const float* feat,
                         const float* target, const int32_t* order, aqs_mlp* model,
                         float* loss_hist, void* stream);

/* Gradient of the mean Huber loss over n <= 65536 samples (one batch, in
 * order) at the weights and standardisation of model: grad receives model
 * with the parameters replaced by their gradients; loss the loss.  DEVICE
 * feat and target as for aqs_mlp_train.  Synchronises. */
aqs_status aqs_mlp_gradients(const aqs_mlp* model, int64_t n, const float* feat,
                             const float* target, float huber_delta, aqs_mlp* grad,
                             float* loss, void* stream);

/* Limits of aqs_mlp_train_static and the size of its device array. */
#define AQS_STATIC_TRAIN_MAX_SAMPLES 65536
#define AQS_STATIC_TRAIN_MAX_BATCH 4096
#define AQS_STATIC_TRAIN_MAX_EPOCHS 4096
#define AQS_STATIC_TRAIN_SCRATCH_BYTES 16525568  /* 15.8 MiB per GPU */

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * training of aqs_mlp_train -- same arguments, same kernels, the same
 * trained weights bit for bit -- with its buffers taken from a fixed array
 * of AQS_STATIC_TRAIN_SCRATCH_BYTES inside this library instead of
 * allocated.  Calls no hipMalloc, hipFree or other allocating routine.
 *
 * Each GPU the library runs on holds its own copy of the array from the
 * first use until the process ends; the call uses the array of the current
 * device (hipGetDevice), which must be the device of feat, target, order and
 * stream.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (the call clears what must start at zero itself):
 * calls that overlap on one GPU -- from two threads, or on two streams whose
 * work interleaves -- race on it and must be serialised by the caller.
 * AQS_ECAPACITY, nothing run, if n > AQS_STATIC_TRAIN_MAX_SAMPLES, if
 * min(batch, n) > AQS_STATIC_TRAIN_MAX_BATCH or if epochs >
 * AQS_STATIC_TRAIN_MAX_EPOCHS; otherwise the errors of aqs_mlp_train.
 * Synchronises. */
aqs_status aqs_mlp_train_static(const aqs_train_params* p, int64_t n, const float* feat,
                                const float* target, const int32_t* order, aqs_mlp* model,
                                float* loss_hist, void* stream);

/* Human-readable description of the last error on this thread. */
const char* aqs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AQS_H */
