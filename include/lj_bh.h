/*
 * lj_bh.h - C ABI of liblj_bh.so, an MI355X (gfx950) library for the hot path
 * of adaptive, parallel Basin Hopping on Lennard-Jones clusters
 * (Carmona et al., arXiv 2510.25938).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers owned by the caller (HBM); scalar
 *     descriptors (lj_batch, parameter structs, state/trace structs) are HOST
 *     structs whose pointer members are device pointers unless noted.
 *   - `stream` is a hipStream_t passed as void*.  Every call only enqueues
 *     work on that stream and returns; results are valid once the stream has
 *     been synchronised.  No call synchronises the host, except
 *     lj_autotune, which times launches.
 *   - Host threads may call concurrently when each uses its own stream and
 *     workspace: the side streams that run size classes concurrently and the
 *     cached step graphs are kept per (device, caller stream).
 *   - No call allocates device memory.  Scratch memory is a caller-provided
 *     workspace whose size comes from the matching *_workspace_bytes query;
 *     the workspace must stay untouched until the enqueued work completes.
 *   - Argument errors are detected on the host before anything is enqueued
 *     and returned as a negative lj_status; lj_last_error() then describes
 *     the failure (thread-local string).
 *   - Numerical outcomes (convergence, line-search failure, overflow) are
 *     per-cluster status codes (LJ_CONVERGED ...), never call errors.
 *   - Reduced units throughout: sigma = epsilon = 1 (Eq. 1).
 *
 * Coordinate layout
 *   A batch of B clusters of uneven size is described by offset[B+1], an
 *   int32 device array of prefix sums: cluster b owns atoms
 *   offset[b] .. offset[b+1]-1, N_b = offset[b+1] - offset[b] >= 0.
 *   Coordinates and gradients are three planes of doubles
 *   [3][total_atoms] = x plane, y plane, z plane.  The paper flattens one
 *   cluster as [x0, y0, z0, x1, ...] (Methodology, Initial Structures and
 *   Input); the planes are its per-component transpose, which makes every
 *   HBM access by consecutive atoms contiguous.
 *
 * Precision modes
 *   LJ_FP64   all arithmetic in FP64.  Per-atom sums run over partners in
 *             ascending order and every sum over atoms is a pairwise
 *             (balanced binary tree) sum over the atom index padded with
 *             zeros to a power of two; FP64 results are therefore identical
 *             bit for bit on every launch schedule.
 *   LJ_MIXED  pair arithmetic (r^-6, r^-12, force factors) and per-tile
 *             per-atom accumulation in FP32; per-cluster energy and all
 *             dot products, L-BFGS curvature pairs and the Armijo test in
 *             FP64; optionally followed by an FP64 polish.
 */
#ifndef LJ_BH_H
#define LJ_BH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lj_status;
#define LJ_OK 0
#define LJ_E_ARG (-1)         /* invalid argument (null pointer, bad size, bad parameter) */
#define LJ_E_HIP (-2)         /* a HIP runtime call failed (see lj_last_error)            */
#define LJ_E_WORKSPACE (-3)   /* workspace missing or smaller than the query returned     */
#define LJ_E_UNSUPPORTED (-4) /* cluster larger than the compiled limit, or no gfx950     */

#define LJ_FP64 0
#define LJ_MIXED 1

/* Per-cluster status written by the minimiser. */
#define LJ_CONVERGED 0 /* ||g||_2 < gtol                                               */
#define LJ_MAXITER 1   /* iteration cap reached                                       */
#define LJ_LSFAIL 2    /* line search failed from the steepest-descent direction      */
#define LJ_NONFINITE 3 /* energy or gradient not finite (e.g. coincident atoms)       */
#define LJ_SWITCHED 4  /* LJ_MIXED without polish: the FP32 phase met its tolerance
                          or stopped making progress at FP32 resolution          */
#define LJ_BADSIZE 5   /* the cluster's N from offset[] is negative or above max_n;
                          the cluster was not processed                          */

#define LJ_MAX_ATOMS_EVAL 4096 /* largest cluster for lj_energy_grad_batch        */
#define LJ_MAX_ATOMS_MIN 1024  /* largest cluster for minimisation and BH         */
#define LJ_MAX_M 10            /* largest L-BFGS history                          */
#define LJ_MAX_CANDS 64        /* largest number of candidates per BH step        */

/* Pair potential of a batch (lj_batch.pair).  LJ_PAIR_LJ is Eq. (1) in
 * reduced units (sigma = epsilon = 1).  LJ_PAIR_MORSE is the Morse pair, an
 * empirical pair force field of the kind the paper's conclusions name as the
 * next potentials, in reduced units with well depth 1 at r = 1:
 *   V(r) = t (t - 2),  t = exp(rho (1 - r)),  rho = lj_batch.pair_rho > 0
 * (rho = 6 has the curvature of Eq. (1) at its minimum).
 * Units (lj_batch.sigma, lj_batch.epsilon; 0 means 1): the coordinates the
 * caller passes and receives are in units of sigma (the well position), the
 * energies in units of epsilon (the well depth).  The kernels divide each
 * loaded coordinate by sigma (one IEEE division) and work in reduced units;
 * they report E = epsilon E_reduced, g = (epsilon / sigma) g_reduced,
 * ||g|| likewise, and coordinates times sigma.  The minimiser's parameters
 * (gtol, max_step, ...) stay in reduced units.  Basin hopping takes reduced
 * units only. */
#define LJ_PAIR_LJ 0
#define LJ_PAIR_MORSE 1

/* A ragged batch.  offset is a device pointer; the other fields are host
 * values that must agree with it: num = B >= 0, max_n >= every N_b,
 * total_atoms = offset[B].  pair and pair_rho select the pair potential,
 * sigma and epsilon the units (zero-initialised: Eq. (1), reduced units). */
typedef struct {
    int32_t num;
    const int32_t* offset;
    int32_t max_n;
    int64_t total_atoms;
    int32_t pair;    /* LJ_PAIR_LJ or LJ_PAIR_MORSE                       */
    double pair_rho; /* Morse range rho (finite, > 0); ignored for Eq. (1) */
    double sigma;    /* length unit (finite, > 0; 0 means 1)              */
    double epsilon;  /* energy unit (finite, > 0; 0 means 1)              */
} lj_batch;

/*
 * lj_energy_grad_batch - Eq. (1) and its analytic gradient for every cluster
 * (or the batch's Morse pair: E_b = sum_{i<j} V(r_ij)).
 *   E_b = 4 sum_{i<j} (r_ij^-12 - r_ij^-6),   g_i = dE/dx_i.
 * Paper: Methodology, "Lennard-Jones Potential", Eq. (1); the gradient is the
 * derivative of Eq. (1) that the L-BFGS-B minimiser consumes.
 *   xyz     [3][total_atoms] device, read only.
 *   energy  [num] device, written.
 *   grad    [3][total_atoms] device, written; may be NULL (energy only).
 *   precision LJ_FP64 or LJ_MIXED.
 * N_b = 0 or 1 gives E = 0 and g = 0.  Coincident atoms give a non-finite E.
 * A cluster above max_n (a broken precondition) is evaluated as usual if it
 * fits the launch shape chosen for max_n; otherwise its E is NaN and its
 * gradient is not written.
 * Errors: LJ_E_ARG, LJ_E_UNSUPPORTED (max_n > LJ_MAX_ATOMS_EVAL), LJ_E_HIP.
 */
lj_status lj_energy_grad_batch(const lj_batch* batch, const double* xyz, double* energy,
                               double* grad, int32_t precision, void* stream);

/* L-BFGS parameters (host struct).  lj_lbfgs_defaults fills the defaults shown. */
typedef struct {
    int32_t m;                  /* stored (s, y) pairs, 0..LJ_MAX_M             [10]   */
    double gtol;                /* stop when ||g||_2 < gtol                     [1e-6] */
    int32_t max_iter;           /* accepted-step cap per phase                  [10000]*/
    double max_step;            /* per-atom cap on the trial displacement       [0.2]  */
    double c1;                  /* Armijo sufficient-decrease constant          [1e-4] */
    int32_t max_ls;             /* backtracking halvings per line search        [30]   */
    double curv_eps;            /* keep (s,y) only if s.y > curv_eps |s||y|     [1e-10]*/
    double gtol_mixed_per_atom; /* LJ_MIXED: FP32 phase ends at
                                   ||g|| < max(gtol, this*N)                    [1e-5] */
    int32_t polish;             /* LJ_MIXED: run the FP64 polish                [1]    */
    double ls_noise;            /* LJ_MIXED: FP32 energy resolution relative to
                                   |E|: the Armijo allowance of the full step
                                   near the FP32 tolerance, and the energy
                                   change below which the FP32 phase judges a
                                   trial by the slope test g_t.d <= (2c1-1) g.d
                                                                                [5e-7] */
} lj_lbfgs_params;

void lj_lbfgs_defaults(lj_lbfgs_params* p);

/* Workspace bytes needed by lj_bh_minimize_batch for this batch shape. */
size_t lj_minimize_workspace_bytes(const lj_batch* batch, const lj_lbfgs_params* params,
                                   int32_t precision);

/*
 * lj_bh_minimize_batch - local minimisation of every cluster of the batch in
 * one persistent launch per cluster-size class (Algorithm Overview, step 2:
 * n candidates minimised in parallel with L-BFGS-B; with no bounds this is
 * L-BFGS: two-loop recursion, per-atom step cap, backtracking Armijo search).
 *   xyz       [3][total_atoms] device: starts in, local minima out.
 *   energy    [num] device: final FP64 energy.
 *   gnorm     [num] device: final ||g||_2 (FP64).
 *   iters     [num] device int32: accepted L-BFGS steps (both phases).
 *   evals     [num] device int32: energy+gradient evaluations (both phases).
 *   status    [num] device int32: LJ_CONVERGED ... LJ_SWITCHED.
 *   xyz_switch [3][total_atoms] device or NULL: LJ_MIXED only, the point where
 *             the FP32 phase ended (the polish starts there).
 *   ws, ws_bytes  workspace of at least lj_minimize_workspace_bytes().
 * Clusters are planned on `stream` (sorted by N, largest first, into size
 * classes); with more than one class present, the classes run concurrently on
 * library-owned side streams forked from and joined back into `stream` with
 * events (also under stream capture, as parallel graph branches).
 * The result of each cluster depends only on its own start and the
 * parameters, never on the batch composition or the launch schedule.
 * Errors: LJ_E_ARG, LJ_E_UNSUPPORTED (max_n > LJ_MAX_ATOMS_MIN), LJ_E_WORKSPACE,
 * LJ_E_HIP.
 */
lj_status lj_bh_minimize_batch(const lj_batch* batch, double* xyz, double* energy, double* gnorm,
                               int32_t* iters, int32_t* evals, int32_t* status,
                               double* xyz_switch, const lj_lbfgs_params* params,
                               int32_t precision, void* ws, size_t ws_bytes, void* stream);

/*
 * lj_bh_minimize_batch_noalloc - lj_bh_minimize_batch with no workspace
 * argument, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * call allocates nothing: its scratch (the work list sorted by N, the
 * size-class table and the claim counters) is a fixed array of
 * LJ_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on
 * until the process ends, and the size classes run one after another on
 * `stream` (no side streams).  Arguments, outputs and per-cluster results are
 * those of lj_bh_minimize_batch, bit for bit.
 * Limits: max_n <= LJ_NOALLOC_MAX_ATOMS (larger clusters keep their L-BFGS
 * history in workspace memory) and num <= LJ_NOALLOC_MAX_CLUSTERS.
 * Concurrency: every call on one device shares that device's array; calls
 * whose work overlaps on one device (other streams, other host threads) race
 * and give wrong results.  Order them, e.g. on one stream.  The array keeps
 * the last call's contents; each call rewrites what it reads before using it.
 * Errors: LJ_E_ARG, LJ_E_UNSUPPORTED (max_n above the limit), LJ_E_WORKSPACE
 * (more clusters than the array holds), LJ_E_HIP.
 */
#define LJ_NOALLOC_SCRATCH_BYTES (1 << 20)
#define LJ_NOALLOC_MAX_ATOMS 256
#define LJ_NOALLOC_MAX_CLUSTERS 262016 /* (LJ_NOALLOC_SCRATCH_BYTES - 512) / 4 */
lj_status lj_bh_minimize_batch_noalloc(const lj_batch* batch, double* xyz, double* energy,
                                       double* gnorm, int32_t* iters, int32_t* evals,
                                       int32_t* status, double* xyz_switch,
                                       const lj_lbfgs_params* params, int32_t precision,
                                       void* stream);

/* Basin-hopping parameters (host struct). */
typedef struct {
    int32_t cands;          /* n candidates per chain and step, 1..LJ_MAX_CANDS        */
    double kT;              /* Metropolis temperature (paper: T = 1.0)                 */
    int32_t adapt_interval; /* adapt the step size every this many steps (paper: 10)   */
    double target_rate;     /* target acceptance rate (paper: 50%)                     */
    double factor;          /* step /= factor above target, *= factor below       [0.9]*/
    uint64_t seed;          /* key of the Philox4x64-10 streams                        */
} lj_bh_params;

/* Per-chain Markov-chain state; every member is a device array over chains
 * (xyz_cur and xyz_best are planes [3][total_atoms] of the chains' batch).
 * The caller initialises it: xyz_cur a local minimum, e_cur its energy,
 * step the initial step size, win_accepts 0, step_index 0, e_best_seen +inf,
 * e_best_acc = e_cur, xyz_best = xyz_cur. */
typedef struct {
    double* xyz_cur;
    double* e_cur;
    double* step;
    int32_t* win_accepts;
    int64_t* step_index;
    double* e_best_seen; /* lowest selected trial energy so far (Fig. 2, running lowest) */
    double* e_best_acc;  /* lowest accepted energy so far (Fig. 3)                        */
    double* xyz_best;    /* structure of e_best_acc                                       */
} lj_bh_state;

/* Optional per-step trace, arrays [chains][capacity_steps] (e_cand:
 * [chains][capacity_steps][cands]); row k is written by step k (0-based
 * step_index) while k < capacity_steps.  Any member may be NULL. */
typedef struct {
    double* e_trial;    /* selected candidate energy, NaN if none finite            */
    int8_t* accepted;   /* Metropolis decision                                       */
    double* e_best;     /* e_best_seen after the step                                */
    double* e_best_acc; /* e_best_acc after the step                                 */
    double* e_cur;      /* e_cur after the step                                      */
    double* step;       /* step size after the step's adaptation                     */
    double* e_cand;     /* every candidate's energy (the values selection used)      */
    int8_t* polish_status; /* LJ_MIXED: status of the accepted candidate's FP64
                              polish (LJ_CONVERGED ...); -1 when nothing was
                              polished (a rejected step, or LJ_FP64)           */
    int32_t capacity_steps;
} lj_bh_trace;

size_t lj_bh_workspace_bytes(const lj_batch* chains, const lj_bh_params* bh,
                             const lj_lbfgs_params* params, int32_t precision);

/*
 * lj_bh_step - num_steps basin-hopping steps of every chain (Algorithm
 * Overview, steps 1-5):
 *   1. perturb: n copies of xyz_cur, each coordinate displaced by s(2u-1),
 *      u uniform in [0,1) from Philox4x64-10 keyed (seed; chain, step,
 *      candidate) - a cube of side 2s;
 *   2. minimise all chains' candidates together (as lj_bh_minimize_batch);
 *   3. select the lowest energy (first index on ties, non-finite ignored);
 *   4. Metropolis: accept if dE <= 0 or u < exp(-dE/kT);
 *   5. every adapt_interval steps: step /= factor if the window's accepted
 *      count exceeds target_rate*interval, step *= factor if below.
 * LJ_MIXED minimises candidates with the FP32 phase only (energies used for
 * selection are FP64 re-evaluations at the FP32 endpoints) and polishes the
 * accepted candidate in FP64 before it becomes the current structure.
 * One step is captured once into a HIP graph per (shapes, pointers,
 * parameters, stream) and replayed num_steps times.  On the legacy NULL
 * stream, which cannot be captured, and on a stream that is itself being
 * captured, the kernels are enqueued directly.
 *   chains  batch descriptor of the chains (offset device, sizes host).
 *   state   per-chain state (device arrays), updated in place.
 *   trace   optional (NULL) per-step trace.
 * Errors: LJ_E_ARG, LJ_E_UNSUPPORTED, LJ_E_WORKSPACE, LJ_E_HIP.
 */
lj_status lj_bh_step(const lj_batch* chains, const lj_bh_state* state, const lj_bh_params* bh,
                     const lj_lbfgs_params* params, int32_t precision, int32_t num_steps,
                     const lj_bh_trace* trace, void* ws, size_t ws_bytes, void* stream);

/*
 * Launch-schedule table (process-wide).  The library picks a workgroup shape
 * per call from this table, falling back to a built-in rule:
 *   LJ_SCHED_EVAL      lj_energy_grad_batch: W wavefronts per workgroup (1, 2,
 *                      4, 8, 16) x A atom slots per lane (1, 2, 4), keyed by
 *                      precision and max_n rounded up to a power of two;
 *                      64*W*A must be >= max_n.
 *   LJ_SCHED_MIN_LARGE minimiser shape for clusters of 257..1024 atoms, keyed by
 *                      precision: w = 0 (16 wavefronts x 1 atom, the LJ_MIXED
 *                      default), 1 (8 x 2, the LJ_FP64 default) or 2 (4 x 4);
 *                      a is ignored.
 *   LJ_SCHED_MIN_CLASS0..2  minimiser shape of the size class of 0..64,
 *                      65..128 and 129..256 atoms (the cluster-per-workgroup
 *                      schedule), keyed by precision, the class of max_n (the
 *                      largest class in the batch) and the class's largest N
 *                      rounded up to a power of two:
 *                        class 0: w = 0 one cluster per wavefront, 1 one
 *                                 cluster reduced over one 16-lane row
 *                                 (N <= 16), 2 two clusters per wavefront
 *                                 (N <= 32), 3 four clusters per wavefront
 *                                 (N <= 16); 4-7 shapes 0-3 compiled to run
 *                                 two wavefronts per SIMD (registers capped
 *                                 at 256, the rest spilled);
 *                        class 1: w = 0 two wavefronts, 1 one wavefront with
 *                                 two atoms per lane;
 *                        class 2: w = 0 four wavefronts, 1 three wavefronts
 *                                 (N <= 192).
 *                      lj_set_schedule: w = -1 removes the entry (built-in
 *                      rule); a is ignored.  lj_get_schedule: *w = the entry
 *                      or -1 (none: the built-in rule, which for class 1 also
 *                      depends on the cluster count), *a = its clusters per
 *                      workgroup.
 * Results never depend on the schedule in LJ_FP64 (fixed summation order).
 */
#define LJ_SCHED_EVAL 0
#define LJ_SCHED_MIN_LARGE 1
#define LJ_SCHED_MIN_CLASS0 2
#define LJ_SCHED_MIN_CLASS1 3
#define LJ_SCHED_MIN_CLASS2 4
lj_status lj_set_schedule(int32_t kind, int32_t precision, int32_t max_n, int32_t w, int32_t a);
lj_status lj_get_schedule(int32_t kind, int32_t precision, int32_t max_n, int32_t* w, int32_t* a);

/*
 * lj_autotune - time every candidate schedule for this batch and record the
 * fastest in the schedule table: all lj_energy_grad_batch shapes holding
 * max_n atoms (at most twice the padded size); for max_n in 257..1024 the
 * three large-cluster minimiser shapes (timed on a 3-iteration minimisation of
 * a copy of xyz); then, for max_n <= 1024, the shapes of size classes 2, 1
 * and 0 in turn, each timed on a whole minimisation of a copy of xyz (default
 * parameters, at most 1000 iterations per phase) with the other classes at
 * their current choice, a shape replacing the current one when at least 2 %
 * faster.  Every candidate is timed as the median of five launches after a
 * warm-up.  xyz [3][total_atoms] is read only.  Unlike every other call this
 * one SYNCHRONISES the stream (it times launches with HIP events).
 *   ws, ws_bytes     scratch of at least lj_autotune_workspace_bytes().
 *   best_eval_ms     fastest pair-kernel time (nullable).
 *   best_min_ms      minimisation time with the chosen shapes, -1 if not
 *                    tuned (max_n above LJ_MAX_ATOMS_MIN) (nullable).
 */
size_t lj_autotune_workspace_bytes(const lj_batch* batch, int32_t precision);
lj_status lj_autotune(const lj_batch* batch, const double* xyz, int32_t precision, void* ws,
                      size_t ws_bytes, void* stream, float* best_eval_ms, float* best_min_ms);

/* Static description of a status code. */
const char* lj_status_string(lj_status s);

/* Description of the last error returned on this thread ("" if none). */
const char* lj_last_error(void);

/* ABI version of this header (incremented on any incompatible change). */
#define LJ_ABI_VERSION 4
int32_t lj_abi_version(void);

/* Number of basin-hopping step graphs captured by this process so far (a
 * diagnostic of the lj_bh_step graph cache: a call whose arguments match a
 * cached graph replays it and captures nothing). */
int64_t lj_bh_graph_captures(void);

#ifdef __cplusplus
}
#endif

#endif /* LJ_BH_H */
