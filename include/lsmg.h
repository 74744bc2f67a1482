/*
 * lsmg — level-set multigrid for the sulfation model on MI355X (gfx950).
 *
 * C ABI of the GPU library.  The method is that of Coco, Semplice and Serra
 * Capizzano (arXiv 1902.07029): a Crank-Nicolson step (section 3.1) of the
 * sulfation model (section 2, eq. maineq) on a uniform Cartesian grid masked by
 * a level set (section 3.2), finite differences on inside nodes and ghost-point
 * boundary rows (section 3.3), Newton-Raphson (section 3.4) whose linear systems
 * are solved by a multigrid V-cycle (section 3.5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns lsmg_status; 0 is success, negative values are
 *   errors and lsmg_last_error() gives a thread-local message.  Nothing else
 *   is reported through exceptions or aborts.
 * - Pointers marked "device" are GPU global-memory addresses owned by the
 *   caller (for example torch tensors' data_ptr()).  The library never frees
 *   them and never keeps them beyond the call.  Pointers marked "host" are
 *   ordinary CPU memory.
 * - The library owns every internal buffer of a hierarchy, of its states and of
 *   a batch.  Their device memory comes from the caller's allocator given at
 *   creation (lsmg_allocator, for example a framework's caching allocator), or
 *   from hipMalloc when none is given.
 * - All GPU work of a hierarchy is enqueued on the HIP stream given to
 *   lsmg_build_hierarchy (NULL = the null stream).  Entry points that return
 *   a scalar through a host pointer synchronise that stream before returning;
 *   the others only enqueue.
 * - Grids: dim = 2 or 3, n nodes per axis on the box [lo, hi]^dim, spacing
 *   h = (hi - lo) / (n - 1) on every axis (Delta x = Delta y [= Delta z] as in
 *   section 3.3).  Grid arrays are n^dim doubles, x fastest.
 * - Compact vectors of level l: 2 * Na doubles, Na = Ni + Ng active nodes,
 *   the s-block then the c-block (section 3.3, "all s variables before the c
 *   ones"); active nodes are ordered as the inside nodes in lexicographic grid
 *   order followed by the ghost nodes in lexicographic grid order (the map M of
 *   eq. maprij).  Level 0 is the finest grid.
 */
#ifndef LSMG_H
#define LSMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LSMG_OK = 0,
    LSMG_EINVAL = -1,      /* bad argument, size or call order */
    LSMG_EGEOM = -2,       /* geometry the method cannot discretise (see lsmg_build_hierarchy) */
    LSMG_ENOCONV = -3,     /* Newton did not reach the tolerance in newton_max iterations */
    LSMG_ENONFINITE = -4,  /* a NaN or infinity appeared in a residual, update or coarse factor */
    LSMG_EOOM = -5,        /* device allocation failed */
    LSMG_EHIP = -6,        /* a HIP runtime call failed */
    LSMG_ENOTIMPL = -7
} lsmg_status;

typedef struct {
    int dim;        /* 2 or 3 */
    int n;          /* nodes per axis; (n - 1) = (coarsest_n - 1) * 2^k */
    double lo, hi;  /* box [lo, hi]^dim */
} lsmg_grid;

typedef struct {
    /* model, section 2 and eq. (dataeq): reaction rates a/m_c and a/m_s,
     * diffusion d, porosity phi(c) = alpha c + beta */
    double a, d, m_s, m_c, alpha, beta;
    /* ghost-row relaxation parameter tau^s of eq. (RelGhost), 0 < tau_s < 1 (eq. CFLcond) */
    double tau_s;
    int nu1, nu2;          /* pre- and post-smoothing steps of the V-cycle */
    int ghost_sweeps;      /* ghost relaxations per smoothing step; 0: 5 in 2-D, 15 in 3-D */
    int ghost_sweeps_coarse; /* the same on levels whose diffusion number d dt / h^2 is below
                              * sweeps_lambda; 0: 20 in 2-D, 30 in 3-D */
    int band_steps;        /* layers of the boundary-defect extension (section 3.5.2) */
    int ghost_c_new;       /* 1: the ghost c-row relaxation uses the new delta s */
    int coarsest_n;        /* nodes per axis of the coarsest grid (>= 3) */
    int precision;         /* 0: FP64 V-cycle; 1: FP32 V-cycle inside FP64 iterative refinement */
    double newton_tol;     /* stop when min(|F|_inf, |dW|_inf / |W|_inf) < newton_tol (section 3.4) */
    int newton_max;
    double lin_rtol;       /* linear solve stops when |J dW - F|_inf <= lin_rtol |F|_inf */
    int cycles_max;        /* V-cycles per linear solve at most */
    double sweeps_lambda;  /* threshold of d dt / h^2 for ghost_sweeps_coarse; 0: 0.3 in 2-D, 0.1 in 3-D */
    int bc;                /* boundary condition for s, fixed at build: 0 Dirichlet s = s_b (eq. BCs);
                            * 1 Neumann ds/dn = s_b (section 3.6, eq. BCsN), with the relaxation
                            * parameter tau_s * 2 sqrt(2) h / 3 per level (eq. CFLcondN; in 3-D
                            * tau_s * 4 h / (3 sqrt(3))) */
    int cycle_gamma;       /* cycle index: 1 V-cycle, 2 W-cycle (the paper's cycle, section 4: the
                            * coarse-grid correction is two cycles on the next level, the second
                            * starting from the first one's result); batches take 1 only */
    int fmg;               /* full multigrid as the first iteration of a linear solve: 0 never,
                            * 1 in the first Newton iteration of a step, 2 in every one (the right-
                            * hand side restricted to every level, the coarsest problem solved, then
                            * on each finer level the prolongated solution as the start of one
                            * cycle); batches take 0 only */
    int fused_sweep;       /* 2-D: 1 runs both colours of a smoothing sweep in one launch over
                            * tiles of rows, the red half-sweep recomputed on a one-node halo
                            * (same bits as one launch per colour); 0 one launch per colour.
                            * A batch fuses its sweeps when every member has fused_sweep = 1 */
    int krylov_m;          /* 0: the linear solve of each Newton iteration iterates V-cycles
                            * (section 3.5); m in 1..200: flexible GMRES(m) on the same system,
                            * right-preconditioned by one V-cycle from a zero correction (the FP32
                            * cycle in mixed precision), restarted from the true defect every m
                            * iterations, stopping when the 2-norm of the defect is at most
                            * lin_rtol times that of F or after cycles_max cycles; fmg is not used.
                            * Not in the paper: it removes the few slow modes that ghost rows with a
                            * tiny self-weight leave to the cycles.  Single hierarchies only (a batch
                            * refuses members with krylov_m > 0, LSMG_ENOTIMPL); its vectors take
                            * (2m + 4) 2 Na doubles of device memory, allocated at the first solve */
} lsmg_params;

typedef struct lsmg_hierarchy lsmg_hierarchy;
typedef struct lsmg_state lsmg_state;

typedef struct {
    int newton_iters;   /* Newton iterations of the step */
    int vcycles;        /* V-cycles executed (one per refinement step in mixed precision) */
    double res_inf;     /* |F(W^{n+1})|_inf at exit */
    double rho_last;    /* last convergence factor |r_q|_inf / |r_{q-1}|_inf (section 4.2) */
    double rho_geo;     /* geometric mean of all convergence factors of the step */
    double dw_rel;      /* last |dW|_inf / |W|_inf */
} lsmg_step_stats;

/* Device memory for the library's internal buffers.  alloc returns `bytes`
 * bytes of device global memory (aligned to at least 256 bytes) on the
 * device that is current, or NULL on failure; free returns a pointer that
 * alloc gave.  The library calls free only after the stream the buffer was
 * used on has been synchronised, so a stream-ordered caching allocator may
 * hand the block out again at once.  Both are called from the thread that
 * calls the library, never concurrently for one hierarchy or batch. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} lsmg_allocator;

/* Default parameters: the model data of eq. (dataeq), tau_s = 0.9 (section
 * 3.5.1), V(2,2), automatic ghost sweeps (0, 0, 0), 3 band layers, ghost_c_new = 1,
 * coarsest 5, FP64, newton_tol 1e-10, newton_max 20, lin_rtol 1e-3,
 * cycles_max 30, Dirichlet boundary, V-cycles, no full multigrid, fused 2-D sweeps. */
void lsmg_default_params(lsmg_params *p);

/* Build the grid hierarchy of one domain (sections 3.2-3.3, 3.5).
 * d_levelset: device, n^dim doubles, the level set phi at the nodes (inside
 *   where phi < 0, eq. ghostdef); read during the call only.
 * Per level (phi injected to every coarser grid): node classification
 * (inside / ghost / inactive), the compact ordering, ghost geometry (normal by
 * central differences, eq. nij; upwind stencil ST; boundary point B by
 * bisection; the biquadratic/triquadratic weights of eq. JssD, with a lower-
 * order fallback where ST reaches an inactive node; where no order is
 * admissible, the ghost's own weight would be negative or B lies outside the
 * stencil: in 2-D the axis rule (B on the grid line to the inside axis
 * neighbour that gives the ghost the largest weight, found by bisection of the
 * quadratic interpolant of phi on that line, and the row the quadratic
 * interpolation along it), in 3-D the constant rule w = 1 on the ghost) and the
 * tables of the boundary-aware restriction.
 * With params->bc = 1 the boundary rows are Neumann rows (section 3.6): the
 * derivative at B of the interpolant of s on ST along the unit gradient of the
 * interpolant of phi at B (eqs. Neumanntilde, JccN), with the fallbacks
 * bilinear gradient -> one-sided differences along the inward axes, each taken
 * only where its nonzero weights sit on active nodes and the ghost's own
 * weight meets eq. CFLcondN.
 * allocator: host, may be NULL (then hipMalloc / hipFree).  Copied: the
 *   hierarchy, its states and their temporaries take every device buffer from
 *   it until lsmg_destroy_hierarchy / lsmg_state_destroy hand them back.
 * stream: a hipStream_t (NULL for the null stream); every later call of this
 *   hierarchy runs on it.
 * Errors: LSMG_EINVAL (bad grid or parameters), LSMG_EGEOM (an inside node on
 *   the box edge, or a Neumann ghost with no admissible row), LSMG_EOOM (also
 *   when the allocator returns NULL), LSMG_EHIP.  *out is NULL on error. */
lsmg_status lsmg_build_hierarchy(const double *d_levelset, const lsmg_grid *grid,
                                 const lsmg_params *params, const lsmg_allocator *allocator, void *stream,
                                 lsmg_hierarchy **out);
void lsmg_destroy_hierarchy(lsmg_hierarchy *h);

/* Set the time step ahead of the first step: the level descriptors and the
 * per-level ghost relaxation maps (whose sweep counts depend on d dt / h^2)
 * are prepared for dt.  Every stepping call does this itself when dt
 * changes.  Synchronises the hierarchy's stream.  Errors: EINVAL. */
lsmg_status lsmg_set_dt(lsmg_hierarchy *h, double dt);

/* Replace the solver parameters (coarsest_n, band_steps and bc are fixed at
 * build: EINVAL if they differ). */
lsmg_status lsmg_set_params(lsmg_hierarchy *h, const lsmg_params *params);

/* ---- preparation of a domain's inputs (full grids, device, x fastest) -------
 * Each call runs on `stream` (a hipStream_t, NULL for the null stream), uses
 * device scratch of a few grid-sized arrays that it frees again, and returns
 * after synchronising the stream.  Errors: EINVAL (bad grid or argument),
 * EOOM, EHIP. */

/* Re-initialisation of a level set towards the signed distance function
 * (section 2): `iterations` forward-Euler steps of d phi/d mu = sgn(phi0)(1 -
 * |grad phi|) with d mu = h / dim.  Nodes next to a sign change of phi0 relax
 * to their distance estimated from phi0 (the subcell fix of Russo and
 * Smereka, which keeps the zero level set in place); the others take the
 * upwind (Godunov) update.  One-sided differences vanish at the box edge.
 * d_phi: n^dim doubles, in place.  The solver itself does not need a distance
 * function (section 2). */
lsmg_status lsmg_reinitialize(double *d_phi, const lsmg_grid *grid, int iterations, void *stream);

/* lsmg_reinitialize for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result, bit for bit, with the
 * working arrays in a fixed device array of the library (52.4 MB per device,
 * held until the process ends) instead of hipMalloc'd ones.  No allocating
 * call is made.  Grids of at most 2^21 nodes (1025^2 in 2-D, 127^3 in 3-D);
 * larger ones return LSMG_EINVAL before any GPU work.  Every call on a device
 * uses that device's one array: calls that overlap on one device (several
 * streams or host threads) race and must be serialised by the caller.
 * Synchronises `stream` before returning. */
lsmg_status lsmg_reinitialize_noalloc(double *d_phi, const lsmg_grid *grid, int iterations, void *stream);

/* A level set from a mask (section 2, images): phi = -1 where d_mask != 0
 * (n^dim bytes), +1 elsewhere, then `iterations` explicit heat steps phi +=
 * (1 / (2 dim)) * (sum of the second differences).  d_phi: n^dim doubles out. */
lsmg_status lsmg_levelset_from_mask(const uint8_t *d_mask, const lsmg_grid *grid, int iterations, double *d_phi,
                                    void *stream);

/* Second-order extrapolation of data (initial s or c, section 3.3) from the
 * inside (phi < 0) to every other node, by the pseudo-time PDE approach the
 * paper cites: the normal derivatives q_n and q_nn by central differences where
 * their stencils are inside, then q_nn extended constantly, q_n linearly and q
 * quadratically along n = grad phi / |grad phi|, `iterations` upwind steps of
 * d tau = h / dim each (20-40 reach the ghost nodes).  d_q: n^dim doubles, in
 * place; values where phi < 0 are unchanged. */
lsmg_status lsmg_extrapolate(const double *d_phi, const lsmg_grid *grid, double *d_q, int iterations, void *stream);

/* Whether the coarse tail of the cycle (the levels of at most 1024 active nodes,
 * run by one workgroup) holds its levels in LDS for the given precision (0:
 * FP64 cycle, 1: FP32 cycle): *in_lds = 1, or 0 where they do not fit or the
 * environment variable LSMG_TAIL_LDS=0 was set when h was built (the tail then
 * reads its levels from HBM; the results are the same bits). */
lsmg_status lsmg_tail_in_lds(const lsmg_hierarchy *h, int precision, int *in_lds);

/* Whether smoothing on `level` runs fused sweeps (fused_sweep, 2-D, pairs of
 * steps) for the given precision: *fused = 1 where the level's active nodes
 * times the value size are at most 1 MiB (launch latency dominates there; on
 * larger levels the fused sweep's halo and whole-tile reads cost more than the
 * launch it saves), else 0.  An odd step of a smoothing block always runs one
 * launch per colour. */
lsmg_status lsmg_sweep_fused(const lsmg_hierarchy *h, int level, int precision, int *fused);

/* Parameters in effect (host out), with automatic choices resolved. */
lsmg_status lsmg_get_params(const lsmg_hierarchy *h, lsmg_params *params);

/* Number of levels (host out). */
lsmg_status lsmg_num_levels(const lsmg_hierarchy *h, int *nlev);

/* Level facts (host outs): nodes per axis, spacing, inside, ghost and
 * boundary-band node counts. */
lsmg_status lsmg_level_info(const lsmg_hierarchy *h, int level, int *n, double *hh,
                            int *n_inside, int *n_ghost, int *n_band);

/* Compact-to-grid map of a level: d_out device, Na int64 lexicographic grid indices. */
lsmg_status lsmg_compact_to_grid(lsmg_hierarchy *h, int level, int64_t *d_out);

/* Ghost table of a level (all device, Ng rows; nst = 3^dim):
 * d_st: Ng*nst int32 compact indices of the stencil ST (k = (k_x, k_y[, k_z]) in
 *   {0,1,2}^dim, x fastest, node G - h (m_x k_x, ...), m = SIGN(normal) except
 *   on the line of an axis-rule row, where G - m_a e_a is the inside
 *   neighbour), -1 where inactive;
 * d_w: Ng*nst weights of the boundary row (eq. JssD); d_B: Ng*dim boundary
 * points; d_normal: Ng*dim unit normals by central differences (eq. nij);
 * d_row_normal: Ng*dim normal of the boundary row (d_normal for Dirichlet
 * rows; for Neumann rows the unit gradient of the interpolated level set at
 * B, eq. Neumanntilde); d_order: Ng int32 (2 quadratic, 1 linear, 0 constant
 * or, for Neumann rows, one-sided); d_bfallback: Ng int32 (0 when B came from
 * bisection along the normal, 1 from the first-order projection, 2 from the
 * axis rule).  Any pointer may be NULL. */
lsmg_status lsmg_ghost_table(lsmg_hierarchy *h, int level, int32_t *d_st, double *d_w, double *d_B,
                             double *d_normal, double *d_row_normal, int32_t *d_order, int32_t *d_bfallback);

/* ---- one Crank-Nicolson step ---------------------------------------------- */

/* A state holds W = (s, c) on the finest active nodes (FP64, device). */
lsmg_status lsmg_state_create(lsmg_hierarchy *h, lsmg_state **out);
void lsmg_state_destroy(lsmg_state *st);
/* d_W: device compact vector of level 0 (2 Na doubles; may be NULL when Na = 0). */
lsmg_status lsmg_state_set(lsmg_state *st, const double *d_W);
lsmg_status lsmg_state_get(const lsmg_state *st, double *d_W);
/* Grid form: d_s, d_c device n^dim doubles; set reads active nodes only,
 * get writes NaN at inactive nodes. */
lsmg_status lsmg_state_set_grid(lsmg_state *st, const double *d_s, const double *d_c);
lsmg_status lsmg_state_get_grid(const lsmg_state *st, double *d_s, double *d_c);

/* Advance st from t_n to t_{n+1} = t_n + dt (sections 3.1, 3.3, 3.4): Newton on
 * F(W) = 0 from W^{(n+1,0)} = W^n, each linear system J dW = F solved by
 * V-cycles from dW = 0, W <- W - dW, stop when
 * min(|F|_inf, |dW|_inf / |W|_inf) < newton_tol after at least one iteration.
 * d_sb: device, Ng boundary values s_b(B_g, t_{n+1}) in ghost order, or NULL to
 *   use sb_const for every ghost (Neumann rows: the values of ds/dn at B_g).
 * d_fn, d_fnp1: device compact vectors [f1 | f2] of the source terms of
 *   section 4.1 at t_n and t_{n+1}, or both NULL.
 * stats: host, may be NULL.  Synchronises the stream.
 * The state is replaced only on LSMG_OK; on LSMG_ENOCONV or LSMG_ENONFINITE it
 * still holds W^n. */
lsmg_status lsmg_newton_cn_step(lsmg_hierarchy *h, lsmg_state *st, double dt, const double *d_sb,
                                double sb_const, const double *d_fn, const double *d_fnp1,
                                lsmg_step_stats *stats);

/* ---- components of the step, on compact device vectors -------------------- */

/* Newton residual F(W) (eqs. FDs, FDc, and the boundary row s~(B) - s_b on
 * ghosts) for the step from W^n = d_Wn with time step dt; d_F out; res_inf
 * (host, may be NULL) receives |F|_inf and synchronises. */
lsmg_status lsmg_residual(lsmg_hierarchy *h, const double *d_W, const double *d_Wn, double dt,
                          const double *d_sb, double sb_const, const double *d_fn,
                          const double *d_fnp1, double *d_F, double *res_inf);

/* Fix the linearisation point of the Jacobian on every level: W on the
 * finest level, injected to the coarser ones; builds and factors the coarsest
 * operator.  Required before the calls below. */
lsmg_status lsmg_set_linearization(lsmg_hierarchy *h, const double *d_W, double dt);

/* Linearisation point of a level (compact, device out). */
lsmg_status lsmg_level_state(lsmg_hierarchy *h, int level, double *d_W);

/* y = J x on a level (section 3.4 Jacobian rows). */
lsmg_status lsmg_apply_J(lsmg_hierarchy *h, int level, const double *d_x, double *d_y);

/* nsweeps smoothing steps (section 3.5.1): red-black collective Gauss-Seidel
 * on inside nodes, then ghost_sweeps ghost relaxations (eq. RelGhost). */
lsmg_status lsmg_smooth(lsmg_hierarchy *h, int level, const double *d_rhs, double *d_x, int nsweeps);

/* Defect r = rhs - J x (section 3.5.2); res_inf as in lsmg_residual. */
lsmg_status lsmg_defect(lsmg_hierarchy *h, int level, const double *d_rhs, const double *d_x,
                        double *d_r, double *res_inf);

/* Boundary-aware restriction of a defect of level `level` to the right-hand
 * side of level+1 (section 3.5.2, Fig. Neigh, with the ghost-defect band
 * extension). */
lsmg_status lsmg_restrict(lsmg_hierarchy *h, int level, const double *d_r, double *d_rhs_coarse);

/* x += bilinear/trilinear prolongation of the coarse correction of level+1
 * (section 3.5.3). */
lsmg_status lsmg_prolong_add(lsmg_hierarchy *h, int level, const double *d_e_coarse, double *d_x);

/* Exact solve on the coarsest level (section 3.5; the coarsest grid is solved
 * directly), FP64.  The operator's c-block is diagonal on that level, so the
 * library eliminates it: S = J^ss - J^sc diag(J^cs / J^cc) (Na x Na, Na the
 * active nodes) is inverted once per linearisation by Gauss-Jordan elimination
 * with partial pivoting, and each call applies
 *   x_s = S^-1 (r_s - J^sc (r_c / J^cc)),   x_c = (r_c - J^cs x_s) / J^cc.
 * d_rhs, d_x: device, 2 Na doubles, [s-block | c-block] of the coarsest level.
 * Needs a linearisation (lsmg_set_linearization or a running step);
 * LSMG_ENONFINITE when S is singular or not finite. */
lsmg_status lsmg_coarse_solve(lsmg_hierarchy *h, const double *d_rhs, double *d_x);

/* One V(nu1, nu2) cycle on `level` with initial guess d_x (in/out);
 * res_inf (host, may be NULL) receives |rhs - J x|_inf after the cycle. */
lsmg_status lsmg_vcycle(lsmg_hierarchy *h, int level, const double *d_rhs, double *d_x, double *res_inf);

/* ---- launch timing ---------------------------------------------------------- */

/* Kernel classes that can be timed. */
enum {
    LSMG_KERNEL_SMOOTH = 0,    /* one smoothing launch: one colour of the collective red-black
                                * sweep, or both colours of a fused 2-D sweep (fused_sweep) */
    LSMG_KERNEL_DEFECT = 1,    /* defect r = rhs - J x */
    LSMG_KERNEL_RESTRICT = 2,  /* restriction onto `level` from level - 1 */
    LSMG_KERNEL_PROLONG = 3,   /* prolongation onto `level` from level + 1 */
    LSMG_KERNEL_GHOST = 4      /* the ghost relaxation of a smoothing step (each of its launches) */
};

/* Start timing every launch of `kernel` on `level` of this hierarchy: a HIP
 * event is recorded on the hierarchy's stream before and after each launch.
 * While timing is on, V-cycles run as direct launches rather than as a
 * replayed graph (events inside a graph cannot be timed).  Synchronises the
 * stream.  Timing adds two event records per launch. */
lsmg_status lsmg_profile_start(lsmg_hierarchy *h, int kernel, int level);

/* Stop timing; host outs: number of timed launches and the sum of their
 * event-to-event durations in milliseconds.  Synchronises the stream. */
lsmg_status lsmg_profile_stop(lsmg_hierarchy *h, int *launches, double *total_ms);

/* Device memory: the bytes a hierarchy holds now (its levels, tables and
 * composed ghost maps) and the bytes of one state of it.  Host pointers;
 * either may be NULL. */
lsmg_status lsmg_memory_bytes(const lsmg_hierarchy *h, size_t *hierarchy_bytes, size_t *state_bytes);

/* The same before building, from the grid and parameters alone: the storage-
 * layout arrays of every level exactly, plus an allowance (10 % and 64 MiB)
 * for the geometry-dependent tables; for admission by memory footprint. */
lsmg_status lsmg_estimate_bytes(const lsmg_grid *grid, const lsmg_params *params, size_t *hierarchy_bytes,
                                size_t *state_bytes);

/* ------------------------------------------------------------------------
 * Batches: many hierarchies advanced by one Crank-Nicolson step together
 * (sections 3.1-3.5 for each member), with one launch per kernel and grid
 * size for all members.  A member's results are bitwise those of
 * lsmg_newton_cn_step on it alone: the batch runs each member's own V-cycle
 * operations in the same order on its own data, and its stopping decisions per
 * member with the same rules.
 * ------------------------------------------------------------------------ */
typedef struct lsmg_batch lsmg_batch;

/* Build a batch over count >= 1 distinct hierarchies (host array of handles).
 * All members must have the same dim and the same parameters (precision,
 * cycle, tolerances, ghost_c_new = 1); a mixed-precision batch needs members
 * built (or set) with precision 1.  The members stay owned by the caller and
 * must outlive the batch; while a batch call runs, a member must not be used
 * on its own.  All batch work runs on `stream` (NULL = null stream); building
 * synchronises it.  The batch holds the members' concatenated level
 * descriptors and work lists, per-member norm slots and flags, in device
 * memory from `allocator` (host, may be NULL: hipMalloc / hipFree).
 * Errors: EINVAL (NULL, duplicates, mismatched members), ENOTIMPL
 * (ghost_c_new = 0), EOOM, EHIP. */
lsmg_status lsmg_batch_create(lsmg_hierarchy *const *members, int count, const lsmg_allocator *allocator,
                              void *stream, lsmg_batch **out);
void lsmg_batch_destroy(lsmg_batch *b);

/* One Crank-Nicolson step with time step dt for every member k: states[k]
 * (host array; a state of members[k]) goes from W^n to W^{n+1}.  Boundary
 * values s_b at t_{n+1}: d_sb[k] (device, Ng doubles of member k) if d_sb and
 * d_sb[k] are non-NULL, else sb_const[k] (host array; 1.0 if sb_const is
 * NULL).  status[k] (host, optional) gets member k's own status with the
 * meaning of lsmg_newton_cn_step's; a member that fails keeps W^n.  stats[k]
 * (host, optional) as for lsmg_newton_cn_step.  Returns LSMG_OK if every
 * member converged, else the first failing member's status.  Synchronises the
 * batch stream.  On the first step the batch autotunes its launch shapes
 * (lsmg_batch_set_autotune), which changes no result. */
lsmg_status lsmg_batch_step(lsmg_batch *b, lsmg_state *const *states, double dt, const double *const *d_sb,
                            const double *sb_const, lsmg_status *status, lsmg_step_stats *stats);

/* Continuous batching at V-cycle granularity.  Every member runs its own
 * Crank-Nicolson steps with the stopping rules of lsmg_newton_cn_step, and
 * each tick of the batch issues, for every member, the next piece of its step:
 * the explicit half and residual of a new step with its first linearisation,
 * one V-cycle (or FP64 refinement step), a Newton update and residual, or the
 * linearisation of a new Newton iteration (with its first cycle).  Members in
 * different phases share every launch of a tick; a member's results are
 * bitwise those of lsmg_newton_cn_step alone.
 * remaining[k] (host): 0 or the number of steps member k still has to do;
 *   a member starts a new step only when remaining[k] > 0, and a step in
 *   progress always continues.  The progress of a step lives with the
 *   hierarchy, so a member can move to a new batch between calls.
 * Runs ticks until some member ends a step (converged or failed) or
 * max_ticks ticks have run, then returns.  Per member (host arrays, each
 * optional): ended[k] = 1 if its step ended in this call, status[k] its
 * outcome (a failed step keeps W^n and the member starts no further step
 * until called with remaining[k] > 0 again), stats[k] that step's statistics,
 * step_ms[k] its wall time from the tick that started it to the tick that
 * ended it.  *ticks_run: ticks run.  Boundary values sb_const[k] (NULL: 1.0).
 * Synchronises the batch stream. */
lsmg_status lsmg_batch_advance(lsmg_batch *b, lsmg_state *const *states, double dt, const double *sb_const,
                               const int *remaining, int max_ticks, int *ended, lsmg_status *status,
                               lsmg_step_stats *stats, double *step_ms, int *ticks_run);

/* Autotuning of the batch's launch shapes (enable != 0, the default): on the
 * first step, for every grid size and kernel class (smoother, ghost
 * relaxation, defect, restriction, prolongation, band), the workgroup size of
 * 1, 2, 4 or 8 wavefronts with the least measured launch time is kept.
 * Disabling it restores the default of 4. */
lsmg_status lsmg_batch_set_autotune(lsmg_batch *b, int enable);

/* The batch's grid sizes (finest first) and their chosen workgroup sizes in
 * wavefronts, 6 per size in the class order above; cap bounds the entries
 * written (host arrays sizes[cap], ipb[6 * cap]); *count gets the number of
 * sizes. */
lsmg_status lsmg_batch_tuning(const lsmg_batch *b, int cap, int *count, int *sizes, int *ipb);

/* The same as lsmg_sweep_fused for the batch's launches at grid size n (the
 * active nodes summed over the member levels of that size outside the coarse
 * tails); *fused = 0 for a size the batch does not have. */
lsmg_status lsmg_batch_sweep_fused(const lsmg_batch *b, int n, int precision, int *fused);

/* Launch timing inside a batch, as lsmg_profile_start / lsmg_profile_stop:
 * every launch of kernel class `kernel` (LSMG_KERNEL_*) at grid size n (for
 * LSMG_KERNEL_RESTRICT: the launch that restricts from size n) is timed by
 * its own dispatch events until lsmg_batch_profile_stop, which returns the
 * number of timed launches and their total time in ms; while timing is on,
 * the batch's V-cycles run as direct launches instead of its captured graph.
 * Both synchronise the batch stream. */
lsmg_status lsmg_batch_profile_start(lsmg_batch *b, int kernel, int n);
lsmg_status lsmg_batch_profile_stop(lsmg_batch *b, int *launches, double *total_ms);

/* Thread-local message for the last non-OK status of this thread. */
const char *lsmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LSMG_H */
