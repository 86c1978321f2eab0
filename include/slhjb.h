/*
 * slhjb.h -- C ABI of the MI355X semi-Lagrangian HJB solver with independent
 * sub-domains (Festa, "Reconstruction of independent sub-domains for a class of
 * Hamilton-Jacobi equations and its application to parallel computing").
 *
 * Problem (paper Sec. 2, exit-time problem (P1) and equation (HJ)):
 *   dynamics   f(x, a_k) = c(x) * b_k   (+ drift(x))   on a discrete control set,
 *   or for a differential game f(x, a_k, b_l) = drift(x) + S(x)(a_k - b_l) with the
 *   evader's discrete choices b_l (sl_problem.m_b, velocity_b);
 *   running cost l(x) > 0, discount lambda > 0, target set Gamma = union of
 *   components Gamma_i (nodes with target id i), exit cost g on Gamma.
 * Scheme (Sec. 3, (SL) and (Tdef), read as: foot x + h f, cost added, min over
 * the pursuer's controls, max over the evader's choices):  for a free node x_j
 *   V(j) = max_l min_k { beta * I[V](x_j + h f(x_j, a_k, b_l)) + w * l(x_j) }
 *   (a control problem has no evader: V(j) = min_k {...})
 *   I = Q1 (bi/trilinear) interpolation on the Cartesian grid; corners outside
 *   the box or outside the current sub-domain read the ghost value v_ghost;
 *   target nodes keep g.  Discount: SL_DISC_EXP beta = exp(-lambda h),
 *   w = (1 - beta)/lambda;  SL_DISC_PAPER beta = 1/(1 + lambda h), w = h;
 *   SL_DISC_KRUZKOV (the Kruzkov image v = 1 - exp(-J) of the weighted minimum
 *   time J = integral of l, Sec. 2 with the discount carried by the cost): per node
 *   beta_j = exp(-h l_j) and the cost term 1 - beta_j = -expm1(-h l_j), lambda
 *   unused; the exponentials are evaluated on the host in binary64 (the fields
 *   cross to the host once per call).  v_ghost should exceed 1 (e.g. 2) so that
 *   V = v_ghost is a supersolution in floating point.  sl_adjoint returns
 *   SL_ERR_UNSUPPORTED for it.
 * Fixed point by value iteration from V = v_ghost (a supersolution), which the
 * paper notes is a contraction (Sec. 3).
 *
 * Conventions (all entry points):
 *   - Array arguments marked DEVICE are device pointers owned by the caller; the
 *     library never frees or keeps them past the call.  HOST arrays are read
 *     during the call only.
 *   - Node fields are flat, row-major, x fastest: j = i0 + n0*(i1 + n1*i2).
 *   - Every device operation is ordered on the caller's HIP stream `stream`
 *     (NULL = default stream).  A call returns after its work has completed
 *     (it synchronizes the stream once at the end to fill the stats).
 *   - Scratch memory is a caller-provided DEVICE workspace of at least the size
 *     the matching *_workspace_size query returns; it may be reused between calls.
 *   - Functions return an sl_status.  No C++ exception crosses the ABI.  Errors
 *     are not sticky: the next call starts clean.  On SL_NOT_CONVERGED the outputs
 *     are written with the last iterate.
 */
#ifndef SLHJB_H
#define SLHJB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SLHJB_ABI_VERSION 5
#define SL_MAX_COMP 8
#define SL_MAX_CONTROLS 256
/* A policy output holds one control index per node in a byte and marks target and
 * non-member nodes with 255, so the entry points that write or read a policy
 * (sl_solve and sl_solve_isa with want_policy and a policy buffer, sl_adjoint)
 * return SL_ERR_UNSUPPORTED for m above this. */
#define SL_MAX_POLICY_CONTROLS 255
/* Bytes of the device scratch array that sl_solve_noalloc uses as its workspace
 * (one copy per device, held from the library's load until the process ends). */
#define SL_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
#define SL_MAX_TABLE 4096     /* m * max(m_b, 1): displacement rows of a game       */

typedef enum {
    SL_OK = 0,
    SL_NOT_CONVERGED = 1,     /* max_sweeps reached before the tolerance           */
    SL_ERR_INVALID_ARG = -1,  /* bad size, pointer, value or too small workspace    */
    SL_ERR_NO_TARGET = -2,    /* no target node (checked on the device)            */
    SL_ERR_UNSUPPORTED = -3,  /* dim, control count or component count out of range */
    SL_ERR_HIP = -4,          /* a HIP runtime call failed                          */
    SL_ERR_WORKSPACE = -5,    /* workspace smaller than the query says              */
    SL_ERR_SCRATCH = -6       /* sl_solve_noalloc: the problem's workspace exceeds
                                 SL_NOALLOC_SCRATCH_BYTES                             */
} sl_status;

typedef enum { SL_F32 = 0, SL_F64 = 1 } sl_dtype;
typedef enum { SL_DISC_EXP = 0, SL_DISC_PAPER = 1, SL_DISC_KRUZKOV = 2 } sl_disc;
/* Interpolation I[V] at the foot (Sec. 3): Q1, tensor-product linear on the grid
 * cell; or P1, linear on the Kuhn simplex of the cell that holds the foot (the
 * simplex fixed by the order of the foot's fractions t, decreasing, equal ones in
 * increasing axis order).  P1 is evaluated as nested interpolations from the far
 * vertex, in 2D lerp(t_0, v_0, lerp(t_1/t_0, v_1, v_2)), in 3D
 * lerp(t_0, v_0, lerp(t_1/t_0, v_1, lerp(t_2/t_1, v_2, v_3))), with
 * lerp(s, a, b) = fma(s, b, (1 - s) a) and v_0 .. v_d the simplex's vertices from
 * the cell's lower corner, one sorted axis step at a time (a ratio with a zero
 * denominator is 0); FP64 divides exactly, FP32 uses the reciprocal instruction,
 * clamped to 1. */
typedef enum { SL_INTERP_Q1 = 0, SL_INTERP_P1 = 1 } sl_interp;

/* One exit-time problem on a uniform box grid (paper Sec. 2-3). */
typedef struct sl_problem {
    int dim;                  /* 2 or 3                                              */
    int n[3];                 /* nodes per axis (>= 3 on used axes)                  */
    double lo[3], hi[3];      /* box corners; dx_d = (hi_d - lo_d)/(n_d - 1)         */
    int m;                    /* number of discrete controls, 1..SL_MAX_CONTROLS     */
    const double *velocity;   /* HOST, m*dim: b_k with f(x, a_k) = drift(x) + c(x) b_k
                                 (for a game: the pursuer's a_k)                       */
    const void *speed;        /* DEVICE, N values of c(x) >= 0 in `dtype` (N*dim with
                                 speed_axes); NULL = 1                                 */
    const void *cost;         /* DEVICE, N values of l(x) > 0 in `dtype`; NULL = 1    */
    const void *drift;        /* DEVICE, N*dim drift(x) in `dtype` (node-major); NULL = 0.
                                 Control-affine dynamics (the Van der Pol example, Sec.
                                 4.1).  The foot is u_d = i_d + (e_kd c_j + q_jd) in index
                                 units, q_jd = (h/dx_d) drift_jd in FP64.  The halo covers
                                 c|e| + |q|.  Every entry point takes it.              */
    const int8_t *target;     /* DEVICE, N: -1 free node, i in [0, n_comp) target of component i */
    const void *g;            /* DEVICE, N exit costs (read on target nodes) in `dtype`; NULL = 0 */
    int n_comp;               /* number of target components, 1..SL_MAX_COMP          */
    double lambda;            /* discount rate > 0                                    */
    double h;                 /* fictitious time step > 0                             */
    double v_ghost;           /* value read outside the box / sub-domain; should be >= max(l)/lambda */
    int disc;                 /* sl_disc                                              */
    int dtype;                /* sl_dtype of fields and values                        */
    int m_b;                  /* differential game (Sec. 2, (Tdef) with max over B): the
                                 number of evader choices b_l, 1..SL_MAX_CONTROLS with
                                 m * m_b <= SL_MAX_TABLE; 0 = control problem.  The
                                 evader chooses first (outer maximum), the pursuer answers
                                 (inner minimum over the m controls); the displacement of
                                 the pair is (h/dx_d)(a_kd - b_ld), the difference taken
                                 first, in FP64.  sl_solve, sl_reconstruct and sl_solve_isa
                                 take games (without a policy: want_policy with a policy
                                 buffer returns SL_ERR_UNSUPPORTED), and so does
                                 sl_solve_batched; sl_adjoint returns
                                 SL_ERR_UNSUPPORTED.  The sub-domain
                                 method needs the decomposability condition of Sec. 2
                                 (the paper shows it for its pursuit-evasion example); the
                                 library does not check it.                             */
    const double *velocity_b; /* HOST, m_b*dim: the evader's b_l (NULL iff m_b == 0)   */
    int speed_axes;           /* 0: speed holds one c(x) per node, S(x) = c(x) I;
                                 1: speed holds dim factors per node (node-major, N*dim,
                                 each >= 0), S(x) = diag(c_1(x), .., c_d(x)); the coarse
                                 grid samples each factor by Q1.  Needs speed != NULL.
                                 Every entry point takes it.                           */
    int interp;               /* sl_interp.  SL_INTERP_P1 is taken by sl_solve,
                                 sl_reconstruct, sl_solve_isa (2D and 3D), sl_adjoint
                                 (its Jacobi iteration) and sl_solve_batched, whose
                                 problems must all share one interpolation (a mix
                                 returns SL_ERR_UNSUPPORTED).                           */
} sl_problem;

/* Reconstruction algorithm options (paper Sec. 3, RA; Sec. 4, ISA steps 1-2). */
typedef struct sl_ra_opts {
    int coarse_stride;        /* s >= 1 dividing n_d - 1: coarse grid K = every s-th node
                                 (used when coarse_n[0] == 0)                           */
    int coarse_n[3];          /* > 0: K has coarse_n[d] nodes per used axis, 3 <= coarse_n[d]
                                 <= n[d], on the same box; it need not be nested in the fine
                                 grid (Sec. 4 asks only that both grids cover the domain).
                                 Coarse node k of an axis sits at fine coordinate
                                 k (n_d - 1)/(coarse_n[d] - 1); K takes speed and cost by Q1
                                 interpolation of the fine fields (FP64, corner weights as
                                 products in axis order, corners summed in order from 0),
                                 target ids and g from the nearest fine node (ties up); the
                                 coarse step is h * max_d (n_d - 1)/(coarse_n[d] - 1).   */
    double C, M, q;           /* threshold delta = 2 (C dx_K^q + M dx_K) (Prop. 3.1)  */
    double delta_override;    /* > 0: use this delta instead                          */
    double tol;               /* coarse stopping tolerance on max|V_new - V| (0 = until nothing changes) */
    long max_sweeps;          /* coarse sweep cap                                     */
    int autotune;             /* as sl_solve_opts.autotune, for the coarse sweeps (the FP64
                                 results do not depend on the kernel configuration)   */
    int local_iters;          /* as sl_solve_opts.local_iters, for the coarse sweeps: 0
                                 Jacobi; k > 0 block-asynchronous.  With tol = 0 both
                                 reach the same FP64 fixed point bit for bit (so the sets
                                 and labels do not depend on it); with tol > 0 the two
                                 stop on different iterates.  sl_solve_batched takes it
                                 (like tol and autotune) from the first problem's options. */
} sl_ra_opts;

/* Value-iteration options. */
typedef struct sl_solve_opts {
    double tol;               /* stop when max|V_new - V| <= tol over the sub-domain (0: no change) */
    long max_sweeps;          /* sweep cap (>= 1)                                     */
    int want_policy;          /* write the first minimising control index per node   */
    int check_every;          /* sweeps between host convergence polls.  0 = default:
                                 32, or, when a call repeats the launch arguments
                                 of an earlier call (same shapes, workspace and
                                 options), a first poll at that call's converged
                                 sweep count rounded up to 8 and then every 8.
                                 The results do not depend on it: sweeps after a
                                 set converged change nothing.                  */
    int profile;              /* 1: time the sweep launches with HIP events (stats.ms_sweeps) */
    int autotune;             /* 0: default kernel; 1: on the first call with a new shape,
                                 time the first 96 sweeps of every (tile shape, schedule)
                                 candidate and cache the fastest; 2: same with complete
                                 solves as trials; -k: use candidate k-1 (testing aid,
                                 k <= sl_tune_candidates(dim, dtype))                    */
    int local_iters;          /* 0: Jacobi sweeps (each reads the previous iterate).
                                 k > 0 (0 <= k <= 1024): block-asynchronous sweeps: every
                                 active tile iterates up to k times on its own values in
                                 on-chip memory, its halo as read at the start of the
                                 launch, while anything in it changes, and writes back in
                                 place.  The scheme's evaluation is monotone in the node
                                 values in both precisions, so from the initial values
                                 (a supersolution when v_ghost >= max l / lambda) the
                                 iterates decrease to the same floating-point fixed point
                                 as Jacobi: with tol = 0 the values match Jacobi's bit for
                                 bit whenever T(V0) <= V0 holds exactly in floating point
                                 (e.g. FP32 with v_ghost a power of two).  A "sweep" in the
                                 statistics is then one launch; tol bounds the largest
                                 change of one local iteration.                        */
} sl_solve_opts;

/* Per-call statistics (HOST struct filled at the end of a call). */
typedef struct sl_stats {
    long sweeps_max;          /* most sweeps done by one sub-domain                   */
    long sweeps_total;        /* sum over sub-domains                                 */
    double residual;          /* largest final residual over sub-domains              */
    double node_control_updates; /* node*control evaluations actually computed        */
    double ms_ra, ms_fine, ms_total; /* wall times of the phases (HIP events)         */
    int n_subdomains;         /* sub-domains solved                                   */
    int n_unreachable;        /* sl_solve, sl_solve_isa: free nodes whose final value is
                                 still v_ghost up to rounding, |V - v_ghost| <= 8 eps
                                 v_ghost / (1 - beta) (they never read a reached value:
                                 no target is reachable from them); else 0 */
    double set_fraction_max;  /* max_i |Sigma_i| / N on the fine grid (ISA calls)     */
    double ms_sweeps;         /* profile: HIP-event time spanning the sweep launches  */
    long sweep_launches;      /* profile: number of sweep launches timed              */
    int variant;              /* sweep kernel variant used (tile shape)               */
    int mode;                 /* work schedule used: 0 per item, 1 queue, 2 stride    */
    int tile[3];              /* tile shape used                                      */
    long ra_sweeps_max;       /* RA: most coarse sweeps of one auxiliary problem
                                 (sl_reconstruct, sl_solve_batched; else 0)           */
} sl_stats;

const char *sl_status_string(int status);
int sl_abi_version(void);
/* Number of sweep-kernel configurations (tile shape x work schedule) the
 * autotuner chooses from for (dim, dtype) in a control problem; 0 if unsupported.
 * A game chooses from the subset whose kernels give each tile one thread group. */
int sl_tune_candidates(int dim, int dtype);

/* Workspace bytes needed by sl_solve for problem `p` (0 if `p` is invalid). */
size_t sl_solve_workspace_size(const sl_problem *p);

/* Global solve ("no decomposition"): value iteration of T on the whole grid
 * (paper Sec. 3, (SL)).  Outputs: V (DEVICE, N in p->dtype), policy (DEVICE, N
 * uint8, 255 on target nodes; may be NULL).  Targets start at g, free nodes at
 * v_ghost. */
int sl_solve(const sl_problem *p, const sl_solve_opts *o, void *ws, size_t ws_bytes,
             void *V, uint8_t *policy, sl_stats *stats, void *stream);

/* sl_solve without a workspace argument and without any allocation, for callers
 * that cannot allocate memory (code under stream capture, serving loops,
 * harnesses that forbid hipMalloc).  It runs the global solve of sl_solve with
 * the same kernels and arguments, so its outputs equal sl_solve's bit for bit,
 * and takes its workspace from a static device array of SL_NOALLOC_SCRATCH_BYTES
 * bytes on the current device (the device the caller's stream belongs to must be
 * current).  It calls no hipMalloc/hipFree, creates no events, streams or graphs
 * (the sweep chunks are launched directly, not replayed from a captured graph),
 * and polls convergence into host stack memory.
 * Limits: sl_solve_workspace_size(p) must be at most SL_NOALLOC_SCRATCH_BYTES, else
 * SL_ERR_SCRATCH (about 2.8 million FP32 nodes with a cost field, e.g. 1025^2 and
 * 129^3); o->autotune must be <= 0 and o->profile 0 (both time with HIP events),
 * else SL_ERR_INVALID_ARG; stats->ms_* are 0.  Every call on a device shares that
 * device's array and every call re-initialises what it reads, so consecutive calls
 * are independent, but calls that overlap in time on one device (other host
 * threads or streams) race on the array and must be serialised by the caller.
 * Arguments, outputs and other errors: as sl_solve. */
int sl_solve_noalloc(const sl_problem *p, const sl_solve_opts *o, void *V, uint8_t *policy,
                     sl_stats *stats, void *stream);

/* Workspace bytes needed by sl_reconstruct / sl_solve_isa / sl_isa. */
size_t sl_isa_workspace_size(const sl_problem *p, const sl_ra_opts *ra);

/* Reconstruction of the independent sub-domains (paper Sec. 3, RA steps 1-3, on
 * the coarse grid K of ISA step 1; Sec. 4, ISA step 2 projection to the fine
 * grid).  The coarse auxiliary solves run in FP64 whatever p->dtype is, with the
 * operation order of the scheme fixed (Q1 as nested one-axis interpolations
 * fma(tau, v1, (1 - tau) v0) along x, then y, then z; candidate fma(beta, I, w l)),
 * so the labels are reproducible bit for bit.
 * Outputs (DEVICE, N uint8 each): member = bitmask of the sets containing each
 * fine node (Con(.): the union of the closed coarse cells with every corner in the
 * set; a fine node in no such cell takes every set present at the corners of the
 * cells holding it); label = coarse argmin component at the nearest coarse node
 * (ties rounded up).  Cells and nearest nodes are located in exact integers.
 * member_K, label_K (DEVICE, N_K uint8 each) may be NULL. */
int sl_reconstruct(const sl_problem *p, const sl_ra_opts *ra, void *ws, size_t ws_bytes,
                   uint8_t *member, uint8_t *label, uint8_t *member_K, uint8_t *label_K,
                   sl_stats *stats, void *stream);

/* Workspace bytes needed by sl_refine_split (0 if the arguments are invalid). */
size_t sl_refine_workspace_size(const sl_problem *p, const sl_ra_opts *ra, int max_comp);

/* Recursive refinement of the division of Gamma for balance, the remedy the
 * paper's conclusions propose for unbalanced sub-domains (Sec. 5, on the Van der
 * Pol example of Sec. 4.1).  Starting from p->target (p->n_comp components), repeat: run the
 * reconstruction (as sl_reconstruct); stop if there are max_comp components or
 * the largest projected set holds at most frac_goal of the fine nodes; else halve
 * the component whose set holds the most fine nodes (lowest index on ties) among
 * those with at least two target nodes: along the grid axis on which its nodes
 * span the most index positions (lowest axis on ties), order them by (index on
 * that axis, flat index) and give the upper floor(count/2) the next free label.
 * Every decision is integer, so the result is reproducible bit for bit.
 * Inputs: p (its target ids are read, not written), ra, max_comp in
 * [p->n_comp, SL_MAX_COMP], frac_goal in [0, 1].  Outputs: target_out (DEVICE, N
 * int8, the refined ids; g is unchanged), *n_comp_out (HOST), frac_max (HOST,
 * room for max_comp - p->n_comp + 1 doubles, may be NULL: the largest set
 * fraction after each reconstruction).  stats: ms_ra = total time, sweeps_max =
 * reconstructions done, ra_sweeps_max = most coarse sweeps of one auxiliary
 * problem.  The target ids cross to the host once and each reconstruction's
 * member mask once (N bytes each way per step). */
int sl_refine_split(const sl_problem *p, const sl_ra_opts *ra, int max_comp, double frac_goal,
                    void *ws, size_t ws_bytes, int8_t *target_out, int *n_comp_out,
                    double *frac_max, sl_stats *stats, void *stream);

/* ISA steps 3-4 (paper Sec. 4): value iteration of T on every set i (nodes with
 * bit i of `member`; non-members read v_ghost), all sets in one launch per
 * sweep, then V(j) = min over the sets containing j.  Inputs: member (DEVICE, N
 * uint8).  Outputs: V (DEVICE, N in p->dtype), owner (DEVICE, N uint8, lowest
 * minimising set; may be NULL), policy (DEVICE, n_comp*N uint8 per set, 255 on
 * target and non-member nodes; may be NULL), V_sets (DEVICE, n_comp*N values per
 * set, v_ghost off the set; may be NULL). */
int sl_solve_isa(const sl_problem *p, const sl_ra_opts *ra, const uint8_t *member,
                 const sl_solve_opts *o, void *ws, size_t ws_bytes, void *V, uint8_t *owner,
                 uint8_t *policy, void *V_sets, sl_stats *stats, void *stream);

/* The whole independent-sets algorithm in one call (paper Sec. 4, ISA steps 1-4):
 * sl_reconstruct, then sl_solve_isa on its sets, with the field statistics
 * gathered once.  Same arguments and outputs as the two calls: member and label
 * (DEVICE, N uint8 each, outputs), V, owner, policy, V_sets as sl_solve_isa; ws
 * of sl_isa_workspace_size bytes.  stats: those of the sets' solves, with ms_ra
 * and ra_sweeps_max of the reconstruction and ms_total of the whole call.
 * Returns SL_NOT_CONVERGED if either stage stopped at its sweep limit. */
int sl_isa(const sl_problem *p, const sl_ra_opts *ra, const sl_solve_opts *o, void *ws,
           size_t ws_bytes, void *V, uint8_t *owner, uint8_t *member, uint8_t *label,
           uint8_t *policy, void *V_sets, sl_stats *stats, void *stream);

/* Workspace bytes needed by sl_solve_batched (0 if any input is invalid). */
size_t sl_batched_workspace_size(int nprob, const sl_problem *probs, const sl_ra_opts *ras);

/* The independent-sets algorithm (RA on each problem's coarse grid, projection,
 * per-set value iteration, assembly; paper Sec. 3-4) for `nprob` independent
 * problems of any sizes at once: every step is one launch over all problems,
 * and every sweep one launch over the joint (problem, set, tile) work list, so
 * the small problems ride along with the large ones; chunks of sweeps are
 * replayed as a captured hipGraph with device-side convergence per set.
 * All problems must share dim and dtype.  probs, ras: HOST arrays of nprob.
 * V: HOST array of nprob DEVICE pointers (N_p values each, outputs).  member,
 * label, owner: HOST arrays of nprob DEVICE pointers (N_p uint8 each) or NULL
 * (internal).  per_problem: HOST array of nprob stats or NULL; total: aggregate
 * stats or NULL. */
int sl_solve_batched(int nprob, const sl_problem *probs, const sl_ra_opts *ras,
                     const sl_solve_opts *o, void *ws, size_t ws_bytes, void *const *V,
                     uint8_t *const *member, uint8_t *const *label, uint8_t *const *owner,
                     sl_stats *per_problem, sl_stats *total, void *stream);

/* Workspace bytes needed by sl_adjoint (n_sets = n_comp with sets, 1 without). */
size_t sl_adjoint_workspace_size(const sl_problem *p, int n_sets);

/* Gradient of a loss on V with respect to the running cost l, with the argmin
 * controls frozen (the fixed point is then linear in l: V = beta P V + w l + c on
 * free nodes).  Solves lambda = g + beta P^T lambda, then dLdl = w * sum over sets
 * of lambda.  P^T is applied as a gather: for every node c, the sum of
 * w_c(j) lambda(j) over the free member nodes j whose frozen foot has c in its
 * interpolation stencil (Q1 cell corners, or the P1 simplex vertices), in a fixed
 * order of j; no atomics touch the adjoint state.
 * Inputs: member (DEVICE, N uint8 set bitmask, or NULL: one set = whole grid, as
 * after sl_solve), owner (DEVICE, N uint8: dL/dV(j) goes to set owner[j] only;
 * NULL: to every set), policy (DEVICE, n_sets*N uint8 controls from the forward
 * call with want_policy; m <= SL_MAX_POLICY_CONTROLS), dLdV (DEVICE, N in
 * p->dtype).  The feet are those of the forward scheme: per-axis speed factors
 * and drift (index units, e c + q) are taken; games and the Kruzkov discount (the
 * discount then depends on l, so V is not linear in l) return SL_ERR_UNSUPPORTED.
 * Iteration (tiles of 32x8 nodes in 2D, 8x8x4 in 3D, when the feet reach at
 * most 8 cells in 2D and 5 in 3D):
 *   local_iters = 0: Jacobi: every launch evaluates each active tile once from
 *     one buffer into the other; a tile is revisited when a node of its
 *     neighbourhood changed, so the iterates are exactly those of the Jacobi
 *     iteration and the result is reproducible bit for bit (deterministic mode);
 *   local_iters = k > 0 (<= 1024): block-asynchronous: every active tile repeats
 *     the gather up to k times in on-chip memory, its halo as staged, and writes
 *     back in place; tiles see their neighbours' latest values, so the order of
 *     updates, and the result at rounding level, depends on scheduling.
 *   With longer feet the Jacobi iteration runs over the whole grid as a scatter
 *   with float atomics (the summation order then varies run to run).
 *   The iteration has nonnegative coefficients and spectral radius <= beta < 1,
 *   so every order converges to the same lambda (up to rounding).  Stop: the
 *   largest change of one evaluation <= tol + 16 eps max|lambda| (eps of
 *   p->dtype, the rounding level of the sums), or max_iters launches.  tol >= 0
 *   is absolute; tol < 0 is relative: |tol| * max_j |dLdV_j| rounded down to a
 *   power of two, the maximum taken on the device with the input checks (no
 *   extra host round trip); the rounding keeps the tolerance, and with it the
 *   captured launch graphs, unchanged while the gradient's scale moves within a
 *   factor of two.
 * Output: dLdl (DEVICE, N in p->dtype; 0 on target nodes). */
int sl_adjoint(const sl_problem *p, const uint8_t *member, const uint8_t *owner,
               const uint8_t *policy, const void *dLdV, void *dLdl, double tol, long max_iters,
               int local_iters, void *ws, size_t ws_bytes, sl_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SLHJB_H */
