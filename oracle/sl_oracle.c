/*
 * FP64 CPU oracle for the semi-Lagrangian (SL) value iteration of the discounted
 * exit-time Hamilton-Jacobi-Bellman problem, and for its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with the
 * HIP library: it is written from the paper's definitions, plainly and slowly.
 *
 * What it computes (paper, Section 3, scheme (SL) and operator (Tdef)):
 *   for a free node x_j of the solve domain
 *     [T(V)]_j = max_l min_k { beta * I[V](x_j + h f(x_j, a_k, b_l)) + w * l(x_j) }
 *   (a differential game, Sec. 2; with one evader choice b_0 = 0 it is the
 *   control problem's min_k)
 *   fixed (target) nodes keep their value, nodes outside the box or outside the
 *   solve domain read the ghost value G (the paper's ghost nodes, finite here).
 *   I is tensor-product linear (Q1) interpolation on the Cartesian grid, or
 *   piecewise linear (P1) interpolation on the Kuhn triangulation of its cells
 *   (Sec. 3 states the scheme with P1 on a simplicial grid).
 *   The fixed point is found by the plain (Jacobi) iteration V <- T(V) (Sec. 3,
 *   "the fixed point ... is found through the iterative map", a contraction).
 *
 * Readings of the paper used here (each is listed in the design notes):
 *   - foot at x + h f and cost added with +, minimum over the discrete controls
 *     (the printed signs of (Tdef) are inconsistent with the Hamiltonian (HJ));
 *   - discount: "exp"   beta = exp(-lam h),  w = (1 - beta)/lam   (default),
 *               "paper" beta = 1/(1 + lam h), w = h               ((Tdef) as printed),
 *               "kruzkov" per node beta_j = exp(-h l_j), w l_j -> 1 - beta_j =
 *               -expm1(-h l_j): the Kruzkov image v = 1 - exp(-J) of the weighted
 *               minimum time J = integral of l along the trajectory (lam unused);
 *   - dynamics f(x, a_k, b_l) = drift(x) + S(x) (a_k - b_l), S(x) = c(x) times the
 *     identity, or diag(c_1(x), .., c_d(x)) when per-axis speed factors are given,
 *     evaluated in grid-index units:
 *       disp_d = (h/dx_d * (a_kd - b_ld)) * c_jd  (+ h/dx_d * drift_jd),
 *       u_d = i_d + disp_d
 *     (for a control problem, without evader choices, the difference is a_kd);
 *   - game order: the evader (maximising b) chooses first, the pursuer (minimising
 *     a) answers, as the max-min of (Tdef) is printed; the policy index of a node is
 *     l m + k for the first maximising l and, within it, the first minimising k;
 *   - interpolation in a fixed operation order: Q1 as the tensor product of
 *     one-axis linear interpolations, along x, then y, then z, each evaluated as
 *     fma(tau, v1, (1 - tau) * v0); an implementation that follows the same order
 *     gets bit-identical FP64 results.  Every rounding step is monotone in the node
 *     values, and a constant field equal to a power of two (the ghost value) is
 *     reproduced exactly;
 *   - P1 on simplices: each cell is split into the d! Kuhn simplices, the simplex of
 *     a point being fixed by the order of its fractions tau (descending; equal
 *     fractions in increasing axis order, which does not change the value).  With
 *     t_0 >= .. >= t_{d-1} the sorted fractions and v_0 .. v_d the vertices (v_0 the
 *     cell's lower corner, each next one a step along the next sorted axis), the
 *     barycentric weights are 1 - t_0, t_0 - t_1, .., t_{d-1}.  The value is taken
 *     as nested one-dimensional interpolations from the far vertex inwards,
 *       acc = v_d;  acc = lerp(t_i / t_{i-1}, v_i, acc) for i = d-1 .. 1;
 *       value = lerp(t_0, v_0, acc),   lerp(s, a, b) = fma(s, b, (1 - s) * a),
 *     (a ratio with t_{i-1} = 0 is 0), which expands to the barycentric form and
 *     keeps the two properties above: every step is monotone in the vertex values
 *     and a power-of-two constant is reproduced exactly.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see oracle/build.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_CORNERS 8

typedef struct {
    int dim;
    long n[3];
    long N;
    int m;                /* pursuer controls a_k (inner minimum)    */
    int mb;               /* evader choices b_l (outer maximum), >= 1 */
    double *e;            /* (mb*m)*dim, row l*m + k: (h/dx_d) * (a_kd - b_ld) */
    double *q;            /* N*dim: (h/dx_d) * drift_jd, or NULL     */
    const double *c;      /* speed per node (or per node and axis), or NULL (= 1) */
    int c_axes;           /* 1: c holds dim factors per node          */
    int interp;           /* 0: Q1 on cells; 1: P1 on Kuhn simplices  */
    double *wl;           /* w * l_j per node                        */
    double *bn;           /* per-node discount (Kruzkov form) or NULL */
    double beta;
    double G;
    const uint8_t *fixed; /* 1: value fixed (target node)            */
    const uint8_t *dom;   /* NULL (whole box) or 1: node in domain   */
} orc_prob;

/* Discount beta and cost weight w of one SL step of length h. */
int orc_scheme_constants(double lam, double h, int disc, double *beta, double *w)
{
    if (!(lam > 0.0) || !(h > 0.0) || !beta || !w) return -1;
    if (disc == 0) {                 /* exact integral of e^{-lam s} over [0, h] */
        *beta = exp(-lam * h);
        *w = -expm1(-lam * h) / lam;
    } else if (disc == 1) {          /* the printed (Tdef): 1/(1+lam h) and h    */
        *beta = 1.0 / (1.0 + lam * h);
        *w = h;
    } else if (disc == 2) {          /* Kruzkov form with l = 1: exp(-h), 1 - exp(-h) */
        *beta = exp(-h);
        *w = -expm1(-h);
    } else {
        return -1;
    }
    return 0;
}

static int prob_init(orc_prob *P, int dim, const int *n, const double *lo, const double *hi,
                     double h, int m, const double *b, const double *c, int mb,
                     const double *bb, int c_axes, int interp, const double *l, const double *drift,
                     double lam, int disc, double G, const uint8_t *fixed, const uint8_t *dom)
{
    double beta, w, t[3];
    memset(P, 0, sizeof(*P));
    if (dim < 1 || dim > 3 || m < 1) return -1;
    if (interp != 0 && interp != 1) return -1;
    if (bb ? mb < 1 : mb > 1) return -1;
    if (mb < 1) mb = 1;
    P->dim = dim;
    P->N = 1;
    for (int d = 0; d < 3; ++d) P->n[d] = 1;
    for (int d = 0; d < dim; ++d) {
        if (n[d] < 2) return -1;
        P->n[d] = n[d];
        P->N *= n[d];
        t[d] = h / ((hi[d] - lo[d]) / (double)(n[d] - 1));
    }
    if (orc_scheme_constants(lam, h, disc, &beta, &w)) return -1;
    P->m = m;
    P->mb = mb;
    P->e = (double *)malloc(sizeof(double) * (size_t)mb * m * dim);
    P->wl = (double *)malloc(sizeof(double) * (size_t)P->N);
    if (!P->e || !P->wl) return -2;
    for (int lb = 0; lb < mb; ++lb)
        for (int k = 0; k < m; ++k)
            for (int d = 0; d < dim; ++d) {
                const double rel = bb ? b[k * dim + d] - bb[lb * dim + d] : b[k * dim + d];
                P->e[((size_t)lb * m + k) * dim + d] = t[d] * rel;
            }
    if (drift) {
        P->q = (double *)malloc(sizeof(double) * (size_t)P->N * dim);
        if (!P->q) return -2;
        for (long j = 0; j < P->N; ++j)
            for (int d = 0; d < dim; ++d) P->q[j * dim + d] = t[d] * drift[j * dim + d];
    }
    if (disc == 2 && l) {
        P->bn = (double *)malloc(sizeof(double) * (size_t)P->N);
        if (!P->bn) return -2;
        for (long j = 0; j < P->N; ++j) {
            P->bn[j] = exp(-h * l[j]);
            P->wl[j] = -expm1(-h * l[j]);
        }
    } else {
        for (long j = 0; j < P->N; ++j) P->wl[j] = w * (l ? l[j] : 1.0);
    }
    P->c = c;
    P->c_axes = c_axes ? 1 : 0;
    P->interp = interp;
    P->beta = beta;
    P->G = G;
    P->fixed = fixed;
    P->dom = dom;
    return 0;
}

static void prob_free(orc_prob *P)
{
    free(P->e);
    free(P->q);
    free(P->wl);
    free(P->bn);
}

static inline void node_index(const orc_prob *P, long j, long *ij)
{
    ij[0] = j % P->n[0];
    ij[1] = (j / P->n[0]) % P->n[1];
    ij[2] = j / (P->n[0] * P->n[1]);
}

/* Speed factor of node j on axis d. */
static inline double speed_at(const orc_prob *P, long j, int d)
{
    if (!P->c) return 1.0;
    return P->c_axes ? P->c[j * P->dim + d] : P->c[j];
}

/* Fractional parts tau_d of the foot of table row k (= l m + k_a) from node j
 * (index units). */
static void foot_fractions(const orc_prob *P, long j, const long *ij, int k, double *tau)
{
    for (int d = 0; d < P->dim; ++d) {
        double disp = P->e[k * P->dim + d] * speed_at(P, j, d);
        if (P->q) disp = disp + P->q[j * P->dim + d];
        double u = (double)ij[d] + disp;
        tau[d] = u - floor(u);
    }
}

/* Axes in the order of decreasing fraction, equal fractions in increasing axis
 * order (insertion sort of at most three entries). */
static void kuhn_order(int dim, const double *tau, int *ax)
{
    for (int d = 0; d < dim; ++d) {
        int i = d;
        while (i > 0 && tau[ax[i - 1]] < tau[d]) {
            ax[i] = ax[i - 1];
            --i;
        }
        ax[i] = d;
    }
}

/* Interpolation stencil at the foot of control k from node j (Q1: the 2^dim cell
 * corners, bit d = upper node on axis d; P1: the dim + 1 simplex vertices in order
 * v_0 .. v_dim): corner node indices (-1 = ghost:
 * outside the box or outside the domain) and weights.  Returns the corner count. */
static int stencil(const orc_prob *P, long j, const long *ij, int k, long *cidx, double *wt)
{
    const int dim = P->dim;
    double tau[3];
    long p[3];
    for (int d = 0; d < dim; ++d) {
        double disp = P->e[k * dim + d] * speed_at(P, j, d);
        if (P->q) disp = disp + P->q[j * dim + d];
        double u = (double)ij[d] + disp;
        double fl = floor(u);
        tau[d] = u - fl;
        p[d] = (long)fl;
    }
    const int K = 1 << dim;
    if (P->interp == 1) {
        /* P1: the d + 1 vertices of the point's Kuhn simplex with their barycentric
         * weights, then the unused slots as absent corners of weight 0 */
        int ax[3];
        kuhn_order(dim, tau, ax);
        long pv[3] = {p[0], p[1], p[2]};
        for (int s = 0; s <= dim; ++s) {
            if (s > 0) pv[ax[s - 1]] += 1;
            double w;
            if (s == 0) w = 1.0 - tau[ax[0]];
            else if (s < dim) w = tau[ax[s - 1]] - tau[ax[s]];
            else w = tau[ax[dim - 1]];
            long idx = 0, stride = 1;
            int inside = 1;
            for (int d = 0; d < dim; ++d) {
                if (pv[d] < 0 || pv[d] >= P->n[d]) inside = 0;
                idx += pv[d] * stride;
                stride *= P->n[d];
            }
            if (inside && P->dom && !P->dom[idx]) inside = 0;
            cidx[s] = inside ? idx : -1;
            wt[s] = w;
        }
        for (int s = dim + 1; s < K; ++s) {
            cidx[s] = -1;
            wt[s] = 0.0;
        }
        return dim + 1;
    }
    for (int s = 0; s < K; ++s) {
        double w = 0.0;
        long idx = 0, stride = 1;
        int inside = 1;
        for (int d = 0; d < dim; ++d) {
            int bit = (s >> d) & 1;
            double f = bit ? tau[d] : 1.0 - tau[d];
            w = (d == 0) ? f : w * f;
            long pd = p[d] + bit;
            if (pd < 0 || pd >= P->n[d]) inside = 0;
            idx += pd * stride;
            stride *= P->n[d];
        }
        if (inside && P->dom && !P->dom[idx]) inside = 0;
        cidx[s] = inside ? idx : -1;
        wt[s] = w;
    }
    return K;
}

/* P1 value at the foot from the vertex values val[0..dim] of its Kuhn simplex
 * (stencil order): nested linear interpolations from the far vertex inwards. */
static double interp_p1(int dim, const double *tau, const double *val)
{
    int ax[3];
    kuhn_order(dim, tau, ax);
    double acc = val[dim];
    for (int i = dim - 1; i >= 0; --i) {
        double s;
        if (i == 0) s = tau[ax[0]];
        else s = tau[ax[i - 1]] > 0.0 ? tau[ax[i]] / tau[ax[i - 1]] : 0.0;
        acc = fma(s, acc, (1.0 - s) * val[i]);
    }
    return acc;
}

/* Q1 value at the foot from the corner values val[0..2^dim) (bit d of the corner
 * index = upper node on axis d): linear interpolation along axis 0 between corner
 * pairs (2s, 2s+1), then along axis 1 between the results, and so on. */
static double interp_q1(int dim, const double *tau, double *val)
{
    int cnt = 1 << dim;
    for (int d = 0; d < dim; ++d) {
        const double t = tau[d], a = 1.0 - t;
        for (int s = 0; s < cnt / 2; ++s) val[s] = fma(t, val[2 * s + 1], a * val[2 * s]);
        cnt /= 2;
    }
    return val[0];
}

/* One application of T at node j: the maximum over the evader's choices l of the
 * minimum over the pursuer's controls k.  *arg = l m + k of the first maximising l
 * and, within it, the first minimising k. */
static double apply_node(const orc_prob *P, long j, const double *V, int *arg)
{
    long ij[3], cidx[ORC_MAX_CORNERS];
    double wt[ORC_MAX_CORNERS], tau[3], val[ORC_MAX_CORNERS];
    node_index(P, j, ij);
    double best = 0.0;
    int bk = -1;
    for (int lb = 0; lb < P->mb; ++lb) {
        double inner = 0.0;
        int ik = -1;
        for (int ka = 0; ka < P->m; ++ka) {
            const int k = lb * P->m + ka;
            int K = stencil(P, j, ij, k, cidx, wt);
            foot_fractions(P, j, ij, k, tau);
            for (int s = 0; s < K; ++s) val[s] = cidx[s] >= 0 ? V[cidx[s]] : P->G;
            double r = P->interp == 1 ? interp_p1(P->dim, tau, val)
                                      : interp_q1(P->dim, tau, val);
            double cand = fma(P->bn ? P->bn[j] : P->beta, r, P->wl[j]);
            if (ik < 0 || cand < inner) {
                inner = cand;
                ik = k;
            }
        }
        if (bk < 0 || inner > best) {
            best = inner;
            bk = ik;
        }
    }
    *arg = bk;
    return best;
}

static inline int is_free(const orc_prob *P, long j)
{
    return !(P->fixed && P->fixed[j]) && !(P->dom && !P->dom[j]);
}

/* One Jacobi sweep Vn = T(V); returns max |Vn - V| over free domain nodes. */
static double sweep(const orc_prob *P, const double *V, double *Vn, int32_t *policy)
{
    double res = 0.0;
    const long N = P->N;
#pragma omp parallel for schedule(static) reduction(max : res)
    for (long j = 0; j < N; ++j) {
        if (P->dom && !P->dom[j]) {
            Vn[j] = P->G;
            if (policy) policy[j] = -1;
            continue;
        }
        if (P->fixed && P->fixed[j]) {
            Vn[j] = V[j];
            if (policy) policy[j] = -1;
            continue;
        }
        int arg;
        double v = apply_node(P, j, V, &arg);
        Vn[j] = v;
        if (policy) policy[j] = arg;
        double dv = fabs(v - V[j]);
        if (dv > res) res = dv;
    }
    return res;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    /* 0 = every host thread (the count OpenMP starts with), whatever an earlier
     * call with an explicit count set */
    static int all_threads = 0;
    if (!all_threads) all_threads = omp_get_max_threads();
    omp_set_num_threads(nthreads > 0 ? nthreads : all_threads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Apply T once: TV = T(V), policy (first minimising control, -1 on fixed or
 * non-domain nodes) optional.  Returns 0 or a negative error. */
int orc_apply(int dim, const int *n, const double *lo, const double *hi, double h, int m,
              const double *b, const double *c, int mb, const double *bb, int c_axes, int interp,
              const double *l, const double *drift, double lam, int disc, double G,
              const uint8_t *fixed, const uint8_t *dom, const double *V, double *TV,
              int32_t *policy, int nthreads)
{
    orc_prob P;
    int rc = prob_init(&P, dim, n, lo, hi, h, m, b, c, mb, bb, c_axes, interp, l, drift, lam, disc, G,
                       fixed, dom);
    if (rc) { prob_free(&P); return rc; }
    set_threads(nthreads);
    (void)sweep(&P, V, TV, policy);
    prob_free(&P);
    return 0;
}

/* Jacobi iteration V <- T(V) from the caller's V (fixed nodes hold their values)
 * until max|V_new - V| <= tol (tol = 0: until nothing changes) or max_sweeps.
 * Returns the number of sweeps done (the last one's residual in *residual), or a
 * negative error.  On return V holds the last iterate, policy (optional) the
 * first minimising control of the last sweep. */
long orc_solve(int dim, const int *n, const double *lo, const double *hi, double h, int m,
               const double *b, const double *c, int mb, const double *bb, int c_axes, int interp,
               const double *l, const double *drift, double lam, int disc, double G,
               const uint8_t *fixed, const uint8_t *dom, double *V, int32_t *policy,
               double tol, long max_sweeps, double *residual, int nthreads)
{
    orc_prob P;
    int rc = prob_init(&P, dim, n, lo, hi, h, m, b, c, mb, bb, c_axes, interp, l, drift, lam, disc, G,
                       fixed, dom);
    if (rc) { prob_free(&P); return rc; }
    set_threads(nthreads);
    double *W = (double *)malloc(sizeof(double) * (size_t)P.N);
    if (!W) { prob_free(&P); return -2; }
    for (long j = 0; j < P.N; ++j)
        if (P.dom && !P.dom[j]) V[j] = G;
    double res = INFINITY;
    long s = 0;
    while (s < max_sweeps) {
        res = sweep(&P, V, W, policy);
        memcpy(V, W, sizeof(double) * (size_t)P.N);
        ++s;
        if (res <= tol) break;
    }
    if (residual) *residual = res;
    free(W);
    prob_free(&P);
    return s;
}

/* Interpolation stencil of the frozen policy: for every node j with policy[j] >= 0,
 * corner indices (-1 = ghost) and weights of I at its foot, 2^dim per node. */
int orc_policy_stencil(int dim, const int *n, const double *lo, const double *hi, double h, int m,
                       const double *b, const double *c, int mb, const double *bb, int c_axes, int interp,
                       const double *drift, const uint8_t *dom, const int32_t *policy,
                       int64_t *cidx, double *wts)
{
    orc_prob P;
    int rc = prob_init(&P, dim, n, lo, hi, h, m, b, c, mb, bb, c_axes, interp, NULL, drift, 1.0, 0, 0.0,
                       NULL, dom);
    if (rc) { prob_free(&P); return rc; }
    const int K = 1 << dim;
    for (long j = 0; j < P.N; ++j) {
        long ij[3], ci[ORC_MAX_CORNERS];
        double wt[ORC_MAX_CORNERS];
        if (policy[j] < 0) {
            for (int s = 0; s < K; ++s) { cidx[j * K + s] = -1; wts[j * K + s] = 0.0; }
            continue;
        }
        node_index(&P, j, ij);
        stencil(&P, j, ij, policy[j], ci, wt);
        for (int s = 0; s < K; ++s) { cidx[j * K + s] = ci[s]; wts[j * K + s] = wt[s]; }
    }
    prob_free(&P);
    return 0;
}

/* Adjoint of the policy-frozen scheme.  With the policy frozen, on free domain
 * nodes V = beta P V + w l + (constants from fixed and ghost corners), so for a
 * loss with gradient gV = dL/dV the adjoint state solves
 *     lambda = gV + beta P^T lambda      (free domain nodes only)
 * and dL/dl_j = w lambda_j.  Plain Jacobi iteration from lambda = gV, scattering
 * beta * weight * lambda_j to the free corners of node j's foot, until
 * max|lambda_new - lambda| <= tol.  Output: lam_out (N, zero off free nodes) and,
 * if dLdl != NULL, w * lambda.  Returns iterations or a negative error. */
long orc_adjoint(int dim, const int *n, const double *lo, const double *hi, double h, int m,
                 const double *b, const double *c, int mb, const double *bb, int c_axes, int interp,
                 const double *drift, double lam, int disc, const uint8_t *fixed,
                 const uint8_t *dom, const int32_t *policy, const double *gV, double *lam_out,
                 double *dLdl, double tol, long max_iters, double *residual)
{
    orc_prob P;
    if (disc == 2) return -1;        /* the discount depends on l: not a linear adjoint in w l */
    int rc = prob_init(&P, dim, n, lo, hi, h, m, b, c, mb, bb, c_axes, interp, NULL, drift, lam, disc, 0.0,
                       fixed, dom);
    if (rc) { prob_free(&P); return rc; }
    double beta = P.beta, w;
    orc_scheme_constants(lam, h, disc, &beta, &w);
    const long N = P.N;
    const int K = 1 << dim;
    double *X = (double *)calloc((size_t)N, sizeof(double));
    double *Y = (double *)calloc((size_t)N, sizeof(double));
    if (!X || !Y) { free(X); free(Y); prob_free(&P); return -2; }
    for (long j = 0; j < N; ++j) X[j] = is_free(&P, j) ? gV[j] : 0.0;
    long it = 0;
    double res = INFINITY;
    while (it < max_iters) {
        for (long j = 0; j < N; ++j) Y[j] = is_free(&P, j) ? gV[j] : 0.0;
        for (long j = 0; j < N; ++j) {
            if (!is_free(&P, j) || X[j] == 0.0) continue;
            long ij[3], ci[ORC_MAX_CORNERS];
            double wt[ORC_MAX_CORNERS];
            node_index(&P, j, ij);
            stencil(&P, j, ij, policy[j], ci, wt);
            for (int s = 0; s < K; ++s)
                if (ci[s] >= 0 && is_free(&P, ci[s])) Y[ci[s]] += beta * wt[s] * X[j];
        }
        res = 0.0;
        for (long j = 0; j < N; ++j) {
            double dv = fabs(Y[j] - X[j]);
            if (dv > res) res = dv;
        }
        double *T = X; X = Y; Y = T;
        ++it;
        if (res <= tol) break;
    }
    memcpy(lam_out, X, sizeof(double) * (size_t)N);
    if (dLdl)
        for (long j = 0; j < N; ++j) dLdl[j] = w * X[j];
    if (residual) *residual = res;
    free(X); free(Y);
    prob_free(&P);
    return it;
}

/* Tangent of the policy-frozen scheme: Vdot = beta P Vdot + w * dl on free domain
 * nodes (zero elsewhere), plain Jacobi from zero.  Used for the dot-product test
 * <lambda, w dl> = <gV, Vdot>.  Returns iterations or a negative error. */
long orc_tangent(int dim, const int *n, const double *lo, const double *hi, double h, int m,
                 const double *b, const double *c, int mb, const double *bb, int c_axes, int interp,
                 const double *drift, double lam, int disc, const uint8_t *fixed,
                 const uint8_t *dom, const int32_t *policy, const double *dl, double *Vdot,
                 double tol, long max_iters, double *residual)
{
    orc_prob P;
    if (disc == 2) return -1;
    int rc = prob_init(&P, dim, n, lo, hi, h, m, b, c, mb, bb, c_axes, interp, dl, drift, lam, disc, 0.0,
                       fixed, dom);
    if (rc) { prob_free(&P); return rc; }
    const long N = P.N;
    const int K = 1 << dim;
    double *X = (double *)calloc((size_t)N, sizeof(double));
    double *Y = (double *)calloc((size_t)N, sizeof(double));
    if (!X || !Y) { free(X); free(Y); prob_free(&P); return -2; }
    long it = 0;
    double res = INFINITY;
    while (it < max_iters) {
        res = 0.0;
#pragma omp parallel for schedule(static) reduction(max : res)
        for (long j = 0; j < N; ++j) {
            if (!is_free(&P, j)) { Y[j] = 0.0; continue; }
            long ij[3], ci[ORC_MAX_CORNERS];
            double wt[ORC_MAX_CORNERS];
            node_index(&P, j, ij);
            stencil(&P, j, ij, policy[j], ci, wt);
            double r = 0.0;
            for (int s = 0; s < K; ++s)
                if (ci[s] >= 0 && is_free(&P, ci[s])) r += wt[s] * X[ci[s]];
            Y[j] = P.beta * r + P.wl[j];
            double dv = fabs(Y[j] - X[j]);
            if (dv > res) res = dv;
        }
        double *T = X; X = Y; Y = T;
        ++it;
        if (res <= tol) break;
    }
    memcpy(Vdot, X, sizeof(double) * (size_t)N);
    if (residual) *residual = res;
    free(X); free(Y);
    prob_free(&P);
    return it;
}
