// C-ABI entry points of the slhjb library (declared in include/slhjb.h).
//
// Host side of every call:
//   1. validate the arguments on the host; lay out the caller's workspace;
//   2. one device pass gathers input statistics (max speed for the halo, value
//      checks, target counts); one stream sync reads them back;
//   3. build the sub-domain descriptors and the device work list;
//   4. run sweeps in chunks of `check_every` launches; convergence is decided on
//      the device, the host reads one counter per chunk;
//   5. assemble outputs, copy the per-sub-domain states back for the stats.
#include "internal.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

using namespace slhjb;

namespace {

// ------------------------------------------------------------------ workspace
struct Arena {
    char *base;          // nullptr: dry run (size query)
    size_t cap;
    size_t off = 0;
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    bool fits() const { return base == nullptr || off <= cap; }
};

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return SL_ERR_HIP;   \
    } while (0)

size_t nodes_of(const sl_problem *p) {
    size_t N = 1;
    for (int d = 0; d < p->dim; ++d) N *= (size_t)p->n[d];
    return N;
}

int validate(const sl_problem *p) {
    if (!p) return SL_ERR_INVALID_ARG;
    if (p->dim != 2 && p->dim != 3) return SL_ERR_UNSUPPORTED;
    if (p->m < 1 || p->m > SL_MAX_CONTROLS) return SL_ERR_UNSUPPORTED;
    if (p->n_comp < 1 || p->n_comp > SL_MAX_COMP) return SL_ERR_UNSUPPORTED;
    if (!p->velocity || !p->target) return SL_ERR_INVALID_ARG;
    double N = 1;
    for (int d = 0; d < p->dim; ++d) {
        if (p->n[d] < 3) return SL_ERR_INVALID_ARG;
        if (!(p->hi[d] > p->lo[d]) || !std::isfinite(p->hi[d] - p->lo[d])) return SL_ERR_INVALID_ARG;
        N *= p->n[d];
    }
    if (N > 2147483647.0) return SL_ERR_UNSUPPORTED;
    for (int i = 0; i < p->m * p->dim; ++i)
        if (!std::isfinite(p->velocity[i])) return SL_ERR_INVALID_ARG;
    if (!(p->lambda > 0.0) || !std::isfinite(p->lambda)) return SL_ERR_INVALID_ARG;
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return SL_ERR_INVALID_ARG;
    if (!std::isfinite(p->v_ghost)) return SL_ERR_INVALID_ARG;
    if (p->disc != SL_DISC_EXP && p->disc != SL_DISC_PAPER) return SL_ERR_INVALID_ARG;
    if (p->dtype != SL_F32 && p->dtype != SL_F64) return SL_ERR_INVALID_ARG;
    if (p->drift) return SL_ERR_UNSUPPORTED;
    return SL_OK;
}

int validate_solve_opts(const sl_solve_opts *o) {
    if (!o) return SL_ERR_INVALID_ARG;
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return SL_ERR_INVALID_ARG;
    if (o->max_sweeps < 1 || o->max_sweeps > 100000000L) return SL_ERR_INVALID_ARG;
    if (o->check_every < 0) return SL_ERR_INVALID_ARG;
    return SL_OK;
}

int validate_ra(const sl_problem *p, const sl_ra_opts *ra) {
    if (!ra) return SL_ERR_INVALID_ARG;
    if (ra->coarse_stride < 1) return SL_ERR_INVALID_ARG;
    for (int d = 0; d < p->dim; ++d) {
        if ((p->n[d] - 1) % ra->coarse_stride) return SL_ERR_INVALID_ARG;
        if ((p->n[d] - 1) / ra->coarse_stride + 1 < 3) return SL_ERR_INVALID_ARG;
    }
    if (!std::isfinite(ra->C) || !std::isfinite(ra->M) || !std::isfinite(ra->q))
        return SL_ERR_INVALID_ARG;
    if (!(ra->delta_override >= 0.0) && !(ra->delta_override < 0.0)) return SL_ERR_INVALID_ARG;
    if (!(ra->tol >= 0.0) || ra->max_sweeps < 1) return SL_ERR_INVALID_ARG;
    return SL_OK;
}

// Discount and cost weight of one step (same formulas as the scheme's statement).
void scheme_constants(double lam, double h, int disc, double *beta, double *w) {
    if (disc == SL_DISC_EXP) {
        *beta = std::exp(-lam * h);
        *w = -std::expm1(-lam * h) / lam;
    } else {
        *beta = 1.0 / (1.0 + lam * h);
        *w = h;
    }
}

// Control displacements in cells per unit speed: e_kd = (h/dx_d) * b_kd.
void control_table(const sl_problem *p, const int *n, double h, std::vector<double> &e,
                   double *emax) {
    double t[3];
    for (int d = 0; d < p->dim; ++d) t[d] = h / ((p->hi[d] - p->lo[d]) / (double)(n[d] - 1));
    e.resize((size_t)p->m * p->dim);
    *emax = 0.0;
    for (int k = 0; k < p->m; ++k)
        for (int d = 0; d < p->dim; ++d) {
            e[(size_t)k * p->dim + d] = t[d] * p->velocity[(size_t)k * p->dim + d];
            *emax = std::max(*emax, std::fabs(e[(size_t)k * p->dim + d]));
        }
}

int halo_for(double speed_max, double emax) {
    const double D = speed_max * emax;
    if (!std::isfinite(D)) return INT_MAX;
    // floor(D) + 1 covers both corners of every foot; the margin absorbs the
    // rounding of c*e and of the foot coordinate.
    return (int)std::floor(D * (1.0 + 1e-6) + 1e-3) + 1;
}

int default_variant(int dim, int dtype) {
    if (dim == 2) return dtype == SL_F32 ? 0 : 4;
    return dtype == SL_F32 ? 5 : 8;
}

LaunchCfg make_cfg(int dim, int dtype, int halo, int variant) {
    LaunchCfg all[16];
    const int nv = sweep_variants(dim, all, 16);
    LaunchCfg c{};
    for (int i = 0; i < nv && i < 16; ++i)
        if (all[i].variant == variant) c = all[i];
    c.halo = halo;
    return c;
}

// Pinned host scratch for the per-chunk convergence poll.
struct Pinned {
    int *active = nullptr;
    Pinned() {
        if (hipHostMalloc((void **)&active, sizeof(int) * 16, hipHostMallocDefault) != hipSuccess)
            active = nullptr;
    }
};
Pinned &pinned() {
    static thread_local Pinned p;
    return p;
}

// --------------------------------------------------------------- executor
template <typename T>
struct Exec {
    LaunchCfg cfg{};
    SdDesc<T> *sds = nullptr;       // device
    SdState *st = nullptr;          // device
    WorkItem *items = nullptr;      // device
    ExecCounters *cnt = nullptr;    // device
    int *prefix = nullptr;          // device
    int n_sd = 0;
    int total_tiles = 0;
    std::vector<SdDesc<T>> host_sds;
    std::vector<int> host_prefix;

    void reserve(Arena &a, int nsd, int tiles_total) {
        sds = a.take<SdDesc<T>>(nsd);
        st = a.take<SdState>(nsd);
        items = a.take<WorkItem>(tiles_total > 0 ? tiles_total : 1);
        cnt = a.take<ExecCounters>(1);
        prefix = a.take<int>(nsd);
    }

    static int tiles_of(const LaunchCfg &cfg, const int *n, int dim, int *t) {
        int tot = 1;
        for (int d = 0; d < 3; ++d) {
            const int nd = d < dim ? n[d] : 1;
            const int td = d < dim ? cfg.tile[d] : 1;
            t[d] = (nd + td - 1) / td;
            tot *= t[d];
        }
        return tot;
    }

    // Upload descriptors and states, build the work list.
    int prepare(hipStream_t s) {
        n_sd = (int)host_sds.size();
        host_prefix.resize(n_sd);
        int acc = 0;
        for (int i = 0; i < n_sd; ++i) {
            host_sds[i].tile_offset = acc;
            host_prefix[i] = acc;
            acc += host_sds[i].tiles[0] * host_sds[i].tiles[1] * host_sds[i].tiles[2];
        }
        total_tiles = acc;
        std::vector<SdState> hs(n_sd);
        for (auto &x : hs) {
            x.res[0] = x.res[1] = x.res[2] = 0ull;
            x.conv_at = -1;
            x.final_buf = 0;
            x.done_sweeps = 0;
            x.pad = 0;
            x.final_res = 0ull;
            x.scale[0] = x.scale[1] = x.scale[2] = 0ull;
        }
        HIPCHK(hipMemcpyAsync(sds, host_sds.data(), sizeof(SdDesc<T>) * n_sd,
                              hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(st, hs.data(), sizeof(SdState) * n_sd, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(prefix, host_prefix.data(), sizeof(int) * n_sd,
                              hipMemcpyHostToDevice, s));
        HIPCHK(hipMemsetAsync(cnt, 0, sizeof(ExecCounters), s));
        HIPCHK(launch_build_items(cfg, sds, n_sd, total_tiles, prefix, items, cnt, s));
        return SL_OK;
    }

    // Sweeps until every sd meets tol or max_sweeps.  Returns SL_OK or
    // SL_NOT_CONVERGED; *sweeps_done = sweeps launched.
    // Profiling (optional): HIP events around each chunk of back-to-back sweep
    // launches; ms_sweeps / sweep_launches is the mean launch duration.
    double ms_sweeps = 0.0;
    long sweep_launches = 0;

    int run(double tol, long max_sweeps, int check_every, int want_policy, hipStream_t s,
            long *sweeps_done, int profile = 0) {
        int *active = pinned().active;
        if (!active) return SL_ERR_HIP;
        const int chunk = check_every > 0 ? check_every : 32;
        long S = 0;
        int status = SL_NOT_CONVERGED;
        hipEvent_t ev[2] = {nullptr, nullptr};
        if (profile) {
            HIPCHK(hipEventCreate(&ev[0]));
            HIPCHK(hipEventCreate(&ev[1]));
        }
        while (S < max_sweeps) {
            const long todo = std::min<long>(chunk, max_sweeps - S);
            if (profile) HIPCHK(hipEventRecord(ev[0], s));
            for (long i = 0; i < todo; ++i, ++S)
                HIPCHK(launch_sweep(cfg, sds, st, n_sd, items, cnt, total_tiles, (int)S, tol, 0, s));
            if (profile) HIPCHK(hipEventRecord(ev[1], s));
            HIPCHK(launch_bookkeep(st, n_sd, (int)S, tol, cnt, 0, s));
            HIPCHK(hipMemcpyAsync(active, &cnt->n_active, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (profile) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
                ms_sweeps += ms;
                sweep_launches += todo;
            }
            if (*active == 0) {
                status = SL_OK;
                break;
            }
        }
        if (profile) {
            (void)hipEventDestroy(ev[0]);
            (void)hipEventDestroy(ev[1]);
        }
        HIPCHK(launch_bookkeep(st, n_sd, (int)S, tol, cnt, 1, s));
        if (want_policy) {
            HIPCHK(launch_sweep(cfg, sds, st, n_sd, items, cnt, total_tiles, (int)S, tol, 1, s));
            HIPCHK(launch_flip(st, n_sd, s));
        }
        *sweeps_done = S;
        return status;
    }

    int read_stats(hipStream_t s, std::vector<SdState> &out, unsigned long long *nc) {
        out.resize(n_sd);
        ExecCounters c{};
        HIPCHK(hipMemcpyAsync(out.data(), st, sizeof(SdState) * n_sd, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&c, cnt, sizeof(ExecCounters), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *nc = c.nc_updates;
        return SL_OK;
    }
};

void fill_stats(sl_stats *stats, const std::vector<SdState> &hs, unsigned long long nc,
                long S) {
    if (!stats) return;
    long smax = 0, stot = 0;
    double res = 0.0;
    for (const auto &x : hs) {
        const long sw = x.conv_at >= 0 ? x.conv_at + 1 : S;
        smax = std::max(smax, sw);
        stot += sw;
        double r;
        const unsigned long long bits = x.final_res;
        std::memcpy(&r, &bits, sizeof(r));
        res = std::max(res, r);
    }
    stats->sweeps_max = smax;
    stats->sweeps_total = stot;
    stats->residual = res;
    stats->node_control_updates = (double)nc;
    stats->n_subdomains = (int)hs.size();
    stats->n_unreachable = 0;
}

struct Timer {
    hipEvent_t e[4]{};
    bool ok = false;
    Timer() {
        ok = true;
        for (auto &x : e) ok = ok && hipEventCreate(&x) == hipSuccess;
    }
    ~Timer() {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
    void mark(int i, hipStream_t s) {
        if (ok) (void)hipEventRecord(e[i], s);
    }
    double ms(int a, int b) {
        float v = 0.f;
        if (ok && hipEventElapsedTime(&v, e[a], e[b]) == hipSuccess) return v;
        return 0.0;
    }
};

// ------------------------------------------------------------ field statistics
template <typename T>
int gather_field_stats(const sl_problem *p, const int8_t *target, const T *speed,
                       const T *cost, size_t N, int n_comp, FieldStats *fs_dev,
                       FieldStats *host, hipStream_t s) {
    FieldStats init{};
    for (int i = 0; i < SL_MAX_COMP; ++i) init.first_node[i] = INT_MAX;
    HIPCHK(hipMemcpyAsync(fs_dev, &init, sizeof(init), hipMemcpyHostToDevice, s));
    HIPCHK(launch_field_stats<T>(speed, cost, (const T *)nullptr, p->dim, target, N, n_comp,
                                 fs_dev, s));
    HIPCHK(hipMemcpyAsync(host, fs_dev, sizeof(FieldStats), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return SL_OK;
}

double bits_to_double(unsigned long long b) {
    double d;
    std::memcpy(&d, &b, sizeof(d));
    return d;
}

int check_fields(const FieldStats &fs) {
    if (fs.bad_speed || fs.bad_cost || fs.bad_target) return SL_ERR_INVALID_ARG;
    if (fs.n_target == 0) return SL_ERR_NO_TARGET;
    return SL_OK;
}

// ------------------------------------------------------------ global solve
template <typename T>
int plan_global(const sl_problem *p, Arena &a, Exec<T> &ex, T **Vb, T **wl, T **ctrl,
                FieldStats **fs, int variant) {
    const size_t N = nodes_of(p);
    const LaunchCfg cfg = make_cfg(p->dim, p->dtype, 1, variant);
    int t[3];
    const int tiles = Exec<T>::tiles_of(cfg, p->n, p->dim, t);
    Vb[0] = a.take<T>(N);
    Vb[1] = a.take<T>(N);
    *wl = p->cost ? a.take<T>(N) : nullptr;
    *ctrl = a.take<T>((size_t)p->m * p->dim);
    *fs = a.take<FieldStats>(1);
    ex.reserve(a, 1, tiles);
    return SL_OK;
}

template <typename T>
int solve_global(const sl_problem *p, const sl_solve_opts *o, void *ws, size_t ws_bytes,
                 T *V, uint8_t *policy, sl_stats *stats, hipStream_t s) {
    Timer tm;
    tm.mark(0, s);
    const size_t N = nodes_of(p);
    const int variant = default_variant(p->dim, p->dtype);
    Arena a{(char *)ws, ws_bytes};
    Exec<T> ex;
    T *Vb[2], *wl, *ctrl;
    FieldStats *fs_dev;
    plan_global<T>(p, a, ex, Vb, &wl, &ctrl, &fs_dev, variant);
    if (!a.fits()) return SL_ERR_WORKSPACE;

    FieldStats fs{};
    int rc = gather_field_stats<T>(p, p->target, (const T *)p->speed, (const T *)p->cost, N,
                                   p->n_comp, fs_dev, &fs, s);
    if (rc) return rc;
    if ((rc = check_fields(fs))) return rc;

    double beta, w, emax;
    scheme_constants(p->lambda, p->h, p->disc, &beta, &w);
    std::vector<double> e;
    control_table(p, p->n, p->h, e, &emax);
    const double smax = p->speed ? bits_to_double(fs.speed_max) : 1.0;
    const int H = halo_for(smax, emax);
    if (H > kMaxHalo) return SL_ERR_UNSUPPORTED;
    ex.cfg = make_cfg(p->dim, p->dtype, H, variant);

    std::vector<T> et(e.size());
    for (size_t i = 0; i < e.size(); ++i) et[i] = (T)e[i];
    HIPCHK(hipMemcpyAsync(ctrl, et.data(), sizeof(T) * et.size(), hipMemcpyHostToDevice, s));
    if (p->cost) HIPCHK((launch_scale_field<T, T>((const T *)p->cost, wl, N, w, s)));
    for (int b = 0; b < 2; ++b)
        HIPCHK(launch_init_values<T>(Vb[b], p->target, (const T *)p->g, (T)p->v_ghost, -1, N, s));

    SdDesc<T> d{};
    d.V[0] = Vb[0];
    d.V[1] = Vb[1];
    d.speed = (const T *)p->speed;
    d.wl = wl;
    d.drift = nullptr;
    d.target = p->target;
    d.member = nullptr;
    d.policy = policy;
    d.ctrl = ctrl;
    d.wl_const = (T)w;
    d.beta = (T)beta;
    d.G = (T)p->v_ghost;
    for (int k = 0; k < 3; ++k) d.n[k] = k < p->dim ? p->n[k] : 1;
    d.m = p->m;
    d.bit = 0;
    Exec<T>::tiles_of(ex.cfg, p->n, p->dim, d.tiles);
    d.halo = H;
    ex.host_sds.push_back(d);
    if ((rc = ex.prepare(s))) return rc;
    if (o->want_policy && policy) HIPCHK(hipMemsetAsync(policy, 0xFF, N, s));
    tm.mark(1, s);
    long S = 0;
    const int status = ex.run(o->tol, o->max_sweeps, o->check_every, o->want_policy && policy, s, &S,
                              o->profile);
    if (status < 0) return status;
    HIPCHK(launch_copy_final<T>(ex.sds, ex.st, 0, V, N, s));
    tm.mark(2, s);
    std::vector<SdState> hs;
    unsigned long long nc = 0;
    if ((rc = ex.read_stats(s, hs, &nc))) return rc;
    fill_stats(stats, hs, nc, S);
    if (stats) {
        stats->ms_ra = 0.0;
        stats->ms_fine = tm.ms(1, 2);
        stats->ms_total = tm.ms(0, 2);
        stats->set_fraction_max = 1.0;
        stats->ms_sweeps = ex.ms_sweeps;
        stats->sweep_launches = ex.sweep_launches;
    }
    return status;
}

// --------------------------------------------------------------- RA and ISA
struct CoarseGeom {
    int nK[3];
    size_t NK;
    double hK;
};

CoarseGeom coarse_geom(const sl_problem *p, int s) {
    CoarseGeom g{};
    g.NK = 1;
    for (int d = 0; d < 3; ++d) {
        g.nK[d] = d < p->dim ? (p->n[d] - 1) / s + 1 : 1;
        g.NK *= (size_t)g.nK[d];
    }
    g.hK = p->h * s;
    return g;
}

template <typename T>
struct IsaPlan {
    // coarse
    T *cK_t = nullptr;             // gathered speed (dtype)
    T *lK_t = nullptr;             // gathered cost (dtype)
    double *cK = nullptr, *wlK = nullptr, *gK = nullptr, *ctrlK = nullptr, *gK_src = nullptr;
    T *gK_t = nullptr;
    int8_t *tK = nullptr;
    double *Vaux = nullptr;        // n_comp * 2 * NK
    double *Vpack = nullptr;       // n_comp * NK final auxiliary values
    uint8_t *mK = nullptr, *lbK = nullptr;
    FieldStats *fsK = nullptr;
    Exec<double> exK;
    // fine
    T *Vf = nullptr;               // n_comp * 2 * N
    T *wl = nullptr, *ctrl = nullptr;
    FieldStats *fs = nullptr;
    unsigned long long *counts = nullptr;
    Exec<T> ex;
};

template <typename T>
void plan_isa(const sl_problem *p, const sl_ra_opts *ra, Arena &a, IsaPlan<T> &P) {
    const size_t N = nodes_of(p);
    const CoarseGeom cg = coarse_geom(p, ra->coarse_stride);
    const int nc = p->n_comp;
    const LaunchCfg cfgK = make_cfg(p->dim, SL_F64, 1, default_variant(p->dim, SL_F64));
    int t[3];
    const int tilesK = Exec<double>::tiles_of(cfgK, cg.nK, p->dim, t);
    P.cK_t = a.take<T>(cg.NK);
    P.lK_t = a.take<T>(cg.NK);
    P.gK_t = a.take<T>(cg.NK);
    P.cK = a.take<double>(cg.NK);
    P.wlK = a.take<double>(cg.NK);
    P.gK = a.take<double>(cg.NK);
    P.ctrlK = a.take<double>((size_t)p->m * p->dim);
    P.tK = a.take<int8_t>(cg.NK);
    P.Vaux = a.take<double>((size_t)nc * 2 * cg.NK);
    P.Vpack = a.take<double>((size_t)nc * cg.NK);
    P.mK = a.take<uint8_t>(cg.NK);
    P.lbK = a.take<uint8_t>(cg.NK);
    P.fsK = a.take<FieldStats>(1);
    P.exK.reserve(a, nc, tilesK * nc);
    const LaunchCfg cfg = make_cfg(p->dim, p->dtype, 1, default_variant(p->dim, p->dtype));
    const int tiles = Exec<T>::tiles_of(cfg, p->n, p->dim, t);
    P.Vf = a.take<T>((size_t)nc * 2 * N);
    P.wl = p->cost ? a.take<T>(N) : nullptr;
    P.ctrl = a.take<T>((size_t)p->m * p->dim);
    P.fs = a.take<FieldStats>(1);
    P.counts = a.take<unsigned long long>(8);
    P.ex.reserve(a, nc, tiles * nc);
}

template <typename T>
int reconstruct_impl(const sl_problem *p, const sl_ra_opts *ra, void *ws, size_t ws_bytes,
                     uint8_t *member, uint8_t *label, uint8_t *member_K, uint8_t *label_K,
                     sl_stats *stats, hipStream_t s) {
    Timer tm;
    tm.mark(0, s);
    const size_t N = nodes_of(p);
    Arena a{(char *)ws, ws_bytes};
    IsaPlan<T> P;
    plan_isa<T>(p, ra, a, P);
    if (!a.fits()) return SL_ERR_WORKSPACE;
    const int sK = ra->coarse_stride;
    const CoarseGeom cg = coarse_geom(p, sK);
    const int nc = p->n_comp;

    // fine-grid statistics: validation and lowest node per component
    FieldStats fs{};
    int rc = gather_field_stats<T>(p, p->target, (const T *)p->speed, (const T *)p->cost, N, nc,
                                   P.fs, &fs, s);
    if (rc) return rc;
    if ((rc = check_fields(fs))) return rc;

    // coarse problem data: every s-th node, widened to FP64
    if (p->speed) {
        HIPCHK(launch_gather_coarse<T>((const T *)p->speed, P.cK_t, p->n, cg.nK, p->dim, sK, 1, s));
        HIPCHK((launch_scale_field<T, double>(P.cK_t, P.cK, cg.NK, 1.0, s)));
    }
    double betaK, wK, emaxK;
    scheme_constants(p->lambda, cg.hK, p->disc, &betaK, &wK);
    if (p->cost) {
        HIPCHK(launch_gather_coarse<T>((const T *)p->cost, P.lK_t, p->n, cg.nK, p->dim, sK, 1, s));
        HIPCHK((launch_scale_field<T, double>(P.lK_t, P.wlK, cg.NK, wK, s)));
    }
    if (p->g)
        HIPCHK(launch_gather_coarse<T>((const T *)p->g, P.gK_t, p->n, cg.nK, p->dim, sK, 1, s));
    HIPCHK(launch_gather_coarse_i8(p->target, P.tK, p->n, cg.nK, p->dim, sK, s));
    // components without a coincident coarse node: place them (in the field's own
    // dtype), then widen g to FP64
    {
        FieldStats init{};
        for (int i = 0; i < SL_MAX_COMP; ++i) init.first_node[i] = INT_MAX;
        HIPCHK(hipMemcpyAsync(P.fsK, &init, sizeof(init), hipMemcpyHostToDevice, s));
        HIPCHK(launch_field_stats<double>(nullptr, nullptr, nullptr, p->dim, P.tK, cg.NK, nc,
                                          P.fsK, s));
        const int *first_fine = reinterpret_cast<const int *>(
            reinterpret_cast<const char *>(P.fs) + offsetof(FieldStats, first_node));
        const int *firstK = reinterpret_cast<const int *>(
            reinterpret_cast<const char *>(P.fsK) + offsetof(FieldStats, first_node));
        HIPCHK(launch_place_missing<T>(P.tK, p->g ? P.gK_t : nullptr, (const T *)p->g,
                                       first_fine, firstK, p->n, cg.nK, p->dim, sK, nc, s));
        if (p->g) HIPCHK((launch_scale_field<T, double>(P.gK_t, P.gK, cg.NK, 1.0, s)));
    }

    // coarse auxiliary problems (RA step 1), FP64
    std::vector<double> e;
    control_table(p, cg.nK, cg.hK, e, &emaxK);
    HIPCHK(hipMemcpyAsync(P.ctrlK, e.data(), sizeof(double) * e.size(), hipMemcpyHostToDevice, s));
    const double smax = p->speed ? bits_to_double(fs.speed_max) : 1.0;
    const int HK = halo_for(smax, emaxK);
    if (HK > kMaxHalo) return SL_ERR_UNSUPPORTED;
    P.exK.cfg = make_cfg(p->dim, SL_F64, HK, default_variant(p->dim, SL_F64));
    for (int i = 0; i < nc; ++i) {
        double *V0 = P.Vaux + (size_t)i * 2 * cg.NK;
        for (int b = 0; b < 2; ++b)
            HIPCHK(launch_init_values<double>(V0 + b * cg.NK, P.tK, p->g ? P.gK : nullptr,
                                              p->v_ghost, i, cg.NK, s));
        SdDesc<double> d{};
        d.V[0] = V0;
        d.V[1] = V0 + cg.NK;
        d.speed = p->speed ? P.cK : nullptr;
        d.wl = p->cost ? P.wlK : nullptr;
        d.target = P.tK;
        d.member = nullptr;
        d.policy = nullptr;
        d.ctrl = P.ctrlK;
        d.wl_const = wK;
        d.beta = betaK;
        d.G = p->v_ghost;
        for (int k = 0; k < 3; ++k) d.n[k] = cg.nK[k];
        d.m = p->m;
        d.bit = i;
        Exec<double>::tiles_of(P.exK.cfg, cg.nK, p->dim, d.tiles);
        d.halo = HK;
        P.exK.host_sds.push_back(d);
    }
    if ((rc = P.exK.prepare(s))) return rc;
    long S = 0;
    const int status = P.exK.run(ra->tol, ra->max_sweeps, 32, 0, s, &S);
    if (status < 0) return status;

    // RA steps 2-3: min, threshold, label on the final auxiliary iterates.
    for (int i = 0; i < nc; ++i)
        HIPCHK(launch_copy_final<double>(P.exK.sds, P.exK.st, i, P.Vpack + (size_t)i * cg.NK,
                                         cg.NK, s));
    double dxK = 0.0;
    for (int d = 0; d < p->dim; ++d)
        dxK = std::max(dxK, (p->hi[d] - p->lo[d]) / (double)(cg.nK[d] - 1));
    const double delta = ra->delta_override > 0.0
                             ? ra->delta_override
                             : 2.0 * (ra->C * std::pow(dxK, ra->q) + ra->M * dxK);
    uint8_t *mK = member_K ? member_K : P.mK;
    uint8_t *lbK = label_K ? label_K : P.lbK;
    HIPCHK(launch_ra_combine(P.Vpack, nc, cg.NK, P.tK, delta, mK, lbK, s));
    // ISA step 2: projection to the fine grid
    HIPCHK(launch_project(mK, lbK, cg.nK, p->n, p->dim, sK, member, label, s));
    tm.mark(1, s);
    std::vector<SdState> hs;
    unsigned long long ncu = 0;
    if ((rc = P.exK.read_stats(s, hs, &ncu))) return rc;
    fill_stats(stats, hs, ncu, S);
    if (stats) {
        stats->ms_ra = tm.ms(0, 1);
        stats->ms_fine = 0.0;
        stats->ms_total = tm.ms(0, 1);
        stats->set_fraction_max = 0.0;
        stats->ms_sweeps = 0.0;
        stats->sweep_launches = 0;
    }
    return status;
}

template <typename T>
int isa_impl(const sl_problem *p, const sl_ra_opts *ra, const uint8_t *member,
             const sl_solve_opts *o, void *ws, size_t ws_bytes, T *V, uint8_t *owner,
             uint8_t *policy, T *V_sets, sl_stats *stats, hipStream_t s) {
    Timer tm;
    tm.mark(0, s);
    const size_t N = nodes_of(p);
    Arena a{(char *)ws, ws_bytes};
    IsaPlan<T> P;
    plan_isa<T>(p, ra, a, P);
    if (!a.fits()) return SL_ERR_WORKSPACE;
    const int nc = p->n_comp;
    FieldStats fs{};
    int rc = gather_field_stats<T>(p, p->target, (const T *)p->speed, (const T *)p->cost, N, nc,
                                   P.fs, &fs, s);
    if (rc) return rc;
    if ((rc = check_fields(fs))) return rc;

    double beta, w, emax;
    scheme_constants(p->lambda, p->h, p->disc, &beta, &w);
    std::vector<double> e;
    control_table(p, p->n, p->h, e, &emax);
    const double smax = p->speed ? bits_to_double(fs.speed_max) : 1.0;
    const int H = halo_for(smax, emax);
    if (H > kMaxHalo) return SL_ERR_UNSUPPORTED;
    P.ex.cfg = make_cfg(p->dim, p->dtype, H, default_variant(p->dim, p->dtype));
    std::vector<T> et(e.size());
    for (size_t i = 0; i < e.size(); ++i) et[i] = (T)e[i];
    HIPCHK(hipMemcpyAsync(P.ctrl, et.data(), sizeof(T) * et.size(), hipMemcpyHostToDevice, s));
    if (p->cost) HIPCHK((launch_scale_field<T, T>((const T *)p->cost, P.wl, N, w, s)));
    for (int i = 0; i < nc; ++i) {
        T *V0 = P.Vf + (size_t)i * 2 * N;
        for (int b = 0; b < 2; ++b)
            HIPCHK(launch_init_values<T>(V0 + b * N, p->target, (const T *)p->g, (T)p->v_ghost,
                                         -1, N, s));
        SdDesc<T> d{};
        d.V[0] = V0;
        d.V[1] = V0 + N;
        d.speed = (const T *)p->speed;
        d.wl = P.wl;
        d.target = p->target;
        d.member = member;
        d.policy = policy ? policy + (size_t)i * N : nullptr;
        d.ctrl = P.ctrl;
        d.wl_const = (T)w;
        d.beta = (T)beta;
        d.G = (T)p->v_ghost;
        for (int k = 0; k < 3; ++k) d.n[k] = k < p->dim ? p->n[k] : 1;
        d.m = p->m;
        d.bit = i;
        Exec<T>::tiles_of(P.ex.cfg, p->n, p->dim, d.tiles);
        d.halo = H;
        P.ex.host_sds.push_back(d);
    }
    if ((rc = P.ex.prepare(s))) return rc;
    if (o->want_policy && policy) HIPCHK(hipMemsetAsync(policy, 0xFF, (size_t)nc * N, s));
    tm.mark(1, s);
    long S = 0;
    const int status = P.ex.run(o->tol, o->max_sweeps, o->check_every, o->want_policy && policy,
                                s, &S, o->profile);
    if (status < 0) return status;
    tm.mark(2, s);
    HIPCHK(launch_assemble<T>(P.ex.sds, P.ex.st, nc, member, N, (T)p->v_ghost, V, owner, s));
    if (V_sets)
        for (int i = 0; i < nc; ++i)
            HIPCHK(launch_copy_final<T>(P.ex.sds, P.ex.st, i, V_sets + (size_t)i * N, N, s));
    HIPCHK(hipMemsetAsync(P.counts, 0, sizeof(unsigned long long) * 8, s));
    HIPCHK(launch_member_counts(member, N, P.counts, s));
    unsigned long long counts[8];
    HIPCHK(hipMemcpyAsync(counts, P.counts, sizeof(counts), hipMemcpyDeviceToHost, s));
    tm.mark(3, s);
    std::vector<SdState> hs;
    unsigned long long ncu = 0;
    if ((rc = P.ex.read_stats(s, hs, &ncu))) return rc;
    fill_stats(stats, hs, ncu, S);
    if (stats) {
        double fr = 0.0;
        for (int i = 0; i < nc; ++i) fr = std::max(fr, (double)counts[i] / (double)N);
        stats->set_fraction_max = fr;
        stats->ms_ra = 0.0;
        stats->ms_fine = tm.ms(1, 2);
        stats->ms_total = tm.ms(0, 3);
        stats->ms_sweeps = P.ex.ms_sweeps;
        stats->sweep_launches = P.ex.sweep_launches;
    }
    return status;
}

// ------------------------------------------------------------------- adjoint
template <typename T>
struct AdjPlan {
    T *lam = nullptr, *acc = nullptr, *ctrl = nullptr;
    AdjDesc<T> *ads = nullptr;
    SdState *st = nullptr;
    ExecCounters *cnt = nullptr;
    FieldStats *fs = nullptr;
};

template <typename T>
void plan_adjoint(const sl_problem *p, int n_sets, Arena &a, AdjPlan<T> &P) {
    const size_t N = nodes_of(p);
    P.lam = a.take<T>((size_t)n_sets * N);
    P.acc = a.take<T>((size_t)n_sets * 2 * N);
    P.ctrl = a.take<T>((size_t)p->m * p->dim);
    P.ads = a.take<AdjDesc<T>>(n_sets);
    P.st = a.take<SdState>(n_sets);
    P.cnt = a.take<ExecCounters>(1);
    P.fs = a.take<FieldStats>(1);
}

template <typename T>
int adjoint_impl(const sl_problem *p, const uint8_t *member, const uint8_t *owner,
                 const uint8_t *policy, const T *dLdV, T *dLdl, double tol, long max_iters,
                 void *ws, size_t ws_bytes, sl_stats *stats, hipStream_t s) {
    Timer tm;
    tm.mark(0, s);
    const size_t N = nodes_of(p);
    const int n_sets = member ? p->n_comp : 1;
    Arena a{(char *)ws, ws_bytes};
    AdjPlan<T> P;
    plan_adjoint<T>(p, n_sets, a, P);
    if (!a.fits()) return SL_ERR_WORKSPACE;
    FieldStats fs{};
    int rc = gather_field_stats<T>(p, p->target, (const T *)p->speed, (const T *)p->cost, N,
                                   p->n_comp, P.fs, &fs, s);
    if (rc) return rc;
    if ((rc = check_fields(fs))) return rc;
    double beta, w, emax;
    scheme_constants(p->lambda, p->h, p->disc, &beta, &w);
    std::vector<double> e;
    control_table(p, p->n, p->h, e, &emax);
    std::vector<T> et(e.size());
    for (size_t i = 0; i < e.size(); ++i) et[i] = (T)e[i];
    HIPCHK(hipMemcpyAsync(P.ctrl, et.data(), sizeof(T) * et.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(P.lam, 0, sizeof(T) * (size_t)n_sets * N, s));
    HIPCHK(hipMemsetAsync(P.acc, 0, sizeof(T) * (size_t)n_sets * 2 * N, s));
    std::vector<AdjDesc<T>> hd(n_sets);
    for (int i = 0; i < n_sets; ++i) {
        AdjDesc<T> &d = hd[i];
        d.lam = P.lam + (size_t)i * N;
        d.acc[0] = P.acc + (size_t)i * 2 * N;
        d.acc[1] = d.acc[0] + N;
        d.g = dLdV;
        d.owner = member ? owner : nullptr;
        d.policy = policy + (size_t)i * N;
        d.speed = (const T *)p->speed;
        d.target = p->target;
        d.member = member;
        d.ctrl = P.ctrl;
        d.beta = (T)beta;
        for (int k = 0; k < 3; ++k) d.n[k] = k < p->dim ? p->n[k] : 1;
        d.m = p->m;
        d.bit = i;
        d.set = i;
    }
    HIPCHK(hipMemcpyAsync(P.ads, hd.data(), sizeof(AdjDesc<T>) * n_sets, hipMemcpyHostToDevice, s));
    std::vector<SdState> hs(n_sets);
    for (auto &x : hs) {
        x = SdState{};
        x.conv_at = -1;
    }
    HIPCHK(hipMemcpyAsync(P.st, hs.data(), sizeof(SdState) * n_sets, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(P.cnt, 0, sizeof(ExecCounters), s));
    // rounding-level stop: atomics reorder the sums, so the state settles to
    // within a few ulps of its largest entry
    const double scale_rel = 16.0 * (sizeof(T) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16);
    int bps = (int)((N + kThreads - 1) / kThreads);
    bps = std::max(1, std::min(bps, 2048));
    int *active = pinned().active;
    if (!active) return SL_ERR_HIP;
    tm.mark(1, s);
    long it = 0;
    int status = SL_NOT_CONVERGED;
    const int chunk = 32;
    while (it < max_iters) {
        const long todo = std::min<long>(chunk, max_iters - it);
        for (long i = 0; i < todo; ++i, ++it)
            HIPCHK(launch_adjoint_iter<T>(p->dim, P.ads, P.st, n_sets, bps, P.cnt, (int)it, tol,
                                          scale_rel, s));
        HIPCHK(launch_bookkeep(P.st, n_sets, (int)it, tol, P.cnt, 0, s, scale_rel));
        HIPCHK(hipMemcpyAsync(active, &P.cnt->n_active, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (*active == 0) {
            status = SL_OK;
            break;
        }
    }
    HIPCHK(launch_bookkeep(P.st, n_sets, (int)it, tol, P.cnt, 1, s, scale_rel));
    HIPCHK(launch_adjoint_combine<T>(P.ads, n_sets, p->target, N, (T)w, dLdl, s));
    tm.mark(2, s);
    ExecCounters c{};
    HIPCHK(hipMemcpyAsync(hs.data(), P.st, sizeof(SdState) * n_sets, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&c, P.cnt, sizeof(c), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    fill_stats(stats, hs, c.nc_updates, it);
    if (stats) {
        stats->ms_ra = 0.0;
        stats->ms_fine = tm.ms(1, 2);
        stats->ms_total = tm.ms(0, 2);
        stats->set_fraction_max = 0.0;
        stats->ms_sweeps = 0.0;
        stats->sweep_launches = it;
    }
    return status;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char *sl_status_string(int status) {
    switch (status) {
    case SL_OK: return "ok";
    case SL_NOT_CONVERGED: return "not converged (sweep cap reached)";
    case SL_ERR_INVALID_ARG: return "invalid argument";
    case SL_ERR_NO_TARGET: return "no target node";
    case SL_ERR_UNSUPPORTED: return "unsupported configuration";
    case SL_ERR_HIP: return "HIP runtime error";
    case SL_ERR_WORKSPACE: return "workspace too small";
    default: return "unknown status";
    }
}

int sl_abi_version(void) { return SLHJB_ABI_VERSION; }

size_t sl_solve_workspace_size(const sl_problem *p) {
    if (validate(p) != SL_OK) return 0;
    Arena a{nullptr, 0};
    const int v = default_variant(p->dim, p->dtype);
    if (p->dtype == SL_F32) {
        Exec<float> ex;
        float *Vb[2], *wl, *ctrl;
        FieldStats *fs;
        plan_global<float>(p, a, ex, Vb, &wl, &ctrl, &fs, v);
    } else {
        Exec<double> ex;
        double *Vb[2], *wl, *ctrl;
        FieldStats *fs;
        plan_global<double>(p, a, ex, Vb, &wl, &ctrl, &fs, v);
    }
    return a.off + 256;
}

int sl_solve(const sl_problem *p, const sl_solve_opts *o, void *ws, size_t ws_bytes, void *V,
             uint8_t *policy, sl_stats *stats, void *stream) {
    int rc = validate(p);
    if (rc) return rc;
    if ((rc = validate_solve_opts(o))) return rc;
    if (!V || !ws) return SL_ERR_INVALID_ARG;
    if (ws_bytes < sl_solve_workspace_size(p)) return SL_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == SL_F32)
        return solve_global<float>(p, o, ws, ws_bytes, (float *)V, policy, stats, s);
    return solve_global<double>(p, o, ws, ws_bytes, (double *)V, policy, stats, s);
}

size_t sl_isa_workspace_size(const sl_problem *p, const sl_ra_opts *ra) {
    if (validate(p) != SL_OK || validate_ra(p, ra) != SL_OK) return 0;
    Arena a{nullptr, 0};
    if (p->dtype == SL_F32) {
        IsaPlan<float> P;
        plan_isa<float>(p, ra, a, P);
    } else {
        IsaPlan<double> P;
        plan_isa<double>(p, ra, a, P);
    }
    return a.off + 256;
}

int sl_reconstruct(const sl_problem *p, const sl_ra_opts *ra, void *ws, size_t ws_bytes,
                   uint8_t *member, uint8_t *label, uint8_t *member_K, uint8_t *label_K,
                   sl_stats *stats, void *stream) {
    int rc = validate(p);
    if (rc) return rc;
    if ((rc = validate_ra(p, ra))) return rc;
    if (!member || !label || !ws) return SL_ERR_INVALID_ARG;
    if (ws_bytes < sl_isa_workspace_size(p, ra)) return SL_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == SL_F32)
        return reconstruct_impl<float>(p, ra, ws, ws_bytes, member, label, member_K, label_K,
                                       stats, s);
    return reconstruct_impl<double>(p, ra, ws, ws_bytes, member, label, member_K, label_K,
                                    stats, s);
}

int sl_solve_isa(const sl_problem *p, const sl_ra_opts *ra, const uint8_t *member,
                 const sl_solve_opts *o, void *ws, size_t ws_bytes, void *V, uint8_t *owner,
                 uint8_t *policy, void *V_sets, sl_stats *stats, void *stream) {
    int rc = validate(p);
    if (rc) return rc;
    if ((rc = validate_ra(p, ra))) return rc;
    if ((rc = validate_solve_opts(o))) return rc;
    if (!member || !V || !ws) return SL_ERR_INVALID_ARG;
    if (ws_bytes < sl_isa_workspace_size(p, ra)) return SL_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == SL_F32)
        return isa_impl<float>(p, ra, member, o, ws, ws_bytes, (float *)V, owner, policy,
                               (float *)V_sets, stats, s);
    return isa_impl<double>(p, ra, member, o, ws, ws_bytes, (double *)V, owner, policy,
                            (double *)V_sets, stats, s);
}

size_t sl_adjoint_workspace_size(const sl_problem *p, int n_sets) {
    if (validate(p) != SL_OK || n_sets < 1 || n_sets > SL_MAX_COMP) return 0;
    Arena a{nullptr, 0};
    if (p->dtype == SL_F32) {
        AdjPlan<float> P;
        plan_adjoint<float>(p, n_sets, a, P);
    } else {
        AdjPlan<double> P;
        plan_adjoint<double>(p, n_sets, a, P);
    }
    return a.off + 256;
}

int sl_adjoint(const sl_problem *p, const uint8_t *member, const uint8_t *owner,
               const uint8_t *policy, const void *dLdV, void *dLdl, double tol, long max_iters,
               void *ws, size_t ws_bytes, sl_stats *stats, void *stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!policy || !dLdV || !dLdl || !ws) return SL_ERR_INVALID_ARG;
    if (!(tol >= 0.0) || !std::isfinite(tol) || max_iters < 1) return SL_ERR_INVALID_ARG;
    const int n_sets = member ? p->n_comp : 1;
    if (ws_bytes < sl_adjoint_workspace_size(p, n_sets)) return SL_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == SL_F32)
        return adjoint_impl<float>(p, member, owner, policy, (const float *)dLdV, (float *)dLdl,
                                   tol, max_iters, ws, ws_bytes, stats, s);
    return adjoint_impl<double>(p, member, owner, policy, (const double *)dLdV, (double *)dLdl,
                                tol, max_iters, ws, ws_bytes, stats, s);
}

}  // extern "C"
