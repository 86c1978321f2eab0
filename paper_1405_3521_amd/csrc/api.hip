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
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

using namespace slhjb;

// ------------------------------------------------------- no-allocation scratch
// The workspace of sl_solve_noalloc: a file-scope device array that the code
// object carries, so each device holds its own copy from module load until the
// process ends.  Host code never passes `scratch` itself to a kernel (its host
// name is a stand-in, not a device address): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[SL_NOALLOC_SCRATCH_BYTES];

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

// Rows of the displacement table: the pursuer's controls for every evader choice.
int table_rows(const sl_problem *p) { return p->m * (p->m_b > 0 ? p->m_b : 1); }
bool is_game(const sl_problem *p) { return p->m_b > 0; }
// Values per node of the speed field.
int speed_comps(const sl_problem *p) { return p->speed && p->speed_axes ? p->dim : 1; }

int validate(const sl_problem *p) {
    if (!p) return SL_ERR_INVALID_ARG;
    if (p->dim != 2 && p->dim != 3) return SL_ERR_UNSUPPORTED;
    if (p->m < 1 || p->m > SL_MAX_CONTROLS) return SL_ERR_UNSUPPORTED;
    if (p->m_b < 0 || p->m_b > SL_MAX_CONTROLS) return SL_ERR_UNSUPPORTED;
    if ((p->m_b > 0) != (p->velocity_b != nullptr)) return SL_ERR_INVALID_ARG;
    if (table_rows(p) > SL_MAX_TABLE) return SL_ERR_UNSUPPORTED;
    if (p->speed_axes != 0 && p->speed_axes != 1) return SL_ERR_INVALID_ARG;
    if (p->speed_axes && !p->speed) return SL_ERR_INVALID_ARG;
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
    for (int i = 0; i < p->m_b * p->dim; ++i)
        if (!std::isfinite(p->velocity_b[i])) return SL_ERR_INVALID_ARG;
    if (!(p->lambda > 0.0) || !std::isfinite(p->lambda)) return SL_ERR_INVALID_ARG;
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return SL_ERR_INVALID_ARG;
    if (!std::isfinite(p->v_ghost)) return SL_ERR_INVALID_ARG;
    if (p->disc != SL_DISC_EXP && p->disc != SL_DISC_PAPER && p->disc != SL_DISC_KRUZKOV)
        return SL_ERR_INVALID_ARG;
    if (p->dtype != SL_F32 && p->dtype != SL_F64) return SL_ERR_INVALID_ARG;
    if (p->interp != SL_INTERP_Q1 && p->interp != SL_INTERP_P1) return SL_ERR_INVALID_ARG;
    return SL_OK;
}

int validate_solve_opts(const sl_solve_opts *o) {
    if (!o) return SL_ERR_INVALID_ARG;
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return SL_ERR_INVALID_ARG;
    if (o->max_sweeps < 1 || o->max_sweeps > 100000000L) return SL_ERR_INVALID_ARG;
    if (o->check_every < 0) return SL_ERR_INVALID_ARG;
    if (o->autotune > 2) return SL_ERR_INVALID_ARG;
    if (o->local_iters < 0 || o->local_iters > 1024) return SL_ERR_INVALID_ARG;
    return SL_OK;
}

int validate_ra(const sl_problem *p, const sl_ra_opts *ra) {
    if (!ra) return SL_ERR_INVALID_ARG;
    if (ra->coarse_n[0] > 0) {
        for (int d = 0; d < p->dim; ++d)
            if (ra->coarse_n[d] < 3 || ra->coarse_n[d] > p->n[d]) return SL_ERR_INVALID_ARG;
    } else {
        if (ra->coarse_stride < 1) return SL_ERR_INVALID_ARG;
        for (int d = 0; d < p->dim; ++d) {
            if ((p->n[d] - 1) % ra->coarse_stride) return SL_ERR_INVALID_ARG;
            if ((p->n[d] - 1) / ra->coarse_stride + 1 < 3) return SL_ERR_INVALID_ARG;
        }
    }
    if (!std::isfinite(ra->C) || !std::isfinite(ra->M) || !std::isfinite(ra->q))
        return SL_ERR_INVALID_ARG;
    if (!(ra->delta_override >= 0.0) && !(ra->delta_override < 0.0)) return SL_ERR_INVALID_ARG;
    if (!(ra->tol >= 0.0) || ra->max_sweeps < 1) return SL_ERR_INVALID_ARG;
    if (ra->autotune > 2) return SL_ERR_INVALID_ARG;
    if (ra->local_iters < 0 || ra->local_iters > 1024) return SL_ERR_INVALID_ARG;
    return SL_OK;
}

// Discount and cost weight of one step (same formulas as the scheme's statement).
void scheme_constants(double lam, double h, int disc, double *beta, double *w) {
    if (disc == SL_DISC_EXP) {
        *beta = std::exp(-lam * h);
        *w = -std::expm1(-lam * h) / lam;
    } else if (disc == SL_DISC_KRUZKOV) {     // the per-node form with l = 1
        *beta = std::exp(-h);
        *w = -std::expm1(-h);
    } else {
        *beta = 1.0 / (1.0 + lam * h);
        *w = h;
    }
}

// Per-node discount and cost term of the Kruzkov form, beta_j = exp(-h l_j) and
// 1 - beta_j = -expm1(-h l_j), evaluated on the host in binary64 (the problem
// statement's transcendentals; the running cost crosses to the host once).
// wl may alias l.
bool uses_node_discount(const sl_problem *p) { return p->disc == SL_DISC_KRUZKOV && p->cost; }

template <typename T>
int kruzkov_fields(const T *l, size_t n, double h, T *beta, T *wl, hipStream_t s) {
    std::vector<T> hl(n), hb(n), hw(n);
    HIPCHK(hipMemcpyAsync(hl.data(), l, sizeof(T) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (size_t j = 0; j < n; ++j) {
        const double x = -h * (double)hl[j];
        hb[j] = (T)std::exp(x);
        hw[j] = (T)(-std::expm1(x));
    }
    HIPCHK(hipMemcpyAsync(beta, hb.data(), sizeof(T) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(wl, hw.data(), sizeof(T) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return SL_OK;
}

// Displacements in cells per unit speed, row l*m + k: e_d = (h/dx_d) * (a_kd - b_ld)
// (the difference first, in FP64), or (h/dx_d) * a_kd for a control problem.
void control_table(const sl_problem *p, const int *n, double h, std::vector<double> &e,
                   double *emax) {
    double t[3];
    for (int d = 0; d < p->dim; ++d) t[d] = h / ((p->hi[d] - p->lo[d]) / (double)(n[d] - 1));
    const int mb = p->m_b > 0 ? p->m_b : 1;
    e.resize((size_t)table_rows(p) * p->dim);
    *emax = 0.0;
    for (int l = 0; l < mb; ++l)
        for (int k = 0; k < p->m; ++k)
            for (int d = 0; d < p->dim; ++d) {
                const double a = p->velocity[(size_t)k * p->dim + d];
                const double rel = p->m_b > 0 ? a - p->velocity_b[(size_t)l * p->dim + d] : a;
                const size_t i = ((size_t)l * p->m + k) * p->dim + d;
                e[i] = t[d] * rel;
                *emax = std::max(*emax, std::fabs(e[i]));
            }
}

// Cells a foot can reach: c * |e| over the controls plus the drift's |q| (index units).
int halo_for(double speed_max, double emax, double drift_reach = 0.0) {
    const double D = speed_max * emax + drift_reach;
    if (!std::isfinite(D)) return INT_MAX;
    // floor(D) + 1 covers both corners of every foot; the margin absorbs the
    // rounding of c*e and of the foot coordinate.
    return (int)std::floor(D * (1.0 + 1e-6) + 1e-3) + 1;
}

int max_halo(int dim) { return dim == 2 ? kMaxHalo : kMaxHalo3D; }

int default_variant(int dim, int dtype) {
    if (dim == 2) return dtype == SL_F32 ? 0 : 4;
    return dtype == SL_F32 ? 5 : 8;
}

LaunchCfg make_cfg(int dim, int dtype, int halo, int variant) {
    LaunchCfg all[kMaxVariants];
    const int nv = sweep_variants(dim, all, kMaxVariants);
    LaunchCfg c{};
    for (int i = 0; i < nv && i < kMaxVariants; ++i)
        if (all[i].variant == variant) c = all[i];
    c.halo = halo;
    c.mode = 0;
    return c;
}

// Pinned host scratch for the per-chunk convergence poll, for statistics read
// back after a later synchronisation (kPinnedStats bytes), and for the read-backs
// that end a call (kPinnedReadback bytes, see Readback).
constexpr size_t kPinnedStats = 16384;
constexpr size_t kPinnedReadback = 262144;
struct Pinned {
    int *active = nullptr;
    char *stats = nullptr;
    char *readback = nullptr;
    Pinned() {
        if (hipHostMalloc((void **)&active, sizeof(int) * 16, hipHostMallocDefault) != hipSuccess)
            active = nullptr;
        if (hipHostMalloc((void **)&stats, kPinnedStats, hipHostMallocDefault) != hipSuccess)
            stats = nullptr;
        if (hipHostMalloc((void **)&readback, kPinnedReadback, hipHostMallocDefault) != hipSuccess)
            readback = nullptr;
    }
};
Pinned &pinned() {
    static thread_local Pinned p;
    return p;
}

// Device-to-host copies that end a call, completed by one synchronisation of
// the stream.  A copy into pageable memory waits for the stream by itself, so
// several of them cost one round trip each; here they land in the pinned
// read-back buffer in stream order and are moved to their destinations after
// finish().  Without that buffer (the no-allocation path) or when it is full,
// a copy goes to its destination directly.  Destinations must stay valid and
// untouched until finish().  One Readback at a time per thread: every call
// that uses the buffer ends with finish().
struct Readback {
    hipStream_t s;
    char *buf;
    size_t used = 0;
    struct Item {
        void *dst;
        size_t off, n;
    };
    std::vector<Item> items;
    Readback(hipStream_t s_, bool use_pinned) : s(s_), buf(use_pinned ? pinned().readback : nullptr) {}
    hipError_t add(void *dst, const void *src, size_t n) {
        const size_t off = (used + 63) & ~(size_t)63;
        if (!buf || n > kPinnedReadback || off > kPinnedReadback - n)
            return hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s);
        const hipError_t e = hipMemcpyAsync(buf + off, src, n, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        items.push_back({dst, off, n});
        used = off + n;
        return hipSuccess;
    }
    hipError_t finish() {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        for (const Item &it : items) std::memcpy(it.dst, buf + it.off, it.n);
        items.clear();
        used = 0;
        return hipSuccess;
    }
};

// A private stream for graph capture (captured graphs are launched on the
// caller's stream; capture itself needs a non-default stream).  Default priority.
hipStream_t capture_stream() {
    static thread_local hipStream_t cs = nullptr;
    if (!cs && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) cs = nullptr;
    return cs;
}

// Instantiated chunk graphs kept across calls, keyed by everything their launches
// take as arguments (device pointers, sizes, kernel configurations, tolerance), so
// a call that repeats an earlier call's launches -- the same problem shape in the
// same workspace -- replays the earlier graph without capturing it again.  The
// node fields themselves are not in the key: kernels read them through the
// descriptors, which every call uploads.  Bounded: when the cache is full the
// least recently used entry is destroyed (a hit moves its entry to the back), so
// the graphs that a loop replays every step outlive those of one-off calls.
// The chunk loop waits for every chunk before it enqueues the next (or captures
// a new graph), so on one host thread an evicted graph is never in flight.
struct GraphCache {
    static constexpr size_t kMax = 32;
    std::vector<std::pair<std::vector<unsigned long long>, hipGraphExec_t>> entries;
    std::mutex mu;
    hipGraphExec_t find(const std::vector<unsigned long long> &key) {
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < entries.size(); ++i)
            if (entries[i].first == key) {
                std::rotate(entries.begin() + i, entries.begin() + i + 1, entries.end());
                return entries.back().second;
            }
        return nullptr;
    }
    void insert(std::vector<unsigned long long> key, hipGraphExec_t exec) {
        std::lock_guard<std::mutex> lk(mu);
        if (entries.size() >= kMax) {
            (void)hipGraphExecDestroy(entries.front().second);
            entries.erase(entries.begin());
        }
        entries.emplace_back(std::move(key), exec);
    }
};
GraphCache &graph_cache() {
    static GraphCache c;
    return c;
}

// Converged sweep counts of earlier calls, keyed like the graph cache: a call
// that repeats an earlier call's launches polls first near that call's count
// instead of every 32 sweeps (the results do not depend on where the host
// polls: sweeps of converged sets change nothing).  The key holds the launch
// arguments, not the field values, so a call on new data in the same workspace
// inherits the count; if it converges sooner, the launches up to the first
// poll find nothing to do (a few microseconds each).  Bounded: cleared when
// full.
struct SweepHints {
    static constexpr size_t kMax = 64;
    std::map<std::vector<unsigned long long>, long> m;
    std::mutex mu;
    long find(const std::vector<unsigned long long> &key) {
        std::lock_guard<std::mutex> lk(mu);
        const auto it = m.find(key);
        return it == m.end() ? 0 : it->second;
    }
    void put(const std::vector<unsigned long long> &key, long v) {
        std::lock_guard<std::mutex> lk(mu);
        if (m.size() >= kMax && !m.count(key)) m.clear();
        m[key] = v;
    }
};
SweepHints &sweep_hints() {
    static SweepHints h;
    return h;
}

// Runs `enqueue(stream, todo)` -- `todo` iterations, then a bookkeeping launch
// that advances the device-side iteration base, then a copy of the active-set
// counter to pinned host memory -- in chunks until the counter is zero or
// max_steps iterations are done.  The first chunk has `first` iterations, the
// others `chunk`.  Full chunks are captured as hipGraphs (one per length) and
// replayed on the caller's stream (from the graph cache when `key` is given);
// a short last chunk is launched directly.
struct ChunkLoop {
    double ms = 0.0;         // HIP-event time of the chunks (profile)
    long launches = 0;
    // `active`: host int the enqueued copy writes the active-set counter to
    template <class F>
    int run(F enqueue, long max_steps, int first, int chunk, hipStream_t s, int use_graph,
            int profile, long *done, int *status, int *active,
            const std::vector<unsigned long long> *key = nullptr) {
        if (!active) return SL_ERR_HIP;
        struct Slot {
            int len = 0;
            hipGraph_t graph = nullptr;
            hipGraphExec_t exec = nullptr;
            bool cached = false;
        } slots[2];
        // the replayable graph of a full chunk of `len` iterations (nullptr on error)
        auto graph_of = [&](int len) -> hipGraphExec_t {
            Slot *g = nullptr;
            for (auto &x : slots)
                if (x.len == len) g = &x;
            if (!g) {
                for (auto &x : slots)
                    if (!g && x.len == 0) g = &x;
                if (!g) return nullptr;
                g->len = len;
            }
            if (g->exec) return g->exec;
            std::vector<unsigned long long> k2;
            if (key) {
                k2 = *key;
                k2.push_back((unsigned long long)len);
                g->exec = graph_cache().find(k2);
                if (g->exec) {
                    g->cached = true;
                    return g->exec;
                }
            }
            hipStream_t cs = capture_stream();
            if (!cs || hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return nullptr;
            const hipError_t e1 = enqueue(cs, len);
            const hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
            if (e1 != hipSuccess || e2 != hipSuccess ||
                hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
                g->exec = nullptr;
                return nullptr;
            }
            if (key) {
                graph_cache().insert(k2, g->exec);
                g->cached = true;
            }
            return g->exec;
        };
        hipEvent_t ev[2] = {nullptr, nullptr};
        int rc = SL_OK;
        long S = 0;
        *status = SL_NOT_CONVERGED;
        if (profile && (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess))
            rc = SL_ERR_HIP;
        for (long c = 0; rc == SL_OK && S < max_steps; ++c) {
            const int len = c == 0 && first > 0 ? first : chunk;
            const int todo = (int)std::min<long>(len, max_steps - S);
            if (profile && hipEventRecord(ev[0], s) != hipSuccess) { rc = SL_ERR_HIP; break; }
            if (use_graph && todo == len) {
                const hipGraphExec_t exec = graph_of(len);
                if (!exec || hipGraphLaunch(exec, s) != hipSuccess) { rc = SL_ERR_HIP; break; }
            } else if (enqueue(s, todo) != hipSuccess) {
                rc = SL_ERR_HIP;
                break;
            }
            if (profile && hipEventRecord(ev[1], s) != hipSuccess) { rc = SL_ERR_HIP; break; }
            if (hipStreamSynchronize(s) != hipSuccess) { rc = SL_ERR_HIP; break; }
            S += todo;
            if (profile) {
                float t = 0.f;
                if (hipEventElapsedTime(&t, ev[0], ev[1]) == hipSuccess) ms += t;
                launches += todo;
            }
            if (*active == 0) {
                *status = SL_OK;
                break;
            }
        }
        for (auto &g : slots) {
            if (g.exec && !g.cached) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
        }
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        *done = S;
        return rc;
    }
};

// ------------------------------------------------------------------ autotuner
// Kernel configurations are chosen per problem shape by timing candidates on
// the caller's problem; the winner is cached for the life of the process.
struct TuneKey {
    int dim, dtype, m, m_inner, halo, nsd, size_class, local_iters, interp;
    bool operator<(const TuneKey &o) const {
        const int a[9] = {dim, dtype, m, m_inner, halo, nsd, size_class, local_iters, interp};
        const int b[9] = {o.dim,  o.dtype, o.m,          o.m_inner,     o.halo,
                          o.nsd,  o.size_class, o.local_iters, o.interp};
        return std::lexicographical_compare(a, a + 9, b, b + 9);
    }
};
std::map<TuneKey, std::pair<int, int>> &tune_cache() {
    static std::map<TuneKey, std::pair<int, int>> c;
    return c;
}
std::mutex &tune_mutex() {
    static std::mutex m;
    return m;
}

// Candidates for (dim, dtype); a game leaves out the variants that split the
// controls over several thread groups, P1 the variants without P1 kernels.
std::vector<LaunchCfg> tune_candidates(int dim, int dtype, int halo, bool game = false,
                                       int interp = SL_INTERP_Q1) {
    LaunchCfg all[kMaxVariants];
    const int nv = sweep_variants(dim, all, kMaxVariants);
    std::vector<LaunchCfg> out;
    for (int i = 0; i < nv && i < kMaxVariants; ++i) {
        if (all[i].dtype != dtype) continue;
        if (game && all[i].groups > 1) continue;
        if (interp == SL_INTERP_P1 && !sweep_has_p1(all[i].variant)) continue;
        for (int mode = 0; mode < 3; ++mode) {
            LaunchCfg c = all[i];
            c.halo = halo;
            c.mode = mode;
            c.interp = interp;
            out.push_back(c);
        }
    }
    return out;
}

// Most tiles any variant of (dim, dtype) needs on a grid of n nodes.
int max_tiles(int dim, int dtype, const int *n) {
    LaunchCfg all[kMaxVariants];
    const int nv = sweep_variants(dim, all, kMaxVariants);
    int best = 1;
    for (int i = 0; i < nv && i < kMaxVariants; ++i) {
        if (all[i].dtype != dtype) continue;
        int tot = 1;
        for (int d = 0; d < dim; ++d) tot *= (n[d] + all[i].tile[d] - 1) / all[i].tile[d];
        best = std::max(best, tot);
    }
    return best;
}

// --------------------------------------------------------------- executor
template <typename T>
struct Exec {
    LaunchCfg cfg{};
    SdDesc<T> *sds = nullptr;       // device
    SdState *st = nullptr;          // device
    WorkItem *items = nullptr;      // device
    WorkItem *lists = nullptr;      // device, 2 x tiles: active lists by sweep parity
    ExecCounters *cnt = nullptr;    // device
    int *prefix = nullptr;          // device
    int *stamp = nullptr;           // device, 2 x tiles: sweep each tile must be computed in
    int *class_off_dev = nullptr;   // device, kMaxClasses: item segment of each halo class
    // class_off_dev, prefix, st, sds and cnt share one block (one upload per prepare)
    char *hdr = nullptr;
    size_t hdr_bytes = 0, o_class = 0, o_prefix = 0, o_st = 0, o_sds = 0, o_cnt = 0;
    int n_sd = 0;
    int total_tiles = 0;
    int stamp_stride = 1;           // tiles reserved (stride of the two stamp arrays)
    std::vector<SdDesc<T>> host_sds;
    std::vector<int> host_prefix;
    // halo classes: sub-domains grouped by the halo they need; one launch per
    // class and sweep, each with the kernel instantiated for that halo
    std::vector<LaunchCfg> ccfg;
    std::vector<int> class_off, class_cap;
    int kind = 0;                   // 0: forward sweeps; 1: adjoint tiles (2D)
    double scale_rel = 0.0;         // rounding-aware stopping term (adjoint)

    void reserve(Arena &a, int nsd, int tiles_total) {
        size_t off = 0;
        auto put = [&off](size_t bytes) {
            const size_t o = off;
            off = (off + bytes + 255) & ~size_t(255);
            return o;
        };
        o_class = put(sizeof(int) * kMaxClasses);
        o_prefix = put(sizeof(int) * (size_t)nsd);
        o_st = put(sizeof(SdState) * (size_t)nsd);
        o_sds = put(sizeof(SdDesc<T>) * (size_t)nsd);
        o_cnt = put(sizeof(ExecCounters));
        hdr_bytes = off;
        hdr = a.take<char>(hdr_bytes);
        class_off_dev = hdr ? reinterpret_cast<int *>(hdr + o_class) : nullptr;
        prefix = hdr ? reinterpret_cast<int *>(hdr + o_prefix) : nullptr;
        st = hdr ? reinterpret_cast<SdState *>(hdr + o_st) : nullptr;
        sds = hdr ? reinterpret_cast<SdDesc<T> *>(hdr + o_sds) : nullptr;
        cnt = hdr ? reinterpret_cast<ExecCounters *>(hdr + o_cnt) : nullptr;
        items = a.take<WorkItem>(tiles_total > 0 ? tiles_total : 1);
        lists = a.take<WorkItem>(2 * (size_t)(tiles_total > 0 ? tiles_total : 1));
        stamp_stride = tiles_total > 0 ? tiles_total : 1;
        stamp = a.take<int>(2 * (size_t)stamp_stride);
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
        // block-asynchronous sweeps update in place: both Jacobi buffers are one array
        if (cfg.local_iters > 0)
            for (auto &d : host_sds) d.V[1] = d.V[0];
        host_prefix.resize(n_sd);
        int acc = 0;
        for (int i = 0; i < n_sd; ++i) {
            host_sds[i].tile_offset = acc;
            host_prefix[i] = acc;
            acc += host_sds[i].tiles[0] * host_sds[i].tiles[1] * host_sds[i].tiles[2];
        }
        total_tiles = acc;
        // halo classes (ascending halo)
        std::vector<int> halos;
        for (const auto &d : host_sds) halos.push_back(d.halo > 0 ? d.halo : cfg.halo);
        // in 2D a launch per class costs more than the wider staging of one class
        // at the largest halo while the staged region grows by at most 3x (the
        // region is loaded once per launch, the local iterations reuse it), so the
        // classes merge into one
        if (cfg.dim == 2 && kind == 0 && !halos.empty()) {
            const int hmin = *std::min_element(halos.begin(), halos.end());
            const int hmax = *std::max_element(halos.begin(), halos.end());
            const double rmin = (double)(cfg.tile[0] + 2 * hmin) * (cfg.tile[1] + 2 * hmin);
            const double rmax = (double)(cfg.tile[0] + 2 * hmax) * (cfg.tile[1] + 2 * hmax);
            if (rmax <= 3.0 * rmin)
                for (auto &h : halos) h = hmax;
        }
        std::vector<int> uniq = halos;
        std::sort(uniq.begin(), uniq.end());
        uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
        if ((int)uniq.size() > kMaxClasses) return SL_ERR_UNSUPPORTED;
        ccfg.assign(uniq.size(), cfg);
        class_cap.assign(uniq.size(), 0);
        class_off.assign(kMaxClasses, 0);
        for (int i = 0; i < n_sd; ++i) {
            const int c = (int)(std::lower_bound(uniq.begin(), uniq.end(), halos[i]) - uniq.begin());
            host_sds[i].cls = c;
            class_cap[c] += host_sds[i].tiles[0] * host_sds[i].tiles[1] * host_sds[i].tiles[2];
        }
        for (size_t c = 0; c < uniq.size(); ++c) {
            ccfg[c].halo = uniq[c];
            if (c > 0) class_off[c] = class_off[c - 1] + class_cap[c - 1];
            HIPCHK(kind == 1 ? adjoint_tiles_set_attributes(ccfg[c]) : sweep_set_attributes(ccfg[c]));
        }
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
        // class offsets, prefix, states, descriptors and zeroed counters in one copy
        if (!hdr || o_cnt + sizeof(ExecCounters) > hdr_bytes ||
            o_sds + sizeof(SdDesc<T>) * (size_t)n_sd > o_cnt)
            return SL_ERR_WORKSPACE;
        std::vector<char> h(hdr_bytes, 0);
        std::memcpy(h.data() + o_class, class_off.data(), sizeof(int) * kMaxClasses);
        std::memcpy(h.data() + o_prefix, host_prefix.data(), sizeof(int) * (size_t)n_sd);
        std::memcpy(h.data() + o_st, hs.data(), sizeof(SdState) * (size_t)n_sd);
        std::memcpy(h.data() + o_sds, host_sds.data(), sizeof(SdDesc<T>) * (size_t)n_sd);
        HIPCHK(hipMemcpyAsync(hdr, h.data(), hdr_bytes, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemsetAsync(stamp, 0xFF, sizeof(int) * 2 * (size_t)stamp_stride, s));
        HIPCHK(launch_build_items(cfg, sds, n_sd, total_tiles, prefix, items, cnt, class_off_dev, s));
        return SL_OK;
    }

    // One sweep (or the policy pass): one launch per non-empty halo class.
    hipError_t launch_classes(int sweep_rel, double tol, int want_policy, hipStream_t q) {
        bool first = true;
        for (size_t c = 0; c < ccfg.size(); ++c) {
            if (class_cap[c] == 0) continue;
            const hipError_t e =
                kind == 1
                    ? launch_adjoint_tiles<T>(ccfg[c], sds, st, n_sd, items + class_off[c],
                                              lists + class_off[c], cnt,
                                              class_cap[c], sweep_rel, tol, scale_rel, stamp,
                                              stamp_stride, (int)c, first ? 1 : 0, q)
                    : launch_sweep(ccfg[c], sds, st, n_sd, items + class_off[c],
                                   lists + class_off[c], cnt,
                                   class_cap[c], sweep_rel, tol, want_policy, stamp,
                                   stamp_stride, (int)c, first ? 1 : 0, q);
            if (e != hipSuccess) return e;
            first = false;
        }
        return hipSuccess;
    }

    // Sweeps until every sd meets tol or max_sweeps.  Returns SL_OK or
    // SL_NOT_CONVERGED; *sweeps_done = sweeps launched.
    // Profiling (optional): HIP events around each chunk of sweep launches
    // (a chunk also holds one bookkeeping launch and a 4-byte copy);
    // ms_sweeps / sweep_launches is the mean launch duration.
    double ms_sweeps = 0.0;
    long sweep_launches = 0;
    int use_graph = 1;
    // no_alloc: no graph capture, no events, and the convergence poll lands in a
    // plain host int (no pinned allocation) -- the path of sl_solve_noalloc
    int no_alloc = 0;
    int poll_host = 0;
    std::vector<unsigned long long> last_key;   // key of the last default-schedule run

    int run(double tol, long max_sweeps, int check_every, int want_policy, hipStream_t s,
            long *sweeps_done, int profile = 0) {
        int *active = no_alloc ? &poll_host : pinned().active;
        if (!active) return SL_ERR_HIP;
        int chunk = check_every > 0 ? check_every : 32;
        auto enqueue = [&](hipStream_t q, int todo) -> hipError_t {
            for (int i = 0; i < todo; ++i) {
                const hipError_t e = launch_classes(i, tol, 0, q);
                if (e != hipSuccess) return e;
            }
            hipError_t e = launch_bookkeep(st, n_sd, todo, tol, cnt, 0, q, scale_rel, todo);
            if (e != hipSuccess) return e;
            return hipMemcpyAsync(active, &cnt->n_active, sizeof(int), hipMemcpyDeviceToHost, q);
        };
        // everything the chunk's launches take as arguments
        std::vector<unsigned long long> key;
        auto put = [&key](const void *p) { key.push_back((unsigned long long)(uintptr_t)p); };
        auto putd = [&key](double v) {
            unsigned long long b;
            std::memcpy(&b, &v, sizeof(b));
            key.push_back(b);
        };
        key.push_back((unsigned long long)kind);
        key.push_back((unsigned long long)n_sd);
        key.push_back((unsigned long long)stamp_stride);
        key.push_back((unsigned long long)chunk);
        put(sds); put(st); put(items); put(lists); put(cnt); put(stamp); put(active);
        putd(tol);
        putd(scale_rel);
        for (size_t c = 0; c < ccfg.size(); ++c) {
            const LaunchCfg &g = ccfg[c];
            for (int v : {g.dim, g.dtype, g.tile[0], g.tile[1], g.tile[2], g.halo, g.variant,
                          g.mode, g.threads, g.grid_cap, g.local_iters, g.interp, class_off[c],
                          class_cap[c]})
                key.push_back((unsigned long long)(long long)v);
        }
        // default schedule: a repeat of an earlier call's launches polls first at
        // that call's converged count rounded up to a multiple of 8 (one poll and
        // at most 7 launches past convergence when it converges alike), then
        // every 8 sweeps
        int first = chunk;
        last_key.clear();
        if (check_every == 0 && !no_alloc) {
            last_key = key;
            const long h = sweep_hints().find(key);
            if (h > 0) {
                chunk = 8;
                first = (int)std::min<long>((h + 7) / 8 * 8, 1 << 20);
            }
        }
        ChunkLoop loop;
        long S = 0;
        int status = SL_NOT_CONVERGED;
        int rc = loop.run(enqueue, max_sweeps, first, chunk, s, no_alloc ? 0 : use_graph,
                          no_alloc ? 0 : profile, &S, &status, active, &key);
        if (rc) return rc;
        ms_sweeps += loop.ms;
        sweep_launches += loop.launches;
        HIPCHK(launch_bookkeep(st, n_sd, 0, tol, cnt, 1, s, scale_rel));
        if (want_policy) {
            HIPCHK(launch_classes(0, tol, 1, s));
            HIPCHK(launch_flip(st, n_sd, s));
        }
        *sweeps_done = S;
        return status;
    }

    void retile() {
        for (auto &d : host_sds) tiles_of(cfg, d.n, cfg.dim, d.tiles);
    }

    // Initial values (reinit(stream)), descriptors, work list and the sweeps,
    // with the kernel configuration taken from the tuner when autotune > 0.
    template <class Reinit>
    int solve_tuned(int autotune, Reinit reinit, double tol, long max_sweeps, int check_every,
                    int want_policy, hipStream_t s, long *sweeps_done, int profile) {
        const int local_iters = cfg.local_iters;   // not a tuned parameter
        bool game = false;
        for (const auto &d : host_sds) game = game || (d.m_inner > 0 && d.m_inner < d.m);
        if (autotune < 0) {                  // forced candidate (testing)
            const std::vector<LaunchCfg> cands =
                tune_candidates(cfg.dim, cfg.dtype, cfg.halo, game, cfg.interp);
            const int k = -autotune - 1;
            if (k >= (int)cands.size()) return SL_ERR_INVALID_ARG;
            cfg = cands[k];
            cfg.local_iters = local_iters;
        }
        if (autotune > 0) {
            long nodes = 0;
            for (const auto &d : host_sds) nodes += (long)d.n[0] * d.n[1] * d.n[2];
            int sc = 0;
            while ((1L << sc) < nodes) ++sc;
            const TuneKey key{cfg.dim,
                              cfg.dtype,
                              host_sds.empty() ? 0 : host_sds[0].m,
                              host_sds.empty() ? 0 : host_sds[0].m_inner,
                              cfg.halo,
                              (int)host_sds.size(),
                              sc,
                              local_iters,
                              cfg.interp};
            bool found = false;
            std::pair<int, int> pick;
            {
                std::lock_guard<std::mutex> lk(tune_mutex());
                auto it = tune_cache().find(key);
                if (it != tune_cache().end()) {
                    found = true;
                    pick = it->second;
                }
            }
            if (!found) {
                const std::vector<LaunchCfg> cands =
                    tune_candidates(cfg.dim, cfg.dtype, cfg.halo, game, cfg.interp);
                hipEvent_t e0, e1;
                HIPCHK(hipEventCreate(&e0));
                HIPCHK(hipEventCreate(&e1));
                double best = 1e300;
                pick = {cfg.variant, cfg.mode};
                const long trial = autotune == 1 ? std::min<long>(96, max_sweeps) : max_sweeps;
                for (const LaunchCfg &c : cands) {
                    cfg = c;
                    cfg.local_iters = local_iters;
                    retile();
                    HIPCHK(reinit(s));
                    int rc = prepare(s);
                    if (rc) return rc;
                    HIPCHK(hipEventRecord(e0, s));
                    long Sx = 0;
                    rc = run(tol, trial, check_every, 0, s, &Sx, 0);
                    if (rc < 0) return rc;
                    HIPCHK(hipEventRecord(e1, s));
                    HIPCHK(hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                    const double score = autotune == 1 ? ms / std::max<long>(Sx, 1) : ms;
                    if (score < best) {
                        best = score;
                        pick = {c.variant, c.mode};
                    }
                }
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                std::lock_guard<std::mutex> lk(tune_mutex());
                tune_cache()[key] = pick;
            }
            const int halo = cfg.halo, interp = cfg.interp;
            cfg = make_cfg(cfg.dim, cfg.dtype, halo, pick.first);
            cfg.interp = interp;
            cfg.mode = pick.second;
            cfg.local_iters = local_iters;
            ms_sweeps = 0.0;
            sweep_launches = 0;
        }
        retile();
        HIPCHK(reinit(s));
        int rc = prepare(s);
        if (rc) return rc;
        return run(tol, max_sweeps, check_every, want_policy, s, sweeps_done, profile);
    }

    unsigned long long unreached = 0;   // from the last read_stats
    // The states and counters queued on rb; take_stats after rb.finish().
    hipError_t queue_stats(Readback &rb, std::vector<SdState> &out, ExecCounters &c) const {
        out.resize(n_sd);
        const hipError_t e = rb.add(out.data(), st, sizeof(SdState) * n_sd);
        return e != hipSuccess ? e : rb.add(&c, cnt, sizeof(ExecCounters));
    }
    void take_stats(const std::vector<SdState> &out, const ExecCounters &c,
                    unsigned long long *nc) {
        *nc = c.nc_updates;
        unreached = c.n_unreached;
        remember(out, last_key);
    }
    int read_stats(hipStream_t s, std::vector<SdState> &out, unsigned long long *nc) {
        Readback rb(s, !no_alloc);
        ExecCounters c{};
        HIPCHK(queue_stats(rb, out, c));
        HIPCHK(rb.finish());
        take_stats(out, c, nc);
        return SL_OK;
    }

    // The states and counters copied to pinned `host` in stream order, to be read
    // after a later synchronisation of the stream (read_copied).
    static size_t copied_bytes(int n) { return sizeof(SdState) * n + sizeof(ExecCounters); }
    int copy_stats(hipStream_t s, char *host) const {
        if (!host || copied_bytes(n_sd) > kPinnedStats) return SL_ERR_HIP;
        HIPCHK(hipMemcpyAsync(host, st, sizeof(SdState) * n_sd, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(host + sizeof(SdState) * n_sd, cnt, sizeof(ExecCounters),
                              hipMemcpyDeviceToHost, s));
        return SL_OK;
    }
    static void read_copied(const char *host, int n, std::vector<SdState> &out,
                            unsigned long long *nc) {
        out.resize(n);
        std::memcpy(out.data(), host, sizeof(SdState) * n);
        ExecCounters c;
        std::memcpy(&c, host + sizeof(SdState) * n, sizeof(c));
        *nc = c.nc_updates;
    }

    // the poll hint of a default-schedule run: the number of sweeps after which
    // the bookkeeping sees every set converged
    static void remember(const std::vector<SdState> &out,
                         const std::vector<unsigned long long> &key) {
        if (key.empty()) return;
        long smax = 0;
        bool all = true;
        for (const auto &x : out) {
            all = all && x.conv_at >= 0;
            smax = std::max<long>(smax, (long)x.conv_at + 1);
        }
        if (all && smax > 0) sweep_hints().put(key, smax);
    }
};

// Statistics of a reconstruction whose read-back waits for the next
// synchronisation of the stream (the whole-ISA call): the coarse states are
// copied to pinned memory in stream order, so the host enqueues the fine solve
// without waiting for the reconstruction to finish.
struct DeferredRaStats {
    char *host = nullptr;
    int n_sd = 0;
    long launches = 0;
    std::vector<unsigned long long> key;
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
    stats->ra_sweeps_max = 0;
}

// Most sweeps over sub-domains [b, e) of a state vector (S for unconverged ones).
long sweeps_of(const std::vector<SdState> &hs, size_t b, size_t e, long S) {
    long smax = 0;
    for (size_t i = b; i < e && i < hs.size(); ++i)
        smax = std::max(smax, hs[i].conv_at >= 0 ? (long)hs[i].conv_at + 1 : S);
    return smax;
}

void fill_cfg(sl_stats *stats, const LaunchCfg &c) {
    if (!stats) return;
    stats->variant = c.variant;
    stats->mode = c.mode;
    for (int d = 0; d < 3; ++d) stats->tile[d] = c.tile[d];
}

struct Timer {
    hipEvent_t e[4]{};
    bool ok = false;
    explicit Timer(bool on = true) {
        ok = on;
        if (on)
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
        if (ok && hipEventSynchronize(e[b]) == hipSuccess &&
            hipEventElapsedTime(&v, e[a], e[b]) == hipSuccess)
            return v;
        return 0.0;
    }
};

// ------------------------------------------------------------ field statistics
template <typename T>
int gather_field_stats(const sl_problem *p, const int8_t *target, const T *speed,
                       const T *cost, size_t N, int n_comp, FieldStats *fs_dev,
                       FieldStats *host, hipStream_t s, const T *g_abs = nullptr) {
    FieldStats init{};
    for (int i = 0; i < SL_MAX_COMP; ++i) init.first_node[i] = INT_MAX;
    HIPCHK(hipMemcpyAsync(fs_dev, &init, sizeof(init), hipMemcpyHostToDevice, s));
    HIPCHK(launch_field_stats<T>(speed, speed_comps(p), cost, (const T *)p->drift, p->dim,
                                 target, N, n_comp, fs_dev, s));
    if (g_abs) HIPCHK(launch_abs_max<T>(g_abs, N, &fs_dev->g_absmax, s));
    HIPCHK(hipMemcpyAsync(host, fs_dev, sizeof(FieldStats), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return SL_OK;
}

double bits_to_double(unsigned long long b) {
    double d;
    std::memcpy(&d, &b, sizeof(d));
    return d;
}

// Index-unit factors t_d = h / dx_d of a grid with n nodes per axis (the same
// expression as the control table's).
void index_units(const sl_problem *p, const int *n, double h, double *t) {
    for (int d = 0; d < 3; ++d)
        t[d] = d < p->dim ? h / ((p->hi[d] - p->lo[d]) / (double)(n[d] - 1)) : 0.0;
}

// Largest drift displacement per step in cells, max_d t_d * max|b|.
double drift_reach(const sl_problem *p, const int *n, double h, const FieldStats &fs) {
    if (!p->drift) return 0.0;
    double t[3];
    index_units(p, n, h, t);
    double tm = 0.0;
    for (int d = 0; d < p->dim; ++d) tm = std::max(tm, t[d]);
    return tm * bits_to_double(fs.drift_max);
}

int check_fields(const FieldStats &fs) {
    if (fs.bad_speed || fs.bad_cost || fs.bad_target) return SL_ERR_INVALID_ARG;
    if (fs.n_target == 0) return SL_ERR_NO_TARGET;
    return SL_OK;
}

// A free node that never reads a reached value keeps v_ghost up to rounding: the
// iteration V = beta V + w l settles within about eps G / (1 - beta) of G (the
// rounding of one step, amplified by the contraction).  Values within eight
// times that count as unreached.
template <typename T>
T unreached_level(const sl_problem *p) {
    const double eps = sizeof(T) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16;
    double beta, w;
    scheme_constants(p->lambda, p->h, p->disc, &beta, &w);
    const double G = p->v_ghost;
    return (T)(G - 8.0 * eps * std::fabs(G) / std::max(1.0 - beta, 1e-12));
}

// ------------------------------------------------------------ global solve
template <typename T>
int plan_global(const sl_problem *p, Arena &a, Exec<T> &ex, T **Vb, T **wl, T **ctrl,
                FieldStats **fs, int variant, T **q = nullptr, T **bn = nullptr) {
    const size_t N = nodes_of(p);
    (void)variant;
    const int tiles = max_tiles(p->dim, p->dtype, p->n);
    Vb[0] = a.take<T>(2 * N);       // both buffers back to back (one init launch)
    Vb[1] = Vb[0] ? Vb[0] + N : nullptr;
    *wl = p->cost ? a.take<T>(N) : nullptr;
    T *bb = uses_node_discount(p) ? a.take<T>(N) : nullptr;
    if (bn) *bn = bb;
    T *qq = p->drift ? a.take<T>(N * (size_t)p->dim) : nullptr;
    if (q) *q = qq;
    *ctrl = a.take<T>((size_t)table_rows(p) * p->dim);
    *fs = a.take<FieldStats>(1);
    ex.reserve(a, 1, tiles);
    return SL_OK;
}

template <typename T>
int solve_global(const sl_problem *p, const sl_solve_opts *o, void *ws, size_t ws_bytes,
                 T *V, uint8_t *policy, sl_stats *stats, hipStream_t s, bool no_alloc = false) {
    Timer tm(!no_alloc);
    tm.mark(0, s);
    const size_t N = nodes_of(p);
    const int variant = default_variant(p->dim, p->dtype);
    Arena a{(char *)ws, ws_bytes};
    Exec<T> ex;
    ex.no_alloc = no_alloc ? 1 : 0;
    T *Vb[2], *wl, *ctrl, *q = nullptr, *bn = nullptr;
    FieldStats *fs_dev;
    plan_global<T>(p, a, ex, Vb, &wl, &ctrl, &fs_dev, variant, &q, &bn);
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
    const int H = halo_for(smax, emax, drift_reach(p, p->n, p->h, fs));
    if (H > max_halo(p->dim)) return SL_ERR_UNSUPPORTED;
    ex.cfg = make_cfg(p->dim, p->dtype, H, variant);
    ex.cfg.interp = p->interp;
    ex.cfg.local_iters = o->local_iters;
    if (p->drift) {
        double t[3];
        index_units(p, p->n, p->h, t);
        HIPCHK(launch_scale_drift<T>((const T *)p->drift, q, N, p->dim, t, s));
    }

    std::vector<T> et(e.size());
    for (size_t i = 0; i < e.size(); ++i) et[i] = (T)e[i];
    HIPCHK(hipMemcpyAsync(ctrl, et.data(), sizeof(T) * et.size(), hipMemcpyHostToDevice, s));
    if (uses_node_discount(p)) {
        if ((rc = kruzkov_fields<T>((const T *)p->cost, N, p->h, bn, wl, s))) return rc;
    } else if (p->cost) {
        HIPCHK((launch_scale_field<T, T>((const T *)p->cost, wl, N, w, s)));
    }
    // both buffers (Vb[1] follows Vb[0]) in one launch
    auto reinit = [&](hipStream_t q) -> hipError_t {
        return launch_init_values<T>(Vb[0], p->target, (const T *)p->g, (T)p->v_ghost, -1, N, q,
                                     2);
    };
    SdDesc<T> d{};
    d.V[0] = Vb[0];
    d.V[1] = Vb[1];
    d.speed = (const T *)p->speed;
    d.wl = wl;
    d.beta_n = bn;
    d.drift = q;
    d.target = p->target;
    d.member = nullptr;
    d.policy = policy;
    d.ctrl = ctrl;
    d.wl_const = (T)w;
    d.beta = (T)beta;
    d.G = (T)p->v_ghost;
    for (int k = 0; k < 3; ++k) d.n[k] = k < p->dim ? p->n[k] : 1;
    d.m = table_rows(p);
    d.m_inner = p->m;
    d.speed_axes = speed_comps(p) > 1;
    d.bit = 0;
    Exec<T>::tiles_of(ex.cfg, p->n, p->dim, d.tiles);
    d.halo = H;
    ex.host_sds.push_back(d);
    if (o->want_policy && policy) HIPCHK(hipMemsetAsync(policy, 0xFF, N, s));
    tm.mark(1, s);
    long S = 0;
    const int status = ex.solve_tuned(o->autotune, reinit, o->tol, o->max_sweeps, o->check_every,
                                      o->want_policy && policy, s, &S, o->profile);
    if (status < 0) return status;
    HIPCHK(launch_copy_final<T>(ex.sds, ex.st, 0, V, N, s));
    HIPCHK(launch_count_unreached<T>(V, p->target, N, unreached_level<T>(p),
                                     &ex.cnt->n_unreached, s));
    tm.mark(2, s);
    std::vector<SdState> hs;
    unsigned long long nc = 0;
    if ((rc = ex.read_stats(s, hs, &nc))) return rc;
    fill_stats(stats, hs, nc, S);
    if (stats) stats->n_unreachable = (int)ex.unreached;
    if (stats) {
        stats->ms_ra = 0.0;
        stats->ms_fine = tm.ms(1, 2);
        stats->ms_total = tm.ms(0, 2);
        stats->set_fraction_max = 1.0;
        stats->ms_sweeps = ex.ms_sweeps;
        stats->sweep_launches = ex.sweep_launches;
    }
    fill_cfg(stats, ex.cfg);
    return status;
}

// --------------------------------------------------------------- RA and ISA
struct CoarseGeom {
    int nK[3];
    size_t NK;
    double hK;
};

// The coarse grid K: coarse_n nodes per axis, else every s-th fine node; the SL
// step on K is h times the largest spacing ratio (n_d - 1)/(nK_d - 1).
CoarseGeom coarse_geom(const sl_problem *p, const sl_ra_opts *ra) {
    CoarseGeom g{};
    g.NK = 1;
    double ratio = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (d >= p->dim) {
            g.nK[d] = 1;
            continue;
        }
        g.nK[d] = ra->coarse_n[0] > 0 ? ra->coarse_n[d] : (p->n[d] - 1) / ra->coarse_stride + 1;
        g.NK *= (size_t)g.nK[d];
        ratio = std::max(ratio, (double)(p->n[d] - 1) / (double)(g.nK[d] - 1));
    }
    g.hK = p->h * ratio;
    return g;
}

template <typename T>
struct IsaPlan {
    // coarse
    double *cK = nullptr, *wlK = nullptr, *gK = nullptr, *ctrlK = nullptr, *gK_src = nullptr;
    double *qK = nullptr;          // coarse drift in index units (NK * dim)
    double *betaK = nullptr;       // coarse per-node discount (Kruzkov form)
    T *gK_t = nullptr;
    int8_t *tK = nullptr;
    double *Vaux = nullptr;        // n_comp * 2 * NK
    uint8_t *mK = nullptr, *lbK = nullptr;
    FieldStats *fsK = nullptr;
    Exec<double> exK;
    // fine
    T *Vf = nullptr;               // n_comp * 2 * N
    T *wl = nullptr, *ctrl = nullptr;
    T *q = nullptr;                // fine drift in index units (N * dim)
    T *bn = nullptr;               // fine per-node discount (Kruzkov form)
    FieldStats *fs = nullptr;
    unsigned long long *counts = nullptr;
    Exec<T> ex;
};

template <typename T>
void plan_isa(const sl_problem *p, const sl_ra_opts *ra, Arena &a, IsaPlan<T> &P) {
    const size_t N = nodes_of(p);
    const CoarseGeom cg = coarse_geom(p, ra);
    const int nc = p->n_comp;
    const int tilesK = max_tiles(p->dim, SL_F64, cg.nK);
    P.gK_t = a.take<T>(cg.NK);
    P.cK = a.take<double>(cg.NK * (size_t)speed_comps(p));
    P.wlK = a.take<double>(cg.NK);
    P.qK = p->drift ? a.take<double>(cg.NK * (size_t)p->dim) : nullptr;
    P.betaK = uses_node_discount(p) ? a.take<double>(cg.NK) : nullptr;
    P.gK = a.take<double>(cg.NK);
    P.ctrlK = a.take<double>((size_t)table_rows(p) * p->dim);
    P.tK = a.take<int8_t>(cg.NK);
    P.Vaux = a.take<double>((size_t)nc * 2 * cg.NK);
    P.mK = a.take<uint8_t>(cg.NK);
    P.lbK = a.take<uint8_t>(cg.NK);
    P.fsK = a.take<FieldStats>(1);
    P.exK.reserve(a, nc, tilesK * nc);
    const int tiles = max_tiles(p->dim, p->dtype, p->n);
    P.Vf = a.take<T>((size_t)nc * 2 * N);
    P.wl = p->cost ? a.take<T>(N) : nullptr;
    P.q = p->drift ? a.take<T>(N * (size_t)p->dim) : nullptr;
    P.bn = uses_node_discount(p) ? a.take<T>(N) : nullptr;
    P.ctrl = a.take<T>((size_t)table_rows(p) * p->dim);
    P.fs = a.take<FieldStats>(1);
    P.counts = a.take<unsigned long long>(8);
    P.ex.reserve(a, nc, tiles * nc);
}

template <typename T>
int reconstruct_impl(const sl_problem *p, const sl_ra_opts *ra, void *ws, size_t ws_bytes,
                     uint8_t *member, uint8_t *label, uint8_t *member_K, uint8_t *label_K,
                     sl_stats *stats, hipStream_t s, FieldStats *fs_out = nullptr,
                     DeferredRaStats *defer = nullptr) {
    Timer tm(defer == nullptr);
    tm.mark(0, s);
    const size_t N = nodes_of(p);
    Arena a{(char *)ws, ws_bytes};
    IsaPlan<T> P;
    plan_isa<T>(p, ra, a, P);
    if (!a.fits()) return SL_ERR_WORKSPACE;
    const CoarseGeom cg = coarse_geom(p, ra);
    const int nc = p->n_comp;

    // fine-grid statistics: validation and lowest node per component
    FieldStats fs{};
    int rc = gather_field_stats<T>(p, p->target, (const T *)p->speed, (const T *)p->cost, N, nc,
                                   P.fs, &fs, s);
    if (rc) return rc;
    if ((rc = check_fields(fs))) return rc;
    if (fs_out) *fs_out = fs;

    // coarse problem data: speed and cost by Q1 interpolation in FP64 (exact copies
    // at coincident nodes), target ids and g from the nearest fine node
    double betaK, wK, emaxK;
    scheme_constants(p->lambda, cg.hK, p->disc, &betaK, &wK);
    if (p->speed)
        HIPCHK(launch_sample_coarse<T>((const T *)p->speed, P.cK, p->n, cg.nK, p->dim,
                                       speed_comps(p), 1.0, s));
    if (uses_node_discount(p)) {
        // Q1 samples of l, then the Kruzkov discount and cost term at the coarse step
        HIPCHK(launch_sample_coarse<T>((const T *)p->cost, P.wlK, p->n, cg.nK, p->dim, 1, 1.0, s));
        if ((rc = kruzkov_fields<double>(P.wlK, cg.NK, cg.hK, P.betaK, P.wlK, s))) return rc;
    } else if (p->cost) {
        HIPCHK(launch_sample_coarse<T>((const T *)p->cost, P.wlK, p->n, cg.nK, p->dim, 1, wK, s));
    }
    if (p->g) HIPCHK(launch_gather_nearest<T>((const T *)p->g, P.gK_t, p->n, cg.nK, p->dim, s));
    if (p->drift) {
        // Q1 samples of the drift, then index units of the coarse step
        double tK[3];
        index_units(p, cg.nK, cg.hK, tK);
        HIPCHK(launch_sample_coarse<T>((const T *)p->drift, P.qK, p->n, cg.nK, p->dim, p->dim,
                                       1.0, s));
        HIPCHK(launch_scale_drift<double>(P.qK, P.qK, cg.NK, p->dim, tK, s));
    }
    HIPCHK(launch_gather_nearest<int8_t>(p->target, P.tK, p->n, cg.nK, p->dim, s));
    // components without a coincident coarse node: place them (in the field's own
    // dtype), then widen g to FP64
    {
        FieldStats init{};
        for (int i = 0; i < SL_MAX_COMP; ++i) init.first_node[i] = INT_MAX;
        HIPCHK(hipMemcpyAsync(P.fsK, &init, sizeof(init), hipMemcpyHostToDevice, s));
        HIPCHK(launch_field_stats<double>(nullptr, 1, nullptr, nullptr, p->dim, P.tK, cg.NK,
                                          nc, P.fsK, s));
        const int *first_fine = reinterpret_cast<const int *>(
            reinterpret_cast<const char *>(P.fs) + offsetof(FieldStats, first_node));
        const int *firstK = reinterpret_cast<const int *>(
            reinterpret_cast<const char *>(P.fsK) + offsetof(FieldStats, first_node));
        HIPCHK(launch_place_missing<T>(P.tK, p->g ? P.gK_t : nullptr, (const T *)p->g,
                                       first_fine, firstK, p->n, cg.nK, p->dim, nc, s));
        if (p->g) HIPCHK((launch_scale_field<T, double>(P.gK_t, P.gK, cg.NK, 1.0, s)));
    }

    // coarse auxiliary problems (RA step 1), FP64
    std::vector<double> e;
    control_table(p, cg.nK, cg.hK, e, &emaxK);
    HIPCHK(hipMemcpyAsync(P.ctrlK, e.data(), sizeof(double) * e.size(), hipMemcpyHostToDevice, s));
    const double smax = p->speed ? bits_to_double(fs.speed_max) : 1.0;
    const int HK = halo_for(smax, emaxK, drift_reach(p, cg.nK, cg.hK, fs));
    if (HK > max_halo(p->dim)) return SL_ERR_UNSUPPORTED;
    P.exK.cfg = make_cfg(p->dim, SL_F64, HK, default_variant(p->dim, SL_F64));
    P.exK.cfg.interp = p->interp;
    P.exK.cfg.local_iters = ra->local_iters;
    // the two buffers of every auxiliary problem i (component i keeps g) in one launch
    auto reinit = [&](hipStream_t q) -> hipError_t {
        return launch_init_values<double>(P.Vaux, P.tK, p->g ? P.gK : nullptr, p->v_ghost, -1,
                                          cg.NK, q, 2 * nc, 1);
    };
    for (int i = 0; i < nc; ++i) {
        double *V0 = P.Vaux + (size_t)i * 2 * cg.NK;
        SdDesc<double> d{};
        d.V[0] = V0;
        d.V[1] = V0 + cg.NK;
        d.speed = p->speed ? P.cK : nullptr;
        d.wl = p->cost ? P.wlK : nullptr;
        d.beta_n = P.betaK;
        d.drift = P.qK;
        d.target = P.tK;
        d.member = nullptr;
        d.policy = nullptr;
        d.ctrl = P.ctrlK;
        d.wl_const = wK;
        d.beta = betaK;
        d.G = p->v_ghost;
        for (int k = 0; k < 3; ++k) d.n[k] = cg.nK[k];
        d.m = table_rows(p);
        d.m_inner = p->m;
        d.speed_axes = speed_comps(p) > 1;
        d.bit = i;
        Exec<double>::tiles_of(P.exK.cfg, cg.nK, p->dim, d.tiles);
        d.halo = HK;
        P.exK.host_sds.push_back(d);
    }
    long S = 0;
    const int status =
        P.exK.solve_tuned(ra->autotune, reinit, ra->tol, ra->max_sweeps, 0, 0, s, &S, 0);
    if (status < 0) return status;

    // RA steps 2-3: min, threshold, label on the final auxiliary iterates.
    double dxK = 0.0;
    for (int d = 0; d < p->dim; ++d)
        dxK = std::max(dxK, (p->hi[d] - p->lo[d]) / (double)(cg.nK[d] - 1));
    const double delta = ra->delta_override > 0.0
                             ? ra->delta_override
                             : 2.0 * (ra->C * std::pow(dxK, ra->q) + ra->M * dxK);
    uint8_t *mK = member_K ? member_K : P.mK;
    uint8_t *lbK = label_K ? label_K : P.lbK;
    HIPCHK(launch_ra_combine(P.exK.sds, P.exK.st, nc, cg.NK, P.tK, delta, mK, lbK, s));
    // ISA step 2: projection to the fine grid
    HIPCHK(launch_project(mK, lbK, cg.nK, p->n, p->dim, member, label, s));
    if (defer) {
        defer->host = pinned().stats;
        defer->n_sd = P.exK.n_sd;
        defer->launches = S;
        defer->key = P.exK.last_key;
        if (P.exK.copy_stats(s, defer->host) != SL_OK) return SL_ERR_HIP;
        return status;
    }
    tm.mark(1, s);
    std::vector<SdState> hs;
    unsigned long long ncu = 0;
    if ((rc = P.exK.read_stats(s, hs, &ncu))) return rc;
    fill_stats(stats, hs, ncu, S);
    if (stats) {
        stats->ra_sweeps_max = sweeps_of(hs, 0, hs.size(), S);
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
             uint8_t *policy, T *V_sets, sl_stats *stats, hipStream_t s,
             const FieldStats *fs_in = nullptr) {
    Timer tm;
    tm.mark(0, s);
    const size_t N = nodes_of(p);
    Arena a{(char *)ws, ws_bytes};
    IsaPlan<T> P;
    plan_isa<T>(p, ra, a, P);
    if (!a.fits()) return SL_ERR_WORKSPACE;
    const int nc = p->n_comp;
    // fs_in: the statistics the reconstruction of the same call gathered
    FieldStats fs{};
    int rc = SL_OK;
    if (fs_in) {
        fs = *fs_in;
    } else {
        rc = gather_field_stats<T>(p, p->target, (const T *)p->speed, (const T *)p->cost, N, nc,
                                   P.fs, &fs, s);
        if (rc) return rc;
        if ((rc = check_fields(fs))) return rc;
    }

    double beta, w, emax;
    scheme_constants(p->lambda, p->h, p->disc, &beta, &w);
    std::vector<double> e;
    control_table(p, p->n, p->h, e, &emax);
    const double smax = p->speed ? bits_to_double(fs.speed_max) : 1.0;
    const int H = halo_for(smax, emax, drift_reach(p, p->n, p->h, fs));
    if (H > max_halo(p->dim)) return SL_ERR_UNSUPPORTED;
    P.ex.cfg = make_cfg(p->dim, p->dtype, H, default_variant(p->dim, p->dtype));
    P.ex.cfg.interp = p->interp;
    P.ex.cfg.local_iters = o->local_iters;
    if (p->drift) {
        double t[3];
        index_units(p, p->n, p->h, t);
        HIPCHK(launch_scale_drift<T>((const T *)p->drift, P.q, N, p->dim, t, s));
    }
    std::vector<T> et(e.size());
    for (size_t i = 0; i < e.size(); ++i) et[i] = (T)e[i];
    HIPCHK(hipMemcpyAsync(P.ctrl, et.data(), sizeof(T) * et.size(), hipMemcpyHostToDevice, s));
    if (uses_node_discount(p)) {
        if ((rc = kruzkov_fields<T>((const T *)p->cost, N, p->h, P.bn, P.wl, s))) return rc;
    } else if (p->cost) {
        HIPCHK((launch_scale_field<T, T>((const T *)p->cost, P.wl, N, w, s)));
    }
    // the two buffers of every set in one launch
    auto reinit = [&](hipStream_t q) -> hipError_t {
        return launch_init_values<T>(P.Vf, p->target, (const T *)p->g, (T)p->v_ghost, -1, N, q,
                                     2 * nc);
    };
    for (int i = 0; i < nc; ++i) {
        T *V0 = P.Vf + (size_t)i * 2 * N;
        SdDesc<T> d{};
        d.V[0] = V0;
        d.V[1] = V0 + N;
        d.speed = (const T *)p->speed;
        d.wl = P.wl;
        d.beta_n = P.bn;
        d.drift = P.q;
        d.target = p->target;
        d.member = member;
        d.policy = policy ? policy + (size_t)i * N : nullptr;
        d.ctrl = P.ctrl;
        d.wl_const = (T)w;
        d.beta = (T)beta;
        d.G = (T)p->v_ghost;
        for (int k = 0; k < 3; ++k) d.n[k] = k < p->dim ? p->n[k] : 1;
        d.m = table_rows(p);
        d.m_inner = p->m;
        d.speed_axes = speed_comps(p) > 1;
        d.bit = i;
        Exec<T>::tiles_of(P.ex.cfg, p->n, p->dim, d.tiles);
        d.halo = H;
        P.ex.host_sds.push_back(d);
    }
    if (o->want_policy && policy) HIPCHK(hipMemsetAsync(policy, 0xFF, (size_t)nc * N, s));
    tm.mark(1, s);
    long S = 0;
    const int status = P.ex.solve_tuned(o->autotune, reinit, o->tol, o->max_sweeps,
                                        o->check_every, o->want_policy && policy, s, &S,
                                        o->profile);
    if (status < 0) return status;
    tm.mark(2, s);
    HIPCHK(launch_assemble<T>(P.ex.sds, P.ex.st, nc, member, N, (T)p->v_ghost, V, owner, s));
    if (V_sets)
        for (int i = 0; i < nc; ++i)
            HIPCHK(launch_copy_final<T>(P.ex.sds, P.ex.st, i, V_sets + (size_t)i * N, N, s));
    HIPCHK(hipMemsetAsync(P.counts, 0, sizeof(unsigned long long) * 8, s));
    HIPCHK(launch_member_counts(member, N, P.counts, s));
    HIPCHK(launch_count_unreached<T>(V, p->target, N, unreached_level<T>(p),
                                     &P.ex.cnt->n_unreached, s));
    unsigned long long counts[8];
    Readback rb(s, true);
    HIPCHK(rb.add(counts, P.counts, sizeof(counts)));
    tm.mark(3, s);
    std::vector<SdState> hs;
    ExecCounters c{};
    unsigned long long ncu = 0;
    HIPCHK(P.ex.queue_stats(rb, hs, c));
    HIPCHK(rb.finish());
    P.ex.take_stats(hs, c, &ncu);
    fill_stats(stats, hs, ncu, S);
    if (stats) {
        stats->n_unreachable = (int)P.ex.unreached;
        double fr = 0.0;
        for (int i = 0; i < nc; ++i) fr = std::max(fr, (double)counts[i] / (double)N);
        stats->set_fraction_max = fr;
        stats->ms_ra = 0.0;
        stats->ms_fine = tm.ms(1, 2);
        stats->ms_total = tm.ms(0, 3);
        stats->ms_sweeps = P.ex.ms_sweeps;
        stats->sweep_launches = P.ex.sweep_launches;
    }
    fill_cfg(stats, P.ex.cfg);
    return status;
}

// The whole ISA in one call: reconstruction, then the sets' solves and the
// assembly, sharing the field statistics (one host round trip fewer).
template <typename T>
int isa_all_impl(const sl_problem *p, const sl_ra_opts *ra, const sl_solve_opts *o, void *ws,
                 size_t ws_bytes, T *V, uint8_t *owner, uint8_t *member, uint8_t *label,
                 uint8_t *policy, T *V_sets, sl_stats *stats, hipStream_t s) {
    Timer tm;
    tm.mark(0, s);
    FieldStats fs{};
    DeferredRaStats dra;
    const int ra_status = reconstruct_impl<T>(p, ra, ws, ws_bytes, member, label, nullptr,
                                              nullptr, nullptr, s, &fs, &dra);
    if (ra_status < 0) return ra_status;
    tm.mark(1, s);
    const int status = isa_impl<T>(p, ra, member, o, ws, ws_bytes, V, owner, policy, V_sets,
                                   stats, s, &fs);
    if (status < 0) return status;
    tm.mark(2, s);
    // isa_impl ended with a stream synchronisation: the coarse states are in
    std::vector<SdState> hs;
    unsigned long long ncK = 0;
    Exec<double>::read_copied(dra.host, dra.n_sd, hs, &ncK);
    Exec<double>::remember(hs, dra.key);
    if (stats) {
        stats->ms_ra = tm.ms(0, 1);
        stats->ra_sweeps_max = sweeps_of(hs, 0, hs.size(), dra.launches);
        stats->ms_total = tm.ms(0, 2);
    }
    return status != SL_OK ? status : ra_status;
}

// ------------------------------------------------------------------- adjoint
template <typename T>
struct AdjPlan {
    T *lam = nullptr, *acc = nullptr, *ctrl = nullptr, *q = nullptr;
    AdjDesc<T> *ads = nullptr;
    SdState *st = nullptr;
    ExecCounters *cnt = nullptr;
    FieldStats *fs = nullptr;
    Exec<T> ex;                      // gather tile path
};

template <typename T>
void plan_adjoint(const sl_problem *p, int n_sets, Arena &a, AdjPlan<T> &P) {
    const size_t N = nodes_of(p);
    P.lam = a.take<T>((size_t)n_sets * N);
    P.acc = a.take<T>((size_t)n_sets * 2 * N);
    P.ctrl = a.take<T>((size_t)table_rows(p) * p->dim);
    P.q = p->drift ? a.take<T>(N * (size_t)p->dim) : nullptr;
    P.ads = a.take<AdjDesc<T>>(n_sets);
    P.st = a.take<SdState>(n_sets);
    P.cnt = a.take<ExecCounters>(1);
    P.fs = a.take<FieldStats>(1);
    const int tiles = p->dim == 2
                          ? ((p->n[0] + kAdjTX - 1) / kAdjTX) * ((p->n[1] + kAdjTY - 1) / kAdjTY)
                          : ((p->n[0] + kAdjTX3 - 1) / kAdjTX3) *
                                ((p->n[1] + kAdjTY3 - 1) / kAdjTY3) *
                                ((p->n[2] + kAdjTZ3 - 1) / kAdjTZ3);
    P.ex.reserve(a, n_sets, tiles * n_sets);
}

template <typename T>
int adjoint_impl(const sl_problem *p, const uint8_t *member, const uint8_t *owner,
                 const uint8_t *policy, const T *dLdV, T *dLdl, double tol, long max_iters,
                 int local_iters, void *ws, size_t ws_bytes, sl_stats *stats, hipStream_t s) {
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
                                   p->n_comp, P.fs, &fs, s, dLdV);
    if (rc) return rc;
    if ((rc = check_fields(fs))) return rc;
    if (tol < 0.0) {
        // relative to max |dL/dV|, rounded down to a power of two: the stop is at
        // least as strict as asked, and the tolerance (a launch argument, so part
        // of the captured chunk graphs' key) stays the same from one call to the
        // next while the gradient's scale moves within a factor of two, so a
        // training loop replays its adjoint graphs instead of capturing them anew
        const double t = -tol * bits_to_double(fs.g_absmax);
        int ex = 0;
        (void)std::frexp(t, &ex);
        tol = t > 0.0 && std::isfinite(t) ? std::ldexp(0.5, ex) : t;
    }
    double beta, w, emax;
    scheme_constants(p->lambda, p->h, p->disc, &beta, &w);
    std::vector<double> e;
    control_table(p, p->n, p->h, e, &emax);
    std::vector<T> et(e.size());
    for (size_t i = 0; i < e.size(); ++i) et[i] = (T)e[i];
    HIPCHK(hipMemcpyAsync(P.ctrl, et.data(), sizeof(T) * et.size(), hipMemcpyHostToDevice, s));
    if (p->drift) {
        double t[3];
        index_units(p, p->n, p->h, t);
        HIPCHK(launch_scale_drift<T>((const T *)p->drift, P.q, N, p->dim, t, s));
    }
    HIPCHK(hipMemsetAsync(P.lam, 0, sizeof(T) * (size_t)n_sets * N, s));
    std::vector<AdjDesc<T>> hd(n_sets);
    for (int i = 0; i < n_sets; ++i) {
        AdjDesc<T> &d = hd[i];
        d.lam = P.lam + (size_t)i * N;
        d.lam2 = d.lam;
        d.acc[0] = P.acc + (size_t)i * 2 * N;
        d.acc[1] = d.acc[0] + N;
        d.g = dLdV;
        d.owner = member ? owner : nullptr;
        d.policy = policy + (size_t)i * N;
        d.speed = (const T *)p->speed;
        d.drift = P.q;
        d.target = p->target;
        d.member = member;
        d.ctrl = P.ctrl;
        d.beta = (T)beta;
        for (int k = 0; k < 3; ++k) d.n[k] = k < p->dim ? p->n[k] : 1;
        d.m = p->m;
        d.bit = i;
        d.set = i;
        d.speed_axes = speed_comps(p) > 1;
        d.interp = p->interp;
    }
    const double smax = p->speed ? bits_to_double(fs.speed_max) : 1.0;
    const int H = halo_for(smax, emax, drift_reach(p, p->n, p->h, fs));
    // the gather tile path when the feet stay within its halo; otherwise the
    // Jacobi scatter over the whole grid
    const bool tiles = H <= adjoint_tiles_max_halo(p->dim);
    if (tiles && local_iters == 0)          // Jacobi: the second buffer is the acc area
        for (int i = 0; i < n_sets; ++i) hd[i].lam2 = hd[i].acc[0];
    // the scatter and the Jacobi tiles start from zero in the acc area too; the
    // block-asynchronous tiles iterate in place and never read it
    if (!tiles || local_iters == 0)
        HIPCHK(hipMemsetAsync(P.acc, 0, sizeof(T) * (size_t)n_sets * 2 * N, s));
    HIPCHK(hipMemcpyAsync(P.ads, hd.data(), sizeof(AdjDesc<T>) * n_sets, hipMemcpyHostToDevice, s));
    // rounding-level stop: atomics reorder the sums, so the state settles to
    // within a few ulps of its largest entry
    const double scale_rel = 16.0 * (sizeof(T) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16);
    int bps = (int)((N + kThreads - 1) / kThreads);
    bps = std::max(1, std::min(bps, 2048));
    int *active = pinned().active;
    if (!active) return SL_ERR_HIP;
    if (tiles) {
        // gather tiles on the sweep executor
        LaunchCfg cfg{};
        cfg.dim = p->dim;
        cfg.dtype = p->dtype;
        cfg.tile[0] = p->dim == 2 ? kAdjTX : kAdjTX3;
        cfg.tile[1] = p->dim == 2 ? kAdjTY : kAdjTY3;
        cfg.tile[2] = p->dim == 2 ? 1 : kAdjTZ3;
        cfg.halo = H;
        cfg.variant = -1;
        cfg.threads = kThreads;
        cfg.local_iters = local_iters;
        P.ex.cfg = cfg;
        P.ex.kind = 1;
        P.ex.scale_rel = scale_rel;
        P.ex.host_sds.clear();
        for (int i = 0; i < n_sets; ++i) {
            SdDesc<T> sd{};
            sd.V[0] = hd[i].lam;
            sd.V[1] = hd[i].lam2;
            sd.speed = (const T *)p->speed;
            sd.speed_axes = hd[i].speed_axes;
            sd.drift = P.q;
            sd.target = p->target;
            sd.member = member;
            sd.policy = const_cast<uint8_t *>(policy + (size_t)i * N);
            sd.ctrl = P.ctrl;
            sd.beta = (T)beta;
            for (int k = 0; k < 3; ++k) sd.n[k] = hd[i].n[k];
            sd.m = p->m;
            sd.m_inner = p->m;
            sd.bit = i;
            Exec<T>::tiles_of(cfg, sd.n, p->dim, sd.tiles);
            sd.halo = H;
            sd.interp = p->interp;
            sd.g = dLdV;
            sd.owner = member ? owner : nullptr;
            sd.set = i;
            P.ex.host_sds.push_back(sd);
        }
        tm.mark(1, s);
        if ((rc = P.ex.prepare(s))) return rc;
        long it = 0;
        const int status = P.ex.run(tol, max_iters, 0, 0, s, &it, 0);
        if (status < 0) return status;
        HIPCHK(launch_adjoint_combine<T>(P.ads, P.ex.st, n_sets, p->target, N, (T)w, dLdl, s));
        tm.mark(2, s);
        std::vector<SdState> hs2;
        unsigned long long nc = 0;
        if ((rc = P.ex.read_stats(s, hs2, &nc))) return rc;
        fill_stats(stats, hs2, nc, it);
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
    // scatter: its own states and counters
    std::vector<SdState> hs(n_sets);
    for (auto &x : hs) {
        x = SdState{};
        x.conv_at = -1;
    }
    HIPCHK(hipMemcpyAsync(P.st, hs.data(), sizeof(SdState) * n_sets, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(P.cnt, 0, sizeof(ExecCounters), s));
    tm.mark(1, s);
    auto enqueue = [&](hipStream_t q, int todo) -> hipError_t {
        for (int i = 0; i < todo; ++i) {
            const hipError_t e = launch_adjoint_iter<T>(p->dim, P.ads, P.st, n_sets, bps, P.cnt,
                                                        i, tol, scale_rel, q);
            if (e != hipSuccess) return e;
        }
        hipError_t e = launch_bookkeep(P.st, n_sets, todo, tol, P.cnt, 0, q, scale_rel, todo);
        if (e != hipSuccess) return e;
        return hipMemcpyAsync(active, &P.cnt->n_active, sizeof(int), hipMemcpyDeviceToHost, q);
    };
    ChunkLoop loop;
    long it = 0;
    int status = SL_NOT_CONVERGED;
    if ((rc = loop.run(enqueue, max_iters, 32, 32, s, 1, 0, &it, &status, active))) return rc;
    HIPCHK(launch_bookkeep(P.st, n_sets, 0, tol, P.cnt, 1, s, scale_rel));
    HIPCHK(launch_adjoint_combine<T>(P.ads, P.st, n_sets, p->target, N, (T)w, dLdl, s));
    tm.mark(2, s);
    ExecCounters c{};
    Readback rb(s, true);
    HIPCHK(rb.add(hs.data(), P.st, sizeof(SdState) * n_sets));
    HIPCHK(rb.add(&c, P.cnt, sizeof(c)));
    HIPCHK(rb.finish());
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

// ------------------------------------------------------------------- batched
constexpr int kChunk = 4096;     // elements per block of the segmented batched kernels

template <typename T>
struct BatchPlan {
    std::vector<ProbDesc<T>> hp;     // host image of the descriptors
    ProbDesc<T> *pd = nullptr;
    FieldStats *fs = nullptr;        // 2*np: fine stats, coarse presence
    int *blk_N = nullptr, *blk_NK = nullptr, *blk_aux = nullptr;
    std::vector<int> hblk_N, hblk_NK, hblk_aux;
    double *ctrlK = nullptr;         // np * m * dim
    T *ctrl = nullptr;
    Exec<double> exK;
    Exec<T> ex;
    int tot_sd = 0;
    // Kruzkov form, per problem (nullptr otherwise): coarse discount, fine discount
    // and fine cost term
    std::vector<double *> betaK;
    std::vector<T *> bn, wlk;
};

inline int blocks_for(size_t len) { return (int)((len + kChunk - 1) / kChunk); }

template <typename T>
int plan_batched(int np, const sl_problem *probs, const sl_ra_opts *ras, uint8_t *const *member,
                 uint8_t *const *label, uint8_t *const *owner, Arena &a, BatchPlan<T> &B) {
    const int dim = probs[0].dim;
    B.hp.assign(np, ProbDesc<T>{});
    B.hblk_N.assign(np + 1, 0);
    B.hblk_NK.assign(np + 1, 0);
    B.hblk_aux.assign(np + 1, 0);
    B.betaK.assign(np, nullptr);
    B.bn.assign(np, nullptr);
    B.wlk.assign(np, nullptr);
    int tilesK = 0, tiles = 0, nsd = 0;
    size_t ctrl_len = 0;
    for (int q = 0; q < np; ++q) {
        const sl_problem *p = &probs[q];
        ProbDesc<T> &d = B.hp[q];
        const CoarseGeom cg = coarse_geom(p, &ras[q]);
        d.dim = dim;
        for (int k = 0; k < 3; ++k) {
            d.n[k] = k < dim ? p->n[k] : 1;
            d.nK[k] = cg.nK[k];
        }
        d.n_comp = p->n_comp;
        d.N = nodes_of(p);
        d.NK = cg.NK;
        d.tK = a.take<int8_t>(cg.NK);
        d.cK = p->speed ? a.take<double>(cg.NK * (size_t)speed_comps(p)) : nullptr;
        d.wlK = p->cost ? a.take<double>(cg.NK) : nullptr;
        d.qK = p->drift ? a.take<double>(cg.NK * (size_t)dim) : nullptr;
        d.gK = p->g ? a.take<double>(cg.NK) : nullptr;
        d.Vaux = a.take<double>((size_t)p->n_comp * 2 * cg.NK);
        d.memberK = a.take<uint8_t>(cg.NK);
        d.labelK = a.take<uint8_t>(cg.NK);
        d.member = (member && member[q]) ? member[q] : a.take<uint8_t>(d.N);
        d.label = (label && label[q]) ? label[q] : a.take<uint8_t>(d.N);
        d.owner = owner ? owner[q] : nullptr;
        d.Vf = a.take<T>((size_t)p->n_comp * 2 * d.N);
        d.wl = p->cost ? a.take<T>(d.N) : nullptr;
        d.q = p->drift ? a.take<T>(d.N * (size_t)dim) : nullptr;
        if (uses_node_discount(p)) {
            B.betaK[q] = a.take<double>(cg.NK);
            B.bn[q] = a.take<T>(d.N);
            B.wlk[q] = a.take<T>(d.N);
        }
        int t[3];
        tilesK += max_tiles(dim, SL_F64, cg.nK) * p->n_comp;
        tiles += max_tiles(dim, p->dtype, p->n) * p->n_comp;
        d.sd_coarse0 = nsd;
        d.sd_fine0 = nsd;
        nsd += p->n_comp;
        ctrl_len += (size_t)table_rows(p) * dim;
        B.hblk_N[q + 1] = B.hblk_N[q] + blocks_for(d.N);
        B.hblk_NK[q + 1] = B.hblk_NK[q] + blocks_for(d.NK);
        B.hblk_aux[q + 1] = B.hblk_aux[q] + blocks_for((size_t)p->n_comp * d.NK);
    }
    B.tot_sd = nsd;
    B.pd = a.take<ProbDesc<T>>(np);
    B.fs = a.take<FieldStats>(2 * (size_t)np);
    B.blk_N = a.take<int>(np + 1);
    B.blk_NK = a.take<int>(np + 1);
    B.blk_aux = a.take<int>(np + 1);
    B.ctrlK = a.take<double>(ctrl_len);
    B.ctrl = a.take<T>(ctrl_len);
    B.exK.reserve(a, nsd, tilesK);
    B.ex.reserve(a, nsd, tiles);
    return SL_OK;
}

template <typename T>
int batched_impl(int np, const sl_problem *probs, const sl_ra_opts *ras, const sl_solve_opts *o,
                 void *ws, size_t ws_bytes, void *const *V, uint8_t *const *member,
                 uint8_t *const *label, uint8_t *const *owner, sl_stats *per_problem,
                 sl_stats *total, hipStream_t s) {
    Timer tm;
    tm.mark(0, s);
    const int dim = probs[0].dim;
    Arena a{(char *)ws, ws_bytes};
    BatchPlan<T> B;
    plan_batched<T>(np, probs, ras, member, label, owner, a, B);
    if (!a.fits()) return SL_ERR_WORKSPACE;
    // descriptors, statistics slots, block prefixes
    std::vector<FieldStats> fs_init(2 * (size_t)np);
    for (auto &f : fs_init) {
        f = FieldStats{};
        for (int i = 0; i < SL_MAX_COMP; ++i) f.first_node[i] = INT_MAX;
    }
    for (int q = 0; q < np; ++q) {
        const sl_problem *p = &probs[q];
        ProbDesc<T> &d = B.hp[q];
        d.target = p->target;
        d.speed = (const T *)p->speed;
        d.scomp = speed_comps(p);
        d.cost = (const T *)p->cost;
        d.drift = (const T *)p->drift;
        index_units(p, p->n, p->h, d.ut);
        index_units(p, d.nK, coarse_geom(p, &ras[q]).hK, d.utK);
        d.g = (const T *)p->g;
        d.V = (T *)V[q];
        d.fs = B.fs + q;
        d.fsK = B.fs + np + q;
        d.G = p->v_ghost;
        double beta, w, betaK, wK;
        scheme_constants(p->lambda, p->h, p->disc, &beta, &w);
        scheme_constants(p->lambda, coarse_geom(p, &ras[q]).hK, p->disc, &betaK, &wK);
        d.w = w;
        d.wK = uses_node_discount(p) ? 1.0 : wK;     // Kruzkov: wlK holds the samples of l
        double dxK = 0.0;
        for (int k = 0; k < dim; ++k)
            dxK = std::max(dxK, (p->hi[k] - p->lo[k]) / (double)(d.nK[k] - 1));
        d.delta = ras[q].delta_override > 0.0
                      ? ras[q].delta_override
                      : 2.0 * (ras[q].C * std::pow(dxK, ras[q].q) + ras[q].M * dxK);
    }
    HIPCHK(hipMemcpyAsync(B.pd, B.hp.data(), sizeof(ProbDesc<T>) * np, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B.fs, fs_init.data(), sizeof(FieldStats) * 2 * np, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B.blk_N, B.hblk_N.data(), sizeof(int) * (np + 1), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B.blk_NK, B.hblk_NK.data(), sizeof(int) * (np + 1), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B.blk_aux, B.hblk_aux.data(), sizeof(int) * (np + 1), hipMemcpyHostToDevice, s));
    // 1. input statistics of every problem (one launch, one sync)
    HIPCHK(launch_batched<T>(kBatchStats, B.pd, np, B.blk_N, B.hblk_N[np], kChunk, nullptr, nullptr, s));
    std::vector<FieldStats> fs(np);
    HIPCHK(hipMemcpyAsync(fs.data(), B.fs, sizeof(FieldStats) * np, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int HK = 1, H = 1;
    std::vector<int> Hq(np, 1), HKq(np, 1);      // per-problem halos (halo classes)
    std::vector<double> ctrlK, emaxs(np);
    std::vector<T> ctrl;
    for (int q = 0; q < np; ++q) {
        int rc = check_fields(fs[q]);
        if (rc) return rc;
        const sl_problem *p = &probs[q];
        std::vector<double> e, eK;
        double emax, emaxK;
        control_table(p, p->n, p->h, e, &emax);
        control_table(p, B.hp[q].nK, coarse_geom(p, &ras[q]).hK, eK, &emaxK);
        const double smax = p->speed ? bits_to_double(fs[q].speed_max) : 1.0;
        const double hK = coarse_geom(p, &ras[q]).hK;
        Hq[q] = halo_for(smax, emax, drift_reach(p, p->n, p->h, fs[q]));
        HKq[q] = halo_for(smax, emaxK, drift_reach(p, B.hp[q].nK, hK, fs[q]));
        H = std::max(H, Hq[q]);
        HK = std::max(HK, HKq[q]);
        for (double x : e) ctrl.push_back((T)x);
        for (double x : eK) ctrlK.push_back(x);
    }
    if (H > max_halo(dim) || HK > max_halo(dim)) return SL_ERR_UNSUPPORTED;
    HIPCHK(hipMemcpyAsync(B.ctrlK, ctrlK.data(), sizeof(double) * ctrlK.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(B.ctrl, ctrl.data(), sizeof(T) * ctrl.size(), hipMemcpyHostToDevice, s));
    // 2. coarse data, placement of missing components, auxiliary initial values
    HIPCHK(launch_batched<T>(kBatchCoarsePrep, B.pd, np, B.blk_NK, B.hblk_NK[np], kChunk, nullptr, nullptr, s));
    HIPCHK(launch_batched<T>(kBatchPlace, B.pd, np, nullptr, 1, kChunk, nullptr, nullptr, s));
    // Kruzkov form: per-node discount and cost term on the host, coarse and fine
    for (int q = 0; q < np; ++q) {
        const sl_problem *p = &probs[q];
        if (!uses_node_discount(p)) continue;
        const ProbDesc<T> &d = B.hp[q];
        int rk = kruzkov_fields<double>(d.wlK, d.NK, coarse_geom(p, &ras[q]).hK, B.betaK[q],
                                        d.wlK, s);
        if (!rk) rk = kruzkov_fields<T>((const T *)p->cost, d.N, p->h, B.bn[q], B.wlk[q], s);
        if (rk) return rk;
    }
    auto reinitK = [&](hipStream_t q) -> hipError_t {
        return launch_batched<T>(kBatchInitAux, B.pd, np, B.blk_aux, B.hblk_aux[np], kChunk,
                                 nullptr, nullptr, q);
    };
    // 3. RA step 1 for every (problem, component): one launch per sweep
    B.exK.cfg = make_cfg(dim, SL_F64, HK, default_variant(dim, SL_F64));
    B.exK.cfg.interp = probs[0].interp;
    B.exK.cfg.local_iters = ras[0].local_iters;
    size_t coff = 0;
    for (int q = 0; q < np; ++q) {
        const sl_problem *p = &probs[q];
        const ProbDesc<T> &d = B.hp[q];
        double betaK, wK;
        scheme_constants(p->lambda, coarse_geom(p, &ras[q]).hK, p->disc, &betaK, &wK);
        for (int i = 0; i < p->n_comp; ++i) {
            SdDesc<double> sd{};
            sd.V[0] = d.Vaux + (size_t)i * 2 * d.NK;
            sd.V[1] = sd.V[0] + d.NK;
            sd.speed = d.cK;
            sd.speed_axes = d.scomp > 1;
            sd.drift = d.qK;
            sd.wl = d.wlK;
            sd.beta_n = B.betaK[q];
            sd.target = d.tK;
            sd.ctrl = B.ctrlK + coff;
            sd.wl_const = wK;
            sd.beta = betaK;
            sd.G = p->v_ghost;
            for (int k = 0; k < 3; ++k) sd.n[k] = d.nK[k];
            sd.m = table_rows(p);
            sd.m_inner = p->m;
            sd.bit = i;
            Exec<double>::tiles_of(B.exK.cfg, d.nK, dim, sd.tiles);
            sd.halo = HKq[q];
            B.exK.host_sds.push_back(sd);
        }
        coff += (size_t)table_rows(p) * dim;
    }
    int rc = SL_OK;
    long SK = 0;
    int stK = B.exK.solve_tuned(ras[0].autotune, reinitK, ras[0].tol, ras[0].max_sweeps, 0, 0,
                                s, &SK, 0);
    if (stK < 0) return stK;
    // 4. RA steps 2-3, projection, fine initial values
    HIPCHK(launch_batched<T>(kBatchCombine, B.pd, np, B.blk_NK, B.hblk_NK[np], kChunk, B.exK.sds, B.exK.st, s));
    auto reinit = [&](hipStream_t q) -> hipError_t {
        return launch_batched<T>(kBatchProjectInit, B.pd, np, B.blk_N, B.hblk_N[np], kChunk,
                                 nullptr, nullptr, q);
    };
    tm.mark(1, s);
    // 5. ISA step 3 for every (problem, set): one launch per sweep
    B.ex.cfg = make_cfg(dim, probs[0].dtype, H, default_variant(dim, probs[0].dtype));
    B.ex.cfg.interp = probs[0].interp;
    B.ex.cfg.local_iters = o->local_iters;
    coff = 0;
    for (int q = 0; q < np; ++q) {
        const sl_problem *p = &probs[q];
        const ProbDesc<T> &d = B.hp[q];
        double beta, w;
        scheme_constants(p->lambda, p->h, p->disc, &beta, &w);
        for (int i = 0; i < p->n_comp; ++i) {
            SdDesc<T> sd{};
            sd.V[0] = d.Vf + (size_t)i * 2 * d.N;
            sd.V[1] = sd.V[0] + d.N;
            sd.speed = (const T *)p->speed;
            sd.speed_axes = d.scomp > 1;
            sd.drift = d.q;
            sd.wl = B.wlk[q] ? B.wlk[q] : d.wl;
            sd.beta_n = B.bn[q];
            sd.target = p->target;
            sd.member = d.member;
            sd.ctrl = B.ctrl + coff;
            sd.wl_const = (T)w;
            sd.beta = (T)beta;
            sd.G = (T)p->v_ghost;
            for (int k = 0; k < 3; ++k) sd.n[k] = d.n[k];
            sd.m = table_rows(p);
            sd.m_inner = p->m;
            sd.bit = i;
            Exec<T>::tiles_of(B.ex.cfg, d.n, dim, sd.tiles);
            sd.halo = Hq[q];
            B.ex.host_sds.push_back(sd);
        }
        coff += (size_t)table_rows(p) * dim;
    }
    long S = 0;
    const int status = B.ex.solve_tuned(o->autotune, reinit, o->tol, o->max_sweeps,
                                        o->check_every, 0, s, &S, o->profile);
    if (status < 0) return status;
    tm.mark(2, s);
    // 6. ISA step 4 for every problem
    HIPCHK(launch_batched<T>(kBatchAssemble, B.pd, np, B.blk_N, B.hblk_N[np], kChunk, B.ex.sds, B.ex.st, s));
    tm.mark(3, s);
    std::vector<SdState> hsK, hs;
    unsigned long long ncK = 0, nc = 0;
    {
        Readback rb(s, true);
        ExecCounters cK{}, c{};
        HIPCHK(B.exK.queue_stats(rb, hsK, cK));
        HIPCHK(B.ex.queue_stats(rb, hs, c));
        HIPCHK(rb.finish());
        B.exK.take_stats(hsK, cK, &ncK);
        B.ex.take_stats(hs, c, &nc);
    }
    if (per_problem) {
        for (int q = 0; q < np; ++q) {
            const ProbDesc<T> &d = B.hp[q];
            std::vector<SdState> sub(hs.begin() + d.sd_fine0, hs.begin() + d.sd_fine0 + d.n_comp);
            fill_stats(&per_problem[q], sub, 0, S);
            per_problem[q].ra_sweeps_max =
                sweeps_of(hsK, d.sd_coarse0, d.sd_coarse0 + d.n_comp, SK);
            per_problem[q].node_control_updates = 0.0;
            per_problem[q].ms_ra = per_problem[q].ms_fine = per_problem[q].ms_total = 0.0;
            per_problem[q].set_fraction_max = 0.0;
            per_problem[q].ms_sweeps = 0.0;
            per_problem[q].sweep_launches = 0;
        }
    }
    if (total) {
        fill_stats(total, hs, nc, S);
        total->ra_sweeps_max = sweeps_of(hsK, 0, hsK.size(), SK);
        total->ms_ra = tm.ms(0, 1);
        total->ms_fine = tm.ms(1, 2);
        total->ms_total = tm.ms(0, 3);
        total->set_fraction_max = 0.0;
        total->ms_sweeps = B.ex.ms_sweeps;
        total->sweep_launches = B.ex.sweep_launches;
    }
    fill_cfg(total, B.ex.cfg);
    return status == SL_OK && stK == SL_OK ? SL_OK : SL_NOT_CONVERGED;
}

int validate_batch(int np, const sl_problem *probs, const sl_ra_opts *ras) {
    if (np < 1 || !probs || !ras) return SL_ERR_INVALID_ARG;
    for (int q = 0; q < np; ++q) {
        int rc = validate(&probs[q]);
        if (rc) return rc;
        if ((rc = validate_ra(&probs[q], &ras[q]))) return rc;
        if (probs[q].dim != probs[0].dim || probs[q].dtype != probs[0].dtype)
            return SL_ERR_UNSUPPORTED;
        if (probs[q].interp != probs[0].interp) return SL_ERR_UNSUPPORTED;
    }
    return SL_OK;
}

// ------------------------------------------------------- no-allocation scratch
// Device address of `scratch` (declared at file scope above) on the current
// device, taken once per device with that device current.
constexpr int kMaxScratchDevices = 64;

int noalloc_scratch(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices)
        return SL_ERR_HIP;
    static std::mutex mu;
    static void *ptr[kMaxScratchDevices] = {};
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return SL_ERR_HIP;
        ptr[dev] = q;
    }
    *out = ptr[dev];
    return SL_OK;
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
    case SL_ERR_SCRATCH:
        return "problem needs more than the static scratch of the no-allocation entry point";
    default: return "unknown status";
    }
}

int sl_abi_version(void) { return SLHJB_ABI_VERSION; }

int sl_tune_candidates(int dim, int dtype) {
    if ((dim != 2 && dim != 3) || (dtype != SL_F32 && dtype != SL_F64)) return 0;
    return (int)tune_candidates(dim, dtype, 1).size();
}

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
    if (is_game(p) && o->want_policy && policy) return SL_ERR_UNSUPPORTED;
    if (o->want_policy && policy && p->m > SL_MAX_POLICY_CONTROLS) return SL_ERR_UNSUPPORTED;
    if (ws_bytes < sl_solve_workspace_size(p)) return SL_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == SL_F32)
        return solve_global<float>(p, o, ws, ws_bytes, (float *)V, policy, stats, s);
    return solve_global<double>(p, o, ws, ws_bytes, (double *)V, policy, stats, s);
}

int sl_solve_noalloc(const sl_problem *p, const sl_solve_opts *o, void *V, uint8_t *policy,
                     sl_stats *stats, void *stream) {
    int rc = validate(p);
    if (rc) return rc;
    if ((rc = validate_solve_opts(o))) return rc;
    if (!V) return SL_ERR_INVALID_ARG;
    if (o->autotune > 0 || o->profile) return SL_ERR_INVALID_ARG;   // both need HIP events
    if (is_game(p) && o->want_policy && policy) return SL_ERR_UNSUPPORTED;
    if (o->want_policy && policy && p->m > SL_MAX_POLICY_CONTROLS) return SL_ERR_UNSUPPORTED;
    if (sl_solve_workspace_size(p) > SL_NOALLOC_SCRATCH_BYTES) return SL_ERR_SCRATCH;
    void *ws = nullptr;
    if ((rc = noalloc_scratch(&ws))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == SL_F32)
        return solve_global<float>(p, o, ws, SL_NOALLOC_SCRATCH_BYTES, (float *)V, policy, stats,
                                   s, true);
    return solve_global<double>(p, o, ws, SL_NOALLOC_SCRATCH_BYTES, (double *)V, policy, stats,
                                s, true);
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

size_t sl_refine_workspace_size(const sl_problem *p, const sl_ra_opts *ra, int max_comp) {
    if (validate(p) != SL_OK || validate_ra(p, ra) != SL_OK) return 0;
    if (max_comp < p->n_comp || max_comp > SL_MAX_COMP) return 0;
    sl_problem q = *p;
    q.n_comp = max_comp;
    const size_t isa = sl_isa_workspace_size(&q, ra);
    if (!isa) return 0;
    const size_t N = nodes_of(p);
    return ((isa + 255) & ~size_t(255)) + 2 * ((N + 255) & ~size_t(255)) + 256;
}

int sl_refine_split(const sl_problem *p, const sl_ra_opts *ra, int max_comp, double frac_goal,
                    void *ws, size_t ws_bytes, int8_t *target_out, int *n_comp_out,
                    double *frac_max, sl_stats *stats, void *stream) {
    int rc = validate(p);
    if (rc) return rc;
    if ((rc = validate_ra(p, ra))) return rc;
    if (max_comp < p->n_comp || max_comp > SL_MAX_COMP) return SL_ERR_INVALID_ARG;
    if (!(frac_goal >= 0.0 && frac_goal <= 1.0)) return SL_ERR_INVALID_ARG;
    if (!ws || !target_out || !n_comp_out) return SL_ERR_INVALID_ARG;
    if (ws_bytes < sl_refine_workspace_size(p, ra, max_comp)) return SL_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const size_t N = nodes_of(p);
    sl_problem q = *p;
    q.n_comp = max_comp;
    const size_t isa = (sl_isa_workspace_size(&q, ra) + 255) & ~size_t(255);
    uint8_t *member = (uint8_t *)ws + isa;
    uint8_t *label = member + ((N + 255) & ~size_t(255));
    // the target ids live on the host between reconstructions (the split is a
    // handful of integer decisions); every reconstruction runs on the device
    std::vector<int8_t> ht(N);
    std::vector<uint8_t> hm(N);
    HIPCHK(hipMemcpyAsync(ht.data(), p->target, N, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int nc = p->n_comp, steps = 0, last = SL_OK;
    long ra_sweeps = 0;
    Timer tm;
    tm.mark(0, s);
    for (;;) {
        HIPCHK(hipMemcpyAsync(target_out, ht.data(), N, hipMemcpyHostToDevice, s));
        q = *p;
        q.target = target_out;
        q.n_comp = nc;
        sl_stats st{};
        last = p->dtype == SL_F32
                   ? reconstruct_impl<float>(&q, ra, ws, isa, member, label, nullptr, nullptr, &st, s)
                   : reconstruct_impl<double>(&q, ra, ws, isa, member, label, nullptr, nullptr, &st, s);
        if (last < 0) return last;
        ra_sweeps = std::max(ra_sweeps, st.ra_sweeps_max);
        HIPCHK(hipMemcpyAsync(hm.data(), member, N, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        long counts[SL_MAX_COMP] = {0}, sizes[SL_MAX_COMP] = {0};
        for (size_t j = 0; j < N; ++j) {
            for (int i = 0; i < nc; ++i) counts[i] += (hm[j] >> i) & 1;
            if (ht[j] >= 0 && ht[j] < nc) ++sizes[ht[j]];
        }
        long cmax = 0;
        for (int i = 0; i < nc; ++i) cmax = std::max(cmax, counts[i]);
        const double fmax = (double)cmax / (double)N;
        if (frac_max) frac_max[steps] = fmax;
        ++steps;
        if (nc >= max_comp || fmax <= frac_goal) break;
        // the largest set (lowest index on ties) whose component can be halved
        int pick = -1;
        for (int i = 0; i < nc; ++i)
            if (sizes[i] >= 2 && (pick < 0 || counts[i] > counts[pick])) pick = i;
        if (pick < 0) break;
        // halve it along the axis of largest index extent (lowest axis on ties):
        // nodes ordered by (index on that axis, flat index), the upper half relabelled
        int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
        std::vector<std::pair<long long, long long>> nodes;
        for (size_t j = 0; j < N; ++j) {
            if (ht[j] != pick) continue;
            long long r = (long long)j;
            for (int d = 0; d < p->dim; ++d) {
                const int id = (int)(r % p->n[d]);
                r /= p->n[d];
                lo[d] = std::min(lo[d], id);
                hi[d] = std::max(hi[d], id);
            }
        }
        int axis = 0;
        for (int d = 1; d < p->dim; ++d)
            if (hi[d] - lo[d] > hi[axis] - lo[axis]) axis = d;
        long long stride = 1;
        for (int d = 0; d < axis; ++d) stride *= p->n[d];
        for (size_t j = 0; j < N; ++j)
            if (ht[j] == pick) nodes.emplace_back(((long long)j / stride) % p->n[axis], (long long)j);
        std::sort(nodes.begin(), nodes.end());
        const size_t keep = nodes.size() - nodes.size() / 2;
        for (size_t k = keep; k < nodes.size(); ++k) ht[(size_t)nodes[k].second] = (int8_t)nc;
        ++nc;
    }
    tm.mark(1, s);
    *n_comp_out = nc;
    if (stats) {
        *stats = sl_stats{};
        stats->ms_ra = tm.ms(0, 1);
        stats->ms_total = stats->ms_ra;
        stats->ra_sweeps_max = ra_sweeps;
        stats->n_subdomains = nc;
        stats->sweeps_max = steps;
        stats->set_fraction_max = frac_max ? frac_max[steps - 1] : 0.0;
    }
    return last;
}

int sl_solve_isa(const sl_problem *p, const sl_ra_opts *ra, const uint8_t *member,
                 const sl_solve_opts *o, void *ws, size_t ws_bytes, void *V, uint8_t *owner,
                 uint8_t *policy, void *V_sets, sl_stats *stats, void *stream) {
    int rc = validate(p);
    if (rc) return rc;
    if ((rc = validate_ra(p, ra))) return rc;
    if ((rc = validate_solve_opts(o))) return rc;
    if (!member || !V || !ws) return SL_ERR_INVALID_ARG;
    if (is_game(p) && o->want_policy && policy) return SL_ERR_UNSUPPORTED;
    if (o->want_policy && policy && p->m > SL_MAX_POLICY_CONTROLS) return SL_ERR_UNSUPPORTED;
    if (ws_bytes < sl_isa_workspace_size(p, ra)) return SL_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == SL_F32)
        return isa_impl<float>(p, ra, member, o, ws, ws_bytes, (float *)V, owner, policy,
                               (float *)V_sets, stats, s);
    return isa_impl<double>(p, ra, member, o, ws, ws_bytes, (double *)V, owner, policy,
                            (double *)V_sets, stats, s);
}

int sl_isa(const sl_problem *p, const sl_ra_opts *ra, const sl_solve_opts *o, void *ws,
           size_t ws_bytes, void *V, uint8_t *owner, uint8_t *member, uint8_t *label,
           uint8_t *policy, void *V_sets, sl_stats *stats, void *stream) {
    int rc = validate(p);
    if (rc) return rc;
    if ((rc = validate_ra(p, ra))) return rc;
    if ((rc = validate_solve_opts(o))) return rc;
    if (!member || !label || !V || !ws) return SL_ERR_INVALID_ARG;
    if (is_game(p) && o->want_policy && policy) return SL_ERR_UNSUPPORTED;
    if (o->want_policy && policy && p->m > SL_MAX_POLICY_CONTROLS) return SL_ERR_UNSUPPORTED;
    if (ws_bytes < sl_isa_workspace_size(p, ra)) return SL_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == SL_F32)
        return isa_all_impl<float>(p, ra, o, ws, ws_bytes, (float *)V, owner, member, label,
                                   policy, (float *)V_sets, stats, s);
    return isa_all_impl<double>(p, ra, o, ws, ws_bytes, (double *)V, owner, member, label,
                                policy, (double *)V_sets, stats, s);
}

size_t sl_batched_workspace_size(int nprob, const sl_problem *probs, const sl_ra_opts *ras) {
    if (validate_batch(nprob, probs, ras) != SL_OK) return 0;
    Arena a{nullptr, 0};
    if (probs[0].dtype == SL_F32) {
        BatchPlan<float> B;
        plan_batched<float>(nprob, probs, ras, nullptr, nullptr, nullptr, a, B);
    } else {
        BatchPlan<double> B;
        plan_batched<double>(nprob, probs, ras, nullptr, nullptr, nullptr, a, B);
    }
    return a.off + 256;
}

int sl_solve_batched(int nprob, const sl_problem *probs, const sl_ra_opts *ras,
                     const sl_solve_opts *o, void *ws, size_t ws_bytes, void *const *V,
                     uint8_t *const *member, uint8_t *const *label, uint8_t *const *owner,
                     sl_stats *per_problem, sl_stats *total, void *stream) {
    int rc = validate_batch(nprob, probs, ras);
    if (rc) return rc;
    if ((rc = validate_solve_opts(o))) return rc;
    if (!V || !ws) return SL_ERR_INVALID_ARG;
    for (int q = 0; q < nprob; ++q)
        if (!V[q]) return SL_ERR_INVALID_ARG;
    // the size query lays out internal member/label arrays for every problem,
    // so it bounds the need whatever the caller passes
    if (ws_bytes < sl_batched_workspace_size(nprob, probs, ras)) return SL_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (probs[0].dtype == SL_F32)
        return batched_impl<float>(nprob, probs, ras, o, ws, ws_bytes, V, member, label, owner,
                                   per_problem, total, s);
    return batched_impl<double>(nprob, probs, ras, o, ws, ws_bytes, V, member, label, owner,
                                per_problem, total, s);
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
               int local_iters, void *ws, size_t ws_bytes, sl_stats *stats, void *stream) {
    int rc = validate(p);
    if (rc) return rc;
    if (!policy || !dLdV || !dLdl || !ws) return SL_ERR_INVALID_ARG;
    if (!std::isfinite(tol) || max_iters < 1) return SL_ERR_INVALID_ARG;
    if (local_iters < 0 || local_iters > 1024) return SL_ERR_INVALID_ARG;
    if (is_game(p) || p->disc == SL_DISC_KRUZKOV) return SL_ERR_UNSUPPORTED;
    if (p->m > SL_MAX_POLICY_CONTROLS) return SL_ERR_UNSUPPORTED;
    const int n_sets = member ? p->n_comp : 1;
    if (ws_bytes < sl_adjoint_workspace_size(p, n_sets)) return SL_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (p->dtype == SL_F32)
        return adjoint_impl<float>(p, member, owner, policy, (const float *)dLdV, (float *)dLdl,
                                   tol, max_iters, local_iters, ws, ws_bytes, stats, s);
    return adjoint_impl<double>(p, member, owner, policy, (const double *)dLdV, (double *)dLdl,
                                tol, max_iters, local_iters, ws, ws_bytes, stats, s);
}

}  // extern "C"
