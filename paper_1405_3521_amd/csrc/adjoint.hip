// Adjoint of the policy-frozen SL scheme: the gradient of a loss on V with
// respect to the running cost l.
//
// With the argmin controls frozen, on the free nodes of a set the fixed point
// satisfies V = beta P V + w l + (constants from target and ghost corners), so
//     dL/dl = w * lambda,   lambda = g + beta P^T lambda,   g = dL/dV
// (only the owner set of a node receives its g when the value is the minimum
// over sets).  One fused launch per Jacobi iteration:
//   lambda_k(j) = g(j) + acc_k(j)                     (acc_k(j) reset to 0)
//   acc_{k+1}(c) += beta * w_c(j) * lambda_k(j)   for the free member corners c
//                                                 of node j's foot (float atomics)
// The FP64 residual max|lambda_k - lambda_{k-1}| per set drives the same device
// bookkeeping as the forward sweeps.  The scatter is bound by L2 atomics and
// HBM, not by ALU: ~4 (8 in 3D) atomics and ~20 bytes per node and iteration.
#include "device_common.h"

namespace slhjb {
namespace {

template <typename T, int DIM>
__global__ __launch_bounds__(kThreads) void k_adjoint(const AdjDesc<T> *__restrict__ ads,
                                                      SdState *__restrict__ st, int n_sets,
                                                      int blocks_per_set,
                                                      ExecCounters *__restrict__ cnt,
                                                      int iter_rel, double tol, double scale_rel) {
    const int iter = cnt->sweep_base + iter_rel;
    if (blockIdx.x == 0) bookkeep_block(st, n_sets, iter, tol, cnt, 0, scale_rel);
    const int set = blockIdx.x / blocks_per_set;
    const int b = blockIdx.x - set * blocks_per_set;
    SdState *sst = st + set;
    if (sd_skip(sst, iter, tol, scale_rel)) return;
    const AdjDesc<T> &d = ads[set];
    const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
    const size_t N = (size_t)n0 * n1 * n2;
    T *__restrict__ lam = d.lam;
    T *__restrict__ acc_in = d.acc[iter & 1];
    T *__restrict__ acc_out = d.acc[(iter + 1) & 1];
    const uint8_t *__restrict__ mem = d.member;
    const int bit = d.bit;
    const T beta = d.beta;
    double rmax = 0.0, lmax = 0.0;
    unsigned nact = 0;
    for (size_t j = (size_t)b * kThreads + threadIdx.x; j < N;
         j += (size_t)blocks_per_set * kThreads) {
        if (d.target[j] >= 0) continue;
        if (mem && !((mem[j] >> bit) & 1)) continue;
        const T gj = (!d.owner || d.owner[j] == d.set) ? d.g[j] : T(0);
        const T ln = gj + acc_in[j];
        acc_in[j] = T(0);
        const T lo = lam[j];
        lam[j] = ln;
        const double dv = __builtin_fabs((double)ln - (double)lo);
        rmax = dv > rmax ? dv : rmax;
        const double al = __builtin_fabs((double)ln);
        lmax = al > lmax ? al : lmax;
        ++nact;
        const int k = d.policy[j];
        if (ln == T(0) || k >= d.m) continue;
        int ij[3], p[3];
        T tau[3];
        ij[0] = (int)(j % n0);
        ij[1] = (int)((j / n0) % n1);
        ij[2] = (int)(j / ((size_t)n0 * n1));
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            // foot offset e c + q in index units, the forward sweep's order
            const T c = !d.speed ? T(1) : (d.speed_axes ? d.speed[DIM * j + a] : d.speed[j]);
            const T q = d.drift ? d.drift[DIM * j + a] : T(0);
            const T disp = d.ctrl[DIM * k + a] * c + q;
            const T f = __builtin_floor(disp);
            tau[a] = disp - f;
            p[a] = ij[a] + (int)f;
        }
        const T bl = beta * ln;
        if (d.interp == SL_INTERP_P1) {
            // P1: the vertices of the foot's Kuhn simplex (lower corner, then one
            // step along each axis in the order of decreasing fraction, equal
            // fractions lower axis first) with their barycentric weights
            int ax[3] = {0, 1, 2};
#pragma unroll
            for (int a = 1; a < DIM; ++a)
                for (int b = a; b > 0 && tau[ax[b - 1]] < tau[ax[b]]; --b) {
                    const int t = ax[b - 1];
                    ax[b - 1] = ax[b];
                    ax[b] = t;
                }
            int v[3] = {p[0], DIM > 1 ? p[1] : 0, DIM > 2 ? p[2] : 0};
#pragma unroll
            for (int s = 0; s <= DIM; ++s) {
                if (s > 0) v[ax[s - 1]] += 1;
                const T w = s == 0 ? T(1) - tau[ax[0]]
                                   : (s < DIM ? tau[ax[s - 1]] - tau[ax[s]] : tau[ax[DIM - 1]]);
                bool in = true;
                size_t idx = 0, stride = 1;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const int na = a == 0 ? n0 : (a == 1 ? n1 : n2);
                    in = in && v[a] >= 0 && v[a] < na;
                    idx += (size_t)(v[a] < 0 ? 0 : v[a]) * stride;
                    stride *= (size_t)na;
                }
                if (!in || w == T(0)) continue;
                if (d.target[idx] >= 0) continue;
                if (mem && !((mem[idx] >> bit) & 1)) continue;
                atomicAdd(&acc_out[idx], bl * w);
            }
            continue;
        }
#pragma unroll
        for (int q = 0; q < (1 << DIM); ++q) {
            T w = T(1);
            bool in = true;
            size_t idx = 0, stride = 1;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const int bitq = (q >> a) & 1;
                w = w * (bitq ? tau[a] : T(1) - tau[a]);
                const int pa = p[a] + bitq;
                const int na = a == 0 ? n0 : (a == 1 ? n1 : n2);
                in = in && pa >= 0 && pa < na;
                idx += (size_t)(pa < 0 ? 0 : pa) * stride;
                stride *= (size_t)na;
            }
            if (!in || w == T(0)) continue;
            if (d.target[idx] >= 0) continue;
            if (mem && !((mem[idx] >> bit) & 1)) continue;
            atomicAdd(&acc_out[idx], bl * w);
        }
    }
    block_max_to(rmax, &sst->res[iter % 3]);
    block_max_to(lmax, &sst->scale[iter % 3]);
    block_sum_to(nact, &cnt->nc_updates);
}

template <typename T>
__device__ __forceinline__ T floor_(T x);
template <>
__device__ __forceinline__ float floor_<float>(float x) { return __builtin_floorf(x); }
template <>
__device__ __forceinline__ double floor_<double>(double x) { return __builtin_floor(x); }

// Tile shapes of the gather adjoint and the most in-stencil entries a tile node
// keeps on chip (a node with more is summed by rescanning its neighbourhood).
template <int DIM>
struct AdjTile;
template <>
struct AdjTile<2> {
    static constexpr int X = kAdjTX, Y = kAdjTY, Z = 1, K = 12;
};
template <>
struct AdjTile<3> {
    static constexpr int X = kAdjTX3, Y = kAdjTY3, Z = kAdjTZ3, K = 24;
};

// The frozen foot of free member node j (region coordinates l of the node): the
// lower corner of its cell in region coordinates and the fractions, exactly as
// the forward scheme places it (u_a = i_a + (e_a c_a + q_a), split by floor).
template <typename T, int DIM>
__device__ __forceinline__ bool adj_foot(const SdDesc<T> &d, size_t j, const int *l, int *p,
                                         T *tau) {
    const int k = d.policy[j];
    if (k >= d.m) return false;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const T c = !d.speed ? T(1) : (d.speed_axes ? d.speed[(size_t)DIM * j + a] : d.speed[j]);
        const T q = d.drift ? d.drift[(size_t)DIM * j + a] : T(0);
        const T disp = d.ctrl[DIM * k + a] * c + q;
        const T f = floor_(disp);
        tau[a] = disp - f;
        p[a] = l[a] + (int)f;
    }
    return true;
}

// The interpolation stencil of a foot: fn(vertex region coordinates, weight) for
// every vertex with a nonzero weight.  Q1: the 2^DIM cell corners with product
// weights in axis order.  P1: the vertices of the foot's Kuhn simplex (lower
// corner, then one step along each axis in the order of decreasing fraction,
// equal fractions lower axis first) with their barycentric weights.
template <typename T, int DIM, class F>
__device__ __forceinline__ void adj_stencil(int interp, const int *p, const T *tau, F fn) {
    if (interp == SL_INTERP_P1) {
        int ax[3] = {0, 1, 2};
#pragma unroll
        for (int a = 1; a < DIM; ++a)
            for (int b = a; b > 0 && tau[ax[b - 1]] < tau[ax[b]]; --b) {
                const int t = ax[b - 1];
                ax[b - 1] = ax[b];
                ax[b] = t;
            }
        int v[3] = {p[0], DIM > 1 ? p[1] : 0, DIM > 2 ? p[2] : 0};
#pragma unroll
        for (int s = 0; s <= DIM; ++s) {
            if (s > 0) v[ax[s - 1]] += 1;
            const T w = s == 0 ? T(1) - tau[ax[0]]
                               : (s < DIM ? tau[ax[s - 1]] - tau[ax[s]] : tau[ax[DIM - 1]]);
            if (w != T(0)) fn(v, w);
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < (1 << DIM); ++q) {
        T w = T(1);
        int v[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int bq = (q >> a) & 1;
            w = w * (bq ? tau[a] : T(1) - tau[a]);
            v[a] = p[a] + bq;
        }
        if (w != T(0)) fn(v, w);
    }
}

// Gather (pull) adjoint over tiles, 2D and 3D, no atomics on the adjoint state.
//
// lambda(c) = g(c) + beta * sum over the free member nodes j whose frozen foot
// has c in its stencil of w_c(j) lambda(j): the transposed stencil.  For each
// work item the tile plus an H-node halo (every node whose foot can reach the
// tile) is staged in LDS; every region node pushes (j, w_c(j)) into the entry
// list of each tile node c of its stencil (LDS counters give the slots), and
// each list is then sorted by source, so the sum runs in a fixed order and the
// result does not depend on the push order.  A node with more than K entries is
// summed by rescanning its neighbourhood in the same source order.  Then up to
// local_iters times: every tile node gathers from its list (halo values as
// staged), the new values are written after a barrier, and the tile stops when
// no node changed by more than tol + scale_rel |lambda|.
//
// local_iters = 0: one evaluation per launch from buffer it & 1 into the other
// buffer (Jacobi); a tile is revisited when a node of its neighbourhood changed
// at all, so skipped tiles already hold their values in both buffers and the
// iterates are those of the plain Jacobi iteration, reproducible bit for bit.
// local_iters > 0: block-asynchronous in place (both buffers are one array): a
// tile sees its neighbours' latest values when it stages them, so the order of
// updates, and the result at rounding level, depends on scheduling.  The
// iteration has nonnegative coefficients and spectral radius <= beta < 1, so
// every order converges to the same solution.
template <typename T, int DIM, int H>
__global__ __launch_bounds__(kThreads) void k_adjoint_pull(
    const SdDesc<T> *__restrict__ sds, SdState *__restrict__ st, int n_sd,
    const WorkItem *__restrict__ items, WorkItem *__restrict__ lists,
    ExecCounters *__restrict__ cnt, int iter_rel, double tol, double scale_rel,
    int *__restrict__ stamp, int stamp_stride, int mode, int cls, int do_bookkeep,
    int local_iters) {
    using TT = AdjTile<DIM>;
    constexpr int TX = TT::X, TY = TT::Y, TZ = TT::Z, K = TT::K;
    constexpr int HZ = DIM == 3 ? H : 0;
    constexpr int LW = TX + 2 * H, LH = TY + 2 * H, LD = TZ + 2 * HZ;
    constexpr int NR = LW * LH * LD, NT = TX * TY * TZ;
    constexpr int NPT = NT / kThreads;
    constexpr int RX = (H + TX - 1) / TX, RY = (H + TY - 1) / TY;
    constexpr int RZ = DIM == 3 ? (H + TZ - 1) / TZ : 0;
    static_assert(NT % kThreads == 0 && NPT >= 1, "tile/thread mismatch");
    static_assert(NR < 32768, "region offsets must fit in 16 bits");
    extern __shared__ unsigned char lds_raw[];
    T *lam_l = reinterpret_cast<T *>(lds_raw);                 // NR region values
    T *ent_w = lam_l + NR;                                     // NT * K weights
    short *ent_s = reinterpret_cast<short *>(ent_w + NT * K);  // NT * K sources
    int *cnt_l = reinterpret_cast<int *>(ent_s + NT * K);      // NT entry counts
    unsigned char *fr_l = reinterpret_cast<unsigned char *>(cnt_l + NT);  // NT free flags

    const int iter = cnt->sweep_base + iter_rel;
    if (do_bookkeep && blockIdx.x == 0) bookkeep_block(st, n_sd, iter, tol, cnt, 0, scale_rel);
    const ItemList list = sweep_items(items, lists, stamp_stride, cnt, cls, iter, false);
    const int n_items = list.n;
    int *queue = &cnt->class_queue[cls][iter % 3];
    const bool jacobi = local_iters <= 0;
    const int iters = jacobi ? 1 : local_iters;
    unsigned nact = 0;

    for (int item = mode == 1 ? next_item(queue) : (int)blockIdx.x; item < n_items;
         item = mode == 1 ? next_item(queue)
                          : (mode == 2 ? item + (int)gridDim.x : n_items)) {
        const WorkItem it = list.items[item];
        SdState *sst = st + it.sd;
        if (sd_skip(sst, iter, tol, scale_rel)) continue;
        const SdDesc<T> &d = sds[it.sd];
        const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
        const int o[3] = {it.t[0] * TX - H, it.t[1] * TY - H, it.t[2] * TZ - HZ};
        const int src = jacobi ? (iter & 1) : 0;
        const T *__restrict__ Vin = d.V[src];
        T *__restrict__ Vout = d.V[src ^ 1];
        const uint8_t *__restrict__ mem = d.member;
        const int bit = d.bit;
        const T beta = d.beta;
        auto free_at = [&](size_t j) -> bool {
            return d.target[j] < 0 && (!mem || ((mem[j] >> bit) & 1));
        };

        __syncthreads();                 // LDS of the previous item is no longer read
        for (int q = threadIdx.x; q < NR; q += kThreads) {
            const int lx = q % LW, ly = (q / LW) % LH, lz = q / (LW * LH);
            const int gx = o[0] + lx, gy = o[1] + ly, gz = o[2] + lz;
            T lv = T(0);
            if ((unsigned)gx < (unsigned)n0 && (unsigned)gy < (unsigned)n1 &&
                (unsigned)gz < (unsigned)n2) {
                const size_t j = ((size_t)gz * n1 + gy) * n0 + gx;
                if (free_at(j)) lv = Vin[j];
            }
            lam_l[q] = lv;
        }
        for (int i = threadIdx.x; i < NT; i += kThreads) {
            const int x = i % TX, y = (i / TX) % TY, z = i / (TX * TY);
            const int gx = o[0] + H + x, gy = o[1] + H + y, gz = o[2] + HZ + z;
            bool f = false;
            if (gx < n0 && gy < n1 && gz < n2) f = free_at(((size_t)gz * n1 + gy) * n0 + gx);
            fr_l[i] = f ? 1 : 0;
            cnt_l[i] = 0;
        }
        __syncthreads();
        // transposed stencil: every region node pushes its entries to the tile
        for (int q = threadIdx.x; q < NR; q += kThreads) {
            const int l[3] = {q % LW, (q / LW) % LH, q / (LW * LH)};
            const int gx = o[0] + l[0], gy = o[1] + l[1], gz = o[2] + l[2];
            if ((unsigned)gx >= (unsigned)n0 || (unsigned)gy >= (unsigned)n1 ||
                (unsigned)gz >= (unsigned)n2)
                continue;
            const size_t j = ((size_t)gz * n1 + gy) * n0 + gx;
            if (!free_at(j)) continue;
            int p[3] = {0, 0, 0};
            T tau[3] = {T(0), T(0), T(0)};
            if (!adj_foot<T, DIM>(d, j, l, p, tau)) continue;
            adj_stencil<T, DIM>(d.interp, p, tau, [&](const int *v, T w) {
                const int x = v[0] - H, y = v[1] - H, z = DIM == 3 ? v[2] - HZ : 0;
                if ((unsigned)x >= (unsigned)TX || (unsigned)y >= (unsigned)TY ||
                    (unsigned)z >= (unsigned)TZ)
                    return;
                const int ti = (z * TY + y) * TX + x;
                if (!fr_l[ti]) return;
                const int slot = atomicAdd(&cnt_l[ti], 1);
                if (slot < K) {
                    ent_s[ti * K + slot] = (short)q;
                    ent_w[ti * K + slot] = w;
                }
            });
        }
        __syncthreads();
        // this thread's tile nodes: sorted entry lists, owner-routed g
        T gv[NPT];
        int ne[NPT];
        int qn[NPT];
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const int i = threadIdx.x + r * kThreads;
            const int x = i % TX, y = (i / TX) % TY, z = i / (TX * TY);
            qn[r] = ((z + HZ) * LH + (y + H)) * LW + (x + H);
            gv[r] = T(0);
            ne[r] = -1;
            if (!fr_l[i]) continue;
            const size_t j = ((size_t)(o[2] + HZ + z) * n1 + (o[1] + H + y)) * n0 + (o[0] + H + x);
            if (!d.owner || d.owner[j] == d.set) gv[r] = d.g[j];
            ne[r] = cnt_l[i];
            if (ne[r] <= K) {
                for (int a = 1; a < ne[r]; ++a) {        // insertion sort by source
                    const short ks = ent_s[i * K + a];
                    const T kw = ent_w[i * K + a];
                    int b = a - 1;
                    while (b >= 0 && ent_s[i * K + b] > ks) {
                        ent_s[i * K + b + 1] = ent_s[i * K + b];
                        ent_w[i * K + b + 1] = ent_w[i * K + b];
                        --b;
                    }
                    ent_s[i * K + b + 1] = ks;
                    ent_w[i * K + b + 1] = kw;
                }
            }
        }
        double rmax = 0.0, lmax = 0.0;
        unsigned na = 0;
        bool tile_changed = false;
        for (int li = 0; li < iters; ++li) {
            T nv[NPT];
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                nv[r] = T(0);
                if (ne[r] < 0) continue;
                const int i = threadIdx.x + r * kThreads;
                T acc = T(0);
                if (ne[r] <= K) {
                    for (int e = 0; e < ne[r]; ++e)
                        acc = fma_(ent_w[i * K + e], lam_l[ent_s[i * K + e]], acc);
                } else {
                    // more entries than fit: rescan the neighbourhood in source order
                    const int c[3] = {qn[r] % LW, (qn[r] / LW) % LH, qn[r] / (LW * LH)};
                    const int zl = DIM == 3 ? max(c[2] - H - 1, 0) : 0;
                    const int zh = DIM == 3 ? min(c[2] + H, LD - 1) : 0;
                    for (int lz = zl; lz <= zh; ++lz)
                        for (int ly = max(c[1] - H - 1, 0); ly <= min(c[1] + H, LH - 1); ++ly)
                            for (int lx = max(c[0] - H - 1, 0); lx <= min(c[0] + H, LW - 1); ++lx) {
                                const int l[3] = {lx, ly, lz};
                                const int gx = o[0] + lx, gy = o[1] + ly, gz = o[2] + lz;
                                if ((unsigned)gx >= (unsigned)n0 || (unsigned)gy >= (unsigned)n1 ||
                                    (unsigned)gz >= (unsigned)n2)
                                    continue;
                                const size_t j = ((size_t)gz * n1 + gy) * n0 + gx;
                                if (!free_at(j)) continue;
                                int p[3] = {0, 0, 0};
                                T tau[3] = {T(0), T(0), T(0)};
                                if (!adj_foot<T, DIM>(d, j, l, p, tau)) continue;
                                const T lq = lam_l[(lz * LH + ly) * LW + lx];
                                adj_stencil<T, DIM>(d.interp, p, tau, [&](const int *v, T w) {
                                    if (v[0] == c[0] && v[1] == c[1] && (DIM == 2 || v[2] == c[2]))
                                        acc = fma_(w, lq, acc);
                                });
                            }
                }
                nv[r] = fma_(beta, acc, gv[r]);
            }
            __syncthreads();             // every gather of this iteration is done
            int chg = 0;
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (ne[r] < 0) continue;
                const T lo = lam_l[qn[r]];
                const double dv = __builtin_fabs((double)nv[r] - (double)lo);
                const double al = __builtin_fabs((double)nv[r]);
                rmax = dv > rmax ? dv : rmax;
                lmax = al > lmax ? al : lmax;
                chg |= jacobi ? (nv[r] != lo) : (dv > tol + scale_rel * al);
                lam_l[qn[r]] = nv[r];
                ++na;
            }
            if (!__syncthreads_or(chg)) break;
            tile_changed = true;
        }
        if (jacobi || tile_changed) {
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (ne[r] < 0) continue;
                const int i = threadIdx.x + r * kThreads;
                const int x = i % TX, y = (i / TX) % TY, z = i / (TX * TY);
                Vout[((size_t)(o[2] + HZ + z) * n1 + (o[1] + H + y)) * n0 + (o[0] + H + x)] =
                    lam_l[qn[r]];
            }
        }
        nact += na;
        block_max_to(lmax, &sst->scale[iter % 3]);
        (void)block_max_to(rmax, &sst->res[iter % 3]);
        if (threadIdx.x < 64 && tile_changed)
            stamp_and_list<RX, RY, RZ>(stamp + (size_t)((iter + 1) & 1) * stamp_stride, it,
                                       d.tile_offset, d.tiles, iter + 1,
                                       lists + (size_t)((iter + 1) & 1) * stamp_stride,
                                       &cnt->class_count[cls][(iter + 1) % 3]);
    }
    block_sum_to(nact, &cnt->nc_updates);
}

template <typename T, int DIM, int H>
constexpr size_t adj_lds_bytes() {
    using TT = AdjTile<DIM>;
    constexpr int HZ = DIM == 3 ? H : 0;
    constexpr size_t NR = (size_t)(TT::X + 2 * H) * (TT::Y + 2 * H) * (TT::Z + 2 * HZ);
    constexpr size_t NT = (size_t)TT::X * TT::Y * TT::Z;
    return NR * sizeof(T) + NT * TT::K * (sizeof(T) + sizeof(short)) + NT * sizeof(int) + NT;
}

template <typename T>
__global__ void k_adjoint_combine(const AdjDesc<T> *ads, const SdState *st, int n_sets,
                                  const int8_t *target, size_t N, T w, T *dLdl) {
    for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < N;
         j += (size_t)gridDim.x * blockDim.x) {
        T s = T(0);
        if (target[j] < 0)
            for (int i = 0; i < n_sets; ++i) {
                const AdjDesc<T> &d = ads[i];
                if (d.member && !((d.member[j] >> d.bit) & 1)) continue;
                s += (st[i].final_buf ? d.lam2 : d.lam)[j];
            }
        dLdl[j] = w * s;
    }
}

// Instances of the gather adjoint per dimension and halo.
constexpr int kMaxAdjHalo = 8;
constexpr int kMaxAdjHalo3D = 5;
template <typename T, int DIM, int H>
void adj_entry(const void **fn, size_t *lds) {
    fn[H] = (const void *)&k_adjoint_pull<T, DIM, H>;
    lds[H] = adj_lds_bytes<T, DIM, H>();
}
struct AdjTable {
    const void *fn[kMaxAdjHalo + 1] = {};
    size_t lds[kMaxAdjHalo + 1] = {};
};
template <typename T, int DIM>
const AdjTable &adjoint_table() {
    static const AdjTable t = [] {
        AdjTable a;
        adj_entry<T, DIM, 1>(a.fn, a.lds);
        adj_entry<T, DIM, 2>(a.fn, a.lds);
        adj_entry<T, DIM, 3>(a.fn, a.lds);
        adj_entry<T, DIM, 4>(a.fn, a.lds);
        adj_entry<T, DIM, 5>(a.fn, a.lds);
        if constexpr (DIM == 2) {
            adj_entry<T, DIM, 6>(a.fn, a.lds);
            adj_entry<T, DIM, 7>(a.fn, a.lds);
            adj_entry<T, DIM, 8>(a.fn, a.lds);
        }
        return a;
    }();
    return t;
}
template <typename T>
const void *adjoint_tiles_fn(int dim, int H, size_t *lds) {
    if (H < 1 || H > (dim == 2 ? kMaxAdjHalo : kMaxAdjHalo3D)) return nullptr;
    const AdjTable &t = dim == 2 ? adjoint_table<T, 2>() : adjoint_table<T, 3>();
    *lds = t.lds[H];
    return t.fn[H];
}

}  // namespace

int adjoint_tiles_max_halo(int dim) { return dim == 2 ? kMaxAdjHalo : kMaxAdjHalo3D; }

hipError_t adjoint_tiles_set_attributes(LaunchCfg &cfg) {
    size_t lds = 0;
    const void *fn = cfg.dtype == SL_F32 ? adjoint_tiles_fn<float>(cfg.dim, cfg.halo, &lds)
                                         : adjoint_tiles_fn<double>(cfg.dim, cfg.halo, &lds);
    if (!fn) return hipErrorInvalidValue;
    if (lds > 64 * 1024) {
        const hipError_t e =
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int dev = 0, n_cu = 256, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        n_cu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    cfg.grid_cap = per_cu * n_cu;
    return hipSuccess;
}

template <typename T>
hipError_t launch_adjoint_tiles(const LaunchCfg &cfg, const SdDesc<T> *sds, SdState *st,
                                int n_sd, const WorkItem *items, WorkItem *lists,
                                ExecCounters *cnt, int max_items, int iter_rel, double tol,
                                double scale_rel,
                                int *stamp, int stamp_stride, int cls, int do_bookkeep,
                                hipStream_t s) {
    size_t lds = 0;
    const void *fn = adjoint_tiles_fn<T>(cfg.dim, cfg.halo, &lds);
    if (!fn) return hipErrorInvalidValue;
    int grid = max_items > 0 ? max_items : 1;
    int mode = cfg.mode;
    if (mode && cfg.grid_cap > 0 && grid > cfg.grid_cap) grid = cfg.grid_cap;
    int local_iters = cfg.local_iters;
    void *args[] = {(void *)&sds, (void *)&st, (void *)&n_sd, (void *)&items, (void *)&lists,
                    (void *)&cnt, (void *)&iter_rel, (void *)&tol, (void *)&scale_rel, (void *)&stamp,
                    (void *)&stamp_stride, (void *)&mode, (void *)&cls, (void *)&do_bookkeep,
                    (void *)&local_iters};
    return hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, lds, s);
}
template hipError_t launch_adjoint_tiles<float>(const LaunchCfg &, const SdDesc<float> *, SdState *, int, const WorkItem *, WorkItem *, ExecCounters *, int, int, double, double, int *, int, int, int, hipStream_t);
template hipError_t launch_adjoint_tiles<double>(const LaunchCfg &, const SdDesc<double> *, SdState *, int, const WorkItem *, WorkItem *, ExecCounters *, int, int, double, double, int *, int, int, int, hipStream_t);

template <typename T>
hipError_t launch_adjoint_iter(int dim, const AdjDesc<T> *ads, SdState *st, int n_sets,
                               int blocks_per_set, ExecCounters *cnt, int iter, double tol,
                               double scale_rel, hipStream_t s) {
    const dim3 grid(n_sets * blocks_per_set);
    if (dim == 2)
        hipLaunchKernelGGL((k_adjoint<T, 2>), grid, dim3(kThreads), 0, s, ads, st, n_sets,
                           blocks_per_set, cnt, iter, tol, scale_rel);
    else
        hipLaunchKernelGGL((k_adjoint<T, 3>), grid, dim3(kThreads), 0, s, ads, st, n_sets,
                           blocks_per_set, cnt, iter, tol, scale_rel);
    return hipGetLastError();
}
template hipError_t launch_adjoint_iter<float>(int, const AdjDesc<float> *, SdState *, int, int, ExecCounters *, int, double, double, hipStream_t);
template hipError_t launch_adjoint_iter<double>(int, const AdjDesc<double> *, SdState *, int, int, ExecCounters *, int, double, double, hipStream_t);

template <typename T>
hipError_t launch_adjoint_combine(const AdjDesc<T> *ads, const SdState *st, int n_sets,
                                  const int8_t *target, size_t N, T w, T *dLdl, hipStream_t s) {
    size_t g = (N + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_adjoint_combine<T>, dim3((unsigned)g), dim3(kThreads), 0, s, ads, st,
                       n_sets, target, N, w, dLdl);
    return hipGetLastError();
}
template hipError_t launch_adjoint_combine<float>(const AdjDesc<float> *, const SdState *, int, const int8_t *, size_t, float, float *, hipStream_t);
template hipError_t launch_adjoint_combine<double>(const AdjDesc<double> *, const SdState *, int, const int8_t *, size_t, double, double *, hipStream_t);

}  // namespace slhjb
