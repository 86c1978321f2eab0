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

// Block-asynchronous adjoint, 2D, one (set, tile) work item per work-group step.
// The tile plus an H-cell halo is staged in LDS: lambda (0 off the set's free
// nodes), and for every node its frozen foot cell (region coordinates of the
// lower corner, -1 when none of its corners lies in the tile) with the Q1
// fractions.  The inflow from halo nodes is pushed once (LDS float atomics);
// then up to local_iters times: push the tile's own lambda, lambda = g + inflow,
// while some node changes by more than tol + scale_rel * |lambda| (the atomics
// reorder sums, so smaller changes are rounding).  The linear iteration has
// nonnegative coefficients and spectral radius <= beta < 1, so every order of
// updates converges to the same solution (up to rounding).
template <typename T, int H>
__global__ __launch_bounds__(kThreads) void k_adjoint_tiles(
    const SdDesc<T> *__restrict__ sds, SdState *__restrict__ st, int n_sd,
    const WorkItem *__restrict__ items, WorkItem *__restrict__ lists,
    ExecCounters *__restrict__ cnt, int iter_rel,
    double tol, double scale_rel, int *__restrict__ stamp, int stamp_stride, int mode, int cls,
    int do_bookkeep, int local_iters) {
    constexpr int TX = kAdjTX, TY = kAdjTY;
    constexpr int LW = TX + 2 * H, LH = TY + 2 * H, NR = LW * LH, NT = TX * TY;
    constexpr int RSTEP = kThreads / TX, NPT = TY / RSTEP;
    constexpr int RX = (H + TX - 1) / TX, RY = (H + TY - 1) / TY;
    static_assert(kThreads % TX == 0 && TY % RSTEP == 0, "tile/thread mismatch");
    __shared__ T lam_l[NR];
    __shared__ int cell_l[NR];
    __shared__ T fx_l[NR], fy_l[NR];
    __shared__ T acc_h[NT], acc_t[NT];

    const int iter = cnt->sweep_base + iter_rel;
    if (do_bookkeep && blockIdx.x == 0) bookkeep_block(st, n_sd, iter, tol, cnt, 0, scale_rel);
    const ItemList list = sweep_items(items, lists, stamp_stride, cnt, cls, iter, false);
    const int n_items = list.n;
    const int slot = iter % 3;
    int *queue = &cnt->class_queue[cls][slot];
    const int tx = threadIdx.x % TX, ty0 = threadIdx.x / TX;
    unsigned nact = 0;

    for (int item = mode == 1 ? next_item(queue) : (int)blockIdx.x; item < n_items;
         item = mode == 1 ? next_item(queue)
                          : (mode == 2 ? item + (int)gridDim.x : n_items)) {
        const WorkItem it = list.items[item];
        SdState *sst = st + it.sd;
        if (sd_skip(sst, iter, tol, scale_rel)) continue;
        const SdDesc<T> &d = sds[it.sd];
        const int n0 = d.n[0], n1 = d.n[1];
        const int x0 = it.t[0] * TX, y0 = it.t[1] * TY;
        const int ox = x0 - H, oy = y0 - H;
        T *__restrict__ lam = d.V[0];
        const uint8_t *__restrict__ mem = d.member;
        const int bit = d.bit;
        const T beta = d.beta;

        __syncthreads();                 // LDS of the previous item is no longer read
        for (int q = threadIdx.x; q < NR; q += kThreads) {
            const int ly = q / LW, lx = q - ly * LW;
            const int gx = ox + lx, gy = oy + ly;
            T lv = T(0), fx = T(0), fy = T(0);
            int cb = -1;
            if ((unsigned)gx < (unsigned)n0 && (unsigned)gy < (unsigned)n1) {
                const size_t j = (size_t)gy * n0 + gx;
                if (d.target[j] < 0 && (!mem || ((mem[j] >> bit) & 1))) {
                    lv = lam[j];
                    const int k = d.policy[j];
                    if (k < d.m) {
                        T cx = T(1), cy = T(1), qx = T(0), qy = T(0);
                        if (d.speed) {
                            cx = d.speed_axes ? d.speed[2 * j] : d.speed[j];
                            cy = d.speed_axes ? d.speed[2 * j + 1] : cx;
                        }
                        if (d.drift) {
                            qx = d.drift[2 * j];
                            qy = d.drift[2 * j + 1];
                        }
                        const T dx = d.ctrl[2 * k] * cx + qx, dy = d.ctrl[2 * k + 1] * cy + qy;
                        const T flx = floor_(dx), fly = floor_(dy);
                        fx = dx - flx;
                        fy = dy - fly;
                        const int px = lx + (int)flx, py = ly + (int)fly;
                        if (px + 1 >= H && px < H + TX && py + 1 >= H && py < H + TY)
                            cb = py * LW + px;
                    }
                }
            }
            lam_l[q] = lv;
            cell_l[q] = cb;
            fx_l[q] = fx;
            fy_l[q] = fy;
        }
        for (int i = threadIdx.x; i < NT; i += kThreads) acc_h[i] = T(0);
        __syncthreads();
        // inflow from the halo (fixed for this launch)
        for (int q = threadIdx.x; q < NR; q += kThreads) {
            const int ly = q / LW, lx = q - ly * LW;
            if (lx >= H && lx < H + TX && ly >= H && ly < H + TY) continue;
            {
                const int cb = cell_l[q];
                const T lv = lam_l[q];
                if (cb >= 0 && lv != T(0)) {
                    const int py = cb / LW, px = cb - py * LW;
                    const T fx = fx_l[q], fy = fy_l[q];
                    const T bl = beta * lv;
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int cy = py + b;
                        if (cy < H || cy >= H + TY) continue;
                        const T wy = b ? fy : T(1) - fy;
#pragma unroll
                        for (int a2 = 0; a2 < 2; ++a2) {
                            const int cx = px + a2;
                            if (cx < H || cx >= H + TX) continue;
                            const T w = (a2 ? fx : T(1) - fx) * wy;
                            if (w != T(0)) atomicAdd(&acc_h[(cy - H) * TX + (cx - H)], bl * w);
                        }
                    }
                }
            }
        }
        // this thread's tile nodes: free flag and owner-routed g
        T gv[NPT];
        bool fr[NPT];
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const int ty = ty0 + r * RSTEP;
            const int gx = x0 + tx, gy = y0 + ty;
            fr[r] = false;
            gv[r] = T(0);
            if (gx < n0 && gy < n1) {
                const size_t j = (size_t)gy * n0 + gx;
                fr[r] = d.target[j] < 0 && (!mem || ((mem[j] >> bit) & 1));
                if (fr[r] && (!d.owner || d.owner[j] == d.set)) gv[r] = d.g[j];
            }
        }
        const int iters = local_iters > 0 ? local_iters : 1;
        double rmax = 0.0, lmax = 0.0;
        unsigned na = 0;
        bool tile_changed = false;
        for (int li = 0; li < iters; ++li) {
            for (int i = threadIdx.x; i < NT; i += kThreads) acc_t[i] = T(0);
            __syncthreads();             // acc_t cleared; lambda of the last iteration written
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                const int q = (ty0 + r * RSTEP + H) * LW + tx + H;
                {
                const int cb = cell_l[q];
                const T lv = lam_l[q];
                if (cb >= 0 && lv != T(0)) {
                    const int py = cb / LW, px = cb - py * LW;
                    const T fx = fx_l[q], fy = fy_l[q];
                    const T bl = beta * lv;
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int cy = py + b;
                        if (cy < H || cy >= H + TY) continue;
                        const T wy = b ? fy : T(1) - fy;
#pragma unroll
                        for (int a2 = 0; a2 < 2; ++a2) {
                            const int cx = px + a2;
                            if (cx < H || cx >= H + TX) continue;
                            const T w = (a2 ? fx : T(1) - fx) * wy;
                            if (w != T(0)) atomicAdd(&acc_t[(cy - H) * TX + (cx - H)], bl * w);
                        }
                    }
                }
            }
            }
            __syncthreads();             // every push of this iteration is done
            int chg = 0;
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (!fr[r]) continue;
                const int i = (ty0 + r * RSTEP) * TX + tx;
                const int q = (ty0 + r * RSTEP + H) * LW + tx + H;
                const T lo = lam_l[q];
                const T ln = gv[r] + (acc_h[i] + acc_t[i]);
                const double dv = __builtin_fabs((double)ln - (double)lo);
                const double al = __builtin_fabs((double)ln);
                rmax = dv > rmax ? dv : rmax;
                lmax = al > lmax ? al : lmax;
                chg |= dv > tol + scale_rel * al;
                lam_l[q] = ln;
                ++na;
            }
            if (!__syncthreads_or(chg)) break;
            tile_changed = true;
        }
        if (tile_changed) {
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (!fr[r]) continue;
                const int ty = ty0 + r * RSTEP;
                lam[(size_t)(y0 + ty) * n0 + x0 + tx] = lam_l[(ty + H) * LW + tx + H];
            }
        }
        nact += na;
        block_max_to(lmax, &sst->scale[iter % 3]);
        const double bm = block_max_to(rmax, &sst->res[iter % 3]);
        (void)bm;
        if (threadIdx.x < 64 && tile_changed)
            stamp_and_list<RX, RY, 0>(stamp + (size_t)((iter + 1) & 1) * stamp_stride, it,
                                      d.tile_offset, d.tiles, iter + 1,
                                      lists + (size_t)((iter + 1) & 1) * stamp_stride,
                                      &cnt->class_count[cls][(iter + 1) % 3]);
    }
    block_sum_to(nact, &cnt->nc_updates);
}

template <typename T>
__global__ void k_adjoint_combine(const AdjDesc<T> *ads, int n_sets, const int8_t *target,
                                  size_t N, T w, T *dLdl) {
    for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < N;
         j += (size_t)gridDim.x * blockDim.x) {
        T s = T(0);
        if (target[j] < 0)
            for (int i = 0; i < n_sets; ++i) {
                const AdjDesc<T> &d = ads[i];
                if (d.member && !((d.member[j] >> d.bit) & 1)) continue;
                s += d.lam[j];
            }
        dLdl[j] = w * s;
    }
}

// Instances of the adjoint tile kernel per halo (2D; H <= kMaxAdjHalo).
constexpr int kMaxAdjHalo = 8;
template <typename T>
const void *adjoint_tiles_fn(int H) {
    static const void *const table[kMaxAdjHalo + 1] = {
        nullptr,
        (const void *)&k_adjoint_tiles<T, 1>, (const void *)&k_adjoint_tiles<T, 2>,
        (const void *)&k_adjoint_tiles<T, 3>, (const void *)&k_adjoint_tiles<T, 4>,
        (const void *)&k_adjoint_tiles<T, 5>, (const void *)&k_adjoint_tiles<T, 6>,
        (const void *)&k_adjoint_tiles<T, 7>, (const void *)&k_adjoint_tiles<T, 8>};
    return (H >= 1 && H <= kMaxAdjHalo) ? table[H] : nullptr;
}

}  // namespace

int adjoint_tiles_max_halo() { return kMaxAdjHalo; }

hipError_t adjoint_tiles_set_attributes(LaunchCfg &cfg) {
    const void *fn = cfg.dtype == SL_F32 ? adjoint_tiles_fn<float>(cfg.halo)
                                         : adjoint_tiles_fn<double>(cfg.halo);
    if (!fn) return hipErrorInvalidValue;
    int dev = 0, n_cu = 256, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        n_cu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, 0) != hipSuccess ||
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
    const void *fn = adjoint_tiles_fn<T>(cfg.halo);
    if (!fn) return hipErrorInvalidValue;
    int grid = max_items > 0 ? max_items : 1;
    int mode = cfg.mode;
    if (mode && cfg.grid_cap > 0 && grid > cfg.grid_cap) grid = cfg.grid_cap;
    int local_iters = cfg.local_iters;
    void *args[] = {(void *)&sds, (void *)&st, (void *)&n_sd, (void *)&items, (void *)&lists,
                    (void *)&cnt, (void *)&iter_rel, (void *)&tol, (void *)&scale_rel, (void *)&stamp,
                    (void *)&stamp_stride, (void *)&mode, (void *)&cls, (void *)&do_bookkeep,
                    (void *)&local_iters};
    return hipLaunchKernel(fn, dim3(grid), dim3(kThreads), args, 0, s);
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
hipError_t launch_adjoint_combine(const AdjDesc<T> *ads, int n_sets, const int8_t *target,
                                  size_t N, T w, T *dLdl, hipStream_t s) {
    size_t g = (N + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_adjoint_combine<T>, dim3((unsigned)g), dim3(kThreads), 0, s, ads,
                       n_sets, target, N, w, dLdl);
    return hipGetLastError();
}
template hipError_t launch_adjoint_combine<float>(const AdjDesc<float> *, int, const int8_t *, size_t, float, float *, hipStream_t);
template hipError_t launch_adjoint_combine<double>(const AdjDesc<double> *, int, const int8_t *, size_t, double, double *, hipStream_t);

}  // namespace slhjb
