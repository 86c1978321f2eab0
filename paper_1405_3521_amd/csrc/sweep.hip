// Semi-Lagrangian sweep kernels for gfx950 (CDNA4).
//
// One sweep applies the SL operator (paper Sec. 3, (SL)/(Tdef))
//     V_new(j) = max_l min_k  fma(beta, I[V](foot_j,lk), w l_j)
// to every free member node of every active (sub-domain, tile) work item: the
// table holds, per evader choice l, the pursuer's m_inner displacements; a control
// problem has one block (l = 0) and the maximum is over one value.
//
// Mapping to the hardware
//   * one work-group (4 wave64) per work item; the tile plus an H-cell halo
//     (all the corners a foot can reach) is staged in LDS with coalesced row
//     loads, ghost and non-member nodes already replaced by the ghost value, so
//     the inner loop has no branches;
//   * lanes of a wave own consecutive x nodes, so the four (eight) corner reads
//     of neighbouring lanes hit neighbouring LDS banks;
//   * the control loop is uniform across the wave: the displacement table is
//     read through the scalar cache and every lane carries NPT nodes (ILP);
//   * no MFMA: this is a gather + min, not a dense contraction;
//   * FP32 values use tile-local foot coordinates (exact fractional parts, small
//     magnitudes); the FP64 variant uses global grid-index coordinates and the
//     fixed operation order of the scheme, so its results are reproducible bit
//     for bit by any IEEE implementation of the same order.
//   * the per-sd residual max|V_new - V| is reduced in FP64 (wave shuffles, LDS,
//     one 64-bit atomicMax per work-group on the bit pattern).
#include "device_common.h"

#include <algorithm>

namespace slhjb {

namespace {

// ------------------------------------------------------------------ 2D kernel
// Persistent: a resident grid of work-groups takes work items from a per-sweep
// atomic queue until the list is exhausted.
template <typename T, int TX, int TY, int H, bool POLICY, int S, bool P1, int GT>
__global__ __launch_bounds__(GT * S) void k_sweep2d(const SdDesc<T> *__restrict__ sds,
                                                      SdState *__restrict__ st, int n_sd,
                                                      const WorkItem *__restrict__ items,
                                                      WorkItem *__restrict__ lists,
                                                      ExecCounters *__restrict__ cnt,
                                                      int sweep_rel, double tol,
                                                      int *__restrict__ stamp,
                                                      int stamp_stride, int mode, int cls,
                                                      int do_bookkeep, int local_iters) {
    const int sweep = cnt->sweep_base + sweep_rel;
    constexpr int LW = TX + 2 * H;
    constexpr int LH = TY + 2 * H;
    constexpr int RSTEP = GT / TX;
    constexpr int NPT = TY / RSTEP;
    constexpr int RX = (H + TX - 1) / TX, RY = (H + TY - 1) / TY;
    static_assert(GT % 64 == 0 && GT % TX == 0 && TY % RSTEP == 0, "tile/thread mismatch");
    // S groups of GT threads share a tile: the same nodes, every S-th control
    // each (k = g, g + S, ...); group 0 takes the minimum over the groups' partial
    // results (exact, so the values do not depend on S; on ties the lowest control
    // index wins, as in one pass).  Control problems only: a game (more than one
    // evader block) runs with S = 1.
    constexpr int NT = GT * S;
    __shared__ T lds[LW * LH];
    __shared__ T part[S > 1 ? (S - 1) * TX * TY : 1];
    __shared__ int parg[(S > 1 && POLICY) ? (S - 1) * TX * TY : 1];

    if (!POLICY && do_bookkeep && blockIdx.x == 0) bookkeep_block(st, n_sd, sweep, tol, cnt, 0);
    const ItemList list = sweep_items(items, lists, stamp_stride, cnt, cls, sweep, POLICY);
    const int n_items = list.n;
    const int grp = S > 1 ? (int)threadIdx.x / GT : 0;
    const int lt = S > 1 ? (int)threadIdx.x % GT : (int)threadIdx.x;
    unsigned nact = 0;
    const int slot = sweep % 3;
    // mode 0: one item per work-group, scheduled by the hardware;
    // mode 1: resident grid taking items from the sweep's atomic queue;
    // mode 2: resident grid walking the list with a grid stride.
    int *queue = &cnt->class_queue[cls][slot];
    for (int item = mode == 1 ? next_item(queue) : (int)blockIdx.x; item < n_items;
         item = mode == 1 ? next_item(queue)
                          : (mode == 2 ? item + (int)gridDim.x : n_items)) {
        const WorkItem it = list.items[item];
        SdState *sst = st + it.sd;
        if (!POLICY && sd_skip(sst, sweep, tol)) continue;
        const SdDesc<T> &d = sds[it.sd];
        const int n0 = d.n[0], n1 = d.n[1];
        const int x0 = it.t[0] * TX, y0 = it.t[1] * TY;
        const int src = POLICY ? sst->final_buf : (sweep & 1);
        const T *__restrict__ Vin = d.V[src];
        T *__restrict__ Vout = d.V[src ^ 1];
        const uint8_t *__restrict__ mem = d.member;
        const int bit = d.bit;
        const T G = d.G;

        __syncthreads();                 // LDS of the previous item is no longer read
        for (int q = threadIdx.x; q < LW * LH; q += NT) {
            const int ly = q / LW;
            const int lx = q - ly * LW;
            const int gx = x0 - H + lx, gy = y0 - H + ly;
            T v = G;
            if ((unsigned)gx < (unsigned)n0 && (unsigned)gy < (unsigned)n1) {
                const size_t j = (size_t)gy * n0 + gx;
                if (!mem || ((mem[j] >> bit) & 1)) v = Vin[j];
            }
            lds[q] = v;
        }
        __syncthreads();

        // Compaction (one node per thread): the tile's active nodes (free
        // members) take the first threads, in node order, so the threads past
        // the last active node form whole waves that skip the control loop: the
        // inactive lanes of a tile cut by a set's boundary or holding targets
        // become idle waves instead of inactive lanes inside busy ones.  With
        // several nodes per thread every thread keeps its own nodes (rows r of
        // the tile), which keeps neighbouring lanes on neighbouring nodes.
        constexpr bool COMPACT = NPT == 1;
        constexpr int CU = NPT == 1 ? 4 : 2;
        constexpr int NW = GT / 64;                  // waves of one control group
        __shared__ short cidx[COMPACT ? TX * TY : 1];
        __shared__ int ccnt[COMPACT ? NW : 1];
        int n_act = 0;
        if (COMPACT) {
            bool fl = false;
            unsigned long long mk = 0;
            if (grp == 0) {
                const int gxn = x0 + lt % TX, gyn = y0 + lt / TX;
                if (gxn < n0 && gyn < n1) {
                    const size_t j = (size_t)gyn * n0 + gxn;
                    fl = (!mem || ((mem[j] >> bit) & 1)) && d.target[j] < 0;
                }
                mk = __ballot(fl);
                if ((lt & 63) == 0) ccnt[lt >> 6] = (int)__popcll(mk);
            }
            __syncthreads();
            if (grp == 0 && fl) {
                int base = 0;
                for (int p = 0; p < (lt >> 6); ++p) base += ccnt[p];
                cidx[base + (int)__popcll(mk & ((1ull << (lt & 63)) - 1ull))] = (short)lt;
            }
#pragma unroll
            for (int p = 0; p < NW; ++p) n_act += ccnt[p];
            __syncthreads();             // cidx complete
        }

        T cx[NPT], cy[NPT], ux0[NPT], uy0[NPT], qx[NPT], qy[NPT], wl[NPT], bt[NPT], best[NPT];
        int arg[NPT], nx[NPT], ny[NPT];
        bool act[NPT];
        int any = 0;
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            int n = lt + r * GT;
            if (COMPACT) {
                act[r] = lt < n_act;
                n = act[r] ? (int)cidx[lt] : 0;
            }
            nx[r] = n % TX;
            ny[r] = n / TX;
            const int gx = x0 + nx[r], gy = y0 + ny[r];
            if (!COMPACT) {
                act[r] = false;
                if (gx < n0 && gy < n1) {
                    const size_t j = (size_t)gy * n0 + gx;
                    act[r] = (!mem || ((mem[j] >> bit) & 1)) && d.target[j] < 0;
                }
            }
            cx[r] = T(0);                       // inactive lanes: foot = own node
            cy[r] = T(0);
            wl[r] = d.wl_const;
            bt[r] = d.beta;
            T qxv = T(0), qyv = T(0);           // drift in index units
            if (act[r]) {
                const size_t j = (size_t)gy * n0 + gx;
                if (!d.speed) {
                    cx[r] = cy[r] = T(1);
                } else if (d.speed_axes) {
                    cx[r] = d.speed[2 * j];
                    cy[r] = d.speed[2 * j + 1];
                } else {
                    cx[r] = cy[r] = d.speed[j];
                }
                if (d.wl) wl[r] = d.wl[j];
                if (d.beta_n) bt[r] = d.beta_n[j];
                if (d.drift) {
                    qxv = d.drift[2 * j];
                    qyv = d.drift[2 * j + 1];
                }
            }
            any |= act[r];
            if (sizeof(T) == 4) {
                // FP32: the drift folds into the node's tile-local origin
                ux0[r] = (T)(nx[r] + H) + qxv;
                uy0[r] = (T)(ny[r] + H) + qyv;
            } else {
                // FP64: u = i + (e c + q), the reproducible operation order
                ux0[r] = (T)gx;
                uy0[r] = (T)gy;
            }
            qx[r] = sizeof(T) == 4 ? T(0) : qxv;
            qy[r] = sizeof(T) == 4 ? T(0) : qyv;
        }
        const int ox = x0 - H, oy = y0 - H;     // tile-local origin (FP64 path)
        const const_ptr<T> ctrl = as_const(d.ctrl);     // scalar loads
        const int m = d.m;
        const int ma = d.m_inner > 0 ? d.m_inner : m;
        // Jacobi (local_iters == 0): one evaluation per node, written to the other
        // buffer.  Block-asynchronous (local_iters = k > 0): the tile iterates up to
        // k times on its own values in LDS, the halo as staged, while anything in it
        // changes; the values go back in place (both buffers are the same array).
        const bool async = !POLICY && local_iters > 0;
        const int iters = async ? local_iters : 1;
        double rmax = 0.0;
        unsigned na = 0;
        bool tile_changed = false;
        for (int li = 0; li < iters; ++li) {
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            best[r] = -(T)INFINITY;
            arg[r] = 0;
        }
        // evader blocks (maximum) of pursuer controls (minimum); with S groups the
        // groups split the controls of each block (games use S = 1)
        if (__any(any)) {
        for (int kb = 0; kb < m; kb += ma) {
            T inner[NPT];
#pragma unroll
            for (int r = 0; r < NPT; ++r) inner[r] = (T)INFINITY;
            // controls unrolled by 4 with one node per thread, by 2 when each
            // thread carries several nodes (their registers already give ILP)
#pragma unroll CU
            for (int k = kb + grp; k < kb + ma; k += S) {
                const T ex = ctrl[2 * k], ey = ctrl[2 * k + 1];
#pragma unroll
                for (int r = 0; r < NPT; ++r) {
                    T ux, uy;
                    if (sizeof(T) == 4) {
                        ux = fma_(cx[r], ex, ux0[r]);
                        uy = fma_(cy[r], ey, uy0[r]);
                    } else {
                        ux = ux0[r] + (ex * cx[r] + qx[r]);
                        uy = uy0[r] + (ey * cy[r] + qy[r]);
                    }
                    int ix, iy;
                    T fx, fy;
                    Foot<T>::split(ux, ox, ix, fx);
                    Foot<T>::split(uy, oy, iy, fy);
                    // corners lie inside the staged tile (0 <= ix, iy < LW, LH): a
                    // 24-bit multiply is exact and single-pass
                    const int base = (int)__umul24((unsigned)iy, (unsigned)LW) + ix;
                    T acc;
                    if (P1) {
                        // P1 on the cell's Kuhn simplex: lower corner, one step
                        // along the axis of the larger fraction (x on ties), the
                        // upper corner; nested interpolations from the far vertex
                        const bool xf = fx >= fy;
                        const T t0 = xf ? fx : fy, t1 = xf ? fy : fx;
                        const T v00 = lds[base], vm = lds[base + (xf ? 1 : LW)];
                        const T v11 = lds[base + LW + 1];
                        const T sr = simplex_ratio(t1, t0);
                        const T in = lerp_m(sr, vm, v11);
                        acc = lerp_m(t0, v00, in);
                    } else {
                    const T v00 = lds[base], v10 = lds[base + 1];
                    const T v01 = lds[base + LW], v11 = lds[base + LW + 1];
                    // Q1 as nested one-axis interpolations (lerp_m), x then y.
                    // Every rounding step is monotone in the node values (so the
                    // iterates from the ghost value decrease to a bitwise fixed point,
                    // in any update order), and a field equal to a power of two (the
                    // ghost value) is reproduced exactly: the unreached region keeps
                    // its value bit for bit, so its tiles are skipped instead of
                    // drifting.  In FP64 (global index coordinates) this is also the
                    // fixed operation order the reproducible labels rely on.
                    const T a = lerp_m(fx, v00, v10);
                    const T b = lerp_m(fx, v01, v11);
                    acc = lerp_m(fy, a, b);
                    }
                    const T cand = fma_(bt[r], acc, wl[r]);
                    if (POLICY) {
                        if (cand < inner[r]) {
                            inner[r] = cand;
                            arg[r] = k;
                        }
                    } else {
                        inner[r] = min_(inner[r], cand);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < NPT; ++r) best[r] = max_(best[r], inner[r]);
        }
        }
        if (S > 1) {
            if (grp > 0) {
#pragma unroll
                for (int r = 0; r < NPT; ++r) {
                    const int node = lt + r * GT;           // thread slot
                    part[(grp - 1) * TX * TY + node] = best[r];
                    if (POLICY) parg[(grp - 1) * TX * TY + node] = arg[r];
                }
            }
            __syncthreads();
            if (grp == 0) {
#pragma unroll
                for (int r = 0; r < NPT; ++r) {
                    const int node = lt + r * GT;           // thread slot
                    for (int g = 1; g < S; ++g) {
                        const T v = part[(g - 1) * TX * TY + node];
                        if (POLICY) {
                            const int a = parg[(g - 1) * TX * TY + node];
                            if (v < best[r] || (v == best[r] && a < arg[r])) {
                                best[r] = v;
                                arg[r] = a;
                            }
                        } else {
                            best[r] = min_(best[r], v);
                        }
                    }
                }
            }
        }
        if (async) {
            int chg = 0;
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (!act[r] || grp > 0) continue;
                const T old = lds[(ny[r] + H) * LW + nx[r] + H];
                const double dv = __builtin_fabs((double)best[r] - (double)old);
                rmax = dv > rmax ? dv : rmax;
                chg |= best[r] != old;
                ++na;
            }
            __syncthreads();                 // every read of this iteration is done
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (!act[r] || grp > 0) continue;
                lds[(ny[r] + H) * LW + nx[r] + H] = best[r];
            }
            if (!__syncthreads_or(chg)) break;
            tile_changed = true;
        } else {
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (!act[r] || grp > 0) continue;
                const size_t j = (size_t)(y0 + ny[r]) * n0 + x0 + nx[r];
                // a policy pass over in-place (block-asynchronous) values only
                // records the argmin, so that it belongs to the returned values
                if (!POLICY || Vout != Vin) Vout[j] = best[r];
                if (POLICY) d.policy[j] = (uint8_t)arg[r];
                const double dv =
                    __builtin_fabs((double)best[r] - (double)lds[(ny[r] + H) * LW + nx[r] + H]);
                rmax = dv > rmax ? dv : rmax;
                ++na;
            }
        }
        }                                    // local iterations
        if (tile_changed) {
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (!act[r] || grp > 0) continue;
                Vout[(size_t)(y0 + ny[r]) * n0 + x0 + nx[r]] = lds[(ny[r] + H) * LW + nx[r] + H];
            }
        }
        nact += na * (unsigned)m;
        if (!POLICY) {
            const double bm = block_max_to<NT>(rmax, &sst->res[sweep % 3]);
            if (threadIdx.x < 64 && __shfl(bm, 0, 64) > 0.0)
                stamp_and_list<RX, RY, 0>(stamp + (size_t)((sweep + 1) & 1) * stamp_stride, it,
                                          d.tile_offset, d.tiles, sweep + 1,
                                          lists + (size_t)((sweep + 1) & 1) * stamp_stride,
                                          &cnt->class_count[cls][(sweep + 1) % 3]);
        }
    }
    if (!POLICY) block_sum_to<NT>(nact, &cnt->nc_updates);
}

// ------------------------------------------------------------------ 3D kernel
template <typename T, int TX, int TY, int TZ, int H, bool POLICY, bool P1>
__global__ __launch_bounds__(kThreads) void k_sweep3d(const SdDesc<T> *__restrict__ sds,
                                                      SdState *__restrict__ st, int n_sd,
                                                      const WorkItem *__restrict__ items,
                                                      WorkItem *__restrict__ lists,
                                                      ExecCounters *__restrict__ cnt,
                                                      int sweep_rel, double tol,
                                                      int *__restrict__ stamp,
                                                      int stamp_stride, int mode, int cls,
                                                      int do_bookkeep, int local_iters) {
    const int sweep = cnt->sweep_base + sweep_rel;
    constexpr int LW = TX + 2 * H;
    constexpr int LH = TY + 2 * H;
    constexpr int LD = TZ + 2 * H;
    constexpr int PL = LW * LH;
    constexpr int TXY = TX * TY;
    static_assert(kThreads % TXY == 0 || TXY % kThreads == 0, "tile/thread mismatch");
    constexpr int ZSTEP = kThreads / TXY;              // z planes covered per pass
    constexpr int NPT = TZ / ZSTEP;
    constexpr int RX = (H + TX - 1) / TX, RY = (H + TY - 1) / TY, RZ = (H + TZ - 1) / TZ;
    static_assert(ZSTEP >= 1 && TZ % ZSTEP == 0, "tile/thread mismatch");
    extern __shared__ unsigned char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);

    if (!POLICY && do_bookkeep && blockIdx.x == 0) bookkeep_block(st, n_sd, sweep, tol, cnt, 0);
    const ItemList list = sweep_items(items, lists, stamp_stride, cnt, cls, sweep, POLICY);
    const int n_items = list.n;
    const int tx = threadIdx.x % TX;
    const int ty = (threadIdx.x / TX) % TY;
    const int tz0 = threadIdx.x / TXY;
    unsigned nact = 0;
    const int slot = sweep % 3;
    // mode 0: one item per work-group, scheduled by the hardware;
    // mode 1: resident grid taking items from the sweep's atomic queue;
    // mode 2: resident grid walking the list with a grid stride.
    int *queue = &cnt->class_queue[cls][slot];
    for (int item = mode == 1 ? next_item(queue) : (int)blockIdx.x; item < n_items;
         item = mode == 1 ? next_item(queue)
                          : (mode == 2 ? item + (int)gridDim.x : n_items)) {
        const WorkItem it = list.items[item];
        SdState *sst = st + it.sd;
        if (!POLICY && sd_skip(sst, sweep, tol)) continue;
        const SdDesc<T> &d = sds[it.sd];
        const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
        const int x0 = it.t[0] * TX, y0 = it.t[1] * TY, z0 = it.t[2] * TZ;
        const int src = POLICY ? sst->final_buf : (sweep & 1);
        const T *__restrict__ Vin = d.V[src];
        T *__restrict__ Vout = d.V[src ^ 1];
        const uint8_t *__restrict__ mem = d.member;
        const int bit = d.bit;
        const T G = d.G;

        __syncthreads();                 // LDS of the previous item is no longer read
        for (int q = threadIdx.x; q < PL * LD; q += kThreads) {
            const int lz = q / PL;
            const int rem = q - lz * PL;
            const int ly = rem / LW;
            const int lx = rem - ly * LW;
            const int gx = x0 - H + lx, gy = y0 - H + ly, gz = z0 - H + lz;
            T v = G;
            if ((unsigned)gx < (unsigned)n0 && (unsigned)gy < (unsigned)n1 &&
                (unsigned)gz < (unsigned)n2) {
                const size_t j = ((size_t)gz * n1 + gy) * n0 + gx;
                if (!mem || ((mem[j] >> bit) & 1)) v = Vin[j];
            }
            lds[q] = v;
        }
        __syncthreads();

        const int gx = x0 + tx, gy = y0 + ty;
        T cx[NPT], cy[NPT], cz[NPT], ux0[NPT], uy0[NPT], uz0[NPT], qx[NPT], qy[NPT], qz[NPT];
        T wl[NPT], bt[NPT], best[NPT];
        int arg[NPT];
        bool act[NPT];
        int any = 0;
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const int tz = tz0 + r * ZSTEP;
            const int gz = z0 + tz;
            act[r] = false;
            cx[r] = cy[r] = cz[r] = T(0);       // inactive lanes: foot = own node
            wl[r] = d.wl_const;
            bt[r] = d.beta;
            T qxv = T(0), qyv = T(0), qzv = T(0);
            if (gx < n0 && gy < n1 && gz < n2) {
                const size_t j = ((size_t)gz * n1 + gy) * n0 + gx;
                const bool inset = !mem || ((mem[j] >> bit) & 1);
                act[r] = inset && d.target[j] < 0;
                if (act[r]) {
                    if (!d.speed) {
                        cx[r] = cy[r] = cz[r] = T(1);
                    } else if (d.speed_axes) {
                        cx[r] = d.speed[3 * j];
                        cy[r] = d.speed[3 * j + 1];
                        cz[r] = d.speed[3 * j + 2];
                    } else {
                        cx[r] = cy[r] = cz[r] = d.speed[j];
                    }
                    if (d.wl) wl[r] = d.wl[j];
                    if (d.beta_n) bt[r] = d.beta_n[j];
                    if (d.drift) {
                        qxv = d.drift[3 * j];
                        qyv = d.drift[3 * j + 1];
                        qzv = d.drift[3 * j + 2];
                    }
                }
            }
            any |= act[r];
            if (sizeof(T) == 4) {
                ux0[r] = (T)(tx + H) + qxv;
                uy0[r] = (T)(ty + H) + qyv;
                uz0[r] = (T)(tz + H) + qzv;
            } else {
                ux0[r] = (T)gx;
                uy0[r] = (T)gy;
                uz0[r] = (T)gz;
            }
            qx[r] = sizeof(T) == 4 ? T(0) : qxv;
            qy[r] = sizeof(T) == 4 ? T(0) : qyv;
            qz[r] = sizeof(T) == 4 ? T(0) : qzv;
        }
        const int ox = x0 - H, oy = y0 - H, oz = z0 - H;
        const const_ptr<T> ctrl = as_const(d.ctrl);     // scalar loads
        const int m = d.m;
        const int ma = d.m_inner > 0 ? d.m_inner : m;
        // Jacobi or block-asynchronous local iterations, as in the 2D kernel
        const bool async = !POLICY && local_iters > 0;
        const int iters = async ? local_iters : 1;
        double rmax = 0.0;
        unsigned na = 0;
        bool tile_changed = false;
        for (int li = 0; li < iters; ++li) {
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            best[r] = -(T)INFINITY;
            arg[r] = 0;
        }
        if (__any(any)) {
        for (int kb = 0; kb < m; kb += ma) {     // evader blocks, as in the 2D kernel
            T inner[NPT];
#pragma unroll
            for (int r = 0; r < NPT; ++r) inner[r] = (T)INFINITY;
#pragma unroll 2
            for (int k = kb; k < kb + ma; ++k) {
                const T ex = ctrl[3 * k], ey = ctrl[3 * k + 1], ez = ctrl[3 * k + 2];
#pragma unroll
                for (int r = 0; r < NPT; ++r) {
                    T ux, uy, uz;
                    if (sizeof(T) == 4) {
                        ux = fma_(cx[r], ex, ux0[r]);
                        uy = fma_(cy[r], ey, uy0[r]);
                        uz = fma_(cz[r], ez, uz0[r]);
                    } else {
                        ux = ux0[r] + (ex * cx[r] + qx[r]);
                        uy = uy0[r] + (ey * cy[r] + qy[r]);
                        uz = uz0[r] + (ez * cz[r] + qz[r]);
                    }
                    int ix, iy, iz;
                    T fx, fy, fz;
                    Foot<T>::split(ux, ox, ix, fx);
                    Foot<T>::split(uy, oy, iy, fy);
                    Foot<T>::split(uz, oz, iz, fz);
                    // corners lie inside the staged block: 24-bit products are exact
                    const int base = (int)__umul24((unsigned)iz, (unsigned)PL) +
                                     (int)__umul24((unsigned)iy, (unsigned)LW) + ix;
                    T acc;
                    if (P1) {
                        // P1 on the cell's Kuhn simplex: the fractions sorted in
                        // decreasing order with their axis steps (a stable sort:
                        // equal fractions keep the lower axis first), vertices
                        // from the lower corner one sorted step at a time, nested
                        // interpolations from the far vertex
                        T t0 = fx, t1 = fy, t2 = fz;
                        int o0 = 1, o1 = LW, o2 = PL;
                        if (t1 > t0) { const T t = t0; t0 = t1; t1 = t; const int o = o0; o0 = o1; o1 = o; }
                        if (t2 > t1) { const T t = t1; t1 = t2; t2 = t; const int o = o1; o1 = o2; o2 = o; }
                        if (t1 > t0) { const T t = t0; t0 = t1; t1 = t; const int o = o0; o0 = o1; o1 = o; }
                        const T v0 = lds[base], v1 = lds[base + o0], v2 = lds[base + o0 + o1];
                        const T v3 = lds[base + 1 + LW + PL];
                        const T s2 = simplex_ratio(t2, t1), s1 = simplex_ratio(t1, t0);
                        const T i2 = lerp_m(s2, v2, v3);
                        const T i1 = lerp_m(s1, v1, i2);
                        acc = lerp_m(t0, v0, i1);
                        (void)o2;
                    } else {
                    // nested one-axis interpolations, x, then y, then z (as in 2D)
                    const T v000 = lds[base], v100 = lds[base + 1];
                    const T v010 = lds[base + LW], v110 = lds[base + LW + 1];
                    const T *__restrict__ up = lds + base + PL;   // the z + 1 plane
                    const T v001 = up[0], v101 = up[1];
                    const T v011 = up[LW], v111 = up[LW + 1];
                    const T a0 = lerp_m(fx, v000, v100);
                    const T b0 = lerp_m(fx, v010, v110);
                    const T a1 = lerp_m(fx, v001, v101);
                    const T b1 = lerp_m(fx, v011, v111);
                    const T c0 = lerp_m(fy, a0, b0);
                    const T c1 = lerp_m(fy, a1, b1);
                    acc = lerp_m(fz, c0, c1);
                    }
                    const T cand = fma_(bt[r], acc, wl[r]);
                    if (POLICY) {
                        if (cand < inner[r]) {
                            inner[r] = cand;
                            arg[r] = k;
                        }
                    } else {
                        inner[r] = min_(inner[r], cand);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < NPT; ++r) best[r] = max_(best[r], inner[r]);
        }
        }
        if (async) {
            int chg = 0;
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (!act[r]) continue;
                const int tz = tz0 + r * ZSTEP;
                const T old = lds[((tz + H) * LH + ty + H) * LW + tx + H];
                const double dv = __builtin_fabs((double)best[r] - (double)old);
                rmax = dv > rmax ? dv : rmax;
                chg |= best[r] != old;
                ++na;
            }
            __syncthreads();                 // every read of this iteration is done
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (!act[r]) continue;
                lds[((tz0 + r * ZSTEP + H) * LH + ty + H) * LW + tx + H] = best[r];
            }
            if (!__syncthreads_or(chg)) break;
            tile_changed = true;
        } else {
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (!act[r]) continue;
                const int tz = tz0 + r * ZSTEP;
                const size_t j = ((size_t)(z0 + tz) * n1 + gy) * n0 + gx;
                if (!POLICY || Vout != Vin) Vout[j] = best[r];
                if (POLICY) d.policy[j] = (uint8_t)arg[r];
                const double dv = __builtin_fabs(
                    (double)best[r] - (double)lds[((tz + H) * LH + ty + H) * LW + tx + H]);
                rmax = dv > rmax ? dv : rmax;
                ++na;
            }
        }
        }                                    // local iterations
        if (tile_changed) {
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                if (!act[r]) continue;
                const int tz = tz0 + r * ZSTEP;
                Vout[((size_t)(z0 + tz) * n1 + gy) * n0 + gx] =
                    lds[((tz + H) * LH + ty + H) * LW + tx + H];
            }
        }
        nact += na * (unsigned)m;
        if (!POLICY) {
            const double bm = block_max_to(rmax, &sst->res[sweep % 3]);
            if (threadIdx.x < 64 && __shfl(bm, 0, 64) > 0.0)
                stamp_and_list<RX, RY, RZ>(stamp + (size_t)((sweep + 1) & 1) * stamp_stride, it,
                                           d.tile_offset, d.tiles, sweep + 1,
                                           lists + (size_t)((sweep + 1) & 1) * stamp_stride,
                                           &cnt->class_count[cls][(sweep + 1) % 3]);
        }
    }
    if (!POLICY) block_sum_to(nact, &cnt->nc_updates);
}

__global__ void k_flip(SdState *st, int n_sd) {
    for (int i = threadIdx.x; i < n_sd; i += blockDim.x) st[i].final_buf ^= 1;
}

__global__ void k_bookkeep(SdState *st, int n_sd, int sweep_rel, double tol, ExecCounters *cnt,
                           int final_pass, double scale_rel, int advance) {
    const int base = cnt->sweep_base;
    bookkeep_block(st, n_sd, base + sweep_rel, tol, cnt, final_pass, scale_rel);
    if (threadIdx.x == 0) cnt->sweep_base = base + advance;
}

// ------------------------------------------------------------ dispatch tables


struct Variant {
    int dim, dtype, tile[3], threads, groups;
    const void *fn[kMaxHalo + 1][2];    // [H][policy]
    const void *fn_p1[kMaxHalo + 1][2]; // P1 interpolation (null where not built)
    size_t lds_bytes[kMaxHalo + 1];     // dynamic LDS (3D only)
};

template <typename T, int TX, int TY, int H, int S, bool WITH_P1, int GT>
void fill2d(Variant &v) {
    v.fn[H][0] = (const void *)&k_sweep2d<T, TX, TY, H, false, S, false, GT>;
    v.fn[H][1] = (const void *)&k_sweep2d<T, TX, TY, H, true, S, false, GT>;
    if (WITH_P1) {
        v.fn_p1[H][0] = (const void *)&k_sweep2d<T, TX, TY, H, false, S, WITH_P1, GT>;
        v.fn_p1[H][1] = (const void *)&k_sweep2d<T, TX, TY, H, true, S, WITH_P1, GT>;
    }
    v.lds_bytes[H] = 0;
}
template <typename T, int TX, int TY, int TZ, int H, bool WITH_P1>
void fill3d(Variant &v) {
    v.fn[H][0] = (const void *)&k_sweep3d<T, TX, TY, TZ, H, false, false>;
    v.fn[H][1] = (const void *)&k_sweep3d<T, TX, TY, TZ, H, true, false>;
    if (WITH_P1) {
        v.fn_p1[H][0] = (const void *)&k_sweep3d<T, TX, TY, TZ, H, false, WITH_P1>;
        v.fn_p1[H][1] = (const void *)&k_sweep3d<T, TX, TY, TZ, H, true, WITH_P1>;
    }
    v.lds_bytes[H] = sizeof(T) * (size_t)(TX + 2 * H) * (TY + 2 * H) * (TZ + 2 * H);
}

// GT threads per control group (kThreads unless the tile has fewer nodes), S groups
template <typename T, int TX, int TY, int S = 1, bool P = false, int GT = kThreads>
Variant make2d() {
    Variant v{};
    v.dim = 2;
    v.dtype = sizeof(T) == 4 ? SL_F32 : SL_F64;
    v.tile[0] = TX; v.tile[1] = TY; v.tile[2] = 1;
    v.threads = GT * S;
    v.groups = S;
    fill2d<T, TX, TY, 1, S, P, GT>(v); fill2d<T, TX, TY, 2, S, P, GT>(v); fill2d<T, TX, TY, 3, S, P, GT>(v);
    fill2d<T, TX, TY, 4, S, P, GT>(v); fill2d<T, TX, TY, 5, S, P, GT>(v); fill2d<T, TX, TY, 6, S, P, GT>(v);
    fill2d<T, TX, TY, 7, S, P, GT>(v); fill2d<T, TX, TY, 8, S, P, GT>(v); fill2d<T, TX, TY, 9, S, P, GT>(v);
    fill2d<T, TX, TY, 10, S, P, GT>(v); fill2d<T, TX, TY, 11, S, P, GT>(v);
    fill2d<T, TX, TY, 12, S, P, GT>(v); fill2d<T, TX, TY, 13, S, P, GT>(v);
    fill2d<T, TX, TY, 14, S, P, GT>(v); fill2d<T, TX, TY, 15, S, P, GT>(v);
    fill2d<T, TX, TY, 16, S, P, GT>(v);
    return v;
}
template <typename T, int TX, int TY, int TZ, bool P = false>
Variant make3d() {
    Variant v{};
    v.dim = 3;
    v.dtype = sizeof(T) == 4 ? SL_F32 : SL_F64;
    v.tile[0] = TX; v.tile[1] = TY; v.tile[2] = TZ;
    v.threads = kThreads;
    v.groups = 1;
    fill3d<T, TX, TY, TZ, 1, P>(v); fill3d<T, TX, TY, TZ, 2, P>(v);
    fill3d<T, TX, TY, TZ, 3, P>(v); fill3d<T, TX, TY, TZ, 4, P>(v);
    fill3d<T, TX, TY, TZ, 5, P>(v); fill3d<T, TX, TY, TZ, 6, P>(v);
    fill3d<T, TX, TY, TZ, 7, P>(v); fill3d<T, TX, TY, TZ, 8, P>(v);
    return v;
}

const Variant *variants(int *count) {
    static const Variant table[] = {
        make2d<float, 64, 16, 1, true>(),   // 0: default FP32 2D (also P1)
        make2d<float, 64, 8>(),    // 1
        make2d<float, 64, 4>(),    // 2
        make2d<float, 32, 16>(),   // 3
        make2d<double, 64, 8, 1, true>(),   // 4: FP64 2D (also P1)
        make3d<float, 32, 8, 8, true>(),  // 5: default FP32 3D (also P1)
        make3d<float, 32, 8, 4, true>(),  // 6 (also P1)
        make3d<float, 16, 16, 4, true>(), // 7 (also P1)
        make3d<double, 16, 8, 8, true>(), // 8: FP64 3D (also P1)
        make2d<double, 32, 8, 1, true>(),   // 9: FP64 2D, small tiles (coarse grids; also P1)
        make2d<double, 16, 16>(),  // 10
        make3d<double, 8, 8, 8, true>(),  // 11: FP64 3D, small tiles (also P1)
        make3d<double, 16, 8, 4, true>(), // 12 (also P1)
        make2d<float, 32, 16, 2>(), // 13: FP32 2D, controls split over 2 groups
        make2d<float, 32, 16, 4>(), // 14: ... over 4 groups
        make2d<float, 64, 8, 4>(),  // 15
        make2d<double, 16, 16, 2>(), // 16: FP64 2D, controls split over 2 groups: more
        make2d<double, 16, 16, 4>(), // 17: waves per tile for small (coarse) grids
        make2d<float, 32, 8, 1, true>(),    // 18: FP32 2D, one node per thread: finer skipping (also P1)
        make2d<float, 16, 16>(),     // 19: and twice the waves per active region
        make2d<float, 32, 8, 2>(),   // 20
        // tiles of fewer than 256 nodes (control groups of 128 or 64 threads): more
        // tiles for small grids, so a launch spreads over every compute unit and a
        // lone tile's local iterations take less time (the coarse FP64 pass)
        make2d<double, 16, 8, 4, false, 128>(),   // 21
        make2d<double, 8, 8, 4, false, 64>(),     // 22
        make2d<float, 16, 8, 2, false, 128>(),    // 23
    };
    *count = (int)(sizeof(table) / sizeof(table[0]));
    return table;
}

}  // namespace

int sweep_variants(int dim, LaunchCfg *out, int cap) {
    int nv = 0, k = 0;
    const Variant *v = variants(&nv);
    for (int i = 0; i < nv; ++i) {
        if (v[i].dim != dim) continue;
        if (k < cap) {
            out[k].dim = v[i].dim;
            out[k].dtype = v[i].dtype;
            out[k].tile[0] = v[i].tile[0];
            out[k].tile[1] = v[i].tile[1];
            out[k].tile[2] = v[i].tile[2];
            out[k].halo = 0;
            out[k].variant = i;
            out[k].threads = v[i].threads;
            out[k].groups = v[i].groups;
            out[k].interp = SL_INTERP_Q1;
        }
        ++k;
    }
    return k;
}

bool sweep_has_p1(int variant) {
    int nv = 0;
    const Variant *vt = variants(&nv);
    return variant >= 0 && variant < nv && vt[variant].fn_p1[1][0];
}

static const void *sweep_fn(const LaunchCfg &cfg, int want_policy, size_t *lds) {
    int nv = 0;
    const Variant *vt = variants(&nv);
    if (cfg.variant < 0 || cfg.variant >= nv || cfg.halo < 1) return nullptr;
    const Variant &v = vt[cfg.variant];
    if (cfg.halo > (v.dim == 2 ? kMaxHalo : kMaxHalo3D) || !v.fn[cfg.halo][0]) return nullptr;
    *lds = v.lds_bytes[cfg.halo];
    if (cfg.interp == SL_INTERP_P1) return v.fn_p1[cfg.halo][want_policy ? 1 : 0];
    return v.fn[cfg.halo][want_policy ? 1 : 0];
}

hipError_t sweep_set_attributes(LaunchCfg &cfg) {
    static int n_cu = 0;
    if (!n_cu) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            n_cu = 256;
    }
    int caps[2] = {1, 1};
    for (int pol = 0; pol < 2; ++pol) {
        size_t lds = 0;
        const void *fn = sweep_fn(cfg, pol, &lds);
        if (!fn) return hipErrorInvalidValue;
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
        }
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, cfg.threads, lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        caps[pol] = per_cu * n_cu;
    }
    // each kernel's own occupancy: the policy pass keeps more registers (the
    // argmin) and would otherwise hold the sweeps to fewer resident work-groups
    cfg.grid_cap = caps[0];
    cfg.grid_cap_pol = caps[1];
    return hipSuccess;
}

hipError_t launch_sweep(const LaunchCfg &cfg, const void *sds, SdState *st, int n_sd,
                        const WorkItem *items, WorkItem *lists, ExecCounters *cnt, int max_items,
                        int sweep, double tol, int want_policy, int *stamp,
                        int stamp_stride, int cls, int do_bookkeep, hipStream_t s) {
    size_t lds = 0;
    const void *fn = sweep_fn(cfg, want_policy, &lds);
    if (!fn) return hipErrorInvalidValue;
    int grid = max_items > 0 ? max_items : 1;
    int persistent = cfg.mode;
    const int cap = want_policy ? cfg.grid_cap_pol : cfg.grid_cap;
    if (persistent && cap > 0 && grid > cap) grid = cap;
    int local_iters = want_policy ? 0 : cfg.local_iters;
    void *args[] = {(void *)&sds, (void *)&st, (void *)&n_sd, (void *)&items, (void *)&lists,
                    (void *)&cnt, (void *)&sweep, (void *)&tol, (void *)&stamp, (void *)&stamp_stride,
                    (void *)&persistent, (void *)&cls, (void *)&do_bookkeep,
                    (void *)&local_iters};
    return hipLaunchKernel(fn, dim3(grid), dim3(cfg.threads > 0 ? cfg.threads : kThreads), args,
                           lds, s);
}

hipError_t launch_flip(SdState *st, int n_sd, hipStream_t s) {
    hipLaunchKernelGGL(k_flip, dim3(1), dim3(kThreads), 0, s, st, n_sd);
    return hipGetLastError();
}

hipError_t launch_bookkeep(SdState *st, int n_sd, int sweep, double tol, ExecCounters *cnt,
                           int final_pass, hipStream_t s, double scale_rel, int advance) {
    hipLaunchKernelGGL(k_bookkeep, dim3(1), dim3(kThreads), 0, s, st, n_sd, sweep, tol, cnt,
                       final_pass, scale_rel, advance);
    return hipGetLastError();
}

}  // namespace slhjb
