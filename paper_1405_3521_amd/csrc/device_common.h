// Device helpers shared by the sweep and adjoint kernels: explicit fused
// multiply-add (the library is built with -ffp-contract=off), foot splitting,
// FP64 block max-reduction to a residual slot, and the per-sub-domain
// convergence bookkeeping run by one work-group per launch.
#pragma once
#include "internal.h"

namespace slhjb {
namespace {

template <typename T>
__device__ __forceinline__ T fma_(T a, T b, T c);
template <>
__device__ __forceinline__ float fma_<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fma_<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One-axis interpolation (1 - f) v0 + f v1 for 0 <= f <= 1, each rounding step
// monotone in v0 and v1 and a power-of-two constant reproduced exactly (so
// iterates from the ghost value decrease to a bitwise fixed point in any update
// order).  FP64, the order the labels' reproducibility fixes:
// fma(f, v1, RN(1 - f) v0).  FP32: fma(f, v1, fma(-f, v0, v0)), where v0 (1 - f)
// is formed exactly and rounded once: two operations instead of three.  On a
// constant G = 2^k both give G RN(f + RN(1 - f)) = G.
template <typename T>
__device__ __forceinline__ T lerp_m(T f, T v0, T v1);
template <>
__device__ __forceinline__ float lerp_m<float>(float f, float v0, float v1) {
    return __builtin_fmaf(f, v1, __builtin_fmaf(-f, v0, v0));
}
template <>
__device__ __forceinline__ double lerp_m<double>(double f, double v0, double v1) {
    return __builtin_fma(f, v1, (1.0 - f) * v0);
}

template <typename T>
__device__ __forceinline__ T min_(T a, T b) { return a < b ? a : b; }

template <>
__device__ __forceinline__ float min_<float>(float a, float b) { return __builtin_fminf(a, b); }
template <>
__device__ __forceinline__ double min_<double>(double a, double b) { return __builtin_fmin(a, b); }
template <typename T>
__device__ __forceinline__ T max_(T a, T b) { return a > b ? a : b; }

// t1 / t0 for the sorted fractions 0 <= t1 <= t0 of a P1 foot, 0 when t0 = 0:
// FP64 divides exactly; FP32 multiplies by the reciprocal instruction and clamps
// to 1 (any value in [0, 1] keeps the interpolation monotone and exact on
// constants).
template <typename T>
__device__ __forceinline__ T simplex_ratio(T t1, T t0);
template <>
__device__ __forceinline__ float simplex_ratio<float>(float t1, float t0) {
    return t0 > 0.f ? min_(t1 * __builtin_amdgcn_rcpf(t0), 1.f) : 0.f;
}
template <>
__device__ __forceinline__ double simplex_ratio<double>(double t1, double t0) {
    return t0 > 0.0 ? t1 / t0 : 0.0;
}

// Read-only table in the constant address space: uniform indices then compile to
// scalar loads through the scalar data cache instead of vector memory loads (the
// displacement table is not written while a sweep kernel runs).
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ const_ptr<T> as_const(const T *p) {
    return (const_ptr<T>)(p);
}
template <>
__device__ __forceinline__ float max_<float>(float a, float b) { return __builtin_fmaxf(a, b); }
template <>
__device__ __forceinline__ double max_<double>(double a, double b) { return __builtin_fmax(a, b); }

// Split a foot coordinate into the integer cell index (tile-local, >= 0) and the
// fractional part.  FP32: local coordinate u > 0, so truncation is the floor and
// the fractional part is exact.  FP64: global coordinate (may be < 0 near the
// box), floor and subtraction exactly as the scheme's reference order.
template <typename T>
struct Foot;
template <>
struct Foot<float> {
    static __device__ __forceinline__ void split(float u, int origin, int &i, float &t) {
        (void)origin;
        i = (int)u;
        t = __builtin_amdgcn_fractf(u);
    }
};
template <>
struct Foot<double> {
    static __device__ __forceinline__ void split(double u, int origin, int &i, double &t) {
        double f = __builtin_floor(u);
        t = u - f;
        i = (int)f - origin;
    }
};

// ---- coarse grid K and fine grid G on the same box (any node counts)
// Coarse node k of an axis (n fine, nK coarse nodes) lies at fine coordinate
// k (n-1)/(nK-1) = i0 + r/(nK-1): the two fine nodes around it, the fraction, and
// the nearest fine node (ties rounded up).  Integer arithmetic except t.
struct AxisPos {
    int i0, i1, near;
    double t;
};

__device__ __forceinline__ AxisPos fine_pos_of_coarse(int k, int n, int nK) {
    const long long P = (long long)k * (n - 1);
    const int q = nK - 1;
    AxisPos a;
    a.i0 = (int)(P / q);
    const int r = (int)(P - (long long)a.i0 * q);
    a.t = (double)r / (double)q;
    a.i1 = a.i0 + 1 < n ? a.i0 + 1 : n - 1;
    a.near = a.i0 + (2 * r >= q ? 1 : 0);
    return a;
}

// Fine node j of an axis lies at coarse coordinate j (nK-1)/(n-1) = c + r/(n-1):
// the coarse cells [lo, hi] whose closure holds it and its nearest coarse node.
__device__ __forceinline__ void coarse_cells_of_fine(int j, int n, int nK, int &lo, int &hi,
                                                     int &near) {
    const long long P = (long long)j * (nK - 1);
    const int q = n - 1;
    const int c = (int)(P / q);
    const int r = (int)(P - (long long)c * q);
    hi = c < nK - 2 ? c : nK - 2;
    lo = r == 0 ? (c - 1 > 0 ? c - 1 : 0) : hi;
    near = c + (2 * r >= q ? 1 : 0);
    near = near < nK - 1 ? near : nK - 1;
}

// Q1 value of a fine node field (comps values per node, component q) at coarse
// node (ax[0], ax[1], ax[2]), in FP64: corner weights are products over the axes
// in axis order, corner terms summed in corner order from 0 (corner bit d = upper
// node on axis d).  Compiled without contraction, so the value is reproducible.
template <typename T>
__device__ __forceinline__ double sample_q1(const T *f, int comps, int q, int n0, int n1,
                                            int dim, const AxisPos *ax) {
    double acc = 0.0;
    for (int corner = 0; corner < (1 << dim); ++corner) {
        double w = 1.0;
        int id[3] = {0, 0, 0};
        for (int d = 0; d < dim; ++d) {
            const bool up = (corner >> d) & 1;
            w = w * (up ? ax[d].t : 1.0 - ax[d].t);
            id[d] = up ? ax[d].i1 : ax[d].i0;
        }
        const size_t j = ((size_t)id[2] * n1 + id[1]) * n0 + id[0];
        acc = acc + w * (double)f[j * comps + q];
    }
    return acc;
}

// Exact active-tile skipping.  With Jacobi double buffering, if no node of the
// tiles that a tile's halo reaches changed in sweep s-1, the tile's new values
// equal its old ones, and the output buffer already holds them (it holds the
// iterate of sweep s-1, equal to that of sweep s).  A tile that changes in sweep
// s therefore stamps every tile of its neighbourhood (itself included) with s+1,
// and sweep s computes exactly the tiles stamped s.  The stamps are double
// buffered by sweep parity (sweep s writes stamp[(s+1) & 1]).
//
// Active lists.  The first writer of stamp s+1 on a tile (atomic exchange) also
// appends the tile's work item to the active list of sweep s+1 (one list per
// sweep parity and halo class, its length in class_count[cls][(s+1) % 3]).
// Sweep s > 0 launches over that list only, so the work-groups that do work are
// the first ones of the grid: the hardware spreads them evenly over the compute
// units, instead of leaving them wherever they happen to fall among thousands of
// skipped tiles.  Sweep 0 takes every item of the class.
//
// Called by every lane of wave 0 of the work-group: one lane per neighbour tile.
template <int RX, int RY, int RZ>
__device__ __forceinline__ void stamp_and_list(int *next_stamp, const WorkItem &it, int off,
                                               const int *nt, int s, WorkItem *next_list,
                                               int *next_count) {
    constexpr int NX = 2 * RX + 1, NY = 2 * RY + 1, NZ = 2 * RZ + 1;
    static_assert(NX * NY * NZ <= 64, "neighbourhood larger than a wave");
    const int lane = (int)(threadIdx.x & 63);
    bool fresh = false;
    int x = 0, y = 0, z = 0, idx = 0;
    if (lane < NX * NY * NZ) {
        x = it.t[0] + lane % NX - RX;
        y = it.t[1] + (lane / NX) % NY - RY;
        z = it.t[2] + lane / (NX * NY) - RZ;
        if (x >= 0 && x < nt[0] && y >= 0 && y < nt[1] && z >= 0 && z < nt[2]) {
            idx = off + (z * nt[1] + y) * nt[0] + x;
            fresh = atomicExch(&next_stamp[idx], s) != s;
        }
    }
    const unsigned long long mask = __ballot(fresh);
    if (!mask) return;
    int base = 0;
    if (lane == 0) base = atomicAdd(next_count, (int)__popcll(mask));
    base = __shfl(base, 0, 64);
    if (fresh) {
        WorkItem w;
        w.sd = it.sd;
        w.t[0] = x;
        w.t[1] = y;
        w.t[2] = z;
        w.tflat = idx;
        w.pad[0] = w.pad[1] = w.pad[2] = 0;
        next_list[base + (int)__popcll(mask & ((1ull << lane) - 1ull))] = w;
    }
}

// The work items of sweep `sweep` of halo class `cls`: every item of the class
// (sweep 0, and passes that visit every tile), else the class's active list.
// `lists` points at the class's segment of the parity-0 list; the parity-1 list
// starts `list_stride` items later.
struct ItemList {
    const WorkItem *items;
    int n;
};
__device__ __forceinline__ ItemList sweep_items(const WorkItem *items, const WorkItem *lists,
                                                int list_stride, const ExecCounters *cnt,
                                                int cls, int sweep, bool every) {
    if (every || sweep == 0) return {items, cnt->class_items[cls]};
    return {lists + (size_t)(sweep & 1) * list_stride, cnt->class_count[cls][sweep % 3]};
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(v, off, 64);
        v = v > o ? v : o;
    }
    return v;
}

// Block max of v, folded into *dst (FP64 bit pattern, atomicMax); returns the
// block max on thread 0 (0 elsewhere).
template <int NT = kThreads>
__device__ __forceinline__ double block_max_to(double v, unsigned long long *dst) {
    __shared__ double red[NT / 64];
    __syncthreads();                    // a previous call's reader is done with red[]
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double m = 0.0;
    if (threadIdx.x == 0) {
        m = red[0];
#pragma unroll
        for (int i = 1; i < NT / 64; ++i) m = red[i] > m ? red[i] : m;
        if (m > 0.0) atomicMax(dst, (unsigned long long)__double_as_longlong(m));
    }
    return m;
}

template <int NT = kThreads>
__device__ __forceinline__ void block_sum_to(unsigned v, unsigned long long *dst) {
    __shared__ unsigned red[NT / 64];
    __syncthreads();                    // a previous call's reader is done with red[]
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < NT / 64; ++i) s += red[i];
        if (s) atomicAdd(dst, s);
    }
}

// Effective stopping tolerance of a sub-domain: tol plus, for iterations whose
// state only settles to rounding level (the atomic adjoint), scale_rel times the
// largest |state| seen in the same sweep.
__device__ __forceinline__ double eff_tol(const SdState *s, int slot, double tol,
                                          double scale_rel) {
    if (scale_rel <= 0.0) return tol;
    return tol + scale_rel * __longlong_as_double((long long)s->scale[slot]);
}

// Convergence bookkeeping before sweep `sweep` (one work-group).
__device__ void bookkeep_block(SdState *st, int n_sd, int sweep, double tol,
                               ExecCounters *cnt, int final_pass, double scale_rel = 0.0) {
    __shared__ int active;
    if (threadIdx.x == 0) active = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n_sd; i += blockDim.x) {
        SdState &s = st[i];
        if (s.conv_at < 0) {
            const int prev = (sweep + 2) % 3;
            const double r = __longlong_as_double((long long)s.res[prev]);
            if (sweep > 0 && r <= eff_tol(&s, prev, tol, scale_rel)) {
                s.conv_at = sweep - 1;
                s.final_buf = sweep & 1;
                s.done_sweeps = sweep;
                s.final_res = s.res[prev];
            } else {
                if (final_pass) {
                    s.final_buf = sweep & 1;
                    s.done_sweeps = sweep;
                    s.final_res = s.res[prev];
                }
                atomicAdd(&active, 1);
            }
        }
        s.res[(sweep + 1) % 3] = 0ull;
        s.scale[(sweep + 1) % 3] = 0ull;
    }
    __syncthreads();
    if (threadIdx.x < kMaxClasses) {
        cnt->class_queue[threadIdx.x][(sweep + 1) % 3] = 0;
        // the active lists that sweep `sweep` + 1 fills (read by `sweep` + 2)
        cnt->class_count[threadIdx.x][(sweep + 2) % 3] = 0;
    }
    if (threadIdx.x == 0) cnt->n_active = active;   // queues of the next sweep reset above
}

// Next work item of this sweep for the whole work-group (dynamic queue: one
// atomic per item, broadcast through LDS).
__device__ __forceinline__ int next_item(int *queue) {
    __shared__ int s_item;
    __syncthreads();                    // everyone has read the previous s_item
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    return s_item;
}

// Should work items of this sd be skipped at `sweep`?  Reads only data finished
// before this launch started.
__device__ __forceinline__ bool sd_skip(const SdState *s, int sweep, double tol,
                                        double scale_rel = 0.0) {
    if (s->conv_at >= 0) return true;
    if (sweep > 0) {
        const int prev = (sweep + 2) % 3;
        const double r = __longlong_as_double((long long)s->res[prev]);
        if (r <= eff_tol(s, prev, tol, scale_rel)) return true;
    }
    return false;
}

}  // namespace
}  // namespace slhjb
