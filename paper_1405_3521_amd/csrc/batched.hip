// Batched kernels: the element-wise and integer steps of the reconstruction and
// of the independent-sets algorithm for MANY problems in one launch each.
//
// Every kernel runs on a segmented grid: the blocks are split among the problems
// by a prefix array (blk_prefix[p] = first block of problem p), each block owns a
// contiguous chunk of `chunk` elements of one problem, so a block never mixes
// problems and per-problem data are read through the scalar cache.  Together
// with the sweep launches over the joint (problem, set, tile) work list, a batch
// of problems of very different sizes is solved with a fixed number of launches
// per step, independent of the number of problems.
#include "device_common.h"

#include <climits>

namespace slhjb {
namespace {

constexpr int kB = 256;

struct Seg {
    int p;
    size_t begin, end;
};

__device__ __forceinline__ Seg segment(const int *blk_prefix, int np, int chunk, size_t len_of_p_dummy) {
    (void)len_of_p_dummy;
    int lo = 0, hi = np - 1;
    const int b = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk_prefix[mid] <= b) lo = mid; else hi = mid - 1;
    }
    Seg s;
    s.p = lo;
    s.begin = (size_t)(b - blk_prefix[lo]) * chunk;
    s.end = s.begin + chunk;
    return s;
}

template <typename T>
__global__ __launch_bounds__(kB) void k_b_stats(const ProbDesc<T> *pd, const int *blkp, int np,
                                                int chunk) {
    const Seg sg = segment(blkp, np, chunk, 0);
    const ProbDesc<T> &d = pd[sg.p];
    const size_t end = sg.end < d.N ? sg.end : d.N;
    double smax = 0.0, cmax = 0.0, dmax = 0.0;
    int bad_s = 0, bad_c = 0, ntar = 0, bad_t = 0;
    int first[SL_MAX_COMP];
#pragma unroll
    for (int c = 0; c < SL_MAX_COMP; ++c) first[c] = INT_MAX;
    for (size_t i = sg.begin + threadIdx.x; i < end; i += kB) {
        if (d.speed) {
            for (int c = 0; c < d.scomp; ++c) {
                const double v = (double)d.speed[i * d.scomp + c];
                if (!(v >= 0.0) || !(v < INFINITY)) ++bad_s; else smax = v > smax ? v : smax;
            }
        }
        if (d.cost) {
            const double v = (double)d.cost[i];
            if (!(v > 0.0) || !(v < INFINITY)) ++bad_c; else cmax = v > cmax ? v : cmax;
        }
        if (d.drift) {
            for (int c = 0; c < d.dim; ++c) {
                const double v = __builtin_fabs((double)d.drift[i * d.dim + c]);
                if (!(v < INFINITY)) ++bad_s; else dmax = v > dmax ? v : dmax;
            }
        }
        const int t = d.target[i];
        if (t >= 0) {
            ++ntar;
            if (t < d.n_comp) {
#pragma unroll
                for (int c = 0; c < SL_MAX_COMP; ++c)
                    if (c == t && (int)i < first[c]) first[c] = (int)i;
            } else {
                ++bad_t;
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(smax, off, 64); smax = o > smax ? o : smax;
        o = __shfl_xor(cmax, off, 64); cmax = o > cmax ? o : cmax;
        o = __shfl_xor(dmax, off, 64); dmax = o > dmax ? o : dmax;
        bad_s += __shfl_xor(bad_s, off, 64);
        bad_c += __shfl_xor(bad_c, off, 64);
        ntar += __shfl_xor(ntar, off, 64);
        bad_t += __shfl_xor(bad_t, off, 64);
#pragma unroll
        for (int c = 0; c < SL_MAX_COMP; ++c) {
            const int f = __shfl_xor(first[c], off, 64);
            first[c] = f < first[c] ? f : first[c];
        }
    }
    if ((threadIdx.x & 63) == 0) {
        FieldStats *fs = d.fs;
        if (smax > 0.0) atomicMax(&fs->speed_max, (unsigned long long)__double_as_longlong(smax));
        if (cmax > 0.0) atomicMax(&fs->cost_max, (unsigned long long)__double_as_longlong(cmax));
        if (dmax > 0.0) atomicMax(&fs->drift_max, (unsigned long long)__double_as_longlong(dmax));
        if (bad_s) atomicAdd(&fs->bad_speed, bad_s);
        if (bad_c) atomicAdd(&fs->bad_cost, bad_c);
        if (ntar) atomicAdd(&fs->n_target, ntar);
        if (bad_t) atomicAdd(&fs->bad_target, bad_t);
        for (int c = 0; c < d.n_comp; ++c)
            if (first[c] != INT_MAX) atomicMin(&fs->first_node[c], first[c]);
    }
}

// Coarse data of every problem: Q1 interpolation (FP64) of speed and cost at the
// coarse nodes, the cost weighted by the coarse step's w; target id and g from the
// nearest fine node; coarse target presence per component.
template <typename T>
__global__ __launch_bounds__(kB) void k_b_coarse_prep(const ProbDesc<T> *pd, const int *blkp,
                                                      int np, int chunk) {
    const Seg sg = segment(blkp, np, chunk, 0);
    const ProbDesc<T> &d = pd[sg.p];
    const size_t end = sg.end < d.NK ? sg.end : d.NK;
    for (size_t k = sg.begin + threadIdx.x; k < end; k += kB) {
        AxisPos ax[3];
        ax[0] = fine_pos_of_coarse((int)(k % d.nK[0]), d.n[0], d.nK[0]);
        ax[1] = fine_pos_of_coarse((int)((k / d.nK[0]) % d.nK[1]), d.n[1], d.nK[1]);
        ax[2] = d.dim == 3 ? fine_pos_of_coarse((int)(k / ((size_t)d.nK[0] * d.nK[1])), d.n[2], d.nK[2])
                           : AxisPos{0, 0, 0, 0.0};
        const size_t j = ((size_t)ax[2].near * d.n[1] + ax[1].near) * d.n[0] + ax[0].near;
        const int t = d.target[j];
        d.tK[k] = (int8_t)t;
        if (d.speed)
            for (int c = 0; c < d.scomp; ++c)
                d.cK[k * d.scomp + c] = 1.0 * sample_q1(d.speed, d.scomp, c, d.n[0], d.n[1], d.dim, ax);
        // drift: Q1 samples, then index units of the coarse step (FP64 products)
        if (d.drift)
            for (int c = 0; c < d.dim; ++c)
                d.qK[k * d.dim + c] = d.utK[c] * (1.0 * sample_q1(d.drift, d.dim, c, d.n[0], d.n[1], d.dim, ax));
        if (d.cost) d.wlK[k] = d.wK * sample_q1(d.cost, 1, 0, d.n[0], d.n[1], d.dim, ax);
        if (d.g) d.gK[k] = (double)d.g[j];
        if (t >= 0 && t < d.n_comp) atomicMin(&d.fsK->first_node[t], (int)k);
    }
}

template <typename T>
__global__ void k_b_place_missing(const ProbDesc<T> *pd, int np) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const ProbDesc<T> &d = pd[p];
    for (int i = 0; i < d.n_comp; ++i) {
        if (d.fsK->first_node[i] != INT_MAX) continue;
        const int j = d.fs->first_node[i];
        if (j == INT_MAX) continue;
        const int a = j % d.n[0], b = (j / d.n[0]) % d.n[1], c = j / (d.n[0] * d.n[1]);
        int lo, hi, ka, kb, kc = 0;
        coarse_cells_of_fine(a, d.n[0], d.nK[0], lo, hi, ka);
        coarse_cells_of_fine(b, d.n[1], d.nK[1], lo, hi, kb);
        if (d.dim == 3) coarse_cells_of_fine(c, d.n[2], d.nK[2], lo, hi, kc);
        const size_t jk = ((size_t)kc * d.nK[1] + kb) * d.nK[0] + ka;
        if (d.tK[jk] < 0) {
            d.tK[jk] = (int8_t)i;
            if (d.gK) d.gK[jk] = d.g ? (double)d.g[j] : 0.0;
        }
    }
}

// Auxiliary problem i of problem p: component i at g, other targets and free
// nodes at the ghost value; both Jacobi buffers.
template <typename T>
__global__ __launch_bounds__(kB) void k_b_init_aux(const ProbDesc<T> *pd, const int *blkp,
                                                   int np, int chunk) {
    const Seg sg = segment(blkp, np, chunk, 0);
    const ProbDesc<T> &d = pd[sg.p];
    const size_t len = (size_t)d.n_comp * d.NK;
    const size_t end = sg.end < len ? sg.end : len;
    for (size_t q = sg.begin + threadIdx.x; q < end; q += kB) {
        const int i = (int)(q / d.NK);
        const size_t k = q - (size_t)i * d.NK;
        const int t = d.tK[k];
        const double v = (t == i) ? (d.gK ? d.gK[k] : 0.0) : d.G;
        double *V0 = d.Vaux + (size_t)i * 2 * d.NK;
        V0[k] = v;
        V0[d.NK + k] = v;
    }
}

// RA steps 2-3 of every problem, reading the final auxiliary iterates from the
// coarse sub-domains' state.
template <typename T>
__global__ __launch_bounds__(kB) void k_b_combine(const ProbDesc<T> *pd, const SdDesc<double> *sdsK,
                                                  const SdState *stK, const int *blkp, int np,
                                                  int chunk) {
    const Seg sg = segment(blkp, np, chunk, 0);
    const ProbDesc<T> &d = pd[sg.p];
    const size_t end = sg.end < d.NK ? sg.end : d.NK;
    const int sd0 = d.sd_coarse0;
    for (size_t z = sg.begin + threadIdx.x; z < end; z += kB) {
        double V = sdsK[sd0].V[stK[sd0].final_buf][z];
        for (int i = 1; i < d.n_comp; ++i) {
            const double v = sdsK[sd0 + i].V[stK[sd0 + i].final_buf][z];
            V = v < V ? v : V;
        }
        const int t = d.tK[z];
        unsigned bits = 0;
        int label = 255;
        for (int i = d.n_comp - 1; i >= 0; --i) {
            const double v = sdsK[sd0 + i].V[stK[sd0 + i].final_buf][z];
            if (t == i || __builtin_fabs(v - V) <= d.delta) bits |= 1u << i;
            if (v == V) label = i;
        }
        d.memberK[z] = (uint8_t)bits;
        d.labelK[z] = (uint8_t)label;
    }
}

// ISA step 2 of every problem (Con(.) projection, orphan repair, label) and the
// fine initial values / cost weights.
template <typename T>
__global__ __launch_bounds__(kB) void k_b_project_init(const ProbDesc<T> *pd, const int *blkp,
                                                       int np, int chunk) {
    const Seg sg = segment(blkp, np, chunk, 0);
    const ProbDesc<T> &d = pd[sg.p];
    const size_t end = sg.end < d.N ? sg.end : d.N;
    const int dim = d.dim;
    const int k0 = d.nK[0], k1 = d.nK[1];
    for (size_t j = sg.begin + threadIdx.x; j < end; j += kB) {
        const int a = (int)(j % d.n[0]);
        const int b = (int)((j / d.n[0]) % d.n[1]);
        const int c = (int)(j / ((size_t)d.n[0] * d.n[1]));
        int lo[3], hi[3], nr[3];
        coarse_cells_of_fine(a, d.n[0], k0, lo[0], hi[0], nr[0]);
        coarse_cells_of_fine(b, d.n[1], k1, lo[1], hi[1], nr[1]);
        if (dim == 3) coarse_cells_of_fine(c, d.n[2], d.nK[2], lo[2], hi[2], nr[2]);
        else lo[2] = hi[2] = nr[2] = 0;
        unsigned full = 0, anyb = 0;
        for (int ch = 0; ch < (1 << dim); ++ch) {
            const int ca = (ch & 1) ? hi[0] : lo[0];
            const int cb = (ch & 2) ? hi[1] : lo[1];
            const int cc = (ch & 4) ? hi[2] : lo[2];
            unsigned andb = 0xFFu;
            for (int q = 0; q < (1 << dim); ++q) {
                const unsigned v = d.memberK[((size_t)(cc + ((q >> 2) & 1)) * k1 +
                                              (cb + ((q >> 1) & 1))) * k0 + ca + (q & 1)];
                andb &= v;
                anyb |= v;
            }
            full |= andb;
        }
        const unsigned bits = full ? full : anyb;
        d.member[j] = (uint8_t)bits;
        d.label[j] = d.labelK[((size_t)nr[2] * k1 + nr[1]) * k0 + nr[0]];
        // fine initial values (targets at g, others at the ghost value) in every
        // set's two buffers, and the per-node cost weight
        const T v = d.target[j] >= 0 ? (d.g ? d.g[j] : T(0)) : (T)d.G;
        for (int i = 0; i < d.n_comp; ++i) {
            T *V0 = d.Vf + (size_t)i * 2 * d.N;
            V0[j] = v;
            V0[d.N + j] = v;
        }
        if (d.cost) d.wl[j] = (T)(d.w * (double)d.cost[j]);
        if (d.drift)
            for (int q = 0; q < dim; ++q)
                d.q[j * dim + q] = (T)(d.ut[q] * (double)d.drift[j * dim + q]);
    }
}

// ISA step 4 of every problem.
template <typename T>
__global__ __launch_bounds__(kB) void k_b_assemble(const ProbDesc<T> *pd, const SdDesc<T> *sds,
                                                   const SdState *st, const int *blkp, int np,
                                                   int chunk) {
    const Seg sg = segment(blkp, np, chunk, 0);
    const ProbDesc<T> &d = pd[sg.p];
    const size_t end = sg.end < d.N ? sg.end : d.N;
    const int sd0 = d.sd_fine0;
    for (size_t j = sg.begin + threadIdx.x; j < end; j += kB) {
        const unsigned bits = d.member[j];
        T best = (T)INFINITY;
        int arg = 255;
        for (int i = 0; i < d.n_comp; ++i) {
            if (!((bits >> i) & 1)) continue;
            const T v = sds[sd0 + i].V[st[sd0 + i].final_buf][j];
            if (v < best) {
                best = v;
                arg = i;
            }
        }
        d.V[j] = arg == 255 ? (T)d.G : best;
        if (d.owner) d.owner[j] = (uint8_t)arg;
    }
}

}  // namespace

template <typename T>
hipError_t launch_batched(int op, const ProbDesc<T> *pd, int np, const int *blkp, int nblocks,
                          int chunk, const void *sds, const SdState *st, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    const dim3 g(nblocks), b(kB);
    switch (op) {
    case kBatchStats: hipLaunchKernelGGL(k_b_stats<T>, g, b, 0, s, pd, blkp, np, chunk); break;
    case kBatchCoarsePrep: hipLaunchKernelGGL(k_b_coarse_prep<T>, g, b, 0, s, pd, blkp, np, chunk); break;
    case kBatchPlace: hipLaunchKernelGGL(k_b_place_missing<T>, dim3((np + 63) / 64), dim3(64), 0, s, pd, np); break;
    case kBatchInitAux: hipLaunchKernelGGL(k_b_init_aux<T>, g, b, 0, s, pd, blkp, np, chunk); break;
    case kBatchCombine:
        hipLaunchKernelGGL(k_b_combine<T>, g, b, 0, s, pd, (const SdDesc<double> *)sds, st, blkp, np, chunk);
        break;
    case kBatchProjectInit: hipLaunchKernelGGL(k_b_project_init<T>, g, b, 0, s, pd, blkp, np, chunk); break;
    case kBatchAssemble:
        hipLaunchKernelGGL(k_b_assemble<T>, g, b, 0, s, pd, (const SdDesc<T> *)sds, st, blkp, np, chunk);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_batched<float>(int, const ProbDesc<float> *, int, const int *, int, int, const void *, const SdState *, hipStream_t);
template hipError_t launch_batched<double>(int, const ProbDesc<double> *, int, const int *, int, int, const void *, const SdState *, hipStream_t);

}  // namespace slhjb
