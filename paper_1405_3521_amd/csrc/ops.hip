// Element-wise and integer kernels around the sweeps: initial values, coarse-grid
// gathers, the reconstruction algorithm's combine/threshold step, the Con(.)
// projection to the fine grid, the min-assembly of the sub-domain values and the
// construction of the (sub-domain, tile) work list.  All are streaming kernels
// (HBM/L2 bound); grid-stride loops with 256-thread work-groups.
#include "device_common.h"

#include <climits>

namespace slhjb {

namespace {

constexpr int kOpThreads = 256;

inline int grid_for(size_t n) {
    size_t g = (n + kOpThreads - 1) / kOpThreads;
    if (g > 65536) g = 65536;
    return g > 0 ? (int)g : 1;
}

template <typename T>
__global__ void k_fill(T *dst, T v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = v;
}

template <typename Tin, typename Tout>
__global__ void k_scale_field(const Tin *src, Tout *dst, size_t n, double scale) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double v = src ? (double)src[i] : 1.0;
        dst[i] = (Tout)(scale * v);
    }
}

template <typename T>
__global__ void k_absmax(const T *src, size_t n, unsigned long long *out) {
    double m = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        double v = __builtin_fabs((double)src[i]);
        if (!(v == v)) v = INFINITY;             // NaN -> reported as +inf
        m = v > m ? v : m;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0 && m > 0.0)
        atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// Input statistics in one pass: max |speed| and |drift|, max cost, counts of bad
// values (speed < 0, cost <= 0, non-finite), target counts, lowest node index per
// target component, target ids out of range.
template <typename T>
__global__ void k_field_stats(const T *speed, int speed_comps, const T *cost, const T *drift,
                              int dim, const int8_t *target, size_t n, int n_comp,
                              FieldStats *fs) {
    double smax = 0.0, cmax = 0.0, dmax = 0.0;
    int bad_s = 0, bad_c = 0, ntar = 0, bad_t = 0;
    int first[SL_MAX_COMP];
#pragma unroll
    for (int c = 0; c < SL_MAX_COMP; ++c) first[c] = INT_MAX;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if (speed) {
            for (int c = 0; c < speed_comps; ++c) {
                const double v = (double)speed[i * speed_comps + c];
                if (!(v >= 0.0) || !(v < INFINITY)) ++bad_s; else smax = v > smax ? v : smax;
            }
        }
        if (cost) {
            const double v = (double)cost[i];
            if (!(v > 0.0) || !(v < INFINITY)) ++bad_c; else cmax = v > cmax ? v : cmax;
        }
        if (drift) {
            for (int d = 0; d < dim; ++d) {
                const double v = __builtin_fabs((double)drift[i * dim + d]);
                if (!(v < INFINITY)) ++bad_s; else dmax = v > dmax ? v : dmax;
            }
        }
        const int t = target[i];
        if (t >= 0) {
            ++ntar;
            if (t < n_comp) {
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
    // combine the work-group's waves in LDS, then one thread per work-group
    // publishes (few same-address atomics)
    constexpr int NW = kOpThreads / 64;
    __shared__ double r_s[NW], r_c[NW], r_d[NW];
    __shared__ int r_bs[NW], r_bc[NW], r_nt[NW], r_bt[NW], r_f[NW][SL_MAX_COMP];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        r_s[w] = smax;
        r_c[w] = cmax;
        r_d[w] = dmax;
        r_bs[w] = bad_s;
        r_bc[w] = bad_c;
        r_nt[w] = ntar;
        r_bt[w] = bad_t;
        for (int c = 0; c < SL_MAX_COMP; ++c) r_f[w][c] = first[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < NW; ++k) {
            smax = r_s[k] > smax ? r_s[k] : smax;
            cmax = r_c[k] > cmax ? r_c[k] : cmax;
            dmax = r_d[k] > dmax ? r_d[k] : dmax;
            bad_s += r_bs[k];
            bad_c += r_bc[k];
            ntar += r_nt[k];
            bad_t += r_bt[k];
            for (int c = 0; c < SL_MAX_COMP; ++c) first[c] = r_f[k][c] < first[c] ? r_f[k][c] : first[c];
        }
        if (smax > 0.0) atomicMax(&fs->speed_max, (unsigned long long)__double_as_longlong(smax));
        if (cmax > 0.0) atomicMax(&fs->cost_max, (unsigned long long)__double_as_longlong(cmax));
        if (dmax > 0.0) atomicMax(&fs->drift_max, (unsigned long long)__double_as_longlong(dmax));
        if (bad_s) atomicAdd(&fs->bad_speed, bad_s);
        if (bad_c) atomicAdd(&fs->bad_cost, bad_c);
        if (ntar) atomicAdd(&fs->n_target, ntar);
        if (bad_t) atomicAdd(&fs->bad_target, bad_t);
        for (int c = 0; c < n_comp; ++c)
            if (first[c] != INT_MAX) atomicMin(&fs->first_node[c], first[c]);
    }
}

__global__ void k_target_scan(const int8_t *target, size_t n, int n_comp, int *count,
                              int *first_node) {
    int local = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int t = target[i];
        if (t >= 0) {
            ++local;
            if (t < n_comp) atomicMin(&first_node[t], (int)i);
        }
    }
    if (local) atomicAdd(count, local);
}

template <typename T>
__global__ void k_abs_max(const T *x, size_t n, unsigned long long *dst) {
    double m = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double a = __builtin_fabs((double)x[i]);
        m = a > m ? a : m;
    }
    block_max_to<kOpThreads>(m, dst);
}

// Initial iterate of gridDim.y consecutive grids of n nodes (grid r at V + r n):
// g on the target nodes of component c (of every component when c < 0), v_ghost
// elsewhere; c = comp, or c = r / 2 with comp_by_pair (the two buffers of
// auxiliary problem r / 2).
template <typename T>
__global__ void k_init_values(T *V, const int8_t *target, const T *g, T G, int comp,
                              int comp_by_pair, size_t n) {
    const int c = comp_by_pair ? (int)(blockIdx.y >> 1) : comp;
    T *__restrict__ Vr = V + (size_t)blockIdx.y * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int t = target[i];
        T v = G;
        if (t >= 0 && (c < 0 || t == c)) v = g ? g[i] : T(0);
        Vr[i] = v;
    }
}

// Work items of the tiled sds.  Each wave takes kBuildTilesPerWave consecutive
// (sd, tile) pairs and OR-reduces the member bit over each tile's nodes; a tile
// with a member node (every tile of an sd without a member mask) becomes an item
// of its sd's halo class.  The work-group reserves the slots of all its items
// with one global atomic per class (a single counter per class takes every
// append, so one atomic per tile would serialize the whole build on it).
constexpr int kBuildTilesPerWave = 4;
constexpr int kBuildTilesPerBlock = kBuildTilesPerWave * (kOpThreads / 64);

template <typename T>
__global__ void k_build_items(const SdDesc<T> *sds, int n_sd, int total_tiles,
                              const int *tile_prefix, int tx, int ty, int tz,
                              WorkItem *items, ExecCounters *cnt, const int *class_off) {
    __shared__ int s_count[kMaxClasses], s_base[kMaxClasses];
    __shared__ int s_slot[kBuildTilesPerBlock];        // class slot, -1: not an item
    __shared__ WorkItem s_item[kBuildTilesPerBlock];
    __shared__ int s_cls[kBuildTilesPerBlock];
    if (threadIdx.x < kMaxClasses) s_count[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int t = 0; t < kBuildTilesPerWave; ++t) {
        const int k = wave * kBuildTilesPerWave + t;          // tile of this block
        const int g = blockIdx.x * kBuildTilesPerBlock + k;
        if (g >= total_tiles) {
            if (lane == 0) s_slot[k] = -1;
            continue;
        }
        // binary search the sd owning tile g
        int lo = 0, hi = n_sd - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tile_prefix[mid] <= g) lo = mid; else hi = mid - 1;
        }
        const int sd = lo;
        const SdDesc<T> &d = sds[sd];
        const int local = g - tile_prefix[sd];
        const int t0 = local % d.tiles[0];
        const int t1 = (local / d.tiles[0]) % d.tiles[1];
        const int t2 = local / (d.tiles[0] * d.tiles[1]);
        bool hit = true;
        if (d.member) {
            const int cnt_nodes = tx * ty * tz;
            int mine = 0;
            for (int q = lane; q < cnt_nodes; q += 64) {
                const int lx = q % tx, ly = (q / tx) % ty, lz = q / (tx * ty);
                const int gx = t0 * tx + lx, gy = t1 * ty + ly, gz = t2 * tz + lz;
                if (gx < d.n[0] && gy < d.n[1] && gz < d.n[2]) {
                    const size_t j = ((size_t)gz * d.n[1] + gy) * d.n[0] + gx;
                    mine |= (d.member[j] >> d.bit) & 1;
                }
            }
            hit = __any(mine);
        }
        if (lane == 0) {
            s_slot[k] = hit ? atomicAdd(&s_count[d.cls], 1) : -1;
            s_cls[k] = d.cls;
            WorkItem w;
            w.sd = sd;
            w.t[0] = t0;
            w.t[1] = t1;
            w.t[2] = t2;
            w.tflat = g;
            w.pad[0] = w.pad[1] = w.pad[2] = 0;
            s_item[k] = w;
        }
    }
    __syncthreads();
    if (threadIdx.x < kMaxClasses && s_count[threadIdx.x] > 0)
        s_base[threadIdx.x] = atomicAdd(&cnt->class_items[threadIdx.x], s_count[threadIdx.x]);
    __syncthreads();
    if (threadIdx.x < kBuildTilesPerBlock && s_slot[threadIdx.x] >= 0) {
        const int c = s_cls[threadIdx.x];
        items[class_off[c] + s_base[c] + s_slot[threadIdx.x]] = s_item[threadIdx.x];
    }
}

// Coarse data of the RA: Q1 interpolation (FP64) of a fine field at every coarse
// node, times `scale` (1 for speed, the coarse step's w for the cost).
template <typename T>
__global__ void k_sample_coarse(const T *src, double *dst, int n0, int n1, int n2, int k0,
                                int k1, int k2, int dim, int comps, double scale) {
    const size_t NK = (size_t)k0 * k1 * k2;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < NK;
         i += (size_t)gridDim.x * blockDim.x) {
        AxisPos ax[3];
        ax[0] = fine_pos_of_coarse((int)(i % k0), n0, k0);
        ax[1] = fine_pos_of_coarse((int)((i / k0) % k1), n1, k1);
        ax[2] = dim == 3 ? fine_pos_of_coarse((int)(i / ((size_t)k0 * k1)), n2, k2) : AxisPos{0, 0, 0, 0.0};
        for (int q = 0; q < comps; ++q)
            dst[i * comps + q] = scale * sample_q1(src, comps, q, n0, n1, dim, ax);
    }
}

// Drift in index units: dst[j*dim + d] = t_d * src[j*dim + d] (FP64 product; src
// and dst may be the same array).
template <typename T>
__global__ void k_scale_drift(const T *src, T *dst, size_t N, int dim, double t0, double t1,
                              double t2) {
    const size_t n = N * (size_t)dim;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int d = (int)(i % (size_t)dim);
        const double t = d == 0 ? t0 : (d == 1 ? t1 : t2);
        dst[i] = (T)(t * (double)src[i]);
    }
}

// Discrete coarse data (target ids, exit costs): the value at the nearest fine node.
template <typename T>
__global__ void k_gather_nearest(const T *src, T *dst, int n0, int n1, int n2, int k0, int k1,
                                 int k2, int dim) {
    const size_t NK = (size_t)k0 * k1 * k2;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < NK;
         i += (size_t)gridDim.x * blockDim.x) {
        const int a = fine_pos_of_coarse((int)(i % k0), n0, k0).near;
        const int b = fine_pos_of_coarse((int)((i / k0) % k1), n1, k1).near;
        const int c = dim == 3 ? fine_pos_of_coarse((int)(i / ((size_t)k0 * k1)), n2, k2).near : 0;
        dst[i] = src[((size_t)c * n1 + b) * n0 + a];
    }
}

// Components with no coarse node get the coarse node nearest to their
// lowest-index fine node (components in index order; an occupied coarse node is
// not taken over).  firstK: lowest coarse node per component (or INT_MAX).
template <typename T>
__global__ void k_place_missing(int8_t *tK, T *gK, const T *g, const int *first_fine,
                                const int *firstK, int n0, int n1, int n2, int k0, int k1,
                                int k2, int dim, int n_comp) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = 0; i < n_comp; ++i) {
        if (firstK[i] != 0x7fffffff) continue;
        const int j = first_fine[i];
        if (j == 0x7fffffff) continue;
        const int a = j % n0, b = (j / n0) % n1, c = j / (n0 * n1);
        int lo, hi, ka, kb, kc = 0;
        coarse_cells_of_fine(a, n0, k0, lo, hi, ka);
        coarse_cells_of_fine(b, n1, k1, lo, hi, kb);
        if (dim == 3) coarse_cells_of_fine(c, n2, k2, lo, hi, kc);
        const size_t jk = ((size_t)kc * k1 + kb) * k0 + ka;
        if (tK[jk] < 0) {
            tK[jk] = (int8_t)i;
            if (gK) gK[jk] = g ? g[j] : T(0);
        }
    }
}

// RA steps 2-3 on the final auxiliary iterates (sds[i].V[st[i].final_buf]).
__global__ void k_ra_combine(const SdDesc<double> *sds, const SdState *st, int n_comp,
                             size_t NK, const int8_t *tK, double delta, uint8_t *memberK,
                             uint8_t *labelK) {
    const double *Va[SL_MAX_COMP];
#pragma unroll
    for (int i = 0; i < SL_MAX_COMP; ++i) Va[i] = i < n_comp ? sds[i].V[st[i].final_buf] : nullptr;
    for (size_t z = blockIdx.x * (size_t)blockDim.x + threadIdx.x; z < NK;
         z += (size_t)gridDim.x * blockDim.x) {
        double V = Va[0][z];
#pragma unroll
        for (int i = 1; i < SL_MAX_COMP; ++i) {
            if (i < n_comp) {
                const double v = Va[i][z];
                V = v < V ? v : V;
            }
        }
        const int t = tK[z];
        unsigned bits = 0;
        int label = 255;
#pragma unroll
        for (int i = SL_MAX_COMP - 1; i >= 0; --i) {
            if (i < n_comp) {
                const double v = Va[i][z];
                if (t == i || __builtin_fabs(v - V) <= delta) bits |= 1u << i;
                if (v == V) label = i;
            }
        }
        memberK[z] = (uint8_t)bits;
        labelK[z] = (uint8_t)label;
    }
}

__global__ void k_project(const uint8_t *mK, const uint8_t *lK, int k0, int k1, int k2,
                          int n0, int n1, int n2, int dim, uint8_t *member, uint8_t *label) {
    const size_t N = (size_t)n0 * n1 * n2;
    for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < N;
         j += (size_t)gridDim.x * blockDim.x) {
        const int a = (int)(j % n0);
        const int b = (int)((j / n0) % n1);
        const int c = (int)(j / ((size_t)n0 * n1));
        int lo[3], hi[3], nr[3];
        coarse_cells_of_fine(a, n0, k0, lo[0], hi[0], nr[0]);
        coarse_cells_of_fine(b, n1, k1, lo[1], hi[1], nr[1]);
        if (dim == 3) coarse_cells_of_fine(c, n2, k2, lo[2], hi[2], nr[2]);
        else { lo[2] = hi[2] = nr[2] = 0; }
        unsigned full = 0, anyb = 0;
        const int ncell = 1 << dim;
        for (int ch = 0; ch < ncell; ++ch) {
            const int ca = (ch & 1) ? hi[0] : lo[0];
            const int cb = (ch & 2) ? hi[1] : lo[1];
            const int cc = (ch & 4) ? hi[2] : lo[2];
            unsigned andb = 0xFFu;
            for (int q = 0; q < (1 << dim); ++q) {
                const int xa = ca + (q & 1), xb = cb + ((q >> 1) & 1), xc = cc + ((q >> 2) & 1);
                const unsigned v = mK[((size_t)xc * k1 + xb) * k0 + xa];
                andb &= v;
                anyb |= v;
            }
            full |= andb;
        }
        member[j] = (uint8_t)(full ? full : anyb);
        label[j] = lK[((size_t)nr[2] * k1 + nr[1]) * k0 + nr[0]];
    }
}

template <typename T>
__global__ void k_assemble(const SdDesc<T> *sds, const SdState *st, int n_comp,
                           const uint8_t *member, size_t N, T G, T *V, uint8_t *owner) {
    for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < N;
         j += (size_t)gridDim.x * blockDim.x) {
        const unsigned bits = member[j];
        T best = (T)INFINITY;
        int arg = 255;
        for (int i = 0; i < n_comp; ++i) {
            if (!((bits >> i) & 1)) continue;
            const T v = sds[i].V[st[i].final_buf][j];
            if (v < best) {
                best = v;
                arg = i;
            }
        }
        V[j] = arg == 255 ? G : best;
        if (owner) owner[j] = (uint8_t)arg;
    }
}

template <typename T>
__global__ void k_copy_final(const SdDesc<T> *sds, const SdState *st, int i, T *dst, size_t N) {
    const T *src = sds[i].V[st[i].final_buf];
    for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < N;
         j += (size_t)gridDim.x * blockDim.x)
        dst[j] = src[j];
}

template <typename T>
__global__ void k_count_unreached(const T *V, const int8_t *target, size_t N, T G,
                                  unsigned long long *count) {
    unsigned c = 0;
    for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < N;
         j += (size_t)gridDim.x * blockDim.x)
        c += target[j] < 0 && V[j] >= G;
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, (unsigned long long)c);
}

__global__ void k_member_counts(const uint8_t *member, size_t N, unsigned long long *counts) {
    __shared__ unsigned c[8];
    if (threadIdx.x < 8) c[threadIdx.x] = 0;
    __syncthreads();
    unsigned loc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t j = blockIdx.x * (size_t)blockDim.x + threadIdx.x; j < N;
         j += (size_t)gridDim.x * blockDim.x) {
        const unsigned b = member[j];
#pragma unroll
        for (int i = 0; i < 8; ++i) loc[i] += (b >> i) & 1;
    }
    // wave sums by shuffles, then one LDS atomic per wave and bit
#pragma unroll
    for (int i = 0; i < 8; ++i)
        for (int off = 32; off >= 1; off >>= 1) loc[i] += __shfl_xor(loc[i], off, 64);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (loc[i]) atomicAdd(&c[i], loc[i]);
    }
    __syncthreads();
    if (threadIdx.x < 8 && c[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)c[threadIdx.x]);
}

}  // namespace

template <typename T>
hipError_t launch_fill(T *dst, T v, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kOpThreads), 0, s, dst, v, n);
    return hipGetLastError();
}
template hipError_t launch_fill<float>(float *, float, size_t, hipStream_t);
template hipError_t launch_fill<double>(double *, double, size_t, hipStream_t);

template <typename Tin, typename Tout>
hipError_t launch_scale_field(const Tin *src, Tout *dst, size_t n, double scale, hipStream_t s) {
    hipLaunchKernelGGL((k_scale_field<Tin, Tout>), dim3(grid_for(n)), dim3(kOpThreads), 0, s,
                       src, dst, n, scale);
    return hipGetLastError();
}
template hipError_t launch_scale_field<float, float>(const float *, float *, size_t, double, hipStream_t);
template hipError_t launch_scale_field<float, double>(const float *, double *, size_t, double, hipStream_t);
template hipError_t launch_scale_field<double, double>(const double *, double *, size_t, double, hipStream_t);
template hipError_t launch_scale_field<double, float>(const double *, float *, size_t, double, hipStream_t);

template <typename T>
hipError_t launch_absmax(const T *src, size_t n, unsigned long long *out, hipStream_t s) {
    hipLaunchKernelGGL(k_absmax<T>, dim3(grid_for(n) < 2048 ? grid_for(n) : 2048),
                       dim3(kOpThreads), 0, s, src, n, out);
    return hipGetLastError();
}
template hipError_t launch_absmax<float>(const float *, size_t, unsigned long long *, hipStream_t);
template hipError_t launch_absmax<double>(const double *, size_t, unsigned long long *, hipStream_t);

hipError_t launch_target_scan(const int8_t *target, size_t n, int n_comp, int *count,
                              int *first_node, hipStream_t s) {
    hipLaunchKernelGGL(k_target_scan, dim3(grid_for(n) < 2048 ? grid_for(n) : 2048),
                       dim3(kOpThreads), 0, s, target, n, n_comp, count, first_node);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_abs_max(const T *x, size_t n, unsigned long long *dst, hipStream_t s) {
    const int g = grid_for(n) < 1024 ? grid_for(n) : 1024;
    hipLaunchKernelGGL(k_abs_max<T>, dim3(g), dim3(kOpThreads), 0, s, x, n, dst);
    return hipGetLastError();
}
template hipError_t launch_abs_max<float>(const float *, size_t, unsigned long long *, hipStream_t);
template hipError_t launch_abs_max<double>(const double *, size_t, unsigned long long *, hipStream_t);

template <typename T>
hipError_t launch_init_values(T *V, const int8_t *target, const T *g, T G, int comp, size_t n,
                              hipStream_t s, int reps, int comp_by_pair) {
    if (reps <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_values<T>, dim3(grid_for(n), reps), dim3(kOpThreads), 0, s, V,
                       target, g, G, comp, comp_by_pair, n);
    return hipGetLastError();
}
template hipError_t launch_init_values<float>(float *, const int8_t *, const float *, float, int, size_t, hipStream_t, int, int);
template hipError_t launch_init_values<double>(double *, const int8_t *, const double *, double, int, size_t, hipStream_t, int, int);

template <typename T>
hipError_t launch_build_items(const LaunchCfg &cfg, const SdDesc<T> *sds_dev, int n_sd,
                              int total_tiles, const int *tile_prefix_dev, WorkItem *items,
                              ExecCounters *cnt, const int *class_off, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_items<T>,
                       dim3((total_tiles + kBuildTilesPerBlock - 1) / kBuildTilesPerBlock),
                       dim3(kOpThreads), 0, s, sds_dev,
                       n_sd, total_tiles, tile_prefix_dev, cfg.tile[0], cfg.tile[1],
                       cfg.tile[2], items, cnt, class_off);
    return hipGetLastError();
}
template hipError_t launch_build_items<float>(const LaunchCfg &, const SdDesc<float> *, int, int, const int *, WorkItem *, ExecCounters *, const int *, hipStream_t);
template hipError_t launch_build_items<double>(const LaunchCfg &, const SdDesc<double> *, int, int, const int *, WorkItem *, ExecCounters *, const int *, hipStream_t);

template <typename T>
hipError_t launch_sample_coarse(const T *src, double *dst, const int *n, const int *nK, int dim,
                                int comps, double scale, hipStream_t s) {
    const size_t NK = (size_t)nK[0] * nK[1] * (dim == 3 ? nK[2] : 1);
    hipLaunchKernelGGL(k_sample_coarse<T>, dim3(grid_for(NK)), dim3(kOpThreads), 0, s, src, dst,
                       n[0], n[1], dim == 3 ? n[2] : 1, nK[0], nK[1], dim == 3 ? nK[2] : 1, dim,
                       comps, scale);
    return hipGetLastError();
}
template hipError_t launch_sample_coarse<float>(const float *, double *, const int *, const int *, int, int, double, hipStream_t);
template hipError_t launch_sample_coarse<double>(const double *, double *, const int *, const int *, int, int, double, hipStream_t);

template <typename T>
hipError_t launch_scale_drift(const T *src, T *dst, size_t N, int dim, const double *t,
                              hipStream_t s) {
    const size_t n = N * (size_t)dim;
    hipLaunchKernelGGL(k_scale_drift<T>, dim3(grid_for(n)), dim3(kOpThreads), 0, s, src, dst, N,
                       dim, t[0], t[1], t[2]);
    return hipGetLastError();
}
template hipError_t launch_scale_drift<float>(const float *, float *, size_t, int, const double *, hipStream_t);
template hipError_t launch_scale_drift<double>(const double *, double *, size_t, int, const double *, hipStream_t);

template <typename T>
hipError_t launch_gather_nearest(const T *src, T *dst, const int *n, const int *nK, int dim,
                                 hipStream_t s) {
    const size_t NK = (size_t)nK[0] * nK[1] * (dim == 3 ? nK[2] : 1);
    hipLaunchKernelGGL(k_gather_nearest<T>, dim3(grid_for(NK)), dim3(kOpThreads), 0, s, src, dst,
                       n[0], n[1], dim == 3 ? n[2] : 1, nK[0], nK[1], dim == 3 ? nK[2] : 1, dim);
    return hipGetLastError();
}
template hipError_t launch_gather_nearest<float>(const float *, float *, const int *, const int *, int, hipStream_t);
template hipError_t launch_gather_nearest<double>(const double *, double *, const int *, const int *, int, hipStream_t);
template hipError_t launch_gather_nearest<int8_t>(const int8_t *, int8_t *, const int *, const int *, int, hipStream_t);

template <typename T>
hipError_t launch_place_missing(int8_t *tK, T *gK, const T *g, const int *first_fine,
                                const int *firstK, const int *n, const int *nK, int dim,
                                int n_comp, hipStream_t s) {
    hipLaunchKernelGGL(k_place_missing<T>, dim3(1), dim3(64), 0, s, tK, gK, g, first_fine, firstK,
                       n[0], n[1], dim == 3 ? n[2] : 1, nK[0], nK[1], dim == 3 ? nK[2] : 1, dim,
                       n_comp);
    return hipGetLastError();
}
template hipError_t launch_place_missing<float>(int8_t *, float *, const float *, const int *, const int *, const int *, const int *, int, int, hipStream_t);
template hipError_t launch_place_missing<double>(int8_t *, double *, const double *, const int *, const int *, const int *, const int *, int, int, hipStream_t);

template <typename T>
hipError_t launch_field_stats(const T *speed, int speed_comps, const T *cost, const T *drift, int dim,
                              const int8_t *target, size_t n, int n_comp, FieldStats *fs,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_field_stats<T>, dim3(grid_for(n) < 512 ? grid_for(n) : 512),
                       dim3(kOpThreads), 0, s, speed, speed_comps, cost, drift, dim, target, n,
                       n_comp, fs);
    return hipGetLastError();
}
template hipError_t launch_field_stats<float>(const float *, int, const float *, const float *, int, const int8_t *, size_t, int, FieldStats *, hipStream_t);
template hipError_t launch_field_stats<double>(const double *, int, const double *, const double *, int, const int8_t *, size_t, int, FieldStats *, hipStream_t);

hipError_t launch_ra_combine(const SdDesc<double> *sds, const SdState *st, int n_comp, size_t NK,
                             const int8_t *tK, double delta, uint8_t *memberK, uint8_t *labelK,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_ra_combine, dim3(grid_for(NK)), dim3(kOpThreads), 0, s, sds, st, n_comp,
                       NK, tK, delta, memberK, labelK);
    return hipGetLastError();
}

hipError_t launch_project(const uint8_t *memberK, const uint8_t *labelK, const int *nK,
                          const int *n, int dim, uint8_t *member, uint8_t *label,
                          hipStream_t s) {
    const size_t N = (size_t)n[0] * n[1] * (dim == 3 ? n[2] : 1);
    hipLaunchKernelGGL(k_project, dim3(grid_for(N)), dim3(kOpThreads), 0, s, memberK, labelK,
                       nK[0], nK[1], dim == 3 ? nK[2] : 1, n[0], n[1], dim == 3 ? n[2] : 1, dim,
                       member, label);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_assemble(const SdDesc<T> *sds_dev, const SdState *st, int n_comp,
                           const uint8_t *member, size_t N, T G, T *V, uint8_t *owner,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_assemble<T>, dim3(grid_for(N)), dim3(kOpThreads), 0, s, sds_dev, st,
                       n_comp, member, N, G, V, owner);
    return hipGetLastError();
}
template hipError_t launch_assemble<float>(const SdDesc<float> *, const SdState *, int, const uint8_t *, size_t, float, float *, uint8_t *, hipStream_t);
template hipError_t launch_assemble<double>(const SdDesc<double> *, const SdState *, int, const uint8_t *, size_t, double, double *, uint8_t *, hipStream_t);

template <typename T>
hipError_t launch_copy_final(const SdDesc<T> *sds_dev, const SdState *st, int i, T *dst,
                             size_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_final<T>, dim3(grid_for(N)), dim3(kOpThreads), 0, s, sds_dev, st, i,
                       dst, N);
    return hipGetLastError();
}
template hipError_t launch_copy_final<float>(const SdDesc<float> *, const SdState *, int, float *, size_t, hipStream_t);
template hipError_t launch_copy_final<double>(const SdDesc<double> *, const SdState *, int, double *, size_t, hipStream_t);

hipError_t launch_member_counts(const uint8_t *member, size_t N, unsigned long long *counts8,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_member_counts, dim3(grid_for(N) < 128 ? grid_for(N) : 128),
                       dim3(kOpThreads), 0, s, member, N, counts8);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_count_unreached(const T *V, const int8_t *target, size_t N, T G,
                                  unsigned long long *count, hipStream_t s) {
    hipLaunchKernelGGL(k_count_unreached<T>, dim3(grid_for(N) < 1024 ? grid_for(N) : 1024),
                       dim3(kOpThreads), 0, s, V, target, N, G, count);
    return hipGetLastError();
}
template hipError_t launch_count_unreached<float>(const float *, const int8_t *, size_t, float, unsigned long long *, hipStream_t);
template hipError_t launch_count_unreached<double>(const double *, const int8_t *, size_t, double, unsigned long long *, hipStream_t);

}  // namespace slhjb
