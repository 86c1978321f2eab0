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
        const T c = d.speed ? d.speed[j] : T(1);
        int ij[3], p[3];
        T tau[3];
        ij[0] = (int)(j % n0);
        ij[1] = (int)((j / n0) % n1);
        ij[2] = (int)(j / ((size_t)n0 * n1));
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const T disp = c * d.ctrl[DIM * k + a];
            const T f = __builtin_floor(disp);
            tau[a] = disp - f;
            p[a] = ij[a] + (int)f;
        }
        const T bl = beta * ln;
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

}  // namespace

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
