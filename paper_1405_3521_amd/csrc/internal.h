// Internal declarations of the slhjb HIP library (not part of the C ABI).
//
// Execution model
//   A "sub-domain" (sd) is one value-iteration problem on one box grid: the
//   whole grid (global solve), one auxiliary problem of the reconstruction
//   algorithm on the coarse grid, one reconstructed set on the fine grid, or one
//   problem of a batch.  Every sweep is ONE launch over a device-built list of
//   (sd, tile) work items; each work item stages its tile plus a halo of H nodes
//   in LDS and applies the SL operator to its free member nodes (Jacobi: read
//   buffer s%2, write 1-s%2).  Per-sd residuals are max-reduced on the device
//   (FP64, atomicMax on the bit pattern); a converged sd is skipped by later
//   sweeps, so no host round trip is needed per sweep.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/slhjb.h"

namespace slhjb {

constexpr int kMaxHalo = 16;           // largest supported halo (cells), 2D
constexpr int kMaxHalo3D = 8;          // largest supported halo (cells), 3D
constexpr int kMaxClasses = 16;        // halo classes per executor (one launch each per sweep)
constexpr int kThreads = 256;          // threads per sweep work-group (4 waves)
constexpr int kMaxVariants = 32;       // sweep kernel variants of one dimension

// Per-sub-domain description (device memory, read-only during a sweep).
template <typename T>
struct SdDesc {
    T *V[2];                    // Jacobi double buffer
    const T *speed;             // per-node speed c(x) or nullptr (= 1)
    const T *wl;                // per-node w*l(x) or nullptr (= wl_const)
    const T *beta_n;            // per-node discount (Kruzkov form) or nullptr (= beta)
    const T *drift;             // per-node (h/dx)*drift, dim values per node, or nullptr
    const int8_t *target;       // per-node target id (>= 0: fixed node)
    const uint8_t *member;      // per-node set bitmask or nullptr (whole box)
    uint8_t *policy;            // per-node first minimising control (policy pass only)
    const T *ctrl;              // m*dim displacements (h/dx_d)(a_kd - b_ld), row l*m_inner + k
    T wl_const, beta, G;
    int n[3];
    int m;                      // table rows (pursuer controls x evader choices)
    int m_inner;                // pursuer controls per evader choice (= m: control problem)
    int speed_axes;             // 1: speed holds dim factors per node
    int bit;                    // member bit of this sd
    int tiles[3];               // tiles per axis
    int tile_offset;            // first global tile id of this sd
    int halo;                   // halo this sd needs
    int cls;                    // halo class (its work items live in that class's segment)
    // adjoint solves only (V[0] holds lambda; policy is the frozen forward policy)
    const T *g;                 // dL/dV per node
    const uint8_t *owner;       // set owning each node's value, or nullptr (all sets)
    int set;                    // this sd's set index (compared with owner)
    int interp;                 // sl_interp of the frozen feet's stencil
};

// Per-sub-domain convergence state (device memory).
struct SdState {
    unsigned long long res[3];  // residual slots (FP64 bit patterns, >= 0)
    int conv_at;                // sweep whose residual first met tol, -1 if none
    int final_buf;              // buffer holding the latest iterate
    int done_sweeps;            // sweeps applied to this sd
    int pad;
    unsigned long long final_res;  // residual of the last sweep (set by bookkeeping)
    unsigned long long scale[3];   // max |state| per sweep slot (adjoint: rounding level)
};

struct WorkItem {
    int sd;
    int t[3];                   // tile coordinates
    int tflat;                  // global tile index (sd's tile_offset + local index)
    int pad[3];
};

// Counters shared by a launch sequence (device memory).
struct ExecCounters {
    int n_items;                // valid work items
    int n_active;               // sds not yet converged (after the last bookkeeping)
    unsigned long long nc_updates;  // node*control evaluations
    int sweep_base;             // index of the first sweep of the current chunk
    int pad;
    int queue[3];               // unused (kept for layout)
    int pad2;
    int class_items[kMaxClasses];      // work items per halo class
    int class_queue[kMaxClasses][3];   // per-class, per-sweep work-queue heads
    int class_count[kMaxClasses][3];   // per-class, per-sweep active-list lengths
    unsigned long long n_unreached;    // free nodes left at the ghost value (after the solve)
};

// Input statistics gathered on the device in one pass (see launch_field_stats).
struct FieldStats {
    unsigned long long speed_max;   // FP64 bit patterns of non-negative maxima
    unsigned long long cost_max;
    unsigned long long drift_max;
    unsigned long long g_absmax;    // max |dL/dV| (adjoint calls)
    int bad_speed;                  // speed < 0 or non-finite, drift non-finite
    int bad_cost;                   // cost <= 0 or non-finite
    int n_target;                   // nodes with target id >= 0
    int bad_target;                 // target ids >= n_comp
    int first_node[SL_MAX_COMP];    // lowest node index per component (INT_MAX: none)
};

// Per-set description of the adjoint iteration (device memory).
template <typename T>
struct AdjDesc {
    T *lam;                     // adjoint state per node
    T *lam2;                    // second Jacobi buffer of the tile path (= lam otherwise);
                                // the set's final_buf picks the one holding the result
    T *acc[2];                  // inflow accumulators (ping-pong)
    const T *g;                 // dL/dV per node
    const uint8_t *owner;       // set owning each node's value, or nullptr (all)
    const uint8_t *policy;      // frozen control index per node (>= m: none)
    const T *speed;             // speed per node (dim per node if speed_axes) or nullptr (= 1)
    const T *drift;             // per-node drift in index units, dim per node, or nullptr
    const int8_t *target;       // target ids (>= 0: fixed, no adjoint)
    const uint8_t *member;      // set bitmask or nullptr
    const T *ctrl;              // m*dim control displacements
    T beta;
    int n[3];
    int m;
    int bit;
    int set;
    int speed_axes;             // speed holds one factor per axis
    int interp;                 // sl_interp: the feet's stencil
};

// One problem of a batch (device memory): its fine fields (caller's), its
// coarse-grid and fine-grid scratch, outputs and the indices of its first
// coarse and fine sub-domain in the joint executors.
template <typename T>
struct ProbDesc {
    int dim, n[3], nK[3], n_comp;
    size_t N, NK;
    const int8_t *target;
    const T *speed, *cost, *g;
    int8_t *tK;
    double *cK, *wlK, *gK;
    double *Vaux;               // n_comp * 2 * NK
    double wK, delta, G, w;
    uint8_t *memberK, *labelK, *member, *label, *owner;
    T *Vf;                      // n_comp * 2 * N
    T *wl;                      // N (if cost)
    T *V;                       // output
    FieldStats *fs, *fsK;
    int sd_coarse0, sd_fine0;
    // control-affine dynamics and per-axis speed
    const T *drift;             // N*dim drift or nullptr
    int scomp;                  // values per node of speed (1, or dim per-axis factors)
    double ut[3], utK[3];       // index units h/dx_d of the fine and the coarse grid
    double *qK;                 // NK*dim coarse drift in index units
    T *q;                       // N*dim fine drift in index units
};

enum BatchOp {
    kBatchStats = 0,
    kBatchCoarsePrep = 1,
    kBatchPlace = 2,
    kBatchInitAux = 3,
    kBatchCombine = 4,
    kBatchProjectInit = 5,
    kBatchAssemble = 6,
};

struct LaunchCfg {
    int dim;
    int dtype;                  // SL_F32 / SL_F64
    int tile[3];                // tile shape
    int halo;                   // H
    int variant;                // kernel variant id (autotuner)
    int grid_cap;               // resident work-groups (persistent grid), 0 = unset
    int grid_cap_pol;           // the same for the policy-pass kernel
    int mode;                   // 0: one work-group per item; 1: resident grid + atomic
                                // work queue; 2: resident grid + static grid stride
    int threads;                // work-group size of the variant
    int groups;                 // thread groups sharing a tile's controls (1: none)
    int local_iters;            // 0: Jacobi sweeps; k > 0: block-asynchronous, up to k
                                // local iterations per tile and launch (in place)
    int interp;                 // sl_interp of the kernels
};

// ---- launchers (sweep.hip) -------------------------------------------------
// One Jacobi sweep over all work items.  The sweep index is
// cnt->sweep_base + sweep_rel (device-resident base, so a captured chunk of
// launches can be replayed).
// `stamp`: 2 * stamp_stride ints, per sweep parity and tile: the sweep in which
// the tile must be computed (a tile that changes in sweep s stamps its
// neighbourhood with s + 1 in the other parity's array).
// `items` is the segment of halo class `cls` (capacity max_items); only the
// launch with do_bookkeep runs the convergence bookkeeping of the sweep.
hipError_t launch_sweep(const LaunchCfg &cfg, const void *sds, SdState *st, int n_sd,
                        const WorkItem *items, WorkItem *lists, ExecCounters *cnt, int max_items,
                        int sweep_rel, double tol, int want_policy, int *stamp,
                        int stamp_stride, int cls, int do_bookkeep, hipStream_t s);
// Bookkeeping before sweep cnt->sweep_base + sweep_rel (marks sds converged,
// resets slots, counts active sds); `final_pass` also settles final_buf of
// unconverged sds; afterwards sweep_base += advance.
hipError_t launch_bookkeep(SdState *st, int n_sd, int sweep_rel, double tol,
                           ExecCounters *cnt, int final_pass, hipStream_t s,
                           double scale_rel = 0.0, int advance = 0);
// Dynamic-LDS attributes of the kernels of `cfg` (call before graph capture);
// sets cfg.grid_cap (cfg.grid_cap_pol) to the number of resident work-groups of
// the sweep (policy-pass) kernel.
hipError_t sweep_set_attributes(LaunchCfg &cfg);
// Supported tile shapes per (dim) for the autotuner; returns count.
int sweep_variants(int dim, LaunchCfg *out, int cap);
// Whether a variant has P1 kernels.
bool sweep_has_p1(int variant);

// ---- launchers (ops.hip) ----------------------------------------------------
template <typename T>
hipError_t launch_fill(T *dst, T v, size_t n, hipStream_t s);
template <typename Tin, typename Tout>
hipError_t launch_convert(const Tin *src, Tout *dst, size_t n, Tout scale, hipStream_t s);
// dst[j] = scale * (src ? src[j] : 1)
template <typename Tin, typename Tout>
hipError_t launch_scale_field(const Tin *src, Tout *dst, size_t n, double scale, hipStream_t s);
// max over a field (non-negative values), result as double bits in *out (pre-zeroed)
template <typename T>
hipError_t launch_absmax(const T *src, size_t n, unsigned long long *out, hipStream_t s);
// count of nodes with target >= 0 (int atomic) and per-component presence bits
hipError_t launch_target_scan(const int8_t *target, size_t n, int n_comp, int *count,
                              int *first_node, hipStream_t s);
// Fold max_j |x_j| (FP64 bit pattern) into *dst with atomicMax.
template <typename T>
hipError_t launch_abs_max(const T *x, size_t n, unsigned long long *dst, hipStream_t s);
// V init for a solve, `reps` consecutive grids of n nodes: target nodes -> g (only
// those of component comp when comp >= 0; of component r / 2 in grid r with
// comp_by_pair), others -> G.
template <typename T>
hipError_t launch_init_values(T *V, const int8_t *target, const T *g, T G, int comp,
                              size_t n, hipStream_t s, int reps = 1, int comp_by_pair = 0);
// Build work items for sds whose grids are tiled with cfg.tile; sds with member
// masks only get tiles that contain a member node.
// Items of an sd go to the segment of its halo class (class_off[cls] onward).
template <typename T>
hipError_t launch_build_items(const LaunchCfg &cfg, const SdDesc<T> *sds_dev, int n_sd,
                              int total_tiles, const int *tile_prefix_dev, WorkItem *items,
                              ExecCounters *cnt, const int *class_off, hipStream_t s);
// Coarse data: Q1 interpolation (FP64) of a fine field at the coarse nodes, times
// scale; discrete data from the nearest fine node.
template <typename T>
hipError_t launch_sample_coarse(const T *src, double *dst, const int *n, const int *nK, int dim,
                                int comps, double scale, hipStream_t s);
template <typename T>
hipError_t launch_gather_nearest(const T *src, T *dst, const int *n, const int *nK, int dim,
                                 hipStream_t s);
// Drift in index units, dst = t_d * src per component (t: 3 factors).
template <typename T>
hipError_t launch_scale_drift(const T *src, T *dst, size_t N, int dim, const double *t,
                              hipStream_t s);
// Place components without a coarse node (single thread, in order).
template <typename T>
hipError_t launch_place_missing(int8_t *tK, T *gK, const T *g, const int *first_fine,
                                const int *firstK, const int *n, const int *nK, int dim,
                                int n_comp, hipStream_t s);
// One-pass input statistics (fs must be pre-initialised: zeros, first_node = INT_MAX).
template <typename T>
hipError_t launch_field_stats(const T *speed, int speed_comps, const T *cost, const T *drift, int dim,
                              const int8_t *target, size_t n, int n_comp, FieldStats *fs,
                              hipStream_t s);
// Flip final_buf of every sd (after a policy pass).
hipError_t launch_flip(SdState *st, int n_sd, hipStream_t s);
// RA steps 2-3 on K: V = min_i V_i, member bits, argmin label.
hipError_t launch_ra_combine(const SdDesc<double> *sds, const SdState *st, int n_comp, size_t NK,
                             const int8_t *tK, double delta, uint8_t *memberK, uint8_t *labelK,
                             hipStream_t s);
// ISA step 2: Con(.) projection + orphan repair + nearest-node label.
hipError_t launch_project(const uint8_t *memberK, const uint8_t *labelK, const int *nK,
                          const int *n, int dim, uint8_t *member, uint8_t *label,
                          hipStream_t s);
// ISA step 4: V = min over member sets (final buffers from SdState), owner.
template <typename T>
hipError_t launch_assemble(const SdDesc<T> *sds_dev, const SdState *st, int n_comp,
                           const uint8_t *member, size_t N, T G, T *V, uint8_t *owner,
                           hipStream_t s);
// Copy the final buffer of sd `i` to dst.
template <typename T>
hipError_t launch_copy_final(const SdDesc<T> *sds_dev, const SdState *st, int i, T *dst,
                             size_t N, hipStream_t s);
// member popcounts per bit (for set fractions)
// Free nodes whose value is still the ghost value G (no target reached), added
// to *count.
template <typename T>
hipError_t launch_count_unreached(const T *V, const int8_t *target, size_t N, T G,
                                  unsigned long long *count, hipStream_t s);
hipError_t launch_member_counts(const uint8_t *member, size_t N, unsigned long long *counts8,
                                hipStream_t s);

// ---- launchers (batched.hip) ------------------------------------------------
// One batched op over all problems; blkp[p] = first block of problem p (np+1
// entries), each block covers `chunk` elements of its problem.
template <typename T>
hipError_t launch_batched(int op, const ProbDesc<T> *pd, int np, const int *blkp, int nblocks,
                          int chunk, const void *sds, const SdState *st, hipStream_t s);

// ---- launchers (adjoint.hip) ------------------------------------------------
template <typename T>
hipError_t launch_adjoint_iter(int dim, const AdjDesc<T> *ads, SdState *st, int n_sets,
                               int blocks_per_set, ExecCounters *cnt, int iter_rel, double tol,
                               double scale_rel, hipStream_t s);
// Gather adjoint over the tile work items of an executor (2D and 3D): every
// active tile gathers lambda = g + beta P^T lambda through its transposed
// stencil, once per launch into the other buffer (local_iters = 0, Jacobi) or up
// to local_iters times in LDS, writing back in place.
template <typename T>
hipError_t launch_adjoint_tiles(const LaunchCfg &cfg, const SdDesc<T> *sds, SdState *st,
                                int n_sd, const WorkItem *items, WorkItem *lists,
                                ExecCounters *cnt, int max_items, int iter_rel, double tol,
                                double scale_rel,
                                int *stamp, int stamp_stride, int cls, int do_bookkeep,
                                hipStream_t s);
hipError_t adjoint_tiles_set_attributes(LaunchCfg &cfg);
int adjoint_tiles_max_halo(int dim);
// Tile shapes of the gather adjoint: 2D 32x8 (one node per thread), 3D 8x8x4.
constexpr int kAdjTX = 32, kAdjTY = 8;
constexpr int kAdjTX3 = 8, kAdjTY3 = 8, kAdjTZ3 = 4;
template <typename T>
hipError_t launch_adjoint_combine(const AdjDesc<T> *ads, const SdState *st, int n_sets,
                                  const int8_t *target, size_t N, T w, T *dLdl, hipStream_t s);

}  // namespace slhjb
