// pins_launch.h -- host-side launch wrappers of the HIP kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "pins_internal.h"

namespace pins {

// Everything a launch needs to cover one batch.
struct LaunchCtx {
    hipStream_t stream;
    const DevInst* insts;  // device array [count]
    DevInst* insts_mut;    // same array, for the setup kernels that fill scales
    Ctrl* ctrl;            // device array [count]
    KP kp;
    int count;
    int max_m, max_n, max_mn;  // maxima over the batch (max_mn = max m+n)
    int max_tiles;             // max nrb*ncb
    int total_tiles, total_rowblk;  // sums over the batch (flat grids of the tile and row kernels)
    int sp_f32;                // values of S stored in float (fast-mixed precision), else double
    // CG kinds present in the batch (per instance by DevInst::cgfmt): the
    // one-block CG, the wide CG with uint16 / int32 indices; the largest m+n
    // among the one-block instances; one-block instances with m+n up to
    // PCG_SMALL_N (256-thread blocks) and above it (1024-thread blocks)
    bool any_small, any_wide16, any_wide32;
    int max_mn_small;
    bool any_tiny, any_big;
    // some one-block instance whose S may have more row pieces in a half than
    // the CG's LDS holds (the row-contiguous CG form must then be launched):
    // a half holds at most cap/64 + max(m, n) pieces (cap/4 quads in pieces of
    // up to 16 plus one shorter piece per row)
    bool any_rows_form;
};

void launch_row_lse(const LaunchCtx& L, int src, bool f32, int mask);
void launch_col_lse(const LaunchCtx& L, int src, bool f32, int mask);
void launch_col_merge(const LaunchCtx& L, int mask);
void launch_grad(const LaunchCtx& L, int src);
void launch_grad_merge(const LaunchCtx& L, bool early);  // early: only instances whose fused full step was just applied
void launch_sparsify(const LaunchCtx& L, int src);
// wide CG (instances with m+n above WCG_MAX_N, or every instance with
// matrix-free products): begin, one iteration (no-op for instances that
// stopped), end; the host repeats launch_wcg_iter until no instance has
// Ctrl::cg_on set.  src < 0: products with the sparsified Hessian, for the
// instances whose cgfmt selects the wide CG; src >= 0: matrix-free with the full
// Hessian over that cost source, for every instance
void launch_wcg_begin(const LaunchCtx& L, int src);
void launch_wcg_iter(const LaunchCtx& L, int src);  // one iteration; no per-iteration argument
void launch_wcg_end(const LaunchCtx& L, int src);
// the one-block CG of the instances with m+n <= WCG_MAX_N whose S is stored in
// the jagged-diagonal form (jds) or row-contiguous (the others)
void launch_pcg(const LaunchCtx& L, bool jds);
void launch_ls(const LaunchCtx& L, int src, bool first);
void launch_update(const LaunchCtx& L);
void launch_shift(const LaunchCtx& L, int base_src);
void launch_init(const LaunchCtx& L, int base_src);
void launch_points_cost(hipStream_t st, const double* x, const double* y, int m, int n, int d, double* C);
void launch_cost_max(const LaunchCtx& L, double* scratch, int nblk, int exponent_uses_base);
// outputs of every instance (gate = nullptr) or of those with gate[b] != 0 (device array)
void launch_final(const LaunchCtx& L, int base_src, double K, bool write_x, const int* gate = nullptr);
void launch_zero(hipStream_t st, void* p, size_t bytes);  // bytes: a multiple of 8
// device address of the fixed scratch of pins_solve_device_noalloc on `device`
// (PINS_NOALLOC_SCRATCH_BYTES bytes); PINS_OK or PINS_EDEVICE
int noalloc_scratch(int device, void** out);

}  // namespace pins
