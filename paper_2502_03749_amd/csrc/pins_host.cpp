// pins_host.cpp -- C ABI of libpins.so: validation, device workspace, and the
// host sequencing of Alg. 2 (EPPA outer loop; Sinkhorn warm-up; sparse Newton
// with Sparsify, CG, Armijo line search).  Every arithmetic step of the
// method runs in the HIP kernels of pins_kernels.hip; the host only decides,
// from small control blocks read back from the device, when a batch has left
// a loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "pins.h"
#include "pins_internal.h"
#include "pins_launch.h"
#include "pins_live.h"

using namespace pins;

// Resources of one execution lane: a device workspace, a pinned staging
// area, a pool of profiling events and (for lanes > 0) its own HIP stream.
struct Lane {
    int device = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    std::vector<hipEvent_t> events;  // profiling pool, used in pairs
    std::vector<int> ev_kind;
    size_t ev_used = 0;
    bool profile = false;
    int profile_mask = 0;          // kernel classes timed (0 = all)
    hipStream_t stream = nullptr;  // owned stream (default priority)
    // fixed lane (pins_solve_device_noalloc): ws is the library's fixed device
    // scratch and host staging goes through host_buf; nothing is allocated
    bool fixed = false;
    static constexpr size_t HOST_BUF = 16384;
    alignas(256) char host_buf[HOST_BUF];
};

struct pins_ctx {
    int device = 0;
    std::string err;
    std::vector<Lane*> lanes;  // lanes[0] runs single-stream solves on the caller's stream
    Lane* fixed = nullptr;     // the no-allocation lane (created with the context)
};

namespace {

struct HipError {
    hipError_t e;
    const char* what;
};

#define HIPCHK(x)                                     \
    do {                                              \
        hipError_t e_ = (x);                          \
        if (e_ != hipSuccess) throw HipError{e_, #x}; \
    } while (0)

struct Fail {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg) { throw Fail{code, msg}; }

constexpr size_t NONE = (size_t)-1;

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += al256(bytes);
        return o;
    }
};

// Offsets of one instance's device arrays inside the workspace.
struct InstPlan {
    int m, n, d, R, nrb, ncb, cap;
    size_t loga, logb, F, G, Ah, Bh, rc, dir, cgw, part, part2, blk, blk2, hist, rowptr, col, val, colptr,
        rowT, valT, rowbin, cntr, cntc, Ck, Cpts;
    size_t C, x, y, a, b, alpha, beta, X;  // host-API staging
};

// Size class of an instance for params.tile_rows: m in [1, 64), [64, 256),
// [256, 1024), [1024, ...).
int size_class(int m) { return m < 64 ? 0 : m < 256 ? 1 : m < 1024 ? 2 : 3; }

// Rows per tile of the dense passes: params.tile_rows of the instance's class,
// 0 = the class's default (taller tiles for larger m: fewer column partials to
// merge; measured best or near it on 784-, 4096- and 16384-row grids and on
// uneven point clouds).
int tile_rows_for(const pins_params& p, int m) {
    static constexpr int def[4] = {16, 32, 32, 64};
    const int c = size_class(m), r = p.tile_rows[c];
    return r > 0 ? r : def[c];
}

long nnz_capacity(int m, int n, double budget) {
    const double lim = std::ceil(budget * (double)(m + n - 1));
    const double mn = (double)m * (double)n;
    return std::max(1L, (long)std::min(lim, mn));
}

InstPlan plan_instance(Carver& cv, const pins_problem& P, const pins_params& p, bool host_api, bool want_x) {
    InstPlan q;
    const int m = P.m, n = P.n, N = m + n;
    const size_t D = sizeof(double), I4 = sizeof(int);
    q.m = m;
    q.n = n;
    q.d = P.d;
    q.R = std::min(tile_rows_for(p, m), m);
    q.nrb = (m + q.R - 1) / q.R;
    q.ncb = (n + TILE_C - 1) / TILE_C;
    // kept entries plus up to 3 pads per row of S or S^T, rounded to quads
    q.cap = (int)(((nnz_capacity(m, n, p.budget) + 3L * std::max(m, n)) + 3) & ~3L);
    const long tiles = (long)q.nrb * q.ncb;
    // per-block parts: tiles, 4-row sweep groups, 32-entry merge blocks, and
    // (||res||^2, <res, z>) per wide-CG vector block
    const long nblk = std::max({tiles, (long)(m + 3) / 4, (long)(N + 31) / 32, 2L * ((m + WCG_VROWS - 1) / WCG_VROWS)});
    q.loga = cv.take(m * D);
    q.logb = cv.take(n * D);
    q.F = cv.take(m * D);
    q.G = cv.take(n * D);
    q.Ah = cv.take(m * D);
    q.Bh = cv.take(n * D);
    q.rc = cv.take(N * D);
    q.dir = cv.take(N * D);
    q.cgw = cv.take(4 * (size_t)N * D);
    q.part = cv.take((size_t)q.nrb * n * 2 * D);
    q.part2 = cv.take((size_t)q.ncb * m * D);
    q.blk = cv.take((size_t)nblk * LS_T * D);
    q.blk2 = cv.take((size_t)nblk * D);
    q.hist = cv.take((size_t)NLEV * I4);
    q.cntr = cv.take((size_t)m * q.ncb * I4);
    q.cntc = cv.take((size_t)q.nrb * n * I4);
    q.rowptr = cv.take((m + 1) * I4);
    q.col = cv.take((size_t)q.cap * I4);
    q.val = cv.take((size_t)q.cap * D);
    q.colptr = cv.take((n + 1) * I4);
    q.rowT = cv.take((size_t)q.cap * I4);
    q.valT = cv.take((size_t)q.cap * D);
    q.rowbin = cv.take((size_t)N * I4);
    q.Ck = (p.shift_mode == PINS_SHIFT_MATERIALIZED) ? cv.take((size_t)m * n * D) : NONE;
    q.Cpts = (P.kind == PINS_COST_POINTS) ? cv.take((size_t)m * n * D) : NONE;
    q.C = q.x = q.y = q.a = q.b = q.alpha = q.beta = q.X = NONE;
    if (host_api) {
        if (P.kind == PINS_COST_DENSE) q.C = cv.take((size_t)m * n * D);
        if (P.kind == PINS_COST_POINTS) {
            q.x = cv.take((size_t)m * P.d * D);
            q.y = cv.take((size_t)n * P.d * D);
        }
        q.a = cv.take(m * D);
        q.b = cv.take(n * D);
        q.alpha = cv.take(m * D);
        q.beta = cv.take(n * D);
        if (want_x) q.X = cv.take((size_t)m * n * D);
    }
    return q;
}

struct Batch {
    std::vector<InstPlan> plans;
    size_t insts = 0, ctrl = 0, scratch = 0, offs = 0, total = 0;
    int max_m = 0, max_n = 0, max_mn = 0, max_tiles = 0;
    std::vector<int> toff, roff;  // prefix sums of tiles and row blocks (count + 1 each)
};

constexpr int SCRATCH_BLK = 512;

// The CG an instance takes and how its S is stored (DevInst::cgfmt), from its
// sizes alone: the wide CG above WCG_MAX_N rows and columns together, with
// uint16 indices (2 bytes an entry; the wide products stream S from memory)
// when every index fits; else int32 byte offsets (no unpacking in the gather).
int cg_format(int m, int n) {
    if (m + n <= WCG_MAX_N) return 0;
    return 1 | ((m <= 65536 && n <= 65536) ? 2 : 0);
}

Batch plan_batch(const pins_problem* probs, int count, const pins_params& p, bool host_api, const pins_result* res) {
    Batch B;
    Carver cv;
    B.insts = cv.take(sizeof(DevInst) * count);
    B.ctrl = cv.take(sizeof(Ctrl) * count);
    B.scratch = cv.take(sizeof(double) * (size_t)SCRATCH_BLK * count);
    B.offs = cv.take(sizeof(int) * 2 * (size_t)(count + 1));
    B.toff.assign(1, 0);
    B.roff.assign(1, 0);
    for (int q = 0; q < count; ++q) {
        const bool want_x = host_api && res && res[q].X;
        B.plans.push_back(plan_instance(cv, probs[q], p, host_api, want_x));
        const InstPlan& P = B.plans.back();
        B.max_m = std::max(B.max_m, P.m);
        B.max_n = std::max(B.max_n, P.n);
        B.max_mn = std::max(B.max_mn, P.m + P.n);
        B.max_tiles = std::max(B.max_tiles, P.nrb * P.ncb);
        const long nt = (long)B.toff.back() + (long)P.nrb * P.ncb, nr = (long)B.roff.back() + (P.m + 3) / 4;
        if (nt > INT32_MAX || nr > INT32_MAX) fail(PINS_EINVAL, "batch too large for one launch");
        B.toff.push_back((int)nt);
        B.roff.push_back((int)nr);
    }
    B.total = cv.off;
    return B;
}

void check_params(const pins_params& p) {
    if (!(p.eta > 0.0) || !std::isfinite(p.eta)) fail(PINS_EINVAL, "eta must be positive and finite");
    if (p.max_outer < 1) fail(PINS_EINVAL, "max_outer (K) must be >= 1");
    if (p.max_sinkhorn < 0 || p.max_newton < 0 || p.cg_max_iter < 0 || p.ls_max < 1)
        fail(PINS_EINVAL, "iteration caps must be non-negative and ls_max >= 1");
    if (!(p.warm_tol >= 0.0) || !(p.inner_tol >= 0.0) || !(p.final_tol >= 0.0) || !(p.cg_rtol >= 0.0))
        fail(PINS_EINVAL, "tolerances must be non-negative");
    if (!(p.ls_beta > 0.0 && p.ls_beta < 1.0) || !(p.ls_c1 > 0.0 && p.ls_c1 < 1.0))
        fail(PINS_EINVAL, "Armijo constants must lie in (0, 1)");
    if (p.rho_levels < 1 || p.rho_levels > NLEV) fail(PINS_EINVAL, "rho_levels must be in [1, 16]");
    if (!(p.rho > 0.0) || !std::isfinite(p.rho) || !(p.budget > 0.0) || !std::isfinite(p.budget))
        fail(PINS_EINVAL, "rho and budget must be positive and finite");
    if (p.precision != PINS_FP64 && p.precision != PINS_MIXED && p.precision != PINS_MIXED_FAST)
        fail(PINS_EINVAL, "unknown precision");
    if (p.shift_mode != PINS_SHIFT_IMPLICIT && p.shift_mode != PINS_SHIFT_MATERIALIZED)
        fail(PINS_EINVAL, "unknown shift_mode");
    if (p.hvp < 0 || p.hvp > 2) fail(PINS_EINVAL, "hvp must be 0 (sparsified), 1 (matrix-free) or 2 (switch)");
    if (p.hvp_switch < 0) fail(PINS_EINVAL, "hvp_switch must be >= 0");
    for (int c = 0; c < 4; ++c)
        if (p.tile_rows[c] < 0 || p.tile_rows[c] > TILE_RMAX) fail(PINS_EINVAL, "tile_rows must be in [0, 64]");
}

void check_problem_shape(const pins_problem& P) {
    if (P.kind != PINS_COST_DENSE && P.kind != PINS_COST_POINTS && P.kind != PINS_COST_GRID)
        fail(PINS_EINVAL, "unknown cost kind");
    if (P.m < 1 || P.n < 1) fail(PINS_EINVAL, "m and n must be >= 1");
    if (P.kind == PINS_COST_GRID && (P.grid_s < 1 || P.grid_s > 46340 || P.m != P.grid_s * P.grid_s || P.n != P.m))
        fail(PINS_EINVAL, "GRID needs m = n = grid_s^2");
    if ((double)P.m * (double)P.n > 2147483647.0) fail(PINS_EUNSUPPORTED, "m*n must be below 2^31");
    if ((double)P.m + (double)P.n >= 268435456.0) fail(PINS_EUNSUPPORTED, "m+n must be below 2^28");
    if (P.kind == PINS_COST_DENSE && !P.C) fail(PINS_EINVAL, "DENSE needs C");
    if (P.kind == PINS_COST_POINTS && (!P.x || !P.y || P.d < 1)) fail(PINS_EINVAL, "POINTS needs x, y and d >= 1");
    if (!P.a || !P.b) fail(PINS_EINVAL, "a and b are required");
    if (!std::isfinite(P.cost_scale)) fail(PINS_EINVAL, "cost_scale must be finite");
}

void check_marginal(const double* v, int len, const char* name) {
    double s = 0.0;
    for (int i = 0; i < len; ++i) {
        if (!(v[i] > 0.0) || !std::isfinite(v[i])) fail(PINS_EINVAL, std::string(name) + " must be positive and finite");
        s += v[i];
    }
    if (std::fabs(s - 1.0) > 1e-10) fail(PINS_EINVAL, std::string(name) + " must sum to 1 (|sum-1| <= 1e-10)");
}

// Device descriptor of one instance whose arrays are carved at `base` by plan
// L: with host_api the inputs are copied from the host into the staging areas
// of the plan (and the outputs go to its staging areas), else the problem's
// and result's device pointers are used; a point-cloud cost is formed on the
// matrix cores into the plan's cost array.  Everything is enqueued on st.
DevInst build_inst(const InstPlan& L, const pins_problem& P, char* base, bool host_api, bool mat, const pins_result& r,
                   hipStream_t st) {
    auto Dp = [&](size_t off) { return off == NONE ? (double*)nullptr : (double*)(base + off); };
    auto Ip = [&](size_t off) { return (int*)(base + off); };
    DevInst I;
    std::memset(&I, 0, sizeof(I));
    const double *dC = P.C, *dx = P.x, *dy = P.y, *da = P.a, *db = P.b;
    if (host_api) {
        const size_t D = sizeof(double);
        if (P.kind == PINS_COST_DENSE) {
            HIPCHK(hipMemcpyAsync(Dp(L.C), P.C, D * L.m * L.n, hipMemcpyHostToDevice, st));
            dC = Dp(L.C);
        }
        if (P.kind == PINS_COST_POINTS) {
            HIPCHK(hipMemcpyAsync(Dp(L.x), P.x, D * L.m * P.d, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(Dp(L.y), P.y, D * L.n * P.d, hipMemcpyHostToDevice, st));
            dx = Dp(L.x);
            dy = Dp(L.y);
        }
        HIPCHK(hipMemcpyAsync(Dp(L.a), P.a, D * L.m, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(Dp(L.b), P.b, D * L.n, hipMemcpyHostToDevice, st));
        da = Dp(L.a);
        db = Dp(L.b);
    }
    I.m = L.m;
    I.n = L.n;
    I.grid_s = P.grid_s;
    I.R = L.R;
    I.nrb = L.nrb;
    I.ncb = L.ncb;
    I.nnz_cap = L.cap;
    I.cgfmt = cg_format(L.m, L.n);
    I.ldc = L.n;
    I.a = da;
    I.b = db;
    if (P.kind == PINS_COST_DENSE) {
        I.cbase = dC;
    } else if (P.kind == PINS_COST_POINTS) {
        I.cbase = Dp(L.Cpts);
        launch_points_cost(st, dx, dy, L.m, L.n, P.d, Dp(L.Cpts));
        HIPCHK(hipGetLastError());
    }
    if (P.cost_scale > 0.0) {
        I.bscale = P.cost_scale;
    } else if (P.kind == PINS_COST_GRID) {
        I.bscale = P.grid_s > 1 ? 1.0 / (2.0 * (double)(P.grid_s - 1) * (double)(P.grid_s - 1)) : 1.0;
    } else {
        I.bscale = -1.0;  // replaced by 1/max C on the device
    }
    I.Ck = Dp(L.Ck);
    I.csrc = mat ? I.Ck : I.cbase;
    I.cscale = mat ? 1.0 : I.bscale;
    I.loga = Dp(L.loga);
    I.logb = Dp(L.logb);
    I.F = Dp(L.F);
    I.G = Dp(L.G);
    I.Ah = Dp(L.Ah);
    I.Bh = Dp(L.Bh);
    I.rc = Dp(L.rc);
    I.d = Dp(L.dir);
    I.cgw = Dp(L.cgw);
    I.part = Dp(L.part);
    I.part2 = Dp(L.part2);
    I.blk = Dp(L.blk);
    I.blk2 = Dp(L.blk2);
    I.hist = Ip(L.hist);
    I.cntr = Ip(L.cntr);
    I.cntc = Ip(L.cntc);
    I.rowptr = Ip(L.rowptr);
    I.col = Ip(L.col);
    I.val = Dp(L.val);
    I.colptr = Ip(L.colptr);
    I.rowT = Ip(L.rowT);
    I.valT = Dp(L.valT);  // reinterpreted by the kernels per cgfmt and LaunchCtx::sp_f32
    I.rowbin = Ip(L.rowbin);
    if (host_api) {
        I.alpha = Dp(L.alpha);
        I.beta = Dp(L.beta);
        I.X = Dp(L.X);
    } else {
        I.alpha = r.alpha;
        I.beta = r.beta;
        I.X = r.X;
    }
    return I;
}

// Launch-wide facts of a batch of descriptors: sizes, flat-grid totals, the CG
// kinds present and the storage of S.
void fill_launch(LaunchCtx& L, const DevInst* hI, int count, const pins_params& p) {
    L.sp_f32 = p.precision == PINS_MIXED_FAST ? 1 : 0;
    L.any_small = L.any_wide16 = L.any_wide32 = false;
    L.any_tiny = L.any_big = L.any_rows_form = false;
    L.max_mn_small = 0;
    L.max_m = L.max_n = L.max_mn = L.max_tiles = 0;
    for (int q = 0; q < count; ++q) {
        const DevInst& I = hI[q];
        L.max_m = std::max(L.max_m, I.m);
        L.max_n = std::max(L.max_n, I.n);
        L.max_mn = std::max(L.max_mn, I.m + I.n);
        L.max_tiles = std::max(L.max_tiles, I.nrb * I.ncb);
        const int f = I.cgfmt;
        if (!(f & 1)) {
            L.any_small = true;
            L.max_mn_small = std::max(L.max_mn_small, I.m + I.n);
            if (I.m + I.n <= PCG_SMALL_N)
                L.any_tiny = true;
            else
                L.any_big = true;
            const long pieces = (long)I.nnz_cap / (4 * JDS_PQ) + std::max(I.m, I.n) + 1;
            if (pieces > pcg_parts(pcg_ept(I.m + I.n))) L.any_rows_form = true;
        } else if (f & 2) {
            L.any_wide16 = true;
        } else {
            L.any_wide32 = true;
        }
    }
}

// One event pair per launch when profiling; summed per kernel class at the end.
struct Prof {
    Lane* c;
    hipStream_t st;
    int kind = -1;
    Prof(Lane* c_, hipStream_t s, int k) : c(c_), st(s) {
        if (!c->profile || (c->profile_mask && !((c->profile_mask >> k) & 1))) return;
        kind = k;
        if (c->ev_used + 2 > c->events.size()) {
            for (int q = 0; q < 512; ++q) {
                hipEvent_t e;
                HIPCHK(hipEventCreate(&e));
                c->events.push_back(e);
            }
            c->ev_kind.resize(c->events.size() / 2);
        }
        HIPCHK(hipEventRecord(c->events[c->ev_used], st));
    }
    void end() {
        if (kind < 0) return;
        HIPCHK(hipEventRecord(c->events[c->ev_used + 1], st));
        c->ev_kind[c->ev_used / 2] = kind;
        c->ev_used += 2;
        kind = -1;
    }
};

template <class Fn>
void run_launch(Lane* c, hipStream_t st, int kind, Fn&& fn) {
    Prof pr(c, st, kind);
    fn();
    HIPCHK(hipGetLastError());
    pr.end();
}

void* pinned(Lane* c, size_t bytes) {
    if (c->fixed) {
        if (bytes > Lane::HOST_BUF) fail(PINS_ENOMEM, "host staging of the no-allocation entry point too small");
        return c->host_buf;
    }
    if (bytes > c->pinned_bytes) {
        if (c->pinned) HIPCHK(hipHostFree(c->pinned));
        c->pinned = nullptr;
        c->pinned_bytes = 0;
        HIPCHK(hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault));
        c->pinned_bytes = bytes;
    }
    return c->pinned;
}

char* workspace(Lane* c, size_t bytes) {
    if (c->fixed) {
        if (bytes > c->ws_bytes)
            fail(PINS_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes exceeds the fixed scratch of " +
                                  std::to_string(c->ws_bytes) + " bytes (PINS_NOALLOC_SCRATCH_BYTES)");
        return (char*)c->ws;
    }
    if (bytes > c->ws_bytes) {
        if (c->ws) HIPCHK(hipFree(c->ws));
        c->ws = nullptr;
        c->ws_bytes = 0;
        if (hipMalloc(&c->ws, bytes) != hipSuccess) {
            (void)hipGetLastError();
            c->ws = nullptr;
            fail(PINS_ENOMEM, "device workspace allocation failed (" + std::to_string(bytes) + " bytes)");
        }
        c->ws_bytes = bytes;
    }
    return (char*)c->ws;
}

// Read the control blocks back (synchronises the stream).
const Ctrl* readback(Lane* c, hipStream_t st, const Ctrl* d_ctrl, int count) {
    Ctrl* h = (Ctrl*)pinned(c, sizeof(Ctrl) * count + sizeof(DevInst) * count);
    HIPCHK(hipMemcpyAsync(h, d_ctrl, sizeof(Ctrl) * count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return h;
}

// The host sequencing of one outer iteration of Alg. 2 over a batch: the
// shift (when asked), the Sinkhorn warm-up and the Newton steps, until no
// instance is warming up or iterating.  Kept across the outer iterations of a
// solve (or of a live batch) for the warm-up heuristic and the captured graph.
struct GraphHolder {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    ~GraphHolder() {
        if (e) (void)hipGraphExecDestroy(e);
        if (g) (void)hipGraphDestroy(g);
    }
};

struct OuterRunner {
    Lane* ctx;
    hipStream_t st;
    const LaunchCtx& L;
    Ctrl* d_ctrl;
    int count;
    const pins_params& p;
    int src, base_src;
    bool quick_warm = false;  // every warm-up of the last outer iteration took one iteration
    bool graphs_ok = false;   // params.graphs and a batch the captured sequence covers
    GraphHolder gq;

    void run(bool mf, bool do_shift) {
        const bool f32 = p.precision != PINS_FP64;  // float warm-up sweeps
        const int M_WARM = 1 << PH_WARM, M_FB = 1 << PH_FALLBACK;
        // The launches of a Newton round up to its readback: Newton pass and merge,
        // Sparsify, the one-block CG (sparsified products; the wide CG and the
        // matrix-free products run their own loop), the first Armijo trial fused
        // with the next Newton pass, and the early merge and decision.
        auto newton_round = [&](bool mf_) {
            run_k(PINS_K_GRAD, [&] { launch_grad(L, src); });
            run_k(PINS_K_GRAD_MERGE, [&] { launch_grad_merge(L, false); });
            if (!mf_) run_k(PINS_K_FILL, [&] { launch_sparsify(L, src); });
            // sparsified products: the one-block CG for the instances with m + n <=
            // WCG_MAX_N and the wide CG for the others (the choice is each
            // instance's own); matrix-free products: the wide CG for every instance
            // (the storage form of each instance's S is chosen on the device: the
            // row-contiguous form's kernel is launched when some instance's S could
            // need it (LaunchCtx::any_rows_form), each kernel returning at once for
            // the instances stored the other way)
            if (!mf_ && L.any_small) {
                run_k(PINS_K_PCG, [&] { launch_pcg(L, true); });
                if (L.any_rows_form) run_k(PINS_K_PCG_ROWS, [&] { launch_pcg(L, false); });
            }
            if (mf_ || L.any_wide16 || L.any_wide32) {
                // wide or matrix-free CG: iterations in chunks between readbacks of cg_on
                const int hsrc = mf_ ? src : -1;
                run_k(PINS_K_PCG_WIDE, [&] { launch_wcg_begin(L, hsrc); });
                for (int chunk = 4;; chunk = std::min(2 * chunk, 32)) {
                    const Ctrl* hc = readback(ctx, st, d_ctrl, count);
                    bool on = false;
                    for (int q = 0; q < count; ++q) on |= hc[q].phase == PH_NEWTON && hc[q].cg_on;
                    if (!on) break;
                    for (int c = 0; c < chunk; ++c) run_k(PINS_K_PCG_WIDE, [&] { launch_wcg_iter(L, hsrc); });
                }
                run_k(PINS_K_PCG_WIDE, [&] { launch_wcg_end(L, hsrc); });
            }
            run_k(PINS_K_LS, [&] { launch_ls(L, src, true); });
            // instances whose full step the fused first trial applied: the next
            // gradient is formed, so merge it and take the convergence decision
            // now (a subproblem that converged in one step then needs no further
            // round of launches)
            run_k(PINS_K_GRAD_MERGE, [&] { launch_grad_merge(L, true); });
        };
        // params.graphs: an outer iteration on the quick path (a shift, the
        // previous warm-ups all took one iteration, sparsified products,
        // one-block CGs only) launches shift, one warm-up iteration and the first
        // Newton round with no readback in between; that sequence is captured
        // once as a HIP graph and replayed.  Every kernel argument is the same
        // in every outer iteration (the per-instance state lives in the control
        // blocks), so a replay runs exactly the launches the sequence would make.
        auto quick_sequence = [&] {
            run_k(PINS_K_SHIFT, [&] { launch_shift(L, base_src); });
            run_k(PINS_K_ROW_LSE, [&] { launch_row_lse(L, src, f32, M_WARM); });
            run_k(PINS_K_COL_LSE, [&] { launch_col_lse(L, src, f32, M_WARM); });
            run_k(PINS_K_COL_MERGE, [&] { launch_col_merge(L, M_WARM); });
            newton_round(false);
        };
        bool warm_unread = false, round_done = false;
        if (graphs_ok && !mf && do_shift && quick_warm) {
            if (!gq.e) {
                HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
                try {
                    quick_sequence();
                } catch (...) {
                    hipGraph_t bad = nullptr;
                    (void)hipStreamEndCapture(st, &bad);
                    if (bad) (void)hipGraphDestroy(bad);
                    throw;
                }
                HIPCHK(hipStreamEndCapture(st, &gq.g));
                HIPCHK(hipGraphInstantiate(&gq.e, gq.g, nullptr, nullptr, 0));
            }
            HIPCHK(hipGraphLaunch(gq.e, st));
            warm_unread = true;
            round_done = true;
        } else if (do_shift) {
            run_k(PINS_K_SHIFT, [&] { launch_shift(L, base_src); });
        }
        // warm-up sweeps of the instances in the warm-up phase: chunks of W
        // iterations, a readback after each, until none is left; returns the
        // number of chunks
        auto warm_loop = [&](int W) {
            int chunks = 0;
            for (;;) {
                for (int w = 0; w < W; ++w) {
                    run_k(PINS_K_ROW_LSE, [&] { launch_row_lse(L, src, f32, M_WARM); });
                    run_k(PINS_K_COL_LSE, [&] { launch_col_lse(L, src, f32, M_WARM); });
                    run_k(PINS_K_COL_MERGE, [&] { launch_col_merge(L, M_WARM); });
                }
                ++chunks;
                const Ctrl* h = readback(ctx, st, d_ctrl, count);
                bool any = false;
                for (int q = 0; q < count; ++q) any |= h[q].phase == PH_WARM;
                if (!any) return chunks;
                W = std::min(2 * W, 8);
            }
        };
        // After the shift, when every warm-up of the previous outer iteration
        // took a single iteration, one iteration is launched and the first Newton
        // round follows without a readback: the Newton kernels act only on the
        // instances that iteration moved to the Newton phase, and any still in the
        // warm-up finish it after the round's readback and join the next round.
        if (p.max_sinkhorn > 0 && !round_done) {
            if (quick_warm) {
                run_k(PINS_K_ROW_LSE, [&] { launch_row_lse(L, src, f32, M_WARM); });
                run_k(PINS_K_COL_LSE, [&] { launch_col_lse(L, src, f32, M_WARM); });
                run_k(PINS_K_COL_MERGE, [&] { launch_col_merge(L, M_WARM); });
                warm_unread = true;
            } else {
                quick_warm = warm_loop(1) == 1;
            }
        }
        // Newton steps; a readback after each (the first round may have gone out
        // with the captured sequence)
        for (;;) {
            if (!round_done) newton_round(mf);
            round_done = false;
            // one readback per Newton step: who is still iterating, who needs more
            // Armijo trials, who will take the Sinkhorn fallback
            const Ctrl* h = readback(ctx, st, d_ctrl, count);
            bool any = false, pending = false, failed = false, unapplied = false, warm = false;
            for (int q = 0; q < count; ++q) {
                any |= h[q].phase == PH_NEWTON;
                pending |= h[q].phase == PH_NEWTON && h[q].ls_state == LS_PENDING;
                failed |= h[q].phase == PH_NEWTON && h[q].ls_state == LS_FAILED;
                unapplied |= h[q].phase == PH_NEWTON && h[q].ls_state != LS_APPLIED;
                warm |= h[q].phase == PH_WARM;
            }
            if (warm_unread) {
                warm_unread = false;
                quick_warm = !warm;
            }
            if (!any && !warm) break;
            for (int hh = 1; pending && hh < p.ls_max; hh += LS_T) {
                run_k(PINS_K_LS, [&] { launch_ls(L, src, false); });
                const Ctrl* h2 = readback(ctx, st, d_ctrl, count);
                pending = false;
                for (int q = 0; q < count; ++q) {
                    pending |= h2[q].phase == PH_NEWTON && h2[q].ls_state == LS_PENDING;
                    failed |= h2[q].phase == PH_NEWTON && h2[q].ls_state == LS_FAILED;
                }
            }
            // the update (and the step's bookkeeping) of every instance whose full
            // step the fused first trial has not already applied
            if (unapplied) run_k(PINS_K_UPDATE, [&] { launch_update(L); });
            if (failed) {
                run_k(PINS_K_ROW_LSE, [&] { launch_row_lse(L, src, false, M_FB); });
                run_k(PINS_K_COL_LSE, [&] { launch_col_lse(L, src, false, M_FB); });
                run_k(PINS_K_COL_MERGE, [&] { launch_col_merge(L, M_FB); });
            }
            if (warm) warm_loop(2);  // the instances the single warm-up iteration left
        }
    }

    template <class Fn>
    void run_k(int kind, Fn&& fn) {
        run_launch(ctx, st, kind, fn);
    }
};

// A range of outer iterations for pins_solve_resume: start after
// from->outer_done completed iterations (from = nullptr: at the start), stop
// after `stop`, copy the state reached to *save when non-null.
struct ResumeIO {
    const pins_state* from;
    int stop;
    pins_state* save;
};

int solve_impl(Lane* ctx, const pins_problem* probs, int count, const pins_params& p, pins_result* res,
               hipStream_t st, bool host_api, const ResumeIO* rio = nullptr) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    if (count < 1) fail(PINS_EINVAL, "count must be >= 1");
    if (!probs || !res) fail(PINS_EINVAL, "problems and results are required");
    check_params(p);
    const bool grid0 = probs[0].kind == PINS_COST_GRID;
    for (int q = 0; q < count; ++q) {
        check_problem_shape(probs[q]);
        if ((probs[q].kind == PINS_COST_GRID) != grid0)
            fail(PINS_EUNSUPPORTED, "a batch must not mix GRID with DENSE/POINTS costs");
        if (!host_api && (!res[q].alpha || !res[q].beta)) fail(PINS_EINVAL, "res.alpha and res.beta are required");
        if (host_api && (!res[q].alpha || !res[q].beta)) fail(PINS_EINVAL, "res.alpha and res.beta are required");
    }
    HIPCHK(hipSetDevice(ctx->device));
    ctx->profile = p.profile != 0;
    if (ctx->fixed && ctx->profile) fail(PINS_EINVAL, "profiling is not available without allocation (it creates events)");
    ctx->profile_mask = p.profile_mask;
    ctx->ev_used = 0;

    // host marginals are validated here, before any copy; device marginals by
    // the set-up kernel on the solve's stream (ordered after the caller's work
    // on it), read back with the set-up's control blocks
    if (host_api)
        for (int q = 0; q < count; ++q) {
            check_marginal(probs[q].a, probs[q].m, "a");
            check_marginal(probs[q].b, probs[q].n, "b");
        }

    const Batch B = plan_batch(probs, count, p, host_api, res);
    char* ws = workspace(ctx, B.total);
    DevInst* d_insts = (DevInst*)(ws + B.insts);
    Ctrl* d_ctrl = (Ctrl*)(ws + B.ctrl);
    double* d_scratch = (double*)(ws + B.scratch);
    auto Dp = [&](size_t off) { return off == NONE ? (double*)nullptr : (double*)(ws + off); };

    const bool mat = p.shift_mode == PINS_SHIFT_MATERIALIZED;
    const int src = (grid0 && !mat) ? SRC_GRID : SRC_DENSE;  // exponent source
    const int base_src = grid0 ? SRC_GRID : SRC_DENSE;       // unshifted cost

    Prof setup(ctx, st, PINS_K_SETUP);
    std::vector<DevInst> hI(count);
    bool need_max = false;
    for (int q = 0; q < count; ++q) {
        hI[q] = build_inst(B.plans[q], probs[q], ws, host_api, mat, res[q], st);
        if (probs[q].kind != PINS_COST_GRID) need_max = true;
    }
    {
        char* pin = (char*)pinned(ctx, sizeof(Ctrl) * count + sizeof(DevInst) * count +
                                           sizeof(int) * 2 * (size_t)(count + 1));
        DevInst* h = (DevInst*)(pin + sizeof(Ctrl) * count);
        std::memcpy(h, hI.data(), sizeof(DevInst) * count);
        HIPCHK(hipMemcpyAsync(d_insts, h, sizeof(DevInst) * count, hipMemcpyHostToDevice, st));
        int* ho = (int*)(pin + sizeof(Ctrl) * count + sizeof(DevInst) * count);
        std::memcpy(ho, B.toff.data(), sizeof(int) * (count + 1));
        std::memcpy(ho + count + 1, B.roff.data(), sizeof(int) * (count + 1));
        HIPCHK(hipMemcpyAsync(ws + B.offs, ho, sizeof(int) * 2 * (count + 1), hipMemcpyHostToDevice, st));
        launch_zero(st, d_ctrl, sizeof(Ctrl) * count);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));  // the pinned staging area is reused by readback()
    }

    LaunchCtx L;
    L.stream = st;
    L.insts = d_insts;
    L.insts_mut = d_insts;
    L.ctrl = d_ctrl;
    L.count = count;
    // sizes, the CG kinds present in the batch; the CG's copy of S holds float
    // values in the fast-mixed precision only (CG vectors and sums stay double)
    fill_launch(L, hI.data(), count, p);
    L.total_tiles = B.toff.back();
    L.total_rowblk = B.roff.back();
    KP& kp = L.kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.eta = p.eta;
    kp.inv_eta = 1.0 / p.eta;
    kp.warm_tol = p.warm_tol;
    kp.inner_tol = p.inner_tol;
    kp.final_tol = p.final_tol;
    kp.K = p.max_outer;
    kp.cg_rtol = p.cg_rtol;
    kp.ls_beta = p.ls_beta;
    kp.ls_c1 = p.ls_c1;
    kp.log_rho = std::log(p.rho);
    kp.budget = p.budget;
    kp.T1 = p.max_sinkhorn;
    kp.T2 = p.max_newton;
    kp.cg_max = p.cg_max_iter;
    kp.ls_max = p.ls_max;
    kp.nlev = p.rho_levels;
    kp.shift_mode = p.shift_mode;
    kp.count = count;
    kp.toff = (const int*)(ws + B.offs);
    kp.roff = kp.toff + count + 1;

    // a0: cost scale (1/max over the dense cost unless given) and finiteness
    if (need_max) {
        launch_cost_max(L, d_scratch, SCRATCH_BLK, mat ? 0 : 1);
        HIPCHK(hipGetLastError());
    }
    launch_init(L, base_src);
    HIPCHK(hipGetLastError());
    setup.end();
    {
        const Ctrl* h = readback(ctx, st, d_ctrl, count);
        for (int q = 0; q < count; ++q) {
            const std::string at = " (instance " + std::to_string(q) + ")";
            const int mb = h[q].margbad;
            if (mb & 1) fail(PINS_EINVAL, "a must be positive and finite" + at);
            if (mb & 2) fail(PINS_EINVAL, "a must sum to 1 (|sum-1| <= 1e-10)" + at);
            if (mb & 4) fail(PINS_EINVAL, "b must be positive and finite" + at);
            if (mb & 8) fail(PINS_EINVAL, "b must sum to 1 (|sum-1| <= 1e-10)" + at);
            if (h[q].nonfinite) fail(PINS_EINVAL, "C has non-finite entries" + at);
        }
    }
    // resume: the saved (F, G, A, B), kappa = k (k + 1 after the coming shift)
    // and the earlier-subproblem flag replace what the initialisation wrote
    int k_begin = 0, k_end = p.max_outer;
    if (rio) {
        k_end = rio->stop;
        if (rio->from) {
            const pins_state& S = *rio->from;
            const InstPlan& Lp = B.plans[0];
            const size_t D = sizeof(double);
            k_begin = S.outer_done;
            const double kap = (double)S.outer_done;
            const int kprev = S.outer_done - 1;  // the coming shift advances it to outer_done
            const int done_phase = PH_DONE;      // outer iteration outer_done - 1 finished: the shift applies
            const int fl = S.flags & 2;
            HIPCHK(hipMemcpyAsync(Dp(Lp.F), S.F, D * Lp.m, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(Dp(Lp.G), S.G, D * Lp.n, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(Dp(Lp.Ah), S.A, D * Lp.m, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(Dp(Lp.Bh), S.B, D * Lp.n, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(&d_ctrl[0].kappa, &kap, sizeof(double), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(&d_ctrl[0].k_out, &kprev, sizeof(int), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(&d_ctrl[0].phase, &done_phase, sizeof(int), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(&d_ctrl[0].flags, &fl, sizeof(int), hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
    }

    // matrix-free Hessian products (no Sparsify) in outer iteration k
    auto matrix_free = [&](int k) { return p.hvp == 1 || (p.hvp == 2 && k < p.hvp_switch); };
    OuterRunner R{ctx, st, L, d_ctrl, count, p, src, base_src};
    R.graphs_ok = p.graphs && !ctx->profile && st != nullptr && L.any_small && !L.any_wide16 && !L.any_wide32 &&
                  p.max_sinkhorn > 0;
    for (int k = k_begin; k < k_end; ++k) R.run(matrix_free(k), k > 0);
    bool want_x = false;
    for (int q = 0; q < count; ++q) want_x |= hI[q].X != nullptr;
    run_launch(ctx, st, PINS_K_FINAL, [&] { launch_final(L, base_src, (double)k_end, want_x); });
    const Ctrl* h = readback(ctx, st, d_ctrl, count);
    if (rio && rio->save) {
        pins_state& S = *rio->save;
        const InstPlan& Lp = B.plans[0];
        const size_t D = sizeof(double);
        HIPCHK(hipMemcpyAsync(S.F, Dp(Lp.F), D * Lp.m, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(S.G, Dp(Lp.G), D * Lp.n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(S.A, Dp(Lp.Ah), D * Lp.m, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(S.B, Dp(Lp.Bh), D * Lp.n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        S.m = Lp.m;
        S.n = Lp.n;
        S.outer_done = k_end;
        S.flags = h[0].flags & 2;
    }

    // outputs
    if (host_api) {
        for (int q = 0; q < count; ++q) {
            const InstPlan& Lp = B.plans[q];
            HIPCHK(hipMemcpyAsync(res[q].alpha, Dp(Lp.alpha), sizeof(double) * Lp.m, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(res[q].beta, Dp(Lp.beta), sizeof(double) * Lp.n, hipMemcpyDeviceToHost, st));
            if (res[q].X)
                HIPCHK(hipMemcpyAsync(res[q].X, Dp(Lp.X), sizeof(double) * Lp.m * Lp.n, hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipStreamSynchronize(st));
    }
    double kms[PINS_NKERN] = {0};
    int kcalls[PINS_NKERN] = {0};
    if (ctx->profile) {
        HIPCHK(hipStreamSynchronize(st));
        for (size_t e = 0; e + 1 < ctx->ev_used; e += 2) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ctx->events[e], ctx->events[e + 1]));
            const int kd = ctx->ev_kind[e / 2];
            kms[kd] += ms;
            kcalls[kd] += 1;
        }
    }
    const double wall = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    int worst = PINS_OK;
    for (int q = 0; q < count; ++q) {
        pins_result& r = res[q];
        const Ctrl& S = h[q];
        r.cost = S.cost;
        r.eps = p.eta / (double)k_end;
        r.resid = S.resid;
        r.dual = S.dual;
        r.gap = S.cost - S.dual;
        r.entropy = S.entropy;
        r.cost_scale = need_max ? S.scale : hI[q].bscale;
        r.time_ms = wall;
        r.flags = S.flags | (S.nonfinite ? 4 : 0);
        r.outer_iters = k_end;
        r.sinkhorn_iters = S.sink_total;
        r.newton_iters = S.newton_total;
        r.cg_iters = S.cg_total;
        r.fallbacks = S.fb_total;
        r.nnz_last = S.nnz;
        r.status = S.nonfinite ? PINS_ENUMERIC : ((S.flags & 1) ? PINS_NOT_CONVERGED : PINS_OK);
        for (int kk = 0; kk < PINS_NKERN; ++kk) {
            r.kern_ms[kk] = kms[kk];
            r.kern_calls[kk] = kcalls[kk];
            r.kern_work[kk] = 0.0;
        }
        r.kern_work[PINS_K_ROW_LSE] = S.work[W_ROW];
        r.kern_work[PINS_K_COL_LSE] = S.work[W_COL];
        r.kern_work[PINS_K_GRAD] = S.work[W_GRAD];
        r.kern_work[PINS_K_FILL] = S.work[W_FILL];
        r.kern_work[PINS_K_PCG] = S.work[W_CG];
        r.kern_work[PINS_K_PCG_ROWS] = S.work[W_CG_ROWS];
        r.kern_work[PINS_K_PCG_WIDE] = S.work[W_CG_WIDE];
        r.kern_work[PINS_K_LS] = S.work[W_LS];
        r.kern_work[PINS_K_FINAL] = S.work[W_FINAL];
        r.group = 0;
        if (r.status < 0 && (worst >= 0 || r.status < worst)) worst = r.status;
        if (worst >= 0 && r.status > worst) worst = r.status;
    }
    return worst;
}

Lane* lane(pins_ctx* ctx, int q) {
    while ((int)ctx->lanes.size() <= q) {
        Lane* L = new Lane;
        L->device = ctx->device;
        if (!ctx->lanes.empty()) {
            HIPCHK(hipSetDevice(ctx->device));
            HIPCHK(hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking));
        }
        ctx->lanes.push_back(L);
    }
    return ctx->lanes[q];
}

void free_lane(Lane* L) {
    for (hipEvent_t e : L->events) (void)hipEventDestroy(e);
    if (L->ws && !L->fixed) (void)hipFree(L->ws);
    if (L->pinned) (void)hipHostFree(L->pinned);
    if (L->stream) (void)hipStreamDestroy(L->stream);
    delete L;
}

// Number of concurrent lanes for a batch: params.streams (0 or 1: one lane
// on the caller's stream; measured faster than automatic splitting for
// equal-size batches, whose CG phases then overlap poorly).
int lane_count(const pins_params& p, int count, bool host_api) {
    if (host_api || count < 2) return 1;
    int g = p.streams > 1 ? p.streams : 1;
    g = std::max(1, std::min({g, PINS_MAX_LANES, count}));
    return g;
}

int solve_entry(pins_ctx* ctx, const pins_problem* probs, int count, const pins_params& p, pins_result* res,
                hipStream_t st, bool host_api) {
    if (count < 1) fail(PINS_EINVAL, "count must be >= 1");
    if (!probs || !res) fail(PINS_EINVAL, "problems and results are required");
    check_params(p);
    const int G = lane_count(p, count, host_api);
    if (G == 1) return solve_impl(lane(ctx, 0), probs, count, p, res, st, host_api);
    for (int q = 0; q < count; ++q) check_problem_shape(probs[q]);
    // contiguous groups of (nearly) equal instance count
    std::vector<int> start(G + 1);
    for (int g = 0; g <= G; ++g) start[g] = (int)(((long)count * g) / G);
    // the lanes start after the caller's stream has produced the inputs
    HIPCHK(hipSetDevice(ctx->device));
    hipEvent_t ready;
    HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ready, st));
    std::vector<Lane*> L(G);
    for (int g = 0; g < G; ++g) {
        L[g] = lane(ctx, g + 1);
        HIPCHK(hipStreamWaitEvent(L[g]->stream, ready, 0));
    }
    std::vector<int> rc(G, PINS_OK);
    std::vector<std::string> msg(G);
    std::vector<std::thread> th;
    for (int g = 0; g < G; ++g) {
        const int a = start[g], b = start[g + 1];
        if (a >= b) continue;
        th.emplace_back([&, g, a, b] {
            try {
                HIPCHK(hipSetDevice(ctx->device));
                rc[g] = solve_impl(L[g], probs + a, b - a, p, res + a, L[g]->stream, false);
                for (int q = a; q < b; ++q) res[q].group = g;
            } catch (const Fail& f) {
                rc[g] = f.code;
                msg[g] = f.msg;
            } catch (const HipError& e) {
                rc[g] = PINS_EDEVICE;
                msg[g] = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.what;
            } catch (...) {
                rc[g] = PINS_EDEVICE;
                msg[g] = "unexpected internal error";
            }
        });
    }
    for (auto& t : th) t.join();
    (void)hipEventDestroy(ready);
    int worst = PINS_OK;
    for (int g = 0; g < G; ++g) {
        if (rc[g] < 0) fail(rc[g], msg[g]);
        worst = std::max(worst, rc[g]);
    }
    return worst;
}

template <class Fn>
int guarded(pins_ctx* ctx, Fn&& fn) {
    if (!ctx) return PINS_EINVAL;
    try {
        ctx->err.clear();
        return fn();
    } catch (const Fail& f) {
        ctx->err = f.msg;
        return f.code;
    } catch (const HipError& e) {
        ctx->err = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.what;
        return PINS_EDEVICE;
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        return PINS_ENOMEM;
    } catch (...) {
        ctx->err = "unexpected internal error";
        return PINS_EDEVICE;
    }
}

}  // namespace


// ---------------------------------------------------------------------------
// Live batch (pins_live.h): the serving runtime's engine.
// ---------------------------------------------------------------------------
namespace pins {

struct LiveSlot {
    bool live = false, fresh = false;
    bool scaled = false;        // the set-up computes its scale 1/max C on the device
    int64_t id = 0;
    size_t off = 0, bytes = 0;  // arena region
    InstPlan plan;              // offsets relative to the region
    pins_problem prob{};        // sizes and kind (input pointers are not kept)
    int k_done = 0;             // completed outer iterations
    double* alpha_out = nullptr;
    double* beta_out = nullptr;
};

struct LiveBatch {
    int device = 0;
    pins_params p{};
    int max_slots = 0;
    Lane lane;  // its own non-blocking stream and pinned staging; no profiling
    char* arena = nullptr;
    size_t arena_bytes = 0;
    std::map<size_t, size_t> freel;  // free regions of the arena: offset -> bytes
    char* meta = nullptr;            // descriptors, control blocks, offsets, scratch, gates
    size_t o_insts = 0, o_ctrl = 0, o_offs = 0, o_scr = 0, o_gate = 0;
    std::vector<LiveSlot> slots;
    std::vector<DevInst> hI;
    bool grid = false;
    int nlive = 0;
    bool dirty = true;
    LaunchCtx L{};
    std::unique_ptr<OuterRunner> R;
    int src = SRC_DENSE, base_src = SRC_DENSE;
    ~LiveBatch() {
        (void)hipSetDevice(device);
        R.reset();
        if (arena) (void)hipFree(arena);
        if (meta) (void)hipFree(meta);
        for (hipEvent_t e : lane.events) (void)hipEventDestroy(e);
        if (lane.pinned) (void)hipHostFree(lane.pinned);
        if (lane.stream) (void)hipStreamDestroy(lane.stream);
    }
};

namespace {

size_t plan_bytes(const pins_problem& P, const pins_params& p, InstPlan* out) {
    Carver cv;
    const InstPlan q = plan_instance(cv, P, p, true, false);
    if (out) *out = q;
    return al256(cv.off);
}

bool arena_take(LiveBatch* B, size_t need, size_t* off) {
    for (auto it = B->freel.begin(); it != B->freel.end(); ++it) {
        if (it->second < need) continue;
        *off = it->first;
        const size_t rest = it->second - need;
        const size_t at = it->first + need;
        B->freel.erase(it);
        if (rest) B->freel[at] = rest;
        return true;
    }
    return false;
}

void arena_give(LiveBatch* B, size_t off, size_t bytes) {
    auto it = B->freel.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != B->freel.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        B->freel.erase(nx);
    }
    if (it != B->freel.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            B->freel.erase(it);
        }
    }
}

// result scalars of a finished (or rejected) instance from its control block
pins_result live_result(const LiveBatch* B, const Ctrl& S, int K, double scale) {
    pins_result r;
    std::memset(&r, 0, sizeof(r));
    r.cost = S.cost;
    r.eps = B->p.eta / (double)K;
    r.resid = S.resid;
    r.dual = S.dual;
    r.gap = S.cost - S.dual;
    r.entropy = S.entropy;
    r.cost_scale = scale;
    r.flags = S.flags | (S.nonfinite ? 4 : 0);
    r.outer_iters = K;
    r.sinkhorn_iters = S.sink_total;
    r.newton_iters = S.newton_total;
    r.cg_iters = S.cg_total;
    r.fallbacks = S.fb_total;
    r.nnz_last = S.nnz;
    r.status = S.nonfinite ? PINS_ENUMERIC : ((S.flags & 1) ? PINS_NOT_CONVERGED : PINS_OK);
    return r;
}

// The slot leaves: its control block is cleared on the stream (phase DONE, no
// outer iteration left, so no later launch acts on it) before its arena region
// can be handed to another problem.
void live_kill(LiveBatch* B, int q) {
    LiveSlot& Sl = B->slots[q];
    if (!Sl.live) return;
    launch_zero(B->lane.stream, B->meta + B->o_ctrl + sizeof(Ctrl) * (size_t)q, sizeof(Ctrl));
    arena_give(B, Sl.off, Sl.bytes);
    Sl.live = false;
    Sl.fresh = false;
    B->nlive -= 1;
    B->dirty = true;
}

// descriptors and flat-grid offsets of the current slots (dead slots: no tiles,
// phase DONE in their control blocks, so no kernel acts on them)
void live_upload(LiveBatch* B, int count) {
    std::vector<int> toff(1, 0), roff(1, 0);
    std::vector<DevInst> live;
    for (int q = 0; q < count; ++q) {
        const LiveSlot& Sl = B->slots[q];
        const DevInst& I = B->hI[q];
        toff.push_back(toff.back() + (Sl.live ? I.nrb * I.ncb : 0));
        roff.push_back(roff.back() + (Sl.live ? (I.m + 3) / 4 : 0));
        if (Sl.live) live.push_back(I);
    }
    LaunchCtx& L = B->L;
    fill_launch(L, live.data(), (int)live.size(), B->p);
    L.count = count;
    L.kp.count = count;
    L.total_tiles = toff.back();
    L.total_rowblk = roff.back();
    const hipStream_t st = B->lane.stream;
    char* pin = (char*)pinned(&B->lane, sizeof(DevInst) * count + sizeof(int) * 2 * (size_t)(count + 1) + 64);
    std::memcpy(pin, B->hI.data(), sizeof(DevInst) * count);
    HIPCHK(hipMemcpyAsync(B->meta + B->o_insts, pin, sizeof(DevInst) * count, hipMemcpyHostToDevice, st));
    int* ho = (int*)(pin + sizeof(DevInst) * count);
    std::memcpy(ho, toff.data(), sizeof(int) * (count + 1));
    std::memcpy(ho + count + 1, roff.data(), sizeof(int) * (count + 1));
    HIPCHK(hipMemcpyAsync(B->meta + B->o_offs, ho, sizeof(int) * 2 * (count + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));  // the pinned area is reused by the readbacks
    L.kp.toff = (const int*)(B->meta + B->o_offs);
    L.kp.roff = L.kp.toff + count + 1;
    B->dirty = false;
}

int live_round_impl(LiveBatch* B, std::vector<LiveDone>& done) {
    HIPCHK(hipSetDevice(B->device));
    const hipStream_t st = B->lane.stream;
    int count = 0;
    for (int q = 0; q < B->max_slots; ++q)
        if (B->slots[q].live) count = q + 1;
    if (count == 0) return PINS_OK;
    DevInst* d_insts = (DevInst*)(B->meta + B->o_insts);
    Ctrl* d_ctrl = (Ctrl*)(B->meta + B->o_ctrl);
    double* d_scr = (double*)(B->meta + B->o_scr);
    int* d_gate = (int*)(B->meta + B->o_gate);
    // set-up of the problems admitted since the last round
    bool any_fresh = false, any_old = false;
    for (int q = 0; q < count; ++q) {
        any_fresh |= B->slots[q].live && B->slots[q].fresh;
        any_old |= B->slots[q].live && !B->slots[q].fresh;
    }
    if (B->dirty) live_upload(B, count);
    if (any_fresh) {
        for (int q = 0; q < count; ++q) {
            LiveSlot& Sl = B->slots[q];
            if (!Sl.live || !Sl.fresh) continue;
            LaunchCtx Ls = B->L;
            Ls.insts = d_insts + q;
            Ls.insts_mut = d_insts + q;
            Ls.ctrl = d_ctrl + q;
            Ls.count = 1;
            launch_zero(st, d_ctrl + q, sizeof(Ctrl));
            Sl.scaled = Sl.prob.kind != PINS_COST_GRID && !(B->hI[q].bscale > 0.0);
            if (Sl.scaled) launch_cost_max(Ls, d_scr + (size_t)SCRATCH_BLK * q, SCRATCH_BLK, 1);
            launch_init(Ls, B->base_src);
            HIPCHK(hipGetLastError());
        }
        const Ctrl* h = readback(&B->lane, st, d_ctrl, count);
        for (int q = 0; q < count; ++q) {
            LiveSlot& Sl = B->slots[q];
            if (!Sl.live || !Sl.fresh) continue;
            Sl.fresh = false;
            if (h[q].margbad || h[q].nonfinite) {
                LiveDone d;
                d.id = Sl.id;
                d.rc = PINS_EINVAL;
                std::memset(&d.res, 0, sizeof(d.res));
                d.res.status = PINS_EINVAL;
                done.push_back(d);
                live_kill(B, q);
                continue;
            }
            // the scale the set-up chose (1/max C) is kept in the host copy of the descriptor
            if (Sl.scaled) {
                B->hI[q].bscale = h[q].scale;
                B->hI[q].cscale = h[q].scale;
            }
        }
        if (B->dirty) {
            if (B->nlive == 0) return PINS_OK;
            live_upload(B, count);
        }
    }
    // one outer iteration of every problem (the shift acts on those past their first)
    B->R->count = count;
    B->R->run(B->p.hvp == 1, any_old);
    int K = B->p.max_outer;
    bool any_fin = false;
    int* gate = (int*)pinned(&B->lane, sizeof(int) * count);
    for (int q = 0; q < count; ++q) {
        LiveSlot& Sl = B->slots[q];
        gate[q] = 0;
        if (!Sl.live) continue;
        Sl.k_done += 1;
        if (Sl.k_done >= K) {
            gate[q] = 1;
            any_fin = true;
        }
    }
    if (!any_fin) return PINS_OK;
    HIPCHK(hipMemcpyAsync(d_gate, gate, sizeof(int) * count, hipMemcpyHostToDevice, st));
    run_launch(&B->lane, st, PINS_K_FINAL, [&] { launch_final(B->L, B->base_src, (double)K, false, d_gate); });
    std::vector<char> fin(count, 0);
    for (int q = 0; q < count; ++q) fin[q] = (char)gate[q];  // gate's staging is reused by the readback
    const Ctrl* h = readback(&B->lane, st, d_ctrl, count);
    std::vector<Ctrl> hc(h, h + count);
    for (int q = 0; q < count; ++q) {
        if (!fin[q]) continue;
        LiveSlot& Sl = B->slots[q];
        char* base = B->arena + Sl.off;
        HIPCHK(hipMemcpyAsync(Sl.alpha_out, base + Sl.plan.alpha, sizeof(double) * Sl.plan.m, hipMemcpyDeviceToHost,
                              st));
        HIPCHK(hipMemcpyAsync(Sl.beta_out, base + Sl.plan.beta, sizeof(double) * Sl.plan.n, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (int q = 0; q < count; ++q) {
        if (!fin[q]) continue;
        LiveSlot& Sl = B->slots[q];
        LiveDone d;
        d.id = Sl.id;
        d.res = live_result(B, hc[q], K, B->hI[q].bscale);
        d.rc = d.res.status;
        done.push_back(d);
        live_kill(B, q);
    }
    return PINS_OK;
}

}  // namespace

LiveBatch* live_create(int device, const pins_params& p, int max_slots, size_t arena_bytes, std::string* err) {
    try {
        check_params(p);
        if (p.shift_mode != PINS_SHIFT_IMPLICIT) fail(PINS_EUNSUPPORTED, "serving needs the implicit shift");
        if (p.hvp == 2) fail(PINS_EUNSUPPORTED, "serving needs one kind of Hessian product throughout (hvp 0 or 1)");
        if (max_slots < 1 || arena_bytes < 4096) fail(PINS_EINVAL, "bad live batch size");
        std::unique_ptr<LiveBatch> B(new LiveBatch);
        B->device = device;
        B->p = p;
        B->p.profile = 0;
        B->p.graphs = 0;
        B->max_slots = max_slots;
        B->lane.device = device;
        HIPCHK(hipSetDevice(device));
        HIPCHK(hipStreamCreateWithFlags(&B->lane.stream, hipStreamNonBlocking));
        Carver cv;
        B->o_insts = cv.take(sizeof(DevInst) * max_slots);
        B->o_ctrl = cv.take(sizeof(Ctrl) * max_slots);
        B->o_offs = cv.take(sizeof(int) * 2 * (size_t)(max_slots + 1));
        B->o_scr = cv.take(sizeof(double) * (size_t)SCRATCH_BLK * max_slots);
        B->o_gate = cv.take(sizeof(int) * max_slots);
        if (hipMalloc(&B->meta, cv.off) != hipSuccess || hipMalloc(&B->arena, arena_bytes) != hipSuccess) {
            (void)hipGetLastError();
            fail(PINS_ENOMEM, "live batch allocation failed");
        }
        B->arena_bytes = arena_bytes;
        B->freel[0] = arena_bytes;
        B->slots.resize(max_slots);
        B->hI.resize(max_slots);
        std::memset(B->hI.data(), 0, sizeof(DevInst) * max_slots);
        LaunchCtx& L = B->L;
        std::memset(&L, 0, sizeof(L));
        L.stream = B->lane.stream;
        L.insts = (const DevInst*)(B->meta + B->o_insts);
        L.insts_mut = (DevInst*)(B->meta + B->o_insts);
        L.ctrl = (Ctrl*)(B->meta + B->o_ctrl);
        KP& kp = L.kp;
        kp.eta = p.eta;
        kp.inv_eta = 1.0 / p.eta;
        kp.warm_tol = p.warm_tol;
        kp.inner_tol = p.inner_tol;
        kp.final_tol = p.final_tol;
        kp.K = p.max_outer;
        kp.cg_rtol = p.cg_rtol;
        kp.ls_beta = p.ls_beta;
        kp.ls_c1 = p.ls_c1;
        kp.log_rho = std::log(p.rho);
        kp.budget = p.budget;
        kp.T1 = p.max_sinkhorn;
        kp.T2 = p.max_newton;
        kp.cg_max = p.cg_max_iter;
        kp.ls_max = p.ls_max;
        kp.nlev = p.rho_levels;
        kp.shift_mode = PINS_SHIFT_IMPLICIT;
        B->R.reset(new OuterRunner{&B->lane, B->lane.stream, B->L, L.ctrl, 0, B->p, SRC_DENSE, SRC_DENSE});
        // the control blocks of unused slots: phase DONE, no outer iteration left
        launch_zero(B->lane.stream, L.ctrl, sizeof(Ctrl) * max_slots);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(B->lane.stream));
        return B.release();
    } catch (const Fail& f) {
        if (err) *err = f.msg;
    } catch (const HipError& e) {
        (void)hipGetLastError();
        if (err) *err = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.what;
    } catch (...) {
        if (err) *err = "live batch creation failed";
    }
    return nullptr;
}

void live_destroy(LiveBatch* B) { delete B; }

int live_count(const LiveBatch* B) { return B ? B->nlive : 0; }

bool live_grid(const LiveBatch* B) { return B && B->grid; }

size_t live_bytes(const LiveBatch* B, const pins_problem& prob) {
    try {
        check_problem_shape(prob);
        return plan_bytes(prob, B->p, nullptr);
    } catch (...) {
        return 0;
    }
}

bool live_admit(LiveBatch* B, int64_t id, const pins_problem& prob, double* alpha_out, double* beta_out) {
    if (!B || !alpha_out || !beta_out) return false;
    const bool g = prob.kind == PINS_COST_GRID;
    if (B->nlive > 0 && g != B->grid) return false;
    int q = -1;
    for (int k = 0; k < B->max_slots; ++k)
        if (!B->slots[k].live) {
            q = k;
            break;
        }
    if (q < 0) return false;
    try {
        check_problem_shape(prob);
        InstPlan plan;
        const size_t need = plan_bytes(prob, B->p, &plan);
        size_t off = 0;
        if (!arena_take(B, need, &off)) return false;
        HIPCHK(hipSetDevice(B->device));
        pins_result r;
        std::memset(&r, 0, sizeof(r));
        B->hI[q] = build_inst(plan, prob, B->arena + off, true, false, r, B->lane.stream);
        LiveSlot& Sl = B->slots[q];
        Sl.live = true;
        Sl.fresh = true;
        Sl.id = id;
        Sl.off = off;
        Sl.bytes = need;
        Sl.plan = plan;
        Sl.prob = prob;
        Sl.prob.C = Sl.prob.x = Sl.prob.y = Sl.prob.a = Sl.prob.b = nullptr;
        Sl.k_done = 0;
        Sl.alpha_out = alpha_out;
        Sl.beta_out = beta_out;
        // the input copies out of the caller's host arrays complete before admission returns
        HIPCHK(hipStreamSynchronize(B->lane.stream));
        if (B->nlive == 0) {
            B->grid = g;
            B->src = g ? SRC_GRID : SRC_DENSE;
            B->base_src = B->src;
            B->R->src = B->src;
            B->R->base_src = B->base_src;
        }
        B->nlive += 1;
        B->dirty = true;
        return true;
    } catch (...) {
        (void)hipGetLastError();
        return false;
    }
}

int live_round(LiveBatch* B, std::vector<LiveDone>& done, std::string* err) {
    try {
        return live_round_impl(B, done);
    } catch (const Fail& f) {
        if (err) *err = f.msg;
        for (int q = 0; q < B->max_slots; ++q)
            if (B->slots[q].live) {
                LiveDone d;
                d.id = B->slots[q].id;
                d.rc = f.code;
                std::memset(&d.res, 0, sizeof(d.res));
                d.res.status = f.code;
                done.push_back(d);
                live_kill(B, q);
            }
        return f.code;
    } catch (const HipError& e) {
        (void)hipGetLastError();
        if (err) *err = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.what;
        for (int q = 0; q < B->max_slots; ++q)
            if (B->slots[q].live) {
                LiveDone d;
                d.id = B->slots[q].id;
                d.rc = PINS_EDEVICE;
                std::memset(&d.res, 0, sizeof(d.res));
                d.res.status = PINS_EDEVICE;
                done.push_back(d);
                live_kill(B, q);
            }
        return PINS_EDEVICE;
    }
}

}  // namespace pins

extern "C" {

int pins_abi_version(void) { return PINS_ABI_VERSION; }

void pins_params_default(pins_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->eta = 1e-2;
    p->max_outer = 250;
    p->max_sinkhorn = 100;
    p->max_newton = 50;
    p->cg_max_iter = 1000;
    p->warm_tol = 1e-3;
    p->inner_tol = 1e-9;
    p->final_tol = 1e-12;
    p->cg_rtol = 1e-6;
    p->ls_beta = 0.5;
    p->ls_c1 = 1e-4;
    p->ls_max = 30;
    p->rho_levels = 11;
    p->rho = 1e-7;
    p->budget = 64.0;
    p->precision = PINS_FP64;
    p->shift_mode = PINS_SHIFT_IMPLICIT;
    p->profile = 0;
    p->streams = 0;
    p->profile_mask = 0;
    p->hvp = 0;
    p->hvp_switch = 0;
}

int pins_create(int device, pins_ctx** out) {
    if (!out) return PINS_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return PINS_EDEVICE;
    }
    // set-up of the no-allocation lane: the fixed scratch's address on this device
    void* scr = nullptr;
    if (noalloc_scratch(device, &scr) != PINS_OK) return PINS_EDEVICE;
    pins_ctx* c = new (std::nothrow) pins_ctx;
    if (!c) return PINS_ENOMEM;
    c->device = device;
    c->fixed = new (std::nothrow) Lane;
    if (!c->fixed) {
        delete c;
        return PINS_ENOMEM;
    }
    c->fixed->device = device;
    c->fixed->fixed = true;
    c->fixed->ws = scr;
    c->fixed->ws_bytes = PINS_NOALLOC_SCRATCH_BYTES;
    *out = c;
    return PINS_OK;
}

void pins_destroy(pins_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    for (Lane* L : c->lanes) free_lane(L);
    if (c->fixed) free_lane(c->fixed);
    delete c;
}

const char* pins_last_error(const pins_ctx* c) { return c ? c->err.c_str() : "null context"; }

int pins_workspace_bytes(const pins_problem* probs, int count, const pins_params* p, size_t* bytes) {
    if (!probs || !p || !bytes || count < 1) return PINS_EINVAL;
    try {
        check_params(*p);
        for (int q = 0; q < count; ++q) check_problem_shape(probs[q]);
        *bytes = plan_batch(probs, count, *p, false, nullptr).total;
        return PINS_OK;
    } catch (const Fail& f) {
        return f.code;
    } catch (...) {
        return PINS_EINVAL;
    }
}

int pins_solve(pins_ctx* ctx, const pins_problem* prob, const pins_params* p, pins_result* res) {
    return guarded(ctx, [&] {
        if (!prob || !p || !res) fail(PINS_EINVAL, "null argument");
        return solve_entry(ctx, prob, 1, *p, res, nullptr, true);
    });
}

int pins_solve_device(pins_ctx* ctx, const pins_problem* prob, const pins_params* p, pins_result* res,
                      void* stream) {
    return guarded(ctx, [&] {
        if (!prob || !p || !res) fail(PINS_EINVAL, "null argument");
        return solve_entry(ctx, prob, 1, *p, res, (hipStream_t)stream, false);
    });
}

int pins_solve_device_noalloc(pins_ctx* ctx, const pins_problem* prob, const pins_params* p, pins_result* res,
                              void* stream) {
    return guarded(ctx, [&] {
        if (!prob || !p || !res) fail(PINS_EINVAL, "null argument");
        if (!ctx->fixed) fail(PINS_EDEVICE, "context has no fixed scratch");
        return solve_impl(ctx->fixed, prob, 1, *p, res, (hipStream_t)stream, false);
    });
}

int pins_solve_resume(pins_ctx* ctx, const pins_problem* prob, const pins_params* p, const pins_state* from,
                      int32_t stop, pins_state* save, pins_result* res) {
    return guarded(ctx, [&] {
        if (!prob || !p || !res) fail(PINS_EINVAL, "null argument");
        check_params(*p);
        check_problem_shape(*prob);
        if (p->shift_mode != PINS_SHIFT_IMPLICIT)
            fail(PINS_EUNSUPPORTED, "resume needs the implicit shift (shift_mode 0)");
        const int K = p->max_outer;
        if (stop < 0 || stop > K) fail(PINS_EINVAL, "stop must be in [0, max_outer]");
        const ResumeIO io{from, stop > 0 ? stop : K, save};
        if (from) {
            const pins_state& S = *from;
            if (S.m != prob->m || S.n != prob->n) fail(PINS_EINVAL, "state sizes do not match the problem");
            if (S.outer_done < 1 || S.outer_done >= io.stop)
                fail(PINS_EINVAL, "state outer_done must be in [1, stop)");
            if (!S.F || !S.G || !S.A || !S.B) fail(PINS_EINVAL, "state arrays are required");
            for (int i = 0; i < S.m; ++i)
                if (!std::isfinite(S.F[i]) || !std::isfinite(S.A[i])) fail(PINS_EINVAL, "state has non-finite entries");
            for (int j = 0; j < S.n; ++j)
                if (!std::isfinite(S.G[j]) || !std::isfinite(S.B[j])) fail(PINS_EINVAL, "state has non-finite entries");
        }
        if (save && (!save->F || !save->G || !save->A || !save->B)) fail(PINS_EINVAL, "save arrays are required");
        return solve_impl(lane(ctx, 0), prob, 1, *p, res, nullptr, true, &io);
    });
}

int pins_solve_batch_device(pins_ctx* ctx, const pins_problem* probs, int count, const pins_params* p,
                            pins_result* res, void* stream) {
    return guarded(ctx, [&] {
        if (!probs || !p || !res) fail(PINS_EINVAL, "null argument");
        return solve_entry(ctx, probs, count, *p, res, (hipStream_t)stream, false);
    });
}

int pins_tune_batch_device(pins_ctx* ctx, const pins_problem* probs, int count, const pins_params* p,
                           int max_lanes, int reps, pins_result* res, void* stream, pins_params* best,
                           pins_tune_trial* trials, int max_trials, int32_t* ntrials) {
    return guarded(ctx, [&] {
        if (!probs || !p || !res || !best) fail(PINS_EINVAL, "null argument");
        if (max_lanes < 1 || max_lanes > PINS_MAX_LANES) fail(PINS_EINVAL, "max_lanes must be in [1, PINS_MAX_LANES]");
        if (reps < 1) fail(PINS_EINVAL, "reps must be >= 1");
        if (count < 1) fail(PINS_EINVAL, "count must be >= 1");
        check_params(*p);
        using clk = std::chrono::steady_clock;
        int rc = PINS_OK, nt = 0;
        pins_params cur = *p, top = *p;
        double top_ms = -1.0;
        // one configuration: an untimed solve, then the fastest of `reps` timed ones
        auto trial = [&](const pins_params& q) {
            rc = solve_entry(ctx, probs, count, q, res, (hipStream_t)stream, false);
            if (rc < 0) return;
            double t = 0.0;
            for (int r = 0; r < reps; ++r) {
                const auto t0 = clk::now();
                rc = solve_entry(ctx, probs, count, q, res, (hipStream_t)stream, false);
                if (rc < 0) return;
                const double e = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
                t = (r == 0) ? e : std::min(t, e);
            }
            if (trials && nt < max_trials) {
                pins_tune_trial& T = trials[nt];
                T.streams = q.streams;
                T.graphs = q.graphs;
                for (int c = 0; c < 4; ++c) T.tile_rows[c] = q.tile_rows[c];
                T.ms = t;
            }
            ++nt;
            if (top_ms < 0.0 || t < top_ms) {
                top_ms = t;
                top = q;
            }
        };
        // lanes (a batch runs on at most `count` lanes), graphs off, 16-row tiles
        cur.graphs = 0;
        for (int c = 0; c < 4; ++c) cur.tile_rows[c] = 0;
        for (int g = 1; g <= std::min(max_lanes, count); ++g) {
            cur.streams = g;
            trial(cur);
            if (rc < 0) return rc;
        }
        // graph replay at the best lane count
        cur = top;
        cur.graphs = 1;
        trial(cur);
        if (rc < 0) return rc;
        // rows per tile, per size class present in the batch
        bool present[4] = {false, false, false, false};
        for (int q = 0; q < count; ++q) present[size_class(probs[q].m)] = true;
        for (int c = 0; c < 4; ++c) {
            if (!present[c]) continue;
            for (int rows : {8, 32, 64}) {
                cur = top;
                cur.tile_rows[c] = rows;
                trial(cur);
                if (rc < 0) return rc;
            }
        }
        *best = top;
        if (ntrials) *ntrials = nt;
        return rc;
    });
}

}  // extern "C"
