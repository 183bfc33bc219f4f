// pins_kernels.hip -- HIP kernels of the PINS hot path for MI355X (gfx950).
//
// Every kernel covers a batch of independent instances: the tile and row
// kernels run a flat grid whose blocks map to (instance, block) through
// per-instance prefix sums (uneven sizes waste no blocks); the per-instance
// merges and setup kernels use blockIdx.y as the instance.  Each instance's
// control block (Ctrl::phase) decides whether it takes part in a launch.  An instance's arithmetic never
// depends on which other instances are in the batch, so a batched result is
// bitwise the result of the same problem solved alone.
//
// Wave64 throughout.  Reductions are fixed-order trees (wave butterflies,
// then LDS in wave order, then per-block partials summed in block order), so
// every run is bitwise reproducible.  No value atomics: atomics only count
// integers (Sparsify histogram, CSC counts) or hand out tickets.
//
// Paper references: Alg. 1 / Alg. 2 (log-domain Sinkhorn, PINS), eq. (eppa_x)
// recovery map, eq. (eppa-sub-dual) dual objective, eq. (eppa-hess) Hessian.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <mutex>

#include "pins.h"
#include "pins_internal.h"
#include "pins_launch.h"
#include "pins_texp.h"

// Device scratch of the entry point that allocates nothing
// (pins_solve_device_noalloc): one array per GPU, held until the process ends.
// Host code never passes this name to a kernel or a copy (on the host it is a
// stand-in, not a device address): pins::noalloc_scratch() looks up its
// address on each device once and every use goes through that address.
static __device__ __align__(256) char scratch[PINS_NOALLOC_SCRATCH_BYTES];

namespace pins {

static constexpr double INV_LN10 = 0.43429448190325182765;

// load through the global address space (the pointers live in descriptors,
// so the compiler cannot infer it and would otherwise emit flat loads)
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}

// ---------------------------------------------------------------------------
// cost sources
// ---------------------------------------------------------------------------

// Dense row-major cost.  `base` selects the unshifted cost (outputs, shift)
// instead of the exponent source (which is C^k in materialised mode).
struct DenseSrc {
    const double* __restrict__ C;
    long ld;
    double s;
    __device__ __forceinline__ DenseSrc(const DevInst& I, bool base = false)
        : C(base ? I.cbase : I.csrc), ld(I.ldc), s(base ? I.bscale : I.cscale) {}
    __device__ __forceinline__ double at(int i, int j) const { return ldg(C + ((long)i * ld + j)) * s; }
    // walking a row: the row's base, a column cursor advanced by a fixed step
    typedef const double* Row;
    typedef int Col;
    __device__ __forceinline__ Row row(int i) const { return C + (long)i * ld; }
    __device__ __forceinline__ Col col(int j) const { return j; }
    template <int STEP>
    __device__ __forceinline__ void next(Col& c) const { c += STEP; }
    __device__ __forceinline__ double at(Row r, Col c) const { return ldg(r + c) * s; }
};

// Squared distance between pixels p = row*s + col of an s x s grid, times the
// scale; exact integers before scaling, never stored.  The row of a pixel is
// found as (int)((p + 0.5) * (1/s)) in float, exact because p < s^2 < 2^16:
// the relative rounding error (< 2^-22) times p/s (< s) stays far below the
// distance 0.5/s of (p + 0.5)/s to the nearest integer.
struct GridSrc {
    int s;
    float inv_s;
    double sc;
    __device__ __forceinline__ GridSrc(const DevInst& I, bool base = false)
        : s(I.grid_s), inv_s(1.0f / (float)I.grid_s), sc(base ? I.bscale : I.cscale) {}
    __device__ __forceinline__ int quot(int v) const { return (int)(((float)v + 0.5f) * inv_s); }
    __device__ __forceinline__ double at(int i, int j) const {
        const int ri = quot(i), ci = i - ri * s, rj = quot(j), cj = j - rj * s;
        const int dr = ri - rj, dc = ci - cj;
        return (double)(dr * dr + dc * dc) * sc;
    }
    // walking a row: pixel coordinates, the column's advanced by a fixed step
    // of pixels without a division (the same exact integers as at(i, j))
    struct Px {
        int r, c;
    };
    typedef Px Row;
    typedef Px Col;
    __device__ __forceinline__ Px row(int i) const {
        const int r = quot(i);
        return Px{r, i - r * s};
    }
    __device__ __forceinline__ Px col(int j) const { return row(j); }
    template <int STEP>
    __device__ __forceinline__ void next(Px& q) const {
        q.c += STEP % s;
        q.r += STEP / s;
        if (q.c >= s) {
            q.c -= s;
            q.r += 1;
        }
    }
    __device__ __forceinline__ double at(Px a, Px b) const {
        const int dr = a.r - b.r, dc = a.c - b.c;
        return (double)(dr * dr + dc * dc) * sc;
    }
};


// A tile's rows as cursors of its cost source, in LDS: entry r is row
// i0 + min(r, rows - 1), so that every entry of the table is a row in range.
// (For the grid cost this takes each row's pixel coordinates out of the
// per-entry work.)
template <class Src>
__device__ __forceinline__ void tile_row_table(const Src& src, typename Src::Row* sRow, int i0, int rows) {
    if ((int)threadIdx.x < TILE_RMAX) sRow[threadIdx.x] = src.row(i0 + min((int)threadIdx.x, rows - 1));
}

// log of the recovery map, eq. (eppa_x): (F_i + G_j - kappa*C_ij)/eta
__device__ __forceinline__ double expo(double Fi, double Gj, double kap, double c, double ie) {
    return (Fi + Gj - kap * c) * ie;
}

// Sparsify level coordinate: Xt_ij >= rho*10^l*min(a_i,b_j)  <=>  q >= l
__device__ __forceinline__ double lev_q(double x, double log_rho, double la, double lb) {
    return (x - log_rho - fmin(la, lb)) * INV_LN10;
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

// Cross-lane moves through DPP (data-parallel primitives, no LDS round trip).
// CTRL: 0xB1 quad_perm [1,0,3,2] (lane ^ 1), 0x4E quad_perm [2,3,0,1]
// (lane ^ 2), 0x141 row_half_mirror (lane i <-> 7-i within 8), 0x140
// row_mirror (i <-> 15-i within 16).  Each pairs lanes symmetrically, so a
// sum step gives every lane of the group the same value.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

// sum over aligned groups of G lanes (G = 1, 2, 4, 8, 16, 32); every lane of the group gets it
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 32, "group of 1..32 lanes");
    if (G >= 2) v += dpp_f64<0xB1>(v);
    if (G >= 4) v += dpp_f64<0x4E>(v);
    if (G >= 8) v += dpp_f64<0x141>(v);
    if (G >= 16) v += dpp_f64<0x140>(v);
    if (G >= 32) v += __shfl_xor(v, 16);
    return v;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// sum over the 64 lanes of a wave, broadcast (fixed order: 16-lane rows, then rows 0..3)
__device__ __forceinline__ double wave_sum(double v) {
    v = group_sum<16>(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

__device__ __forceinline__ int wave_sum_i(int v) {
    v += dpp_i32<0xB1>(v);
    v += dpp_i32<0x4E>(v);
    v += dpp_i32<0x141>(v);
    v += dpp_i32<0x140>(v);
    return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
           (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

// (max, sum) pairs of log-sum-exp; an empty pair is (-inf, 0).
// ex<T>(y, T64): exp in the sweep's precision (float: hardware exp; double:
// the table-driven texp below with its table T64 in LDS).
__device__ __forceinline__ double texp(double x, const double* T);
template <class T>
__device__ __forceinline__ T ex(double y, const double* T64);
template <>
__device__ __forceinline__ double ex<double>(double y, const double* T64) { return texp(y, T64); }
template <>
__device__ __forceinline__ float ex<float>(double y, const double*) { return __expf((float)y); }
// exp in the sweep's precision of an argument <= 0 (the log-sum-exp sweeps'
// exp(z - max)): double takes the table method's non-positive form
template <class T>
__device__ __forceinline__ T exn(double y, const double* T64);
template <>
__device__ __forceinline__ double exn<double>(double y, const double* T64) { return texp_eval_nonpos(y, T64); }
template <>
__device__ __forceinline__ float exn<float>(double y, const double*) { return __expf((float)y); }
// the same without a table (the few merges of partial pairs)
template <class T>
__device__ __forceinline__ T exs(double y);
template <>
__device__ __forceinline__ double exs<double>(double y) { return exp(y); }
template <>
__device__ __forceinline__ float exs<float>(double y) { return __expf((float)y); }

// exp(x) in double by Tang's table-driven method (pins_texp.h), the table
// 2^(j/64), j = 0..63, in LDS.
__device__ __forceinline__ void texp_table(double* T) {
    if (threadIdx.x < 64) T[threadIdx.x] = texp_table_entry((int)threadIdx.x);
}
__device__ __forceinline__ double texp(double x, const double* T) { return texp_eval(x, T); }

template <class T>
__device__ __forceinline__ void lse_combine(double& mx, T& sm, double m2, T s2) {
    const double M = fmax(mx, m2);
    const T u = (mx == -INFINITY) ? T(0) : sm * exs<T>(mx - M);
    const T v = (m2 == -INFINITY) ? T(0) : s2 * exs<T>(m2 - M);
    mx = M;
    sm = u + v;
}

template <int CTRL, class T>
__device__ __forceinline__ T dpp_t(T v);
template <int CTRL, class T>
__device__ __forceinline__ T dpp_t(T v) {
    if constexpr (sizeof(T) == 8) {
        return dpp_f64<CTRL>(v);
    } else {
        return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
    }
}

template <int CTRL, class T>
__device__ __forceinline__ void lse_step(double& mx, T& sm) {
    const double m2 = dpp_f64<CTRL>(mx);
    const T s2 = dpp_t<CTRL>(sm);
    lse_combine(mx, sm, m2, s2);
}

template <class T>
__device__ __forceinline__ T readlane_t(T v, int lane) {
    if constexpr (sizeof(T) == 8) {
        return readlane_f64(v, lane);
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
    }
}

// (max, sum) combine over a wave (in-row DPP steps, then rows 0..3 in order);
// every lane gets the same pair
template <class T>
__device__ __forceinline__ void wave_lse(double& mx, T& sm) {
    lse_step<0xB1>(mx, sm);
    lse_step<0x4E>(mx, sm);
    lse_step<0x141>(mx, sm);
    lse_step<0x140>(mx, sm);
    double M = readlane_f64(mx, 0);
    T S = readlane_t(sm, 0);
    for (int r = 16; r < 64; r += 16) lse_combine(M, S, readlane_f64(mx, r), readlane_t(sm, r));
    mx = M;
    sm = S;
}

// Sum over a block of NT threads, result broadcast to all; fixed order.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    constexpr int NW = NT / 64;
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) t += sh[k];
    return t;
}

// Two sums over a block at once (one pair of barriers).
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
    constexpr int NW = NT / 64;
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) {
        sh[w] = a;
        sh[NW + w] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        ta += sh[k];
        tb += sh[NW + k];
    }
    a = ta;
    b = tb;
}

// Two sums over a block when no thread can still be reading sh (the caller's
// earlier barriers order the previous readers): one barrier instead of two.
template <int NT>
__device__ __forceinline__ void block_sum2_nolead(double& a, double& b, double* sh) {
    constexpr int NW = NT / 64;
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        sh[w] = a;
        sh[NW + w] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        ta += sh[k];
        tb += sh[NW + k];
    }
    a = ta;
    b = tb;
}

// Sum of p[0..len) by a block of NT threads in a fixed order.
template <int NT>
__device__ __forceinline__ double block_sum_array(const double* p, int len, double* sh) {
    double v = 0.0;
    for (int k = threadIdx.x; k < len; k += NT) v += p[k];
    return block_sum<NT>(v, sh);
}

// Exclusive scan of cnt(k), k < len, by a block of NT threads; writes out[k]
// (clamped to cap) and out[len]; returns the unclamped total.
template <int NT, class CountF>
__device__ __forceinline__ long block_scan_excl(CountF cnt, int len, int* out, int cap, int* sh) {
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    long carry = 0;
    for (int base = 0; base < len; base += NT) {
        const int k = base + threadIdx.x;
        const int c = (k < len) ? cnt(k) : 0;
        int inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o);
            if (l >= o) inc += t;
        }
        __syncthreads();
        if (l == 63) sh[w] = inc;
        __syncthreads();
        int woff = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            const int s = sh[q];
            if (q < w) woff += s;
            tot += s;
        }
        if (k < len) {
            const long e = carry + woff + inc - c;
            out[k] = (int)(e < cap ? e : cap);
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[len] = (int)(carry < cap ? carry : cap);
    __syncthreads();
    return carry;
}

// Last-block detection: every participating block calls this once; it
// returns true in exactly one block, after all others have released their
// writes.  The ticket is reset for the next launch.
__device__ __forceinline__ bool last_block(int* ticket, int nblocks) {
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = atomicAdd(ticket, 1);
        s_last = (t == nblocks - 1);
        if (s_last) atomicExch(ticket, 0);
    }
    __syncthreads();
    if (s_last) __threadfence();
    return s_last != 0;
}

__device__ __forceinline__ bool phase_in(const Ctrl* ctrl, int b, int mask) {
    return (mask >> ctrl[b].phase) & 1;
}

// one writer per instance (its first block) records the entries a pass visits
// l: the block's index inside its instance
__device__ __forceinline__ void count_work(Ctrl* ctrl, int b, int kind, int m, int n, int l) {
    if (l == 0 && threadIdx.x == 0) ctrl[b].work[kind] += (double)m * (double)n;
}

// Flat grids over an uneven batch: block blockIdx.x belongs to the instance b
// with off[b] <= blockIdx.x < off[b + 1] and is its block l = blockIdx.x - off[b]
// (off: count + 1 prefix sums of the per-instance block counts).
struct BlkRef {
    int b, l;
};
__device__ __forceinline__ BlkRef blk_ref(const int* __restrict__ off, int count) {
    const int x = blockIdx.x;
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return BlkRef{lo, x - off[lo]};
}

// ---------------------------------------------------------------------------
// a2: Sinkhorn f-update (row log-sum-exp sweep), one wave per row.
//   F_i <- eta*log a_i - eta*LSE_j((G_j - kappa*C_ij)/eta)
// Also the row-marginal error of the state before the update:
//   r_i = a_i*exp((F_old - F_new)/eta),   blk[block] = sum |r_i - a_i|.
// T = float: exp and the sum in single precision (mixed path); the exponent
// and the running maximum stay double.
// ---------------------------------------------------------------------------
template <class Src, class T>
__global__ __launch_bounds__(256) void k_row_lse(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp,
                                                 int mask) {
    const BlkRef br = blk_ref(kp.roff, kp.count);
    const int b = br.b, rl = br.l;
    if (!phase_in(ctrl, b, mask)) return;
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n;
    count_work(ctrl, b, W_ROW, m, n, rl);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = rl * 4 + w;
    __shared__ double serr[4];
    __shared__ double sT[64];
    texp_table(sT);
    __syncthreads();
    double err = 0.0;
    if (i < m) {
        const double kap = ctrl[b].kappa, ie = kp.inv_eta;
        const Src src(I);
        const double* __restrict__ G = I.G;
        double mx = -INFINITY;
        T sm = T(0);
        constexpr int U = 8;  // columns per lane in flight (8: 0.61 of 8 TB/s in FP64 on a dense cost, 4: 0.60)
        // chunks of 64 U columns: the full ones without bounds tests (so that
        // their U loads of C and G are issued together), then the last partial
        // one; the same operations in the same order either way
        const int nfull = n - n % (64 * U);
        const typename Src::Row ro = src.row(i);
        typename Src::Col co = src.col(lane);  // column j0 + u * 64 + lane below
        int j0 = 0;
        for (; j0 < nfull; j0 += 64 * U) {
            double z[U];
            double cm = -INFINITY;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = j0 + u * 64 + lane;
                z[u] = (ldg(G + j) - kap * src.at(ro, co)) * ie;
                src.template next<64>(co);
                cm = fmax(cm, z[u]);
            }
            if (cm > mx) {
                sm *= exn<T>(mx - cm, sT);
                mx = cm;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) sm += exn<T>(z[u] - mx, sT);
        }
        if (j0 < n) {
            double z[U];
            double cm = -INFINITY;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = j0 + u * 64 + lane;
                z[u] = (j < n) ? (ldg(G + j) - kap * src.at(ro, co)) * ie : -INFINITY;
                src.template next<64>(co);
                cm = fmax(cm, z[u]);
            }
            if (cm > mx) {
                sm *= exn<T>(mx - cm, sT);
                mx = cm;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = j0 + u * 64 + lane;
                if (j < n) sm += exn<T>(z[u] - mx, sT);
            }
        }
        wave_lse(mx, sm);
        if (lane == 0) {
            const double lse = mx + log((double)sm);
            const double Fo = I.F[i];
            const double Fn = kp.eta * (I.loga[i] - lse);
            const double ai = I.a[i];
            err = fabs(ai * exp((Fo - Fn) * ie) - ai);
            I.F[i] = Fn;
        }
    }
    if (lane == 0) serr[w] = err;
    __syncthreads();
    if (threadIdx.x == 0) I.blk[rl] = ((serr[0] + serr[1]) + serr[2]) + serr[3];
}

// ---------------------------------------------------------------------------
// a3: Sinkhorn g-update, column partials.  Tile = R rows x 256 columns, one
// column per thread: part[rb][j] = (max, sum) of (F_i - kappa*C_ij)/eta over
// the tile's rows (with the new F: Gauss-Seidel).
// ---------------------------------------------------------------------------
template <class Src, class T>
__global__ __launch_bounds__(256) void k_col_lse(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp,
                                                 int mask) {
    const BlkRef br = blk_ref(kp.toff, kp.count);
    const int b = br.b, tl = br.l;
    if (!phase_in(ctrl, b, mask)) return;
    const DevInst& I = insts[b];
    const int rb = tl / I.ncb, cb = tl - rb * I.ncb;
    const int m = I.m, n = I.n;
    count_work(ctrl, b, W_COL, m, n, tl);
    const int i0 = rb * I.R, i1 = min(m, i0 + I.R);
    __shared__ double sF[TILE_RMAX + 4];
    __shared__ double sT[64];
    texp_table(sT);
    if ((int)threadIdx.x < TILE_RMAX + 4) sF[threadIdx.x] = (i0 + (int)threadIdx.x < i1) ? I.F[i0 + threadIdx.x] : 0.0;
    const Src src(I);
    __shared__ typename Src::Row sRow[TILE_RMAX];
    tile_row_table(src, sRow, i0, i1 - i0);
    __syncthreads();
    const int j = cb * TILE_C + threadIdx.x;
    if (j >= n) return;
    const double kap = ctrl[b].kappa, ie = kp.inv_eta;
    const typename Src::Col cj = src.col(j);
    double mx = -INFINITY;
    T sm = T(0);
    constexpr int U = 4;
    // groups of U rows: the full ones without bounds tests (their U loads
    // issued together), then the last partial one; the same operations in the
    // same order either way
    int i = i0;
    for (; i + U <= i1; i += U) {
        double z[U];
        double cm = -INFINITY;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            z[u] = (sF[i + u - i0] - kap * src.at(sRow[i + u - i0], cj)) * ie;
            cm = fmax(cm, z[u]);
        }
        if (cm > mx) {
            sm *= exn<T>(mx - cm, sT);
            mx = cm;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) sm += exn<T>(z[u] - mx, sT);
    }
    if (i < i1) {
        double z[U];
        double cm = -INFINITY;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ii = i + u;
            z[u] = (ii < i1) ? (sF[ii - i0] - kap * src.at(sRow[min(ii - i0, TILE_RMAX - 1)], cj)) * ie : -INFINITY;
            cm = fmax(cm, z[u]);
        }
        if (cm > mx) {
            sm *= exn<T>(mx - cm, sT);
            mx = cm;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i + u < i1) sm += exn<T>(z[u] - mx, sT);
    }
    reinterpret_cast<double2*>(I.part)[(long)rb * n + j] = make_double2(mx, (double)sm);
}

// Merge of the column partials: G_j <- eta*log b_j - eta*LSE; the last block
// runs the warm-up control (row error of the sweep, exit test).
__global__ __launch_bounds__(256) void k_col_merge(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp,
                                                   int mask) {
    // 32 columns per block, 8 lanes per column: lane s merges the row blocks
    // s, s + 8, ... (two passes: maximum, then rescaled sum), then the 8
    // (max, sum) pairs of a column are combined in lane order
    const int b = blockIdx.y;
    if (!phase_in(ctrl, b, mask)) return;
    const DevInst& I = insts[b];
    const int n = I.n;
    if ((int)blockIdx.x * 32 >= n) return;
    const int c = threadIdx.x & 31, sl = threadIdx.x >> 5;
    const int j = blockIdx.x * 32 + c;
    __shared__ double smx[8][32], ssm[8][32];
    double mx = -INFINITY, sm = 0.0;
    if (j < n) {
        const double2* __restrict__ P = reinterpret_cast<const double2*>(I.part);
        for (int rb = sl; rb < I.nrb; rb += 8) mx = fmax(mx, P[(long)rb * n + j].x);
        if (mx != -INFINITY)
            for (int rb = sl; rb < I.nrb; rb += 8) {
                const double2 q = P[(long)rb * n + j];
                if (q.x != -INFINITY) sm += q.y * exp(q.x - mx);
            }
    }
    smx[sl][c] = mx;
    ssm[sl][c] = sm;
    __syncthreads();
    if (sl == 0 && j < n) {
        double M = -INFINITY;
        for (int k = 0; k < 8; ++k) M = fmax(M, smx[k][c]);
        double S = 0.0;
        for (int k = 0; k < 8; ++k)
            if (smx[k][c] != -INFINITY) S += ssm[k][c] * exp(smx[k][c] - M);
        I.G[j] = kp.eta * (I.logb[j] - (M + log(S)));
    }
}

// Warm-up control after a g-update (one block per instance; a kernel of its
// own so that no block of k_col_merge sees the phase change).
__global__ __launch_bounds__(256) void k_col_decide(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp,
                                                    int mask) {
    const int b = blockIdx.x;
    if (!phase_in(ctrl, b, mask)) return;
    const DevInst& I = insts[b];
    {
        __shared__ double sh[4];
        const double err = block_sum_array<256>(I.blk, (I.m + 3) / 4, sh);
        if (threadIdx.x == 0) {
            Ctrl& S = ctrl[b];
            if (S.phase == PH_WARM) {
                S.err = err;
                S.t += 1;
                S.sink_total += 1;
                if (!isfinite(err)) {
                    S.nonfinite = 1;
                    S.phase = PH_DONE;
                } else if (err <= kp.warm_tol || S.t >= kp.T1) {
                    S.phase = PH_NEWTON;
                    S.t = 0;
                }
            } else if (S.phase == PH_FALLBACK) {
                S.phase = PH_NEWTON;
            }
        }
    }
}

// Row totals of a tile without a tile-sized LDS array.  v[u] is this
// thread's entry of row r0 + u.  Two exchanges across wave halves (xor 32,
// xor 16) and a 16-lane DPP sum leave the wave's total of row r0 + (lane >> 4)
// in lanes 0, 16, 32 and 48, which store it to wsum[row][wave].  Fixed order.
__device__ __forceinline__ void wave_rows4(const double (&v)[4], int r0, double (*wsum)[4]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const bool h32 = lane >= 32, h16 = (lane & 16) != 0;
    double a0 = h32 ? v[2] : v[0], a1 = h32 ? v[3] : v[1];
    const double s0 = h32 ? v[0] : v[2], s1 = h32 ? v[1] : v[3];
    a0 += __shfl_xor(s0, 32);
    a1 += __shfl_xor(s1, 32);
    double c = h16 ? a1 : a0;
    const double sc = h16 ? a0 : a1;
    c += __shfl_xor(sc, 16);
    c = group_sum<16>(c);
    if ((lane & 15) == 0) wsum[r0 + (lane >> 4)][w] = c;
}

// Tile row totals from the per-wave totals (after a barrier): part2[cb][i].
__device__ __forceinline__ void tile_rows_store(const double (*wsum)[4], int rows, int i0, int cb, int m,
                                                double* __restrict__ part2) {
    const int t = threadIdx.x;
    if (t < rows) part2[(long)cb * m + i0 + t] = (wsum[t][0] + wsum[t][1]) + (wsum[t][2] + wsum[t][3]);
}

// Sparsify level counts of a tile: hb[level * TILE_C + thread] is one byte per
// thread and level (at most TILE_RMAX entries each).  Wave w reads the 64
// words of levels w, w + 4, w + 8, w + 12, adds their bytes and reduces over
// the wave; one atomic per level and wave (integer, so order-free).
__device__ __forceinline__ void tile_level_totals(const unsigned* hw, int nlev, int* __restrict__ hist) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int s4 = 0; s4 < NLEV / 4; ++s4) {
        const int l = w + 4 * s4;
        if (l < nlev) {
            unsigned x = hw[l * (TILE_C / 4) + lane];
            x = (x & 0x00ff00ffu) + ((x >> 8) & 0x00ff00ffu);
            const int v = wave_sum_i((int)((x & 0xffffu) + (x >> 16)));
            if (lane == 0 && v) atomicAdd(&hist[l], v);
        }
    }
}

template <class Src>
__global__ __launch_bounds__(256) void k_grad(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp) {
    const BlkRef br = blk_ref(kp.toff, kp.count);
    const int b = br.b, tl = br.l;
    if (ctrl[b].phase != PH_NEWTON || ctrl[b].grad_ready) return;
    const DevInst& I = insts[b];
    const int rb = tl / I.ncb, cb = tl - rb * I.ncb;
    const int m = I.m, n = I.n;
    count_work(ctrl, b, W_GRAD, m, n, tl);
    const int i0 = rb * I.R, rows = min(I.R, m - i0);
    __shared__ unsigned hw[NLEV * TILE_C / 4];  // [level][thread] byte counters
    __shared__ double wsum[TILE_RMAX][4];
    __shared__ double sF[TILE_RMAX], sLa[TILE_RMAX];
    __shared__ double sT[64];
    texp_table(sT);
    unsigned char* hcol = reinterpret_cast<unsigned char*>(hw);
    for (int k = threadIdx.x; k < NLEV * TILE_C / 4; k += 256) hw[k] = 0u;
    if ((int)threadIdx.x < rows) {
        sF[threadIdx.x] = I.F[i0 + threadIdx.x];
        sLa[threadIdx.x] = I.loga[i0 + threadIdx.x];
    }
    const Src src(I);
    __shared__ typename Src::Row sRow[TILE_RMAX];
    tile_row_table(src, sRow, i0, rows);
    __syncthreads();
    const int j = cb * TILE_C + threadIdx.x;
    const bool valid = j < n;
    const double kap = ctrl[b].kappa, ie = kp.inv_eta, lrho = kp.log_rho;
    const int nlev = kp.nlev;
    const double Gj = valid ? ldg(I.G + j) : 0.0, lbj = valid ? ldg(I.logb + j) : 0.0;
    double colacc = 0.0;
    const int jc = valid ? j : 0;  // a column in range for the loads of idle lanes
    const typename Src::Col cj = src.col(jc);
    for (int r0 = 0; r0 < rows; r0 += 4) {
        // the group's 4 cost values first (clamped in range, so that their
        // loads are issued together), then the entries
        double cv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) cv[u] = src.at(sRow[min(r0 + u, rows - 1)], cj);
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = r0 + u;
            double e = 0.0;
            if (valid && r < rows) {
                const double x = expo(sF[r], Gj, kap, cv[u], ie);
                e = texp(x, sT);
                const double q = lev_q(x, lrho, sLa[r], lbj);
                if (q >= 0.0) {
                    const int l = (q >= (double)(nlev - 1)) ? nlev - 1 : (int)q;
                    hcol[l * TILE_C + threadIdx.x] += 1;
                }
            }
            colacc += e;
            v[u] = e;
        }
        wave_rows4(v, r0, wsum);
    }
    if (valid) I.part[(long)rb * n + j] = colacc;
    __syncthreads();
    tile_rows_store(wsum, rows, i0, cb, m, I.part2);
    tile_level_totals(hw, nlev, I.hist);
}

// Gradient merge: r = Xt e, c = Xt^T e into rc.  32 entries of (r, c) per
// block with 8 lanes each: lane s sums the partials s, s + 8, ..., and the 8
// sums of an entry are combined in lane order; the block's part of
// ||a - r||_1 + ||b - c||_1 goes to blk2 for k_grad_decide.  `early`: right
// after a full step applied by the fused first trial (whose partials are the
// next gradient's), for those instances only; a later round then skips them.
__global__ __launch_bounds__(256) void k_grad_merge(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl,
                                                    KP kp, int early) {
    const int b = blockIdx.y;
    if (ctrl[b].phase != PH_NEWTON || (early ? ctrl[b].ls_state != LS_APPLIED : ctrl[b].decided)) return;
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n, N = m + n;
    if ((int)blockIdx.x * 32 >= N) return;
    const int c = threadIdx.x & 31, sl = threadIdx.x >> 5;
    const int k = blockIdx.x * 32 + c;
    __shared__ double ss[8][32];
    double s = 0.0;
    if (k < m) {
        for (int cb = sl; cb < I.ncb; cb += 8) s += I.part2[(long)cb * m + k];
    } else if (k < N) {
        const int j = k - m;
        for (int rb = sl; rb < I.nrb; rb += 8) s += I.part[(long)rb * n + j];
    }
    ss[sl][c] = s;
    __syncthreads();
    if (threadIdx.x < 32) {
        double dev = 0.0;
        if (k < N) {
            double t = 0.0;
            for (int q = 0; q < 8; ++q) t += ss[q][c];
            I.rc[k] = t;
            dev = fabs(((k < m) ? I.a[k] : I.b[k - m]) - t);
        }
        for (int o = 16; o > 0; o >>= 1) dev += __shfl_xor(dev, o);  // lanes 0..31 of wave 0
        if (threadIdx.x == 0) I.blk2[blockIdx.x] = dev;
    }
}

// Newton control: residual, convergence, Sparsify level (one block per instance).
__global__ __launch_bounds__(256) void k_grad_decide(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl,
                                                     KP kp, int early) {
    const int b = blockIdx.x;
    if (ctrl[b].phase != PH_NEWTON) return;
    if (early && ctrl[b].ls_state != LS_APPLIED) return;
    if (!early && ctrl[b].decided) {  // decided right after the previous step (early)
        __syncthreads();
        if (threadIdx.x == 0) {
            ctrl[b].decided = 0;
            ctrl[b].grad_ready = 0;
        }
        return;
    }
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n;
    __shared__ double sh[4];
    const double res = block_sum_array<256>(I.blk2, (m + n + 31) / 32, sh);
    Ctrl& S = ctrl[b];
    __shared__ int s_go;
    if (threadIdx.x == 0) {
        S.resid = res;
        int go = 0;
        if (!isfinite(res)) {
            S.nonfinite = 1;
            S.phase = PH_DONE;
        } else if (res <= (S.k_out >= S.K_out - 1 ? S.tol_fin : S.tol_in)) {
            S.phase = PH_DONE;
        } else if (S.t >= kp.T2) {
            S.flags |= (S.k_out >= S.K_out - 1) ? 1 : 2;
            S.phase = PH_DONE;
        } else {
            go = 1;
        }
        s_go = go;
    }
    __syncthreads();
    if (s_go) {
        // tot[l] = number of entries whose highest kept level is l
        __shared__ long tot[NLEV];
        const int nlev = kp.nlev;
        if ((int)threadIdx.x < nlev) tot[threadIdx.x] = I.hist[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == 0) {
            const double lim = kp.budget * (double)(m + n - 1);
            // no level within the budget: keep no entry (the Newton system is
            // then its diagonal), never a kept set the CSR/CSC arrays cannot hold
            int lev = LEV_NONE;
            long cum = 0;
            // count kept at level l = sum_{l' >= l} tot[l']; smallest l within the budget
            long kept[NLEV];
            for (int l = nlev - 1; l >= 0; --l) {
                cum += tot[l];
                kept[l] = cum;
            }
            for (int l = 0; l < nlev; ++l)
                if ((double)kept[l] <= lim) {
                    lev = l;
                    break;
                }
            S.level = lev;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < NLEV) I.hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        // early and continuing: the next round skips this instance's Newton
        // pass, merge and decision (the gradient is the fused trial's)
        const int keep = early && S.phase == PH_NEWTON;
        S.grad_ready = keep;
        S.decided = keep;
    }
}

// ---------------------------------------------------------------------------
// a6: Sparsify at the chosen level: keep Xt_ij >= rho*10^lev*min(a_i,b_j).
// Three steps, all tile-parallel and deterministic:
//   k_count  kept entries per (row, column block) and per (row block, column)
//   k_scan   CSR row pointers and CSC column pointers (exclusive scans), and
//            the CG's storage form: jagged-diagonal (one-block CG instances,
//            when it fits) or row-contiguous with a binned row list
//   k_fill   both copies of S in one pass: CSR rows in column order (ballot
//            prefix within the tile row), CSC columns in row order, each entry
//            at the slot the storage form gives it.
// count and fill take the keep decision with the same arithmetic, so the
// pointers match what the fill writes.
// ---------------------------------------------------------------------------
// Position of the e-th entry (in index order) of a row of nq quads starting at
// entry `start`: quads are stored transposed, component u of quad q holding
// entry u*nq + q, so that the lanes reading quads q, q+1, ... of a row gather
// consecutive entries (nearby columns) for each component.
__device__ __forceinline__ int quad_slot(int start, int nq, int e) {
    const unsigned q = (unsigned)e % (unsigned)nq, u = (unsigned)e / (unsigned)nq;
    return start + 4 * (int)q + (int)u;
}

template <class Src>
__global__ __launch_bounds__(256) void k_count(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp) {
    const BlkRef br = blk_ref(kp.toff, kp.count);
    const int b = br.b, tl = br.l;
    if (ctrl[b].phase != PH_NEWTON) return;
    const DevInst& I = insts[b];
    const int rb = tl / I.ncb, cb = tl - rb * I.ncb;
    const int m = I.m, n = I.n;
    count_work(ctrl, b, W_FILL, m, n, tl);
    const int i0 = rb * I.R, rows = min(I.R, m - i0);
    __shared__ double sF[TILE_RMAX], sLa[TILE_RMAX];
    __shared__ int wc[TILE_RMAX][4];
    if ((int)threadIdx.x < rows) {
        sF[threadIdx.x] = I.F[i0 + threadIdx.x];
        sLa[threadIdx.x] = I.loga[i0 + threadIdx.x];
    }
    const Src src(I);
    __shared__ typename Src::Row sRow[TILE_RMAX];
    tile_row_table(src, sRow, i0, rows);
    __syncthreads();
    const int j = cb * TILE_C + threadIdx.x;
    const bool valid = j < n;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double lev = (double)ctrl[b].level, kap = ctrl[b].kappa, ie = kp.inv_eta, lrho = kp.log_rho;
    const double Gj = valid ? ldg(I.G + j) : 0.0, lbj = valid ? ldg(I.logb + j) : 0.0;
    int cc = 0;
    const int jc = valid ? j : 0;  // a column in range for the loads of idle lanes
    const typename Src::Col cj = src.col(jc);
    for (int r0 = 0; r0 < rows; r0 += 4) {
        double cv[4];  // the group's cost values first (loads issued together)
#pragma unroll
        for (int u = 0; u < 4; ++u) cv[u] = src.at(sRow[min(r0 + u, rows - 1)], cj);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = r0 + u;
            if (r < rows) {
                bool keep = false;
                if (valid) keep = lev_q(expo(sF[r], Gj, kap, cv[u], ie), lrho, sLa[r], lbj) >= lev;
                cc += keep ? 1 : 0;
                const unsigned long long bal = __ballot(keep);
                if (lane == 0) wc[r][w] = (int)__popcll(bal);
            }
        }
    }
    __syncthreads();
    if (valid) I.cntc[(long)rb * n + j] = cc;
    if ((int)threadIdx.x < rows) {
        const int r = threadIdx.x;
        I.cntr[(long)(i0 + r) * I.ncb + cb] = wc[r][0] + wc[r][1] + wc[r][2] + wc[r][3];
    }
}

// Exclusive prefix sums in place over len counts at p[0], p[stride], ...;
// returns the total.  Counts are loaded 16 at a time before any is stored, so
// the loads of a chunk are in flight together.
__device__ __forceinline__ int prefix_in_place(int* __restrict__ p, long stride, int len) {
    constexpr int CH = 16;
    int c = 0;
    for (int q0 = 0; q0 < len; q0 += CH) {
        int v[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) v[u] = (q0 + u < len) ? p[(long)(q0 + u) * stride] : 0;
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (q0 + u < len) {
                p[(long)(q0 + u) * stride] = c;
                c += v[u];
            }
    }
    return c;
}

// Per row of M (CSR row, then CSC column): the kept count over the column
// (row) blocks, and those per-block counts turned into exclusive prefix sums in
// place (the fill reads them as the entry index of its first kept entry).
// The totals go to rowbin, which k_scan reads before it writes the row list.
__global__ __launch_bounds__(256) void k_scan_totals(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl) {
    const int b = blockIdx.y;
    if (ctrl[b].phase != PH_NEWTON) return;
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= m + n) return;
    I.rowbin[k] = (k < m) ? prefix_in_place(I.cntr + (long)k * I.ncb, 1, I.ncb)
                          : prefix_in_place(I.cntc + (k - m), n, I.nrb);
}


// Jagged-diagonal storage for the one-block CG (see Ctrl::jds).  Each row of a
// half (rows of S, then rows of S^T) of nq quads is cut into nq / JDS_PQ full
// pieces and, if nq is not a multiple, one shorter piece; the pieces of a half
// are ordered by length, longest first, so that the pieces longer than q take
// positions 0 .. cnt(q) - 1 and quad q of the piece at position v is stored
// at quad jdp[q] + v, jdp[q] = cnt(0) + ... + cnt(q - 1).  The lanes of a
// wave, one piece each, then read consecutive quads.  Per row k, rowbin[k]
// receives jds_info: the position of its first full piece (the full pieces
// are consecutive) in the low 16 bits, 1 + the position of its shorter piece
// (0: none) in the high bits.  Within a length the pieces follow the row
// order (the full pieces of a row consecutive).  Returns false, writing
// nothing but Ctrl::jds = 0, when a half has more pieces than the CG's LDS
// array of partial sums holds (pcg_parts(pcg_ept(N))).
template <class NQ>
__device__ bool jds_layout(const DevInst& I, Ctrl& C, int m, int N, NQ nq_of) {
    __shared__ int hist[2][JDS_PQ + 1];
    const int tid = threadIdx.x;
    if (tid < 2 * (JDS_PQ + 1)) (&hist[0][0])[tid] = 0;
    __syncthreads();
    for (int k = tid; k < N; k += 1024) {
        const int nq = nq_of(k), h = k >= m;
        const int F = nq / JDS_PQ, rem = nq - F * JDS_PQ;
        if (F) atomicAdd(&hist[h][JDS_PQ], F);
        if (rem) atomicAdd(&hist[h][rem], 1);
    }
    __syncthreads();
    if (tid < 2) {
        const int h = tid;
        // hist[h][L] (count of pieces of length L) -> first position of that
        // length = number of pieces longer than L; hist[h][0] = all pieces
        int acc = 0;
        for (int L = JDS_PQ; L >= 1; --L) {
            const int c = hist[h][L];
            hist[h][L] = acc;
            acc += c;
        }
        hist[h][0] = acc;
        int d = 0;
        C.jdp[h][0] = 0;
        for (int q = 0; q < JDS_PQ; ++q) {
            d += hist[h][q];  // pieces longer than q
            C.jdp[h][q + 1] = d;
        }
    }
    __syncthreads();
    const int vmax = pcg_parts(pcg_ept(N));
    if (hist[0][0] > vmax || hist[1][0] > vmax) {
        if (tid == 0) C.jds = 0;
        return false;
    }
    // positions within each length in row order (so that neighbouring lanes
    // take neighbouring rows): per half, chunks of 1024 rows; the full pieces
    // by a block-wide exclusive scan of their counts, the shorter piece of
    // each length by per-wave ballots
    __shared__ int wcnt[16][JDS_PQ + 1];  // per wave: pieces per length (full: [JDS_PQ])
    const int w = tid >> 6, lane = tid & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int h = 0; h < 2; ++h) {
        const int lo = h ? m : 0, hi = h ? N : m;
        for (int c0 = lo; c0 < hi; c0 += 1024) {
            const int k = c0 + tid;
            const int nq = k < hi ? nq_of(k) : 0;
            const int F = nq / JDS_PQ, rem = nq - F * JDS_PQ;
            int incl = F;  // inclusive scan of F over the wave
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(incl, o);
                if (lane >= o) incl += t;
            }
            int rank = 0;
#pragma unroll
            for (int L = 1; L < JDS_PQ; ++L) {
                const unsigned long long bal = __ballot(rem == L);
                if (rem == L) rank = (int)__popcll(bal & below);
                if (lane == 0) wcnt[w][L] = (int)__popcll(bal);
            }
            if (lane == 63) wcnt[w][JDS_PQ] = incl;
            __syncthreads();
            int fb = hist[h][JDS_PQ] + incl - F, pp = -1;
            for (int q = 0; q < w; ++q) fb += wcnt[q][JDS_PQ];
            if (rem) {
                pp = hist[h][rem] + rank;
                for (int q = 0; q < w; ++q) pp += wcnt[q][rem];
            }
            if (k < hi) I.rowbin[k] = (F ? fb : 0) | ((pp + 1) << 16);
            __syncthreads();
            if (tid <= JDS_PQ && tid >= 1) {  // advance the cursors past this chunk
                int t = 0;
                for (int q = 0; q < 16; ++q) t += wcnt[q][tid];
                hist[h][tid] += t;
            }
            __syncthreads();
        }
    }
    if (tid == 0) C.jds = 1;
    return true;
}

// Slot (entry index in the half's arrays) of entry e of a row of nq quads
// with jds_info `info` (see jds_layout); entry e lies in piece e / (4 JDS_PQ).
__device__ __forceinline__ int jds_slot(const int* jdp, int info, int nq, int e) {
    const int p = e / (4 * JDS_PQ), e2 = e - p * (4 * JDS_PQ);
    const int v = (p < nq / JDS_PQ) ? (info & 0xffff) + p : (info >> 16) - 1;
    return 4 * (jdp[e2 >> 2] + v) + (e2 & 3);
}

__global__ __launch_bounds__(1024) void k_scan(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl) {
    const int b = blockIdx.x;
    if (ctrl[b].phase != PH_NEWTON) return;
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n, N = m + n;
    __shared__ int ish[16];
    __shared__ long lsh[16];
    // kept entries of row k of M (k < m: row of S; else column k - m), from k_scan_totals
    const int* __restrict__ tot = I.rowbin;
    auto kept = [&](int k) { return tot[k]; };
    long real = 0;
    block_scan_excl<1024>(
        [&](int i) {
            const int c = kept(i);
            real += c;
            return (c + 3) & ~3;
        },
        m, I.rowptr, I.nnz_cap, ish);
    block_scan_excl<1024>([&](int j) { return (kept(m + j) + 3) & ~3; }, n, I.colptr, I.nnz_cap, ish);
    // unpadded count of S (fixed-order integer sum)
    {
        long v = real;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & 63) == 0) lsh[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            long t = 0;
            for (int w = 0; w < 16; ++w) t += lsh[w];
            ctrl[b].nnz = (int)(t < I.nnz_cap ? t : I.nnz_cap);
        }
    }
    // the pointers written above are visible to the whole block after the barrier
    __syncthreads();
    auto nq_of = [&](int k) {
        return (k < m) ? (I.rowptr[k + 1] - I.rowptr[k]) >> 2 : (I.colptr[k - m + 1] - I.colptr[k - m]) >> 2;
    };
    // one-block CG instances: the jagged-diagonal form when it fits
    if (!(I.cgfmt & 1) && jds_layout(I, ctrl[b], m, N, nq_of)) return;
    if (threadIdx.x == 0) ctrl[b].jds = 0;
    // otherwise rows of M grouped by quad count for the CG's product, in row
    // order within each bin: a counting pass (per-wave ballots, wave totals in
    // LDS), the bin offsets, then a placing pass over 1024-row chunks in order
    constexpr int NG2 = 2 * NBIN;
    __shared__ int wcnt[16][NG2];
    __shared__ int boff[NG2];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    auto bin_of = [&](int k) {
        const int nq = nq_of(k);
        const int t = nq <= 1 ? 0 : nq <= 2 ? 1 : nq <= 4 ? 2 : nq <= 8 ? 3 : nq <= 16 ? 4 : 5;
        return (k < m ? 0 : NBIN) + t;
    };
    {
        int mine[NG2];
#pragma unroll
        for (int g = 0; g < NG2; ++g) mine[g] = 0;
        for (int base = 0; base < N; base += 1024) {
            const int k = base + threadIdx.x;
            const int gk = k < N ? bin_of(k) : -1;
#pragma unroll
            for (int g = 0; g < NG2; ++g) mine[g] += (int)__popcll(__ballot(gk == g));
        }
        if (lane == 0)
#pragma unroll
            for (int g = 0; g < NG2; ++g) wcnt[w][g] = mine[g];
    }
    __syncthreads();
    __shared__ int btot[NG2];
    if ((int)threadIdx.x < NG2) {
        int t = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) t += wcnt[q][threadIdx.x];
        btot[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int off = 0;
#pragma unroll
        for (int g = 0; g < NG2; ++g) {
            boff[g] = off;
            ctrl[b].binoff[g] = off;
            off += btot[g];
        }
        ctrl[b].binoff[NG2] = off;
    }
    __syncthreads();
    for (int base = 0; base < N; base += 1024) {
        const int k = base + threadIdx.x;
        const int gk = k < N ? bin_of(k) : -1;
        unsigned long long myb = 0ull;
#pragma unroll
        for (int g = 0; g < NG2; ++g) {
            const unsigned long long bal = __ballot(gk == g);
            if (gk == g) myb = bal;
            if (lane == 0) wcnt[w][g] = (int)__popcll(bal);
        }
        __syncthreads();
        if (gk >= 0) {
            int woff = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q) woff += q < w ? wcnt[q][gk] : 0;
            I.rowbin[boff[gk] + woff + (int)__popcll(myb & below)] = k;
        }
        __syncthreads();
        if ((int)threadIdx.x < NG2) {
            int tot = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q) tot += wcnt[q][threadIdx.x];
            boff[threadIdx.x] += tot;
        }
        __syncthreads();
    }
}

// Index storage of S and S^T.  uint16: the column (of S) or row (of S^T)
// index itself.  int32: the byte offset of the vector entry the product
// gathers, 8 (o + k) with o = m for the columns of S and o = 0 for the rows of
// S^T, so that a product reads p at base + offset with no unpacking or scaling
// (the host admits int32 storage only while 8 (m + n) fits in an int).
__device__ __forceinline__ void put_ix(unsigned short* p, int slot, int k, int) { p[slot] = (unsigned short)k; }
__device__ __forceinline__ void put_ix(int* p, int slot, int k, int o) { p[slot] = 8 * (o + k); }

template <class Src, class VT>
__global__ __launch_bounds__(256) void k_fill(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp) {
    const BlkRef br = blk_ref(kp.toff, kp.count);
    const int b = br.b, tl = br.l;
    if (ctrl[b].phase != PH_NEWTON) return;
    const DevInst& I = insts[b];
    const int rb = tl / I.ncb, cb = tl - rb * I.ncb;
    const int m = I.m, n = I.n;
    const int i0 = rb * I.R, rows = min(I.R, m - i0);
    __shared__ double sF[TILE_RMAX], sLa[TILE_RMAX];
    __shared__ int sStart[TILE_RMAX], sNq[TILE_RMAX], sE0[TILE_RMAX], sInfo[TILE_RMAX];
    __shared__ int sJd[2][JDS_PQ + 1];
    __shared__ double sT[64];
    texp_table(sT);
    __shared__ int wc[TILE_RMAX][4];
    const int jds = ctrl[b].jds;  // storage form chosen by k_scan (uniform over the block)
    if ((int)threadIdx.x < rows) {
        const int i = i0 + threadIdx.x;
        sF[threadIdx.x] = I.F[i];
        sLa[threadIdx.x] = I.loga[i];
        sE0[threadIdx.x] = I.cntr[(long)i * I.ncb + cb];  // prefix over the column blocks (k_scan)
        sStart[threadIdx.x] = I.rowptr[i];
        sNq[threadIdx.x] = (I.rowptr[i + 1] - I.rowptr[i]) >> 2;
        sInfo[threadIdx.x] = jds ? I.rowbin[i] : 0;
    }
    if (jds && (int)threadIdx.x < 2 * (JDS_PQ + 1)) (&sJd[0][0])[threadIdx.x] = (&ctrl[b].jdp[0][0])[threadIdx.x];
    __shared__ typename Src::Row sRow[TILE_RMAX];
    tile_row_table(Src(I), sRow, i0, rows);
    __syncthreads();
    // slot of entry e of a row of S (jd = sJd[0]) or of S^T (sJd[1])
    auto slot_of = [&](const int* jd, int start, int nq, int info, int e) {
        return jds ? jds_slot(jd, info, nq, e) : quad_slot(start, nq, e);
    };
    const int j = cb * TILE_C + threadIdx.x;
    const bool valid = j < n;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double lev = (double)ctrl[b].level, kap = ctrl[b].kappa, ie = kp.inv_eta, lrho = kp.log_rho;
    const bool u16 = (I.cgfmt & 2) != 0;  // index storage of this instance (uniform over the block)
    auto put = [&](void* arr, int slot, int k, int o) {
        if (u16)
            put_ix(static_cast<unsigned short*>(arr), slot, k, o);
        else
            put_ix(static_cast<int*>(arr), slot, k, o);
    };
    const Src src(I);
    const double Gj = valid ? ldg(I.G + j) : 0.0, lbj = valid ? ldg(I.logb + j) : 0.0;
    int ce = 0, cstart = 0, cnq = 0, cinfo = 0;  // entry index within column j, its start and quad count
    if (valid) {
        ce = I.cntc[(long)rb * n + j];  // prefix over the row blocks (k_scan)
        cstart = I.colptr[j];
        cnq = (I.colptr[j + 1] - cstart) >> 2;
        if (jds) cinfo = I.rowbin[m + j];
    }
    // the column's facts for the write phase, where any lane of the wave may
    // write an entry of this column
    __shared__ int sCs[TILE_C], sCn[TILE_C], sCi[TILE_C];
    sCs[threadIdx.x] = cstart;
    sCn[threadIdx.x] = cnq;
    sCi[threadIdx.x] = cinfo;
    const int jc = valid ? j : 0;  // a column in range for the loads of idle lanes
    const typename Src::Col cj = src.col(jc);
    const unsigned long long below = (1ull << lane) - 1ull;
    // Writes, KCH rows at a time: each wave first lists its kept entries of
    // those rows in LDS (row by row, in lane order within a row), then writes
    // them with every lane taking one listed entry, so that no lane idles
    // while the few kept lanes of a row write theirs.  The value, CSR entry
    // index e and CSC entry index (the column's running count) of each entry
    // are those an entry-by-entry pass gives, so every slot receives the same
    // value.
    constexpr int KCH = 4;
    __shared__ double kX[4][KCH * 64];
    __shared__ int kRL[4][KCH * 64], kE[4][KCH * 64], kCe[4][KCH * 64];
    // the tile's rows in passes of RS (the exponents of a pass in registers)
    constexpr int RS = 16;
#pragma unroll
    for (int h0 = 0; h0 < TILE_RMAX; h0 += RS) {
        if (h0 >= rows) break;  // uniform over the block
        const int hr = min(RS, rows - h0);
        double xr[RS];
        unsigned keepm = 0;
#pragma unroll
        for (int r = 0; r < RS; ++r) xr[r] = src.at(sRow[h0 + min(r, hr - 1)], cj);  // loads issued together
#pragma unroll
        for (int r = 0; r < RS; ++r) {
            const double cr = xr[r];
            xr[r] = 0.0;
            bool keep = false;
            if (r < hr && valid) {
                xr[r] = expo(sF[h0 + r], Gj, kap, cr, ie);
                keep = lev_q(xr[r], lrho, sLa[h0 + r], lbj) >= lev;
            }
            if (r < hr) {
                const unsigned long long bal = __ballot(keep);
                if (lane == 0) wc[h0 + r][w] = (int)__popcll(bal);
            }
            keepm |= keep ? (1u << r) : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int c0 = 0; c0 < RS; c0 += KCH) {
            int cnt = 0;  // listed entries of the wave (uniform over it)
#pragma unroll
            for (int u = 0; u < KCH; ++u) {
                const int r = c0 + u, rt = h0 + r;
                const bool keep = (keepm >> r) & 1u;
                const unsigned long long bal = __ballot(keep);
                if (keep) {
                    int woff = 0;
                    for (int q = 0; q < w; ++q) woff += wc[rt][q];
                    const int rank = (int)__popcll(bal & below);
                    const int pos = cnt + rank;
                    kX[w][pos] = xr[r];
                    kRL[w][pos] = (lane << 8) | rt;
                    kE[w][pos] = sE0[rt] + woff + rank;
                    kCe[w][pos] = ce;
                    ++ce;
                }
                cnt += (int)__popcll(bal);
            }
            __syncthreads();
            for (int it = lane; it < cnt; it += 64) {
                const int rl = kRL[w][it];
                const int r = rl & 0xff, t = w * 64 + (rl >> 8);  // row in the tile, thread of the column
                const VT v = (VT)texp(kX[w][it], sT);
                const int e = kE[w][it], nq = sNq[r];
                if (e < 4 * nq) {
                    const int slot = slot_of(sJd[0], sStart[r], nq, sInfo[r], e);
                    put(I.col, slot, cb * TILE_C + t, m);
                    static_cast<VT*>(I.val)[slot] = v;
                }
                const int cev = kCe[w][it], cq = sCn[t];
                if (cev < 4 * cq) {
                    const int slot = slot_of(sJd[1], sCs[t], cq, sCi[t], cev);
                    put(I.rowT, slot, i0 + r, 0);
                    static_cast<VT*>(I.valT)[slot] = v;
                }
            }
            __syncthreads();  // the lists are rewritten for the next rows
        }
    }
    // pads (index 0, value 0) up to a whole number of quads: rows of S in the
    // last column block, columns of S^T in the last row block
    if (rb == I.nrb - 1 && valid)
        for (; ce < 4 * cnq; ++ce) {
            const int slot = slot_of(sJd[1], cstart, cnq, cinfo, ce);
            put(I.rowT, slot, 0, 0);
            static_cast<VT*>(I.valT)[slot] = (VT)0;
        }
    if (cb == I.ncb - 1 && (int)threadIdx.x < rows) {
        const int r = threadIdx.x, nq = sNq[r];
        for (int e = sE0[r] + wc[r][0] + wc[r][1] + wc[r][2] + wc[r][3]; e < 4 * nq; ++e) {
            const int slot = slot_of(sJd[0], sStart[r], nq, sInfo[r], e);
            put(I.col, slot, 0, m);
            static_cast<VT*>(I.val)[slot] = (VT)0;
        }
    }
}

// ---------------------------------------------------------------------------
// a7: truncated CG on the Newton system M d = eta*grad P, where
// M = [D_r S; S^T D_c] = -eta * (sparsified Hessian of eq. (eppa-hess)),
// D_r = diag(r), D_c = diag(c).  CG runs on the Schur complement of the
// column block,
//   (D_r - S D_c^-1 S^T) x = b_1 - S D_c^-1 b_2,   y = D_c^-1 (b_2 - S^T x),
// with the preconditioner D_r and x0 = 0.  M couples rows only to columns
// (property A), so CG on the reduced system reaches a residual in half the
// iterations CG on M with diag(M) needs, at the same cost per iteration (one
// product with S^T, one with S).  With y eliminated exactly the residual of
// M's system is (reduced residual, 0), so the stop ||res||_2 <= cg_rtol *
// ||b||_2 (or cg_max iterations) is the rule for M's system itself.  For
// m + n <= WCG_MAX_N one block of 1024 threads per instance; each thread owns
// the vector entries k = tid + 1024 t (the row iterate, residual and direction
// in registers, the rest in LDS); the products gather from LDS, one lane per
// row piece when S is stored in the jagged-diagonal form (jds_layout; the
// piece sums then added per row in order), else by lane groups over the
// binned rows.  Larger instances take the wide CG below.
// Afterwards the line-search inputs <grad P, d>, <a,dF>+<b,dG> and the
// resolution test.
// ---------------------------------------------------------------------------
// Off-diagonal part of M times p (S v for a row k < m, S^T u for k >= m), row-
// contiguous form.  Rows are stored in aligned, transposed quads (see quad_slot); the entry
// order inside a row does not matter for the product.  The rows of one bin
// (similar quad counts) are handled by groups of G lanes, so the lanes of a
// wave do rows of about the same length; a lane loads each quad (its 4
// indices and 4 values) with one vector load each and keeps several quads in
// flight.  ptr arrays: CSR row pointers (rp, m+1) and CSC column pointers
// (cp, n+1), in LDS (one-block CG) or global memory (wide CG); bins: the row
// list.
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

typedef double f64x4 __attribute__((ext_vector_type(4)));

// one quad of a row as loaded: its 4 stored indices and its 4 values, one
// vector load each (kept packed until used, so that several quads can be in
// flight without many registers)
template <class IX>
struct QuadIx;
template <>
struct QuadIx<unsigned short> {
    typedef u16x4 T;
};
template <>
struct QuadIx<int> {
    typedef i32x4 T;
};
template <class VT>
struct QuadVal;
template <>
struct QuadVal<float> {
    typedef f32x4 T;
};
template <>
struct QuadVal<double> {
    typedef f64x4 T;
};

// The four arrays of S and S^T, read once per kernel (a per-row load of the
// descriptor's fields would put a dependent global load in front of every row).
template <class IX, class VT>
struct SpArrays {
    const IX* col;
    const VT* val;
    const IX* rowT;
    const VT* valT;
    __device__ __forceinline__ explicit SpArrays(const DevInst& I)
        : col(static_cast<const IX*>(I.col)),
          val(static_cast<const VT*>(I.val)),
          rowT(static_cast<const IX*>(I.rowT)),
          valT(static_cast<const VT*>(I.valT)) {}
};

// entry of the gathered vector named by a stored index (see put_ix): pv is the
// vector's half for uint16 indices, the whole vector for int32 byte offsets
template <class IX>
__device__ __forceinline__ double gat(const double* __restrict__ pv, int x) {
    if constexpr (sizeof(IX) == 4)
        return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(pv) + x);
    else
        return pv[x];
}

template <class IX, class XV, class WV>
__device__ __forceinline__ double quad_dot(const XV& x, const WV& w, const double* __restrict__ pv) {
    return ((double)w.x * gat<IX>(pv, (int)x.x) + (double)w.y * gat<IX>(pv, (int)x.y)) +
           ((double)w.z * gat<IX>(pv, (int)x.z) + (double)w.w * gat<IX>(pv, (int)x.w));
}

// Products of the rows bins[lo..hi) of M's off-diagonal part: G lanes per
// row, lane lg taking the row's quads lg, lg + G, ..., U quads in flight (the
// loads of a step are issued together, also for the lane's last < U quads);
// fin(k, (M p)_k) is called once per row.
template <int G, int U, int NT, class IX, class VT, class Fin>
__device__ __forceinline__ void spmv_bin(const SpArrays<IX, VT>& A, int m, const int* bins, int lo, int hi,
                                         const int* rp, const int* cp, const double* __restrict__ pv, Fin fin) {
    typedef typename QuadIx<IX>::T XV;
    typedef typename QuadVal<VT>::T WV;
    constexpr int NG = NT / G;
    const int g = threadIdx.x / G, lg = threadIdx.x % G;
    for (int t = lo + g; t < hi; t += NG) {
        const int k = bins[t];
        const bool row = k < m;
        const XV* ix = reinterpret_cast<const XV*>(row ? A.col : A.rowT);
        const WV* vl = reinterpret_cast<const WV*>(row ? A.val : A.valT);
        const int* ptr = row ? rp + k : cp + (k - m);
        const double* pvo = (sizeof(IX) == 2 && row) ? pv + m : pv;
        const int q1 = ptr[1] >> 2;
        int q = (ptr[0] >> 2) + lg;
        double s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) s[u] = 0.0;
        for (; q + (U - 1) * G < q1; q += U * G) {
            XV x[U];
            WV w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                x[u] = ldg(ix + q + u * G);
                w[u] = ldg(vl + q + u * G);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) s[u] += quad_dot<IX>(x[u], w[u], pvo);
        }
        if (U > 1 && q < q1) {
            XV x[U > 1 ? U - 1 : 1];
            WV w[U > 1 ? U - 1 : 1];
#pragma unroll
            for (int u = 0; u < U - 1; ++u)
                if (q + u * G < q1) {
                    x[u] = ldg(ix + q + u * G);
                    w[u] = ldg(vl + q + u * G);
                    }
#pragma unroll
            for (int u = 0; u < U - 1; ++u)
                if (q + u * G < q1) s[u] += quad_dot<IX>(x[u], w[u], pvo);
        }
        double tot = s[0];
#pragma unroll
        for (int u = 1; u < U; ++u) tot += s[u];
        const double sum = group_sum<G>(tot);
        if (lg == 0) fin(k, sum);
    }
}

// single-block CG products: a row of up to 2^t quads gets 2^(t - CG_LANE_SHIFT)
// lanes (at least one), each with CG_QUADS quads in flight (measured best of
// shifts 1..3 and 2..4 quads in flight on 28x28 grid instances)
constexpr int CG_LANE_SHIFT = 1;
constexpr int CG_QUADS = 3;
constexpr int cg_lanes(int quads) { return (quads >> CG_LANE_SHIFT) > 1 ? (quads >> CG_LANE_SHIFT) : 1; }
// One half of M's off-diagonal product inside one block: bo = the NBIN + 1
// bin offsets of the rows of S (out[i] = (S v)_i, v = pv[m..]) or of the rows
// of S^T (out[m + j] = (S^T u)_j, u = pv[0..m)).  Bin t holds rows of up to
// 2^t quads (the last bin: more); each row gets cg_lanes(2^t) lanes, so that
// a lane takes a few quads of its row.
template <int NT, class IX, class VT>
__device__ __forceinline__ void spmv_part(const SpArrays<IX, VT>& A, int m, const int* bins, const int* bo,
                                          const int* rp, const int* cp, const double* __restrict__ pv,
                                          double* __restrict__ out) {
    auto fin = [out](int k, double v) { out[k] = v; };
    spmv_bin<1, CG_QUADS, NT, IX, VT>(A, m, bins, bo[0], bo[1], rp, cp, pv, fin);
    spmv_bin<cg_lanes(2), CG_QUADS, NT, IX, VT>(A, m, bins, bo[1], bo[2], rp, cp, pv, fin);
    spmv_bin<cg_lanes(4), CG_QUADS, NT, IX, VT>(A, m, bins, bo[2], bo[3], rp, cp, pv, fin);
    spmv_bin<cg_lanes(8), CG_QUADS, NT, IX, VT>(A, m, bins, bo[3], bo[4], rp, cp, pv, fin);
    spmv_bin<cg_lanes(16), CG_QUADS, NT, IX, VT>(A, m, bins, bo[4], bo[5], rp, cp, pv, fin);
    spmv_bin<cg_lanes(32), CG_QUADS, NT, IX, VT>(A, m, bins, bo[5], bo[6], rp, cp, pv, fin);
}

// One half of M's off-diagonal product in the jagged-diagonal form (see
// jds_layout): a lane sums piece v (its quads in order, U in flight) into
// part[v]; jd = the half's quad offsets jdp[0..JDS_PQ] in LDS.  The lanes of
// a wave take consecutive pieces of about the same length, so each of its
// quad loads reads consecutive memory and no lane waits for a cross-lane
// reduction.
// element k of an array of V, the byte offset formed in 32 bits (so that the
// load takes the array's base from scalar registers; one-block instances' S
// arrays are far below 4 GiB)
template <class V>
__device__ __forceinline__ V ld32(const V* base, int k) {
    return ldg(reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + (unsigned)k * (unsigned)sizeof(V)));
}

template <int U, int NT, class IX, class VT>
__device__ __forceinline__ void jds_half(const IX* ixa, const VT* vla, const int* jd, const double* __restrict__ pv,
                                         double* __restrict__ part) {
    typedef typename QuadIx<IX>::T XV;
    typedef typename QuadVal<VT>::T WV;
    const XV* ix = reinterpret_cast<const XV*>(ixa);
    const WV* vl = reinterpret_cast<const WV*>(vla);
    const int V = jd[1];  // every piece has at least one quad
    for (int v = threadIdx.x; v < V; v += NT) {
        double s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) s[u] = 0.0;
        int q = 0;
        // quads q .. q+U-1 exist while the piece is longer than q+U-1
        // (unrolled twice: 2U quads' loads in flight per lane; fully unrolled,
        // every quad of the piece would be, and the registers spill)
#pragma unroll 2
        for (; q + U <= JDS_PQ && v < jd[q + U] - jd[q + U - 1]; q += U) {
            XV x[U];
            WV w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                x[u] = ld32(ix, jd[q + u] + v);
                w[u] = ld32(vl, jd[q + u] + v);
            }
            // every gather of the U quads is issued before the first product
            double g[U][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                g[u][0] = gat<IX>(pv, (int)x[u].x);
                g[u][1] = gat<IX>(pv, (int)x[u].y);
                g[u][2] = gat<IX>(pv, (int)x[u].z);
                g[u][3] = gat<IX>(pv, (int)x[u].w);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                s[u] += ((double)w[u].x * g[u][0] + (double)w[u].y * g[u][1]) +
                        ((double)w[u].z * g[u][2] + (double)w[u].w * g[u][3]);
        }
        // the piece's last quads (fewer than U)
        if (U > 1) {
            XV x[U > 1 ? U - 1 : 1];
            WV w[U > 1 ? U - 1 : 1];
            bool h[U > 1 ? U - 1 : 1];
#pragma unroll
            for (int u = 0; u < U - 1; ++u) {
                h[u] = q + u < JDS_PQ && v < jd[q + u + 1] - jd[q + u];
                if (h[u]) {
                    x[u] = ld32(ix, jd[q + u] + v);
                    w[u] = ld32(vl, jd[q + u] + v);
                    }
            }
#pragma unroll
            for (int u = 0; u < U - 1; ++u)
                if (h[u]) s[u] += quad_dot<IX>(x[u], w[u], pv);
        }
        double tot = s[0];
#pragma unroll
        for (int u = 1; u < U; ++u) tot += s[u];
        part[v] = tot;
    }
}
constexpr int JDS_QUADS = 2;  // quads in flight per lane in jds_half (2 and 4 measured alike)

// kind: the CG's work class (W_CG, W_CG_ROWS or W_CG_WIDE)
__device__ __forceinline__ void ls_setup(Ctrl& S, int it, double gd, double dab, double fa, const KP& kp,
                                         int kind) {
    S.last_cg = it;
    S.cg_total += it;
    S.work[kind] += 2.0 * (double)S.nnz * (double)it;
    S.fused = 0;
    S.gd = gd;
    S.dab = dab;
    S.fa = fa;
    S.ls_h = 0;
    if (!(gd > 0.0)) {
        S.ls_state = LS_FAILED;
    } else if (kp.ls_c1 * gd <= 64.0 * DBL_EPSILON * fa) {
        S.ls_state = LS_ACCEPTED;  // increase below the evaluation's resolution: full step
        S.alpha = 1.0;
    } else {
        S.ls_state = LS_PENDING;
    }
}

template <int NT, int EPT, class IX, class VT, bool JDS>
__global__ __launch_bounds__(NT) void k_pcg_lds(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp) {
    const int b = blockIdx.x;
    // wide instances take the wide CG; the instances stored the other way the other instantiation
    if (ctrl[b].phase != PH_NEWTON || (insts[b].cgfmt & 1) || ctrl[b].jds != (JDS ? 1 : 0)) return;
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n, N = m + n;
    if (pcg_threads(N) != NT) return;  // the block size is the instance's own (pcg_threads)
    // LDS: sp, the direction p on the rows and D_c^-1 S^T p on the columns;
    // sAp, products of the current half; sdg, the diagonal (r, c); the
    // pointers and the binned row list
    __shared__ double sp[NT * EPT];
    __shared__ double sAp[pcg_parts(EPT)];
    __shared__ double sdg[NT * EPT];
    __shared__ double sh[32];
    __shared__ int sptr[NT * EPT + 2];
    __shared__ int sbin[NT * EPT];
    __shared__ int sbo[2 * NBIN + 1];
    __shared__ int sjd[2][JDS_PQ + 1];
    const int tid = threadIdx.x;
    const SpArrays<IX, VT> A(I);
    for (int k = tid; k <= m; k += NT) sptr[k] = I.rowptr[k];
    for (int k = tid; k <= n; k += NT) sptr[m + 1 + k] = I.colptr[k];
    for (int k = tid; k < N; k += NT) sbin[k] = I.rowbin[k];  // row list, or jds_info per row
    const int* rp = sptr;
    const int* cp = sptr + m + 1;
    const int* bins = sbin;
    if (tid <= 2 * NBIN) sbo[tid] = ctrl[b].binoff[tid];
    if (tid < 2 * (JDS_PQ + 1)) (&sjd[0][0])[tid] = (&ctrl[b].jdp[0][0])[tid];
    // half h of M's off-diagonal product of the vector in sp: row-contiguous
    // form, (M p)_k into sAp[k]; jagged-diagonal form, piece sums into sAp
    auto prod = [&](int h) {
        if constexpr (!JDS)
            spmv_part<NT, IX, VT>(A, m, bins, sbo + h * NBIN, rp, cp, sp, sAp);
        else if (h == 0)
            jds_half<JDS_QUADS, NT, IX, VT>(A.col, A.val, sjd[0], sp, sAp);
        else
            jds_half<JDS_QUADS, NT, IX, VT>(A.rowT, A.valT, sjd[1], sp, sAp);
    };
    // (M p)_k after prod (and a barrier): the sum of row k's pieces in order
    auto rowval = [&](int k) -> double {
        if constexpr (!JDS) return sAp[k];
        const int info = sbin[k];
        const int nf = ((k < m) ? (rp[k + 1] - rp[k]) >> 2 : (cp[k - m + 1] - cp[k - m]) >> 2) / JDS_PQ;
        const int fb = info & 0xffff, pp = (info >> 16) - 1;
        double v = 0.0;
        for (int p = 0; p < nf; ++p) v += sAp[fb + p];
        if (pp >= 0) v += sAp[pp];
        return v;
    };
    const double eta = kp.eta;
    // right-hand side eta (target - diagonal) of entry k (recomputed where needed)
    auto rhs = [&](int k) { return eta * (((k < m) ? I.a[k] : I.b[k - m]) - sdg[k]); };
    // registers: on the rows the iterate x, residual r, direction p; the
    // inverse diagonal dinv (rows: the Jacobi preconditioner D_r^-1; columns:
    // the D_c^-1 of the reduced matrix)
    double x[EPT], r[EPT], p[EPT], dinv[EPT];
    double bb = 0.0;
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const int k = tid + NT * t;
        x[t] = r[t] = p[t] = 0.0;
        dinv[t] = 0.0;
        if (k < N) {
            const double dk = I.rc[k];
            sdg[k] = dk;
            dinv[t] = 1.0 / dk;
            const double tg = (k < m) ? I.a[k] : I.b[k - m];
            const double bk = eta * (tg - dk);
            bb += bk * bk;
            if (k >= m) sp[k] = bk / dk;  // D_c^-1 b_2
        }
    }
    bb = block_sum<NT>(bb, sh);  // also orders the LDS writes above
    const double bn = sqrt(bb);
    prod(0);  // S D_c^-1 b_2 on the rows
    __syncthreads();
    double rr = 0.0, rz = 0.0;
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const int k = tid + NT * t;
        if (k < m) {
            r[t] = rhs(k) - rowval(k);
            p[t] = r[t] * dinv[t];
            sp[k] = p[t];
            rr += r[t] * r[t];
            rz += r[t] * p[t];
        }
    }
    block_sum2<NT>(rr, rz, sh);
    // q_k = ((D_r - S D_c^-1 S^T) p)_k, read twice per iteration from the same
    // products (nothing writes sAp in between)
    auto qval = [&](int k, double pk) { return sdg[k] * pk - rowval(k); };
    constexpr int NW = NT / 64;
    __shared__ double spq[NW];  // per-wave parts of <p, q>
    int it = 0;
    if (bn > 0.0 && sqrt(rr) > kp.cg_rtol * bn) {
        while (it < kp.cg_max) {
            __syncthreads();
            prod(1);  // y = S^T p
            __syncthreads();
            // D_c^-1 y on the columns, and <p, q> = <p, D_r p> - <y, D_c^-1 y>
            // (q = (D_r - S D_c^-1 S^T) p) in per-wave parts that the barrier
            // before the next product publishes
            double pq = 0.0;
#pragma unroll
            for (int t = 0; t < EPT; ++t) {
                const int k = tid + NT * t;
                if (k < m) {
                    pq += sdg[k] * (p[t] * p[t]);
                } else if (k < N) {
                    const double y = rowval(k), z = y * dinv[t];
                    sp[k] = z;
                    pq -= y * z;
                }
            }
            pq = wave_sum(pq);
            if ((tid & 63) == 0) spq[tid >> 6] = pq;
            __syncthreads();
            prod(0);  // S D_c^-1 S^T p
            __syncthreads();
            pq = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) pq += spq[w];
            if (!(pq > 0.0)) break;
            const double al = rz / pq;
            double rz2 = 0.0;
            rr = 0.0;
#pragma unroll
            for (int t = 0; t < EPT; ++t) {
                const int k = tid + NT * t;
                if (k < m) {
                    x[t] += al * p[t];
                    r[t] -= al * qval(k, p[t]);
                    rr += r[t] * r[t];
                    rz2 += r[t] * (r[t] * dinv[t]);
                }
            }
            block_sum2_nolead<NT>(rr, rz2, sh);  // sh's last readers are several barriers back
            ++it;
            if (sqrt(rr) <= kp.cg_rtol * bn) break;
            const double be = rz2 / rz;
            rz = rz2;
#pragma unroll
            for (int t = 0; t < EPT; ++t) {
                const int k = tid + NT * t;
                if (k < m) {
                    p[t] = r[t] * dinv[t] + be * p[t];
                    sp[k] = p[t];
                }
            }
        }
    }
    // the column part y = D_c^-1 (b_2 - S^T x)
    __syncthreads();
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const int k = tid + NT * t;
        if (k < m) sp[k] = x[t];
    }
    __syncthreads();
    prod(1);
    __syncthreads();
    double gd = 0.0, dab = 0.0, fa = 0.0;
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const int k = tid + NT * t;
        if (k < N) {
            if (k >= m) x[t] = (rhs(k) - rowval(k)) / sdg[k];
            const double tg = (k < m) ? I.a[k] : I.b[k - m];
            I.d[k] = x[t];
            gd += (tg - sdg[k]) * x[t];
            dab += tg * x[t];
            fa += fabs(tg * x[t]);
        }
    }
    gd = block_sum<NT>(gd, sh);
    dab = block_sum<NT>(dab, sh);
    fa = block_sum<NT>(fa, sh);
    if (tid == 0) ls_setup(ctrl[b], it, gd, dab, fa, kp, JDS ? W_CG : W_CG_ROWS);
}

// ---------------------------------------------------------------------------
// Wide CG for instances with m + n > WCG_MAX_N: the same Schur-complement CG,
// with each product spread over many blocks (WCG_ROWS rows of one half of M
// per block, over the binned row list) and the vector steps over blocks of
// WCG_VROWS rows, their dot products merged in fixed order from per-block
// parts.  Kernel boundaries order the memory (no device fences); the host
// runs iterations in chunks between readbacks, and an instance that has
// stopped (cg_on = 0) makes every later launch return at once.
// Vectors (global): x = I.d, res = cgw[0..m), bv = cgw[N..2N) (rhs),
// p = cgw[2N..3N) (direction on the rows, D_c^-1 S^T p on the columns),
// q = cgw[3N..4N).
// ---------------------------------------------------------------------------
// One half of M's product for the blocks of rows [lo, hi) of the part's list.
template <class IX, class VT, class Fin>
__device__ __forceinline__ void spmv_range(const DevInst& I, int m, const int* bins, const int* bo, int lo, int hi,
                                           const double* __restrict__ pv, Fin fin) {
    const SpArrays<IX, VT> A(I);
#define WB_(G, g)                                                                                              \
    {                                                                                                          \
        const int a_ = max(lo, bo[g]), b_ = min(hi, bo[g + 1]);                                               \
        if (a_ < b_) spmv_bin<cg_lanes(G), 3, WCG_NT, IX, VT>(A, m, bins, a_, b_, I.rowptr, I.colptr, pv, fin);  \
    }
    WB_(1, 0) WB_(2, 1) WB_(4, 2) WB_(8, 3) WB_(16, 4) WB_(32, 5)
#undef WB_
}

// rhs, x = 0, D_c^-1 b_2 into p's column part; ||rhs||
// Instances that take part: every one with matrix-free products (dense = 1),
// else those whose cgfmt selects the wide CG.
__device__ __forceinline__ bool wcg_member(const DevInst& I, int dense) { return dense || (I.cgfmt & 1); }

__global__ __launch_bounds__(1024) void k_wcg_begin(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp,
                                                    int dense) {
    const int b = blockIdx.x;
    if (ctrl[b].phase != PH_NEWTON) return;
    if (!wcg_member(insts[b], dense)) {
        if (threadIdx.x == 0) ctrl[b].cg_on = 0;
        return;
    }
    if (dense && threadIdx.x == 0) ctrl[b].nnz = insts[b].m * insts[b].n;  // a product reads every entry
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n, N = m + n;
    double* __restrict__ bv = I.cgw + N;
    double* __restrict__ p = I.cgw + 2 * N;
    __shared__ double sh[32];
    double bb = 0.0;
    for (int k = threadIdx.x; k < N; k += 1024) {
        const double tg = (k < m) ? I.a[k] : I.b[k - m];
        const double rh = kp.eta * (tg - I.rc[k]);
        bv[k] = rh;
        I.d[k] = 0.0;
        if (k >= m) p[k] = rh / I.rc[k];
        bb += rh * rh;
    }
    bb = block_sum<1024>(bb, sh);
    if (threadIdx.x == 0) {
        ctrl[b].cg_bnorm = sqrt(bb);
        ctrl[b].cg_it = 0;
        ctrl[b].cg_on = 1;
    }
}

// columns: p[m + j] = (S^T p_rows)_j / c_j (and the iteration count
// advanced), or q[m + j] = (S^T x)_j when `final` (after the iterations); rows: q[i] = (S p_cols)_i for the start
// (`final` = 2), or in the iterations q[i] = r_i p_i - (S p_cols)_i and the
// block's part of <p, q> in blk[block] (blocks of WCG_ROWS rows of the binned
// list, in order)
template <class IX, class VT>
__global__ __launch_bounds__(WCG_NT) void k_wcg_half(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl,
                                                   int cols, int final) {
    const int b = blockIdx.y;
    if (ctrl[b].phase != PH_NEWTON || (!final && !ctrl[b].cg_on)) return;
    const DevInst& I = insts[b];
    // wide instances whose index storage is this launch's
    constexpr int ix16 = sizeof(IX) == 2 ? 2 : 0;
    if (!(I.cgfmt & 1) || (I.cgfmt & 2) != ix16) return;
    const int m = I.m, N = m + I.n;
    const int* bo = ctrl[b].binoff + (cols ? NBIN : 0);
    const int lo = bo[0] + blockIdx.x * WCG_ROWS;
    const int hi = min(bo[NBIN], lo + WCG_ROWS);
    if (lo >= hi) return;
    double* __restrict__ p = I.cgw + 2 * N;
    double* __restrict__ q = I.cgw + 3 * N;
    const double* __restrict__ dg = I.rc;
    if (cols && !final && blockIdx.x == 0 && threadIdx.x == 0) ctrl[b].cg_it += 1;  // iteration t starts: cg_it = t + 1
    if (cols) {
        if (final)
            spmv_range<IX, VT>(I, m, I.rowbin, bo, lo, hi, I.d, [q](int k, double v) { q[k] = v; });
        else
            spmv_range<IX, VT>(I, m, I.rowbin, bo, lo, hi, p, [p, dg](int k, double v) { p[k] = v / dg[k]; });
    } else if (final) {
        spmv_range<IX, VT>(I, m, I.rowbin, bo, lo, hi, p, [q](int k, double v) { q[k] = v; });
    } else {
        __shared__ double sh[32];
        double pq = 0.0;
        spmv_range<IX, VT>(I, m, I.rowbin, bo, lo, hi, p, [&](int k, double v) {
            const double w = dg[k] * p[k] - v;
            q[k] = w;
            pq += p[k] * w;
        });
        pq = block_sum<WCG_NT>(pq, sh);
        if (threadIdx.x == 0) I.blk[blockIdx.x] = pq;
    }
}

// after S D_c^-1 b_2: residual, preconditioned residual, first direction
__global__ __launch_bounds__(1024) void k_wcg_start(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp,
                                                    int dense) {
    const int b = blockIdx.x;
    if (ctrl[b].phase != PH_NEWTON || !wcg_member(insts[b], dense)) return;
    const DevInst& I = insts[b];
    const int m = I.m, N = m + I.n;
    double* __restrict__ res = I.cgw;
    const double* __restrict__ bv = I.cgw + N;
    double* __restrict__ p = I.cgw + 2 * N;
    const double* __restrict__ q = I.cgw + 3 * N;
    __shared__ double sh[32];
    double rr = 0.0, rz = 0.0;
    for (int i = threadIdx.x; i < m; i += 1024) {
        const double r = bv[i] - q[i];
        res[i] = r;
        const double z = r / I.rc[i];
        p[i] = z;
        rr += r * r;
        rz += r * z;
    }
    block_sum2<1024>(rr, rz, sh);
    if (threadIdx.x == 0) {
        Ctrl& S = ctrl[b];
        S.cg_rzs[0] = rz;
        if (!(S.cg_bnorm > 0.0) || sqrt(rr) <= kp.cg_rtol * S.cg_bnorm || kp.cg_max <= 0) S.cg_on = 0;
    }
}

// One iteration's vector work, over blocks of WCG_VROWS rows (the products
// left q = D_r p - S D_c^-1 S^T p and the parts of <p, q> in blk, npq of them
// per instance, pq_rows rows each).  In iteration t the columns half-product
// has set cg_it = t + 1; <res, z> of iteration t is cg_rzs[t & 1], so no block
// reads a scalar that another block of the same launch writes, and no launch of
// an iteration takes a per-iteration argument.  Each block sums the same
// partials in the same order, so every block takes the same step.
// k_wcg_alpha: step length, x and res, the parts of ||res||^2 and <res, z> in blk2.
__global__ __launch_bounds__(256) void k_wcg_alpha(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl,
                                                   int pq_rows) {
    const int b = blockIdx.y;
    if (ctrl[b].phase != PH_NEWTON || !ctrl[b].cg_on) return;
    const DevInst& I = insts[b];
    const int m = I.m, N = m + I.n;
    const int i0 = blockIdx.x * WCG_VROWS;
    if (i0 >= m) return;
    __shared__ double sh[32];
    const double pq = block_sum_array<256>(I.blk, (m + pq_rows - 1) / pq_rows, sh);
    if (!(pq > 0.0)) {
        // every block sees the same pq and returns before reading cg_it; the
        // breakdown iteration does not count
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctrl[b].cg_on = 0;
            ctrl[b].cg_it -= 1;
        }
        return;
    }
    const int t = ctrl[b].cg_it - 1;
    const double al = ctrl[b].cg_rzs[t & 1] / pq;
    double* __restrict__ res = I.cgw;
    const double* __restrict__ p = I.cgw + 2 * N;
    const double* __restrict__ q = I.cgw + 3 * N;
    double* __restrict__ x = I.d;
    const double* __restrict__ dg = I.rc;
    double rr = 0.0, rz = 0.0;
    for (int i = i0 + threadIdx.x; i < min(m, i0 + WCG_VROWS); i += 256) {
        x[i] += al * p[i];
        const double r = res[i] - al * q[i];
        res[i] = r;
        rr += r * r;
        rz += r * (r / dg[i]);
    }
    block_sum2<256>(rr, rz, sh);
    if (threadIdx.x == 0) {
        I.blk2[2 * blockIdx.x] = rr;
        I.blk2[2 * blockIdx.x + 1] = rz;
    }
}

// k_wcg_beta: stop test and the next direction p = D_r^-1 res + beta p.
__global__ __launch_bounds__(256) void k_wcg_beta(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp) {
    const int b = blockIdx.y;
    if (ctrl[b].phase != PH_NEWTON || !ctrl[b].cg_on) return;
    const DevInst& I = insts[b];
    const int m = I.m, N = m + I.n;
    const int i0 = blockIdx.x * WCG_VROWS;
    if (i0 >= m) return;
    const int nv = (m + WCG_VROWS - 1) / WCG_VROWS;
    double rr = 0.0, rz2 = 0.0;
    for (int c = 0; c < nv; ++c) {
        rr += I.blk2[2 * c];
        rz2 += I.blk2[2 * c + 1];
    }
    const int t = ctrl[b].cg_it - 1;
    const double rz = ctrl[b].cg_rzs[t & 1];
    const int go = !(sqrt(rr) <= kp.cg_rtol * ctrl[b].cg_bnorm) && t + 1 < kp.cg_max;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (go)
            ctrl[b].cg_rzs[(t + 1) & 1] = rz2;
        else
            ctrl[b].cg_on = 0;  // read by later launches only (no block of this one needs it)
    }
    if (!go) return;
    const double be = rz2 / rz;
    const double* __restrict__ res = I.cgw;
    double* __restrict__ p = I.cgw + 2 * N;
    const double* __restrict__ dg = I.rc;
    for (int i = i0 + threadIdx.x; i < min(m, i0 + WCG_VROWS); i += 256) p[i] = res[i] / dg[i] + be * p[i];
}

// Matrix-free products with the full Hessian (params.hvp = 1): the coupling
// block is X~ itself, recomputed tile by tile from the potentials and the
// streamed cost as in the Newton pass.  cols = 1: column partials
// part[rb][j] = sum_i X~_ij u_i of the tile (u = the direction on the rows, or
// x when `final`); cols = 0: row partials part2[cb][i] = sum_j X~_ij w_j
// (w = D_c^-1 X~^T p on the columns).  Merged in fixed order by k_mf_merge.
template <class Src, class T>
__global__ __launch_bounds__(256) void k_mf_tile(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp,
                                                 int cols, int final) {
    const BlkRef br = blk_ref(kp.toff, kp.count);
    const int b = br.b, tl = br.l;
    if (ctrl[b].phase != PH_NEWTON || (!final && !ctrl[b].cg_on)) return;
    const DevInst& I = insts[b];
    const int rb = tl / I.ncb, cb = tl - rb * I.ncb;
    const int m = I.m, n = I.n, N = m + n;
    const int i0 = rb * I.R, rows = min(I.R, m - i0);
    const double* __restrict__ p = I.cgw + 2 * N;
    const double* __restrict__ u = final ? I.d : p;
    __shared__ double sF[TILE_RMAX], su[TILE_RMAX], wsum[TILE_RMAX][4];
    __shared__ double sT[64];
    texp_table(sT);
    if ((int)threadIdx.x < rows) {
        sF[threadIdx.x] = I.F[i0 + threadIdx.x];
        su[threadIdx.x] = u[i0 + threadIdx.x];
    }
    const Src src(I);
    __shared__ typename Src::Row sRow[TILE_RMAX];
    tile_row_table(src, sRow, i0, rows);
    __syncthreads();
    const int j = cb * TILE_C + threadIdx.x;
    const bool valid = j < n;
    const double kap = ctrl[b].kappa, ie = kp.inv_eta;
    const typename Src::Col cj = src.col(valid ? j : 0);
    const double Gj = valid ? ldg(I.G + j) : 0.0;
    if (cols) {
        double acc = 0.0;
        if (valid)
            for (int r = 0; r < rows; ++r) acc += (double)ex<T>(expo(sF[r], Gj, kap, src.at(sRow[r], cj), ie), sT) * su[r];
        if (valid) I.part[(long)rb * n + j] = acc;
    } else {
        const double wj = valid ? p[m + j] : 0.0;
        for (int r0 = 0; r0 < rows; r0 += 4) {
            double v[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int r = r0 + t;
                v[t] = (valid && r < rows) ? (double)ex<T>(expo(sF[r], Gj, kap, src.at(sRow[min(r, rows - 1)], cj), ie), sT) * wj : 0.0;
            }
            wave_rows4(v, r0, wsum);
        }
        __syncthreads();
        tile_rows_store(wsum, rows, i0, cb, m, I.part2);
    }
}

// cols = 1: t_j = sum over row blocks -> p[m + j] = t_j / c_j (and the
// iteration count advanced), or q[m + j] = t_j when `final`; cols = 0: t_i = sum over column blocks -> q_i = t_i for the
// start (`final` = 2), or in the iterations q_i = r_i p_i - t_i and the
// block's part of <p, q> in blk[block].
__global__ __launch_bounds__(256) void k_mf_merge(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, int cols,
                                                  int final) {
    const int b = blockIdx.y;
    if (ctrl[b].phase != PH_NEWTON || (!final && !ctrl[b].cg_on)) return;
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n, N = m + n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    double* __restrict__ p = I.cgw + 2 * N;
    double* __restrict__ q = I.cgw + 3 * N;
    if (cols) {
        if (!final && k == 0) ctrl[b].cg_it += 1;  // iteration t starts: cg_it = t + 1
        if (k >= n) return;
        double t = 0.0;
        for (int rb = 0; rb < I.nrb; ++rb) t += I.part[(long)rb * n + k];
        if (final)
            q[m + k] = t;
        else
            p[m + k] = t / I.rc[m + k];
    } else if (final) {
        if (k >= m) return;
        double t = 0.0;
        for (int cb = 0; cb < I.ncb; ++cb) t += I.part2[(long)cb * m + k];
        q[k] = t;
    } else {
        if ((int)blockIdx.x * 256 >= m) return;  // whole block: no partial beyond this instance's rows
        __shared__ double sh[32];
        double pq = 0.0;
        if (k < m) {
            double t = 0.0;
            for (int cb = 0; cb < I.ncb; ++cb) t += I.part2[(long)cb * m + k];
            const double w = I.rc[k] * p[k] - t;
            q[k] = w;
            pq = p[k] * w;
        }
        pq = block_sum<256>(pq, sh);
        if (threadIdx.x == 0) I.blk[blockIdx.x] = pq;
    }
}

// y = D_c^-1 (b_2 - S^T x) and the line-search inputs
__global__ __launch_bounds__(1024) void k_wcg_finish(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp,
                                                     int dense) {
    const int b = blockIdx.x;
    if (ctrl[b].phase != PH_NEWTON || !wcg_member(insts[b], dense)) return;
    const DevInst& I = insts[b];
    const int m = I.m, N = m + I.n;
    const double* __restrict__ bv = I.cgw + N;
    const double* __restrict__ q = I.cgw + 3 * N;
    __shared__ double sh[32];
    double gd = 0.0, dab = 0.0, fa = 0.0;
    for (int k = threadIdx.x; k < N; k += 1024) {
        if (k >= m) I.d[k] = (bv[k] - q[k]) / I.rc[k];
        const double x = I.d[k];
        const double tg = (k < m) ? I.a[k] : I.b[k - m];
        gd += (tg - I.rc[k]) * x;
        dab += tg * x;
        fa += fabs(tg * x);
    }
    gd = block_sum<1024>(gd, sh);
    dab = block_sum<1024>(dab, sh);
    fa = block_sum<1024>(fa, sh);
    if (threadIdx.x == 0) ls_setup(ctrl[b], ctrl[b].cg_it, gd, dab, fa, kp, W_CG_WIDE);
}

// ---------------------------------------------------------------------------
// a8: Armijo trials on P^k (eq. eppa-sub-dual), NT step sizes per pass:
//   P(f+al df, g+al dg) - P(f,g) = al(<a,df>+<b,dg>) - eta sum_ij Xt_ij expm1(al(df_i+dg_j)/eta)
// accept the first al = beta^h with increase >= c1*al*<grad P, d>.
// ---------------------------------------------------------------------------
// First Armijo trial (alpha = 1), fused with the next Newton pass: with
// e = Xt_ij and t = e*expm1(delta_ij), Xt at the trial point is e + t, whose
// row/column sums and Sparsify histogram are exactly what the next k_grad
// would compute if the full step is accepted.
template <class Src>
__global__ __launch_bounds__(256) void k_ls_first(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl,
                                                  KP kp) {
    const BlkRef br = blk_ref(kp.toff, kp.count);
    const int b = br.b, tl = br.l;
    if (ctrl[b].phase != PH_NEWTON || ctrl[b].ls_state != LS_PENDING) return;
    const DevInst& I = insts[b];
    const int rb = tl / I.ncb, cb = tl - rb * I.ncb;
    const int m = I.m, n = I.n;
    count_work(ctrl, b, W_LS, m, n, tl);
    const int i0 = rb * I.R, rows = min(I.R, m - i0);
    __shared__ unsigned hw[NLEV * TILE_C / 4];  // [level][thread] byte counters
    __shared__ double wsum[TILE_RMAX][4];
    __shared__ double sF[TILE_RMAX], sD[TILE_RMAX], sLa[TILE_RMAX], sA[TILE_RMAX], sA1[TILE_RMAX];
    __shared__ double sT[64];
    texp_table(sT);
    unsigned char* hcol = reinterpret_cast<unsigned char*>(hw);
    for (int k = threadIdx.x; k < NLEV * TILE_C / 4; k += 256) hw[k] = 0u;
    if ((int)threadIdx.x < rows) {
        const int i = i0 + threadIdx.x;
        sF[threadIdx.x] = I.F[i];
        sD[threadIdx.x] = I.d[i] * kp.inv_eta;
        sLa[threadIdx.x] = I.loga[i];
        const double A = expm1(I.d[i] * kp.inv_eta);
        sA[threadIdx.x] = A;
        sA1[threadIdx.x] = 1.0 + A;
    }
    const Src src(I);
    __shared__ typename Src::Row sRow[TILE_RMAX];
    tile_row_table(src, sRow, i0, rows);
    __syncthreads();
    const int j = cb * TILE_C + threadIdx.x;
    const bool valid = j < n;
    const double kap = ctrl[b].kappa, ie = kp.inv_eta, lrho = kp.log_rho;
    const int nlev = kp.nlev;
    double acc = 0.0, colacc = 0.0;
    const double Gj = valid ? ldg(I.G + j) : 0.0, dGj = valid ? ldg(I.d + m + j) * ie : 0.0;
    const double lbj = valid ? ldg(I.logb + j) : 0.0;
    // expm1(a_i + b_j) = A_i + B_j (1 + A_i) with A_i = expm1(a_i), B_j = expm1(b_j)
    const double Bj = expm1(dGj);
    const int jc = valid ? j : 0;  // a column in range for the loads of idle lanes
    const typename Src::Col cj = src.col(jc);
    for (int r0 = 0; r0 < rows; r0 += 4) {
        double cv[4];  // the group's cost values first (loads issued together)
#pragma unroll
        for (int u = 0; u < 4; ++u) cv[u] = src.at(sRow[min(r0 + u, rows - 1)], cj);
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = r0 + u;
            double e1 = 0.0;
            if (valid && r < rows) {
                const double x = expo(sF[r], Gj, kap, cv[u], ie);
                const double e = texp(x, sT);
                const double del = sD[r] + dGj;
                const double t = e * fma(Bj, sA1[r], sA[r]);
                acc += t;
                e1 = e + t;
                const double q = lev_q(x + del, lrho, sLa[r], lbj);
                if (q >= 0.0) {
                    const int l = (q >= (double)(nlev - 1)) ? nlev - 1 : (int)q;
                    hcol[l * TILE_C + threadIdx.x] += 1;
                }
            }
            colacc += e1;
            v[u] = e1;
        }
        wave_rows4(v, r0, wsum);
    }
    if (valid) I.part[(long)rb * n + j] = colacc;
    __syncthreads();
    tile_rows_store(wsum, rows, i0, cb, m, I.part2);
    tile_level_totals(hw, nlev, I.hist);
    __shared__ double sh[4];
    const double bs = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) I.blk[tl] = bs;
}

// Armijo test of the first trial: the block partials in fixed order (a kernel
// of its own, so the tile kernel needs no device-scope fence per block).
__global__ __launch_bounds__(256) void k_ls_first_merge(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl,
                                                        KP kp) {
    const int b = blockIdx.x;
    if (ctrl[b].phase != PH_NEWTON || ctrl[b].ls_state != LS_PENDING) return;
    const DevInst& I = insts[b];
    __shared__ double sh[4];
    const double tot = block_sum_array<256>(I.blk, I.nrb * I.ncb, sh);
    __shared__ int s_acc;
    if (threadIdx.x == 0) {
        Ctrl& S = ctrl[b];
        const double inc = S.dab - kp.eta * tot;
        s_acc = inc >= kp.ls_c1 * S.gd;
        if (!s_acc) {
            S.ls_h = 1;
            if (S.ls_h >= kp.ls_max) S.ls_state = LS_FAILED;
        }
    }
    __syncthreads();
    if (!s_acc) return;
    // full step accepted: apply it here (what k_update does for an accepted
    // step; F + 1.0 * d rounds as F + d there), with the next gradient already
    // formed by the fused trial, so the host can skip k_update
    const int m = I.m, N = m + I.n;
    for (int k = threadIdx.x; k < N; k += 256) {
        if (k < m)
            I.F[k] += I.d[k];
        else
            I.G[k - m] += I.d[k];
    }
    if (threadIdx.x == 0) {
        Ctrl& S = ctrl[b];
        S.alpha = 1.0;
        S.fused = 1;
        S.ls_state = LS_APPLIED;
        S.t += 1;
        S.newton_total += 1;
        S.grad_ready = 1;
    }
}

template <class Src, int NT>
__global__ __launch_bounds__(256) void k_ls(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp) {
    const BlkRef br = blk_ref(kp.toff, kp.count);
    const int b = br.b, tl = br.l;
    if (ctrl[b].phase != PH_NEWTON || ctrl[b].ls_state != LS_PENDING) return;
    const DevInst& I = insts[b];
    const int rb = tl / I.ncb, cb = tl - rb * I.ncb;
    const int m = I.m, n = I.n;
    count_work(ctrl, b, W_LS, m, n, tl);
    const int h0 = ctrl[b].ls_h;
    double al[NT];
    {
        double a0 = 1.0;
        for (int h = 0; h < h0; ++h) a0 *= kp.ls_beta;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            al[t] = a0;
            a0 *= kp.ls_beta;
        }
    }
    const int i0 = rb * I.R, rows = min(I.R, m - i0);
    // trial t: expm1(al_t (a_i + b_j)) = A_it + B_jt (1 + A_it)
    __shared__ double sF[TILE_RMAX], sA[TILE_RMAX][NT], sA1[TILE_RMAX][NT];
    __shared__ double sT[64];
    texp_table(sT);
    for (int k = threadIdx.x; k < rows * NT; k += 256) {
        const int r = k / NT, t = k - r * NT;
        const double A = expm1(al[t] * (I.d[i0 + r] * kp.inv_eta));
        sA[r][t] = A;
        sA1[r][t] = 1.0 + A;
    }
    if ((int)threadIdx.x < rows) sF[threadIdx.x] = I.F[i0 + threadIdx.x];
    const Src src(I);
    __shared__ typename Src::Row sRow[TILE_RMAX];
    tile_row_table(src, sRow, i0, rows);
    __syncthreads();
    const int j = cb * TILE_C + threadIdx.x;
    const bool valid = j < n;
    const double kap = ctrl[b].kappa, ie = kp.inv_eta;
    double acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = 0.0;
    if (valid) {
        const double Gj = ldg(I.G + j), bj = ldg(I.d + m + j) * ie;
        double B[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) B[t] = expm1(al[t] * bj);
        const typename Src::Col cj = src.col(j);
        for (int r = 0; r < rows; ++r) {
            const double e = texp(expo(sF[r], Gj, kap, src.at(sRow[r], cj), ie), sT);
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] += e * fma(B[t], sA1[r][t], sA[r][t]);
        }
    }
    __shared__ double sh[4];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const double s = block_sum<256>(acc[t], sh);
        if (threadIdx.x == 0) I.blk[(long)tl * NT + t] = s;
    }
}

// Armijo tests of a pass of NT trials, first acceptable step size wins.
template <int NT>
__global__ __launch_bounds__(256) void k_ls_merge(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp) {
    const int b = blockIdx.x;
    if (ctrl[b].phase != PH_NEWTON || ctrl[b].ls_state != LS_PENDING) return;
    const DevInst& I = insts[b];
    const int nblk = I.nrb * I.ncb;
    const int h0 = ctrl[b].ls_h;
    const int nt = min(NT, kp.ls_max - h0);
    double al[NT];
    {
        double a0 = 1.0;
        for (int h = 0; h < h0; ++h) a0 *= kp.ls_beta;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            al[t] = a0;
            a0 *= kp.ls_beta;
        }
    }
    __shared__ double sh[4];
    double tot[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        double v = 0.0;
        for (int k = threadIdx.x; k < nblk; k += 256) v += I.blk[(long)k * NT + t];
        tot[t] = block_sum<256>(v, sh);
    }
    if (threadIdx.x == 0) {
        Ctrl& S = ctrl[b];
        int acc_t = -1;
        for (int t = 0; t < nt; ++t) {
            const double inc = al[t] * S.dab - kp.eta * tot[t];
            if (inc >= kp.ls_c1 * al[t] * S.gd) {
                acc_t = t;
                break;
            }
        }
        if (acc_t >= 0) {
            S.alpha = al[acc_t];
            S.ls_state = LS_ACCEPTED;
        } else {
            S.ls_h = h0 + nt;
            if (S.ls_h >= kp.ls_max) S.ls_state = LS_FAILED;
        }
    }
}

// a9: (f, g) += alpha*(df, dg); without an accepted step the instance takes
// one Sinkhorn iteration instead (phase FALLBACK).  One block per instance.
__global__ __launch_bounds__(1024) void k_update(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl) {
    const int b = blockIdx.x;
    if (ctrl[b].phase != PH_NEWTON || ctrl[b].ls_state == LS_APPLIED) return;
    const DevInst& I = insts[b];
    const int m = I.m, N = I.m + I.n;
    const int st = ctrl[b].ls_state;
    const double al = ctrl[b].alpha;
    const bool ready = st == LS_ACCEPTED && ctrl[b].fused;
    if (!ready && (int)threadIdx.x < NLEV) I.hist[threadIdx.x] = 0;  // discard a rejected trial's histogram
    if (st == LS_ACCEPTED)
        for (int k = threadIdx.x; k < N; k += 1024) {
            if (k < m)
                I.F[k] += al * I.d[k];
            else
                I.G[k - m] += al * I.d[k];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        Ctrl& S = ctrl[b];
        S.t += 1;
        S.newton_total += 1;
        S.grad_ready = ready ? 1 : 0;
        if (st != LS_ACCEPTED) {
            S.phase = PH_FALLBACK;
            S.fb_total += 1;
        }
    }
}

// ---------------------------------------------------------------------------
// a1: outer shift, C^{k+1} = C^k + C - f (+) g + eta, warm start (f, g) kept.
// Implicit: (F, Ahat) <- (2F - Ahat, F), (G, Bhat) <- (2G - Bhat, G),
// kappa <- kappa + 1.  Materialised: C^k += C - F (+) G (elementwise kernel),
// Ahat += F, Bhat += G.  Both re-enter the warm-up.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_shift_vec(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl,
                                                    int materialised, int start_phase) {
    const int b = blockIdx.x;
    // only instances that finished an outer iteration and have another to run
    // (in a batch solved together that is every instance; in a live batch the
    // ones admitted this round have just been set up and are warming up)
    if (ctrl[b].phase != PH_DONE || ctrl[b].k_out + 1 >= ctrl[b].K_out) return;
    const DevInst& I = insts[b];
    const int m = I.m, N = I.m + I.n;
    for (int k = threadIdx.x; k < N; k += 1024) {
        double* Fv = (k < m) ? I.F + k : I.G + (k - m);
        double* Av = (k < m) ? I.Ah + k : I.Bh + (k - m);
        const double f = *Fv, a = *Av;
        if (materialised) {
            *Av = a + f;
        } else {
            *Fv = 2.0 * f - a;
            *Av = f;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Ctrl& S = ctrl[b];
        if (!materialised) S.kappa += 1.0;
        S.k_out += 1;
        S.t = 0;
        S.phase = S.nonfinite ? PH_DONE : start_phase;
    }
}

template <class Src>
__global__ __launch_bounds__(256) void k_shift_dense(const DevInst* __restrict__ insts) {
    const int b = blockIdx.y;
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n;
    const long mn = (long)m * n;
    const Src base(I, true);
    for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < mn; q += (long)gridDim.x * 256) {
        const int i = (int)(q / n), j = (int)(q - (long)i * n);
        I.Ck[q] = I.Ck[q] + base.at(i, j) - I.F[i] - I.G[j];
    }
}

// ---------------------------------------------------------------------------
// setup: log marginals, initial duals (f = g = 0), X^0 = a b^T; the marginals
// checked against eq. (ot)'s domain (every entry positive and finite, each
// sum 1 within 1e-10) into Ctrl::margbad, read back by the host before any
// iteration runs.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_init(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp) {
    const int b = blockIdx.x;
    const DevInst& I = insts[b];
    const int m = I.m, N = I.m + I.n;
    const double eta = kp.eta;
    const bool mat = kp.shift_mode != 0;
    __shared__ double sh[32];
    __shared__ int sbad;
    if (threadIdx.x == 0) sbad = 0;
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    int bad = 0;
    for (int k = threadIdx.x; k < N; k += 1024) {
        if (k < m) {
            const double av = I.a[k];
            if (!(av > 0.0) || !isfinite(av)) bad |= 1;
            sa += av;
            const double la = log(av);
            I.loga[k] = la;
            I.Ah[k] = eta * la;
            I.F[k] = mat ? -eta : eta * la - eta;
        } else {
            const double bv = I.b[k - m];
            if (!(bv > 0.0) || !isfinite(bv)) bad |= 4;
            sb += bv;
            const double lb = log(bv);
            I.logb[k - m] = lb;
            I.Bh[k - m] = eta * lb;
            I.G[k - m] = mat ? 0.0 : eta * lb;
        }
    }
    if (bad) atomicOr(&sbad, bad);
    for (int t = threadIdx.x; t < NLEV; t += 1024) I.hist[t] = 0;
    sa = block_sum<1024>(sa, sh);  // its barriers also order the LDS flag
    sb = block_sum<1024>(sb, sh);
    if (threadIdx.x == 0) {
        Ctrl& S = ctrl[b];
        int mb = sbad;
        if (!(fabs(sa - 1.0) <= 1e-10)) mb |= 2;
        if (!(fabs(sb - 1.0) <= 1e-10)) mb |= 8;
        S.margbad = mb;
        S.phase = (S.nonfinite || mb) ? PH_DONE : (kp.T1 > 0 ? PH_WARM : PH_NEWTON);
        S.kappa = 1.0;
        S.k_out = 0;
        S.K_out = kp.K;
        S.tol_in = kp.inner_tol;
        S.tol_fin = kp.final_tol;
    }
}

template <class Src>
__global__ __launch_bounds__(256) void k_init_ck(const DevInst* __restrict__ insts, KP kp) {
    const int b = blockIdx.y;
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n;
    const long mn = (long)m * n;
    const Src base(I, true);
    for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < mn; q += (long)gridDim.x * 256) {
        const int i = (int)(q / n), j = (int)(q - (long)i * n);
        I.Ck[q] = base.at(i, j) - kp.eta * (I.loga[i] + I.logb[j]);
    }
}

// a0 for point clouds: C_ij = |x_i|^2 + |y_j|^2 - 2 <x_i, y_j> with the inner
// products on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  Block = 4 waves,
// a 32x32 tile of C; each wave a 16x16 tile, k in steps of 4 (zero-padded past
// d).  Operand layout of the instruction: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; it receives D[4r + l/16][l%16] in its r-th result, r = 0..3.  The squared norms
// come from the same operand loads (partial over the lane's k slots, summed
// over the 4 lanes sharing l%16).  Rounding of nearly equal points can make
// the expansion slightly negative; it is clamped at 0.
__global__ __launch_bounds__(256) void k_points_cost(const double* __restrict__ x, const double* __restrict__ y,
                                                     int m, int n, int d, double* __restrict__ C) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i0 = blockIdx.y * 32 + (w >> 1) * 16, j0 = blockIdx.x * 32 + (w & 1) * 16;
    const int lr = lane & 15, lk = lane >> 4;
    const int ia = i0 + lr, jb = j0 + lr;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    double xn = 0.0, yn = 0.0;
    for (int k0 = 0; k0 < d; k0 += 4) {
        const int k = k0 + lk;
        const double av = (ia < m && k < d) ? x[(long)ia * d + k] : 0.0;
        const double bv = (jb < n && k < d) ? y[(long)jb * d + k] : 0.0;
        xn += av * av;
        yn += bv * bv;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    // |x_ia|^2, |y_jb|^2: sum over the four lanes with the same l % 16
    xn += __shfl_xor(xn, 16);
    xn += __shfl_xor(xn, 32);
    yn += __shfl_xor(yn, 16);
    yn += __shfl_xor(yn, 32);
    double xr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) xr[r] = __shfl(xn, 4 * r + lk);  // norm of row i0 + 4 r + lk
    const int j = j0 + lr;
    if (j < n) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 4 * r + lk;
            if (i < m) C[(long)i * n + j] = fmax(0.0, (xr[r] + yn) - 2.0 * acc[r]);
        }
    }
}

// a0: max of a dense cost (for the 1/max normalisation) and a finiteness
// check; per-block partial maxima, then the last block writes the scale.
__global__ __launch_bounds__(256) void k_cost_max(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl,
                                                  double* __restrict__ scratch) {
    const int b = blockIdx.y;
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n;
    // whole rows per block (no index division per entry); an instance with
    // fewer rows than the grid's blocks uses m of them (the maximum does not
    // depend on the partition)
    const int nb = min((int)gridDim.x, m);
    if ((int)blockIdx.x >= nb) return;
    double mx = 0.0;
    int bad = 0;
    for (int i = blockIdx.x; i < m; i += nb) {
        const double* __restrict__ row = I.cbase + (long)i * I.ldc;
        for (int j = threadIdx.x; j < n; j += 256) {
            const double v = row[j];
            if (!isfinite(v)) bad = 1;
            mx = fmax(mx, v);
        }
    }
    __shared__ double sm[256];
    __shared__ int sb;
    if (threadIdx.x == 0) sb = 0;
    __syncthreads();
    sm[threadIdx.x] = mx;
    if (bad) atomicOr(&sb, 1);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scratch[(long)b * gridDim.x + blockIdx.x] = sm[0];
        if (sb) atomicOr(&ctrl[b].nonfinite, 1);
    }
    if (!last_block(&ctrl[b].ticket, nb)) return;
    if (threadIdx.x == 0) {
        double M = 0.0;
        for (int k = 0; k < nb; ++k) M = fmax(M, scratch[(long)b * gridDim.x + k]);
        ctrl[b].scale = (M > 0.0) ? 1.0 / M : 1.0;
    }
}

// Copy the scale found by k_cost_max into the descriptors of the instances
// whose scale was not given (bscale <= 0 marks them).
__global__ void k_set_scale(DevInst* insts, Ctrl* ctrl, int count, int exponent_uses_base) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    if (!(insts[b].bscale > 0.0)) {
        const double s = ctrl[b].scale;
        insts[b].bscale = s;
        if (exponent_uses_base) insts[b].cscale = s;
    }
    ctrl[b].scale = insts[b].bscale;
}

// ---------------------------------------------------------------------------
// a10: outputs.  Standard-form potentials at eps = eta/K:
//   alpha = (F + [Ahat])/K, beta = (G + [Bhat])/K  ([.] materialised mode),
// gauge <a,alpha> = <b,beta>; then one pass for X^K, <C,X>, entropy and the
// marginals.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_potentials(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp,
                                                     double K, const int* __restrict__ gate) {
    const int b = blockIdx.x;
    if (gate && !gate[b]) return;  // live batch: only the instances finishing now
    const DevInst& I = insts[b];
    const int m = I.m, N = I.m + I.n;
    const bool mat = kp.shift_mode != 0;
    __shared__ double sh[16];
    double sa = 0.0, sb = 0.0;
    for (int k = threadIdx.x; k < N; k += 1024) {
        if (k < m) {
            const double v = (I.F[k] + (mat ? I.Ah[k] : 0.0)) / K;
            I.alpha[k] = v;
            sa += I.a[k] * v;
        } else {
            const double v = (I.G[k - m] + (mat ? I.Bh[k - m] : 0.0)) / K;
            I.beta[k - m] = v;
            sb += I.b[k - m] * v;
        }
    }
    sa = block_sum<1024>(sa, sh);
    sb = block_sum<1024>(sb, sh);
    const double tg = 0.5 * (sb - sa);
    double du = 0.0;
    for (int k = threadIdx.x; k < N; k += 1024) {
        if (k < m) {
            const double v = I.alpha[k] + tg;
            I.alpha[k] = v;
            du += I.a[k] * v;
        } else {
            const double v = I.beta[k - m] - tg;
            I.beta[k - m] = v;
            du += I.b[k - m] * v;
        }
    }
    du = block_sum<1024>(du, sh);
    if (threadIdx.x == 0) ctrl[b].dual = du;
}

template <class Src>
__global__ __launch_bounds__(256) void k_final(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl, KP kp,
                                               double K, int write_x, const int* __restrict__ gate) {
    const BlkRef br = blk_ref(kp.toff, kp.count);
    const int b = br.b, tl = br.l;
    if (gate && !gate[b]) return;
    const DevInst& I = insts[b];
    const int rb = tl / I.ncb, cb = tl - rb * I.ncb;
    const int m = I.m, n = I.n;
    count_work(ctrl, b, W_FINAL, m, n, tl);
    const int i0 = rb * I.R, rows = min(I.R, m - i0);
    // the tile's rows 16 at a time through red (row sums: 16 lanes per row)
    __shared__ double red[16][TILE_C + 1];
    __shared__ double sh[4];
    const int j = cb * TILE_C + threadIdx.x;
    const bool valid = j < n;
    const double ieps = K * kp.inv_eta;
    const Src base(I, true);
    __shared__ double sA[TILE_RMAX];
    if ((int)threadIdx.x < rows) sA[threadIdx.x] = I.alpha[i0 + threadIdx.x];
    __syncthreads();
    const double bj = valid ? I.beta[j] : 0.0;
    double colacc = 0.0, cst = 0.0, ent = 0.0;
    for (int h0 = 0; h0 < rows; h0 += 16) {  // uniform over the block
        const int hr = min(16, rows - h0);
        for (int r = 0; r < hr; ++r) {
            const int i = i0 + h0 + r;
            double xv = 0.0;
            if (valid) {
                const double c = base.at(i, j);
                const double lx = (sA[h0 + r] + bj - c) * ieps;
                xv = exp(lx);
                cst += c * xv;
                if (xv > 0.0) ent -= xv * lx;
                if (write_x && I.X) I.X[(long)i * n + j] = xv;
            }
            colacc += xv;
            red[r][threadIdx.x] = xv;
        }
        __syncthreads();
        {
            const int r = threadIdx.x >> 4, s = threadIdx.x & 15;
            double v = 0.0;
            if (r < hr)
                for (int k = 0; k < 16; ++k) v += red[r][s * 16 + k];
            v = group_sum<16>(v);
            if (r < hr && s == 0) I.part2[(long)cb * m + i0 + h0 + r] = v;
        }
        __syncthreads();  // red is rewritten by the next rows
    }
    if (valid) I.part[(long)rb * n + j] = colacc;
    cst = block_sum<256>(cst, sh);
    ent = block_sum<256>(ent, sh);
    if (threadIdx.x == 0) {
        I.blk[(long)tl * 2] = cst;
        I.blk[(long)tl * 2 + 1] = ent;
    }
}

__global__ __launch_bounds__(256) void k_final_merge(const DevInst* __restrict__ insts, Ctrl* __restrict__ ctrl,
                                                     const int* __restrict__ gate) {
    const int b = blockIdx.y;
    if (gate && !gate[b]) return;
    const DevInst& I = insts[b];
    const int m = I.m, n = I.n, N = m + n;
    const int nb = (N + 255) / 256;
    if ((int)blockIdx.x >= nb) return;
    __shared__ double sh[4];
    const int k = blockIdx.x * 256 + threadIdx.x;
    double dev = 0.0;
    if (k < m) {
        double s = 0.0;
        for (int cb = 0; cb < I.ncb; ++cb) s += I.part2[(long)cb * m + k];
        dev = fabs(s - I.a[k]);
    } else if (k < N) {
        const int j = k - m;
        double s = 0.0;
        for (int rb = 0; rb < I.nrb; ++rb) s += I.part[(long)rb * n + j];
        dev = fabs(s - I.b[j]);
    }
    const double bs = block_sum<256>(dev, sh);
    if (threadIdx.x == 0) I.blk2[blockIdx.x] = bs;
    if (!last_block(&ctrl[b].ticket, nb)) return;
    const double res = block_sum_array<256>(I.blk2, nb, sh);
    const int nblk = I.nrb * I.ncb;
    double c = 0.0, e = 0.0;
    for (int q = threadIdx.x; q < nblk; q += 256) {
        c += I.blk[(long)q * 2];
        e += I.blk[(long)q * 2 + 1];
    }
    c = block_sum<256>(c, sh);
    e = block_sum<256>(e, sh);
    if (threadIdx.x == 0) {
        Ctrl& S = ctrl[b];
        S.resid = res;
        S.cost = c;
        S.entropy = e;
        if (!isfinite(c) || !isfinite(res)) S.nonfinite = 1;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline dim3 g2(int x, int y) { return dim3((unsigned)(x > 0 ? x : 1), (unsigned)y); }

#define PINS_SRC_DISPATCH(src, KERNEL_TMPL, ...)             \
    do {                                                      \
        if ((src) == SRC_GRID)                                \
            KERNEL_TMPL(GridSrc, ##__VA_ARGS__);              \
        else                                                  \
            KERNEL_TMPL(DenseSrc, ##__VA_ARGS__);             \
    } while (0)

void launch_row_lse(const LaunchCtx& L, int src, bool f32, int mask) {
    const dim3 g(L.total_rowblk);
#define K_(S, T) hipLaunchKernelGGL((k_row_lse<S, T>), g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp, mask)
    if (f32) {
        PINS_SRC_DISPATCH(src, K_, float);
    } else {
        PINS_SRC_DISPATCH(src, K_, double);
    }
#undef K_
}

void launch_col_lse(const LaunchCtx& L, int src, bool f32, int mask) {
    const dim3 g(L.total_tiles);
#define K_(S, T) hipLaunchKernelGGL((k_col_lse<S, T>), g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp, mask)
    if (f32) {
        PINS_SRC_DISPATCH(src, K_, float);
    } else {
        PINS_SRC_DISPATCH(src, K_, double);
    }
#undef K_
}

void launch_col_merge(const LaunchCtx& L, int mask) {
    hipLaunchKernelGGL(k_col_merge, g2((L.max_n + 31) / 32, L.count), dim3(256), 0, L.stream, L.insts, L.ctrl,
                       L.kp, mask);
    hipLaunchKernelGGL(k_col_decide, dim3(L.count), dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp, mask);
}

void launch_grad(const LaunchCtx& L, int src) {
    const dim3 g(L.total_tiles);
#define K_(S) hipLaunchKernelGGL((k_grad<S>), g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp)
    PINS_SRC_DISPATCH(src, K_);
#undef K_
}

void launch_grad_merge(const LaunchCtx& L, bool early) {
    hipLaunchKernelGGL(k_grad_merge, g2((L.max_mn + 31) / 32, L.count), dim3(256), 0, L.stream, L.insts, L.ctrl,
                       L.kp, early ? 1 : 0);
    hipLaunchKernelGGL(k_grad_decide, dim3(L.count), dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp, early ? 1 : 0);
}

template <class VT>
static void launch_fill_t(const LaunchCtx& L, int src, dim3 g) {
#define K_(S) hipLaunchKernelGGL((k_fill<S, VT>), g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp)
    PINS_SRC_DISPATCH(src, K_);
#undef K_
}

void launch_sparsify(const LaunchCtx& L, int src) {
    const dim3 g(L.total_tiles);
#define K_(S) hipLaunchKernelGGL((k_count<S>), g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp)
    PINS_SRC_DISPATCH(src, K_);
#undef K_
    hipLaunchKernelGGL(k_scan_totals, g2((L.max_mn + 255) / 256, L.count), dim3(256), 0, L.stream, L.insts, L.ctrl);
    hipLaunchKernelGGL(k_scan, dim3(L.count), dim3(1024), 0, L.stream, L.insts, L.ctrl);
    if (L.sp_f32)
        launch_fill_t<float>(L, src, g);
    else
        launch_fill_t<double>(L, src, g);
}

// instances with m + n <= WCG_MAX_N (the others take the wide CG); every
// vector of such an instance fits the kernel's LDS arrays.  The entries a
// thread owns beyond an instance's m + n add zeros to its sums, so the
// instance's arithmetic does not depend on the batch's largest m + n.
static_assert(WCG_MAX_N <= 4 * 1024, "k_pcg_lds holds at most 4096 vector entries");
// The 1024-thread CG blocks keep their compute unit to themselves: a launch
// reserves the rest of the unit's LDS as dynamic shared memory that the kernel
// does not use, so that no block of another lane's kernels lands on the unit
// and slows the iterations (measured on the 64-pair batch: 285-286 against
// 289 ms per step).  Zero (no reservation) if the attributes cannot be read.
template <int EPT, class IX, class VT, bool JDS>
static size_t pcg_exclusive_lds() {
    static const size_t pad = [] {
        hipFuncAttributes a;
        int dev = 0, maxs = 0;
        if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&k_pcg_lds<1024, EPT, IX, VT, JDS>)) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&maxs, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
            (size_t)maxs <= a.sharedSizeBytes) {
            (void)hipGetLastError();
            return (size_t)0;
        }
        return (size_t)maxs - a.sharedSizeBytes;
    }();
    return pad;
}

template <class IX, class VT, bool JDS>
static void launch_pcg_t(const LaunchCtx& L) {
    const dim3 g(L.count);
    // instances with m + n <= PCG_SMALL_N: 256-thread blocks, one entry per thread
    if (L.any_tiny) hipLaunchKernelGGL((k_pcg_lds<256, 1, IX, VT, JDS>), g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp);
    if (!L.any_big) return;
    const int ept = (L.max_mn_small + 1023) / 1024;
    const dim3 blk(1024);
    if (ept <= 1) {
        const size_t pad = pcg_exclusive_lds<1, IX, VT, JDS>();
        hipLaunchKernelGGL((k_pcg_lds<1024, 1, IX, VT, JDS>), g, blk, pad, L.stream, L.insts, L.ctrl, L.kp);
    } else if (ept <= 2) {
        const size_t pad = pcg_exclusive_lds<2, IX, VT, JDS>();
        hipLaunchKernelGGL((k_pcg_lds<1024, 2, IX, VT, JDS>), g, blk, pad, L.stream, L.insts, L.ctrl, L.kp);
    } else {
        const size_t pad = pcg_exclusive_lds<4, IX, VT, JDS>();
        hipLaunchKernelGGL((k_pcg_lds<1024, 4, IX, VT, JDS>), g, blk, pad, L.stream, L.insts, L.ctrl, L.kp);
    }
}

template <class IX, class VT>
static void launch_wcg_half_t(const LaunchCtx& L, int cols, int final) {
    const int rows = cols ? L.max_n : L.max_m;
    const dim3 g((rows + WCG_ROWS - 1) / WCG_ROWS, L.count);
    hipLaunchKernelGGL((k_wcg_half<IX, VT>), g, dim3(WCG_NT), 0, L.stream, L.insts, L.ctrl, cols, final);
}

// one launch per index storage present among the wide instances (each skips
// the instances stored the other way)
static void launch_wcg_half(const LaunchCtx& L, int cols, int final) {
    if (L.any_wide16) {
        if (L.sp_f32)
            launch_wcg_half_t<unsigned short, float>(L, cols, final);
        else
            launch_wcg_half_t<unsigned short, double>(L, cols, final);
    }
    if (L.any_wide32) {
        if (L.sp_f32)
            launch_wcg_half_t<int, float>(L, cols, final);
        else
            launch_wcg_half_t<int, double>(L, cols, final);
    }
}

// one half of the product: the sparsified Hessian (src < 0) or matrix-free
// with the full Hessian over cost source src
static void launch_half(const LaunchCtx& L, int src, int cols, int final) {
    if (src < 0) {
        launch_wcg_half(L, cols, final);
        return;
    }
    const dim3 g(L.total_tiles);
#define K_(S, T) hipLaunchKernelGGL((k_mf_tile<S, T>), g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp, cols, final)
    if (L.sp_f32) {
        PINS_SRC_DISPATCH(src, K_, float);  // fast-mixed precision: float exp (exponent formed in double)
    } else {
        PINS_SRC_DISPATCH(src, K_, double);
    }
#undef K_
    hipLaunchKernelGGL(k_mf_merge, g2(((cols ? L.max_n : L.max_m) + 255) / 256, L.count), dim3(256), 0, L.stream,
                       L.insts, L.ctrl, cols, final);
}

void launch_wcg_begin(const LaunchCtx& L, int src) {
    hipLaunchKernelGGL(k_wcg_begin, dim3(L.count), dim3(1024), 0, L.stream, L.insts, L.ctrl, L.kp, src >= 0 ? 1 : 0);
    launch_half(L, src, 0, 2);
    hipLaunchKernelGGL(k_wcg_start, dim3(L.count), dim3(1024), 0, L.stream, L.insts, L.ctrl, L.kp, src >= 0 ? 1 : 0);
}

void launch_wcg_iter(const LaunchCtx& L, int src) {
    launch_half(L, src, 1, 0);
    launch_half(L, src, 0, 0);
    const dim3 g = g2((L.max_m + WCG_VROWS - 1) / WCG_VROWS, L.count);
    const int pq_rows = src < 0 ? WCG_ROWS : 256;  // rows per part of <p, q> (k_wcg_half or k_mf_merge blocks)
    hipLaunchKernelGGL(k_wcg_alpha, g, dim3(256), 0, L.stream, L.insts, L.ctrl, pq_rows);
    hipLaunchKernelGGL(k_wcg_beta, g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp);
}

void launch_wcg_end(const LaunchCtx& L, int src) {
    launch_half(L, src, 1, 1);
    hipLaunchKernelGGL(k_wcg_finish, dim3(L.count), dim3(1024), 0, L.stream, L.insts, L.ctrl, L.kp, src >= 0 ? 1 : 0);
}

// the one-block instances always store int32 byte offsets
void launch_pcg(const LaunchCtx& L, bool jds) {
    if (jds) {
        if (L.sp_f32)
            launch_pcg_t<int, float, true>(L);
        else
            launch_pcg_t<int, double, true>(L);
    } else {
        if (L.sp_f32)
            launch_pcg_t<int, float, false>(L);
        else
            launch_pcg_t<int, double, false>(L);
    }
}

void launch_ls(const LaunchCtx& L, int src, bool first) {
    const dim3 g(L.total_tiles);
    if (first) {
#define K_(S) hipLaunchKernelGGL((k_ls_first<S>), g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp)
        PINS_SRC_DISPATCH(src, K_);
#undef K_
    } else {
#define K_(S, NT) hipLaunchKernelGGL((k_ls<S, NT>), g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp)
        PINS_SRC_DISPATCH(src, K_, LS_T);
#undef K_
    }
    if (first)
        hipLaunchKernelGGL(k_ls_first_merge, dim3(L.count), dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp);
    else
        hipLaunchKernelGGL(k_ls_merge<LS_T>, dim3(L.count), dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp);
}

void launch_update(const LaunchCtx& L) {
    hipLaunchKernelGGL(k_update, dim3(L.count), dim3(1024), 0, L.stream, L.insts, L.ctrl);
}

void launch_shift(const LaunchCtx& L, int base_src) {
    const bool mat = L.kp.shift_mode != 0;
    if (mat) {
        const dim3 g = g2(1024, L.count);
#define K_(S) hipLaunchKernelGGL((k_shift_dense<S>), g, dim3(256), 0, L.stream, L.insts)
        PINS_SRC_DISPATCH(base_src, K_);
#undef K_
    }
    hipLaunchKernelGGL(k_shift_vec, dim3(L.count), dim3(1024), 0, L.stream, L.insts, L.ctrl, mat ? 1 : 0,
                       L.kp.T1 > 0 ? (int)PH_WARM : (int)PH_NEWTON);
}

void launch_init(const LaunchCtx& L, int base_src) {
    hipLaunchKernelGGL(k_init, dim3(L.count), dim3(1024), 0, L.stream, L.insts, L.ctrl, L.kp);
    if (L.kp.shift_mode != 0) {
        const dim3 g = g2(1024, L.count);
#define K_(S) hipLaunchKernelGGL((k_init_ck<S>), g, dim3(256), 0, L.stream, L.insts, L.kp)
        PINS_SRC_DISPATCH(base_src, K_);
#undef K_
    }
}

void launch_points_cost(hipStream_t st, const double* x, const double* y, int m, int n, int d, double* C) {
    hipLaunchKernelGGL(k_points_cost, dim3((n + 31) / 32, (m + 31) / 32), dim3(256), 0, st, x, y, m, n, d, C);
}

void launch_cost_max(const LaunchCtx& L, double* scratch, int nblk, int exponent_uses_base) {
    hipLaunchKernelGGL(k_cost_max, dim3(nblk, L.count), dim3(256), 0, L.stream, L.insts, L.ctrl, scratch);
    hipLaunchKernelGGL(k_set_scale, dim3((L.count + 63) / 64), dim3(64), 0, L.stream, L.insts_mut, L.ctrl, L.count,
                       exponent_uses_base);
}

// zero fill of `words` 8-byte words (control blocks at set-up; a kernel
// rather than a memset node, so the clear is an ordinary launch on the stream)
__global__ __launch_bounds__(256) void k_zero(unsigned long long* __restrict__ p, long words) {
    const long k = (long)blockIdx.x * 256 + threadIdx.x;
    if (k < words) p[k] = 0ull;
}

void launch_zero(hipStream_t st, void* p, size_t bytes) {
    const long words = (long)(bytes / 8);
    if (words > 0)
        hipLaunchKernelGGL(k_zero, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st,
                           (unsigned long long*)p, words);
}

// Address of `scratch` on `device`, looked up once per device with that device
// current (each GPU holds its own copy at its own address), the caller's
// current device restored afterwards.
int noalloc_scratch(int device, void** out) {
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static void* ptr[MAXDEV] = {};
    if (device < 0 || device >= MAXDEV) return PINS_EDEVICE;
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[device]) {
        int prev = 0;
        if (hipGetDevice(&prev) != hipSuccess) return PINS_EDEVICE;
        void* p = nullptr;
        hipError_t e = hipSetDevice(device);
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        (void)hipSetDevice(prev);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return PINS_EDEVICE;
        }
        ptr[device] = p;
    }
    *out = ptr[device];
    return PINS_OK;
}

void launch_final(const LaunchCtx& L, int base_src, double K, bool write_x, const int* gate) {
    hipLaunchKernelGGL(k_potentials, dim3(L.count), dim3(1024), 0, L.stream, L.insts, L.ctrl, L.kp, K, gate);
    const dim3 g(L.total_tiles);
#define K_(S) \
    hipLaunchKernelGGL((k_final<S>), g, dim3(256), 0, L.stream, L.insts, L.ctrl, L.kp, K, write_x ? 1 : 0, gate)
    PINS_SRC_DISPATCH(base_src, K_);
#undef K_
    hipLaunchKernelGGL(k_final_merge, g2((L.max_mn + 255) / 256, L.count), dim3(256), 0, L.stream, L.insts, L.ctrl,
                       gate);
}

}  // namespace pins
