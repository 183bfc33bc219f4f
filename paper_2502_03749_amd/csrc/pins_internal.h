// pins_internal.h -- device-side data layout shared by the HIP kernels and
// the host orchestrator of libpins.so.  Not part of the public ABI.
//
// Representation of the shifted cost (Alg. 2, C^k = C - eta log X^k):
// with X^0 = a b^T and the recovery map of eq. (eppa_x), every shifted cost is
//     C^k = (k+1) C - Ahat (+) Bhat
// for two vectors Ahat (m), Bhat (n).  The kernels therefore evaluate the
// exponent of the recovery map as
//     log Xt_ij = (F_i + G_j - kappa * Csrc_ij) / eta
// where (implicit mode) kappa = k+1, Csrc = C, F = f + Ahat - eta, G = g + Bhat,
// or (materialised mode) kappa = 1, Csrc = C^k stored densely, F = f - eta,
// G = g.  (f, g) are the inner duals of Alg. 2; a Sinkhorn or Newton update of
// (f, g) is the same update of (F, G).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pins {

constexpr int NLEV = 16;     // maximum number of Sparsify levels
constexpr int LEV_NONE = 1 << 20;  // Sparsify level meaning "keep no entry" (no level fits the budget)
constexpr int LS_T = 8;      // trial step sizes per line-search pass (after the first)
constexpr int TILE_C = 256;  // columns per tile (one per thread)
constexpr int TILE_RMAX = 64;  // maximum rows per tile
constexpr int NBIN = 6;        // CG row bins: <= 1, 2, 4, 8, 16 and more quads
constexpr int JDS_PQ = 16;     // one-block CG, jagged-diagonal storage: quads per row piece (8, 32 measured slower)
constexpr int WCG_NT = 256;        // wide CG: threads per block of a half-product (256/512/1024 measured)
constexpr int WCG_ROWS = WCG_NT / 8;  // wide CG: rows of one half of M per block
constexpr int WCG_MAX_N = 4096;  // instances with m+n above this take the wide CG
constexpr int PCG_SMALL_N = 256;  // one-block CG: instances with m+n up to this use 256-thread blocks

// Entries per thread of the one-block CG for an instance with m + n = N (the
// kernel is launched with the largest over its batch, never fewer).
__host__ __device__ constexpr int pcg_ept(int N) { return N <= 1024 ? 1 : N <= 2048 ? 2 : 4; }
// Threads of the one-block CG's block for an instance with m + n = N: 256 up
// to PCG_SMALL_N entries (four waves: cheaper barriers and reductions for the
// small instances, whose iterations are latency-bound), else 1024.  A function
// of N alone, so an instance takes the same block alone and in any batch.
__host__ __device__ constexpr int pcg_threads(int N) { return N <= PCG_SMALL_N ? 256 : 1024; }
// Size of the one-block CG's LDS array of products / piece sums for EPT
// entries per thread (at least 1024 EPT; what the LDS leaves for EPT = 4).
__host__ __device__ constexpr int pcg_parts(int ept) { return ept <= 2 ? 2048 * ept : 6144; }
constexpr int WCG_VROWS = 1024;  // wide CG: rows per block of the vector steps

enum Phase : int { PH_DONE = 0, PH_WARM = 1, PH_NEWTON = 2, PH_FALLBACK = 3 };
// LS_APPLIED: the full step accepted by the fused first trial and already applied
enum LsState : int { LS_PENDING = 0, LS_ACCEPTED = 1, LS_FAILED = 2, LS_APPLIED = 3 };
enum SrcKind : int { SRC_DENSE = 0, SRC_GRID = 1 };

// Per-instance descriptor (device memory, read-only in kernels).
struct DevInst {
    int m, n;
    int grid_s;   // SRC_GRID: side of the grid (m = n = s*s)
    int R;        // rows per tile of the tile kernels (<= TILE_RMAX)
    int nrb, ncb; // row blocks (ceil(m/R)), column blocks (ceil(n/TILE_C))
    int nnz_cap;  // capacity of the CSR/CSC arrays
    int cgfmt;    // CG of this instance: bit 0 set = the wide CG (m + n > WCG_MAX_N), else the
                  // one-block CG; bit 1 set = uint16 indices in S and S^T (wide CG with m, n <= 65536),
                  // else int32 byte offsets.  A function of (m, n) only, so an instance takes the
                  // same CG and storage alone and in any batch
    long ldc;                 // leading dimension of csrc / cbase
    const double* csrc;       // exponent cost source: C (implicit) or C^k (materialised)
    double cscale;            // scale applied to csrc entries
    const double* cbase;      // unshifted cost for the outputs (dense kinds)
    double bscale;            // its scale
    const double* a;
    const double* b;
    double* loga;
    double* logb;
    double* F;
    double* G;
    double* Ah;  // Ahat
    double* Bh;  // Bhat
    double* rc;  // r = Xt e (m) followed by c = Xt^T e (n)
    double* d;   // Newton direction (m+n)
    double* cgw; // CG work: res, z, p, Ap (4*(m+n))
    double* part;   // column partials of tile kernels: nrb * n * 2
    double* part2;  // row partials of tile kernels: ncb * m * LS_T
    double* blk;    // per-block scalars: >= max blocks * LS_T
    double* blk2;   // second per-block scalar area (merge kernels)
    int* hist;      // NLEV Sparsify histogram (entries per highest kept level)
    int* cntr;      // m * ncb kept entries per (row, column block) at the chosen level,
                    // turned by the scan into exclusive prefix sums over the column blocks
    int* cntc;      // nrb * n the same per (row block, column), prefix sums over the row blocks
    // S (CSR) and S^T (CSC).  Every row of S and of S^T starts at a multiple
    // of 4 entries and is padded to one with (index 0, value 0), so the CG
    // reads them in aligned quads; within a row of nq quads the quads are
    // stored transposed (component u of quad q holds the row's entry u*nq + q).
    // nnz_cap (a multiple of 4) includes the padding.
    // Index arrays hold uint16 or int32 per instance (cgfmt bit 1); value arrays
    // hold float in the fast-mixed precision, else double (the buffers are sized
    // for int32/double).
    int* rowptr;    // m+1
    void* col;      // nnz_cap column indices of S
    void* val;      // nnz_cap values of S
    int* colptr;    // n+1
    void* rowT;     // nnz_cap row indices of S^T
    void* valT;     // nnz_cap values of S^T
    int* rowbin;    // m+n rows of M = [. S; S^T .]: rows of S by quad count (NBIN bins), then rows of S^T;
                    // with Ctrl::jds, per row k the positions of its pieces instead (jds_info)
    double* Ck;     // materialised shifted cost (m*n) or nullptr
    double* alpha;  // outputs
    double* beta;
    double* X;      // optional dense plan
};

// Per-instance control block (device memory; the host reads it back).
struct Ctrl {
    int phase, t, ticket, ls_state;
    int level, nnz, ls_h, flags;
    int sink_total, newton_total, cg_total, fb_total;
    int last_cg, fused, nonfinite, grad_ready;  // fused: the Armijo pass also produced the next gradient
    double kappa, err, resid, alpha;
    double gd, dab, fa, cost;
    double entropy, dual, scale, pad2;
    double work[9];  // matrix entries visited per pass kind (W_* below); W_CG*: stored entries read by CG
    int binoff[16];  // rowbin offsets: NBIN bins of rows of S, then NBIN bins of rows of S^T; [2 NBIN] = m+n
    int cg_it, cg_on;        // wide CG (many blocks per instance): iterations, still iterating
    int decided;             // 1: the next round's gradient already merged and decided (after the fused trial)
    int margbad;             // set up: bit 0 a has an entry <= 0 or non-finite, bit 1 |sum a - 1| > 1e-10,
                             // bits 2, 3 the same for b
    double cg_rzs[2], cg_bnorm;  // wide CG: <res, z> of iteration t in cg_rzs[t & 1]; ||rhs||
    // outer loop of this instance: the current subproblem k_out (advanced by the
    // shift), the number K_out of outer iterations, and the marginal tolerances
    // of the subproblems before the last (tol_in) and of the last (tol_fin)
    int k_out, K_out;
    double tol_in, tol_fin;
    // one-block CG storage of S and S^T chosen at the last Sparsify: jds = 1 for
    // the jagged-diagonal form (rows cut into pieces of at most JDS_PQ quads,
    // pieces of one half ordered by length, longest first; quad q of the piece
    // at position v is quad jdp[h][q] + v of the half's arrays), else 0 for the
    // row-contiguous form with the binned row list
    int jds;
    int jdp[2][JDS_PQ + 1];
};

// pass kinds counted in Ctrl::work
// (W_CG: one-block CG over jagged-diagonal S, W_CG_ROWS: over row-contiguous S)
enum WorkKind : int {
    W_ROW = 0, W_COL = 1, W_GRAD = 2, W_FILL = 3, W_CG = 4, W_LS = 5, W_FINAL = 6, W_CG_WIDE = 7, W_CG_ROWS = 8
};

// Kernel-wide parameters (passed by value).
struct KP {
    double eta, inv_eta;
    double warm_tol;
    double inner_tol, final_tol;  // marginal tolerances (copied into each instance's Ctrl at set-up)
    double cg_rtol, ls_beta, ls_c1, log_rho;
    double budget;
    int T1, T2, cg_max, ls_max;
    int nlev, shift_mode, K, count;  // K: outer iterations; count: instances in the batch
    // flat grids over uneven batches: toff / roff hold count + 1 prefix sums of
    // the per-instance tile counts (nrb * ncb) and row-block counts (ceil(m/4))
    const int* toff;
    const int* roff;
};

}  // namespace pins
