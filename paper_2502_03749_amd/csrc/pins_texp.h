// pins_texp.h -- exp(x) in double by Tang's table-driven method (P. T. P.
// Tang, "Table-driven implementation of the exponential function in IEEE
// floating-point arithmetic", ACM TOMS 15(2), 1989), used by the FP64 dense
// passes of the hot path.  Host and device share this code, so that the CPU
// test of the method (tests/test_texp_cpu.py) runs exactly what the kernels run.
//
// x = (64 k + j) ln2/64 + r with |r| <= ln2/128 (ln2/64 split into a leading
// part exact in 43 bits and a trailing part), so that
//     exp(x) = 2^k 2^(j/64) (1 + q),  q = e^r - 1,
// q from its degree-5 Taylor polynomial (truncation below 4e-17 relative),
// 2^(j/64) from a 64-entry table.  About 1 ulp; x < -746 gives 0, x > 710
// gives inf (through the final scaling), NaN stays NaN.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace pins {

// entry j (0..63) of the table: 2^(j/64)
__host__ __device__ inline double texp_table_entry(int j) { return exp2((double)j * (1.0 / 64.0)); }

__host__ __device__ inline double texp_eval(double x, const double* T) {
    x = (x < -746.0) ? -746.0 : x;
    x = (x > 710.0) ? 710.0 : x;
    const double nd = rint(x * 92.33248261689366);  // 64 / ln 2
    const int nk = (x != x) ? 0 : (int)nd;         // NaN: any table entry (the result is NaN)
    double r = fma(-nd, 0x1.62e42fefa39efp-7, x);   // ln 2 / 64, leading part
    r = fma(-nd, 0x1.abc9e3b39803fp-62, r);         // ln 2 / 64, trailing part
    double q = fma(r, 1.0 / 120.0, 1.0 / 24.0);
    q = fma(q, r, 1.0 / 6.0);
    q = fma(q, r, 0.5);
    q = fma(q, r, 1.0);
    q *= r;
    const double tj = T[nk & 63];
    return ldexp(fma(tj, q, tj), nk >> 6);
}

// The same for arguments x <= 0 or -inf (the log-sum-exp sweeps' exp(z - max)):
// one maximum replaces the clamps and the NaN guard (a NaN argument is not
// expected here and gives 0).  Bitwise the value of texp_eval for x <= 0.
__host__ __device__ inline double texp_eval_nonpos(double x, const double* T) {
    x = fmax(x, -746.0);
    const double nd = rint(x * 92.33248261689366);  // 64 / ln 2
    const int nk = (int)nd;
    double r = fma(-nd, 0x1.62e42fefa39efp-7, x);   // ln 2 / 64, leading part
    r = fma(-nd, 0x1.abc9e3b39803fp-62, r);         // ln 2 / 64, trailing part
    double q = fma(r, 1.0 / 120.0, 1.0 / 24.0);
    q = fma(q, r, 1.0 / 6.0);
    q = fma(q, r, 0.5);
    q = fma(q, r, 1.0);
    q *= r;
    const double tj = T[nk & 63];
    return ldexp(fma(tj, q, tj), nk >> 6);
}

}  // namespace pins
