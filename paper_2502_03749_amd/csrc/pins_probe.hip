// Measurement support: the issue rate of the hardware exponential.
//
// Every entry of a streamed warm-up sweep evaluates one exponential (in mixed
// precision the float hardware one, v_exp_f32, which computes 2^x), and nothing
// but the potentials moves through memory, so the rate of that instruction
// bounds the sweep.  The probe measures it: each thread runs PROBE_CHAINS
// independent chains v <- 2^v * (-0.75), enough to hide the instruction's
// latency.  For v in [-1, 0], 2^v lies in [0.5, 1] and the product in
// [-0.75, -0.375], so every value stays in [-1, 0] and finite.  One
// multiply accompanies each exponential.
#include <hip/hip_runtime.h>

#include "pins.h"
#include "pins_texp.h"

namespace {

constexpr int PROBE_CHAINS = 8;
constexpr int PROBE_NT = 256;

__global__ __launch_bounds__(PROBE_NT) void k_probe_exp(float* __restrict__ out, int iters) {
    const int gid = blockIdx.x * PROBE_NT + threadIdx.x;
    float v[PROBE_CHAINS];
#pragma unroll
    for (int u = 0; u < PROBE_CHAINS; ++u) v[u] = -0.0009765625f * (float)((gid + 97 * u) & 1023);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < PROBE_CHAINS; ++u) v[u] = __builtin_amdgcn_exp2f(v[u]) * -0.75f;
    }
    float s = 0.0f;
#pragma unroll
    for (int u = 0; u < PROBE_CHAINS; ++u) s += v[u];
    out[gid] = s;
}

// the FP64 dense passes' exp (pins_texp.h) on the device, table in LDS as in the kernels
__global__ __launch_bounds__(256) void k_probe_texp(const double* __restrict__ x, double* __restrict__ y, int n) {
    __shared__ double T[64];
    if (threadIdx.x < 64) T[threadIdx.x] = pins::texp_table_entry((int)threadIdx.x);
    __syncthreads();
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < n) y[k] = pins::texp_eval(x[k], T);
}

}  // namespace

extern "C" int pins_probe_texp(const double* x, double* y, int n, void* stream) {
    if (!x || !y || n < 0) return PINS_EINVAL;
    if (n == 0) return PINS_OK;
    hipLaunchKernelGGL(k_probe_texp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, x, y, n);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return PINS_EDEVICE;
    return PINS_OK;
}

extern "C" int pins_probe_exp_rate(int device, int blocks, int iters, double* exps_per_s, double* ms) {
    if (!exps_per_s || blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20)) return PINS_EINVAL;
    float* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PINS_EDEVICE;
    float t = 0.0f;
    if (hipSetDevice(device) != hipSuccess) return PINS_EDEVICE;
    if (hipMalloc(&out, sizeof(float) * (size_t)blocks * PROBE_NT) != hipSuccess) return PINS_ENOMEM;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        // one short untimed launch (code load), then the timed one
        hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(PROBE_NT), 0, nullptr, out, 16);
        const bool r0 = hipEventRecord(e0, nullptr) == hipSuccess;
        hipLaunchKernelGGL(k_probe_exp, dim3(blocks), dim3(PROBE_NT), 0, nullptr, out, iters);
        const bool r1 = hipEventRecord(e1, nullptr) == hipSuccess;
        if (r0 && r1 && hipGetLastError() == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&t, e0, e1) == hipSuccess && t > 0.0f) {
            *exps_per_s = (double)blocks * PROBE_NT * (double)iters * PROBE_CHAINS / (1e-3 * (double)t);
            if (ms) *ms = t;
            rc = PINS_OK;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}
