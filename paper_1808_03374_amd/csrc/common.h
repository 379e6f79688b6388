// Internal helpers shared by the gfx950 kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/gkl.h"

namespace gkl {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxKrylov = 96;     // largest projected matrix the in-LDS SVD handles
constexpr int kMaxBlockedKrylov = 128;  // largest projected matrix whose SVD runs in LDS with logged rotations

// ---------------------------------------------------------------------------
// Error plumbing: internal code throws gkl::Error, the ABI layer converts it.
// ---------------------------------------------------------------------------
struct Error {
    gkl_status status;
    std::string msg;
};

[[noreturn]] void fail(gkl_status s, const std::string& msg);
void check_hip(hipError_t e, const char* what);

#define GKL_HIP(call) ::gkl::check_hip((call), #call)
#define GKL_LAUNCH_CHECK(what) ::gkl::check_hip(hipGetLastError(), what)

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
    // butterfly over the 64 lanes; every lane ends with the same total and the
    // order of additions is fixed, so results are deterministic
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum of one double per thread over a block of blockDim.x threads (multiple of
// 64, at most 1024).  Result valid in every thread.  scratch: >= 16 doubles.
__device__ __forceinline__ double block_sum(double v, double* scratch)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += scratch[w];
    return t;
}

// Sum of x[q * stride] for q = 0 .. count - 1, added in increasing q exactly as
// a plain loop would (same result bit for bit), with the loads issued eight at
// a time: indices past count re-read element count - 1 and are not added.
// With kPair each term is x[q * stride] + x[q * stride + pair_off].
template <bool kPair = false>
__device__ __forceinline__ double strided_sum(const double* __restrict__ x, int64_t stride,
                                              int count, int64_t pair_off = 0)
{
    double s = 0.0;
    for (int b = 0; b < count; b += 8) {
        double v[8], w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t q = b + u < count ? b + u : count - 1;
            v[u] = x[q * stride];
            if (kPair) w[u] = x[q * stride + pair_off];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (b + u < count) s += kPair ? v[u] + w[u] : v[u];
    }
    return s;
}

// "Last block reduces" handshake for two-stage deterministic reductions: each
// block writes its partials, then calls this; exactly one block (the last to
// arrive) gets true and may read every block's partials.  The counter is
// reset by that block so the kernel can be replayed.
__device__ __forceinline__ bool last_block_arrived(unsigned int* counter, unsigned int nblocks)
{
    __shared__ bool is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int prev = atomicAdd(counter, 1u);
        is_last = (prev == nblocks - 1);
    }
    __syncthreads();
    if (is_last) {
        __threadfence();
        if (threadIdx.x == 0) atomicExch(counter, 0u);
    }
    return is_last;
}

inline unsigned int ceil_div(int64_t a, int64_t b) { return (unsigned int)((a + b - 1) / b); }

// Workgroups for a grid-stride loop over `total` items with `block` threads per
// workgroup.  A HIP launch counts its work-items in 32 bits (workgroups times
// workgroup size), so any kernel whose item count can exceed that loops instead
// of launching one thread per item.
inline unsigned int stride_grid(int64_t total, int block)
{
    const int64_t g = (total + block - 1) / block;
    const int64_t cap = (int64_t)1 << 20;
    return (unsigned int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace gkl
