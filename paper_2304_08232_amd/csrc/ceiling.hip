// Device ceilings for the benchmark's measurement (not part of the solver):
// the read bandwidth a plain streaming kernel reaches on this part, the
// practical ceiling against which the HBM-bound passes are compared.
//
// k_stream_read: every thread reads 16-byte words with non-temporal loads in
// a grid-stride loop, UNROLL independent loads in flight per thread, and
// folds them into a sum that one thread per workgroup stores (so the loads
// cannot be dropped).  Built as its own small library (libceiling.so).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 8;
typedef double v2d __attribute__((ext_vector_type(2)));  // one 16-byte word

__global__ __launch_bounds__(kThreads) void k_stream_read(const v2d *__restrict__ a, int64_t n2,
                                                          double *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double acc = 0.0;
    for (; i + (kUnroll - 1) * stride < n2; i += kUnroll * stride) {
        v2d v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(a + i + u * stride);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += v[u].x + v[u].y;
    }
    for (; i < n2; i += stride) {
        const v2d v = __builtin_nontemporal_load(a + i);
        acc += v.x + v.y;
    }
    __shared__ double sh[kThreads];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

}  // namespace

extern "C" {

// Reads n2 16-byte words from a (DEVICE, 16-byte aligned) once with `blocks`
// workgroups of 256 threads on `stream`; out (DEVICE) receives one double per
// workgroup.  Returns a hipError_t value (0 on success).
int ceiling_stream_read(const void *a, int64_t n2, double *out, int blocks, hipStream_t stream) {
    if (!a || !out || n2 < 0 || blocks < 1) return (int)hipErrorInvalidValue;
    if (((uintptr_t)a) % 16 != 0) return (int)hipErrorInvalidValue;
    k_stream_read<<<blocks, kThreads, 0, stream>>>((const v2d *)a, n2, out);
    return (int)hipGetLastError();
}

}  // extern "C"
