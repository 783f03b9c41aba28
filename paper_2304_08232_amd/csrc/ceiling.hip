// Device ceilings and floors for the benchmark's measurement (not part of the
// solver), built as its own small library (libceiling.so):
//
// k_stream_read: the read bandwidth a plain streaming kernel reaches on this
//   part, the practical ceiling against which the HBM-bound passes are
//   compared.  Every thread reads 16-byte words with non-temporal loads in a
//   grid-stride loop, UNROLL independent loads in flight per thread, and folds
//   them into a sum that one thread per workgroup stores (so the loads cannot
//   be dropped).
// k_empty: a kernel that does nothing, for the floor one dependent launch
//   costs on a stream (eagerly or replayed from a graph).
// k_barrier: `rounds` barriers among the participating workgroups of one
//   launch (those whose index is a multiple of `stride`: stride 8 keeps them
//   on one XCD, since workgroup b is dispatched to XCD b % 8), for the cost of
//   one barrier round of the kinds a persistent multi-phase kernel could use.
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

__global__ void k_empty() {}

// Barrier kinds:
//   kFenced  - every participant's stores are released to the whole device
//              and its caches refreshed afterwards (agent-scope release and
//              acquire fences around the flag exchange): what a barrier needs
//              when ordinary loads and stores carry the data between phases;
//   kRelaxed - the flag exchange alone (agent-scope relaxed atomics, which
//              bypass the non-coherent caches): what a barrier costs when the
//              data itself travels as agent-scope atomics.
// Participant q (of P) publishes the round it reached in flags[q]; a round
// ends when every flag has reached it.  Every wait is bounded: after
// spin_limit polls the waiter raises *err and every participant stops.
enum BarrierKind { kFenced = 0, kRelaxed = 1 };

template <int KIND>
__global__ __launch_bounds__(64) void k_barrier(unsigned *flags, int stride, int rounds, int *err,
                                                long long spin_limit) {
    if (blockIdx.x % stride != 0) return;
    const int P = (gridDim.x + stride - 1) / stride, q = blockIdx.x / stride;
    for (unsigned epoch = 1; epoch <= (unsigned)rounds; ++epoch) {
        if (KIND == kFenced) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0) __hip_atomic_store(&flags[q], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        long long spins = 0;
        for (;;) {
            int mine = 1;
            for (int j = threadIdx.x; j < P; j += 64)
                mine &= __hip_atomic_load(&flags[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch;
            if (__all(mine)) break;
            // another participant's failure is looked for every 64 polls
            // only, so that the check does not slow the polling down
            if ((++spins & 63) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                return;
            if (spins > spin_limit) {
                if (threadIdx.x == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
        }
        if (KIND == kFenced) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
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

// One launch of an empty kernel of `blocks` workgroups of `threads` threads
// (1..1024) on `stream`.  Returns a hipError_t value.
int ceiling_empty(int blocks, int threads, hipStream_t stream) {
    if (blocks < 1 || threads < 1 || threads > 1024) return (int)hipErrorInvalidValue;
    k_empty<<<blocks, threads, 0, stream>>>();
    return (int)hipGetLastError();
}

// `rounds` barriers of kind `kind` (0 fenced, 1 relaxed) among the workgroups
// of a `blocks`-workgroup launch (64 threads each) whose index is a multiple
// of `stride`.  flags (DEVICE) holds one unsigned per participant and must be
// zero on entry; err (DEVICE) must be zero and is set to 1 if a wait exceeded
// spin_limit polls.  At most 1024 participants.  Returns a hipError_t value.
int ceiling_barrier(int kind, int blocks, int stride, int rounds, unsigned *flags, int *err, long long spin_limit,
                    hipStream_t stream) {
    if ((kind != kFenced && kind != kRelaxed) || blocks < 1 || stride < 1 || rounds < 1 || !flags || !err ||
        spin_limit < 1)
        return (int)hipErrorInvalidValue;
    if ((blocks + stride - 1) / stride > 1024) return (int)hipErrorInvalidValue;
    if (kind == kFenced)
        k_barrier<kFenced><<<blocks, 64, 0, stream>>>(flags, stride, rounds, err, spin_limit);
    else
        k_barrier<kRelaxed><<<blocks, 64, 0, stream>>>(flags, stride, rounds, err, spin_limit);
    return (int)hipGetLastError();
}

}  // extern "C"
