// HBM streaming probe: plain read, write and copy streams with the access
// pattern of a tuned bandwidth kernel (16 bytes per lane per access, 4 or 16
// accesses in flight per lane, a grid of several workgroups per CU striding
// over the buffer, non-temporal loads and stores on request). It computes
// nothing of the method; it measures the rates that a read stream, a write
// stream and a one-to-one copy reach on the device, so that each pass of the
// solver can be set against the stream of its own read/write mix.
#include <hip/hip_runtime.h>

#include "vofl.h"

namespace vofl {
int api_fail(int code, const char* msg);  // vofl_plan.cpp: sets vofl_last_error
}

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int PROBE_THREADS = 256;

template <bool NT>
__device__ __forceinline__ f4 ld(const f4* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void st(f4* p, f4 v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Each thread handles U vectors per trip, PROBE_THREADS apart, so a
// wavefront's accesses of one instruction are 1 KiB contiguous and a
// workgroup moves U x 4 KiB per trip (a copy reads all of it, then writes).
template <bool NT, int U>
__global__ __launch_bounds__(PROBE_THREADS) void k_read(const f4* __restrict__ src, long long nvec,
                                                        float* __restrict__ partial) {
    const long long step = (long long)gridDim.x * PROBE_THREADS * U;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    for (long long base = (long long)blockIdx.x * PROBE_THREADS * U + threadIdx.x; base < nvec;
         base += step) {
        f4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + (long long)u * PROBE_THREADS;
            v[u] = i < nvec ? ld<NT>(src + i) : f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
    // a store that depends on every load keeps the loads live; it happens
    // only for one improbable sum (dst holds one float per workgroup)
    const float tot = acc.x + acc.y + acc.z + acc.w;
    if (tot == -1.0e-37f) partial[blockIdx.x] = tot;
}

template <bool NT, int U>
__global__ __launch_bounds__(PROBE_THREADS) void k_write(f4* __restrict__ dst, long long nvec) {
    const long long step = (long long)gridDim.x * PROBE_THREADS * U;
    for (long long base = (long long)blockIdx.x * PROBE_THREADS * U + threadIdx.x; base < nvec;
         base += step) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + (long long)u * PROBE_THREADS;
            const float x = (float)(i & 1023);
            if (i < nvec) st<NT>(dst + i, f4{x, x + 1.f, x + 2.f, x + 3.f});
        }
    }
}

template <bool NT, int U>
__global__ __launch_bounds__(PROBE_THREADS) void k_copy(const f4* __restrict__ src, f4* __restrict__ dst,
                                                        long long nvec) {
    const long long step = (long long)gridDim.x * PROBE_THREADS * U;
    for (long long base = (long long)blockIdx.x * PROBE_THREADS * U + threadIdx.x; base < nvec;
         base += step) {
        f4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + (long long)u * PROBE_THREADS;
            v[u] = i < nvec ? ld<NT>(src + i) : f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + (long long)u * PROBE_THREADS;
            if (i < nvec) st<NT>(dst + i, v[u]);
        }
    }
}

template <bool NT, int U>
hipError_t launch(int kind, const f4* src, f4* dst, long long nvec, int blocks, hipStream_t s) {
    if (kind == VOFL_PROBE_READ)
        k_read<NT, U><<<blocks, PROBE_THREADS, 0, s>>>(src, nvec, reinterpret_cast<float*>(dst));
    else if (kind == VOFL_PROBE_WRITE)
        k_write<NT, U><<<blocks, PROBE_THREADS, 0, s>>>(dst, nvec);
    else
        k_copy<NT, U><<<blocks, PROBE_THREADS, 0, s>>>(src, dst, nvec);
    return hipGetLastError();
}

}  // namespace

extern "C" int vofl_stream_probe(int kind, const void* src, void* dst, size_t bytes, int blocks, int flags,
                                 void* stream) {
    if (kind != VOFL_PROBE_READ && kind != VOFL_PROBE_WRITE && kind != VOFL_PROBE_COPY)
        return vofl::api_fail(VOFL_ERR_INVALID, "vofl_stream_probe: unknown kind");
    if (bytes == 0 || bytes % 16 != 0)
        return vofl::api_fail(VOFL_ERR_INVALID, "vofl_stream_probe: bytes must be a positive multiple of 16");
    if (flags & ~(VOFL_PROBE_NONTEMPORAL | VOFL_PROBE_DEEP))
        return vofl::api_fail(VOFL_ERR_INVALID, "vofl_stream_probe: unknown flag");
    if (blocks <= 0 || blocks > (1 << 20))
        return vofl::api_fail(VOFL_ERR_INVALID, "vofl_stream_probe: blocks must be in 1..2^20");
    if (!dst || (kind != VOFL_PROBE_WRITE && !src))
        return vofl::api_fail(VOFL_ERR_INVALID, "vofl_stream_probe: null buffer");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
        return vofl::api_fail(VOFL_ERR_INVALID, "vofl_stream_probe: buffers must be 16-byte aligned");
    const long long nvec = (long long)(bytes / 16);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const auto* sp = static_cast<const f4*>(src);
    auto* dp = static_cast<f4*>(dst);
    const bool nt = flags & VOFL_PROBE_NONTEMPORAL, deep = flags & VOFL_PROBE_DEEP;
    const hipError_t e = nt ? (deep ? launch<true, 16>(kind, sp, dp, nvec, blocks, s)
                                    : launch<true, 4>(kind, sp, dp, nvec, blocks, s))
                            : (deep ? launch<false, 16>(kind, sp, dp, nvec, blocks, s)
                                    : launch<false, 4>(kind, sp, dp, nvec, blocks, s));
    if (e != hipSuccess) return vofl::api_fail(VOFL_ERR_DEVICE, "vofl_stream_probe: launch failed");
    return VOFL_OK;
}
