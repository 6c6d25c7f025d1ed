// Allocation-free apply of the M-term operator (2.13) on a 1D grid, for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops that forbid allocation). Everything the apply needs beyond
// the caller's input and output (the grid mean of s, delta = s - s0, the
// symbol table |mu_k|^2 and the twiddle tables) is formed on the device in
// one file-scope array, `scratch`, of NOALLOC_SCRATCH_BYTES; the transforms
// then run in the same single-workgroup kernel as vofl_apply's 1D path.
// Each GPU holds its own copy of the array until the process ends; calls
// that overlap on one GPU race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.hpp"
#include "vofl.h"

namespace vofl {
int api_fail(int code, const char* msg);  // vofl_plan.cpp: sets vofl_last_error
}

namespace {

using vofl::cpx;

constexpr size_t NOALLOC_SCRATCH_BYTES = 256 * 1024;
constexpr int NOALLOC_MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_mtx;
unsigned char* g_scratch[NOALLOC_MAX_DEVICES] = {};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// byte offsets of the tables inside the scratch array
struct Layout {
    size_t sc, delta, mu2, tw64, tw, total;
};
Layout layout(int n, size_t cpx_bytes) {
    Layout l{};
    l.sc = 0;
    l.delta = align256(sizeof(vofl::SolveScalars));
    l.mu2 = l.delta + align256((size_t)n * 8);
    l.tw64 = l.mu2 + align256((size_t)n * 8);
    l.tw = l.tw64 + align256((size_t)n * 16);
    l.total = l.tw + align256((size_t)n * cpx_bytes);
    return l;
}

// One workgroup: s0 = grid mean of s (fixed summation order), delta,
// |mu_k|^2 (bin j holds k = j for j < n/2, j - n otherwise, mu = 2 pi k/L),
// twiddles exp(-2 pi i j/n) in FP64 and in T, and the scalars.
template <typename T>
__global__ __launch_bounds__(256) void k_noalloc_prep(const double* __restrict__ s, int n, double L,
                                                      unsigned char* base, Layout l) {
    __shared__ double part[256];
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) acc += s[j];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    const double mean = part[0] / double(n);
    double* delta = reinterpret_cast<double*>(base + l.delta);
    double* mu2 = reinterpret_cast<double*>(base + l.mu2);
    cpx<double>* tw64 = reinterpret_cast<cpx<double>*>(base + l.tw64);
    cpx<T>* tw = reinterpret_cast<cpx<T>*>(base + l.tw);
    for (int j = threadIdx.x; j < n; j += 256) {
        delta[j] = s[j] - mean;
        const int k = (j < n / 2) ? j : j - n;
        const double mu = 2.0 * M_PI * double(k) / L;
        mu2[j] = mu * mu;
        double sn, cs;
        sincospi(2.0 * double(j) / double(n), &sn, &cs);
        tw64[j] = {cs, -sn};
        tw[j] = {T(cs), T(-sn)};
    }
    if (threadIdx.x == 0) {
        vofl::SolveScalars sc{};
        sc.sig1 = mean;
        sc.sig2 = mean;
        *reinterpret_cast<vofl::SolveScalars*>(base + l.sc) = sc;
    }
}

// Address of this device's scratch array (looked up once per device, with
// the device current): in host code the array's name is not a device address.
unsigned char* device_scratch(int& rc) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        rc = vofl::api_fail(VOFL_ERR_DEVICE, "no current HIP device");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mtx);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            rc = vofl::api_fail(VOFL_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed");
            return nullptr;
        }
        g_scratch[dev] = static_cast<unsigned char*>(ptr);
    }
    return g_scratch[dev];
}

template <typename T>
int apply_noalloc(int n, double lo, double hi, const double* s, int M, const void* u, void* out, int nfields,
                  hipStream_t st) {
    const Layout l = layout(n, sizeof(cpx<T>));
    if (l.total > NOALLOC_SCRATCH_BYTES)
        return vofl::api_fail(VOFL_ERR_INVALID, "grid too large for the allocation-free apply's scratch");
    int rc = VOFL_OK;
    unsigned char* base = device_scratch(rc);
    if (!base) return rc;
    k_noalloc_prep<T><<<dim3(1), dim3(256), 0, st>>>(s, n, hi - lo, base, l);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return vofl::api_fail(VOFL_ERR_DEVICE, "prep launch failed");
    vofl::Args1D<T> a{};
    a.u_in = static_cast<const T*>(u);
    a.u_out = static_cast<T*>(out);
    a.N = n;
    a.mu2 = reinterpret_cast<const double*>(base + l.mu2);
    a.tw = reinterpret_cast<const cpx<T>*>(base + l.tw);
    a.tw64 = reinterpret_cast<const cpx<double>*>(base + l.tw64);
    a.delta = reinterpret_cast<const double*>(base + l.delta);
    a.coef_stride = 0;
    a.sc = reinterpret_cast<const vofl::SolveScalars*>(base + l.sc);
    a.sc_stride = 0;
    a.M = M;
    a.op = VOFL_OP_S1;
    a.invN = 1.0 / double(n);
    a.sub = 1;
    e = vofl::Launch<T>::d1_apply(n, a, nfields, st);
    if (e != hipSuccess) return vofl::api_fail(VOFL_ERR_DEVICE, "apply launch failed");
    return VOFL_OK;
}

}  // namespace

extern "C" int vofl_apply_noalloc(int n, double lo, double hi, const double* s, int M, int precision,
                                  const void* u, void* out, int nfields, void* stream) {
    if (!s || !u || !out) return vofl::api_fail(VOFL_ERR_INVALID, "s, u and out must be device pointers");
    if (u == out) return vofl::api_fail(VOFL_ERR_INVALID, "out must not alias u");
    if (n < 2 || n % 2) return vofl::api_fail(VOFL_ERR_INVALID, "n must be even and >= 2");
    if (!(hi > lo)) return vofl::api_fail(VOFL_ERR_INVALID, "the box must satisfy lo < hi");
    if (M < 0 || M > 64) return vofl::api_fail(VOFL_ERR_INVALID, "M must be in [0, 64]");
    if (nfields < 1 || nfields > 65535) return vofl::api_fail(VOFL_ERR_INVALID, "nfields must be in [1, 65535]");
    if (precision != VOFL_FP64 && precision != VOFL_FP32)
        return vofl::api_fail(VOFL_ERR_INVALID, "precision must be VOFL_FP64 or VOFL_FP32");
    const bool fp32 = precision == VOFL_FP32;
    if (!(fp32 ? vofl::Launch<float>::supported_1d(n) : vofl::Launch<double>::supported_1d(n)))
        return vofl::api_fail(VOFL_ERR_UNSUPPORTED, "no compiled 1D transform of this length");
    hipStream_t st = static_cast<hipStream_t>(stream);
    return fp32 ? apply_noalloc<float>(n, lo, hi, s, M, u, out, nfields, st)
                : apply_noalloc<double>(n, lo, hi, s, M, u, out, nfields, st);
}
