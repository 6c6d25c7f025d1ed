// Host-side launchers: map a runtime transform length onto the compiled
// kernel instantiations (kernels_f32.hip, kernels_f64.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace vofl {

// Elements per thread of each kernel class for a transform length N (the
// last-axis kernel uses 8 at 256, with LDS layouts free of bank conflicts;
// the 4-per-thread schedule, one 64-thread pencil per wavefront, is the
// autotuner's alternative and measured no faster at 256^3). Lengths
// with a factor 3 (3 * 2^k) use 12 elements per thread (radix 4 stages and
// one radix-3 stage); lengths with a factor 5 (1000 = 2^3 5^3) use 10
// (radix-5 and radix-2 stages, 100 threads per pencil).
constexpr bool has3(int N) { return N % 3 == 0; }
constexpr bool has5(int N) { return N % 5 == 0; }
constexpr int e_contig(int N) { return has5(N) ? 10 : has3(N) ? 12 : (N < 8 ? N : (N >= 1024 ? 4 : 8)); }
constexpr int e_mid(int N) { return has5(N) ? 10 : has3(N) ? 12 : (N < 16 ? N : 16); }
constexpr int e_r2c0(int N) { return has5(N) ? 10 : has3(N) ? 12 : (N < 16 ? N : 16); }
constexpr int e_c2r0(int N) { return has5(N) ? 10 : has3(N) ? 12 : (N < 8 ? N : 8); }
// 1D: one workgroup of at most 512 threads per field
constexpr int e_1d(int N) {
    return has5(N) ? 10 : has3(N) ? (N <= 1536 ? 6 : 12) : (N < 4 ? N : (N <= 2048 ? 4 : 8));
}
// The autotuner's alternative for the last-axis pass (contig variant 1): the
// other of 4 and 8 elements per thread (radix schedules 4-4-4-4 and 8-8-4 at
// 256) for power-of-two lengths 64..1024; other lengths have none.
constexpr int e_contig_alt(int N) {
    return (has3(N) || has5(N) || N < 64 || N > 1024) ? e_contig(N) : (e_contig(N) == 4 ? 8 : 4);
}
// pencils per workgroup of k_contig: about 256 threads
constexpr int p_contig_e(int N, int E) { return (256 / (N / E)) > 0 ? (256 / (N / E)) : 1; }
constexpr int p_contig(int N) { return p_contig_e(N, e_contig(N)); }

template <typename T>
struct Launch {
    static bool supported_multi(int N);
    static bool supported_1d(int N);
    static int tile_w(int N);
    static int c2r_w(int N);
    static int c2r_tile(int N, int variant);
    static int c2r_default(int N);
    // whether an axis-0 variant has its own kernel for length N (else it falls back to 0)
    static bool c2r_variant_exists(int N, int variant);
    // variant 0: e_contig(N) elements per thread; 1: e_contig_alt(N)
    template <typename TI>
    static hipError_t contig(int N, const ContigArgs<T, TI>& a, int items, hipStream_t s, int variant = 0);
    static bool contig_variant_exists(int N, int variant);
    static hipError_t mid(int N, int dir, const MidArgs<T>& a, int planes, int items, hipStream_t s,
                          int variant = 0);
    static int mid_tile(int N, int variant);
    // forward axis-0 transform of real T data into FP64 half spectra
    static hipError_t r2c0(int N, const R2CArgs<T>& a, int items, hipStream_t s);
    static int r2c0_w(int N);
    // variant 0: W columns x 8 elements per thread; 1: W x 16 (fewer threads
    // per workgroup); 2: W/2 x 8 (W = c2r_width)
    static hipError_t c2r0(int N, const C2RArgs<T>& a, int items, hipStream_t s, int variant = 0);
    static hipError_t d1_apply(int N, const Args1D<T>& a, int items, hipStream_t s);
    static hipError_t d1_step(int N, const Args1D<T>& a, int items, hipStream_t s);
    static hipError_t d1_lffp(int N, const Args1D<T>& a, int items, hipStream_t s);
    // element-wise T <-> FP64 copies of n values
    static hipError_t to_f64(const T* in, double* out, long long n, hipStream_t s);
    static hipError_t from_f64(const double* in, T* out, long long n, hipStream_t s);
    // Crank-Nicolson vector kernels (see k_lincomb, k_dot2); dot2 leaves the
    // two sums in out[0], out[1] (device) using partial[2 * dot_blocks]
    static constexpr int dot_blocks = 512;
    static hipError_t lincomb(T* out, const T* x0, double c0, const T* x1, double c1, const T* x2, double c2,
                              const T* xq, double cq, long long n, hipStream_t s);
    static hipError_t dot2(const T* a0, const T* b0, const T* a1, const T* b1, long long n, double* partial,
                           double* out, hipStream_t s);
};

extern template struct Launch<float>;
extern template struct Launch<double>;

}  // namespace vofl
