// Definitions of the launchers, included once per precision.
#pragma once

#include "launch.hpp"

namespace vofl {

#define VOFL_MULTI_SIZES(X) X(8) X(16) X(32) X(48) X(64) X(96) X(128) X(256) X(512) X(768) X(1000) X(1024)
#define VOFL_1D_SIZES(X) \
    X(8) X(16) X(32) X(48) X(64) X(96) X(128) X(256) X(512) X(768) X(1000) X(1024) X(2048) X(4096)

template <typename T>
bool Launch<T>::supported_multi(int N) {
    switch (N) {
#define C_(n) case n:
        VOFL_MULTI_SIZES(C_)
#undef C_
        return true;
        default: return false;
    }
}

template <typename T>
bool Launch<T>::supported_1d(int N) {
    switch (N) {
#define C_(n) case n:
        VOFL_1D_SIZES(C_)
#undef C_
        return true;
        default: return false;
    }
}

template <typename T>
int Launch<T>::tile_w(int N) {
    switch (N) {
#define C_(n) case n: return tile_width<T, n>();
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return 0;
    }
}

template <typename T>
int Launch<T>::r2c0_w(int N) {
    switch (N) {
#define C_(n) case n: return tile_width<double, n>();
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return 0;
    }
}

template <typename T>
int Launch<T>::c2r_w(int N) {
    switch (N) {
#define C_(n) case n: return c2r_width<T, n>();
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return 0;
    }
}

// Term slots a step's last-axis launch writes: above the 256 MB last-level
// cache they are stored with the non-temporal policy, except in 3D FP64
// plans, where the default policy measured faster (256^3 step 3.73 -> 3.67
// ms: the axis-0 pass reads some slot lines from the last-level cache);
// 3D FP32 (2.05 -> 2.07 ms) and 2D FP64 (1024^2: 0.218 -> 0.250 ms) were
// slower without the non-temporal stores.
template <typename T, typename TI>
bool contig_streams(const ContigArgs<T, TI>& a, int items) {
    if (a.emit_kind != EMIT_STEP || (sizeof(T) == 8 && a.n1 > 1)) return false;
    return 2LL * (a.M + 1) * a.H * (long long)sizeof(cpx<T>) * items > (256LL << 20);
}

// Pointers every k_contig launch dereferences whatever its kind (the
// twiddle tables are staged into LDS at the start, the symbol tables and the
// scalars are read per element), and those its input and output kinds need.
template <typename T, typename TI>
bool contig_args_ok(const ContigArgs<T, TI>& a) {
    if (!a.tw || !a.tw_in || !a.mu2_0 || !a.mu2_l || !a.sc) return false;
    if ((a.in_kind == IN_INIT || a.in_kind == IN_KICK || a.in_kind == IN_APPLY) && !a.in) return false;
    if (a.in_kind != IN_APPLY && (!a.U || !a.V)) return false;
    if (a.emit_kind != EMIT_NONE && !a.out) return false;
    return true;
}

template <typename T, typename TI, int n, int E>
hipError_t contig_launch(const ContigArgs<T, TI>& a, int items, hipStream_t s) {
    constexpr int P = p_contig_e(n, E);
    if (a.rs < (long long)a.n1 * n) return hipErrorInvalidValue;  // rows hold n1 pencils
    dim3 grid((a.npencils + P - 1) / P, items);
    if (contig_streams(a, items)) k_contig<T, TI, n, E, P, true><<<grid, dim3(P * (n / E)), 0, s>>>(a);
    else k_contig<T, TI, n, E, P><<<grid, dim3(P * (n / E)), 0, s>>>(a);
    return hipGetLastError();
}

template <typename T>
template <typename TI>
hipError_t Launch<T>::contig(int N, const ContigArgs<T, TI>& a, int items, hipStream_t s, int variant) {
    if (!contig_args_ok(a)) return hipErrorInvalidValue;
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        if constexpr (e_contig_alt(n) != e_contig(n))                                   \
            if (variant == 1) return contig_launch<T, TI, n, e_contig_alt(n)>(a, items, s); \
        return contig_launch<T, TI, n, e_contig(n)>(a, items, s);                       \
    }
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
bool Launch<T>::contig_variant_exists(int N, int variant) {
    switch (N) {
#define C_(n)                                                                           \
    case n: return variant == 0 || (variant == 1 && e_contig_alt(n) != e_contig(n));
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return false;
    }
}

// One middle-axis launch of tile width W; nt: the launch moves more than
// the 256 MB last-level cache holds, so slots are loaded and stored with the
// non-temporal policy.
template <typename T, int n, int E, int W>
void mid_launch(int dir, bool nt, dim3 grid, const MidArgs<T>& a, hipStream_t s) {
    const dim3 block(W * (n / E));
    if (nt) {
        if (dir < 0) k_mid<T, n, E, W, -1, true><<<grid, block, 0, s>>>(a);
        else k_mid<T, n, E, W, +1, true><<<grid, block, 0, s>>>(a);
    } else {
        if (dir < 0) k_mid<T, n, E, W, -1><<<grid, block, 0, s>>>(a);
        else k_mid<T, n, E, W, +1><<<grid, block, 0, s>>>(a);
    }
}

// variants: 0 -> W = tile_width columns; 1 -> 2W columns when the FFT
// buffer stays within 66 KB of LDS
template <typename T>
hipError_t Launch<T>::mid(int N, int dir, const MidArgs<T>& a, int planes, int items,
                          hipStream_t s, int variant) {
    if (a.rs < (long long)N * a.n2) return hipErrorInvalidValue;  // a plane holds N rows of n2
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        constexpr int E = e_mid(n), W = tile_width<T, n>();                             \
        constexpr int W2 = (2 * W * n * int(sizeof(cpx<T>)) <= 67584) ? 2 * W : W;      \
        constexpr int W4 = (4 * W * n * int(sizeof(cpx<T>)) <= 135168 &&               \
                            4 * W * (n / E) <= 1024) ? 4 * W : W2;                      \
        const int w = (variant == 2) ? W4 : (variant == 1) ? W2 : W;                   \
        dim3 grid(planes * ((a.n2 + w - 1) / w), items * a.nf);                         \
        const bool nt = (long long)planes * n * a.n2 * items * a.nf * (long long)sizeof(cpx<T>) > \
                        (256LL << 20);                                                  \
        if (variant == 2 && W4 != W2) mid_launch<T, n, E, W4>(dir, nt, grid, a, s);     \
        else if ((variant == 1 || variant == 2) && W2 != W) mid_launch<T, n, E, W2>(dir, nt, grid, a, s); \
        else mid_launch<T, n, E, W>(dir, nt, grid, a, s);                               \
        return hipGetLastError();                                                       \
    }
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
int Launch<T>::mid_tile(int N, int variant) {
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        constexpr int W = tile_width<T, n>(), E = e_mid(n);                             \
        constexpr int W2 = (2 * W * n * int(sizeof(cpx<T>)) <= 67584) ? 2 * W : W;      \
        constexpr int W4 = (4 * W * n * int(sizeof(cpx<T>)) <= 135168 &&               \
                            4 * W * (n / E) <= 1024) ? 4 * W : W2;                      \
        return variant == 2 ? W4 : variant == 1 ? W2 : W;                               \
    }
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return 0;
    }
}

template <typename T>
hipError_t Launch<T>::r2c0(int N, const R2CArgs<T>& a, int items, hipStream_t s) {
    if (a.rs < a.inner) return hipErrorInvalidValue;
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        constexpr int E = e_r2c0(n), W = tile_width<double, n>();                       \
        dim3 grid((a.inner + W - 1) / W, items);                                        \
        k_r2c0<T, n, E, W><<<grid, dim3(W * (n / E)), 0, s>>>(a);                       \
        return hipGetLastError();                                                       \
    }
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return hipErrorInvalidValue;
    }
}

// the paired layout puts positions t and TP - t W lanes apart in a wavefront
template <int n, int E, int W>
constexpr bool paired_ok() {
    return E % 2 == 0 && n / E >= 2 && W <= 32 && (64 / W) % 2 == 0 && ((n / E) * W) % 64 == 0;
}

template <typename T, int n, int E, int W, int WPE, int PD = 1, bool PAIRED = false, bool STAGED = false,
          bool NT = false>
hipError_t c2r0_mode(const C2RArgs<T>& a, int items, hipStream_t s) {
    const dim3 block(W * (n / E));
    const dim3 grid((a.inner + W - 1) / W, items);
    switch (a.mode) {
        case C2R_APPLY: k_c2r0<T, n, E, W, C2R_APPLY, WPE, PD, PAIRED, STAGED, NT><<<grid, block, 0, s>>>(a); break;
        case C2R_KICK: k_c2r0<T, n, E, W, C2R_KICK, WPE, PD, PAIRED, STAGED, NT><<<grid, block, 0, s>>>(a); break;
        case C2R_EXPORT: k_c2r0<T, n, E, W, C2R_EXPORT, WPE, 1, PAIRED, STAGED, NT><<<grid, block, 0, s>>>(a); break;
        case C2R_KICK_GENERIC:
            k_c2r0<T, n, E, W, C2R_KICK_GENERIC, WPE, PD, PAIRED, STAGED, NT><<<grid, block, 0, s>>>(a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Bytes of term slots one k_c2r0 launch reads: above the 256 MB last-level
// cache the paired default streams them with the non-temporal policy (only
// on tiles whose rows fill a 128-byte line: a half line loaded
// non-temporally is fetched again for the neighbouring tile).
template <typename T>
bool c2r0_streams(const C2RArgs<T>& a, int items) {
    const long long slots = a.mode == C2R_EXPORT ? 2 : a.mode == C2R_APPLY ? a.M + 1
                          : a.mode == C2R_KICK ? 2LL * (a.M + 1) : a.M + 2;
    return slots * a.H * (long long)sizeof(cpx<T>) * items > (256LL << 20);
}

template <typename T, int n, int E, int NW>
hipError_t c2r0w_mode(const C2RArgs<T>& a, int items, hipStream_t s) {
    using G = C2RW<T, n, E, NW>;
    const dim3 grid((a.inner + G::W - 1) / G::W, items);
    switch (a.mode) {
        case C2R_APPLY: k_c2r0w<T, n, E, NW, C2R_APPLY><<<grid, dim3(G::NT), 0, s>>>(a); break;
        case C2R_KICK: k_c2r0w<T, n, E, NW, C2R_KICK><<<grid, dim3(G::NT), 0, s>>>(a); break;
        case C2R_KICK_GENERIC: k_c2r0w<T, n, E, NW, C2R_KICK_GENERIC><<<grid, dim3(G::NT), 0, s>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// variants of the axis-0 kernel: 0 -> k_c2r0 (W columns, direct register
// loads of rows min(k, N-k)); 2 -> k_c2r0 with W/2 columns; 11, 12 ->
// k_c2r0 loading each stored row once (paired layout), with 1 and 2 slot
// pairs in flight; 13 -> paired layout with W/2 columns; 14 -> k_c2r0
// staging each stored row once through LDS; 5 -> k_c2r0w (wave-local
// transforms, E = 8, 4 waves);
// 6 -> k_c2r0w with 8 waves. A variant that does not exist for a length
// (see c2r_variant_exists) falls back to variant 0; variants 5 and 6 also
// fall back to 0 in the export mode.
template <typename T>
hipError_t Launch<T>::c2r0(int N, const C2RArgs<T>& a, int items, hipStream_t s, int variant) {
    if (a.rs < a.inner) return hipErrorInvalidValue;
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        constexpr int W = c2r_width<T, n>(), E = e_c2r0(n);                             \
        constexpr int W2 = (W >= 8) ? W / 2 : W;                                        \
        if (variant == 2 && W2 != W) return c2r0_mode<T, n, E, W2, 1>(a, items, s);     \
        if constexpr (E % 2 == 0)                                                       \
            if (variant == 14) return c2r0_mode<T, n, E, W, 1, 1, false, true>(a, items, s); \
        if constexpr (paired_ok<n, E, W2>() && W2 != W)                                  \
            if (variant == 13)                                                          \
                return (c2r0_streams(a, items) && W2 * int(sizeof(cpx<T>)) >= 128)        \
                           ? c2r0_mode<T, n, E, W2, 1, 1, true, false, true>(a, items, s) \
                           : c2r0_mode<T, n, E, W2, 1, 1, true>(a, items, s);            \
        if constexpr (paired_ok<n, E, W>()) {                                           \
            if (variant == 11)                                                          \
                return c2r0_streams(a, items) ? c2r0_mode<T, n, E, W, 1, 1, true, false, true>(a, items, s) \
                                              : c2r0_mode<T, n, E, W, 1, 1, true>(a, items, s); \
            if constexpr (sizeof(T) == 4 && E <= 8)                                       \
                if (variant == 12) return c2r0_mode<T, n, E, W, 1, 2, true>(a, items, s); \
        }                                                                               \
        if constexpr (C2RW<T, n, 8, 4>::ok && sizeof(T) == 4)                           \
            if (variant == 5 && a.mode != C2R_EXPORT) return c2r0w_mode<T, n, 8, 4>(a, items, s); \
        if constexpr (C2RW<T, n, 8, 8>::ok && sizeof(T) == 4)                           \
            if (variant == 6 && a.mode != C2R_EXPORT) return c2r0w_mode<T, n, 8, 8>(a, items, s); \
        return c2r0_mode<T, n, E, W, 1>(a, items, s);                                   \
    }
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
bool Launch<T>::c2r_variant_exists(int N, int variant) {
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        constexpr int W = c2r_width<T, n>(), E = e_c2r0(n);                             \
        if (variant == 0) return true;                                                  \
        if (variant == 2) return W >= 8;                                                \
        if (variant == 11) return paired_ok<n, E, W>();                                 \
        if (variant == 12) return paired_ok<n, E, W>() && sizeof(T) == 4 && E <= 8;     \
        if (variant == 13) return W >= 8 && paired_ok<n, E, (W >= 8 ? W / 2 : W)>();    \
        if (variant == 14) return E % 2 == 0;                                           \
        if (variant == 5) return C2RW<T, n, 8, 4>::ok && sizeof(T) == 4;                \
        if (variant == 6) return C2RW<T, n, 8, 8>::ok && sizeof(T) == 4;                \
        return false;                                                                   \
    }
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return false;
    }
}

// Default axis-0 variant: each stored row loaded once. Columns of 768 points
// and more stage their rows through LDS (14: measured faster there, e.g. the
// 1024^2 FP64 kick 0.116 -> 0.105 ms, where the tiles are 4 columns wide);
// shorter ones use the paired layout on the narrowest tile whose rows still
// fill a 128-byte line (13: half-width tiles, the FP64 case; 11: full
// width), else the LDS-staged loads (14), else direct loads (0). Narrower
// tiles give more workgroups per CU at the same register count; rows shorter
// than a line would be fetched twice.
template <typename T>
int Launch<T>::c2r_default(int N) {
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        constexpr int W = c2r_width<T, n>(), E = e_c2r0(n);                             \
        constexpr int W2 = (W >= 8) ? W / 2 : W;                                        \
        if (n >= 768 && E % 2 == 0) return 14;                                          \
        if (W2 != W && paired_ok<n, E, W2>() && W2 * int(sizeof(cpx<T>)) >= 128) return 13; \
        if (paired_ok<n, E, W>()) return 11;                                            \
        return (E % 2 == 0) ? 14 : 0;                                                   \
    }
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return 0;
    }
}

template <typename T>
int Launch<T>::c2r_tile(int N, int variant) {
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        constexpr int W = c2r_width<T, n>();                                            \
        return ((variant == 2 || variant == 13) && W >= 8) ? W / 2 : W;                 \
    }
        VOFL_MULTI_SIZES(C_)
#undef C_
        default: return 0;
    }
}

template <typename T>
hipError_t Launch<T>::d1_apply(int N, const Args1D<T>& a, int items, hipStream_t s) {
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        constexpr int E = e_1d(n);                                                      \
        k_1d_apply<T, n, E><<<dim3(items), dim3(n / E), 0, s>>>(a);                     \
        return hipGetLastError();                                                       \
    }
        VOFL_1D_SIZES(C_)
#undef C_
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t Launch<T>::d1_step(int N, const Args1D<T>& a, int items, hipStream_t s) {
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        constexpr int E = e_1d(n);                                                      \
        k_1d_step<T, n, E><<<dim3(items), dim3(n / E), 0, s>>>(a);                      \
        return hipGetLastError();                                                       \
    }
        VOFL_1D_SIZES(C_)
#undef C_
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t Launch<T>::d1_lffp(int N, const Args1D<T>& a, int items, hipStream_t s) {
    switch (N) {
#define C_(n)                                                                           \
    case n: {                                                                           \
        constexpr int E = e_1d(n);                                                      \
        k_1d_lffp<T, n, E><<<dim3(items), dim3(n / E), 0, s>>>(a);                      \
        return hipGetLastError();                                                       \
    }
        VOFL_1D_SIZES(C_)
#undef C_
        default: return hipErrorInvalidValue;
    }
}

inline unsigned convert_blocks(long long n) {
    const long long b = (n + 255) / 256;
    return unsigned(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

template <typename T>
hipError_t Launch<T>::to_f64(const T* in, double* out, long long n, hipStream_t s) {
    k_convert<T, double><<<dim3(convert_blocks(n)), dim3(256), 0, s>>>(in, out, n);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::from_f64(const double* in, T* out, long long n, hipStream_t s) {
    k_convert<double, T><<<dim3(convert_blocks(n)), dim3(256), 0, s>>>(in, out, n);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::lincomb(T* out, const T* x0, double c0, const T* x1, double c1, const T* x2, double c2,
                              const T* xq, double cq, long long n, hipStream_t s) {
    k_lincomb<T><<<dim3(convert_blocks(n)), dim3(256), 0, s>>>(out, x0, c0, x1, c1, x2, c2, xq, cq, n);
    return hipGetLastError();
}

template <typename T>
hipError_t Launch<T>::dot2(const T* a0, const T* b0, const T* a1, const T* b1, long long n, double* partial,
                           double* out, hipStream_t s) {
    k_dot2<T><<<dim3(dot_blocks), dim3(256), 0, s>>>(a0, b0, a1, b1, n, partial);
    k_dot2_finish<T><<<dim3(1), dim3(256), 0, s>>>(partial, dot_blocks, out);
    return hipGetLastError();
}

}  // namespace vofl
