// Device-side FFT building blocks for gfx950 (64-wide wavefronts).
//
// A length-N transform ("pencil") is spread over TP = N/E threads; thread t
// of a pencil holds the E elements t + TP*e (e = 0..E-1) in registers, both
// before and after the transform, so global loads and stores of a pencil are
// coalesced. The transform is a Stockham autosort FFT: each stage does E/R
// radix-R butterflies per thread in registers, and stages exchange data
// through LDS (one write + one read per element per exchange). Twiddles come
// from a per-axis FP64-accurate table tw[j] = exp(-2 pi i j/N) rounded to the
// working precision. DIR = -1 is the forward DFT sum_j x_j e^{-2 pi i jk/N},
// DIR = +1 the unscaled inverse.
#pragma once

#include <hip/hip_runtime.h>

namespace vofl {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (DIR = -1) or +i (DIR = +1)
template <int DIR, typename T>
__device__ __forceinline__ cpx<T> mul_i(cpx<T> a) {
    if constexpr (DIR < 0) return {a.y, -a.x};
    else return {-a.y, a.x};
}
// twiddle from the forward table: forward uses w, inverse uses conj(w)
template <int DIR, typename T>
__device__ __forceinline__ cpx<T> twmul(cpx<T> a, cpx<T> w) {
    if constexpr (DIR > 0) w.y = -w.y;
    return cmul(a, w);
}

// Raw buffer load of one complex value: the descriptor (base, byte size)
// lives in scalar registers, the lane supplies a 32-bit byte offset; the
// hardware returns zero for offsets past the size. The third descriptor word
// is the gfx9 raw-buffer format (no swizzle, 32-bit data).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// NT: non-temporal cache policy (data read once from a stream larger than
// the caches).
template <typename T, bool NT = false>
__device__ __forceinline__ cpx<T> buffer_load_cpx(__amdgpu_buffer_rsrc_t r, unsigned off) {
    constexpr int policy = NT ? 2 : 0;
    cpx<T> c;
    if constexpr (sizeof(T) == 4) {
        auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, policy);
        __builtin_memcpy(&c, &v, 8);
    } else {
        auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, policy);
        __builtin_memcpy(&c, &v, 16);
    }
    return c;
}

// ---------------------------------------------------------------------------
// small DFTs in registers
// ---------------------------------------------------------------------------
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cpx<T>* v) {
    cpx<T> a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft3(cpx<T>* v) {
    const T h = T(0.86602540378443864676);  // sqrt(3)/2
    cpx<T> s = cadd(v[1], v[2]);
    cpx<T> d = csub(v[1], v[2]);
    cpx<T> m = {v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
    cpx<T> r = mul_i<DIR>(cscale(d, h));  // DIR*i*(sqrt3/2)(v1 - v2)
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

// 5-point DFT: with a1 = v1+v4, b1 = v1-v4, a2 = v2+v3, b2 = v2-v3 and
// theta = 2 pi/5, X1,4 = v0 + a1 cos(theta) + a2 cos(2 theta) -/+ i s (b1 sin(theta) + b2 sin(2 theta))
// and X2,3 = v0 + a1 cos(2 theta) + a2 cos(theta) -/+ i s (b1 sin(2 theta) - b2 sin(theta)),
// s = -DIR (the sign of the exponent)
template <int DIR, typename T>
__device__ __forceinline__ void dft5(cpx<T>* v) {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);  // cos(2 pi/5), cos(4 pi/5)
    const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);   // sin(2 pi/5), sin(4 pi/5)
    const cpx<T> a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const cpx<T> a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const cpx<T> m1 = {v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
    const cpx<T> m2 = {v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
    const cpx<T> t1 = mul_i<DIR>(cpx<T>{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    const cpx<T> t2 = mul_i<DIR>(cpx<T>{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(m1, t1);
    v[4] = csub(m1, t1);
    v[2] = cadd(m2, t2);
    v[3] = csub(m2, t2);
}

// 10-point DFT from two 5-point DFTs of the even and odd samples:
// X_k = E_k + w^k O_k, X_{k+5} = E_k - w^k O_k (k < 5), w = exp(s 2 pi i/10),
// s = DIR (the sign of the exponent)
template <int DIR, typename T>
__device__ __forceinline__ void dft10(cpx<T>* v) {
    cpx<T> e[5] = {v[0], v[2], v[4], v[6], v[8]};
    cpx<T> o[5] = {v[1], v[3], v[5], v[7], v[9]};
    dft5<DIR>(e);
    dft5<DIR>(o);
    // cos and sin of k pi/5, k = 1..4
    const T c[4] = {T(0.80901699437494742410), T(0.30901699437494742410), T(-0.30901699437494742410),
                    T(-0.80901699437494742410)};
    const T sn[4] = {T(0.58778525229247312917), T(0.95105651629515357212), T(0.95105651629515357212),
                     T(0.58778525229247312917)};
#pragma unroll
    for (int k = 1; k < 5; ++k) {
        const T ss = DIR < 0 ? -sn[k - 1] : sn[k - 1];
        o[k] = {o[k].x * c[k - 1] - o[k].y * ss, o[k].x * ss + o[k].y * c[k - 1]};
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        v[k] = cadd(e[k], o[k]);
        v[k + 5] = csub(e[k], o[k]);
    }
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cpx<T>* v) {
    cpx<T> a0 = cadd(v[0], v[2]);
    cpx<T> a1 = csub(v[0], v[2]);
    cpx<T> a2 = cadd(v[1], v[3]);
    cpx<T> a3 = mul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a1, a3);
    v[3] = csub(a1, a3);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cpx<T>* v) {
    const T r2 = T(0.70710678118654752440);
    cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<DIR>(e);
    dft4<DIR>(o);
    // o[k] *= W8^k, W8 = exp(DIR * i pi/4)
    cpx<T> o1 = o[1], o3 = o[3];
    if constexpr (DIR < 0) {
        o[1] = {r2 * (o1.x + o1.y), r2 * (o1.y - o1.x)};
        o[3] = {r2 * (-o3.x + o3.y), r2 * (-o3.y - o3.x)};
    } else {
        o[1] = {r2 * (o1.x - o1.y), r2 * (o1.y + o1.x)};
        o[3] = {r2 * (-o3.x - o3.y), r2 * (-o3.y + o3.x)};
    }
    o[2] = mul_i<DIR>(o[2]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = cadd(e[k], o[k]);
        v[k + 4] = csub(e[k], o[k]);
    }
}

template <int DIR, typename T>
__device__ __forceinline__ void dft16(cpx<T>* v) {
    // n = 4*n1 + n2, k = k1 + 4*k2: DFT4 over n1, twiddle W16^{n2 k1}, DFT4 over n2
    cpx<T> y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        cpx<T> a[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
        dft4<DIR>(a);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = a[k1];
    }
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
    const T r2 = T(0.70710678118654752440);
    // W16^j for j = n2*k1 in {1,2,3,4,6,9}; forward exp(-2 pi i j/16)
    auto tw = [&](cpx<T> a, int j) -> cpx<T> {
        T c, s;
        switch (j) {
            case 1: c = c1; s = s1; break;
            case 2: c = r2; s = r2; break;
            case 3: c = s1; s = c1; break;
            case 4: c = T(0); s = T(1); break;
            case 6: c = -r2; s = r2; break;
            case 9: c = -c1; s = -s1; break;
            default: c = T(1); s = T(0); break;
        }
        // forward: multiply by (c - i s); inverse: (c + i s)
        if constexpr (DIR < 0) return {a.x * c + a.y * s, a.y * c - a.x * s};
        else return {a.x * c - a.y * s, a.y * c + a.x * s};
    };
#pragma unroll
    for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) y[n2][k1] = tw(y[n2][k1], n2 * k1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cpx<T> b[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        dft4<DIR>(b);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
    }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cpx<T>* v) {
    if constexpr (R == 2) dft2<DIR>(v);
    else if constexpr (R == 3) dft3<DIR>(v);
    else if constexpr (R == 4) dft4<DIR>(v);
    else if constexpr (R == 5) dft5<DIR>(v);
    else if constexpr (R == 10) dft10<DIR>(v);
    else if constexpr (R == 8) dft8<DIR>(v);
    else if constexpr (R == 16) dft16<DIR>(v);
    else static_assert(R == 1, "unsupported radix");
}

// radix of the next stage: the first of 16, 10, 8, 5, 4, 3, 2 dividing both
// the remaining length and E
constexpr int pick_radix(int rem, int E) {
    return (rem % 16 == 0 && E % 16 == 0) ? 16
         : (rem % 10 == 0 && E % 10 == 0) ? 10
         : (rem % 8 == 0 && E % 8 == 0)   ? 8
         : (rem % 5 == 0 && E % 5 == 0)   ? 5
         : (rem % 4 == 0 && E % 4 == 0)   ? 4
         : (rem % 3 == 0 && E % 3 == 0)   ? 3
         : (rem % 2 == 0 && E % 2 == 0)   ? 2
                                          : 1;
}
constexpr int num_stages(int N, int E) {
    int s = 0, rem = N;
    while (rem > 1) {
        int r = pick_radix(rem, E);
        if (r == 1) return -1;
        rem /= r;
        ++s;
    }
    return s;
}

// LDS views. Pencil-major: element i of a pencil at base[i + i/8] (one pad
// slot per 8 elements: the radix-8 Stockham writes at stride 8, 64 and the
// unit-stride reads then fall on distinct banks for 32 lanes).
// Column-interleaved: element i of column c at base[i*W + c] (columns of a
// tile side by side; consecutive lanes hit consecutive addresses).
template <typename T>
struct LdsPencil {
    cpx<T>* base;
    __device__ __forceinline__ cpx<T>& operator[](int i) const { return base[i + (i >> 3)]; }
    static constexpr int footprint(int N) { return N + N / 8; }
};
// Swizzled pencil layout: element i at base[i ^ x(i)], x(i) built from
// single index bits XORed into lower bits, chosen per length, elements per
// thread and element size so that the exchanges of the Stockham stages
// (blocked writes, strided writes, cyclic reads) reach distinct LDS banks.
// The tables follow the bank behaviour measured on gfx950 with a probe of
// single-wavefront access patterns: 64 banks of 4 bytes, 64-bit reads
// served 32 lanes per cycle, 64-bit writes 16 lanes per cycle over 32 banks,
// 128-bit writes 8 lanes per cycle over 32 banks; every FP32 entry and the
// FP64 entries of 8 elements per thread measured conflict-free there (the
// FP64 4-per-thread entry keeps about 12% conflict cycles, against twice the
// cycles for the one-pad-per-8 layout). Lengths without an entry use the
// one-pad-per-8 layout.
struct SwzMasks {
    int src[5];  // source bit for low bit b, or -1
};
constexpr SwzMasks pencil_swizzle(int N, int E, int bytes) {
    if (bytes == 8) {
        if ((N == 256 || N == 512) && E == 8) return {{3, 4, 5, 6, -1}};
        if ((N == 256 || N == 1024) && E == 4) return {{3, 4, 4, 5, -1}};
    } else if (bytes == 16) {
        if ((N == 128 || N == 256 || N == 512) && E == 8) return {{3, 4, 5, -1, -1}};
        if ((N == 256 || N == 1024) && E == 4) return {{3, 4, 4, -1, -1}};
    }
    return {{-1, -1, -1, -1, -1}};
}
template <typename T, int N, int E>
struct LdsPencilX {
    static constexpr SwzMasks S = pencil_swizzle(N, E, int(sizeof(cpx<T>)));
    static constexpr bool SWZ = S.src[0] >= 0;
    cpx<T>* base;
    __device__ __forceinline__ static int map(int i) {
        if constexpr (!SWZ) {
            return i + (i >> 3);
        } else {
            int x = i;
#pragma unroll
            for (int b = 0; b < 5; ++b)
                if (S.src[b] >= 0) x ^= ((i >> S.src[b]) & 1) << b;
            return x;
        }
    }
    __device__ __forceinline__ cpx<T>& operator[](int i) const { return base[map(i)]; }
    static constexpr int footprint(int n) { return SWZ ? n : n + n / 8; }
};
template <typename T, int W>
struct LdsColumn {
    cpx<T>* base;  // already offset by the column index
    __device__ __forceinline__ cpx<T>& operator[](int i) const { return base[i * W]; }
    static constexpr int footprint(int N) { return N * W; }
};

// Synchronisation between the LDS write and read of an exchange. A
// transform whose threads all sit in one wavefront only needs its own LDS
// operations completed and ordered (no workgroup barrier); otherwise the
// whole workgroup synchronises.
template <bool WAVE>
__device__ __forceinline__ void exchange_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Twiddle sources for the stages. TwTable reads the length-N table
// tw[j] = exp(-2 pi i j/N) (global memory or LDS). TwRegs reads a thread's
// own twiddles from registers (filled once by load_twiddles), for kernels
// that run many transforms: for every stage after the first, its Q
// butterflies' R-1 twiddles, in stage order.
constexpr int tw_count(int N, int E) {
    int c = 0, ns = 1;
    while (ns < N) {
        const int r = pick_radix(N / ns, E);
        if (r <= 1) return -1;
        if (ns > 1) c += (E / r) * (r - 1);
        ns *= r;
    }
    return c;
}
// offset of the stage with stride NS in a TwRegs array
constexpr int tw_offset(int N, int E, int NS) {
    int c = 0, ns = 1;
    while (ns < NS) {
        const int r = pick_radix(N / ns, E);
        if (ns > 1) c += (E / r) * (r - 1);
        ns *= r;
    }
    return c;
}

template <typename T>
struct TwTable {
    const cpx<T>* __restrict__ tw;
    template <int N, int E, int NS, int R>
    __device__ __forceinline__ cpx<T> get(int, int r, int k) const {
        return tw[k * r * (N / (NS * R))];
    }
};
template <typename T, int C>
struct TwRegs {
    const cpx<T> (&w)[C];
    template <int N, int E, int NS, int R>
    __device__ __forceinline__ cpx<T> get(int q, int r, int) const {
        return w[tw_offset(N, E, NS) + q * (R - 1) + r - 1];
    }
};

// TwThread reads a thread's own twiddles from an LDS table laid out
// [twiddle index][pencil position] (filled once by stage_thread_twiddles):
// consecutive lanes read consecutive entries, free of bank conflicts, and no
// registers hold them between transforms.
template <typename T, int TP>
struct TwThread {
    const cpx<T>* tws;  // table base
    int t;              // this thread's pencil position
    template <int N, int E, int NS, int R>
    __device__ __forceinline__ cpx<T> get(int q, int r, int) const {
        return tws[(tw_offset(N, E, NS) + q * (R - 1) + r - 1) * TP + t];
    }
};

template <typename T, int N, int E, int NS, int C>
__device__ __forceinline__ void load_twiddles_at(cpx<T> (&w)[C], const int t, const cpx<T>* __restrict__ tw) {
    if constexpr (NS < N) {
        constexpr int R = pick_radix(N / NS, E);
        constexpr int TP = N / E, Q = E / R, OFF = tw_offset(N, E, NS);
        if constexpr (NS > 1) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int k = (t + q * TP) % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) w[OFF + q * (R - 1) + r - 1] = tw[k * r * (N / (NS * R))];
            }
        }
        load_twiddles_at<T, N, E, NS * R, C>(w, t, tw);
    }
}

// Fill w with thread t's twiddles (tw: the length-N table, e.g. in LDS).
template <typename T, int N, int E, int C>
__device__ __forceinline__ void load_twiddles(cpx<T> (&w)[C], const int t, const cpx<T>* __restrict__ tw) {
    static_assert(C == tw_count(N, E), "twiddle register count");
    load_twiddles_at<T, N, E, 1, C>(w, t, tw);
}

// Synchronisation of the exchanges (SYNC):
//  SYNC_BOTH  single LDS buffer, sync between an exchange's writes and reads
//             and again after the reads (the next stage overwrites it);
//  SYNC_PP    two buffers ("ping-pong") for kernels that run many transforms
//             in a row: exchange s uses buffer s mod 2, so only the sync
//             between writes and reads is needed. A wave that starts the
//             next exchange writes the other buffer, which every wave has
//             finished reading (it read it before the sync it just passed).
//             With an odd number of exchanges the transform ends with one
//             sync, so that the next transform's first exchange (buffer 0)
//             cannot overwrite the last one's (also buffer 0) under a slower
//             wave;
//  SYNC_ONCE  one transform per workgroup with a single exchange: one
//             buffer, one sync (nothing reuses the buffer afterwards).
enum { SYNC_BOTH = 0, SYNC_PP = 1, SYNC_ONCE = 2 };

// One Stockham stage with stride NS (product of the radices done before);
// S counts the stages done.
template <typename T, int N, int E, int DIR, int NS, int S, int SYNC, bool WAVE, class Lds, class TW>
__device__ __forceinline__ void fft_stages(cpx<T> (&v)[E], const int t, const Lds& l0, const Lds& l1,
                                           const TW& tws) {
    constexpr int R = pick_radix(N / NS, E);
    static_assert(R > 1, "length not supported by the radix set");
    constexpr int TP = N / E;
    constexpr int Q = E / R;  // butterflies per thread in this stage
    constexpr bool LAST = (NS * R == N);
    const Lds& lds = (SYNC == SYNC_PP && S % 2 == 1) ? l1 : l0;
    cpx<T> out[E];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int b = t + q * TP;  // butterfly index in [0, N/R)
        cpx<T> w[R];
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = v[q + r * Q];
        if constexpr (NS > 1) {
            const int k = b % NS;
#pragma unroll
            for (int r = 1; r < R; ++r) w[r] = twmul<DIR>(w[r], tws.template get<N, E, NS, R>(q, r, k));
        }
        dft<R, DIR>(w);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) out[q + r * Q] = w[r];
        } else {
            const int k = b % NS;
            const int base = (b / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[base + r * NS] = w[r];
        }
    }
    if constexpr (LAST) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = out[e];
        if constexpr (SYNC == SYNC_PP && S % 2 == 1) exchange_sync<WAVE>();  // odd number of exchanges
    } else {
        exchange_sync<WAVE>();
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = lds[t + e * TP];
        if constexpr (SYNC == SYNC_BOTH) exchange_sync<WAVE>();
        fft_stages<T, N, E, DIR, NS * R, S + 1, SYNC, WAVE, Lds, TW>(v, t, l0, l1, tws);
    }
}

// Full length-N transform of the pencil held as v[e] = x[t + TP*e].
// With WAVE = false every thread of the workgroup must call this (it
// contains workgroup barriers); with WAVE = true the pencil's TP threads
// must lie in one wavefront and only they synchronise.
template <typename T, int N, int E, int DIR, class Lds, bool WAVE = false>
__device__ __forceinline__ void fft_pencil(cpx<T> (&v)[E], const int t, const Lds& lds,
                                           const cpx<T>* __restrict__ tw) {
    static_assert(N % E == 0, "E must divide N");
    static_assert(num_stages(N, E) > 0, "length not supported");
    static_assert(!WAVE || (N / E) <= 64, "a wave-synchronised pencil must fit in one wavefront");
    fft_stages<T, N, E, DIR, 1, 0, SYNC_BOTH, WAVE>(v, t, lds, lds, TwTable<T>{tw});
}

// Fill the [twiddle index][pencil position] table of TwThread for positions
// t = 0..TP-1 from the length-N table tw (threads 0..TP-1 write; the caller
// synchronises before use).
template <typename T, int N, int E, int NS>
__device__ __forceinline__ void thread_twiddles_at(cpx<T>* dst, const int t, const cpx<T>* __restrict__ tw) {
    if constexpr (NS < N) {
        constexpr int R = pick_radix(N / NS, E);
        constexpr int TP = N / E, Q = E / R, OFF = tw_offset(N, E, NS);
        if constexpr (NS > 1) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int k = (t + q * TP) % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) dst[(OFF + q * (R - 1) + r - 1) * TP + t] = tw[k * r * (N / (NS * R))];
            }
        }
        thread_twiddles_at<T, N, E, NS * R>(dst, t, tw);
    }
}

// Transform with the thread's twiddles from the TwThread table.
template <typename T, int N, int E, int DIR, class Lds, bool WAVE>
__device__ __forceinline__ void fft_pencil_t(cpx<T> (&v)[E], const int t, const Lds& lds, const cpx<T>* tws) {
    static_assert(N % E == 0 && num_stages(N, E) > 0, "length not supported");
    static_assert(!WAVE || (N / E) <= 64, "a wave-synchronised pencil must fit in one wavefront");
    fft_stages<T, N, E, DIR, 1, 0, SYNC_BOTH, WAVE>(v, t, lds, lds, TwThread<T, N / E>{tws, t});
}

// The same with the thread's twiddles in registers (see load_twiddles).
template <typename T, int N, int E, int DIR, class Lds, bool WAVE, int C>
__device__ __forceinline__ void fft_pencil_r(cpx<T> (&v)[E], const int t, const Lds& lds, const cpx<T> (&w)[C]) {
    static_assert(N % E == 0 && num_stages(N, E) > 0, "length not supported");
    static_assert(!WAVE || (N / E) <= 64, "a wave-synchronised pencil must fit in one wavefront");
    fft_stages<T, N, E, DIR, 1, 0, SYNC_BOTH, WAVE>(v, t, lds, lds, TwRegs<T, C>{w});
}

// Two-buffer transform (SYNC_PP): every thread of the workgroup calls it,
// and between two calls the buffers are used for nothing else.
template <typename T, int N, int E, int DIR, class Lds>
__device__ __forceinline__ void fft_pencil_pp(cpx<T> (&v)[E], const int t, const Lds& l0, const Lds& l1,
                                              const cpx<T>* __restrict__ tw) {
    static_assert(N % E == 0 && num_stages(N, E) > 0, "length not supported");
    fft_stages<T, N, E, DIR, 1, 0, SYNC_PP, false>(v, t, l0, l1, TwTable<T>{tw});
}
template <typename T, int N, int E, int DIR, class Lds, int C>
__device__ __forceinline__ void fft_pencil_ppr(cpx<T> (&v)[E], const int t, const Lds& l0, const Lds& l1,
                                               const cpx<T> (&w)[C]) {
    static_assert(N % E == 0 && num_stages(N, E) > 0, "length not supported");
    fft_stages<T, N, E, DIR, 1, 0, SYNC_PP, false>(v, t, l0, l1, TwRegs<T, C>{w});
}

// Single transform per workgroup with one exchange (SYNC_ONCE).
template <typename T, int N, int E, int DIR, class Lds>
__device__ __forceinline__ void fft_pencil_once(cpx<T> (&v)[E], const int t, const Lds& l0,
                                                const cpx<T>* __restrict__ tw) {
    static_assert(num_stages(N, E) == 2, "one exchange only");
    fft_stages<T, N, E, DIR, 1, 0, SYNC_ONCE, false>(v, t, l0, l0, TwTable<T>{tw});
}

}  // namespace vofl
