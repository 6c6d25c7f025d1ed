// HIP kernels of the variable-order operator (2.13) and the TSFP2 step
// (3.13) on gfx950.
//
// Spectral layout: a real field of shape (n0[, n1][, n2]) has its spectrum
// stored for k0 = 0..n0/2 only ("half" along the OUTERMOST axis, Hermitian
// symmetry gives the rest), as complex [n0/2+1][n1][n2] (3D) or
// [n0/2+1][n1] (2D), last index fastest. Transforms along the last
// (contiguous) axis run on pencils; the other axes run on tiles of W
// consecutive columns, so every global access is coalesced along the last
// axis. The real<->half step happens along axis 0, inside the kernels that
// read/write physical data, where a column of a tile is a whole line.
//
// Kernel classes:
//   k_contig   last-axis transforms fused with the spectral pointwise work:
//              the 1/N scale, the kick update v_hat += dt*dv_hat, the exact
//              damped-oscillator sub-step (3.10)-(3.11), and the M+1 (or
//              2(M+1)) multiplied term spectra l_m |mu|^{2 sigma} u_hat of
//              (2.13), each inverse-transformed along the last axis.
//   k_mid      3D middle-axis C2C transforms of a range of fields (tiles).
//   k_r2c0     axis-0 forward transform of real fields (tiles), half output.
//   k_c2r0     axis-0 inverse transform of pairs of half spectra (two real
//              results from one complex transform) fused with the
//              delta-power sum of (2.13) and either the operator output, the
//              kick right-hand side plus its forward axis-0 transform, or the
//              export of (u, v).
//   k_1d_*     whole 1D apply / step loop of one field per workgroup in LDS.
#pragma once

#include "fft_engine.hpp"
#include <type_traits>

namespace vofl {

// IN_STATE: the spectral state (u_hat, v_hat) itself is the input (no
// transform), for steps resumed from the plan's state.
enum InKind : int { IN_APPLY = 0, IN_INIT = 1, IN_KICK = 2, IN_STATE = 3 };
enum EmitKind : int { EMIT_NONE = 0, EMIT_APPLY = 1, EMIT_STEP = 2, EMIT_EXPORT = 3, EMIT_GENERIC = 4 };
enum C2RMode : int { C2R_APPLY = 0, C2R_KICK = 1, C2R_EXPORT = 2, C2R_KICK_GENERIC = 3 };
enum ModelKind : int { MODEL_SEISMIC = 0, MODEL_GENERIC = 1 };

// Per-solve scalars: mean orders sig1 (1+gbar or s0) and sig2 (1/2+gbar),
// exact-part coefficients kappa0 = A(gbar), beta0 = B(gbar), and the
// coefficient of the cubic term (generic model).
struct SolveScalars {
    double sig1, sig2, kappa0, beta0, lambda, pad0, pad1, pad2;
};

// ---------------------------------------------------------------------------
// workgroup-to-tile order
// ---------------------------------------------------------------------------
// Workgroups are dispatched to the 8 XCDs in turn (b mod 8), each XCD with
// its own L2. Tiles whose rows are shorter than a 128-byte line share every
// line with their neighbours; xcd_group_tile gives workgroups b, b + 8, ...,
// b + 8(G-1) (one XCD) the G neighbouring tiles Gj .. Gj + G - 1 of a group
// of 8G, so each line is fetched into one L2 only. A last partial group
// keeps the identity order. The map is a permutation of [0, nb).
template <int G>
__device__ __forceinline__ int xcd_group_tile(int b, int nb) {
    if constexpr (G <= 1) {
        return b;
    } else {
        const int span = 8 * G, g = b / span, r = b % span;
        if ((g + 1) * span > nb) return b;
        return g * span + (r % 8) * G + r / 8;
    }
}
// tiles per 128-byte line for tile rows of W elements of B bytes
constexpr int line_group(int W, int B) {
    return (W * B >= 128) ? 1 : ((128 / (W * B)) > 8 ? 8 : 128 / (W * B));
}

// Non-temporal global load / store of one complex value (data streamed once
// through a pass larger than the caches).
template <typename T>
__device__ __forceinline__ cpx<T> nt_load(const cpx<T>* p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 r = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return {r.x, r.y};
}
template <typename T>
__device__ __forceinline__ void nt_store(cpx<T>* p, cpx<T> c) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 r;
    r.x = c.x;
    r.y = c.y;
    __builtin_nontemporal_store(r, reinterpret_cast<v2*>(p));
}

// ---------------------------------------------------------------------------
// pointwise helpers (FP64)
// ---------------------------------------------------------------------------

// The rarely taken overdamped branch of damped_flow, kept out of line; it
// returns its pair by value (in registers: reference outputs of an
// out-of-line call go through per-lane stack memory on every point, and the
// wait on that load also waits for every vector memory access in flight).
struct CoshSinh {
    double C, S;
};
__device__ __noinline__ CoshSinh overdamped_cs(double w2m, double t) {
    const double w = sqrt(w2m);
    return {cosh(w * t), sinh(w * t) / w};
}

// Exact flow over time t of u' = v, v' = -kappa0 P1 u - beta0 P2 v (one mode).
// b = beta0 P2/2, q = kappa0 P1, w^2 = q - b^2; the k = 0 mode (P1 = P2 = 0)
// gives u += t v (eq. (3.11)); beta0 = 0 gives the rotation (3.10).
__device__ __forceinline__ void damped_flow(double P1, double P2, double kappa0, double beta0,
                                            double t, double& g11, double& g12, double& g21,
                                            double& g22) {
    const double b = 0.5 * beta0 * P2;
    const double q = kappa0 * P1;
    const double w2 = q - b * b;
    double C, S;
    if (w2 > 0.0) {
        const double w = sqrt(w2);
        double sn, cs;
        sincos(w * t, &sn, &cs);
        C = cs;
        S = sn / w;
    } else if (w2 < 0.0) {
        const CoshSinh r = overdamped_cs(-w2, t);
        C = r.C;
        S = r.S;
    } else {
        C = 1.0;
        S = t;
    }
    const double e = (b != 0.0) ? exp(-b * t) : 1.0;
    g11 = e * (C + b * S);
    g12 = e * S;
    g21 = -e * q * S;
    g22 = e * (C - b * S);
}

template <typename T>
__device__ __forceinline__ cpx<double> to_d(cpx<T> a) {
    return {double(a.x), double(a.y)};
}
template <typename T>
__device__ __forceinline__ cpx<T> from_d(cpx<double> a) {
    return {T(a.x), T(a.y)};
}

// Tile width (columns per workgroup) of the strided kernels: the widest of
// 16/8/4 whose staged half columns fit in about 66 KB of LDS.
template <typename T, int N>
constexpr int tile_width() {
    constexpr int col = (N + 2) * int(sizeof(cpx<T>));
    return (16 * col <= 67584) ? 16 : (8 * col <= 67584) ? 8 : 4;
}
// Tile width of k_c2r0: 16 columns unless the FFT buffer (N x W complex)
// would exceed about 66 KB of LDS, and at most 512 threads (a power of two).
template <typename T, int N>
constexpr int c2r_width() {
    constexpr int col = N * int(sizeof(cpx<T>));
    constexpr int w = (16 * col <= 67584) ? 16 : (8 * col <= 67584) ? 8 : 4;
    // elements per thread of k_c2r0 (e_c2r0)
    constexpr int e = (N % 5 == 0) ? 10 : (N % 3 == 0) ? 12 : (N < 8 ? N : 8);
    int lim = (512 / (N / e)) < 1 ? 1 : (512 / (N / e));
    int p2 = 1;
    while (2 * p2 <= lim) p2 *= 2;
    return w < p2 ? w : p2;
}

// Copy a length-N twiddle table into LDS (called by every thread before
// any transform; ends with a barrier). Reading twiddles from LDS keeps the
// FFT stages from waiting on outstanding global loads.
template <typename T, int N>
__device__ __forceinline__ void stage_twiddles(cpx<T>* dst, const cpx<T>* __restrict__ src) {
    for (int i = threadIdx.x; i < N; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// ---------------------------------------------------------------------------
// k_contig: last-axis pencils
// ---------------------------------------------------------------------------
template <typename T, typename TI>
struct ContigArgs {
    const cpx<TI>* in;       // input half fields: item b, field f at in + b*in_istride + f*in_fstride
    long long in_istride, in_fstride;
    int nin;
    cpx<double>* U;          // spectral state u_hat, item b at U + b*H
    cpx<double>* V;          // spectral state v_hat
    cpx<T>* out;             // output slots: item b, slot s at out + b*out_istride + s*H
    long long out_istride;
    long long H;             // complex elements one half field occupies
    long long rs;            // row stride of a half field along axis 0 (>= n1 * N)
    int npencils;            // pencils of one field
    int n1;                  // pencils per k0 plane (3D: n1, 2D: 1)
    const double* mu2_0;     // mu^2 of axis 0 by bin
    const double* mu2_1;     // axis 1 (3D) or null
    const double* mu2_l;     // last axis
    const cpx<TI>* tw_in;    // last-axis twiddles for the input transform (precision TI)
    const cpx<T>* tw;        // last-axis twiddles for the output transforms
    const SolveScalars* sc;  // per item (sc_stride 1) or shared (0)
    int sc_stride;
    int in_kind, emit_kind, do_prop, M, op;
    int no_store;            // 1: leave the spectral state unchanged (IN_STATE exports)
    double tprop, dt, invN;
};

// Input spectra (forward transforms of caller data, and the FP64 staging)
// are transformed in precision TI; the term spectra in precision T.
// NT: the step's term slots are stored with the non-temporal policy (launches
// whose slots exceed the last-level cache).
template <typename T, typename TI, int N, int E, int P, bool NT = false>
__global__ __launch_bounds__(P*(N / E)) void k_contig(ContigArgs<T, TI> a) {
    constexpr int TP = N / E;
    // swizzled pencils: the exchanges of every stage are free of LDS bank
    // conflicts (one-pad-per-8 layout where the length has no table entry)
    using LPI = LdsPencilX<TI, N, E>;
    using LPT = LdsPencilX<T, N, E>;
    constexpr int FPI = LPI::footprint(N);
    constexpr int FP = LPT::footprint(N);
    __shared__ cpx<TI> lds_raw[P * FPI];  // holds P pencils of TI (>= size of T)
    __shared__ cpx<TI> twi_s[N];
    __shared__ cpx<T> tw_s[N];
    stage_twiddles<TI, N>(twi_s, a.tw_in);
    stage_twiddles<T, N>(tw_s, a.tw);
    const int lp = threadIdx.x / TP;
    const int t = threadIdx.x % TP;
    const int p = blockIdx.x * P + lp;
    const int bi = blockIdx.y;
    const bool active = p < a.npencils;
    const int pc = active ? p : 0;
    const LPI ldsi{lds_raw + lp * FPI};
    const LPT lds{reinterpret_cast<cpx<T>*>(lds_raw) + lp * FP};
    const int k0 = pc / a.n1;
    const int k1 = pc % a.n1;
    const double m2base = a.mu2_0[k0] + (a.mu2_1 ? a.mu2_1[k1] : 0.0);
    // pencil (k0, k1) of a half field: row k0 (stride rs), k1-th run of N
    const long long pen = (long long)k0 * a.rs + (long long)k1 * N;
    const SolveScalars sc = a.sc[bi * a.sc_stride];
    // a pencil's TP threads are consecutive and TP divides 64: every
    // transform stays inside one wavefront
    constexpr bool WV = (TP <= 64) && (64 % TP == 0);
    // Twiddles of the terms' inverse transforms (radix-4/8 schedules with at
    // most 16 per thread): for a pencil of one wavefront or less, from a
    // per-position LDS table (conflict-free, consecutive lanes read
    // consecutive entries); for longer pencils, from registers loaded once
    // (the table holds TP entries per twiddle: 12 x 256 x 16 bytes = 48 KiB
    // for a 1024-point FP64 pencil, a third of the workgroups per CU). The
    // schedules of 10 and 12 elements per thread (factors 5 or 3) read the
    // length-N table: with the per-position table the 768-point pass was 3.7
    // times slower.
    constexpr int TWC = tw_count(N, E);
    constexpr bool TWFEW = E <= 8 && TWC > 0 && TWC <= 16;
    constexpr bool TWT = TWFEW && TP <= 64;
    constexpr bool TWREG = TWFEW && !TWT;
    __shared__ cpx<T> twt_s[TWT ? TWC * TP : 1];
    if constexpr (TWT) {
        if (lp == 0) thread_twiddles_at<T, N, E, 1>(twt_s, t, tw_s);
        __syncthreads();
    }
    cpx<T> twr[TWREG ? TWC : 1];
    if constexpr (TWREG) load_twiddles<T, N, E, TWC>(twr, t, tw_s);
    auto inv_fft = [&](cpx<T> (&x)[E]) __attribute__((always_inline)) {
        if constexpr (TWT) fft_pencil_t<T, N, E, +1, LPT, WV>(x, t, lds, twt_s);
        else if constexpr (TWREG) fft_pencil_r<T, N, E, +1, LPT, WV, TWC>(x, t, lds, twr);
        else fft_pencil<T, N, E, +1, LPT, WV>(x, t, lds, tw_s);
    };

    cpx<double> uh[E], vh[E];
    if (a.in_kind == IN_STATE) {
        const cpx<double>* Us = a.U + (long long)bi * a.H + pen;
        const cpx<double>* Vs = a.V + (long long)bi * a.H + pen;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            uh[e] = Us[t + TP * e];
            vh[e] = Vs[t + TP * e];
        }
    } else if (a.in_kind == IN_KICK) {
        cpx<TI> d[E];
        const cpx<TI>* src = a.in + (long long)bi * a.in_istride + pen;
#pragma unroll
        for (int e = 0; e < E; ++e) d[e] = src[t + TP * e];
        fft_pencil<TI, N, E, -1, LPI, WV>(d, t, ldsi, twi_s);
        const cpx<double>* Us = a.U + (long long)bi * a.H + pen;
        const cpx<double>* Vs = a.V + (long long)bi * a.H + pen;
        const double s = a.dt * a.invN;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            uh[e] = Us[t + TP * e];
            const cpx<double> vv = Vs[t + TP * e];
            vh[e] = {vv.x + s * double(d[e].x), vv.y + s * double(d[e].y)};
        }
    } else {
        for (int f = 0; f < a.nin; ++f) {
            cpx<TI> d[E];
            const cpx<TI>* src = a.in + (long long)bi * a.in_istride + (long long)f * a.in_fstride + pen;
#pragma unroll
            for (int e = 0; e < E; ++e) d[e] = src[t + TP * e];
            fft_pencil<TI, N, E, -1, LPI, WV>(d, t, ldsi, twi_s);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const cpx<double> z = {double(d[e].x) * a.invN, double(d[e].y) * a.invN};
                if (f == 0) uh[e] = z;
                else vh[e] = z;
            }
        }
        if (a.nin < 2) {
#pragma unroll
            for (int e = 0; e < E; ++e) vh[e] = {0.0, 0.0};
        }
    }

    // per element: ln|mu|^2, the symbols |mu|^{2 sig} (zero at k = 0), the
    // exact sub-step, the state store, and the first multiplier of the terms
    double L[E];
    cpx<double>* Ud = a.U + (long long)bi * a.H + pen;
    cpx<double>* Vd = a.V + (long long)bi * a.H + pen;
    const bool store_state = (a.in_kind != IN_APPLY) && !a.no_store && active;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const double m2 = m2base + a.mu2_l[t + TP * e];
        double P1 = 0.0, P2 = 0.0;
        L[e] = 0.0;
        if (m2 > 0.0) {
            L[e] = log(m2);
            P1 = exp(sc.sig1 * L[e]);
            P2 = exp(sc.sig2 * L[e]);
        }
        if (a.do_prop) {
            double g11, g12, g21, g22;
            damped_flow(P1, P2, sc.kappa0, sc.beta0, a.tprop, g11, g12, g21, g22);
            const cpx<double> u0 = uh[e], v0 = vh[e];
            uh[e] = {g11 * u0.x + g12 * v0.x, g11 * u0.y + g12 * v0.y};
            vh[e] = {g21 * u0.x + g22 * v0.x, g21 * u0.y + g22 * v0.y};
        }
        if (store_state) {
            Ud[t + TP * e] = uh[e];
            Vd[t + TP * e] = vh[e];
        }
        if (a.emit_kind == EMIT_STEP) {
            uh[e] = {P1 * uh[e].x, P1 * uh[e].y};
            vh[e] = {P2 * vh[e].x, P2 * vh[e].y};
        } else if (a.emit_kind == EMIT_GENERIC) {
            vh[e] = uh[e];  // u_hat itself, for the nonlinear term
            uh[e] = {P1 * uh[e].x, P1 * uh[e].y};
        } else if (a.emit_kind == EMIT_APPLY) {
            const double c = (a.op == 2) ? P2 : P1;
            uh[e] = {c * uh[e].x, c * uh[e].y};
        }
    }

    cpx<T>* dst0 = a.out + (long long)bi * a.out_istride + pen;
    if (a.emit_kind == EMIT_GENERIC) {
        // slot M+1: u_hat itself (inverse along the last axis)
        {
            cpx<T> x[E];
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = from_d<T>(vh[e]);
            inv_fft(x);
            if (active) {
                cpx<T>* d = dst0 + (long long)(a.M + 1) * a.H;
#pragma unroll
                for (int e = 0; e < E; ++e) d[t + TP * e] = x[e];
            }
        }
    }
    if (a.emit_kind == EMIT_APPLY || a.emit_kind == EMIT_GENERIC) {
        // x_m = l_m |mu|^{2 sig} u_hat, l_{m+1} = l_m L/(m+1)
        for (int m = 0; m <= a.M; ++m) {
            cpx<T> x[E];
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = from_d<T>(uh[e]);
            inv_fft(x);
            if (active) {
                cpx<T>* d = dst0 + (long long)m * a.H;
#pragma unroll
                for (int e = 0; e < E; ++e) d[t + TP * e] = x[e];
            }
            const double inv = 1.0 / double(m + 1);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double f = L[e] * inv;
                uh[e] = {uh[e].x * f, uh[e].y * f};
            }
        }
    } else if (a.emit_kind == EMIT_STEP) {
        for (int m = 0; m <= a.M; ++m) {
            cpx<T> x[E];
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = from_d<T>(uh[e]);
            inv_fft(x);
            if (active) {
                cpx<T>* d = dst0 + (long long)(2 * m) * a.H;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if constexpr (NT) nt_store(d + t + TP * e, x[e]);
                    else d[t + TP * e] = x[e];
                }
            }
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = from_d<T>(vh[e]);
            inv_fft(x);
            if (active) {
                cpx<T>* d = dst0 + (long long)(2 * m + 1) * a.H;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if constexpr (NT) nt_store(d + t + TP * e, x[e]);
                    else d[t + TP * e] = x[e];
                }
            }
            const double inv = 1.0 / double(m + 1);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double f = L[e] * inv;
                uh[e] = {uh[e].x * f, uh[e].y * f};
                vh[e] = {vh[e].x * f, vh[e].y * f};
            }
        }
    } else if (a.emit_kind == EMIT_EXPORT) {
        for (int f = 0; f < 2; ++f) {
            cpx<T> x[E];
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = from_d<T>(f == 0 ? uh[e] : vh[e]);
            inv_fft(x);
            if (active) {
                cpx<T>* d = dst0 + (long long)f * a.H;
#pragma unroll
                for (int e = 0; e < E; ++e) d[t + TP * e] = x[e];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// k_mid: 3D axis-1 C2C on a range of fields, in place
// ---------------------------------------------------------------------------
template <typename T>
struct MidArgs {
    cpx<T>* buf;            // item b, field f at buf + b*istride + f*H
    long long istride;
    int nf;                 // fields per item
    long long H;
    long long rs;           // stride of the k0 planes (>= n1 * n2)
    int n2;                 // columns of a k0 plane (last axis length)
    int tiles_per_plane;    // ceil(n2 / W)
    const cpx<T>* tw;       // axis-1 twiddles
};

template <typename T, int N, int E, int W, int DIR, bool NT = false>
__global__ __launch_bounds__(W*(N / E)) void k_mid(MidArgs<T> a) {
    constexpr int TP = N / E;
    __shared__ cpx<T> lds_raw[N * W];
    __shared__ cpx<T> tw_s[N];
    stage_twiddles<T, N>(tw_s, a.tw);
    const int c = threadIdx.x % W;
    const int t = threadIdx.x / W;
    const int tiles = (a.n2 + W - 1) / W;
    const int bl = xcd_group_tile<line_group(W, int(sizeof(cpx<T>)))>(blockIdx.x, gridDim.x);
    const int plane = bl / tiles;
    const int col = (bl % tiles) * W + c;
    const bool active = col < a.n2;
    const int colc = active ? col : 0;
    const int item = blockIdx.y / a.nf;
    const int f = blockIdx.y % a.nf;
    cpx<T>* base = a.buf + (long long)item * a.istride + (long long)f * a.H + (long long)plane * a.rs + colc;
    const LdsColumn<T, W> lds{lds_raw + c};
    cpx<T> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const cpx<T>* q = base + (long long)(t + TP * e) * a.n2;
        v[e] = NT ? nt_load(q) : *q;
    }
    if constexpr (num_stages(N, E) == 2) fft_pencil_once<T, N, E, DIR>(v, t, lds, tw_s);
    else fft_pencil<T, N, E, DIR>(v, t, lds, tw_s);
    if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            cpx<T>* q = base + (long long)(t + TP * e) * a.n2;
            if constexpr (NT) nt_store(q, v[e]);
            else *q = v[e];
        }
    }
}

// ---------------------------------------------------------------------------
// k_r2c0: axis-0 forward transform of real fields -> half spectra
// ---------------------------------------------------------------------------
template <typename TR>
struct R2CArgs {
    const TR* in;           // real fields: item b at in + b*Nreal
    const TR* in2;          // optional second fields: the input is c1 in + c2 in2 (FP64)
    double c1, c2;
    long long Nreal;
    cpx<double>* out;       // FP64 half spectra: item b at out + b*H, row k at + k*rs
    long long H;
    long long rs;
    int inner;              // columns (product of the other axes)
    const cpx<double>* tw;  // axis-0 twiddles (FP64)
};

// Forward axis-0 transform of caller data, in FP64 whatever the plan
// precision: the operator amplifies rounding noise of the input spectrum by
// up to |mu_max|^{2 s}, so the first transform is kept exact to FP64.
template <typename TR, int N, int E, int W>
__global__ __launch_bounds__(W*(N / E)) void k_r2c0(R2CArgs<TR> a) {
    constexpr int TP = N / E;
    __shared__ cpx<double> lds_raw[N * W];
    __shared__ cpx<double> tw_s[N];
    stage_twiddles<double, N>(tw_s, a.tw);
    const int c = threadIdx.x % W;
    const int t = threadIdx.x / W;
    const int col = xcd_group_tile<line_group(W, int(sizeof(TR)))>(blockIdx.x, gridDim.x) * W + c;
    const bool active = col < a.inner;
    const int colc = active ? col : 0;
    const int item = blockIdx.y;
    const TR* src = a.in + (long long)item * a.Nreal + colc;
    const LdsColumn<double, W> lds{lds_raw + c};
    cpx<double> v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = {double(src[(long long)(t + TP * e) * a.inner]), 0.0};
    if (a.in2) {  // uniform: a combination of two fields, formed in FP64 while loading
        const TR* src2 = a.in2 + (long long)item * a.Nreal + colc;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e].x = a.c1 * v[e].x + a.c2 * double(src2[(long long)(t + TP * e) * a.inner]);
    }
    fft_pencil<double, N, E, -1>(v, t, lds, tw_s);
    if (active) {
        cpx<double>* dst = a.out + (long long)item * a.H + colc;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + TP * e;
            if (k <= N / 2) {
                cpx<double> z = v[e];
                if (k == 0 || k == N / 2) z.y = 0.0;
                dst[(long long)k * a.rs] = z;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// k_c2r0: axis-0 inverse of pairs of half spectra + (2.13) sum + epilogue
// ---------------------------------------------------------------------------
template <typename T>
struct C2RArgs {
    const cpx<T>* in;       // half slots: item b, slot s at in + b*istride + s*H, row k at + k*rs
    long long istride;
    long long H;
    long long rs;           // row stride of the half slots (>= inner); physical rows: inner
    int inner;
    const cpx<T>* tw;       // axis-0 twiddles
    int mode, M, model;
    // per-point coefficients (physical layout); stride 0 if shared by items
    const double* delta;
    const T* A;
    const T* B;
    long long coef_stride;
    const SolveScalars* sc;
    int sc_stride;
    // outputs
    cpx<T>* dv_out;         // kick: half field of item b at dv_out + b*istride
    T* r0;                  // apply: out; export: u (item b at r0 + b*Nreal)
    T* r1;                  // export: v
    long long Nreal;
    int* flag;              // set to 1 on a non-finite kick value
    // leap-frog (lffp = 1): FP64 fields of item b at s_prev + b*Nreal,
    // s_cur + b*Nreal; per point prev <- cur, cur <- new with
    //   apply mode (1.5): new = lf_cb*cur + lf_ca*prev + lf_cf*(-kappa acc + lambda cur^3),
    //     acc = the operator (2.13) applied to cur;
    //   kick mode (1.1): new = lf_cb*cur + lf_ca*prev + lf_cf*acc, acc = -A L1 u - B L2 w
    //     summed in full (the exact-part coefficients kappa0, beta0 are not
    //     subtracted), from the term pairs of (u, w) = (cur, difference quotient)
    int lffp;
    double* s_prev;
    double* s_cur;
    double lf_cb, lf_ca, lf_cf;
};

// One leap-frog update (3.4a) at a point (see C2RArgs); returns false if the
// new value is not finite.
__device__ __forceinline__ bool lffp_point(double* prev, double* cur, double Lu, double kappa, double lambda,
                                           double cb, double ca, double cf) {
    const double u = *cur;
    const double nw = cb * u + ca * (*prev) + cf * (-kappa * Lu + lambda * u * u * u);
    *prev = u;
    *cur = nw;
    return isfinite(nw);
}

// Y = a + i b, with a, b the Hermitian extensions of two half columns.
template <typename T, int N, int W>
__device__ __forceinline__ cpx<T> hermitian_pair(const cpx<T>* h1, const cpx<T>* h2, int c, int k) {
    if (k <= N / 2) {
        cpx<T> p = h1[k * W + c];
        cpx<T> q = h2 ? h2[k * W + c] : cpx<T>{T(0), T(0)};
        if (k == 0 || k == N / 2) {
            p.y = T(0);
            q.y = T(0);
        }
        return {p.x - q.y, p.y + q.x};
    }
    const int kk = N - k;
    const cpx<T> p = h1[kk * W + c];
    const cpx<T> q = h2 ? h2[kk * W + c] : cpx<T>{T(0), T(0)};
    return {p.x + q.y, q.x - p.y};
}

// Transforms of one k_c2r0 launch: transform i reads the slot pair
// (2i, 2i+1); the second slot is absent (-1) past the last slot.
// The export transforms u and v one at a time: v is far smaller than u
// early in a solve (v0 = 0), and a shared complex transform would add
// rounding relative to u to it.
__device__ __forceinline__ int c2r_transforms(int mode, int M) {
    switch (mode) {
        case C2R_EXPORT: return 2;
        case C2R_APPLY: return (M + 2) / 2;         // slots 0..M
        case C2R_KICK: return M + 1;                // slots 0..2M+1
        default: return (M + 3) / 2;                // generic: slots 0..M+1
    }
}
__device__ __forceinline__ int c2r_nslots(int mode, int M) {
    switch (mode) {
        case C2R_EXPORT: return 2;
        case C2R_APPLY: return M + 1;
        case C2R_KICK: return 2 * M + 2;
        default: return M + 2;
    }
}

// PD: slot pairs kept in flight (loaded into registers PD transforms ahead).
// PAIRED: each stored row is loaded once. Pencil positions t and TP - t hold
// each other's mirror rows (N - (t + TP e) = (TP - t) + TP (E-1-e)), so they
// are placed in the same wavefront, W lanes apart, and swap their loaded
// rows with lane shuffles; t = 0 and t = TP/2 are their own mirrors.
// STAGED: each stored row is loaded once, by one thread, into an LDS stage
// (rows t + TP e for e < E/2 and the Nyquist row), and every thread reads
// its rows min(k, N - k) from there; for lengths whose pencil positions
// cannot be paired inside a wavefront.
// NT: the slot loads use the non-temporal policy (launches whose slots are
// larger than the last-level cache: they are read once and not kept).
template <typename T, int N, int E, int W, int MODE, int WPE, int PD = 1, bool PAIRED = false,
          bool STAGED = false, bool NT = false>
__global__ __launch_bounds__(W*(N / E)) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_c2r0(C2RArgs<T> a) {
    static_assert(MODE >= 0 && MODE <= 3, "mode");
    constexpr int TP = N / E;
    static_assert(!PAIRED || (E % 2 == 0 && TP >= 2 && W <= 32 && (64 / W) % 2 == 0 && (TP * W) % 64 == 0),
                  "paired layout needs pencil-position pairs inside a wavefront");
    static_assert(!(PAIRED && STAGED) && (!STAGED || E % 2 == 0), "staged layout");
    constexpr int NL = (PAIRED || STAGED) ? E / 2 + 1 : E;  // rows loaded per slot and thread
    constexpr int HR = N / 2 + 1;                            // stored rows
    // the paired variants also use a second FFT buffer (one barrier per exchange)
    __shared__ cpx<T> lds_fft[N * W];
    __shared__ cpx<T> lds_fft2[PAIRED ? N * W : 1];
    __shared__ cpx<T> stg[STAGED ? 2 * HR * W : 1];
    __shared__ cpx<T> tw_s[N];
    stage_twiddles<T, N>(tw_s, a.tw);
    constexpr int TW = (W <= 64) ? 64 / W : 1;  // pencil positions per wavefront
    const int lane = threadIdx.x % 64, jw = lane / W;
    const int pr = int(threadIdx.x / 64) * (TW / 2) + jw / 2;  // PAIRED: pair index
    const int c = PAIRED ? lane % W : threadIdx.x % W;
    const int t = PAIRED ? ((jw % 2 == 0) ? pr : (pr == 0 ? TP / 2 : TP - pr)) : threadIdx.x / W;
    // grouped by the narrowest per-point array read (A, B in the plan precision)
    const int tile = xcd_group_tile<line_group(W, int(sizeof(T)))>(blockIdx.x, gridDim.x);
    const int col = tile * W + c;
    const bool active = col < a.inner;
    const int colc = active ? col : 0;
    const int item = blockIdx.y;
    const LdsColumn<T, W> lds{lds_fft + c};
    const LdsColumn<T, W> lds2{lds_fft2 + (PAIRED ? c : 0)};
    // the paired variants with E <= 8 keep this thread's twiddles in
    // registers for all the transforms of the kernel
    constexpr bool TWREG = PAIRED && E <= 8 && tw_count(N, E) > 0 && tw_count(N, E) <= 16;
    constexpr int TWC = TWREG ? tw_count(N, E) : 1;
    cpx<T> twr[TWC];
    if constexpr (TWREG) load_twiddles<T, N, E, TWC>(twr, t, tw_s);
    auto fft = [&](cpx<T> (&x)[E], auto dir) __attribute__((always_inline)) {
        if constexpr (TWREG)
            fft_pencil_ppr<T, N, E, decltype(dir)::value, LdsColumn<T, W>, TWC>(x, t, lds, lds2, twr);
        else if constexpr (PAIRED) fft_pencil_pp<T, N, E, decltype(dir)::value, LdsColumn<T, W>>(x, t, lds, lds2, tw_s);
        else fft_pencil<T, N, E, decltype(dir)::value>(x, t, lds, tw_s);
    };
    const cpx<T>* ibase = a.in + (long long)item * a.istride;  // uniform
    const int nT = c2r_transforms(MODE, a.M);
    const int nS = c2r_nslots(MODE, a.M);

    // Each thread loads, for its rows k = t + TP*e, the stored row
    // min(k, N-k) of both slots of a pair directly into registers (the
    // mirror rows of two threads coincide and come from cache the second
    // time); the next pair is loaded while the current one is transformed.
    // Per-lane 32-bit byte offsets (a half field is below 4 GiB, checked by
    // the plan); the slot base is uniform.
    unsigned roff[NL];
    auto row_off = [&](int e) __attribute__((always_inline)) -> unsigned {
        if constexpr (PAIRED || STAGED) {
            // rows t + TP e for e < E/2, and the Nyquist row (used by t = 0
            // only; the other positions load the same cached row and drop it)
            const int r = (e == E / 2) ? N / 2 : t + TP * e;
            return (unsigned(r) * unsigned(a.rs) + unsigned(colc)) * unsigned(sizeof(cpx<T>));
        }
        const int k = t + TP * e;
        const int r = (k <= N / 2) ? k : N - k;
        return (unsigned(r) * unsigned(a.rs) + unsigned(colc)) * unsigned(sizeof(cpx<T>));
    };
#pragma unroll
    for (int e = 0; e < NL; ++e) roff[e] = row_off(e);
    cpx<T> p1[PD][E], p2[PD][E];
    // Loads of pair tr into (q1, q2). A pair past the last one reads through
    // an empty buffer descriptor (zeros, no memory traffic), and a lone last
    // slot is loaded twice and masked in build(), so that no branch depends
    // on the pair index and the compiler can keep PD pairs in flight.
    auto load_pair = [&](int tr, cpx<T> (&q1)[E], cpx<T> (&q2)[E]) __attribute__((always_inline)) {
        const bool live = tr < nT;
        const int s1 = live ? (MODE == C2R_EXPORT ? tr : 2 * tr) : 0;
        const int s2 = live ? (MODE == C2R_EXPORT ? tr : min(2 * tr + 1, nS - 1)) : 0;
        const unsigned bytes = live ? unsigned(a.H * (long long)sizeof(cpx<T>)) : 0u;
        const auto r1 = make_rsrc(ibase + (long long)s1 * a.H, bytes);
        const auto r2 = make_rsrc(ibase + (long long)s2 * a.H, bytes);
#pragma unroll
        for (int e = 0; e < NL; ++e) {
            q1[e] = buffer_load_cpx<T, NT>(r1, roff[e]);
            q2[e] = buffer_load_cpx<T, NT>(r2, roff[e]);
        }
    };
    auto shfl = [&](cpx<T> v) __attribute__((always_inline)) -> cpx<T> {
        return {__shfl_xor(v.x, W), __shfl_xor(v.y, W)};
    };
    // Y = a + i b with a, b the Hermitian extensions along axis 0 (selects,
    // no branches); two = false when the pair has a single slot
    auto build = [&](cpx<T> (&y)[E], const cpx<T> (&q1)[E], const cpx<T> (&q2)[E], bool two)
        __attribute__((always_inline)) {
        if constexpr (PAIRED) {
            cpx<T> m1[E / 2], m2[E / 2];  // the partner position's loaded rows
#pragma unroll
            for (int e = 0; e < E / 2; ++e) {
                m1[e] = shfl(q1[e]);
                m2[e] = shfl(q2[e]);
            }
            // Y = a + i b from the rows a (slot 1) and b (slot 2) of element
            // e: rows k <= N/2 as loaded (lo), rows k > N/2 as the conjugate
            // of the mirror row N - k
            auto pair_lo = [&](cpx<T> a, cpx<T> b) __attribute__((always_inline)) -> cpx<T> {
                return two ? cpx<T>{a.x - b.y, a.y + b.x} : a;
            };
            auto pair_hi = [&](cpx<T> a, cpx<T> b) __attribute__((always_inline)) -> cpx<T> {
                return two ? cpx<T>{a.x + b.y, b.x - a.y} : cpx<T>{a.x, -a.y};
            };
            // positions other than 0 and TP/2: rows t + TP e for e < E/2 are
            // this thread's loads; the mirror rows of the others are the
            // partner's loads of elements E - 1 - e
#pragma unroll
            for (int e = 0; e < E; ++e)
                y[e] = (e < E / 2) ? pair_lo(q1[e], q2[e]) : pair_hi(m1[E - 1 - e], m2[E - 1 - e]);
            // positions 0 and TP/2 (two lanes of one wavefront per column
            // group): position 0 holds rows 0 and N/2 (real: zero imaginary
            // parts) and mirrors itself at TP (E - e); TP/2 mirrors itself
            if (t == 0) {
                const cpx<T> a0 = {q1[0].x, T(0)}, b0 = {q2[0].x, T(0)};
                const cpx<T> an = {q1[E / 2].x, T(0)}, bn = {q2[E / 2].x, T(0)};
                y[0] = pair_lo(a0, b0);
                y[E / 2] = pair_lo(an, bn);
#pragma unroll
                for (int e = E / 2 + 1; e < E; ++e) y[e] = pair_hi(q1[E - e], q2[E - e]);
            } else if (t == TP / 2) {
#pragma unroll
                for (int e = E / 2; e < E; ++e) y[e] = pair_hi(q1[E - 1 - e], q2[E - 1 - e]);
            }
            return;
        }
        if constexpr (STAGED) {
            // the previous pair's stage reads are complete once every thread
            // has passed an exchange barrier of its transform; a transform
            // without an exchange needs a barrier here
            if constexpr (num_stages(N, E) < 2) __syncthreads();
#pragma unroll
            for (int e = 0; e < E / 2; ++e) {
                const int r = t + TP * e;
                stg[r * W + c] = q1[e];
                stg[(HR + r) * W + c] = q2[e];
            }
            if (t == 0) {
                stg[(N / 2) * W + c] = q1[E / 2];
                stg[(HR + N / 2) * W + c] = q2[E / 2];
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = t + TP * e;
                const int r = (k <= N / 2) ? k : N - k;
                const cpx<T> u1 = stg[r * W + c], u2 = stg[(HR + r) * W + c];
                const bool lo = k <= N / 2;
                const bool edge = (k == 0) || (k == N / 2);
                const T ax = u1.x, ay = edge ? T(0) : u1.y;
                const T bx = two ? u2.x : T(0);
                const T by = (two && !edge) ? u2.y : T(0);
                y[e] = {lo ? ax - by : ax + by, lo ? ay + bx : bx - ay};
            }
            return;
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + TP * e;
            const bool lo = k <= N / 2;
            const bool edge = (k == 0) || (k == N / 2);
            const T ax = q1[e].x, ay = edge ? T(0) : q1[e].y;
            const T bx = two ? q2[e].x : T(0);
            const T by = (two && !edge) ? q2[e].y : T(0);
            y[e] = {lo ? ax - by : ax + by, lo ? ay + bx : bx - ay};
        }
    };

    // delta at this thread's points, held in registers (FP64)
    const SolveScalars sc = a.sc[item * a.sc_stride];
    // the leap-frog kick sums the full operators (no exact part to subtract)
    const double kap0 = a.lffp ? 0.0 : sc.kappa0;
    const double bet0 = a.lffp ? 0.0 : sc.beta0;
    double dl[E];
    if constexpr (MODE != C2R_EXPORT) {
        const double* dptr = a.delta + (long long)item * a.coef_stride + colc;
#pragma unroll
        for (int e = 0; e < E; ++e) dl[e] = dptr[(long long)(t + TP * e) * a.inner];
    }

    // Accumulation in the plan precision T (FP32 or FP64); the powers
    // delta^m and the coefficients (kappa0 - A), (beta0 - B), -A delta^m,
    // -B delta^m are formed in FP64 and rounded once:
    //  apply:   acc = sum_m delta^m t_m
    //  kick:    acc = (kappa0 - A) t1_0 + (beta0 - B) t2_0 + sum_{m>=1} delta^m (-A t1_m - B t2_m)
    //  generic: acc = -kappa sum_{s=1..M} delta^s t_s, uu = IDFT(u_hat)
    // FP32 kick (SPLIT): the m >= 1 part is accumulated as S1 = sum delta^m t1_m
    // and S2 = sum delta^m t2_m (delta^m rounded once) and multiplied by -A,
    // -B at the end; these sums are small corrections to the m = 0 term, and
    // the split saves three instructions per point and transform.
    constexpr bool SPLIT = MODE == C2R_KICK && sizeof(T) == 4 && E <= 8;
    T acc[E], cA[E], cB[E];
    T S1[SPLIT ? E : 1], S2[SPLIT ? E : 1];
    T ux[MODE == C2R_EXPORT ? E : 1];  // export: u from the first transform
    double dm[E];
    cpx<T> y[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        acc[e] = T(0);
        dm[e] = 1.0;
        cA[e] = T(0);
        cB[e] = T(0);
        if constexpr (SPLIT) {
            S1[e] = T(0);
            S2[e] = T(0);
        }
    }
    if constexpr (MODE == C2R_KICK) {
        const T* Ap = a.A + (long long)item * a.coef_stride + colc;
        const T* Bp = a.B + (long long)item * a.coef_stride + colc;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const long long off = (long long)(t + TP * e) * a.inner;
            cA[e] = -Ap[off];
            cB[e] = -Bp[off];
        }
    }

    // transform tr of the pair held in y: inverse axis-0 FFT and accumulation
    auto transform = [&](int tr) __attribute__((always_inline)) {
        fft(y, std::integral_constant<int, +1>{});
        if constexpr (MODE == C2R_EXPORT) {
            if (tr == 0) {
#pragma unroll
                for (int e = 0; e < E; ++e) ux[e] = y[e].x;
            }
        } else if constexpr (MODE == C2R_APPLY) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double d = dl[e];
                acc[e] += T(dm[e]) * y[e].x + T(dm[e] * d) * y[e].y;
                dm[e] *= d * d;
            }
        } else if constexpr (SPLIT) {
            if (tr == 0) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    acc[e] = T(kap0 + double(cA[e])) * y[e].x + T(bet0 + double(cB[e])) * y[e].y;
                    dm[e] = dl[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const T w = T(dm[e]);
                    S1[e] += w * y[e].x;
                    S2[e] += w * y[e].y;
                    dm[e] *= dl[e];
                }
            }
        } else if constexpr (MODE == C2R_KICK) {
            const double k0c = (tr == 0) ? kap0 : 0.0;
            const double b0c = (tr == 0) ? bet0 : 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T ca = T(k0c + double(cA[e]) * dm[e]);
                const T cb = T(b0c + double(cB[e]) * dm[e]);
                acc[e] += ca * y[e].x + cb * y[e].y;
                dm[e] *= dl[e];
            }
        } else if constexpr (MODE == C2R_KICK_GENERIC) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double d = dl[e];
                for (int h = 0; h < 2; ++h) {
                    const int sidx = 2 * tr + h;
                    if (sidx >= nS) break;
                    const T val = h == 0 ? y[e].x : y[e].y;
                    if (sidx == a.M + 1) {
                        cB[e] = val;  // u at the half step, for the cubic term
                    } else {
                        if (sidx > 0) acc[e] -= T(sc.kappa0 * dm[e]) * val;
                        dm[e] *= d;
                    }
                }
            }
        }
    };

    // software pipeline: PD pairs in flight; buffer d holds the pairs tr = d
    // (mod PD). The pair count is padded to a multiple of PD with empty pairs
    // (zero data: they add nothing to the sums).
    const int nTp = ((nT + PD - 1) / PD) * PD;
    // (scheduling barriers keep each pair's loads together, in issue order,
    // so that the in-order load counter can wait for one pair at a time)
#pragma unroll
    for (int d = 0; d < PD; ++d) {
        load_pair(d, p1[d], p2[d]);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int base = 0; base < nTp; base += PD) {
#pragma unroll
        for (int d = 0; d < PD; ++d) {
            const int tr = base + d;
            build(y, p1[d], p2[d], MODE != C2R_EXPORT && 2 * tr + 1 < nS);
            __builtin_amdgcn_sched_barrier(0);
            load_pair(tr + PD, p1[d], p2[d]);  // in flight during the next transforms
            __builtin_amdgcn_sched_barrier(0);
            transform(tr);
        }
    }

    if constexpr (MODE == C2R_EXPORT) {
        if (active) {
            T* u = a.r0 + (long long)item * a.Nreal + colc;
            T* v = a.r1 + (long long)item * a.Nreal + colc;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                u[(long long)(t + TP * e) * a.inner] = ux[e];
                v[(long long)(t + TP * e) * a.inner] = y[e].x;
            }
        }
        return;
    }
    if constexpr (MODE == C2R_APPLY) {
        if (active) {
            if (a.lffp) {
                const long long ib = (long long)item * a.Nreal + colc;
                bool ok = true;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const long long ix = ib + (long long)(t + TP * e) * a.inner;
                    ok &= lffp_point(a.s_prev + ix, a.s_cur + ix, double(acc[e]), sc.kappa0, sc.lambda, a.lf_cb,
                                     a.lf_ca, a.lf_cf);
                }
                if (!ok) a.flag[0] = 1;
            } else {
                T* o = a.r0 + (long long)item * a.Nreal + colc;
#pragma unroll
                for (int e = 0; e < E; ++e) o[(long long)(t + TP * e) * a.inner] = acc[e];
            }
        }
        return;
    }
    if constexpr (MODE == C2R_KICK) {
        if (a.lffp) {  // leap-frog update of (1.1) at this thread's points
            if (active) {
                const long long ib = (long long)item * a.Nreal + colc;
                bool ok = true;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    T f = acc[e];
                    if constexpr (SPLIT) f += cA[e] * S1[e] + cB[e] * S2[e];
                    const long long ix = ib + (long long)(t + TP * e) * a.inner;
                    ok &= lffp_point(a.s_prev + ix, a.s_cur + ix, double(f), -1.0, 0.0, a.lf_cb, a.lf_ca, a.lf_cf);
                }
                if (!ok) a.flag[0] = 1;
            }
            return;  // uniform over the workgroup
        }
    }
    // kick: right-hand side, finiteness flag, forward axis-0 transform, half rows out
    cpx<T> z[E];
    bool bad = false;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        T dv = acc[e];
        if constexpr (SPLIT) dv += cA[e] * S1[e] + cB[e] * S2[e];
        if constexpr (MODE == C2R_KICK_GENERIC) dv += T(sc.lambda) * cB[e] * cB[e] * cB[e];
        bad |= !isfinite(dv);
        z[e] = {dv, T(0)};
    }
    if (bad && active) a.flag[0] = 1;
    fft(z, std::integral_constant<int, -1>{});
    if (active) {
        cpx<T>* dst = a.dv_out + (long long)item * a.istride + colc;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + TP * e;
            if (k <= N / 2) {
                cpx<T> w = z[e];
                if (k == 0 || k == N / 2) w.y = T(0);
                dst[(long long)k * a.rs] = w;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// k_c2r0w: axis-0 kernel with wave-local transforms (apply, kick, generic)
// ---------------------------------------------------------------------------
// The workgroup stages the stored half rows (n0/2+1 rows of W columns) of a
// slot pair into LDS with coalesced loads (each stored row read once), then
// every wavefront transforms WV = 64/TP whole columns: its 16-element-per-
// thread radix-16 FFT exchanges data only inside the wavefront, so the
// transform needs no workgroup barrier. The next pair is loaded into
// registers while the current one is transformed. Outputs are staged
// through LDS and written with coalesced stores.
template <typename T, int N, int E_, int NW_>
struct C2RW {
    static constexpr int E = E_;              // elements per thread
    static constexpr int TP = N / E;          // threads per column
    static constexpr int WV = 64 / TP;        // columns per wavefront
    static constexpr int NW = NW_;            // wavefronts per workgroup
    static constexpr int W = WV * NW;         // columns per workgroup
    static constexpr int HR = N / 2 + 1;      // stored rows
    static constexpr int NT = 64 * NW;
    static constexpr int ST = (HR * W + NT - 1) / NT;  // staged elements per thread per slot
    static constexpr int FPW = N + N / 8 + 16;         // one column's exchange region (padded)
    static constexpr bool ok = (N % E == 0) && (TP <= 64) && (64 % TP == 0) && (TP >= 4) &&
                               (num_stages(N, E) > 0);
};

template <typename T, int N, int E_, int NW_, int MODE>
__global__ __launch_bounds__(64 * NW_) void k_c2r0w(C2RArgs<T> a) {
    using G = C2RW<T, N, E_, NW_>;
    static_assert(G::ok, "shape not supported by the wave-local axis-0 kernel");
    static_assert(MODE == C2R_APPLY || MODE == C2R_KICK || MODE == C2R_KICK_GENERIC, "mode");
    constexpr int E = G::E, TP = G::TP, WV = G::WV, W = G::W, HR = G::HR, NT = G::NT, ST = G::ST;
    __shared__ cpx<T> stg[2 * HR * W];             // two staged half slots
    __shared__ cpx<T> xch[G::NW * WV * G::FPW];     // per-column FFT exchange
    __shared__ cpx<T> tw_s[N];
    stage_twiddles<T, N>(tw_s, a.tw);
    const int wv = threadIdx.x / 64, l = threadIdx.x % 64;
    const int cw = l % WV, t = l / WV;
    const int c = wv * WV + cw;                     // column within the tile
    const int col0 = xcd_group_tile<line_group(W, int(sizeof(cpx<T>)))>(blockIdx.x, gridDim.x) * W;
    const int col = col0 + c;
    const bool active = col < a.inner;
    const int colc = active ? col : 0;
    const int item = blockIdx.y;
    const LdsPencil<T> lds{xch + (wv * WV + cw) * G::FPW};
    const cpx<T>* ibase = a.in + (long long)item * a.istride;
    const int nT = c2r_transforms(MODE, a.M);
    const int nS = c2r_nslots(MODE, a.M);
    const unsigned bytes = unsigned(a.H * (long long)sizeof(cpx<T>));

    // staged element j of this thread: i = threadIdx.x + j*NT -> (row, column)
    unsigned soff[ST];
#pragma unroll
    for (int j = 0; j < ST; ++j) {
        const int i = threadIdx.x + j * NT;
        const int row = (i < HR * W) ? i / W : 0;
        const int cg = col0 + i % W;
        soff[j] = (unsigned(row) * unsigned(a.rs) + unsigned(cg < a.inner ? cg : 0)) *
                  unsigned(sizeof(cpx<T>));
    }
    cpx<T> pf1[ST], pf2[ST];
    auto load_pair = [&](int tr) __attribute__((always_inline)) {
        const int s1 = 2 * tr, s2 = 2 * tr + 1;
        const bool two = s2 < nS;
        const auto r1 = make_rsrc(ibase + (long long)s1 * a.H, bytes);
        const auto r2 = make_rsrc(ibase + (long long)(two ? s2 : s1) * a.H, bytes);
#pragma unroll
        for (int j = 0; j < ST; ++j) {
            pf1[j] = buffer_load_cpx<T>(r1, soff[j]);
            pf2[j] = two ? buffer_load_cpx<T>(r2, soff[j]) : cpx<T>{T(0), T(0)};
        }
    };
    auto commit = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < ST; ++j) {
            const int i = threadIdx.x + j * NT;
            if (i < HR * W) {
                stg[i] = pf1[j];
                stg[HR * W + i] = pf2[j];
            }
        }
    };

    const SolveScalars sc = a.sc[item * a.sc_stride];
    double dl[E];
    {
        const double* dptr = a.delta + (long long)item * a.coef_stride + colc;
#pragma unroll
        for (int e = 0; e < E; ++e) dl[e] = dptr[(long long)(t + TP * e) * a.inner];
    }
    // accumulation in T; delta^m and the coefficients in FP64 (see k_c2r0)
    T acc[E], cA[E], cB[E];
    double dm[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        acc[e] = T(0);
        dm[e] = 1.0;
        cA[e] = T(0);
        cB[e] = T(0);
    }
    if constexpr (MODE == C2R_KICK) {
        const T* Ap = a.A + (long long)item * a.coef_stride + colc;
        const T* Bp = a.B + (long long)item * a.coef_stride + colc;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const long long off = (long long)(t + TP * e) * a.inner;
            cA[e] = -Ap[off];
            cB[e] = -Bp[off];
        }
    }

    cpx<T> y[E];
    load_pair(0);
    for (int tr = 0; tr < nT; ++tr) {
        commit();
        __syncthreads();  // staged pair visible to every wavefront
        const bool two = (2 * tr + 1) < nS;
#pragma unroll
        for (int e = 0; e < E; ++e) y[e] = hermitian_pair<T, N, W>(stg, two ? stg + HR * W : nullptr, c, t + TP * e);
        __syncthreads();  // staging free for the next pair
        if (tr + 1 < nT) load_pair(tr + 1);  // in flight during the transform
        fft_pencil<T, N, E, +1, LdsPencil<T>, true>(y, t, lds, tw_s);
        if constexpr (MODE == C2R_APPLY) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                acc[e] += T(dm[e]) * y[e].x + T(dm[e] * dl[e]) * y[e].y;
                dm[e] *= dl[e] * dl[e];
            }
        } else if constexpr (MODE == C2R_KICK) {
            const double k0c = (tr == 0 && !a.lffp) ? sc.kappa0 : 0.0;
            const double b0c = (tr == 0 && !a.lffp) ? sc.beta0 : 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T ca = T(k0c + double(cA[e]) * dm[e]);
                const T cb = T(b0c + double(cB[e]) * dm[e]);
                acc[e] += ca * y[e].x + cb * y[e].y;
                dm[e] *= dl[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                for (int h = 0; h < 2; ++h) {
                    const int sidx = 2 * tr + h;
                    if (sidx >= nS) break;
                    const T val = h == 0 ? y[e].x : y[e].y;
                    if (sidx == a.M + 1) {
                        cB[e] = val;
                    } else {
                        if (sidx > 0) acc[e] -= T(sc.kappa0 * dm[e]) * val;
                        dm[e] *= dl[e];
                    }
                }
            }
        }
    }

    if constexpr (MODE == C2R_APPLY) {
        // stage the real output (N rows x W columns) and store it coalesced
        T* ost = reinterpret_cast<T*>(stg);
#pragma unroll
        for (int e = 0; e < E; ++e) ost[(t + TP * e) * W + c] = acc[e];
        __syncthreads();
        T* o = a.r0 + (long long)item * a.Nreal;
        bool ok = true;
        for (int i = threadIdx.x; i < N * W; i += NT) {
            const int row = i / W, cg = col0 + i % W;
            if (cg < a.inner) {
                const long long ix = (long long)row * a.inner + cg;
                if (a.lffp) {
                    const long long iz = (long long)item * a.Nreal + ix;
                    ok &= lffp_point(a.s_prev + iz, a.s_cur + iz, double(ost[i]), sc.kappa0, sc.lambda, a.lf_cb,
                                     a.lf_ca, a.lf_cf);
                } else {
                    o[ix] = ost[i];
                }
            }
        }
        if (!ok) a.flag[0] = 1;
        return;
    }
    if constexpr (MODE == C2R_KICK) {
        if (a.lffp) {  // leap-frog update of (1.1) at this thread's points
            if (active) {
                const long long ib = (long long)item * a.Nreal + colc;
                bool ok = true;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const long long ix = ib + (long long)(t + TP * e) * a.inner;
                    ok &= lffp_point(a.s_prev + ix, a.s_cur + ix, double(acc[e]), -1.0, 0.0, a.lf_cb, a.lf_ca,
                                     a.lf_cf);
                }
                if (!ok) a.flag[0] = 1;
            }
            return;  // uniform over the workgroup
        }
    }
    // kick: right-hand side, finiteness flag, forward transform, half rows out
    cpx<T> z[E];
    bool bad = false;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        T dv = acc[e];
        if constexpr (MODE == C2R_KICK_GENERIC) dv += T(sc.lambda) * cB[e] * cB[e] * cB[e];
        bad |= !isfinite(dv);
        z[e] = {dv, T(0)};
    }
    if (bad && active) a.flag[0] = 1;
    fft_pencil<T, N, E, -1, LdsPencil<T>, true>(z, t, lds, tw_s);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + TP * e;
        if (k <= N / 2) {
            cpx<T> w = z[e];
            if (k == 0 || k == N / 2) w.y = T(0);
            stg[k * W + c] = w;
        }
    }
    __syncthreads();
    cpx<T>* dst = a.dv_out + (long long)item * a.istride;
    for (int i = threadIdx.x; i < HR * W; i += NT) {
        const int row = i / W, cg = col0 + i % W;
        if (cg < a.inner) dst[(long long)row * a.rs + cg] = stg[i];
    }
}

// ---------------------------------------------------------------------------
// 1D: one workgroup per field, everything in LDS/registers
// ---------------------------------------------------------------------------
template <typename T>
struct Args1D {
    const T* u_in;          // apply: input fields; step: u
    const T* v_in;
    T* u_out;               // apply: out; step: u
    T* v_out;
    int N;
    const double* mu2;      // axis table
    const cpx<T>* tw;       // twiddles in the working precision
    const cpx<double>* tw64;  // FP64 twiddles for the forward transform of caller data
    const double* delta;    // per point (stride coef_stride per item)
    const T* A;
    const T* B;
    long long coef_stride;
    const SolveScalars* sc;
    int sc_stride;
    int M, op, nsteps, model;
    double dt, invN;
    int* flag;
    double lf_cb, lf_ca, lf_cf;   // leap-frog first-step coefficients (k_1d_lffp)
    double lf_wc, lf_wp;          // (1.1): first-step damping argument w = lf_wc cur + lf_wp prev
    // sub-steps per step (1: TSFP2; 3: the fourth-order composition with
    // sub-step weights w1, w0, w1)
    int sub;
    double w1, w0;
};

// Length of sub-step k of a composed step (weights w1, w0, w1) or dt.
__device__ __forceinline__ double substep_len(double dt, int sub, double w1, double w0, int k) {
    return sub == 3 ? dt * ((k % 3 == 1) ? w0 : w1) : dt;
}

template <typename T, int N, int E>
__global__ __launch_bounds__(N / E) void k_1d_apply(Args1D<T> a) {
    constexpr int TP = N / E;
    __shared__ cpx<double> lds_raw[LdsPencil<double>::footprint(N)];
    const LdsPencil<double> lds64{lds_raw};
    const LdsPencil<T> lds{reinterpret_cast<cpx<T>*>(lds_raw)};
    // twiddles from LDS up to N = 1024; longer 1D transforms read them from
    // global memory (the tables would not fit next to the data)
    constexpr int NTW = (N <= 1024) ? N : 1;
    __shared__ cpx<double> tw64_l[NTW];
    __shared__ cpx<T> tw_l[NTW];
    const cpx<double>* tw64_s = a.tw64;
    const cpx<T>* tw_s = a.tw;
    if constexpr (N <= 1024) {
        stage_twiddles<double, N>(tw64_l, a.tw64);
        stage_twiddles<T, N>(tw_l, a.tw);
        tw64_s = tw64_l;
        tw_s = tw_l;
    }
    const int t = threadIdx.x;
    const int item = blockIdx.x;
    const SolveScalars sc = a.sc[item * a.sc_stride];
    const T* u = a.u_in + (long long)item * N;
    cpx<double> x[E];  // forward transform of the input in FP64
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = {double(u[t + TP * e]), 0.0};
    fft_pencil<double, N, E, -1>(x, t, lds64, tw64_s);
    const double sig = (a.op == 2) ? sc.sig2 : sc.sig1;
    cpx<double> r[E];
    double L[E], dl[E], acc[E], dp[E];
    const double* dd = a.delta + (long long)item * a.coef_stride;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const double m2 = a.mu2[t + TP * e];
        double P = 0.0;
        L[e] = 0.0;
        if (m2 > 0.0) {
            L[e] = log(m2);
            P = exp(sig * L[e]);
        }
        r[e] = {P * double(x[e].x) * a.invN, P * double(x[e].y) * a.invN};
        dl[e] = dd[t + TP * e];
        acc[e] = 0.0;
        dp[e] = 1.0;
    }
    for (int m = 0; m <= a.M; m += 2) {
        const bool pair = (m + 1 <= a.M);
        cpx<T> y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const cpx<double> x0 = r[e];
            const double f = L[e] / double(m + 1);
            const cpx<double> x1 = pair ? cpx<double>{x0.x * f, x0.y * f} : cpx<double>{0.0, 0.0};
            y[e] = {T(x0.x - x1.y), T(x0.y + x1.x)};
            const double g = pair ? L[e] / double(m + 2) : 0.0;
            r[e] = {x1.x * g, x1.y * g};
        }
        fft_pencil<T, N, E, +1>(y, t, lds, tw_s);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            acc[e] += dp[e] * (double(y[e].x) + dl[e] * double(y[e].y));
            dp[e] *= dl[e] * dl[e];
        }
    }
    T* o = a.u_out + (long long)item * N;
#pragma unroll
    for (int e = 0; e < E; ++e) o[t + TP * e] = T(acc[e]);
}

// Symbols of one mode: ln|mu|^2 and |mu|^{2 sig1}, |mu|^{2 sig2} (zero at k = 0).
__device__ __forceinline__ void mode_symbols(double m2, double sig1, double sig2, double& L,
                                             double& P1, double& P2) {
    L = 0.0;
    P1 = 0.0;
    P2 = 0.0;
    if (m2 > 0.0) {
        L = log(m2);
        P1 = exp(sig1 * L);
        P2 = exp(sig2 * L);
    }
}

template <typename T, int N, int E>
__global__ __launch_bounds__(N / E) void k_1d_step(Args1D<T> a) {
    constexpr int TP = N / E;
    __shared__ cpx<double> lds_raw[LdsPencil<double>::footprint(N)];
    const LdsPencil<double> lds64{lds_raw};
    const LdsPencil<T> lds{reinterpret_cast<cpx<T>*>(lds_raw)};
    // twiddles from LDS up to N = 1024; longer 1D transforms read them from
    // global memory (the tables would not fit next to the data)
    constexpr int NTW = (N <= 1024) ? N : 1;
    __shared__ cpx<double> tw64_l[NTW];
    __shared__ cpx<T> tw_l[NTW];
    const cpx<double>* tw64_s = a.tw64;
    const cpx<T>* tw_s = a.tw;
    if constexpr (N <= 1024) {
        stage_twiddles<double, N>(tw64_l, a.tw64);
        stage_twiddles<T, N>(tw_l, a.tw);
        tw64_s = tw64_l;
        tw_s = tw_l;
    }
    const int t = threadIdx.x;
    const int item = blockIdx.x;
    const SolveScalars sc = a.sc[item * a.sc_stride];
    const long long co = (long long)item * a.coef_stride;
    cpx<double> uh[E], vh[E];
    {
        cpx<double> x[E];  // forward transforms of the caller's (u, v) in FP64
        const T* u = a.u_in + (long long)item * N;
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = {double(u[t + TP * e]), 0.0};
        fft_pencil<double, N, E, -1>(x, t, lds64, tw64_s);
#pragma unroll
        for (int e = 0; e < E; ++e) uh[e] = {x[e].x * a.invN, x[e].y * a.invN};
        const T* v = a.v_in + (long long)item * N;
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = {double(v[t + TP * e]), 0.0};
        fft_pencil<double, N, E, -1>(x, t, lds64, tw64_s);
#pragma unroll
        for (int e = 0; e < E; ++e) vh[e] = {x[e].x * a.invN, x[e].y * a.invN};
    }
    auto propagate = [&](double tp) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            double L, P1, P2, g11, g12, g21, g22;
            mode_symbols(a.mu2[t + TP * e], sc.sig1, sc.sig2, L, P1, P2);
            damped_flow(P1, P2, sc.kappa0, sc.beta0, tp, g11, g12, g21, g22);
            const cpx<double> u0 = uh[e], v0 = vh[e];
            uh[e] = {g11 * u0.x + g12 * v0.x, g11 * u0.y + g12 * v0.y};
            vh[e] = {g21 * u0.x + g22 * v0.x, g21 * u0.y + g22 * v0.y};
        }
    };
    bool bad = false;
    const int K = a.nsteps * a.sub;  // sub-steps
    if (K > 0) propagate(0.5 * substep_len(a.dt, a.sub, a.w1, a.w0, 0));
    for (int s = 0; s < K; ++s) {
        const double ds = substep_len(a.dt, a.sub, a.w1, a.w0, s);
        double acc[E];
        if (a.model == MODEL_GENERIC) {
            // dv = -kappa sum_{s=1..M} delta^s t_s + lambda u^3, with t_s from
            // l_s |mu|^{2 s0} u_hat (s <= M) and u from u_hat (s = M+1), two per transform
            double uu[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                acc[e] = 0.0;
                uu[e] = 0.0;
            }
            const int ns = a.M + 2;
            for (int s0 = 0; s0 < ns; s0 += 2) {
                cpx<T> y[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    double L, P1, P2;
                    mode_symbols(a.mu2[t + TP * e], sc.sig1, sc.sig2, L, P1, P2);
                    cpx<double> xs[2];
                    for (int h = 0; h < 2; ++h) {
                        const int sidx = s0 + h;
                        double c = 0.0;
                        if (sidx <= a.M) {
                            c = P1;
                            for (int j = 1; j <= sidx; ++j) c *= L / double(j);
                        } else if (sidx == a.M + 1) {
                            c = 1.0;
                        }
                        xs[h] = {c * uh[e].x, c * uh[e].y};
                    }
                    y[e] = {T(xs[0].x - xs[1].y), T(xs[0].y + xs[1].x)};
                }
                fft_pencil<T, N, E, +1>(y, t, lds, tw_s);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int k = t + TP * e;
                    const double d = a.delta[co + k];
                    for (int h = 0; h < 2; ++h) {
                        const int sidx = s0 + h;
                        const double val = h == 0 ? double(y[e].x) : double(y[e].y);
                        if (sidx == a.M + 1) {
                            uu[e] = val;
                        } else if (sidx > 0 && sidx <= a.M) {
                            double dm = 1.0;
                            for (int j = 0; j < sidx; ++j) dm *= d;
                            acc[e] -= sc.kappa0 * dm * val;
                        }
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] += sc.lambda * uu[e] * uu[e] * uu[e];
        } else {
            // kick: dv = (kappa0 - A) t1_0 + (beta0 - B) t2_0 + sum_{m>=1} delta^m (-A t1_m - B t2_m)
            cpx<T> y[E];
            {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    double L, P1, P2;
                    mode_symbols(a.mu2[t + TP * e], sc.sig1, sc.sig2, L, P1, P2);
                    // m = 0 pair: |mu|^{2 sig1} u_hat + i |mu|^{2 sig2} v_hat
                    y[e] = {T(P1 * uh[e].x - P2 * vh[e].y), T(P1 * uh[e].y + P2 * vh[e].x)};
                    acc[e] = 0.0;
                }
            }
            double lm = 1.0;  // running 1/m! for the multipliers
            for (int m = 0; m <= a.M; ++m) {
                fft_pencil<T, N, E, +1>(y, t, lds, tw_s);
                const double k0c = (m == 0) ? sc.kappa0 : 0.0;
                const double b0c = (m == 0) ? sc.beta0 : 0.0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int k = t + TP * e;
                    const double d = a.delta[co + k];
                    double dm = 1.0;
                    for (int j = 0; j < m; ++j) dm *= d;
                    const double ca = -double(a.A[co + k]) * dm;
                    const double cb = -double(a.B[co + k]) * dm;
                    acc[e] += (k0c + ca) * double(y[e].x) + (b0c + cb) * double(y[e].y);
                }
                if (m < a.M) {
                    lm /= double(m + 1);
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        double L, P1, P2;
                        mode_symbols(a.mu2[t + TP * e], sc.sig1, sc.sig2, L, P1, P2);
                        double lp = lm;
                        for (int j = 0; j <= m; ++j) lp *= L;
                        const double c1 = lp * P1, c2 = lp * P2;
                        y[e] = {T(c1 * uh[e].x - c2 * vh[e].y), T(c1 * uh[e].y + c2 * vh[e].x)};
                    }
                }
            }
        }
        cpx<T> z[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            bad |= !isfinite(acc[e]);
            z[e] = {T(acc[e]), T(0)};
        }
        fft_pencil<T, N, E, -1>(z, t, lds, tw_s);
        const double sc2 = ds * a.invN;
#pragma unroll
        for (int e = 0; e < E; ++e) vh[e] = {vh[e].x + sc2 * double(z[e].x), vh[e].y + sc2 * double(z[e].y)};
        propagate(s + 1 < K ? 0.5 * (ds + substep_len(a.dt, a.sub, a.w1, a.w0, s + 1)) : 0.5 * ds);
    }
    if (bad) a.flag[0] = 1;
    // u and v transformed one at a time (v can be far smaller than u)
    T* uo = a.u_out + (long long)item * N;
    T* vo = a.v_out + (long long)item * N;
    for (int f = 0; f < 2; ++f) {
        cpx<T> y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) y[e] = from_d<T>(f == 0 ? uh[e] : vh[e]);
        fft_pencil<T, N, E, +1>(y, t, lds, tw_s);
        T* o = f == 0 ? uo : vo;
#pragma unroll
        for (int e = 0; e < E; ++e) o[t + TP * e] = y[e].x;
    }
}

// ---------------------------------------------------------------------------
// element-wise precision conversion (leap-frog state in and out)
// ---------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_convert(const TI* __restrict__ in, TO* __restrict__ out, long long n) {
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256LL)
        out[i] = TO(in[i]);
}

// ---------------------------------------------------------------------------
// 1D leap-frog (3.4): one workgroup per field, the state in FP64 registers
// for all nsteps steps; (u_in, v_in) = (cur, prev) in, (u_out, v_out) =
// (cur, prev) out (may alias the inputs: every value is read before any is
// written, by the thread that owns it). Generic model: kappa0 = kappa.
// Seismic model (1.1): new = cb cur + ca prev + cf (-A L1 cur - B L2 w) with
// w = (cur - prev)/dt (first step: lf_wc cur + lf_wp prev).
// ---------------------------------------------------------------------------
template <typename T, int N, int E>
__global__ __launch_bounds__(N / E) void k_1d_lffp(Args1D<T> a) {
    constexpr int TP = N / E;
    __shared__ cpx<double> lds_raw[LdsPencil<double>::footprint(N)];
    const LdsPencil<double> lds64{lds_raw};
    const LdsPencil<T> lds{reinterpret_cast<cpx<T>*>(lds_raw)};
    constexpr int NTW = (N <= 1024) ? N : 1;
    __shared__ cpx<double> tw64_l[NTW];
    __shared__ cpx<T> tw_l[NTW];
    const cpx<double>* tw64_s = a.tw64;
    const cpx<T>* tw_s = a.tw;
    if constexpr (N <= 1024) {
        stage_twiddles<double, N>(tw64_l, a.tw64);
        stage_twiddles<T, N>(tw_l, a.tw);
        tw64_s = tw64_l;
        tw_s = tw_l;
    }
    // long transforms keep ln|mu|^2 and |mu|^{2 s0} of their points in LDS
    // (registers would spill), shorter ones in registers
    constexpr bool LP_LDS = N > 1024;
    __shared__ double lp_s[LP_LDS ? 2 * N : 1];
    const int t = threadIdx.x;
    const int item = blockIdx.x;
    const SolveScalars sc = a.sc[item * a.sc_stride];
    double cur[E], prev[E], Lr[LP_LDS ? 1 : E], Pr[LP_LDS ? 1 : E], dl[E];
    auto Lv = [&](int e) __attribute__((always_inline)) -> double {
        if constexpr (LP_LDS) return lp_s[t + TP * e];
        else return Lr[e];
    };
    auto Pv = [&](int e) __attribute__((always_inline)) -> double {
        if constexpr (LP_LDS) return lp_s[N + t + TP * e];
        else return Pr[e];
    };
    const double* dd = a.delta + (long long)item * a.coef_stride;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = t + TP * e;
        cur[e] = double(a.u_in[(long long)item * N + j]);
        prev[e] = double(a.v_in[(long long)item * N + j]);
        const double m2 = a.mu2[j];
        double Le = 0.0, Pe = 0.0;
        if (m2 > 0.0) {
            Le = log(m2);
            Pe = exp(sc.sig1 * Le);
        }
        if constexpr (LP_LDS) {
            lp_s[j] = Le;   // read back only by this thread
            lp_s[N + j] = Pe;
        } else {
            Lr[e] = Le;
            Pr[e] = Pe;
        }
        dl[e] = dd[j];
    }
    const bool seismic = a.model == MODEL_SEISMIC;
    double Ar[E], Br[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const long long j = (long long)item * a.coef_stride + t + TP * e;
        Ar[e] = double(a.A[j]);
        Br[e] = double(a.B[j]);
    }
    bool ok = true;
    for (int step = 0; step < a.nsteps; ++step) {
        const double cb = step == 0 ? a.lf_cb : 2.0, ca = step == 0 ? a.lf_ca : -1.0;
        const double cf = step == 0 ? a.lf_cf : a.dt * a.dt;
        if (seismic) {
            // L1 cur and L2 w: both forward transforms in FP64, then one
            // complex inverse transform per term carrying the pair (t1_m, t2_m)
            const double wc = step == 0 ? a.lf_wc : 1.0 / a.dt;
            const double wp = step == 0 ? a.lf_wp : -1.0 / a.dt;
            cpx<double> x1[E], x2[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                x1[e] = {cur[e], 0.0};
                x2[e] = {wc * cur[e] + wp * prev[e], 0.0};
            }
            fft_pencil<double, N, E, -1>(x1, t, lds64, tw64_s);
            fft_pencil<double, N, E, -1>(x2, t, lds64, tw64_s);
            double acc1[E], acc2[E], dp[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double P1 = Pv(e);
                const double P2 = P1 > 0.0 ? exp(sc.sig2 * Lv(e)) : 0.0;  // zero at k = 0 like P1
                x1[e] = {P1 * x1[e].x * a.invN, P1 * x1[e].y * a.invN};
                x2[e] = {P2 * x2[e].x * a.invN, P2 * x2[e].y * a.invN};
                acc1[e] = 0.0;
                acc2[e] = 0.0;
                dp[e] = 1.0;
            }
            for (int m = 0; m <= a.M; ++m) {
                cpx<T> y[E];
#pragma unroll
                for (int e = 0; e < E; ++e) y[e] = {T(x1[e].x - x2[e].y), T(x1[e].y + x2[e].x)};
                fft_pencil<T, N, E, +1>(y, t, lds, tw_s);
                const double inv = 1.0 / double(m + 1);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    acc1[e] += dp[e] * double(y[e].x);
                    acc2[e] += dp[e] * double(y[e].y);
                    dp[e] *= dl[e];
                    const double f = Lv(e) * inv;
                    x1[e] = {x1[e].x * f, x1[e].y * f};
                    x2[e] = {x2[e].x * f, x2[e].y * f};
                }
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const double u = cur[e];
                const double nw = cb * u + ca * prev[e] + cf * (-Ar[e] * acc1[e] - Br[e] * acc2[e]);
                ok &= isfinite(nw);
                prev[e] = u;
                cur[e] = nw;
            }
            continue;
        }
        cpx<double> x[E];
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = {cur[e], 0.0};
        fft_pencil<double, N, E, -1>(x, t, lds64, tw64_s);
        cpx<double> r[E];
        double acc[E], dp[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            r[e] = {Pv(e) * x[e].x * a.invN, Pv(e) * x[e].y * a.invN};
            acc[e] = 0.0;
            dp[e] = 1.0;
        }
        for (int m = 0; m <= a.M; m += 2) {
            const bool pair = (m + 1 <= a.M);
            cpx<T> y[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const cpx<double> x0 = r[e];
                const double f = Lv(e) / double(m + 1);
                const cpx<double> x1 = pair ? cpx<double>{x0.x * f, x0.y * f} : cpx<double>{0.0, 0.0};
                y[e] = {T(x0.x - x1.y), T(x0.y + x1.x)};
                const double g = pair ? Lv(e) / double(m + 2) : 0.0;
                r[e] = {x1.x * g, x1.y * g};
            }
            fft_pencil<T, N, E, +1>(y, t, lds, tw_s);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                acc[e] += dp[e] * (double(y[e].x) + dl[e] * double(y[e].y));
                dp[e] *= dl[e] * dl[e];
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const double u = cur[e];
            const double nw = cb * u + ca * prev[e] + cf * (-sc.kappa0 * acc[e] + sc.lambda * u * u * u);
            ok &= isfinite(nw);
            prev[e] = u;
            cur[e] = nw;
        }
    }
    if (!ok) a.flag[0] = 1;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = t + TP * e;
        a.u_out[(long long)item * N + j] = T(cur[e]);
        a.v_out[(long long)item * N + j] = T(prev[e]);
    }
}

// ---------------------------------------------------------------------------
// vector kernels of the Crank-Nicolson solver (plan precision vectors,
// FP64 arithmetic and FP64 dot products)
// ---------------------------------------------------------------------------
// out = c0 x0 + c1 x1 + c2 x2 + cq xq^3 (a null input is skipped; out may
// alias an input: each element is read before it is written by its thread)
template <typename T>
__global__ __launch_bounds__(256) void k_lincomb(T* out, const T* x0, double c0, const T* x1, double c1,
                                                 const T* x2, double c2, const T* xq, double cq, long long n) {
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256LL) {
        double r = 0.0;
        if (x0) r += c0 * double(x0[i]);
        if (x1) r += c1 * double(x1[i]);
        if (x2) r += c2 * double(x2[i]);
        if (xq) {
            const double q = double(xq[i]);
            r += cq * q * q * q;
        }
        out[i] = T(r);
    }
}

// Partial sums of a0.b0 and a1.b1 (a1 may be null): one pair per workgroup,
// over a fixed grid, so the summation order does not depend on timing.
template <typename T>
__global__ __launch_bounds__(256) void k_dot2(const T* a0, const T* b0, const T* a1, const T* b1, long long n,
                                              double* partial) {
    __shared__ double red[2][256];
    double s0 = 0.0, s1 = 0.0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256LL) {
        s0 += double(a0[i]) * double(b0[i]);
        if (a1) s1 += double(a1[i]) * double(b1[i]);
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = red[0][0];
        partial[2 * blockIdx.x + 1] = red[1][0];
    }
}

// out[0..1] = sums of the nb partial pairs (one workgroup)
template <typename T>
__global__ __launch_bounds__(256) void k_dot2_finish(const double* partial, int nb, double* out) {
    __shared__ double red[2][256];
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        s0 += partial[2 * b];
        s1 += partial[2 * b + 1];
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

}  // namespace vofl
