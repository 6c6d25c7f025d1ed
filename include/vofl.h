/*
 * vofl.h -- C ABI of libvofl: the matrix-free variable-order fractional
 * Laplacian and the second-order time-splitting Fourier pseudospectral
 * (TSFP2) wave solver of Zhang, Zhao and Zhou, "Fourier pseudospectral methods
 * for the variable-order space fractional wave equations" (arXiv 2311.13049),
 * on AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 1, eq. (1.1); Section 2 for the grid):
 *   (1/c^2) u_tt = eta (-Lap)^{1+gamma(x)} u + tau d/dt[(-Lap)^{1/2+gamma(x)} u]
 * on a periodic box [lo, hi) with n[i] points per axis (n even), with
 *   c = c0 cos(pi gamma/2), eta = -c0^{2 gamma} omega0^{-2 gamma} cos(pi gamma),
 *   tau = -c0^{2 gamma - 1} omega0^{-2 gamma} sin(pi gamma), gamma = atan(1/Q)/pi.
 * Written as u_t = v, v_t = -A(x) L1 u - B(x) L2 v with A = -c^2 eta,
 * B = -c^2 tau, L1 = (-Lap)^{1+gamma(x)}, L2 = (-Lap)^{1/2+gamma(x)}.
 *
 * The generic model (1.5), u_tt = -kappa (-Lap)^{s(x)} u + lambda u^3, is
 * selected with model = VOFL_MODEL_GENERIC (then s replaces gamma/Q and
 * L1 = (-Lap)^{s(x)}).
 *
 * Discrete operator (eq. (2.13)): with s0 the grid mean of s,
 * delta = s - s0, l_m(k) = (ln|mu_k|^2)^m / m!,
 *   (L u)_j = sum_{m=0..M} delta_j^m  IDFT[ l_m |mu|^{2 s0} u_hat ]_j ,
 * u_hat = DFT(u)/N, mu_k = 2 pi k / L per axis, the k = 0 term omitted.
 *
 * Arrays are real, C-ordered (last index fastest), in the plan's precision
 * (double for VOFL_FP64, float for VOFL_FP32). Device pointers are HIP device
 * memory owned by the caller (for example torch tensors); host pointers are
 * read during vofl_plan only. Every call returns VOFL_OK (0) or a negative
 * status; vofl_last_error() returns the message of the calling thread's last
 * failure. No call allocates device memory after vofl_plan.
 */
#ifndef VOFL_H
#define VOFL_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define VOFL_OK              0
#define VOFL_ERR_INVALID    -1  /* argument outside the documented domain           */
#define VOFL_ERR_NOMEM      -2  /* device allocation failed or hbm_budget exceeded   */
#define VOFL_ERR_DEVICE     -3  /* HIP runtime error (no device, launch failure)     */
#define VOFL_ERR_UNSTABLE   -4  /* a non-finite value appeared (time step too large,
                                   see the stability condition (3.5))               */
#define VOFL_ERR_UNSUPPORTED -5 /* grid size without a compiled FFT length, or a
                                   scheme not provided for the plan's model          */

/* precision of the transforms and pointwise work; the expansion coefficients,
   the spectral multipliers, the propagator and the spectral state are FP64 in
   both */
#define VOFL_FP64 0
#define VOFL_FP32 1

/* models */
#define VOFL_MODEL_SEISMIC 0   /* eq. (1.1), gamma(x) from Q(x) or given      */
#define VOFL_MODEL_GENERIC 1   /* eq. (1.5), s(x) given, f(u) = lambda u^3      */

/* operators for vofl_apply */
#define VOFL_OP_S1 1   /* (-Lap)^{1+gamma(x)} (seismic) or (-Lap)^{s(x)} (generic) */
#define VOFL_OP_S2 2   /* (-Lap)^{1/2+gamma(x)} (seismic model only)                */

typedef struct vofl_desc {
    int ndim;            /* 1, 2 or 3                                                  */
    int n[3];            /* points per axis, even, first ndim entries used             */
    double lo[3], hi[3]; /* periodic box [lo, hi) per axis, hi > lo                    */
    int model;           /* VOFL_MODEL_SEISMIC or VOFL_MODEL_GENERIC                   */
    double c0, omega0;   /* seismic: phase velocity and reference frequency, > 0       */
    const double* Q;     /* seismic: host, N values, Q > 0 (+inf gives gamma = 0), or NULL */
    const double* gamma; /* seismic: host, N values in [0, 1/2), or NULL; exactly one of Q, gamma */
    const double* s;     /* generic: host, N values in (0, 2)                           */
    double kappa;        /* generic: kappa > 0                                          */
    double lambda;       /* generic: coefficient of the cubic term f(u) = lambda u^3    */
    int M;               /* upper index of the expansion (M+1 terms), 0 <= M <= 64     */
    double dt;           /* time step > 0                                              */
    int precision;       /* VOFL_FP64 or VOFL_FP32                                     */
    int max_batch;       /* largest nfields accepted by vofl_apply (>= 1; 0 means 1)   */
    int batch;           /* independent solves advanced together by vofl_step (0 means 1);
                            u and v then hold batch * N values, solve after solve      */
    int coef_per_solve;  /* 0: one coefficient field (Q, gamma or s: N values) shared by
                            all solves; 1: batch fields (batch * N values), one per solve */
    size_t hbm_budget;   /* bytes of device memory the plan may take; 0 = no limit     */
    int tune_steps;      /* 0: default kernel variants; > 0: vofl_plan times each
                            candidate over this many steps on temporary buffers and
                            keeps the fastest: the axis-0 kernel variants x the
                            middle-axis tile widths, then the last-axis radix
                            schedule (4 or 8 elements per thread for power-of-two
                            lengths 64..1024) with the best pair (cached in the
                            file named by VOFL_TUNE_CACHE, when set)                 */
    int order;           /* time splitting of vofl_step: 0 or 2: TSFP2 (3.13); 4: the
                            higher-order splitting named after (3.13), built as the
                            symmetric composition of three TSFP2 steps of lengths
                            w1 dt, w0 dt, w1 dt (w1 = 1/(2 - 2^{1/3}), w0 = 1 - 2 w1);
                            generic model only (its kick is exact), else
                            VOFL_ERR_UNSUPPORTED                                       */
    const double* c0_field; /* seismic: host, per-point phase velocity c0(x) > 0 (N values,
                            or batch * N with coef_per_solve = 1) for layered media, as
                            in Example 3 (Section 4); A(x), B(x) then use c0(x), the
                            exact part of vofl_step uses the grid mean of c0(x), and
                            the scalar c0 is ignored. NULL: c0 everywhere             */
} vofl_desc;

typedef struct vofl_plan_s* vofl_plan_t;

/* Build a plan (Section 2.3 grid and symbol, eq. (2.13) expansion,
 * eqs. (3.10)-(3.11) propagator): validates the descriptor on the host,
 * computes gamma = atan(1/Q)/pi, the grid means, delta, A(x), B(x) in FP64,
 * uploads the per-axis tables and allocates all device workspace.
 * stream: HIP stream (hipStream_t) used for the uploads; may be NULL.
 * On success *out owns all device memory of the plan. Errors:
 * VOFL_ERR_INVALID (bad descriptor), VOFL_ERR_UNSUPPORTED (no FFT length),
 * VOFL_ERR_NOMEM (allocation failed or footprint above hbm_budget),
 * VOFL_ERR_DEVICE (no HIP device). The descriptor and host arrays are not
 * retained. The environment variables VOFL_C2R_VARIANT (axis-0 kernel: 0, 2,
 * 5, 6, 11, 12, 13, 14) and VOFL_MID_VARIANT (middle-axis tile: 0, 1, 2)
 * force a kernel variant instead of the default (a variant without a kernel
 * for the plan's length runs as variant 0) and VOFL_CONTIG_VARIANT (last-axis
 * radix schedule: 0, 1); results agree to rounding. The plan keeps its half
 * spectra (2D/3D) with rows along axis 0 padded by 128 bytes when a row spans
 * 4 KiB or more; VOFL_HALF_ROW_PAD (complex elements, 0 = none) sets the
 * padding instead (results are the same; the layout is internal). */
int vofl_plan(const vofl_desc* desc, void* stream, vofl_plan_t* out);

/* Device bytes a plan for desc would allocate (same validation as vofl_plan,
 * no device access). Returns VOFL_OK and writes *bytes, or an error code. */
int vofl_plan_footprint(const vofl_desc* desc, size_t* bytes);

/* Apply the M-term operator (2.13) to nfields real fields (the proposal of
 * one field per call is widened to nfields so that the L1 u / L2 v pair of a
 * step, or a batch of fields, shares the launches):
 * out_f = (L_op u_f) for f < nfields, with op VOFL_OP_S1 or VOFL_OP_S2.
 * u, out: device, nfields * N values each, plan precision, out != u,
 * no overlap. Asynchronous on stream. 1 <= nfields <= max_batch; with
 * coef_per_solve = 1, field f uses solve f's coefficients (nfields <= batch). */
int vofl_apply(vofl_plan_t plan, int op, const void* u, void* out, int nfields,
               void* stream);

/* Advance (u, v = u_t) by nsteps TSFP2 steps (eqs. (3.13)-(3.14); for (1.1)
 * the exact part is the damped oscillator of the mean orders and the kick
 * carries the variable-order remainder). u, v: device, batch * N values
 * each, overwritten in place. nsteps >= 0. Asynchronous on stream; a
 * non-finite value sets the plan's device flag, reported as
 * VOFL_ERR_UNSTABLE by the next vofl_sync_status (and by later vofl_step
 * calls after a sync).
 * Order in dt: second for the generic model (1.5) (the kick is exact in
 * time there), and for (1.1) when gamma is constant (the remainder is then
 * zero and the step is exact in time). For (1.1) with a non-constant gamma
 * the kick holds v at its half-step value inside the variable damping term
 * -(B(x) L2 - beta0 |mu|^{2(1/2+gbar)}) v, so the split is first order in
 * dt; for the same reason order = 4 is refused for the seismic model.
 * Every call on a plan (vofl_apply, vofl_step*, vofl_lffp_*, vofl_cnfp_step)
 * uses the plan's work slots and spectral blocks: calls on one plan must be
 * issued on one stream, or ordered with events; two streams using one plan
 * at once race. */
int vofl_step(vofl_plan_t plan, void* u, void* v, int nsteps, void* stream);

/* Resumable TSFP2 run (eqs. (3.13)-(3.14)) with the spectral state kept in
 * the plan between calls, for callers that advance a solve in chunks
 * (request servers, graph replays) or read the wavefield while stepping.
 *
 * vofl_step_begin: imports (u, v) (device, batch * N values each, plan
 * precision; read only) into the plan's FP64 spectral state at t_0.
 * vofl_step_advance: nsteps >= 0 TSFP2 steps of the run. It touches no
 * caller memory, so its launches depend on nsteps alone; use_graph != 0
 * replays a HIP graph captured once per nsteps (up to 8 kept per plan; no
 * device memory allocated by the library). The state is carried between
 * calls in FP64 exactly as vofl_step carries it between steps, so a run of
 * n steps split into any advance calls equals vofl_step's n steps bit for
 * bit (2D/3D; in 1D each advance is a vofl_step on the run's own copy of
 * (u, v), which matches a single vofl_step to rounding).
 * vofl_step_end: writes the run's current (u, v) (device, batch * N values
 * each, u != v) and leaves the run open: advance may continue afterwards.
 * Each call costs the steps it advances: no re-import per call (one extra
 * last-axis pass at the start of each advance and a light one at its end,
 * in place of vofl_step's merged half steps).
 * A run ends when any other call (vofl_apply, vofl_step, vofl_step_graph,
 * vofl_lffp_*, vofl_cnfp_step, vofl_step_batch) uses the plan; advance and
 * end then fail with VOFL_ERR_INVALID until the next begin. All three are
 * asynchronous on stream; calls on one plan must be issued on one stream or
 * ordered with events (they share the plan's buffers). */
int vofl_step_begin(vofl_plan_t plan, const void* u, const void* v, void* stream);
int vofl_step_advance(vofl_plan_t plan, int nsteps, int use_graph, void* stream);
int vofl_step_end(vofl_plan_t plan, void* u, void* v, void* stream);

/* u = u0, v = v0, then nsteps steps as vofl_step. u0/v0 may equal u/v. */
int vofl_solve(vofl_plan_t plan, const void* u0, const void* v0, int nsteps,
               void* u, void* v, void* stream);

/* Leap-frog Fourier pseudospectral scheme LFFP (eq. (3.4)).
 * Generic model (1.5): u^{n+1} = 2 u^n - u^{n-1} + dt^2 F(u^n) with
 * F(u) = -kappa L u + lambda u^3, L the M-term operator (2.13) of s(x).
 * Seismic model (1.1), the scheme of Example 3 (Section 4): with
 * w^n = (u^n - u^{n-1})/dt standing for u_t in the damping term,
 * u^{n+1} = 2 u^n - u^{n-1} + dt^2 (-A L1 u^n - B L2 w^n), L1, L2 the M-term
 * operators of orders 1+gamma(x), 1/2+gamma(x) (first order in dt through
 * the damping term, second order when gamma = 0).
 *
 * vofl_lffp_start: the start (3.4b, c): u_prev = phi and
 * u = phi + dt psi + dt^2/2 F(phi) (seismic: F(phi) = -A L1 phi - B L2 psi).
 * vofl_lffp_step: nsteps >= 0 steps on (u_prev, u) = (u^{n-1}, u^n), in
 * place; on return they hold (u^{n+nsteps-1}, u^{n+nsteps}).
 * All fields: device, batch * N values each, plan precision; u_prev != u
 * (the inputs of vofl_lffp_start may alias the outputs). Within one call the
 * state is carried in FP64 (in registers in 1D, in plan memory in 2D/3D).
 * Asynchronous on stream; a non-finite value sets the device flag reported by
 * vofl_sync_status. */
int vofl_lffp_start(vofl_plan_t plan, const void* phi, const void* psi, void* u_prev, void* u,
                    void* stream);
int vofl_lffp_step(vofl_plan_t plan, void* u_prev, void* u, int nsteps, void* stream);

/* Crank-Nicolson Fourier pseudospectral scheme CNFP (eq. (3.2)) for the
 * generic model (1.5): per step u^{n+1} = w solves
 *   w + a L w - b lambda w^3 = 2 u^n - u^{n-1} - a L u^{n-1} + b lambda (u^{n-1})^3,
 * a = kappa dt^2/2, b = dt^2/2, L = (2.13). The nonlinear term is handled by
 * fixed-point iteration and every linear solve with I + a L by BiCGSTAB
 * (the operator is not symmetric), each to the relative tolerance tol in
 * (0, 1), at most max_iter (>= 1) iterations per solve. The start (3.3) is
 * the leap-frog start: use vofl_lffp_start. u_prev, u: as vofl_lffp_step.
 * The solves of a batched plan are advanced one after another, each with
 * its own coefficients (the solver's vectors hold one solve).
 * *iterations (host, may be NULL) receives the total BiCGSTAB iterations
 * over all solves. The call synchronises stream (the iteration reads its
 * scalars back). Errors: VOFL_ERR_UNSUPPORTED (seismic model),
 * VOFL_ERR_UNSTABLE (a solve did not reach tol). */
int vofl_cnfp_step(vofl_plan_t plan, void* u_prev, void* u, int nsteps, double tol, int max_iter,
                   long long* iterations, void* stream);

/* vofl_step replayed from a HIP graph (for callers that step the same
 * buffers repeatedly). The first call with a given (u, v, nsteps) captures
 * vofl_step's launch sequence on an internal stream into a graph and
 * instantiates it; every call then launches the graph on stream. The
 * library allocates no device memory here (the HIP runtime keeps the
 * instantiated graph). Up to 8 graphs are kept per plan. Results equal
 * vofl_step's bit for bit. */
int vofl_step_graph(vofl_plan_t plan, void* u, void* v, int nsteps, void* stream);

/* Advance several independent solves, one plan each, by nsteps[i] steps,
 * each plan on an internal stream forked from (and joined back into)
 * stream, so the device overlaps their work. Plans may differ in grid, M
 * and precision. Each solve's result equals what vofl_step gives for it
 * alone, bit for bit. */
int vofl_step_batch(vofl_plan_t* plans, void** u, void** v, const int* nsteps,
                    int count, void* stream);

/* Allocation-free apply, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops that forbid allocation; no
 * plan is needed). Computes the M-term operator (2.13) of order s(x) on a 1D
 * periodic grid of n points on [lo, hi) for nfields fields, as vofl_apply
 * does for a plan of that grid, order field and M:
 *   out_f = sum_{m=0..M} delta^m IDFT[l_m |mu|^{2 s0} DFT(u_f)/N],
 * s0 the grid mean of s, delta = s - s0 (for (1.1) pass s = 1 + gamma or
 * 1/2 + gamma). s: device, n FP64 values in (0, 2]; u, out: device,
 * nfields * n values in the given precision, out != u. n must be a compiled
 * 1D length (8 ... 4096) whose tables fit the library's 256 KiB static
 * scratch array (every compiled length does), else VOFL_ERR_UNSUPPORTED or
 * VOFL_ERR_INVALID. The call allocates nothing: the grid mean, delta, the
 * symbol and twiddle tables are formed on the device in the static array
 * (one per GPU, kept until the process ends, reused by every call), so
 * calls that overlap on one GPU race; order them on one stream.
 * Asynchronous on stream. */
int vofl_apply_noalloc(int n, double lo, double hi, const double* s, int M, int precision,
                       const void* u, void* out, int nfields, void* stream);

/* Measurement support (computes nothing of the method): stream `bytes`
 * through HBM as a plain read (kind VOFL_PROBE_READ: src is read, dst holds
 * one float per workgroup that is written only for one improbable sum),
 * a plain write (VOFL_PROBE_WRITE: dst is filled with vector i holding
 * (i mod 1024) + 0, 1, 2, 3; src unused) or a one-to-one copy
 * (VOFL_PROBE_COPY: src to dst), with 16 bytes per lane per access,
 * `blocks` workgroups of 256 threads striding over the buffer, 4 accesses in
 * flight per lane (16 with VOFL_PROBE_DEEP in flags) and non-temporal loads
 * and stores with VOFL_PROBE_NONTEMPORAL. Device pointers, 16-byte aligned;
 * bytes a positive multiple of 16; blocks in 1..2^20; src and dst must not
 * overlap. Used to measure the read, write and copy rates that each pass's
 * own read/write mix is set against. Asynchronous on stream;
 * VOFL_ERR_INVALID for arguments outside these ranges. */
#define VOFL_PROBE_READ  0
#define VOFL_PROBE_WRITE 1
#define VOFL_PROBE_COPY  2
#define VOFL_PROBE_NONTEMPORAL 1
#define VOFL_PROBE_DEEP        2
int vofl_stream_probe(int kind, const void* src, void* dst, size_t bytes, int blocks, int flags,
                      void* stream);

/* Synchronize stream, then report VOFL_ERR_UNSTABLE if the plan's
 * non-finite flag is set (the flag is cleared by the read). */
int vofl_sync_status(vofl_plan_t plan, void* stream);

/* Record per-kernel-class device time (HIP events) during later calls;
 * enable = 0 stops recording. vofl_kernel_times writes up to cap entries of
 * (name, total milliseconds, launch count) for the kernel classes seen since
 * the last reset and returns their number. */
int vofl_set_timing(vofl_plan_t plan, int enable);
int vofl_kernel_times(vofl_plan_t plan, const char** names, double* ms,
                      long long* launches, int cap);

/* Plan scalars (FP64): out[0] = gbar (or s0), out[1] = kappa0, out[2] = beta0,
 * out[3] = N, out[4] = device bytes held, out[5] = axis-0 kernel variant,
 * out[6] = middle-axis kernel variant, out[7] = last-axis schedule (0: the
 * default elements per thread, 1: the alternative). Writes min(cap, 8)
 * values. Returns VOFL_OK. */
int vofl_plan_info(vofl_plan_t plan, double* out, int cap);

int vofl_destroy(vofl_plan_t plan);
const char* vofl_last_error(void);
/* Library version string. */
const char* vofl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VOFL_H */
