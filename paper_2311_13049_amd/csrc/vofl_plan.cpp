// libvofl host side: descriptor validation, FP64 plan tables, device
// workspace, and the launch sequences of vofl_apply / vofl_step.
//
// Launch sequences (2D/3D; axis 0 is the half-spectrum axis, the last axis is
// contiguous; the 3D middle axis is transformed by k_mid):
//   apply (2.13): r2c0(u) -> [mid fwd] -> contig(1/N, |mu|^{2 s0} l_m, inverse
//                 last axis, m = 0..M) -> [mid inv] -> c2r0(sum_m delta^m t_m)
//   step (3.13):  r2c0(u), r2c0(v) -> [mid fwd] -> contig(state, G(dt/2), terms)
//                 then per step: [mid inv] -> c2r0(kick rhs, forward axis 0)
//                 -> [mid fwd] -> contig(v_hat += dt dv_hat, G(dt) or G(dt/2)
//                 on the last step, next terms or export) ; finally
//                 [mid inv] -> c2r0(export u, v).
// 1D runs one workgroup per field with the whole loop in one kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <thread>
#include <string>
#include <vector>

#include "launch.hpp"
#include "vofl.h"

using namespace vofl;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(VOFL_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Sizes derived from a validated descriptor (no device access).
// Crank-Nicolson solver storage (generic model, one solve at a time): vectors of N
// values in the plan precision and FP64 reduction scalars
constexpr int CN_VECTORS = 11;
constexpr int CN_SCALARS = 2 * 512 + 8;

struct Geometry {
    int ndim = 0;
    int n[3] = {1, 1, 1};
    long long Nreal = 0;   // points of one field
    int n0h = 0;           // n0/2 + 1
    long long H = 0;       // complex elements one half spectrum occupies (2D/3D): n0h rows of rs
    long long rs = 0;      // row stride of a half spectrum along axis 0 (inner, padded)
    int inner = 0;         // columns of the axis-0 transform
    int nlast = 0;         // last-axis length
    int npencils = 0;      // last-axis pencils of one half spectrum
    int batch = 1, max_batch = 1, ncoef = 1;
    int nterm = 0;         // term slots of one step
    int step_slots = 0, apply_slots = 0;
    int stage_fields = 0;  // FP64 half fields of the state/staging block
    size_t elt = 0;        // bytes of one working-precision real
    size_t bytes = 0;      // total device bytes
};

bool is_fp32(const vofl_desc* d) { return d->precision == VOFL_FP32; }

// FP64 fields of the leap-frog state per solve (2D/3D plans): u^{n-1}, u^n
int lffp_fields(int) { return 2; }

bool supported_len(int ndim, int n, bool fp32) {
    if (ndim == 1) return fp32 ? Launch<float>::supported_1d(n) : Launch<double>::supported_1d(n);
    return fp32 ? Launch<float>::supported_multi(n) : Launch<double>::supported_multi(n);
}

int derive(const vofl_desc* d, Geometry& g) {
    if (!d) return fail(VOFL_ERR_INVALID, "desc is NULL");
    if (d->ndim < 1 || d->ndim > 3) return fail(VOFL_ERR_INVALID, "ndim must be 1, 2 or 3 (got %d)", d->ndim);
    if (d->precision != VOFL_FP64 && d->precision != VOFL_FP32)
        return fail(VOFL_ERR_INVALID, "precision must be VOFL_FP64 or VOFL_FP32");
    if (d->model != VOFL_MODEL_SEISMIC && d->model != VOFL_MODEL_GENERIC)
        return fail(VOFL_ERR_INVALID, "unknown model %d", d->model);
    g.ndim = d->ndim;
    g.Nreal = 1;
    for (int i = 0; i < d->ndim; ++i) {
        const int n = d->n[i];
        if (n < 2 || n % 2) return fail(VOFL_ERR_INVALID, "n[%d] = %d must be even and >= 2", i, n);
        if (!(std::isfinite(d->lo[i]) && std::isfinite(d->hi[i]) && d->hi[i] > d->lo[i]))
            return fail(VOFL_ERR_INVALID, "box axis %d must satisfy lo < hi (finite)", i);
        if (!supported_len(d->ndim, n, is_fp32(d)))
            return fail(VOFL_ERR_UNSUPPORTED, "no compiled transform of length %d (axis %d)", n, i);
        g.n[i] = n;
        g.Nreal *= n;
    }
    if (g.Nreal > (1LL << 31)) return fail(VOFL_ERR_INVALID, "grid too large");
    if (d->M < 0 || d->M > 64) return fail(VOFL_ERR_INVALID, "M must be in [0, 64] (got %d)", d->M);
    if (!(std::isfinite(d->dt) && d->dt > 0)) return fail(VOFL_ERR_INVALID, "dt must be finite and > 0");
    if (d->max_batch < 0 || d->max_batch > 4096) return fail(VOFL_ERR_INVALID, "max_batch out of range");
    if (d->batch < 0 || d->batch > 4096) return fail(VOFL_ERR_INVALID, "batch out of range");
    if (d->coef_per_solve != 0 && d->coef_per_solve != 1)
        return fail(VOFL_ERR_INVALID, "coef_per_solve must be 0 or 1");
    if (d->tune_steps < 0 || d->tune_steps > 1000) return fail(VOFL_ERR_INVALID, "tune_steps must be in [0, 1000]");
    if (d->order != 0 && d->order != 2 && d->order != 4) return fail(VOFL_ERR_INVALID, "order must be 2 or 4");
    if (d->order == 4 && d->model != VOFL_MODEL_GENERIC)
        return fail(VOFL_ERR_UNSUPPORTED, "the fourth-order composition is provided for the generic model (1.5)");
    g.batch = d->batch ? d->batch : 1;
    g.max_batch = d->max_batch ? d->max_batch : 1;
    g.ncoef = d->coef_per_solve ? g.batch : 1;
    const long long ncv = (long long)g.ncoef * g.Nreal;
    if (d->model == VOFL_MODEL_SEISMIC) {
        if (!(std::isfinite(d->omega0) && d->omega0 > 0)) return fail(VOFL_ERR_INVALID, "omega0 must be finite and > 0");
        if (d->c0_field) {
            for (long long i = 0; i < ncv; ++i) {
                const double c = d->c0_field[i];
                if (!(std::isfinite(c) && c > 0)) return fail(VOFL_ERR_INVALID, "c0_field[%lld] = %g must be > 0", i, c);
            }
        } else if (!(std::isfinite(d->c0) && d->c0 > 0)) {
            return fail(VOFL_ERR_INVALID, "c0 must be finite and > 0");
        }
        if ((d->Q == nullptr) == (d->gamma == nullptr))
            return fail(VOFL_ERR_INVALID, "give exactly one of Q and gamma");
        if (d->Q) {
            for (long long i = 0; i < ncv; ++i) {
                const double q = d->Q[i];
                if (!(q > 0)) return fail(VOFL_ERR_INVALID, "Q[%lld] = %g must be > 0", i, q);
            }
        } else {
            for (long long i = 0; i < ncv; ++i) {
                const double gm = d->gamma[i];
                if (!(std::isfinite(gm) && gm >= 0 && gm < 0.5))
                    return fail(VOFL_ERR_INVALID, "gamma[%lld] = %g must be in [0, 1/2)", i, gm);
            }
        }
    } else {
        if (!d->s) return fail(VOFL_ERR_INVALID, "generic model needs s");
        if (!(std::isfinite(d->kappa) && d->kappa > 0)) return fail(VOFL_ERR_INVALID, "kappa must be > 0");
        if (!std::isfinite(d->lambda)) return fail(VOFL_ERR_INVALID, "lambda must be finite");
        for (long long i = 0; i < ncv; ++i) {
            const double sv = d->s[i];
            if (!(std::isfinite(sv) && sv > 0 && sv < 2))
                return fail(VOFL_ERR_INVALID, "s[%lld] = %g must be in (0, 2)", i, sv);
        }
    }
    g.elt = is_fp32(d) ? 4 : 8;
    const size_t celt = 2 * g.elt;
    size_t bytes = 0;
    // per-axis tables: twiddles (working precision and FP64) and mu^2 (FP64)
    for (int i = 0; i < d->ndim; ++i) bytes += g.n[i] * (celt + 16 + 8);
    // per-point coefficients: delta (FP64), A and B (working precision), scalars
    bytes += (size_t)ncv * (8 + 2 * g.elt) + (size_t)g.ncoef * sizeof(SolveScalars) + 256;
    if (d->ndim >= 2) {
        g.n0h = g.n[0] / 2 + 1;
        g.nlast = g.n[d->ndim - 1];
        g.inner = (int)(g.Nreal / g.n[0]);
        // Rows of a half spectrum along axis 0 (one k0 plane in 3D) are
        // padded by 128 bytes when they span 4 KiB or more: the axis-0 pass
        // reads a narrow column of every row, and at power-of-two row
        // strides those reads gather on few memory channels (a read probe of
        // that pattern at 256^3 ran 21% faster with the padding).
        g.rs = g.inner;
        if ((size_t)g.inner * celt >= 4096) g.rs += (long long)(128 / celt);
        if (const char* ev = std::getenv("VOFL_HALF_ROW_PAD")) g.rs = g.inner + std::max(0, std::atoi(ev));
        g.H = (long long)g.n0h * g.rs;
        g.npencils = (int)((long long)g.n0h * g.inner / g.nlast);
        if ((unsigned long long)g.H * 16ULL >= (1ULL << 32))
            return fail(VOFL_ERR_UNSUPPORTED, "half spectrum of %lld elements exceeds 32-bit byte offsets", g.H);
        g.nterm = (d->model == VOFL_MODEL_SEISMIC) ? 2 * (d->M + 1) : d->M + 2;
        g.step_slots = g.nterm + 3;   // terms, dv, export pair
        g.apply_slots = d->M + 1;     // terms
        const long long slots =
            std::max((long long)g.batch * g.step_slots, (long long)g.max_batch * g.apply_slots);
        if ((long long)g.batch * g.step_slots > 65535 || (long long)g.max_batch * g.apply_slots > 65535)
            return fail(VOFL_ERR_INVALID, "batch x slots exceeds the launch grid limit");
        bytes += (size_t)slots * g.H * celt;                  // work slots
        g.stage_fields = std::max(2 * g.batch, g.max_batch);
        bytes += (size_t)g.stage_fields * g.H * 16;           // FP64 state / forward staging
        // FP64 leap-frog state (u^{n-1}, u^n)
        bytes += (size_t)lffp_fields(d->model) * g.batch * g.Nreal * 8;
    }
    else
        bytes += (size_t)2 * g.batch * g.Nreal * g.elt;      // 1D resumable run: (u, v) between calls
    if (d->model == VOFL_MODEL_GENERIC)
        bytes += (size_t)CN_VECTORS * g.Nreal * g.elt + CN_SCALARS * 8;  // Crank-Nicolson solver vectors
    g.bytes = bytes;
    if (d->hbm_budget && bytes > d->hbm_budget)
        return fail(VOFL_ERR_NOMEM, "plan needs %zu bytes, above hbm_budget %zu", bytes, d->hbm_budget);
    return VOFL_OK;
}

// Coefficients (1.1): c = c0 cos(pi g/2), eta = -c0^{2g} w0^{-2g} cos(pi g),
// tau = -c0^{2g-1} w0^{-2g} sin(pi g); A = -c^2 eta, B = -c^2 tau.
void seismic_AB(double g, double c0, double w0, double& A, double& B) {
    const double c = c0 * std::cos(M_PI * g / 2.0);
    const double eta = -std::pow(c0, 2.0 * g) * std::pow(w0, -2.0 * g) * std::cos(M_PI * g);
    const double tau = -std::pow(c0, 2.0 * g - 1.0) * std::pow(w0, -2.0 * g) * std::sin(M_PI * g);
    A = -c * c * eta;
    B = -c * c * tau;
}

struct TimedRec {
    int cls;
    hipEvent_t a, b;
};

}  // namespace

struct vofl_plan_s {
    Geometry g;
    int model = 0, precision = 0, M = 0;
    double dt = 0;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    std::vector<SolveScalars> sc_host;
    // device memory
    double* mu2[3] = {nullptr, nullptr, nullptr};
    void* tw[3] = {nullptr, nullptr, nullptr};      // working precision
    cpx<double>* tw64[3] = {nullptr, nullptr, nullptr};
    double* delta = nullptr;
    double* LS = nullptr;              // leap-frog FP64 state: u^{n-1} of every solve, then u^n
    void* cnv = nullptr;               // Crank-Nicolson vectors (CN_VECTORS x N, one solve at a time)
    int coef_item = 0;                 // solve whose coefficients single-field launches use
                                       // (set by the Crank-Nicolson solver; else 0)
    double* cns = nullptr;             // Crank-Nicolson reduction scalars
    int sub = 1;                       // sub-steps per step (3: fourth-order composition)
    double w1 = 1.0, w0 = 1.0;         // composition weights
    void* A = nullptr;
    void* B = nullptr;
    SolveScalars* sc = nullptr;
    void* U = nullptr;
    void* V = nullptr;
    void* work = nullptr;
    int* flag = nullptr;
    std::vector<void*> allocs;
    int c2r_variant = 0;               // axis-0 kernel variant (see Launch::c2r0)
    double tuned_ms = 0;               // best time per tuning run (0: not tuned)
    struct GraphEntry {
        void* u;
        void* v;
        int nsteps;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;    // vofl_step_graph cache, oldest first
    int mid_variant = 1;               // k_mid tile variant (1: double-width tiles)
    int contig_variant = 0;            // last-axis elements per thread (1: the alternative radix schedule)
    // resumable run (vofl_step_begin / advance / end): 0 none; 1 the state is
    // (u_hat, v_hat) at t_n itself (after begin); 2 the state is the one right
    // after the kick of the last step (the step's closing half sub-step pending)
    int run = 0;
    long long run_steps = 0;           // steps advanced since begin
    struct RunGraph {
        int nsteps, phase;
        hipGraphExec_t exec;
    };
    std::vector<RunGraph> run_graphs;  // vofl_step_advance graph cache, oldest first
    hipStream_t own_stream = nullptr;  // used by vofl_step_batch
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    // timing
    bool timing = false;
    std::vector<TimedRec> pending;
    std::vector<hipEvent_t> pool;
    std::vector<std::string> cls_names;
    std::map<int, std::pair<double, long long>> totals;

    ~vofl_plan_s() {
        for (auto& r : pending) {
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
        for (auto& gr : graphs) (void)hipGraphExecDestroy(gr.exec);
        for (auto& gr : run_graphs) (void)hipGraphExecDestroy(gr.exec);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (join_ev) (void)hipEventDestroy(join_ev);
        if (own_stream) (void)hipStreamDestroy(own_stream);
        for (void* p : allocs) (void)hipFree(p);
    }

    int cls_id(const char* name) {
        for (size_t i = 0; i < cls_names.size(); ++i)
            if (cls_names[i] == name) return (int)i;
        cls_names.emplace_back(name);
        return (int)cls_names.size() - 1;
    }
    hipEvent_t get_event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    // wrap one launch: returns the launch status
    template <class F>
    hipError_t timed(const char* name, hipStream_t s, F&& launch) {
        if (!timing) return launch();
        TimedRec r{cls_id(name), get_event(), get_event()};
        (void)hipEventRecord(r.a, s);
        hipError_t e = launch();
        (void)hipEventRecord(r.b, s);
        pending.push_back(r);
        return e;
    }
    void drain_timing() {
        for (auto& r : pending) {
            (void)hipEventSynchronize(r.b);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, r.a, r.b);
            auto& t = totals[r.cls];
            t.first += ms;
            t.second += 1;
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
};

namespace {

template <typename P>
int dalloc(vofl_plan_s* p, P** ptr, size_t bytes) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(VOFL_ERR_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    p->allocs.push_back(q);
    *ptr = static_cast<P*>(q);
    return VOFL_OK;
}

// Host loops over grid points (coefficient maps) split over threads; each
// element is computed independently, so the result does not depend on the split.
template <class F>
void parallel_for(long long n, F&& fn) {
    const unsigned hw = std::thread::hardware_concurrency();
    const long long nt = std::min<long long>(std::max(1u, std::min(hw, 16u)), std::max(1LL, n / (1LL << 16)));
    if (nt <= 1) {
        for (long long i = 0; i < n; ++i) fn(i);
        return;
    }
    std::vector<std::thread> th;
    const long long per = (n + nt - 1) / nt;
    for (long long t = 0; t < nt; ++t) {
        const long long a = t * per, b = std::min(n, a + per);
        th.emplace_back([a, b, &fn] {
            for (long long i = a; i < b; ++i) fn(i);
        });
    }
    for (auto& x : th) x.join();
}

template <typename T>
int upload_tables(vofl_plan_s* p, const std::vector<double>& delta, const std::vector<double>& A,
                  const std::vector<double>& B) {
    const Geometry& g = p->g;
    for (int ax = 0; ax < g.ndim; ++ax) {
        const int n = g.n[ax];
        std::vector<cpx<T>> tw(n);
        std::vector<double> mu2(n);
        const double L = p->hi[ax] - p->lo[ax];
        for (int j = 0; j < n; ++j) {
            const double ang = 2.0 * M_PI * (double)j / (double)n;
            tw[j] = {T(std::cos(ang)), T(-std::sin(ang))};
            const int k = (j < n / 2) ? j : j - n;  // bin j holds wavenumber k (eq. (2.2))
            const double mu = 2.0 * M_PI * (double)k / L;
            mu2[j] = mu * mu;
        }
        std::vector<cpx<double>> tw64(n);
        for (int j = 0; j < n; ++j) {
            const double ang = 2.0 * M_PI * (double)j / (double)n;
            tw64[j] = {std::cos(ang), -std::sin(ang)};
        }
        int rc;
        if ((rc = dalloc(p, (cpx<T>**)&p->tw[ax], n * sizeof(cpx<T>)))) return rc;
        if ((rc = dalloc(p, &p->tw64[ax], n * sizeof(cpx<double>)))) return rc;
        if ((rc = dalloc(p, &p->mu2[ax], n * sizeof(double)))) return rc;
        hipError_t e = hipMemcpy(p->tw[ax], tw.data(), n * sizeof(cpx<T>), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(p->tw64[ax], tw64.data(), n * sizeof(cpx<double>), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(p->mu2[ax], mu2.data(), n * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "table upload");
    }
    const size_t ncv = delta.size();
    std::vector<T> At(ncv), Bt(ncv);
    parallel_for((long long)ncv, [&](long long i) {
        At[i] = T(A[i]);
        Bt[i] = T(B[i]);
    });
    int rc;
    if ((rc = dalloc(p, &p->delta, ncv * sizeof(double)))) return rc;
    if ((rc = dalloc(p, (T**)&p->A, ncv * sizeof(T)))) return rc;
    if ((rc = dalloc(p, (T**)&p->B, ncv * sizeof(T)))) return rc;
    if ((rc = dalloc(p, &p->sc, p->sc_host.size() * sizeof(SolveScalars)))) return rc;
    if ((rc = dalloc(p, &p->flag, 256))) return rc;
    hipError_t e = hipMemcpy(p->delta, delta.data(), ncv * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->A, At.data(), ncv * sizeof(T), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->B, Bt.data(), ncv * sizeof(T), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->sc, p->sc_host.data(), p->sc_host.size() * sizeof(SolveScalars), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->flag, 0, 256);
    if (e != hipSuccess) return hip_fail(e, "coefficient upload");
    if (g.ndim >= 2) {
        const long long slots = std::max((long long)g.batch * g.step_slots, (long long)g.max_batch * g.apply_slots);
        if ((rc = dalloc(p, (cpx<T>**)&p->work, (size_t)slots * g.H * sizeof(cpx<T>)))) return rc;
        // one block: u_hat of every solve, then v_hat of every solve; also the
        // FP64 staging of forward transforms (apply fields use it from the start)
        if ((rc = dalloc(p, (cpx<double>**)&p->U, (size_t)g.stage_fields * g.H * sizeof(cpx<double>)))) return rc;
        p->V = (cpx<double>*)p->U + (size_t)g.batch * g.H;
        if ((rc = dalloc(p, &p->LS, (size_t)lffp_fields(p->model) * g.batch * g.Nreal * sizeof(double))))
            return rc;
    } else {
        // 1D resumable run: the fields (u, v) of every solve between calls
        if ((rc = dalloc(p, (T**)&p->U, (size_t)2 * g.batch * g.Nreal * sizeof(T)))) return rc;
        p->V = (T*)p->U + (size_t)g.batch * g.Nreal;
    }
    if (p->model == VOFL_MODEL_GENERIC) {
        if ((rc = dalloc(p, (T**)&p->cnv, (size_t)CN_VECTORS * g.Nreal * sizeof(T)))) return rc;
        if ((rc = dalloc(p, &p->cns, (size_t)CN_SCALARS * sizeof(double)))) return rc;
    }
    return VOFL_OK;
}

// ---------------------------------------------------------------------------
// launch sequences
// ---------------------------------------------------------------------------

// coefficient offsets of the solve p->coef_item (plans with one coefficient
// field per solve; 0 otherwise)
long long coef_off(const vofl_plan_s* p) { return p->g.ncoef > 1 ? (long long)p->coef_item * p->g.Nreal : 0; }
int sc_off(const vofl_plan_s* p) { return p->g.ncoef > 1 ? p->coef_item : 0; }

template <typename T, typename TI>
ContigArgs<T, TI> contig_base(vofl_plan_s* p) {
    const Geometry& g = p->g;
    ContigArgs<T, TI> a{};
    a.H = g.H;
    a.rs = g.rs;
    a.npencils = g.npencils;
    a.n1 = (g.ndim == 3) ? g.n[1] : 1;
    a.mu2_0 = p->mu2[0];
    a.mu2_1 = (g.ndim == 3) ? p->mu2[1] : nullptr;
    a.mu2_l = p->mu2[g.ndim - 1];
    a.tw = (const cpx<T>*)p->tw[g.ndim - 1];
    // input-transform twiddles: every launch stages them, whatever it reads
    if constexpr (std::is_same<TI, double>::value) a.tw_in = p->tw64[g.ndim - 1];
    else a.tw_in = (const cpx<TI>*)p->tw[g.ndim - 1];
    a.sc = p->sc + sc_off(p);
    a.sc_stride = g.ncoef > 1 ? 1 : 0;
    a.U = (cpx<double>*)p->U;
    a.V = (cpx<double>*)p->V;
    a.M = p->M;
    a.dt = p->dt;
    a.invN = 1.0 / (double)g.Nreal;
    return a;
}

// 3D middle-axis transform of nf fields per item (item stride istride)
template <typename T>
hipError_t mid(vofl_plan_s* p, const char* name, int dir, cpx<T>* buf, long long istride, int nf,
               int items, const cpx<T>* tw, hipStream_t s) {
    const Geometry& g = p->g;
    if (g.ndim != 3) return hipSuccess;
    MidArgs<T> m{};
    m.buf = buf;
    m.istride = istride;
    m.nf = nf;
    m.H = g.H;
    m.rs = g.rs;
    m.n2 = g.n[2];
    const int W = Launch<T>::mid_tile(g.n[1], p->mid_variant);
    m.tiles_per_plane = (g.n[2] + W - 1) / W;
    m.tw = tw;
    return p->timed(name, s, [&] { return Launch<T>::mid(g.n[1], dir, m, g.n0h, items, s, p->mid_variant); });
}

// forward transform of real fields (items of Nreal values) into the FP64
// staging block at stage + item*H, including the 3D middle axis
template <typename T>
hipError_t forward_to_stage(vofl_plan_s* p, const T* in, cpx<double>* stage, int items, hipStream_t s,
                           const T* in2 = nullptr, double c1 = 1.0, double c2 = 0.0) {
    const Geometry& g = p->g;
    R2CArgs<T> r{};
    r.in = in;
    r.in2 = in2;  // optional: transform c1 in + c2 in2
    r.c1 = c1;
    r.c2 = c2;
    r.Nreal = g.Nreal;
    r.out = stage;
    r.H = g.H;
    r.rs = g.rs;
    r.inner = g.inner;
    r.tw = p->tw64[0];
    hipError_t e = p->timed("r2c0", s, [&] { return Launch<T>::r2c0(g.n[0], r, items, s); });
    return e;
}

template <typename T>
C2RArgs<T> c2r_base(vofl_plan_s* p) {
    const Geometry& g = p->g;
    C2RArgs<T> c{};
    c.H = g.H;
    c.rs = g.rs;
    c.inner = g.inner;
    c.tw = (const cpx<T>*)p->tw[0];
    c.M = p->M;
    c.model = p->model;
    c.delta = p->delta + coef_off(p);
    c.A = (const T*)p->A + coef_off(p);
    c.B = (const T*)p->B + coef_off(p);
    c.coef_stride = g.ncoef > 1 ? g.Nreal : 0;
    c.sc = p->sc + sc_off(p);
    c.sc_stride = g.ncoef > 1 ? 1 : 0;
    c.Nreal = g.Nreal;
    c.flag = p->flag;
    return c;
}

// leap-frog update fused into the apply's last pass (see C2RArgs)
struct LffpPass {
    double cb, ca, cf;
    double* prev;
    double* cur;
};

template <typename T, typename TIN = T>
int apply_multi(vofl_plan_s* p, int op, const TIN* u, T* out, int nf, hipStream_t s,
                const LffpPass* lf = nullptr) {
    const Geometry& g = p->g;
    const long long AS = (long long)g.apply_slots * g.H;  // item stride of the term slots
    cpx<T>* W = (cpx<T>*)p->work;
    cpx<double>* stage = (cpx<double>*)p->U;
    hipError_t e = forward_to_stage<TIN>(p, u, stage, nf, s);
    if (e != hipSuccess) return hip_fail(e, "r2c0 launch");
    if ((e = mid<double>(p, "mid_apply_fwd", -1, stage, g.H, 1, nf, p->tw64[1 % g.ndim], s)) != hipSuccess)
        return hip_fail(e, "mid launch");
    ContigArgs<T, double> a = contig_base<T, double>(p);
    a.in = stage;
    a.in_istride = g.H;
    a.nin = 1;
    a.tw_in = p->tw64[g.ndim - 1];
    a.out = W;
    a.out_istride = AS;
    a.in_kind = IN_APPLY;
    a.emit_kind = EMIT_APPLY;
    a.do_prop = 0;
    a.op = op;
    e = p->timed("contig_apply", s, [&] { return Launch<T>::contig(g.nlast, a, nf, s, p->contig_variant); });
    if (e != hipSuccess) return hip_fail(e, "contig launch");
    if ((e = mid<T>(p, "mid_apply_terms", +1, W, AS, p->M + 1, nf, (const cpx<T>*)p->tw[1 % g.ndim], s)) != hipSuccess)
        return hip_fail(e, "mid launch");
    C2RArgs<T> c = c2r_base<T>(p);
    c.in = W;
    c.istride = AS;
    c.mode = C2R_APPLY;
    c.r0 = out;
    if (lf) {
        c.lffp = 1;
        c.s_prev = lf->prev;
        c.s_cur = lf->cur;
        c.lf_cb = lf->cb;
        c.lf_ca = lf->ca;
        c.lf_cf = lf->cf;
    }
    e = p->timed(lf ? "c2r0_lffp" : "c2r0_apply", s, [&] { return Launch<T>::c2r0(g.n[0], c, nf, s, p->c2r_variant); });
    if (e != hipSuccess) return hip_fail(e, "c2r0 launch");
    return VOFL_OK;
}

// nsteps leap-frog steps (3.4a) on the plan's FP64 state; the first uses
// (cb0, ca0, cf0) in place of (2, -1, dt^2) (the start (3.4c) is such a step
// with (1, dt, dt^2/2) on (prev, cur) = (psi, phi))
template <typename T>
int lffp_seismic_multi(vofl_plan_s* p, double cb0, double ca0, double cf0, double wc0, double wp0, int nsteps,
                       hipStream_t s);

template <typename T>
int lffp_multi(vofl_plan_s* p, double cb0, double ca0, double cf0, double wc0, double wp0, int nsteps,
               hipStream_t s) {
    if (p->model == VOFL_MODEL_SEISMIC) return lffp_seismic_multi<T>(p, cb0, ca0, cf0, wc0, wp0, nsteps, s);
    const Geometry& g = p->g;
    double* prev = p->LS;
    double* cur = p->LS + (size_t)g.batch * g.Nreal;
    for (int k = 0; k < nsteps; ++k) {
        const LffpPass lf{k == 0 ? cb0 : 2.0, k == 0 ? ca0 : -1.0, k == 0 ? cf0 : p->dt * p->dt, prev, cur};
        const int rc = apply_multi<T, double>(p, VOFL_OP_S1, cur, (T*)nullptr, g.batch, s, &lf);
        if (rc) return rc;
    }
    return VOFL_OK;
}



// Leap-frog steps for (1.1) on the plan's FP64 state (u^{n-1}, u^n):
// per step forward transforms in FP64 of u^n and of w = wc u^n + wp u^{n-1}
// ((u^n - u^{n-1})/dt, formed while loading; the first step uses (wc0, wp0)), the 2(M+1) term
// spectra l_m |mu|^{2 sigma_1} u_hat and l_m |mu|^{2 sigma_2} w_hat along the
// last (and middle) axis, and the axis-0 pass that sums -A L1 u - B L2 w by
// (2.13) and updates the state in place.
template <typename T>
int lffp_seismic_multi(vofl_plan_s* p, double cb0, double ca0, double cf0, double wc0, double wp0, int nsteps,
                       hipStream_t s) {
    const Geometry& g = p->g;
    const int items = g.batch;
    const long long n = (long long)items * g.Nreal;
    const long long SS = (long long)g.step_slots * g.H;
    double* prev = p->LS;
    double* cur = p->LS + n;
    cpx<T>* W = (cpx<T>*)p->work;
    cpx<double>* U = (cpx<double>*)p->U;
    cpx<double>* V = (cpx<double>*)p->V;
    hipError_t e;
    ContigArgs<T, double> a = contig_base<T, double>(p);
    a.in = U;
    a.in_istride = g.H;
    a.in_fstride = (long long)items * g.H;
    a.nin = 2;
    a.tw_in = p->tw64[g.ndim - 1];
    a.out = W;
    a.out_istride = SS;
    a.in_kind = IN_APPLY;     // no state in the spectral blocks
    a.emit_kind = EMIT_STEP;  // slot pairs (t1_m, t2_m), m = 0..M
    a.do_prop = 0;
    C2RArgs<T> c = c2r_base<T>(p);
    c.in = W;
    c.istride = SS;
    c.mode = C2R_KICK;
    c.lffp = 1;
    c.s_prev = prev;
    c.s_cur = cur;
    for (int k = 0; k < nsteps; ++k) {
        const double wc = k == 0 ? wc0 : 1.0 / p->dt, wp = k == 0 ? wp0 : -1.0 / p->dt;
        c.lf_cb = k == 0 ? cb0 : 2.0;
        c.lf_ca = k == 0 ? ca0 : -1.0;
        c.lf_cf = k == 0 ? cf0 : p->dt * p->dt;
        if ((e = forward_to_stage<double>(p, cur, U, items, s)) != hipSuccess) return hip_fail(e, "r2c0 launch");
        // w: the start passes psi itself in the prev slot
        e = (wc == 0.0 && wp == 1.0) ? forward_to_stage<double>(p, prev, V, items, s)
                                     : forward_to_stage<double>(p, cur, V, items, s, prev, wc, wp);
        if (e != hipSuccess) return hip_fail(e, "r2c0 launch");
        if ((e = mid<double>(p, "mid_lffp_fwd", -1, U, g.H, 1, 2 * items, p->tw64[1 % g.ndim], s)) != hipSuccess)
            return hip_fail(e, "mid launch");
        e = p->timed("contig_lffp", s, [&] { return Launch<T>::contig(g.nlast, a, items, s, p->contig_variant); });
        if (e != hipSuccess) return hip_fail(e, "contig launch");
        if ((e = mid<T>(p, "mid_lffp_terms", +1, W, SS, g.nterm, items, (const cpx<T>*)p->tw[1 % g.ndim], s)) !=
            hipSuccess)
            return hip_fail(e, "mid launch");
        e = p->timed("c2r0_lffp", s, [&] { return Launch<T>::c2r0(g.n[0], c, items, s, p->c2r_variant); });
        if (e != hipSuccess) return hip_fail(e, "c2r0 launch");
    }
    return VOFL_OK;
}

// length of sub-step k (dt for TSFP2; dt w1, dt w0, dt w1 for the composition)
double substep_len_h(const vofl_plan_s* p, int k) {
    return p->sub == 3 ? p->dt * ((k % 3 == 1) ? p->w0 : p->w1) : p->dt;
}

template <typename T>
int step_multi(vofl_plan_s* p, T* u, T* v, int nsteps, hipStream_t s) {
    if (nsteps == 0) return VOFL_OK;
    const Geometry& g = p->g;
    const long long SS = (long long)g.step_slots * g.H;  // item stride of the step slots
    const int nterm = g.nterm;
    const int dv = nterm, h0 = nterm + 1;
    const int items = g.batch;
    const bool generic = p->model == VOFL_MODEL_GENERIC;
    const int emit_terms = generic ? EMIT_GENERIC : EMIT_STEP;
    cpx<T>* W = (cpx<T>*)p->work;
    const cpx<T>* twm = (const cpx<T>*)p->tw[1 % g.ndim];
    cpx<double>* U = (cpx<double>*)p->U;
    cpx<double>* V = (cpx<double>*)p->V;
    hipError_t e;

    // forward transforms of (u, v) in FP64 into the state block, then the
    // first half step of the exact part and the first terms
    if ((e = forward_to_stage<T>(p, u, U, items, s)) != hipSuccess) return hip_fail(e, "r2c0 launch");
    if ((e = forward_to_stage<T>(p, v, V, items, s)) != hipSuccess) return hip_fail(e, "r2c0 launch");
    if ((e = mid<double>(p, "mid_init", -1, U, g.H, 1, 2 * items, p->tw64[1 % g.ndim], s)) != hipSuccess)
        return hip_fail(e, "mid launch");
    {
        ContigArgs<T, double> a = contig_base<T, double>(p);
        a.in = U;
        a.in_istride = g.H;
        a.in_fstride = (long long)items * g.H;
        a.nin = 2;
        a.tw_in = p->tw64[g.ndim - 1];
        a.out = W;
        a.out_istride = SS;
        a.in_kind = IN_INIT;
        a.emit_kind = emit_terms;
        a.do_prop = 1;
        a.tprop = 0.5 * substep_len_h(p, 0);
        e = p->timed("contig_init", s, [&] { return Launch<T>::contig(g.nlast, a, items, s, p->contig_variant); });
        if (e != hipSuccess) return hip_fail(e, "contig launch");
    }

    C2RArgs<T> c = c2r_base<T>(p);
    c.in = W;
    c.istride = SS;
    c.mode = generic ? C2R_KICK_GENERIC : C2R_KICK;
    c.dv_out = W + (long long)dv * g.H;

    ContigArgs<T, T> a = contig_base<T, T>(p);
    a.in = W + (long long)dv * g.H;
    a.in_istride = SS;
    a.nin = 1;
    a.tw_in = (const cpx<T>*)p->tw[g.ndim - 1];
    a.out_istride = SS;
    a.in_kind = IN_KICK;
    a.do_prop = 1;

    const int K = nsteps * p->sub;  // sub-steps (TSFP2: one per step)
    for (int st = 0; st < K; ++st) {
        const bool last = (st + 1 == K);
        const double ds = substep_len_h(p, st);
        a.dt = ds;  // the kick of this sub-step
        if ((e = mid<T>(p, "mid_terms", +1, W, SS, nterm, items, twm, s)) != hipSuccess) return hip_fail(e, "mid launch");
        e = p->timed("c2r0_kick", s, [&] { return Launch<T>::c2r0(g.n[0], c, items, s, p->c2r_variant); });
        if (e != hipSuccess) return hip_fail(e, "c2r0 launch");
        if ((e = mid<T>(p, "mid_dv", -1, W + (long long)dv * g.H, SS, 1, items, twm, s)) != hipSuccess)
            return hip_fail(e, "mid launch");
        a.tprop = last ? 0.5 * ds : 0.5 * (ds + substep_len_h(p, st + 1));
        a.emit_kind = last ? EMIT_EXPORT : emit_terms;
        a.out = W + (last ? (long long)h0 * g.H : 0);
        e = p->timed("contig_kick", s, [&] { return Launch<T>::contig(g.nlast, a, items, s, p->contig_variant); });
        if (e != hipSuccess) return hip_fail(e, "contig launch");
    }
    if ((e = mid<T>(p, "mid_export", +1, W + (long long)h0 * g.H, SS, 2, items, twm, s)) != hipSuccess)
        return hip_fail(e, "mid launch");
    C2RArgs<T> x = c2r_base<T>(p);
    x.in = W + (long long)h0 * g.H;
    x.istride = SS;
    x.mode = C2R_EXPORT;
    x.r0 = u;
    x.r1 = v;
    e = p->timed("c2r0_export", s, [&] { return Launch<T>::c2r0(g.n[0], x, items, s, p->c2r_variant); });
    if (e != hipSuccess) return hip_fail(e, "c2r0 launch");
    return VOFL_OK;
}

// Resumable run (2D/3D). The state between calls is kept in the plan's
// FP64 spectral blocks: after begin, (u_hat, v_hat) at t_0; after advance,
// the state right after the kick of the last step, whose closing exact half
// sub-step (3.13) is applied by the next advance (merged with the next
// step's opening half, as inside vofl_step) or by end (for the export only).
// The arithmetic is that of vofl_step: the state passes through memory in
// FP64 where vofl_step keeps it in registers, so a run of n steps in any
// number of advance calls gives vofl_step's result for n steps bit for bit.
template <typename T>
int run_begin_multi(vofl_plan_s* p, const T* u, const T* v, hipStream_t s) {
    const Geometry& g = p->g;
    const int items = g.batch;
    cpx<double>* U = (cpx<double>*)p->U;
    cpx<double>* V = (cpx<double>*)p->V;
    hipError_t e;
    if ((e = forward_to_stage<T>(p, u, U, items, s)) != hipSuccess) return hip_fail(e, "r2c0 launch");
    if ((e = forward_to_stage<T>(p, v, V, items, s)) != hipSuccess) return hip_fail(e, "r2c0 launch");
    if ((e = mid<double>(p, "mid_init", -1, U, g.H, 1, 2 * items, p->tw64[1 % g.ndim], s)) != hipSuccess)
        return hip_fail(e, "mid launch");
    ContigArgs<T, double> a = contig_base<T, double>(p);
    a.in = U;
    a.in_istride = g.H;
    a.in_fstride = (long long)items * g.H;
    a.nin = 2;
    a.tw_in = p->tw64[g.ndim - 1];
    a.out = (cpx<T>*)p->work;
    a.out_istride = (long long)g.step_slots * g.H;
    a.in_kind = IN_INIT;
    a.emit_kind = EMIT_NONE;
    a.do_prop = 0;
    e = p->timed("contig_begin", s, [&] { return Launch<T>::contig(g.nlast, a, items, s, p->contig_variant); });
    return e == hipSuccess ? VOFL_OK : hip_fail(e, "contig launch");
}

template <typename T>
int run_advance_multi(vofl_plan_s* p, int nsteps, int phase, hipStream_t s) {
    if (nsteps == 0) return VOFL_OK;
    const Geometry& g = p->g;
    const long long SS = (long long)g.step_slots * g.H;
    const int nterm = g.nterm;
    const int dv = nterm;
    const int items = g.batch;
    const int emit_terms = p->model == VOFL_MODEL_GENERIC ? EMIT_GENERIC : EMIT_STEP;
    cpx<T>* W = (cpx<T>*)p->work;
    const cpx<T>* twm = (const cpx<T>*)p->tw[1 % g.ndim];
    hipError_t e;
    // reopen: the pending half sub-step(s) from the state, then the terms
    {
        ContigArgs<T, T> a = contig_base<T, T>(p);
        a.out = W;
        a.out_istride = SS;
        a.in_kind = IN_STATE;
        a.emit_kind = emit_terms;
        a.do_prop = 1;
        const double first = substep_len_h(p, 0);
        a.tprop = phase == 1 ? 0.5 * first : 0.5 * (substep_len_h(p, p->sub - 1) + first);
        e = p->timed("contig_resume", s, [&] { return Launch<T>::contig(g.nlast, a, items, s, p->contig_variant); });
        if (e != hipSuccess) return hip_fail(e, "contig launch");
    }
    C2RArgs<T> c = c2r_base<T>(p);
    c.in = W;
    c.istride = SS;
    c.mode = p->model == VOFL_MODEL_GENERIC ? C2R_KICK_GENERIC : C2R_KICK;
    c.dv_out = W + (long long)dv * g.H;
    ContigArgs<T, T> a = contig_base<T, T>(p);
    a.in = W + (long long)dv * g.H;
    a.in_istride = SS;
    a.nin = 1;
    a.tw_in = (const cpx<T>*)p->tw[g.ndim - 1];
    a.out = W;
    a.out_istride = SS;
    a.in_kind = IN_KICK;
    const int K = nsteps * p->sub;
    for (int st = 0; st < K; ++st) {
        const bool last = (st + 1 == K);
        const double ds = substep_len_h(p, st);
        a.dt = ds;
        if ((e = mid<T>(p, "mid_terms", +1, W, SS, nterm, items, twm, s)) != hipSuccess) return hip_fail(e, "mid launch");
        e = p->timed("c2r0_kick", s, [&] { return Launch<T>::c2r0(g.n[0], c, items, s, p->c2r_variant); });
        if (e != hipSuccess) return hip_fail(e, "c2r0 launch");
        if ((e = mid<T>(p, "mid_dv", -1, W + (long long)dv * g.H, SS, 1, items, twm, s)) != hipSuccess)
            return hip_fail(e, "mid launch");
        // the last kick of the call stores the state and stops there
        a.do_prop = last ? 0 : 1;
        a.tprop = last ? 0.0 : 0.5 * (ds + substep_len_h(p, st + 1));
        a.emit_kind = last ? EMIT_NONE : emit_terms;
        e = p->timed(last ? "contig_close" : "contig_kick", s, [&] { return Launch<T>::contig(g.nlast, a, items, s, p->contig_variant); });
        if (e != hipSuccess) return hip_fail(e, "contig launch");
    }
    return VOFL_OK;
}

template <typename T>
int run_end_multi(vofl_plan_s* p, T* u, T* v, int phase, hipStream_t s) {
    const Geometry& g = p->g;
    const long long SS = (long long)g.step_slots * g.H;
    const int h0 = g.nterm + 1;
    const int items = g.batch;
    cpx<T>* W = (cpx<T>*)p->work;
    const cpx<T>* twm = (const cpx<T>*)p->tw[1 % g.ndim];
    hipError_t e;
    ContigArgs<T, T> a = contig_base<T, T>(p);
    a.out = W + (long long)h0 * g.H;
    a.out_istride = SS;
    a.in_kind = IN_STATE;
    a.no_store = 1;
    a.emit_kind = EMIT_EXPORT;
    a.do_prop = phase == 2 ? 1 : 0;
    a.tprop = 0.5 * substep_len_h(p, p->sub - 1);
    e = p->timed("contig_end", s, [&] { return Launch<T>::contig(g.nlast, a, items, s, p->contig_variant); });
    if (e != hipSuccess) return hip_fail(e, "contig launch");
    if ((e = mid<T>(p, "mid_export", +1, W + (long long)h0 * g.H, SS, 2, items, twm, s)) != hipSuccess)
        return hip_fail(e, "mid launch");
    C2RArgs<T> x = c2r_base<T>(p);
    x.in = W + (long long)h0 * g.H;
    x.istride = SS;
    x.mode = C2R_EXPORT;
    x.r0 = u;
    x.r1 = v;
    e = p->timed("c2r0_export", s, [&] { return Launch<T>::c2r0(g.n[0], x, items, s, p->c2r_variant); });
    return e == hipSuccess ? VOFL_OK : hip_fail(e, "c2r0 launch");
}

template <typename T>
Args1D<T> args_1d(vofl_plan_s* p) {
    const Geometry& g = p->g;
    Args1D<T> a{};
    a.N = g.n[0];
    a.mu2 = p->mu2[0];
    a.tw = (const cpx<T>*)p->tw[0];
    a.tw64 = p->tw64[0];
    a.delta = p->delta + coef_off(p);
    a.A = (const T*)p->A + coef_off(p);
    a.B = (const T*)p->B + coef_off(p);
    a.coef_stride = g.ncoef > 1 ? g.Nreal : 0;
    a.sc = p->sc + sc_off(p);
    a.sc_stride = g.ncoef > 1 ? 1 : 0;
    a.M = p->M;
    a.model = p->model;
    a.dt = p->dt;
    a.invN = 1.0 / (double)g.Nreal;
    a.flag = p->flag;
    a.sub = p->sub;
    a.w1 = p->w1;
    a.w0 = p->w0;
    return a;
}

// leap-frog on caller fields: (cur, prev) in, nsteps steps, (cur, prev) out
template <typename T>
int lffp_any(vofl_plan_s* p, const void* cur_in, const void* prev_in, void* cur_out, void* prev_out,
             double cb0, double ca0, double cf0, double wc0, double wp0, int nsteps, hipStream_t s) {
    const Geometry& g = p->g;
    if (g.ndim == 1) {
        Args1D<T> a = args_1d<T>(p);
        a.u_in = (const T*)cur_in;
        a.v_in = (const T*)prev_in;
        a.u_out = (T*)cur_out;
        a.v_out = (T*)prev_out;
        a.nsteps = nsteps;
        a.lf_cb = cb0;
        a.lf_ca = ca0;
        a.lf_cf = cf0;
        a.lf_wc = wc0;
        a.lf_wp = wp0;
        hipError_t e = p->timed("1d_lffp", s, [&] { return Launch<T>::d1_lffp(a.N, a, g.batch, s); });
        return e == hipSuccess ? VOFL_OK : hip_fail(e, "1d leap-frog launch");
    }
    const long long n = (long long)g.batch * g.Nreal;
    double* prev = p->LS;
    double* cur = p->LS + n;
    hipError_t e = Launch<T>::to_f64((const T*)cur_in, cur, n, s);
    if (e == hipSuccess) e = Launch<T>::to_f64((const T*)prev_in, prev, n, s);
    if (e != hipSuccess) return hip_fail(e, "state load");
    int rc = lffp_multi<T>(p, cb0, ca0, cf0, wc0, wp0, nsteps, s);
    if (rc) return rc;
    e = Launch<T>::from_f64(cur, (T*)cur_out, n, s);
    if (e == hipSuccess) e = Launch<T>::from_f64(prev, (T*)prev_out, n, s);
    return e == hipSuccess ? VOFL_OK : hip_fail(e, "state store");
}


template <typename T>
int apply_any(vofl_plan_s* p, int op, const void* u, void* out, int nf, hipStream_t s) {
    if (p->g.ndim >= 2) return apply_multi<T>(p, op, (const T*)u, (T*)out, nf, s);
    Args1D<T> a = args_1d<T>(p);
    a.u_in = (const T*)u;
    a.u_out = (T*)out;
    a.op = op;
    hipError_t e = p->timed("1d_apply", s, [&] { return Launch<T>::d1_apply(a.N, a, nf, s); });
    if (e != hipSuccess) return hip_fail(e, "1d apply launch");
    return VOFL_OK;
}

// Crank-Nicolson scheme (3.2) for one solve of the generic model: per step,
// w = u^{n+1} solves w + a L w - b f(w) = r with
// r = 2 u^n - u^{n-1} - a L u^{n-1} + b f(u^{n-1}), a = kappa dt^2/2,
// b = dt^2/2, f(w) = lambda w^3; fixed-point iteration on f(w), each linear
// solve with I + a L by BiCGSTAB (the operator (2.13) is not symmetric).
// Host-driven: the scalars of every iteration are read back.
template <typename T>
int cnfp_solve(vofl_plan_s* p, T* up, T* u, int nsteps, double tol, int max_iter, long long* iters,
               hipStream_t s);

// Crank-Nicolson steps of every solve of the plan, one solve after another
// (each solve's applies use its own coefficients; the solver vectors are
// reused)
template <typename T>
int cnfp_run(vofl_plan_s* p, T* up, T* u, int nsteps, double tol, int max_iter, long long* iters,
             hipStream_t s) {
    const long long n = p->g.Nreal;
    long long total = 0;
    int rc = VOFL_OK;
    for (int b = 0; b < p->g.batch && rc == VOFL_OK; ++b) {
        p->coef_item = b;
        long long it = 0;
        rc = cnfp_solve<T>(p, up + b * n, u + b * n, nsteps, tol, max_iter, &it, s);
        total += it;
    }
    p->coef_item = 0;
    if (iters) *iters = total;
    return rc;
}

template <typename T>
int cnfp_solve(vofl_plan_s* p, T* up, T* u, int nsteps, double tol, int max_iter, long long* iters,
               hipStream_t s) {
    const long long n = p->g.Nreal;
    T* V = (T*)p->cnv;
    T *r = V, *w = V + n, *x = V + 2 * n, *b = V + 3 * n, *res = V + 4 * n, *rh = V + 5 * n, *pv = V + 6 * n,
      *vv = V + 7 * n, *sv = V + 8 * n, *tv = V + 9 * n, *lw = V + 10 * n;
    double* part = p->cns;
    double* dres = p->cns + 2 * Launch<T>::dot_blocks;
    const SolveScalars sc = p->sc_host[sc_off(p)];
    const double kap = sc.kappa0, lam = sc.lambda;
    const double a = 0.5 * kap * p->dt * p->dt, bb = 0.5 * p->dt * p->dt;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t ee) { if (e == hipSuccess) e = ee; };
    auto L = [&](const T* in, T* out) { return apply_any<T>(p, VOFL_OP_S1, in, out, 1, s); };
    // (I + a L) in -> out, with lw as scratch
    auto A = [&](const T* in, T* out) {
        int rc = L(in, lw);
        if (rc) return rc;
        chk(Launch<T>::lincomb(out, in, 1.0, lw, a, nullptr, 0.0, nullptr, 0.0, n, s));
        return e == hipSuccess ? VOFL_OK : hip_fail(e, "lincomb");
    };
    double host2[2];
    auto dot2 = [&](const T* a0, const T* b0, const T* a1, const T* b1) -> int {
        chk(Launch<T>::dot2(a0, b0, a1, b1, n, part, dres, s));
        if (e == hipSuccess) chk(hipMemcpyAsync(host2, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        if (e == hipSuccess) chk(hipStreamSynchronize(s));
        return e == hipSuccess ? VOFL_OK : hip_fail(e, "dot product");
    };
    long long total = 0;
    int rc;
    for (int step = 0; step < nsteps; ++step) {
        // r = 2u - up - a L up + b lambda up^3
        if ((rc = L(up, lw))) return rc;
        chk(Launch<T>::lincomb(r, u, 2.0, up, -1.0, lw, -a, up, bb * lam, n, s));
        chk(Launch<T>::lincomb(w, u, 2.0, up, -1.0, nullptr, 0.0, nullptr, 0.0, n, s));
        if (e != hipSuccess) return hip_fail(e, "lincomb");
        bool outer_done = false;
        for (int outer = 0; outer < 100 && !outer_done; ++outer) {
            // b = r + b lambda w^3; x0 = w
            chk(Launch<T>::lincomb(b, r, 1.0, nullptr, 0.0, nullptr, 0.0, w, bb * lam, n, s));
            chk(Launch<T>::lincomb(x, w, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr, 0.0, n, s));
            if ((rc = A(x, res))) return rc;
            chk(Launch<T>::lincomb(res, b, 1.0, res, -1.0, nullptr, 0.0, nullptr, 0.0, n, s));
            chk(Launch<T>::lincomb(rh, res, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr, 0.0, n, s));
            if ((rc = dot2(b, b, res, res))) return rc;
            const double bnorm = std::sqrt(host2[0]);
            double rr = host2[1];
            double rho = 1.0, alpha = 1.0, omega = 1.0;
            bool conv = std::sqrt(rr) <= tol * bnorm;
            for (int it = 0; it < max_iter && !conv; ++it) {
                ++total;
                if ((rc = dot2(rh, res, nullptr, nullptr))) return rc;
                const double rho_new = host2[0];
                if (it == 0) {
                    chk(Launch<T>::lincomb(pv, res, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr, 0.0, n, s));
                } else {
                    const double beta = (rho_new / rho) * (alpha / omega);
                    // p = r + beta (p - omega v)
                    chk(Launch<T>::lincomb(pv, res, 1.0, pv, beta, vv, -beta * omega, nullptr, 0.0, n, s));
                }
                rho = rho_new;
                if ((rc = A(pv, vv))) return rc;
                if ((rc = dot2(rh, vv, nullptr, nullptr))) return rc;
                alpha = rho / host2[0];
                chk(Launch<T>::lincomb(sv, res, 1.0, vv, -alpha, nullptr, 0.0, nullptr, 0.0, n, s));
                if ((rc = dot2(sv, sv, nullptr, nullptr))) return rc;
                if (std::sqrt(host2[0]) <= tol * bnorm) {
                    chk(Launch<T>::lincomb(x, x, 1.0, pv, alpha, nullptr, 0.0, nullptr, 0.0, n, s));
                    conv = true;
                    break;
                }
                if ((rc = A(sv, tv))) return rc;
                if ((rc = dot2(tv, sv, tv, tv))) return rc;
                omega = host2[0] / host2[1];
                chk(Launch<T>::lincomb(x, x, 1.0, pv, alpha, sv, omega, nullptr, 0.0, n, s));
                chk(Launch<T>::lincomb(res, sv, 1.0, tv, -omega, nullptr, 0.0, nullptr, 0.0, n, s));
                if ((rc = dot2(res, res, nullptr, nullptr))) return rc;
                if (!std::isfinite(host2[0])) break;
                conv = std::sqrt(host2[0]) <= tol * bnorm;
            }
            if (!conv) return fail(VOFL_ERR_UNSTABLE, "BiCGSTAB did not reach the tolerance in %d iterations", max_iter);
            // fixed point on f(w): stop when the iterate no longer moves
            chk(Launch<T>::lincomb(lw, x, 1.0, w, -1.0, nullptr, 0.0, nullptr, 0.0, n, s));
            if ((rc = dot2(lw, lw, x, x))) return rc;
            outer_done = std::sqrt(host2[0]) <= tol * std::sqrt(host2[1]) || lam == 0.0;
            chk(Launch<T>::lincomb(w, x, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr, 0.0, n, s));
            if (e != hipSuccess) return hip_fail(e, "lincomb");
        }
        if (!outer_done) return fail(VOFL_ERR_UNSTABLE, "fixed-point iteration on f(u) did not converge");
        // (up, u) <- (u, w)
        chk(Launch<T>::lincomb(up, u, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr, 0.0, n, s));
        chk(Launch<T>::lincomb(u, w, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr, 0.0, n, s));
        if (e != hipSuccess) return hip_fail(e, "lincomb");
    }
    if (iters) *iters = total;
    return VOFL_OK;
}

template <typename T>
int step_any(vofl_plan_s* p, void* u, void* v, int nsteps, hipStream_t s) {
    if (p->g.ndim >= 2) return step_multi<T>(p, (T*)u, (T*)v, nsteps, s);
    Args1D<T> a = args_1d<T>(p);
    a.u_in = (const T*)u;
    a.v_in = (const T*)v;
    a.u_out = (T*)u;
    a.v_out = (T*)v;
    a.nsteps = nsteps;
    hipError_t e = p->timed("1d_step", s, [&] { return Launch<T>::d1_step(a.N, a, p->g.batch, s); });
    if (e != hipSuccess) return hip_fail(e, "1d step launch");
    return VOFL_OK;
}

// Resumable run in 1D: (u, v) are kept in the plan's run buffers between
// calls, and every advance is one vofl_step on them (the 1D step kernel
// keeps the spectral state in registers within a call).
template <typename T>
int run_begin_any(vofl_plan_s* p, const void* u, const void* v, hipStream_t s) {
    if (p->g.ndim >= 2) return run_begin_multi<T>(p, (const T*)u, (const T*)v, s);
    const size_t bytes = (size_t)p->g.batch * p->g.Nreal * sizeof(T);
    hipError_t e = hipMemcpyAsync(p->U, u, bytes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(p->V, v, bytes, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? VOFL_OK : hip_fail(e, "run copy");
}

template <typename T>
int run_advance_any(vofl_plan_s* p, int nsteps, int phase, hipStream_t s) {
    if (p->g.ndim >= 2) return run_advance_multi<T>(p, nsteps, phase, s);
    return step_any<T>(p, p->U, p->V, nsteps, s);
}

template <typename T>
int run_end_any(vofl_plan_s* p, void* u, void* v, int phase, hipStream_t s) {
    if (p->g.ndim >= 2) return run_end_multi<T>(p, (T*)u, (T*)v, phase, s);
    const size_t bytes = (size_t)p->g.batch * p->g.Nreal * sizeof(T);
    hipError_t e = hipMemcpyAsync(u, p->U, bytes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(v, p->V, bytes, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? VOFL_OK : hip_fail(e, "run copy");
}

}  // namespace

namespace vofl {
// error reporting for the entry points defined outside this file (noalloc.hip,
// stream_probe.hip)
int api_fail(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace vofl

// ---------------------------------------------------------------------------
// autotuning of the axis-0 and middle-axis kernel variants
// ---------------------------------------------------------------------------
std::string tune_key(const vofl_plan_s* p) {
    std::ostringstream k;
    k << "vofl3 ndim=" << p->g.ndim << " n=" << p->g.n[0] << "x" << p->g.n[1] << "x" << p->g.n[2]
      << " M=" << p->M << " prec=" << p->precision << " model=" << p->model << " batch=" << p->g.batch;
    return k.str();
}

bool tune_cache_lookup(vofl_plan_s* p, const std::string& key) {
    const char* path = std::getenv("VOFL_TUNE_CACHE");
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const size_t bar = line.find(" | ");
        if (bar == std::string::npos || line.substr(0, bar) != key) continue;
        std::istringstream rest(line.substr(bar + 3));
        int c = 0, m = 0, cv = 0;
        double ms = 0;
        if (rest >> c >> m >> cv >> ms) {
            p->c2r_variant = c;                    // a variant without a kernel runs as 0
            p->mid_variant = (m >= 0 && m <= 2) ? m : 0;
            p->contig_variant = cv == 1 ? 1 : 0;   // likewise
            p->tuned_ms = ms;
            found = true;  // the last matching line wins
        }
    }
    return found;
}

// Time each candidate over `steps` TSFP2 steps on temporary zero fields and
// keep the fastest. Runs inside vofl_plan (the only place that allocates).
template <typename T>
int autotune(vofl_plan_s* p, int steps) {
    const Geometry& g = p->g;
    if (g.ndim < 2) return VOFL_OK;
    const std::string key = tune_key(p);
    if (tune_cache_lookup(p, key)) return VOFL_OK;
    const size_t bytes = (size_t)g.batch * g.Nreal * sizeof(T);
    T* u = nullptr;
    T* v = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&u, bytes);
    if (e == hipSuccess) e = hipMalloc(&v, bytes);
    if (e == hipSuccess) e = hipMemset(u, 0, bytes);
    if (e == hipSuccess) e = hipMemset(v, 0, bytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();  // zero fields and tables in place before s runs
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int rc = (e == hipSuccess) ? VOFL_OK : hip_fail(e, "autotune setup");
    std::vector<int> c2r, mid;
    for (int c : {0, 2, 5, 6, 11, 12, 13, 14})
        if (Launch<T>::c2r_variant_exists(g.n[0], c)) c2r.push_back(c);
    mid.push_back(0);
    if (g.ndim == 3)
        for (int m = 1; m <= 2; ++m)
            if (Launch<T>::mid_tile(g.n[1], m) != Launch<T>::mid_tile(g.n[1], m - 1)) mid.push_back(m);
    const bool timing = p->timing;
    p->timing = false;
    double best = 1e300;
    int bc = p->c2r_variant, bm = p->mid_variant, bv = p->contig_variant;
    // one candidate: (axis-0 variant, middle-axis tile, last-axis schedule)
    auto time_one = [&](int c, int m, int cv) {
        if (rc) return;
        p->c2r_variant = c;
        p->mid_variant = m;
        p->contig_variant = cv;
        rc = step_any<T>(p, u, v, 1, s);
        if (rc) return;
        (void)hipEventRecord(e0, s);
        rc = step_any<T>(p, u, v, steps, s);
        (void)hipEventRecord(e1, s);
        if (rc) return;
        e = hipEventSynchronize(e1);
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune run");
            return;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            bc = c;
            bm = m;
            bv = cv;
        }
    };
    // axis-0 variants x middle-axis tiles with the default last-axis schedule,
    // then the last-axis schedules (elements per thread, hence radices) with
    // the best pair
    for (int c : c2r)
        for (int m : mid) time_one(c, m, 0);
    if (Launch<T>::contig_variant_exists(g.nlast, 1)) time_one(bc, bm, 1);
    p->timing = timing;
    p->c2r_variant = bc;
    p->mid_variant = bm;
    p->contig_variant = bv;
    p->tuned_ms = (best < 1e300) ? best / steps : 0.0;
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (u) (void)hipFree(u);
    if (v) (void)hipFree(v);
    (void)hipMemset(p->flag, 0, 256);
    (void)hipDeviceSynchronize();
    if (rc == VOFL_OK) {
        if (const char* path = std::getenv("VOFL_TUNE_CACHE")) {
            std::ofstream f(path, std::ios::app);
            f << key << " | " << bc << " " << bm << " " << bv << " " << p->tuned_ms << "\n";
        }
    }
    return rc;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* vofl_last_error(void) { return g_err.c_str(); }

const char* vofl_version(void) { return "vofl 0.1 (gfx950)"; }

int vofl_plan_footprint(const vofl_desc* desc, size_t* bytes) {
    Geometry g;
    int rc = derive(desc, g);
    if (rc) return rc;
    if (!bytes) return fail(VOFL_ERR_INVALID, "bytes is NULL");
    *bytes = g.bytes;
    return VOFL_OK;
}

int vofl_plan(const vofl_desc* d, void* stream, vofl_plan_t* out) {
    (void)stream;
    if (!out) return fail(VOFL_ERR_INVALID, "out is NULL");
    *out = nullptr;
    Geometry g;
    int rc = derive(d, g);
    if (rc) return rc;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(VOFL_ERR_DEVICE, "no HIP device available");
    }
    // FP64 coefficient maps on the host (Section 1 coefficients of (1.1);
    // grid means of gamma or s; delta = field - mean)
    const long long N = g.Nreal;
    const int ncoef = g.ncoef;
    std::vector<double> delta((size_t)ncoef * N), A((size_t)ncoef * N), B((size_t)ncoef * N);
    std::vector<SolveScalars> sc(ncoef);
    for (int c = 0; c < ncoef; ++c) {
        const long long off = (long long)c * N;
        std::vector<double> f(N);
        parallel_for(N, [&](long long i) {
            if (d->model == VOFL_MODEL_GENERIC) f[i] = d->s[off + i];
            else if (d->Q) f[i] = std::atan2(1.0, d->Q[off + i]) / M_PI;
            else f[i] = d->gamma[off + i];
        });
        long double sum = 0.0L;
        for (long long i = 0; i < N; ++i) sum += f[i];
        const double mean = (double)(sum / (long double)N);
        SolveScalars s{};
        if (d->model == VOFL_MODEL_GENERIC) {
            for (long long i = 0; i < N; ++i) {
                delta[off + i] = f[i] - mean;
                A[off + i] = d->kappa;
                B[off + i] = 0.0;
            }
            s.sig1 = mean;
            s.sig2 = 0.0;
            s.kappa0 = d->kappa;
            s.beta0 = 0.0;
            s.lambda = d->lambda;
        } else {
            // per-point phase velocity (layered media) or the scalar c0; the
            // exact part uses the grid mean of c0
            const double* cf = d->c0_field ? d->c0_field + off : nullptr;
            parallel_for(N, [&](long long i) {
                delta[off + i] = f[i] - mean;
                seismic_AB(f[i], cf ? cf[i] : d->c0, d->omega0, A[off + i], B[off + i]);
            });
            double cbar = d->c0;
            if (cf) {
                long double cs = 0.0L;
                for (long long i = 0; i < N; ++i) cs += cf[i];
                cbar = (double)(cs / (long double)N);
            }
            double k0, b0;
            seismic_AB(mean, cbar, d->omega0, k0, b0);
            s.sig1 = 1.0 + mean;
            s.sig2 = 0.5 + mean;
            s.kappa0 = k0;
            s.beta0 = b0;
        }
        sc[c] = s;
    }
    vofl_plan_s* p = new vofl_plan_s();
    p->g = g;
    p->model = d->model;
    p->precision = d->precision;
    p->M = d->M;
    p->dt = d->dt;
    for (int i = 0; i < 3; ++i) {
        p->lo[i] = d->lo[i];
        p->hi[i] = d->hi[i];
    }
    p->sc_host = sc;
    if (d->order == 4) {
        // fourth-order composition of three TSFP2 steps (symmetric triple jump)
        const double c = std::cbrt(2.0);
        p->sub = 3;
        p->w1 = 1.0 / (2.0 - c);
        p->w0 = -c / (2.0 - c);
    }
    // default axis-0 kernel: each stored row loaded once (see c2r_default)
    if (g.ndim >= 2)
        p->c2r_variant = (d->precision == VOFL_FP32) ? Launch<float>::c2r_default(g.n[0])
                                                     : Launch<double>::c2r_default(g.n[0]);
    if (const char* ev = std::getenv("VOFL_C2R_VARIANT")) p->c2r_variant = std::atoi(ev);
    if (const char* ev = std::getenv("VOFL_CONTIG_VARIANT")) p->contig_variant = std::atoi(ev) == 1 ? 1 : 0;
    if (const char* ev = std::getenv("VOFL_MID_VARIANT")) {
        // only 0, 1, 2 exist; the launcher's grid and kernel tile must agree
        const int v = std::atoi(ev);
        p->mid_variant = (v >= 0 && v <= 2) ? v : 0;
    }
    rc = (d->precision == VOFL_FP32) ? upload_tables<float>(p, delta, A, B)
                                     : upload_tables<double>(p, delta, A, B);
    if (rc == VOFL_OK && d->tune_steps > 0)
        rc = (d->precision == VOFL_FP32) ? autotune<float>(p, d->tune_steps) : autotune<double>(p, d->tune_steps);
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    return VOFL_OK;
}

int vofl_destroy(vofl_plan_t plan) {
    if (!plan) return fail(VOFL_ERR_INVALID, "plan is NULL");
    (void)hipDeviceSynchronize();
    delete plan;
    return VOFL_OK;
}

int vofl_apply(vofl_plan_t p, int op, const void* u, void* out, int nfields, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    p->run = 0;  // these calls reuse the buffers that hold a resumable run
    if (!u || !out) return fail(VOFL_ERR_INVALID, "u and out must be device pointers");
    if (u == out) return fail(VOFL_ERR_INVALID, "out must not alias u");
    if (op != VOFL_OP_S1 && op != VOFL_OP_S2) return fail(VOFL_ERR_INVALID, "op must be VOFL_OP_S1 or VOFL_OP_S2");
    if (op == VOFL_OP_S2 && p->model == VOFL_MODEL_GENERIC)
        return fail(VOFL_ERR_INVALID, "VOFL_OP_S2 belongs to the seismic model");
    if (nfields < 1 || nfields > p->g.max_batch) return fail(VOFL_ERR_INVALID, "nfields must be in [1, max_batch]");
    if (p->g.ncoef > 1 && nfields > p->g.ncoef)
        return fail(VOFL_ERR_INVALID, "nfields exceeds the number of coefficient fields");
    hipStream_t s = (hipStream_t)stream;
    return p->precision == VOFL_FP32 ? apply_any<float>(p, op, u, out, nfields, s)
                                     : apply_any<double>(p, op, u, out, nfields, s);
}

int vofl_step(vofl_plan_t p, void* u, void* v, int nsteps, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    p->run = 0;  // these calls reuse the buffers that hold a resumable run
    if (!u || !v) return fail(VOFL_ERR_INVALID, "u and v must be device pointers");
    if (u == v) return fail(VOFL_ERR_INVALID, "u and v must be distinct");
    if (nsteps < 0) return fail(VOFL_ERR_INVALID, "nsteps must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    return p->precision == VOFL_FP32 ? step_any<float>(p, u, v, nsteps, s)
                                     : step_any<double>(p, u, v, nsteps, s);
}

int vofl_step_graph(vofl_plan_t p, void* u, void* v, int nsteps, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    p->run = 0;  // these calls reuse the buffers that hold a resumable run
    if (!u || !v) return fail(VOFL_ERR_INVALID, "u and v must be device pointers");
    if (u == v) return fail(VOFL_ERR_INVALID, "u and v must be distinct");
    if (nsteps < 0) return fail(VOFL_ERR_INVALID, "nsteps must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    for (auto& gr : p->graphs)
        if (gr.u == u && gr.v == v && gr.nsteps == nsteps) {
            hipError_t e = hipGraphLaunch(gr.exec, s);
            return e == hipSuccess ? VOFL_OK : hip_fail(e, "graph launch");
        }
    hipError_t e = hipSuccess;
    if (!p->own_stream) {
        e = hipStreamCreateWithFlags(&p->own_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "stream");
    }
    const bool timing = p->timing;
    p->timing = false;  // no event records inside the graph
    e = hipStreamBeginCapture(p->own_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        p->timing = timing;
        return hip_fail(e, "begin capture");
    }
    int rc = p->precision == VOFL_FP32 ? step_any<float>(p, u, v, nsteps, p->own_stream)
                                       : step_any<double>(p, u, v, nsteps, p->own_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(p->own_stream, &graph);
    p->timing = timing;
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    if (p->graphs.size() >= 8) {
        (void)hipDeviceSynchronize();  // the oldest graph may still be running
        (void)hipGraphExecDestroy(p->graphs.front().exec);
        p->graphs.erase(p->graphs.begin());
    }
    p->graphs.push_back({u, v, nsteps, exec});
    e = hipGraphLaunch(exec, s);
    return e == hipSuccess ? VOFL_OK : hip_fail(e, "graph launch");
}

int vofl_step_begin(vofl_plan_t p, const void* u, const void* v, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    if (!u || !v) return fail(VOFL_ERR_INVALID, "u and v must be device pointers");
    p->run = 0;
    hipStream_t s = (hipStream_t)stream;
    const int rc = p->precision == VOFL_FP32 ? run_begin_any<float>(p, u, v, s) : run_begin_any<double>(p, u, v, s);
    if (rc) return rc;
    p->run = 1;
    p->run_steps = 0;
    return VOFL_OK;
}

int vofl_step_advance(vofl_plan_t p, int nsteps, int use_graph, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    if (!p->run) return fail(VOFL_ERR_INVALID, "no run in progress (call vofl_step_begin first)");
    if (nsteps < 0) return fail(VOFL_ERR_INVALID, "nsteps must be >= 0");
    if (nsteps == 0) return VOFL_OK;
    hipStream_t s = (hipStream_t)stream;
    const int phase = p->run;
    auto launch = [&](hipStream_t st) {
        return p->precision == VOFL_FP32 ? run_advance_any<float>(p, nsteps, phase, st)
                                         : run_advance_any<double>(p, nsteps, phase, st);
    };
    int rc = VOFL_OK;
    if (!use_graph) {
        rc = launch(s);
    } else {
        hipGraphExec_t exec = nullptr;
        for (auto& gr : p->run_graphs)
            if (gr.nsteps == nsteps && gr.phase == phase) exec = gr.exec;
        if (!exec) {
            hipError_t e = hipSuccess;
            if (!p->own_stream) {
                e = hipStreamCreateWithFlags(&p->own_stream, hipStreamNonBlocking);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming);
                if (e != hipSuccess) return hip_fail(e, "stream");
            }
            const bool timing = p->timing;
            p->timing = false;  // no event records inside the graph
            e = hipStreamBeginCapture(p->own_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) {
                p->timing = timing;
                return hip_fail(e, "begin capture");
            }
            rc = launch(p->own_stream);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(p->own_stream, &graph);
            p->timing = timing;
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "end capture");
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "graph instantiate");
            if (p->run_graphs.size() >= 8) {
                (void)hipDeviceSynchronize();  // the oldest graph may still be running
                (void)hipGraphExecDestroy(p->run_graphs.front().exec);
                p->run_graphs.erase(p->run_graphs.begin());
            }
            p->run_graphs.push_back({nsteps, phase, exec});
        }
        hipError_t e = hipGraphLaunch(exec, s);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
    }
    if (rc) return rc;
    p->run = 2;
    p->run_steps += nsteps;
    return VOFL_OK;
}

int vofl_step_end(vofl_plan_t p, void* u, void* v, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    if (!p->run) return fail(VOFL_ERR_INVALID, "no run in progress (call vofl_step_begin first)");
    if (!u || !v) return fail(VOFL_ERR_INVALID, "u and v must be device pointers");
    if (u == v) return fail(VOFL_ERR_INVALID, "u and v must be distinct");
    hipStream_t s = (hipStream_t)stream;
    return p->precision == VOFL_FP32 ? run_end_any<float>(p, u, v, p->run, s)
                                     : run_end_any<double>(p, u, v, p->run, s);
}

int vofl_solve(vofl_plan_t p, const void* u0, const void* v0, int nsteps, void* u, void* v, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    if (!u0 || !v0 || !u || !v) return fail(VOFL_ERR_INVALID, "null device pointer");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)p->g.batch * p->g.Nreal * p->g.elt;
    hipError_t e = hipSuccess;
    if (u0 != u) e = hipMemcpyAsync(u, u0, bytes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && v0 != v) e = hipMemcpyAsync(v, v0, bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "initial copy");
    return vofl_step(p, u, v, nsteps, stream);
}

int vofl_lffp_start(vofl_plan_t p, const void* phi, const void* psi, void* u_prev, void* u, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    p->run = 0;  // these calls reuse the buffers that hold a resumable run
    if (!phi || !psi || !u_prev || !u) return fail(VOFL_ERR_INVALID, "phi, psi, u_prev and u must be device pointers");
    if (u_prev == u) return fail(VOFL_ERR_INVALID, "u_prev and u must be distinct");
    hipStream_t s = (hipStream_t)stream;
    const double dt = p->dt;
    // (prev, cur) = (psi, phi): u^1 = phi + dt psi + dt^2/2 F(phi, w = psi)
    return p->precision == VOFL_FP32
               ? lffp_any<float>(p, phi, psi, u, u_prev, 1.0, dt, 0.5 * dt * dt, 0.0, 1.0, 1, s)
               : lffp_any<double>(p, phi, psi, u, u_prev, 1.0, dt, 0.5 * dt * dt, 0.0, 1.0, 1, s);
}

int vofl_lffp_step(vofl_plan_t p, void* u_prev, void* u, int nsteps, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    p->run = 0;  // these calls reuse the buffers that hold a resumable run
    if (!u_prev || !u) return fail(VOFL_ERR_INVALID, "u_prev and u must be device pointers");
    if (u_prev == u) return fail(VOFL_ERR_INVALID, "u_prev and u must be distinct");
    if (nsteps < 0) return fail(VOFL_ERR_INVALID, "nsteps must be >= 0");
    if (nsteps == 0) return VOFL_OK;
    hipStream_t s = (hipStream_t)stream;
    const double dt2 = p->dt * p->dt, idt = 1.0 / p->dt;
    return p->precision == VOFL_FP32
               ? lffp_any<float>(p, u, u_prev, u, u_prev, 2.0, -1.0, dt2, idt, -idt, nsteps, s)
               : lffp_any<double>(p, u, u_prev, u, u_prev, 2.0, -1.0, dt2, idt, -idt, nsteps, s);
}

int vofl_cnfp_step(vofl_plan_t p, void* u_prev, void* u, int nsteps, double tol, int max_iter,
                   long long* iterations, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    p->run = 0;  // these calls reuse the buffers that hold a resumable run
    if (!u_prev || !u) return fail(VOFL_ERR_INVALID, "u_prev and u must be device pointers");
    if (u_prev == u) return fail(VOFL_ERR_INVALID, "u_prev and u must be distinct");
    if (nsteps < 0) return fail(VOFL_ERR_INVALID, "nsteps must be >= 0");
    if (!(tol > 0.0 && tol < 1.0)) return fail(VOFL_ERR_INVALID, "tol must be in (0, 1)");
    if (max_iter < 1) return fail(VOFL_ERR_INVALID, "max_iter must be >= 1");
    if (p->model != VOFL_MODEL_GENERIC)
        return fail(VOFL_ERR_UNSUPPORTED, "the Crank-Nicolson scheme is provided for the generic model (1.5)");
    if (iterations) *iterations = 0;
    if (nsteps == 0) return VOFL_OK;
    hipStream_t s = (hipStream_t)stream;
    return p->precision == VOFL_FP32
               ? cnfp_run<float>(p, (float*)u_prev, (float*)u, nsteps, tol, max_iter, iterations, s)
               : cnfp_run<double>(p, (double*)u_prev, (double*)u, nsteps, tol, max_iter, iterations, s);
}

int vofl_step_batch(vofl_plan_t* plans, void** u, void** v, const int* nsteps, int count, void* stream) {
    if (!plans || !u || !v || !nsteps || count < 0) return fail(VOFL_ERR_INVALID, "null argument");
    hipStream_t s = (hipStream_t)stream;
    // fork: every plan runs on its own stream after the caller's prior work
    hipEvent_t start = nullptr;
    hipError_t e = hipEventCreateWithFlags(&start, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "event");
    (void)hipEventRecord(start, s);
    int rc = VOFL_OK;
    for (int i = 0; i < count && rc == VOFL_OK; ++i) {
        vofl_plan_s* p = plans[i];
        if (!p) {
            rc = fail(VOFL_ERR_INVALID, "plans[%d] is NULL", i);
            break;
        }
        if (!p->own_stream) {
            e = hipStreamCreateWithFlags(&p->own_stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming);
            if (e != hipSuccess) {
                rc = hip_fail(e, "stream");
                break;
            }
        }
        (void)hipStreamWaitEvent(p->own_stream, start, 0);
        rc = vofl_step(p, u[i], v[i], nsteps[i], p->own_stream);
        (void)hipEventRecord(p->join_ev, p->own_stream);
    }
    for (int i = 0; i < count; ++i)
        if (plans[i] && plans[i]->join_ev) (void)hipStreamWaitEvent(s, plans[i]->join_ev, 0);
    (void)hipEventDestroy(start);
    return rc;
}

int vofl_sync_status(vofl_plan_t p, void* stream) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    int flag = 0;
    e = hipMemcpy(&flag, p->flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "flag read");
    if (flag) {
        e = hipMemset(p->flag, 0, sizeof(int));
        if (e != hipSuccess) return hip_fail(e, "flag reset");
        return fail(VOFL_ERR_UNSTABLE, "non-finite value during a step (time step above the stability limit?)");
    }
    return VOFL_OK;
}

int vofl_set_timing(vofl_plan_t p, int enable) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    p->timing = enable != 0;
    if (enable) p->totals.clear();
    return VOFL_OK;
}

int vofl_kernel_times(vofl_plan_t p, const char** names, double* ms, long long* launches, int cap) {
    if (!p) return fail(VOFL_ERR_INVALID, "plan is NULL");
    p->drain_timing();
    int k = 0;
    for (auto& kv : p->totals) {
        if (k < cap) {
            if (names) names[k] = p->cls_names[kv.first].c_str();
            if (ms) ms[k] = kv.second.first;
            if (launches) launches[k] = kv.second.second;
        }
        ++k;
    }
    return k;
}

int vofl_plan_info(vofl_plan_t p, double* out, int cap) {
    if (!p || !out) return fail(VOFL_ERR_INVALID, "null argument");
    const double v[8] = {p->model == VOFL_MODEL_GENERIC ? p->sc_host[0].sig1 : p->sc_host[0].sig1 - 1.0,
                         p->sc_host[0].kappa0, p->sc_host[0].beta0, (double)p->g.Nreal, (double)p->g.bytes,
                         (double)p->c2r_variant, (double)p->mid_variant, (double)p->contig_variant};
    for (int i = 0; i < cap && i < 8; ++i) out[i] = v[i];
    return VOFL_OK;
}

}  // extern "C"
