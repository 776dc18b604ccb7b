// fl_api.hip -- the C-ABI entry points: argument checks, operator lifetime,
// the matvec entry and host copies of the coefficients and eigenvalues.
#include <cmath>
#include <cstdarg>
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "fl_internal.hpp"

namespace fl {

static thread_local char g_err[512] = {0};

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

fl_status build_coeffs(fl_op op, hipStream_t s);

static int next_pow2(long x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// exp(-2 pi i m / P) for m < P, computed in long double and rounded
static fl_status make_twiddles(fl_op op) {
    const int P = op->P;
    std::vector<double2> t64(P);
    std::vector<float2> t32(P);
    const long double tau = 6.283185307179586476925286766559005768L;
    for (int m = 0; m < P; ++m) {
        long double ang = tau * (long double)m / (long double)P;
        long double c = cosl(ang), s = -sinl(ang);
        // exact values at the quarter turns
        if (m * 4 % P == 0) {
            int q = m * 4 / P;
            c = q == 0 ? 1.0L : q == 2 ? -1.0L : 0.0L;
            s = q == 1 ? -1.0L : q == 3 ? 1.0L : 0.0L;
        }
        t64[m].x = (double)c;
        t64[m].y = (double)s;
        t32[m].x = (float)c;
        t32[m].y = (float)s;
    }
    FL_HIP_TRY(hipMalloc((void **)&op->tw64, sizeof(double2) * P));
    FL_HIP_TRY(hipMalloc((void **)&op->tw32, sizeof(float2) * P));
    if (!large_op(op)) {
        FL_HIP_TRY(hipMalloc((void **)&op->sch64, sizeof(double2) * sched_len(P)));
        FL_HIP_TRY(hipMalloc((void **)&op->sch32, sizeof(float2) * sched_len(P)));
    }
    FL_HIP_TRY(hipMemcpy(op->tw64, t64.data(), sizeof(double2) * P, hipMemcpyHostToDevice));
    FL_HIP_TRY(hipMemcpy(op->tw32, t32.data(), sizeof(float2) * P, hipMemcpyHostToDevice));
    return FL_OK;
}

void free_solver_workspace(fl_op op);

static void destroy(fl_op op) {
    if (!op) return;
    (void)hipFree(op->a);
    (void)hipFree(op->lam64);
    (void)hipFree(op->lam64t);
    (void)hipFree(op->lam32t);
    (void)hipFree(op->tw64);
    (void)hipFree(op->tw32);
    (void)hipFree(op->sch64);
    (void)hipFree(op->sch32);
    (void)hipFree(op->T1);
    (void)hipFree(op->T2);
    (void)hipFree(op->mu64t);
    (void)hipFree(op->mu32t);
    free_solver_workspace(op);
    delete op;
}

// Nk: intervals per axis (x first) of a box; nullptr for the square of N per axis.
// The coefficients and the symbol are those of the square of side L = N h,
// N = max Nk (Sec. 2 takes L as the longest side and N_x = N); the box keeps
// Nk - 1 interior nodes per axis.
static fl_status create(int d, double alpha, double gamma, double h, int N, const int *Nk, fl_op *out) {
    fl_op op = new (std::nothrow) fl_op_s();
    if (!op) {
        set_error("host allocation failed");
        return FL_E_NOMEM;
    }
    op->d = d;
    op->N = N;
    op->n = N - 1;
    op->alpha = alpha;
    op->gamma = gamma;
    op->h = h;
    op->c = std::pow(2.0, alpha - 1.0) * alpha * std::tgamma(0.5 * (d + alpha)) /
            (std::pow(M_PI, 0.5 * d) * std::tgamma(1.0 - 0.5 * alpha));
    op->P = next_pow2(2L * op->n - 1);
    if (op->P < 8) op->P = 8;
    op->Q = op->P / 2 + 1;
    op->Qp = ((op->Q + 31) / 32) * 32;  // a whole number of the four-step passes' 32-column groups
    for (int k = 0; k < 3; ++k) op->nk[k] = k >= d ? 1 : (Nk ? Nk[k] - 1 : op->n);
    op->M = (int64_t)op->nk[0] * op->nk[1] * op->nk[2];
    (void)hipGetDevice(&op->device);
    const long V = N + 1;
    long nv = 1, ql = 1;
    for (int k = 0; k < d; ++k) {
        nv *= V;
        ql *= op->Q;
    }
    const long qrest = ql / op->Q;
    // tiled spectra: ntiles * C <= Q + C - 1 columns per line, sized for the
    // widest tile and 16-byte (FP64) values; lines: the x pass's rows (T1),
    // the z lines times P y frequencies (T2, 3D).  Large operators (FFT length
    // above the LDS path's) instead hold two P x Qp complex work buffers and
    // lambda in natural order only (Q x Q, with an FP32 copy).
    const long w32 = op->Q + kMaxTile - 1, w64 = op->Q + kMaxTile - 1;
    const size_t colb = sizeof(double2) * w64;
    const bool large = large_op(op);
    const long lam64t_len = large ? 0 : qrest * w64, lam32t_len = large ? ql : qrest * w32;
    if (large) {
        op->T1_bytes = op->T2_bytes = sizeof(double2) * (size_t)op->P * op->Qp;
    } else {
        op->T1_bytes = colb * (size_t)op->nk[1] * op->nk[2];
        op->T2_bytes = d != 3 ? 0 : colb * (size_t)op->nk[2] * op->P;
    }
    fl_status st = FL_OK;
    auto fail = [&](fl_status s) {
        destroy(op);
        return s;
    };
    hipError_t e;
    if ((e = hipMalloc((void **)&op->a, sizeof(double) * nv)) != hipSuccess ||
        (e = hipMalloc((void **)&op->lam64, sizeof(double) * ql)) != hipSuccess ||
        (lam64t_len && (e = hipMalloc((void **)&op->lam64t, sizeof(double) * lam64t_len)) != hipSuccess) ||
        (e = hipMalloc((void **)&op->lam32t, sizeof(float) * lam32t_len)) != hipSuccess ||
        (e = hipMalloc(&op->T1, op->T1_bytes)) != hipSuccess ||
        (op->T2_bytes && (e = hipMalloc(&op->T2, op->T2_bytes)) != hipSuccess)) {
        set_error("device allocation: %s", hipGetErrorString(e));
        return fail(e == hipErrorOutOfMemory ? FL_E_NOMEM : FL_E_DEVICE);
    }
    if ((st = make_twiddles(op)) != FL_OK) return fail(st);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        set_error("stream creation failed");
        return fail(FL_E_DEVICE);
    }
    st = make_schedules(op, s);
    if (st == FL_OK) st = build_coeffs(op, s);
    if (st == FL_OK) st = build_symbol(op, s);
    if (st == FL_OK) {
        e = hipMemcpyAsync(&op->a0, op->a, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_error("reading a_0: %s", hipGetErrorString(e));
            st = FL_E_DEVICE;
        }
    }
    (void)hipStreamDestroy(s);
    if (st != FL_OK) return fail(st);
    *out = op;
    return FL_OK;
}

static bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

}  // namespace fl

using namespace fl;

// ---------------------------------------------------------------------------
// the autotuner's choices on disk, keyed by (d, FFT length, precision): one
// line "fl-tune 1 <d> <P> <prec> <variants> <best> <ms>" per tuning.  The file
// is $FL_TUNE_CACHE, else $HOME/.cache/fl_tune_gfx950.txt; an empty
// FL_TUNE_CACHE turns caching and tuning off (variant 0).  A line whose
// variant count differs from the built tables is ignored; the last matching
// line wins.  Appends are whole lines, so concurrent writers at worst repeat a key.
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;

static bool tune_path(std::string *path) {
    const char *env = std::getenv("FL_TUNE_CACHE");
    if (env) {
        *path = env;
        return !path->empty();
    }
    const char *home = std::getenv("HOME");
    if (!home || !*home) return false;
    *path = std::string(home) + "/.cache/fl_tune_gfx950.txt";
    return true;
}

static int tune_lookup(const std::string &path, int d, int P, int prec, int nv) {
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return -1;
    int found = -1;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        int ver = 0, dd = 0, pp = 0, pr = 0, n = 0, best = 0;
        float ms = 0.f;
        if (std::sscanf(line, "fl-tune %d %d %d %d %d %d %f", &ver, &dd, &pp, &pr, &n, &best, &ms) == 7 && ver == 1 &&
            dd == d && pp == P && pr == prec && n == nv && best >= 0 && best < nv)
            found = best;
    }
    std::fclose(f);
    return found;
}

static void tune_record(const std::string &path, int d, int P, int prec, int nv, int best, float ms) {
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "fl-tune 1 %d %d %d %d %d %.6f\n", d, P, prec, nv, best, ms);
    std::fclose(f);
}

namespace fl {
// the variant to use for (op's d and P, prec): from the cache, else timed now
// (fl_autotune, 10 matvecs per variant) and recorded; selects it on op
fl_status tuned_variant(fl_op op, int prec, int *k) {
    *k = 0;
    if (large_op(op)) return FL_OK;
    const int nv = variant_count(op, prec);
    std::string path;
    if (nv <= 1 || !tune_path(&path)) return fl_select_variant(op, prec, 0);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    int best = tune_lookup(path, op->d, op->P, prec, nv);
    if (best >= 0) {
        *k = best;
        return fl_select_variant(op, prec, best);
    }
    std::vector<float> ms(nv);
    hipStream_t s = nullptr;
    FL_HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    fl_status st = fl_autotune(op, prec, 10, s, &best, ms.data());
    (void)hipStreamDestroy(s);
    FL_TRY(st);
    tune_record(path, op->d, op->P, prec, nv, best, ms[best]);
    *k = best;
    return FL_OK;
}
}  // namespace fl

extern "C" {

const char *fl_last_error(void) { return g_err; }

const char *fl_status_string(fl_status s) {
    switch (s) {
        case FL_OK: return "FL_OK";
        case FL_E_INVAL: return "FL_E_INVAL";
        case FL_E_NOMEM: return "FL_E_NOMEM";
        case FL_E_DEVICE: return "FL_E_DEVICE";
        case FL_E_NOCONV: return "FL_E_NOCONV";
        case FL_E_BREAKDOWN: return "FL_E_BREAKDOWN";
        case FL_E_UNSUPPORTED: return "FL_E_UNSUPPORTED";
    }
    return "unknown status";
}

static fl_status check_args(int d, double alpha, double gamma, double h, fl_op *out) {
    if (!(gamma > alpha && gamma <= 2.0)) {
        set_error("gamma must lie in (alpha, 2] (got gamma=%g, alpha=%g)", gamma, alpha);
        return FL_E_INVAL;
    }
    if (!out) { set_error("out is NULL"); return FL_E_INVAL; }
    if (d < 1 || d > 3) { set_error("d must be 1, 2 or 3 (got %d)", d); return FL_E_INVAL; }
    if (!(alpha > 0.0 && alpha < 2.0)) { set_error("alpha must lie in (0,2) (got %g)", alpha); return FL_E_INVAL; }
    if (!(h > 0.0) || !std::isfinite(h)) { set_error("h must be positive and finite"); return FL_E_INVAL; }
    return FL_OK;
}

static fl_status check_N(int d, int N) {
    if (N < 2) { set_error("N must be >= 2 (got %d)", N); return FL_E_INVAL; }
    // FFT lengths up to 2048 in LDS; 2D up to 16384 by the large-operator passes
    const int nmax = d == 2 ? 8193 : (d == 3 ? 513 : 1025);
    if (N > nmax) { set_error("N=%d exceeds the built range (N <= %d for d=%d)", N, nmax, d); return FL_E_UNSUPPORTED; }
    return FL_OK;
}

fl_status fl_coeffs_gamma(int d, double alpha, double gamma, double h, int N, fl_op *out) {
    g_err[0] = 0;
    fl_status st = check_args(d, alpha, gamma, h, out);
    if (st == FL_OK) st = check_N(d, N);
    return st == FL_OK ? create(d, alpha, gamma, h, N, nullptr, out) : st;
}

fl_status fl_coeffs_box(int d, double alpha, double gamma, double h, const int *Nk, fl_op *out) {
    g_err[0] = 0;
    fl_status st = check_args(d, alpha, gamma, h, out);
    if (st != FL_OK) return st;
    if (!Nk) { set_error("Nk is NULL"); return FL_E_INVAL; }
    int N = 0;
    for (int k = 0; k < d; ++k) {
        if (Nk[k] < 2) { set_error("Nk[%d] must be >= 2 (got %d)", k, Nk[k]); return FL_E_INVAL; }
        N = Nk[k] > N ? Nk[k] : N;
    }
    st = check_N(d, N);
    return st == FL_OK ? create(d, alpha, gamma, h, N, Nk, out) : st;
}

fl_status fl_coeffs(int d, double alpha, double h, int N, fl_op *out) {
    if (!(alpha > 0.0 && alpha < 2.0)) {
        g_err[0] = 0;
        set_error("alpha must lie in (0,2) (got %g)", alpha);
        return FL_E_INVAL;
    }
    return fl_coeffs_gamma(d, alpha, 2.0, h, N, out);
}

fl_status fl_op_destroy(fl_op op) {
    destroy(op);
    return FL_OK;
}

fl_status fl_op_describe(fl_op op, fl_op_desc *desc) {
    if (!op || !desc) { set_error("NULL argument"); return FL_E_INVAL; }
    desc->d = op->d;
    desc->N = op->N;
    desc->n = op->n;
    desc->P = op->P;
    desc->Q = op->Q;
    desc->M = op->M;
    desc->alpha = op->alpha;
    desc->h = op->h;
    desc->c = op->c;
    desc->a0 = op->a0;
    desc->gamma = op->gamma;
    for (int k = 0; k < 3; ++k) desc->nk[k] = op->nk[k];
    return FL_OK;
}

fl_status fl_apply(fl_op op, const void *u, void *y, int prec, void *stream) {
    if (!op || !u || !y) { set_error("NULL argument"); return FL_E_INVAL; }
    if (prec != FL_FP64 && prec != FL_FP32) { set_error("prec must be FL_FP64 or FL_FP32"); return FL_E_INVAL; }
    const size_t es = prec == FL_FP64 ? sizeof(double) : sizeof(float);
    if (overlap(u, es * op->M, y, es * op->M)) { set_error("u and y overlap"); return FL_E_INVAL; }
    hipStream_t s = (hipStream_t)stream;
    if (prec == FL_FP64) return matvec<double>(op, (const double *)u, (double *)y, s);
    return matvec<float>(op, (const float *)u, (float *)y, s);
}

fl_status fl_residual(fl_op op, const double *f, const double *u, double *r, void *stream) {
    if (!op || !f || !u || !r) { set_error("NULL argument"); return FL_E_INVAL; }
    if (overlap(u, sizeof(double) * op->M, r, sizeof(double) * op->M)) { set_error("u and r overlap"); return FL_E_INVAL; }
    Epi<double> ep;
    ep.w1 = f;
    ep.a1 = 1.0;
    ep.scale = -1.0;
    return matvec_ex<double>(op, u, r, ep, nullptr, (hipStream_t)stream);
}

fl_status fl_tau_apply(fl_op op, const double *r, double *z, double s0, double s1, void *stream) {
    if (!op || !r || !z) { set_error("NULL argument"); return FL_E_INVAL; }
    if (overlap(r, sizeof(double) * op->M, z, sizeof(double) * op->M)) { set_error("r and z overlap"); return FL_E_INVAL; }
    hipStream_t s = (hipStream_t)stream;
    FL_TRY(tau_prepare(op, s0, s1, s));
    return tau_apply(op, r, z, nullptr, s);
}

fl_status fl_apply_profiled(fl_op op, const void *u, void *y, int prec, int reps, void *stream, float *pass_ms,
                            int *npass) {
    if (!op || !u || !y || !pass_ms || !npass || reps < 1) { set_error("bad argument"); return FL_E_INVAL; }
    if (prec != FL_FP64 && prec != FL_FP32) { set_error("prec must be FL_FP64 or FL_FP32"); return FL_E_INVAL; }
    const size_t es = prec == FL_FP64 ? sizeof(double) : sizeof(float);
    if (overlap(u, es * op->M, y, es * op->M)) { set_error("u and y overlap"); return FL_E_INVAL; }
    if (large_op(op)) { set_error("per-pass timing covers FFT lengths up to %d", kMaxLdsP); return FL_E_UNSUPPORTED; }
    const int np = op->d == 1 ? 1 : op->d == 2 ? 3 : 5;
    hipStream_t s = (hipStream_t)stream;
    constexpr int kChunk = 64;
    std::vector<hipEvent_t> ev(2 * 5 * kChunk);
    const int chunk = reps < kChunk ? reps : kChunk;
    for (int i = 0; i < 2 * np * chunk; ++i) FL_HIP_TRY(hipEventCreate(&ev[i]));
    double acc[5] = {0, 0, 0, 0, 0};
    fl_status st = FL_OK;
    for (int done = 0; done < reps && st == FL_OK; done += chunk) {
        const int k = reps - done < chunk ? reps - done : chunk;
        for (int r = 0; r < k && st == FL_OK; ++r) {
            hipEvent_t *e = ev.data() + 2 * np * r;
            st = prec == FL_FP64 ? matvec_ex<double>(op, (const double *)u, (double *)y, Epi<double>{}, nullptr, s, e)
                                 : matvec_ex<float>(op, (const float *)u, (float *)y, Epi<float>{}, nullptr, s, e);
        }
        if (hipStreamSynchronize(s) != hipSuccess) st = FL_E_DEVICE;
        for (int r = 0; r < k && st == FL_OK; ++r) {
            hipEvent_t *e = ev.data() + 2 * np * r;
            for (int p = 0; p < np; ++p) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, e[2 * p], e[2 * p + 1]) != hipSuccess) st = FL_E_DEVICE;
                acc[p] += ms;
            }
        }
    }
    for (int i = 0; i < 2 * np * chunk; ++i) (void)hipEventDestroy(ev[i]);
    if (st != FL_OK) { set_error("profiled apply failed"); return st; }
    for (int p = 0; p < np; ++p) pass_ms[p] = (float)(acc[p] / reps);
    *npass = np;
    return FL_OK;
}

fl_status fl_variant_count(fl_op op, int prec, int *count) {
    if (!op || !count || (prec != FL_FP64 && prec != FL_FP32)) { set_error("bad argument"); return FL_E_INVAL; }
    *count = variant_count(op, prec);
    return FL_OK;
}

fl_status fl_variant_info(fl_op op, int prec, int k, int *desc4) {
    if (!op || !desc4 || (prec != FL_FP64 && prec != FL_FP32)) { set_error("bad argument"); return FL_E_INVAL; }
    if (k < 0 || k >= variant_count(op, prec)) { set_error("variant %d out of range", k); return FL_E_INVAL; }
    const VariantDesc v = variant_desc(op, prec, k);
    desc4[0] = v.ex;
    desc4[1] = v.ey;
    desc4[2] = v.c;
    desc4[3] = v.lpb;
    desc4[4] = v.kind;
    return FL_OK;
}

fl_status fl_select_variant(fl_op op, int prec, int k) {
    if (!op || (prec != FL_FP64 && prec != FL_FP32)) { set_error("bad argument"); return FL_E_INVAL; }
    hipStream_t s = nullptr;
    FL_HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    fl_status st = select_variant(op, prec, k, s);
    hipError_t e = hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    FL_TRY(st);
    FL_HIP_TRY(e);
    return FL_OK;
}

fl_status fl_autotune(fl_op op, int prec, int reps, void *stream, int *best, float *ms_out) {
    if (!op || reps < 1 || (prec != FL_FP64 && prec != FL_FP32)) { set_error("bad argument"); return FL_E_INVAL; }
    if (large_op(op)) { set_error("no kernel variants above FFT length %d", kMaxLdsP); return FL_E_UNSUPPORTED; }
    const int nv = variant_count(op, prec);
    const size_t es = prec == FL_FP64 ? sizeof(double) : sizeof(float);
    hipStream_t s = (hipStream_t)stream;
    void *buf = nullptr;
    FL_HIP_TRY(hipMalloc(&buf, 2 * es * (size_t)op->M));
    fl_status st = FL_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMemsetAsync(buf, 0, 2 * es * (size_t)op->M, s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        st = FL_E_DEVICE;
    void *u = buf, *y = (char *)buf + es * op->M;
    // two rounds over the variants, each variant's time the smaller of its two:
    // the first variant of a single round ran while the clocks were still
    // rising and always lost a few per cent
    std::vector<float> tmin(nv, 1e30f);
    for (int round = 0; round < 2 && st == FL_OK; ++round) {
        for (int k = 0; k < nv && st == FL_OK; ++k) {
            st = select_variant(op, prec, k, s);
            for (int r = 0; r < 3 + reps && st == FL_OK; ++r) {
                if (r == 3 && hipEventRecord(e0, s) != hipSuccess) st = FL_E_DEVICE;
                st = prec == FL_FP64 ? matvec<double>(op, (const double *)u, (double *)y, s)
                                     : matvec<float>(op, (const float *)u, (float *)y, s);
            }
            float ms = 0.f;
            if (st == FL_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = FL_E_DEVICE;
            ms /= reps;
            if (ms < tmin[k]) tmin[k] = ms;
        }
    }
    int bi = 0;
    for (int k = 0; k < nv; ++k) {
        if (ms_out) ms_out[k] = tmin[k];
        if (tmin[k] < tmin[bi]) bi = k;
    }
    if (st == FL_OK) st = select_variant(op, prec, bi, s);
    (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (st != FL_OK) return st;
    if (best) *best = bi;
    return FL_OK;
}

fl_status fl_tune(fl_op op, int prec, int *variant) {
    if (!op || !variant || (prec != FL_FP64 && prec != FL_FP32)) { set_error("bad argument"); return FL_E_INVAL; }
    return tuned_variant(op, prec, variant);
}

fl_status fl_get_coeffs(fl_op op, double *a_host) {
    if (!op || !a_host) { set_error("NULL argument"); return FL_E_INVAL; }
    const long V = op->N + 1;
    long nv = 1;
    for (int k = 0; k < op->d; ++k) nv *= V;
    FL_HIP_TRY(hipMemcpy(a_host, op->a, sizeof(double) * nv, hipMemcpyDeviceToHost));
    return FL_OK;
}

fl_status fl_get_symbol(fl_op op, double *lam_host) {
    if (!op || !lam_host) { set_error("NULL argument"); return FL_E_INVAL; }
    const long Q = op->Q;
    long ql = 1;
    for (int k = 0; k < op->d; ++k) ql *= Q;
    FL_HIP_TRY(hipMemcpy(lam_host, op->lam64, sizeof(double) * ql, hipMemcpyDeviceToHost));
    return FL_OK;
}

}  // extern "C"
