// fl_solve.hip -- conjugate gradients on K = s0 I + s1 A with the FFT matvec:
//   * the fractional Poisson problem A u = f (Sec. 5.2; K = A),
//   * each semi-implicit Allen--Cahn step (Sec. 5.3; K = I + theta tau eps^2 A).
// CG keeps every scalar on the device: per iteration one matvec, one fused
// dot (p, Kp), one fused update of x and r with the partial (r, r), and one
// fused update of p.  Reductions are two-level with a fixed assignment of
// vector chunks to blocks, so results are bitwise reproducible.  The host
// polls the scalars once per chunk of iterations; a device `done` flag turns
// the remaining launches of a chunk into no-ops.
//
// Mixed precision: the outer loop evaluates r = b - K x in FP64 and stops on
// ||r||_2 <= tol ||b||_2; each inner solve K d = r runs in FP32 (vectors and
// matvec, FP64 dot products) and x += d in FP64.  Plain FP64 CG is the same
// loop with an FP64 inner solve.
#include <chrono>
#include <cmath>

#include "fl_internal.hpp"

namespace fl {

constexpr int kVecBlock = 256;
constexpr int kMaxParts = 1024;

// device scalar slots
enum : int {
    S_RR0 = 0,  // (r, r) ping
    S_RR1 = 1,  // (r, r) pong
    S_DONE = 2,
    S_BRK = 3,
    S_ITER = 4,
    S_TARGET = 5,  // stop when (r, r) <= target
    S_DOT = 6,     // result slot of a standalone dot
    S_COUNT = 16
};

struct VecLayout {
    long n, chunk;
    int blocks;
};
static VecLayout layout(long n) {
    long per = (n + kMaxParts - 1) / kMaxParts;
    long chunk = ((per + 4 * kVecBlock - 1) / (4 * kVecBlock)) * (4 * kVecBlock);
    if (chunk < 4 * kVecBlock) chunk = 4 * kVecBlock;
    int blocks = (int)((n + chunk - 1) / chunk);
    if (blocks < 1) blocks = 1;
    return {n, chunk, blocks};
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int k = kVecBlock / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// every block adds the partials in the same order: identical scalars everywhere
__device__ __forceinline__ double sum_parts(const double *__restrict__ part, int np, double *sh) {
    double a = 0.0;
    for (int i = threadIdx.x; i < np; i += kVecBlock) a += part[i];
    return block_sum(a, sh);
}

template <typename V>
__global__ __launch_bounds__(kVecBlock) void k_dot(const V *__restrict__ a, const V *__restrict__ b, long n, long chunk,
                                                   double *part, const double *done) {
    __shared__ double sh[kVecBlock];
    if (done && *done != 0.0) return;
    const long beg = (long)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
    double acc = 0.0;
    for (long i = beg + threadIdx.x; i < end; i += kVecBlock) acc += (double)a[i] * (double)b[i];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// slot <- sum of partials (single block)
__global__ __launch_bounds__(kVecBlock) void k_finish(const double *part, int np, double *scal, int slot) {
    __shared__ double sh[kVecBlock];
    double s = sum_parts(part, np, sh);
    if (threadIdx.x == 0) scal[slot] = s;
}

// start of a CG run: rr[0] = sum(part), flags cleared, target = rel^2 * rr
__global__ __launch_bounds__(kVecBlock) void k_cg_init(const double *part, int np, double *scal, double rel2,
                                                       double abs2) {
    __shared__ double sh[kVecBlock];
    double s = sum_parts(part, np, sh);
    if (threadIdx.x == 0) {
        scal[S_RR0] = s;
        scal[S_RR1] = s;
        scal[S_ITER] = 0.0;
        scal[S_BRK] = std::isfinite(s) ? 0.0 : 1.0;
        const double tgt = rel2 * s > abs2 ? rel2 * s : abs2;
        scal[S_TARGET] = tgt;
        scal[S_DONE] = (s <= tgt || !std::isfinite(s)) ? 1.0 : 0.0;
    }
}

// alpha = rr / (p, Kp); x += alpha p; r -= alpha Kp; partial (r, r)
template <typename V>
__global__ __launch_bounds__(kVecBlock) void k_cg_xr(V *__restrict__ x, V *__restrict__ r, const V *__restrict__ p,
                                                     const V *__restrict__ kp, long n, long chunk,
                                                     const double *__restrict__ part_pkp, int np, double *part_rr,
                                                     double *scal, int parity) {
    __shared__ double sh[kVecBlock];
    if (scal[S_DONE] != 0.0) return;
    const double pkp = sum_parts(part_pkp, np, sh);
    const double rr = scal[parity ? S_RR1 : S_RR0];
    const double al = rr / pkp;
    if (!(pkp > 0.0) || !std::isfinite(al)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[S_BRK] = 1.0;
            scal[S_DONE] = 1.0;
        }
        return;
    }
    const V a = (V)al;
    const long beg = (long)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
    double acc = 0.0;
    for (long i = beg + threadIdx.x; i < end; i += kVecBlock) {
        x[i] += a * p[i];
        const V ri = r[i] - a * kp[i];
        r[i] = ri;
        acc += (double)ri * (double)ri;
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = s;
}

// beta = rr_new / rr; p = r + beta p; block 0 advances the scalars
template <typename V>
__global__ __launch_bounds__(kVecBlock) void k_cg_p(V *__restrict__ p, const V *__restrict__ r, long n, long chunk,
                                                    const double *__restrict__ part_rr, int np, double *scal,
                                                    int parity) {
    __shared__ double sh[kVecBlock];
    if (scal[S_DONE] != 0.0) return;
    const double rr_new = sum_parts(part_rr, np, sh);
    const double rr = scal[parity ? S_RR1 : S_RR0];
    const double be = rr_new / rr;
    const bool stop = rr_new <= scal[S_TARGET] || !std::isfinite(rr_new);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[parity ? S_RR0 : S_RR1] = rr_new;
        scal[S_ITER] += 1.0;
        if (!std::isfinite(rr_new)) scal[S_BRK] = 1.0;
        if (stop) scal[S_DONE] = 1.0;
    }
    if (stop) return;
    const V b = (V)be;
    const long beg = (long)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
    for (long i = beg + threadIdx.x; i < end; i += kVecBlock) p[i] = r[i] + b * p[i];
}

template <typename D, typename S>
__global__ void k_copy_cast(D *__restrict__ d, const S *__restrict__ s, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        d[i] = (D)s[i];
}

template <typename S>
__global__ void k_axpy_to64(double *__restrict__ x, const S *__restrict__ d, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] += (double)d[i];
}

template <typename V>
__global__ void k_zero(V *__restrict__ x, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = V(0);
}

// Allen--Cahn right-hand side b = u - (1-theta) s A u + tau (u - u^3)
__global__ void k_ac_rhs(const double *__restrict__ u, const double *__restrict__ au, double *__restrict__ b, long n,
                         double tau, double s, double theta) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double ui = u[i];
        b[i] = ui - (1.0 - theta) * s * au[i] + tau * (ui - ui * ui * ui);
    }
}

static inline int ew_grid(long n) {
    long g = (n + 255) / 256;
    return (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

// ---------------------------------------------------------------------------
// solver workspace
// ---------------------------------------------------------------------------
struct Work {
    double *r64, *p64, *kp64, *d64, *b64;
    float *r32, *p32, *kp32, *d32;
    double *partA, *partB;
};

static Work work_of(fl_op op) {
    Work w;
    const long M = op->M;
    double *base = (double *)op->sw;
    w.r64 = base;
    w.p64 = w.r64 + M;
    w.kp64 = w.p64 + M;
    w.d64 = w.kp64 + M;
    w.b64 = w.d64 + M;
    w.partA = w.b64 + M;
    w.partB = w.partA + kMaxParts;
    float *f = (float *)(w.partB + kMaxParts);
    w.r32 = f;
    w.p32 = w.r32 + M;
    w.kp32 = w.p32 + M;
    w.d32 = w.kp32 + M;
    return w;
}

void free_solver_workspace(fl_op op) {
    if (op->sw) (void)hipFree(op->sw);
    if (op->scal) (void)hipFree(op->scal);
    if (op->hscal) (void)hipHostFree(op->hscal);
    op->sw = nullptr;
    op->scal = nullptr;
    op->hscal = nullptr;
}

static fl_status ensure_workspace(fl_op op) {
    if (op->sw) return FL_OK;
    const long M = op->M;
    size_t bytes = sizeof(double) * (5 * M + 2 * kMaxParts) + sizeof(float) * (4 * M + 64);
    FL_HIP_TRY(hipMalloc(&op->sw, bytes));
    op->sw_bytes = bytes;
    FL_HIP_TRY(hipMalloc((void **)&op->scal, sizeof(double) * S_COUNT));
    FL_HIP_TRY(hipHostMalloc((void **)&op->hscal, sizeof(double) * S_COUNT, hipHostMallocDefault));
    return FL_OK;
}

static fl_status read_scalars(fl_op op, hipStream_t s) {
    FL_HIP_TRY(hipMemcpyAsync(op->hscal, op->scal, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, s));
    FL_HIP_TRY(hipStreamSynchronize(s));
    return FL_OK;
}

template <typename V>
static fl_status dot(fl_op op, const V *a, const V *b, double *part, double *out_host, hipStream_t s) {
    VecLayout L = layout(op->M);
    hipLaunchKernelGGL(k_dot<V>, dim3(L.blocks), dim3(kVecBlock), 0, s, a, b, L.n, L.chunk, part, nullptr);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kVecBlock), 0, s, part, L.blocks, op->scal, (int)S_DOT);
    FL_HIP_TRY(hipGetLastError());
    FL_TRY(read_scalars(op, s));
    *out_host = op->hscal[S_DOT];
    return FL_OK;
}

// K v = s0 v + s1 A v (epilogue of the last pass when s0 != 0 or s1 != 1)
template <typename V>
static fl_status apply_K(fl_op op, const V *v, V *kv, double s0, double s1, const double *done, hipStream_t s) {
    Epi<V> ep;
    ep.scale = (V)s1;
    if (s0 != 0.0) {
        ep.w1 = v;
        ep.a1 = (V)s0;
    }
    return matvec_ex<V>(op, v, kv, ep, done, s);
}

// r64 = b - K x in FP64
static fl_status residual64(fl_op op, const double *b, const double *x, double *r, double s0, double s1,
                            hipStream_t s) {
    Epi<double> ep;
    ep.w1 = b;
    ep.a1 = 1.0;
    ep.scale = -s1;
    if (s0 != 0.0) {
        ep.w2 = x;
        ep.a2 = -s0;
    }
    return matvec_ex<double>(op, x, r, ep, nullptr, s);
}

struct CgResult {
    int iters = 0;
    bool breakdown = false;
};

// CG on K d = r from d = 0, in place on (d, r), until (r,r) <= rel^2 (r0,r0)
// or max_it iterations.
template <typename V>
static fl_status cg_run(fl_op op, double s0, double s1, V *d, V *r, V *p, V *kp, double rel, int max_it,
                        int check_every, const Work &w, hipStream_t s, CgResult *res) {
    VecLayout L = layout(op->M);
    const long M = op->M;
    hipLaunchKernelGGL(k_zero<V>, dim3(ew_grid(M)), dim3(256), 0, s, d, M);
    hipLaunchKernelGGL((k_copy_cast<V, V>), dim3(ew_grid(M)), dim3(256), 0, s, p, r, M);
    hipLaunchKernelGGL(k_dot<V>, dim3(L.blocks), dim3(kVecBlock), 0, s, r, r, L.n, L.chunk, w.partB, nullptr);
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(kVecBlock), 0, s, w.partB, L.blocks, op->scal, rel * rel, 0.0);
    FL_HIP_TRY(hipGetLastError());
    const double *done = op->scal + S_DONE;
    int launched = 0;
    int chunk = check_every > 0 ? check_every : 8;
    res->iters = 0;
    res->breakdown = false;
    while (launched < max_it) {
        const int k = chunk < max_it - launched ? chunk : max_it - launched;
        for (int i = 0; i < k; ++i) {
            const int parity = (launched + i) & 1;
            FL_TRY(apply_K<V>(op, p, kp, s0, s1, done, s));
            hipLaunchKernelGGL(k_dot<V>, dim3(L.blocks), dim3(kVecBlock), 0, s, p, kp, L.n, L.chunk, w.partA, done);
            hipLaunchKernelGGL(k_cg_xr<V>, dim3(L.blocks), dim3(kVecBlock), 0, s, d, r, p, kp, L.n, L.chunk,
                               w.partA, L.blocks, w.partB, op->scal, parity);
            hipLaunchKernelGGL(k_cg_p<V>, dim3(L.blocks), dim3(kVecBlock), 0, s, p, r, L.n, L.chunk, w.partB,
                               L.blocks, op->scal, parity);
        }
        FL_HIP_TRY(hipGetLastError());
        launched += k;
        FL_TRY(read_scalars(op, s));
        if (op->hscal[S_DONE] != 0.0) break;
        if (check_every <= 0 && chunk < 128) chunk *= 2;
    }
    FL_TRY(read_scalars(op, s));
    res->iters = (int)op->hscal[S_ITER];
    res->breakdown = op->hscal[S_BRK] != 0.0;
    return FL_OK;
}

// Solve K x = b to ||b - K x|| <= tol ||b||; x holds the initial guess.
// inner64: FP64 inner solves (plain CG), else FP32 inner solves.
static fl_status refine(fl_op op, double s0, double s1, const double *b, double *x, double tol, bool inner64,
                        double inner_tol, int max_iter, int check_every, fl_info *info, hipStream_t s) {
    FL_TRY(ensure_workspace(op));
    Work w = work_of(op);
    const long M = op->M;
    double bb = 0.0;
    FL_TRY(dot<double>(op, b, b, w.partA, &bb, s));
    const double bn = std::sqrt(bb);
    info->iters = 0;
    info->outer_iters = 0;
    info->relres = 0.0;
    if (!std::isfinite(bn)) {
        set_error("right-hand side is not finite");
        info->relres = NAN;
        return FL_E_BREAKDOWN;
    }
    if (bn == 0.0) {
        hipLaunchKernelGGL(k_zero<double>, dim3(ew_grid(M)), dim3(256), 0, s, x, M);
        FL_HIP_TRY(hipGetLastError());
        FL_HIP_TRY(hipStreamSynchronize(s));
        return FL_OK;
    }
    const int max_outer = 200;
    double last = INFINITY;
    int stalls = 0;
    for (int outer = 0;; ++outer) {
        FL_TRY(residual64(op, b, x, w.r64, s0, s1, s));
        double rr = 0.0;
        FL_TRY(dot<double>(op, w.r64, w.r64, w.partA, &rr, s));
        const double rel = std::sqrt(rr) / bn;
        info->relres = rel;
        info->outer_iters = outer + 1;
        if (!std::isfinite(rel)) {
            set_error("residual is not finite");
            return FL_E_BREAKDOWN;
        }
        if (rel <= tol) return FL_OK;
        if (info->iters >= max_iter || outer >= max_outer) {
            set_error("no convergence: relres %.3e after %d iterations", rel, info->iters);
            return FL_E_NOCONV;
        }
        // three outer steps in a row that gain less than 10% mean the solve has stalled
        if (rel > 0.9 * last) {
            if (++stalls >= 3) {
                set_error("stagnation at relres %.3e after %d iterations", rel, info->iters);
                return FL_E_NOCONV;
            }
        } else {
            stalls = 0;
        }
        last = rel;
        // inner target relative to this residual: no tighter than needed
        double want = 0.5 * tol / rel;
        double itol = inner64 ? want : (want > inner_tol ? want : inner_tol);
        if (itol >= 1.0) itol = 0.5;
        CgResult cr;
        const int budget = max_iter - info->iters;
        if (inner64) {
            FL_TRY(cg_run<double>(op, s0, s1, w.d64, w.r64, w.p64, w.kp64, itol, budget, check_every, w, s, &cr));
            hipLaunchKernelGGL(k_axpy_to64<double>, dim3(ew_grid(M)), dim3(256), 0, s, x, w.d64, M);
        } else {
            hipLaunchKernelGGL((k_copy_cast<float, double>), dim3(ew_grid(M)), dim3(256), 0, s, w.r32, w.r64, M);
            FL_TRY(cg_run<float>(op, s0, s1, w.d32, w.r32, w.p32, w.kp32, itol, budget, check_every, w, s, &cr));
            hipLaunchKernelGGL(k_axpy_to64<float>, dim3(ew_grid(M)), dim3(256), 0, s, x, w.d32, M);
        }
        FL_HIP_TRY(hipGetLastError());
        info->iters += cr.iters;
        if (cr.breakdown && cr.iters == 0) {
            set_error("CG breakdown (p^T K p <= 0 or non-finite)");
            return FL_E_BREAKDOWN;
        }
    }
}

static int default_max_iter(fl_op op) {
    return (int)(50.0 * std::pow((double)op->M, 1.0 / op->d) + 1000.0);
}

}  // namespace fl

using namespace fl;

extern "C" {

fl_status fl_poisson_solve_ex(fl_op op, const double *f, double tol, double *u, const fl_solve_opts *opts,
                              fl_info *info, void *stream) {
    if (!op || !f || !u) { set_error("NULL argument"); return FL_E_INVAL; }
    if (!(tol > 0.0) || !std::isfinite(tol)) { set_error("tol must be positive"); return FL_E_INVAL; }
    if (f == u) { set_error("f and u must differ"); return FL_E_INVAL; }
    fl_solve_opts o = {FL_SOLVE_AUTO, 0, 0, 0, 0.0};
    if (opts) o = *opts;
    if (o.solver < FL_SOLVE_AUTO || o.solver > FL_SOLVE_FPCG) { set_error("unknown solver"); return FL_E_INVAL; }
    if (o.solver == FL_SOLVE_FPCG) {
        set_error("FPCG needs a preconditioner attached to the operator");
        return FL_E_INVAL;
    }
    fl_info local;
    fl_info *inf = info ? info : &local;
    *inf = fl_info{};
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    if (!o.use_x0) {
        hipLaunchKernelGGL(k_zero<double>, dim3(ew_grid(op->M)), dim3(256), 0, s, u, op->M);
    }
    const int max_iter = o.max_iter > 0 ? o.max_iter : default_max_iter(op);
    const bool inner64 = o.solver == FL_SOLVE_CG64;
    const double itol = o.inner_tol > 0.0 ? o.inner_tol : 1e-3;
    fl_status st = refine(op, 0.0, 1.0, f, u, tol, inner64, itol, max_iter, o.check_every, inf, s);
    inf->status = st;
    inf->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

fl_status fl_poisson_solve(fl_op op, const double *f, double tol, double *u, fl_info *info, void *stream) {
    return fl_poisson_solve_ex(op, f, tol, u, nullptr, info, stream);
}

fl_status fl_allen_cahn_step_ex(fl_op op, double *u, double tau, double eps, double theta, double tol, int solver,
                                fl_info *info, void *stream) {
    if (!op || !u) { set_error("NULL argument"); return FL_E_INVAL; }
    if (!(tau > 0.0) || !std::isfinite(tau)) { set_error("tau must be positive"); return FL_E_INVAL; }
    if (!(eps > 0.0) || !std::isfinite(eps)) { set_error("eps must be positive"); return FL_E_INVAL; }
    if (!(theta > 0.0 && theta <= 1.0)) { set_error("theta must lie in (0,1]"); return FL_E_INVAL; }
    if (!(tol > 0.0)) { set_error("tol must be positive"); return FL_E_INVAL; }
    if (solver != FL_SOLVE_AUTO && solver != FL_SOLVE_REFINE && solver != FL_SOLVE_CG64) {
        set_error("solver must be AUTO, REFINE or CG64");
        return FL_E_INVAL;
    }
    fl_info local;
    fl_info *inf = info ? info : &local;
    *inf = fl_info{};
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    FL_TRY(ensure_workspace(op));
    Work w = work_of(op);
    const double sc = tau * eps * eps;
    // b = u - (1-theta) s A u + tau (u - u^3), A u in FP64
    FL_TRY(matvec<double>(op, u, w.kp64, s));
    hipLaunchKernelGGL(k_ac_rhs, dim3(ew_grid(op->M)), dim3(256), 0, s, u, w.kp64, w.b64, op->M, tau, sc, theta);
    FL_HIP_TRY(hipGetLastError());
    // (I + theta s A) u+ = b, initial guess u
    fl_status st = refine(op, 1.0, theta * sc, w.b64, u, tol, solver == FL_SOLVE_CG64, 1e-4,
                          default_max_iter(op), 0, inf, s);
    inf->status = st;
    inf->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

fl_status fl_allen_cahn_step(fl_op op, double *u, double tau, double eps, fl_info *info, void *stream) {
    return fl_allen_cahn_step_ex(op, u, tau, eps, 0.5, 1e-8, FL_SOLVE_AUTO, info, stream);
}

}  // extern "C"
