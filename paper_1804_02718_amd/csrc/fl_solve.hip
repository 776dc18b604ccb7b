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
#include <new>
#include <type_traits>
#include <vector>

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
    // flexible PCG: current (r, r), (r, z) ping / pong, best (r, r) so far and
    // iterations since it last dropped by 4 (the residual by 2)
    S_FRR = 7,
    S_FRZ0 = 8,
    S_FRZ1 = 9,
    S_FBEST = 10,
    S_FSINCE = 11,
    S_COUNT = 16
};
// flexible PCG break codes in S_BRK
enum : int { BRK_PAP = 1, BRK_RZ = 2, BRK_NAN = 3, BRK_STALL = 4 };

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
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
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

// Batched use: blockIdx.y = problem z; vectors of problem z start at z*n,
// its partial sums at z*kMaxParts and its scalars at z*S_COUNT.
template <typename V>
__global__ __launch_bounds__(kVecBlock) void k_dot(const V *__restrict__ a, const V *__restrict__ b, long n, long chunk,
                                                   double *part, const double *done) {
    __shared__ double sh[kVecBlock];
    const int z = blockIdx.y;
    if (done && done[z * S_COUNT] != 0.0) return;
    a += z * n;
    b += z * n;
    part += z * kMaxParts;
    const long beg = (long)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
    double acc = 0.0;
    for (long i = beg + threadIdx.x; i < end; i += kVecBlock) acc += (double)a[i] * (double)b[i];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// slot <- sum of partials (single block)
__global__ __launch_bounds__(kVecBlock) void k_finish(const double *part, int np, double *scal, int slot) {
    __shared__ double sh[kVecBlock];
    const int z = blockIdx.y;
    part += z * kMaxParts;
    scal += z * S_COUNT;
    double s = sum_parts(part, np, sh);
    if (threadIdx.x == 0) scal[slot] = s;
}

// start of a CG run: rr[0] = sum(part), flags cleared, target = rel^2 * rr;
// rel2z (optional, per problem) overrides rel2, a negative entry marks the
// problem as already finished
__global__ __launch_bounds__(kVecBlock) void k_cg_init(const double *part, int np, double *scal, double rel2,
                                                       double abs2, const double *rel2z) {
    __shared__ double sh[kVecBlock];
    const int z = blockIdx.y;
    part += z * kMaxParts;
    scal += z * S_COUNT;
    bool skip = false;
    if (rel2z) {
        rel2 = rel2z[z];
        skip = rel2 < 0.0;
    }
    double s = sum_parts(part, np, sh);
    if (threadIdx.x == 0) {
        scal[S_RR0] = s;
        scal[S_RR1] = s;
        scal[S_ITER] = 0.0;
        scal[S_BRK] = std::isfinite(s) ? 0.0 : 1.0;
        const double tgt = rel2 * s > abs2 ? rel2 * s : abs2;
        scal[S_TARGET] = tgt;
        scal[S_DONE] = (skip || s <= tgt || !std::isfinite(s)) ? 1.0 : 0.0;
    }
}

// alpha = rr / (p, Kp); x += alpha p; r -= alpha Kp; partial (r, r)
template <typename V>
__global__ __launch_bounds__(kVecBlock) void k_cg_xr(V *__restrict__ x, V *__restrict__ r, const V *__restrict__ p,
                                                     const V *__restrict__ kp, long n, long chunk,
                                                     const double *__restrict__ part_pkp, int np, double *part_rr,
                                                     double *scal, int parity) {
    __shared__ double sh[kVecBlock];
    const int z = blockIdx.y;
    scal += z * S_COUNT;
    if (scal[S_DONE] != 0.0) return;
    x += z * n;
    r += z * n;
    p += z * n;
    kp += z * n;
    part_pkp += z * kMaxParts;
    part_rr += z * kMaxParts;
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
    const int z = blockIdx.y;
    scal += z * S_COUNT;
    if (scal[S_DONE] != 0.0) return;
    p += z * n;
    r += z * n;
    part_rr += z * kMaxParts;
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

// start of a preconditioned CG run (batched: blockIdx.y = problem): the S_RR
// slots take (r, z), the stop target rel2 * (r, r), rel2z[z] overriding rel2
// when given (a negative entry marks the problem as finished); (r, z) <= 0 or
// a non-finite sum is a breakdown
__global__ __launch_bounds__(kVecBlock) void k_pcg_init(const double *part_rr, const double *part_rz, int np,
                                                        double *scal, double rel2_all, const double *rel2z) {
    __shared__ double sh[kVecBlock];
    const int z = blockIdx.y;
    part_rr += z * kMaxParts;
    part_rz += z * kMaxParts;
    scal += z * S_COUNT;
    const double rel2 = rel2z ? rel2z[z] : rel2_all;
    const double rr = sum_parts(part_rr, np, sh);
    const double rz = sum_parts(part_rz, np, sh);
    if (threadIdx.x == 0) {
        scal[S_RR0] = rz;
        scal[S_RR1] = rz;
        scal[S_ITER] = 0.0;
        const bool bad = !std::isfinite(rr) || !std::isfinite(rz) || !(rz > 0.0);
        scal[S_BRK] = bad && rr > 0.0 ? 1.0 : 0.0;
        const double tgt = rel2 * rr;
        scal[S_TARGET] = tgt;
        scal[S_DONE] = (rel2 < 0.0 || rr <= tgt || bad) ? 1.0 : 0.0;
    }
}

// preconditioned direction: stop on (r, r) <= target; beta = (r, z)_new / (r, z);
// p = z + beta p; block 0 advances the scalars
template <typename V>
__global__ __launch_bounds__(kVecBlock) void k_pcg_p(V *__restrict__ p, const V *__restrict__ zv, long n, long chunk,
                                                     const double *__restrict__ part_rr,
                                                     const double *__restrict__ part_rz, int np, double *scal,
                                                     int parity) {
    __shared__ double sh[kVecBlock];
    const int z = blockIdx.y;
    scal += z * S_COUNT;
    if (scal[S_DONE] != 0.0) return;
    p += z * n;
    zv += z * n;
    part_rr += z * kMaxParts;
    part_rz += z * kMaxParts;
    const double rr_new = sum_parts(part_rr, np, sh);
    const double rz_new = sum_parts(part_rz, np, sh);
    const double be = rz_new / scal[parity ? S_RR1 : S_RR0];
    const bool bad = !std::isfinite(rr_new) || !std::isfinite(be) || !(rz_new > 0.0);
    const bool stop = rr_new <= scal[S_TARGET] || bad;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[parity ? S_RR0 : S_RR1] = rz_new;
        scal[S_ITER] += 1.0;
        if (bad && !(rr_new <= scal[S_TARGET])) scal[S_BRK] = 1.0;
        if (stop) scal[S_DONE] = 1.0;
    }
    if (stop) return;
    const V b = (V)be;
    const long beg = (long)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
    for (long i = beg + threadIdx.x; i < end; i += kVecBlock) p[i] = zv[i] + b * p[i];
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

// Allen--Cahn right-hand side b = u - (1-theta) s A u + tau gamma (w - w^3),
// w = u - shift, and the residual of the initial guess u for
// (I + theta s A) u+ = b from the same A u: r = b - u - theta s A u
__global__ void k_ac_rhs(const double *__restrict__ u, const double *__restrict__ au, double *__restrict__ b,
                         double *__restrict__ r, long n, double tau, double s, double theta, double gamma,
                         double shift) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double ui = u[i], ai = au[i], wi = ui - shift, g = tau * gamma * (wi - wi * wi * wi);
        b[i] = ui - (1.0 - theta) * s * ai + g;
        r[i] = g - s * ai;
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
    double *r64, *p64, *kp64, *d64, *b64, *q64;
    float *r32, *p32, *kp32, *d32, *z32;
    double *partA, *partB, *partC;
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
    w.q64 = w.b64 + M;
    w.partA = w.q64 + M;
    w.partB = w.partA + kMaxParts;
    w.partC = w.partB + kMaxParts;
    float *f = (float *)(w.partC + kMaxParts);
    w.r32 = f;
    w.p32 = w.r32 + M;
    w.kp32 = w.p32 + M;
    w.d32 = w.kp32 + M;
    w.z32 = w.d32 + M;
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
    size_t bytes = sizeof(double) * (6 * M + 3 * kMaxParts) + sizeof(float) * (5 * M + 64);
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

// K v = s0 v + s1 A v (epilogue of the last pass when s0 != 0 or s1 != 1);
// with dpart, the last pass also leaves per-workgroup partials of (v, K v)
template <typename V>
static fl_status apply_K(fl_op op, const V *v, V *kv, double s0, double s1, const double *done, hipStream_t s,
                         double *dpart = nullptr) {
    Epi<V> ep;
    ep.scale = (V)s1;
    if (s0 != 0.0) {
        ep.w1 = v;
        ep.a1 = (V)s0;
    }
    if (dpart) {
        ep.dotw = v;
        ep.dpart = dpart;
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
// or max_it iterations.  tau (FP32 only): preconditioned by the sine transform
// (prepared by tau_prepare32), with (r, z) in the S_RR slots.
template <typename V>
static fl_status cg_run(fl_op op, double s0, double s1, V *d, V *r, V *p, V *kp, double rel, int max_it,
                        int check_every, const Work &w, hipStream_t s, CgResult *res, bool tau = false) {
    VecLayout L = layout(op->M);
    const long M = op->M;
    hipLaunchKernelGGL(k_zero<V>, dim3(ew_grid(M)), dim3(256), 0, s, d, M);
    hipLaunchKernelGGL(k_dot<V>, dim3(L.blocks), dim3(kVecBlock), 0, s, r, r, L.n, L.chunk, w.partB, nullptr);
    if constexpr (std::is_same<V, float>::value) {
        if (tau) {
            // z = M^{-1} r, p = z, (r, z)
            FL_TRY(tau_apply32(op, r, w.z32, nullptr, s));
            hipLaunchKernelGGL((k_copy_cast<float, float>), dim3(ew_grid(M)), dim3(256), 0, s, p, w.z32, M);
            hipLaunchKernelGGL(k_dot<float>, dim3(L.blocks), dim3(kVecBlock), 0, s, r, w.z32, L.n, L.chunk, w.partC,
                               nullptr);
            hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(kVecBlock), 0, s, w.partB, w.partC, L.blocks, op->scal,
                               rel * rel, (const double *)nullptr);
        }
    }
    if (!tau) {
        hipLaunchKernelGGL((k_copy_cast<V, V>), dim3(ew_grid(M)), dim3(256), 0, s, p, r, M);
        hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(kVecBlock), 0, s, w.partB, L.blocks, op->scal, rel * rel, 0.0,
                           (const double *)nullptr);
    }
    FL_HIP_TRY(hipGetLastError());
    const double *done = op->scal + S_DONE;
    // (p, Kp) from the matvec's last pass when its workgroups fit the partials array
    const int np_x = xinv_parts(op->d, (long)(op->M / op->nk[0]), op->P, sizeof(V) == 8 ? FL_FP64 : FL_FP32,
                                sizeof(V) == 8 ? op->var64 : op->var32);
    const bool fused = np_x > 0 && np_x <= kMaxParts;
    int launched = 0;
    // the preconditioned solves need a few iterations: check after 4, then every 2
    int chunk = check_every > 0 ? check_every : (tau ? 4 : 8);
    res->iters = 0;
    res->breakdown = false;
    while (launched < max_it) {
        const int k = chunk < max_it - launched ? chunk : max_it - launched;
        for (int i = 0; i < k; ++i) {
            const int parity = (launched + i) & 1;
            FL_TRY(apply_K<V>(op, p, kp, s0, s1, done, s, fused ? w.partA : nullptr));
            if (!fused)
                hipLaunchKernelGGL(k_dot<V>, dim3(L.blocks), dim3(kVecBlock), 0, s, p, kp, L.n, L.chunk, w.partA,
                                   done);
            hipLaunchKernelGGL(k_cg_xr<V>, dim3(L.blocks), dim3(kVecBlock), 0, s, d, r, p, kp, L.n, L.chunk,
                               w.partA, fused ? np_x : L.blocks, w.partB, op->scal, parity);
            if constexpr (std::is_same<V, float>::value) {
                if (tau) {
                    FL_TRY(tau_apply32(op, r, w.z32, done, s));
                    hipLaunchKernelGGL(k_dot<float>, dim3(L.blocks), dim3(kVecBlock), 0, s, r, w.z32, L.n, L.chunk,
                                       w.partC, done);
                    hipLaunchKernelGGL(k_pcg_p<float>, dim3(L.blocks), dim3(kVecBlock), 0, s, p, w.z32, L.n,
                                       L.chunk, w.partB, w.partC, L.blocks, op->scal, parity);
                }
            }
            if (!tau)
                hipLaunchKernelGGL(k_cg_p<V>, dim3(L.blocks), dim3(kVecBlock), 0, s, p, r, L.n, L.chunk, w.partB,
                                   L.blocks, op->scal, parity);
        }
        FL_HIP_TRY(hipGetLastError());
        launched += k;
        FL_TRY(read_scalars(op, s));
        if (op->hscal[S_DONE] != 0.0) break;
        if (check_every <= 0) chunk = tau ? 2 : (chunk < 128 ? 2 * chunk : chunk);
    }
    FL_TRY(read_scalars(op, s));
    res->iters = (int)op->hscal[S_ITER];
    res->breakdown = op->hscal[S_BRK] != 0.0;
    return FL_OK;
}

// Solve K x = b to ||b - K x|| <= tol ||b||; x holds the initial guess.
// inner64: FP64 inner solves (plain CG), else FP32 inner solves; tau: the FP32
// inner solves preconditioned by the sine transform.
// r_given: w.r64 already holds b - K x for the initial x (saves the first FP64 matvec)
static fl_status refine(fl_op op, double s0, double s1, const double *b, double *x, double tol, bool inner64,
                        double inner_tol, int max_iter, int check_every, fl_info *info, hipStream_t s,
                        bool r_given = false, bool tau = false) {
    FL_TRY(ensure_workspace(op));
    if (tau) FL_TRY(tau_prepare32(op, s0, s1, s));
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
        if (!(r_given && outer == 0)) FL_TRY(residual64(op, b, x, w.r64, s0, s1, s));
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
            FL_TRY(cg_run<float>(op, s0, s1, w.d32, w.r32, w.p32, w.kp32, itol, budget, check_every, w, s, &cr,
                                 tau));
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

// x += a p; rold = r; r -= a kp
// flexible PCG start (one block): (r, r) and (r, z) from partials; target, flags
__global__ __launch_bounds__(kVecBlock) void k_fpcg_init(const double *part_rr, const double *part_rz, int np,
                                                         double *scal, double target) {
    __shared__ double sh[kVecBlock];
    const double rr = sum_parts(part_rr, np, sh);
    const double rz = sum_parts(part_rz, np, sh);
    if (threadIdx.x == 0) {
        scal[S_FRR] = rr;
        scal[S_FRZ0] = rz;
        scal[S_ITER] = 0.0;
        scal[S_TARGET] = target;
        scal[S_FBEST] = rr;
        scal[S_FSINCE] = 0.0;
        const int brk = !std::isfinite(rr) ? BRK_NAN : (!(rz > 0.0) || !std::isfinite(rz) ? BRK_RZ : 0);
        scal[S_BRK] = (double)brk;
        scal[S_DONE] = (brk != 0 || rr <= target) ? 1.0 : 0.0;
    }
}
// alpha = (r, z) / (p, A p); x += alpha p; r_old = r; r -= alpha A p; partial (r, r)
__global__ __launch_bounds__(kVecBlock) void k_fpcg_xr(double *__restrict__ x, double *__restrict__ r,
                                                       double *__restrict__ rold, const double *__restrict__ p,
                                                       const double *__restrict__ kp, long n, long chunk,
                                                       const double *__restrict__ part_pkp, int np,
                                                       double *__restrict__ part_rr, double *scal, int parity) {
    __shared__ double sh[kVecBlock];
    if (scal[S_DONE] != 0.0) return;
    const double pkp = sum_parts(part_pkp, np, sh);
    const double al = scal[parity ? S_FRZ1 : S_FRZ0] / pkp;
    if (!(pkp > 0.0) || !std::isfinite(al)) {  // every block sees the same sums
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[S_BRK] = (double)BRK_PAP;
            scal[S_DONE] = 1.0;
        }
        return;
    }
    const long beg = (long)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
    double acc = 0.0;
    for (long i = beg + threadIdx.x; i < end; i += kVecBlock) {
        x[i] += al * p[i];
        const double ri = r[i];
        rold[i] = ri;
        const double rn = ri - al * kp[i];
        r[i] = rn;
        acc += rn * rn;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = t;
}
// (r, r) bookkeeping (one block): iteration count, convergence, finiteness, and
// the stall test (the residual has not halved in 50 iterations)
__global__ __launch_bounds__(kVecBlock) void k_fpcg_rr(const double *part_rr, int np, double *scal) {
    __shared__ double sh[kVecBlock];
    if (scal[S_DONE] != 0.0) return;
    const double rr = sum_parts(part_rr, np, sh);
    if (threadIdx.x == 0) {
        scal[S_FRR] = rr;
        scal[S_ITER] += 1.0;
        if (!std::isfinite(rr)) {
            scal[S_BRK] = (double)BRK_NAN;
            scal[S_DONE] = 1.0;
        } else if (rr <= scal[S_TARGET]) {
            scal[S_DONE] = 1.0;
        } else if (rr < 0.25 * scal[S_FBEST]) {
            scal[S_FBEST] = rr;
            scal[S_FSINCE] = 0.0;
        } else if ((scal[S_FSINCE] += 1.0) > 50.0) {
            scal[S_BRK] = (double)BRK_STALL;
            scal[S_DONE] = 1.0;
        }
    }
}
// partials of (r, z) and (r_old, z) in one pass
__global__ __launch_bounds__(kVecBlock) void k_fpcg_dot2(const double *__restrict__ r, const double *__restrict__ z,
                                                         const double *__restrict__ rold, long n, long chunk,
                                                         double *part_rz, double *part_roz, const double *done) {
    __shared__ double sh[kVecBlock];
    if (done && done[0] != 0.0) return;
    const long beg = (long)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
    double a = 0.0, b = 0.0;
    for (long i = beg + threadIdx.x; i < end; i += kVecBlock) {
        const double zi = z[i];
        a += r[i] * zi;
        b += rold[i] * zi;
    }
    const double sa = block_sum(a, sh);
    const double sb = block_sum(b, sh);
    if (threadIdx.x == 0) {
        part_rz[blockIdx.x] = sa;
        part_roz[blockIdx.x] = sb;
    }
}
// Polak--Ribiere beta = ((r, z) - (r_old, z)) / (r_old, z_old); p = z + beta p;
// block 0 stores the new (r, z) in the other slot
__global__ __launch_bounds__(kVecBlock) void k_fpcg_dir(double *__restrict__ p, const double *__restrict__ z, long n,
                                                        long chunk, const double *part_rz, const double *part_roz,
                                                        int np, double *scal, int parity) {
    __shared__ double sh[kVecBlock];
    if (scal[S_DONE] != 0.0) return;
    const double rzn = sum_parts(part_rz, np, sh);
    const double zro = sum_parts(part_roz, np, sh);
    const double be = (rzn - zro) / scal[parity ? S_FRZ1 : S_FRZ0];
    if (!(rzn > 0.0) || !std::isfinite(be)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            scal[S_BRK] = (double)BRK_RZ;
            scal[S_DONE] = 1.0;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[parity ? S_FRZ0 : S_FRZ1] = rzn;
    const long beg = (long)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
    for (long i = beg + threadIdx.x; i < end; i += kVecBlock) p[i] = z[i] + be * p[i];
}

// preconditioners of the flexible PCG
enum : int {
    PREC_NET = 0,  // learned: z = ||r|| Net(r / ||r||, alpha)
    PREC_TAU = 1   // sine-transform (tau) preconditioner of K, prepared by tau_prepare
};

// z = M r; `done` (optional) turns the application into a no-op once set
static fl_status apply_prec(fl_op op, int kind, const double *r, double *z, const double *done, hipStream_t s) {
    if (kind == PREC_TAU) return tau_apply(op, r, z, done, s);
    return unet_apply(op->net, r, op->n, op->alpha, z, op->scal + S_FRR, s);
}

// Flexible PCG (Notay's flexible CG with the Polak--Ribiere beta) on
// K x = f, K = s0 I + s1 A, x holding the initial guess, with the learned or
// the sine-transform preconditioner.  Falls back to plain FP64 CG from the
// current iterate when (r, z) <= 0, a scalar is not finite, or the residual
// stops decreasing.
// r_given: w.r64 already holds f - K x for the initial x (saves the first FP64 matvec)
static fl_status fpcg(fl_op op, int kind, double s0, double s1, const double *f, double *x, double tol,
                      int max_iter, fl_info *info, hipStream_t s, bool r_given = false) {
    FL_TRY(ensure_workspace(op));
    Work w = work_of(op);
    const long M = op->M;
    VecLayout L = layout(M);
    double *r = w.r64, *z = w.d64, *p = w.p64, *kp = w.kp64, *rold = w.q64;
    double bb = 0.0;
    FL_TRY(dot<double>(op, f, f, w.partA, &bb, s));
    const double bn = std::sqrt(bb);
    if (!std::isfinite(bn)) { set_error("right-hand side is not finite"); return FL_E_BREAKDOWN; }
    if (bn == 0.0) {
        hipLaunchKernelGGL(k_zero<double>, dim3(ew_grid(M)), dim3(256), 0, s, x, M);
        FL_HIP_TRY(hipStreamSynchronize(s));
        return FL_OK;
    }
    // r = f - K x; (r, r) into S_FRR for the network's scaling; z = M r; (r, z); p = z
    if (!r_given) FL_TRY(residual64(op, f, x, r, s0, s1, s));
    double *scal = op->scal;
    const double *done = scal + S_DONE;
    hipLaunchKernelGGL(k_dot<double>, dim3(L.blocks), dim3(kVecBlock), 0, s, r, r, L.n, L.chunk, w.partA, nullptr);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kVecBlock), 0, s, w.partA, L.blocks, scal, (int)S_FRR);
    FL_TRY(apply_prec(op, kind, r, z, nullptr, s));
    hipLaunchKernelGGL(k_dot<double>, dim3(L.blocks), dim3(kVecBlock), 0, s, r, z, L.n, L.chunk, w.partB, nullptr);
    hipLaunchKernelGGL(k_fpcg_init, dim3(1), dim3(kVecBlock), 0, s, w.partA, w.partB, L.blocks, scal,
                       tol * tol * bb);
    hipLaunchKernelGGL((k_copy_cast<double, double>), dim3(ew_grid(M)), dim3(256), 0, s, p, z, M);
    FL_HIP_TRY(hipGetLastError());
    // (p, A p) from the matvec's last pass when its workgroups fit the partials array
    const int np_x = xinv_parts(op->d, (long)(op->M / op->nk[0]), op->P, FL_FP64, op->var64);
    const bool fused = np_x > 0 && np_x <= kMaxParts;
    // scalars stay on the device; the host reads them every kCheck iterations
    // (the network does not test the done flag, so at most kCheck - 1 of its
    // applications follow convergence).  The sine-transform preconditioner
    // converges in 6-9 iterations at 1e-8: its first check comes after 6, then
    // every 2, so few no-op iterations are launched after convergence.
    constexpr int kCheck = 4;
    int launched = 0;
    FL_TRY(read_scalars(op, s));
    while (op->hscal[S_DONE] == 0.0 && launched < max_iter) {
        const int want = kind == PREC_TAU ? (launched == 0 ? 6 : 2) : kCheck;
        const int k = want < max_iter - launched ? want : max_iter - launched;
        for (int i = 0; i < k; ++i) {
            const int parity = (launched + i) & 1;
            FL_TRY(apply_K<double>(op, p, kp, s0, s1, done, s, fused ? w.partA : nullptr));
            if (!fused)
                hipLaunchKernelGGL(k_dot<double>, dim3(L.blocks), dim3(kVecBlock), 0, s, p, kp, L.n, L.chunk,
                                   w.partA, done);
            hipLaunchKernelGGL(k_fpcg_xr, dim3(L.blocks), dim3(kVecBlock), 0, s, x, r, rold, p, kp, L.n, L.chunk,
                               w.partA, fused ? np_x : L.blocks, w.partB, scal, parity);
            hipLaunchKernelGGL(k_fpcg_rr, dim3(1), dim3(kVecBlock), 0, s, w.partB, L.blocks, scal);
            FL_TRY(apply_prec(op, kind, r, z, done, s));
            hipLaunchKernelGGL(k_fpcg_dot2, dim3(L.blocks), dim3(kVecBlock), 0, s, r, z, rold, L.n, L.chunk,
                               w.partA, w.partB, done);
            hipLaunchKernelGGL(k_fpcg_dir, dim3(L.blocks), dim3(kVecBlock), 0, s, p, z, L.n, L.chunk, w.partA,
                               w.partB, L.blocks, scal, parity);
        }
        FL_HIP_TRY(hipGetLastError());
        launched += k;
        FL_TRY(read_scalars(op, s));
    }
    const int it = (int)op->hscal[S_ITER];
    const int brk = (int)op->hscal[S_BRK];
    info->iters = it;
    info->relres = std::sqrt(op->hscal[S_FRR]) / bn;
    bool fallback = brk != 0;
    switch (brk) {
        case BRK_PAP: set_error("FPCG: (p, A p) <= 0 at iteration %d; plain CG takes over", it); break;
        case BRK_RZ: set_error("FPCG: (r, z) <= 0 at iteration %d; plain CG takes over", it); break;
        case BRK_NAN: set_error("FPCG: residual not finite at iteration %d; plain CG takes over", it); break;
        case BRK_STALL:
            set_error("FPCG: residual %.3e not halved in 50 iterations (at %d); plain CG takes over", info->relres,
                      it);
            break;
        default: break;
    }
    if (!fallback) {
        // verify with a fresh FP64 residual
        FL_TRY(residual64(op, f, x, r, s0, s1, s));
        double rr = 0.0;
        FL_TRY(dot<double>(op, r, r, w.partA, &rr, s));
        info->relres = std::sqrt(rr) / bn;
        info->outer_iters = 1;
        if (info->relres <= tol) return FL_OK;
        if (launched >= max_iter) { set_error("FPCG: no convergence"); return FL_E_NOCONV; }
    }
    // plain FP64 CG from the current iterate
    info->fell_back = 1;
    fl_info sub{};
    fl_status st = refine(op, s0, s1, f, x, tol, true, 0.0, max_iter, 0, &sub, s);
    info->iters += sub.iters;
    info->outer_iters += sub.outer_iters;
    info->relres = sub.relres;
    return st;
}

// AUTO takes the FP32 inner solves (TAU32) from this many unknowns up.  Each
// refinement step costs an FP64 residual and a host check, which the cheaper
// FP32 passes repay only on large grids: 3D N = 256 (16.6M unknowns) to 1e-8 in
// 15 ms against 21 ms with TAU; 2D N = 1024 (1M) in 1.5 ms against 1.3 ms.
constexpr int64_t kTau32Min = (int64_t)1 << 22;

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
    if (o.solver < FL_SOLVE_AUTO || o.solver > FL_SOLVE_TAU32) { set_error("unknown solver"); return FL_E_INVAL; }
    if ((o.solver == FL_SOLVE_TAU || o.solver == FL_SOLVE_TAU32) && !tau_supported(op)) {
        set_error("TAU needs at most P/2 - 1 nodes per axis (N not 2^k + 1)");
        return FL_E_INVAL;
    }
    if (o.solver == FL_SOLVE_FPCG && (!op->net || op->d != 2 || op->n > unet_size(op->net) ||
                                      op->nk[0] != op->n || op->nk[1] != op->n)) {
        set_error("FPCG needs a learned preconditioner attached to a 2D square operator with n <= its grid size");
        return FL_E_INVAL;
    }
    fl_info local;
    fl_info *inf = info ? info : &local;
    *inf = fl_info{};
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    // from x0 = 0 the initial residual is f itself: the solvers take it as given
    // instead of spending an FP64 matvec on f - A 0
    const bool r0 = !o.use_x0;
    if (r0) {
        FL_TRY(ensure_workspace(op));
        hipLaunchKernelGGL(k_zero<double>, dim3(ew_grid(op->M)), dim3(256), 0, s, u, op->M);
        hipLaunchKernelGGL((k_copy_cast<double, double>), dim3(ew_grid(op->M)), dim3(256), 0, s, work_of(op).r64, f,
                           op->M);
    }
    const int max_iter = o.max_iter > 0 ? o.max_iter : default_max_iter(op);
    fl_status st = FL_OK;
    bool solved = false;
    // AUTO: the sine-transform preconditioned CG wherever it applies (square and
    // cubic operators; a handful of iterations at every size, against hundreds
    // for CG at alpha >= 1): the FP64 flexible solve (TAU), or from kTau32Min
    // unknowns up FP32 inner solves in FP64 refinement (TAU32), which falls back
    // to TAU from the current iterate if it fails
    if (o.solver == FL_SOLVE_TAU || o.solver == FL_SOLVE_TAU32 ||
        (o.solver == FL_SOLVE_AUTO && tau_supported(op))) {
        const bool t32 = o.solver == FL_SOLVE_TAU32 || (o.solver == FL_SOLVE_AUTO && op->M >= kTau32Min);
        st = t32 ? tau_prepare32(op, 0.0, 1.0, s) : tau_prepare(op, 0.0, 1.0, s);
        if (st == FL_OK && t32) {
            const double itol = o.inner_tol > 0.0 ? o.inner_tol : 1e-4;
            st = refine(op, 0.0, 1.0, f, u, tol, false, itol, max_iter, o.check_every, inf, s, r0, true);
            if (st != FL_OK && o.solver == FL_SOLVE_AUTO && std::isfinite(inf->relres) &&
                tau_prepare(op, 0.0, 1.0, s) == FL_OK) {
                fl_info sub{};
                st = fpcg(op, PREC_TAU, 0.0, 1.0, f, u, tol, max_iter, &sub, s);
                inf->iters += sub.iters;
                inf->outer_iters += sub.outer_iters;
                inf->relres = sub.relres;
                inf->fell_back = 1;
            }
            solved = true;
        } else if (st == FL_OK) {
            st = fpcg(op, PREC_TAU, 0.0, 1.0, f, u, tol, max_iter, inf, s, r0);  // falls back to CG itself
            solved = true;
        } else {
            // AUTO without a positive symbol on the sine modes takes the plain solvers
            solved = o.solver != FL_SOLVE_AUTO || st != FL_E_BREAKDOWN;
        }
    }
    if (!solved && o.solver == FL_SOLVE_FPCG) {
        st = fpcg(op, PREC_NET, 0.0, 1.0, f, u, tol, max_iter, inf, s, r0);
    } else if (!solved) {
        // otherwise FP32-matvec refinement up to alpha = 1.25, FP64 CG above.  Each
        // refinement step restarts CG, and for the stiffer operators the restarts cost
        // more iterations than the cheaper FP32 matvec saves (2D N = 1024 to 1e-8:
        // refinement 5-10 % faster at alpha <= 1, 7 % and 16 % slower at alpha = 1.5 and 1.9)
        const bool inner64 = o.solver == FL_SOLVE_CG64 || (o.solver == FL_SOLVE_AUTO && op->alpha > 1.25);
        const double itol = o.inner_tol > 0.0 ? o.inner_tol : 1e-3;
        *inf = fl_info{};
        st = refine(op, 0.0, 1.0, f, u, tol, inner64, itol, max_iter, o.check_every, inf, s, r0);
    }
    inf->status = st;
    inf->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

fl_status fl_set_preconditioner(fl_op op, fl_unet net) {
    if (!op) { set_error("NULL operator"); return FL_E_INVAL; }
    op->net = net;
    return FL_OK;
}

fl_status fl_poisson_solve(fl_op op, const double *f, double tol, double *u, fl_info *info, void *stream) {
    return fl_poisson_solve_ex(op, f, tol, u, nullptr, info, stream);
}

fl_status fl_allen_cahn_step_gen(fl_op op, double *u, double tau, double kappa, double gamma, double shift,
                                 double theta, double tol, int solver, fl_info *info, void *stream) {
    if (!op || !u) { set_error("NULL argument"); return FL_E_INVAL; }
    if (!(tau > 0.0) || !std::isfinite(tau)) { set_error("tau must be positive"); return FL_E_INVAL; }
    if (!(kappa >= 0.0) || !std::isfinite(kappa)) { set_error("kappa must be >= 0"); return FL_E_INVAL; }
    if (!std::isfinite(gamma) || !std::isfinite(shift)) { set_error("gamma and shift must be finite"); return FL_E_INVAL; }
    if (!(theta > 0.0 && theta <= 1.0)) { set_error("theta must lie in (0,1]"); return FL_E_INVAL; }
    if (!(tol > 0.0)) { set_error("tol must be positive"); return FL_E_INVAL; }
    if (solver != FL_SOLVE_AUTO && solver != FL_SOLVE_REFINE && solver != FL_SOLVE_CG64 && solver != FL_SOLVE_TAU &&
        solver != FL_SOLVE_TAU32) {
        set_error("solver must be AUTO, REFINE, CG64, TAU or TAU32");
        return FL_E_INVAL;
    }
    if ((solver == FL_SOLVE_TAU || solver == FL_SOLVE_TAU32) && !tau_supported(op)) {
        set_error("TAU needs at most P/2 - 1 nodes per axis (N not 2^k + 1)");
        return FL_E_INVAL;
    }
    fl_info local;
    fl_info *inf = info ? info : &local;
    *inf = fl_info{};
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    FL_TRY(ensure_workspace(op));
    Work w = work_of(op);
    const double sc = tau * kappa;
    // b = u - (1-theta) s A u + tau gamma (w - w^3), A u in FP64
    FL_TRY(matvec<double>(op, u, w.kp64, s));
    hipLaunchKernelGGL(k_ac_rhs, dim3(ew_grid(op->M)), dim3(256), 0, s, u, w.kp64, w.b64, w.r64, op->M, tau, sc,
                       theta, gamma, shift);
    FL_HIP_TRY(hipGetLastError());
    // (I + theta s A) u+ = b, initial guess u, whose residual k_ac_rhs left in r64: the
    // sine-transform preconditioned CG (TAU; AUTO where it applies and the system is
    // not close to the identity), else CG or FP32-matvec refinement.  The spectral
    // radius of A is at most 2 A_ii = -2 c a_0 (its symbol is a_0 + sum of the
    // off-diagonal terms, which sum to at most -a_0); when theta s times that is
    // small, plain CG converges in a few iterations and the preconditioner's extra
    // FP64 pass per iteration does not pay (the paper's two-bubble runs at N = 1024:
    // the preconditioned solve is faster at 1.05, refinement at 0.11).
    const double spread = theta * sc * 2.0 * (-op->c * op->a0);
    fl_status st = FL_OK;
    bool solved = false;
    if (solver == FL_SOLVE_TAU || solver == FL_SOLVE_TAU32 ||
        (solver == FL_SOLVE_AUTO && tau_supported(op) && spread > 0.5)) {
        const bool t32 = solver == FL_SOLVE_TAU32 || (solver == FL_SOLVE_AUTO && op->M >= kTau32Min);
        st = t32 ? tau_prepare32(op, 1.0, theta * sc, s) : tau_prepare(op, 1.0, theta * sc, s);
        if (st == FL_OK && t32) {
            st = refine(op, 1.0, theta * sc, w.b64, u, tol, false, 1e-4, default_max_iter(op), 0, inf, s, true,
                        true);
            if (st != FL_OK && solver == FL_SOLVE_AUTO && std::isfinite(inf->relres) &&
                tau_prepare(op, 1.0, theta * sc, s) == FL_OK) {
                fl_info sub{};
                st = fpcg(op, PREC_TAU, 1.0, theta * sc, w.b64, u, tol, default_max_iter(op), &sub, s);
                inf->iters += sub.iters;
                inf->outer_iters += sub.outer_iters;
                inf->relres = sub.relres;
                inf->fell_back = 1;
            }
            solved = true;
        } else if (st == FL_OK) {
            st = fpcg(op, PREC_TAU, 1.0, theta * sc, w.b64, u, tol, default_max_iter(op), inf, s, true);
            solved = true;
        } else {
            // r64 still holds the initial residual for refine
            solved = solver != FL_SOLVE_AUTO || st != FL_E_BREAKDOWN;
        }
    }
    if (!solved)
        st = refine(op, 1.0, theta * sc, w.b64, u, tol, solver == FL_SOLVE_CG64, 1e-4, default_max_iter(op), 0,
                    inf, s, true);
    inf->status = st;
    inf->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

fl_status fl_allen_cahn_step_ex(fl_op op, double *u, double tau, double eps, double theta, double tol, int solver,
                                fl_info *info, void *stream) {
    if (!(eps > 0.0) || !std::isfinite(eps)) { set_error("eps must be positive"); return FL_E_INVAL; }
    return fl_allen_cahn_step_gen(op, u, tau, eps * eps, 1.0, 0.0, theta, tol, solver, info, stream);
}

fl_status fl_allen_cahn_step(fl_op op, double *u, double tau, double eps, fl_info *info, void *stream) {
    return fl_allen_cahn_step_ex(op, u, tau, eps, 0.5, 1e-8, FL_SOLVE_AUTO, info, stream);
}

}  // extern "C"

// ===========================================================================
// Batched Poisson solves.  Problems are grouped into size classes (same N,
// hence the same FFT length and kernels).  Each class keeps its problems'
// vectors packed ([problem][M]) and runs every FFT pass and CG kernel of all
// of them in one launch (blockIdx.z / blockIdx.y = problem).  The inner FP32
// CG iterations of a class are captured once in a hipGraph (a chunk of
// kGraphIters iterations) and replayed; classes run concurrently on their own
// streams.  Each problem has its own device scalars and done flag, so a
// converged problem turns its share of every later launch into a no-op.
// ===========================================================================
namespace fl {

constexpr int kGraphIters = 16;    // inner CG iterations per captured graph (even: parity)
constexpr int kGraphItersTau = 4;  // inner preconditioned iterations per graph (they converge in a few)

struct BatchClass {
    int N = 0, n = 0, P = 0, Q = 0, B = 0;
    long M = 0;
    std::vector<int> idx;    // user indices of the problems
    std::vector<fl_op> ops;  // per-problem operators (coefficients, lambda)
    int var32 = 0, var64 = 0;
    void *buf = nullptr;     // all packed device buffers
    double *x = nullptr, *b = nullptr, *r64 = nullptr, *rel2 = nullptr;
    float *r32 = nullptr, *p32 = nullptr, *kp32 = nullptr, *d32 = nullptr;
    double *partA = nullptr, *partB = nullptr, *scal = nullptr, *hscal = nullptr;
    void *T1 = nullptr, *T2 = nullptr, *lam32 = nullptr, *lam64 = nullptr;
    long zs_t = 0, zs_t2 = 0, lamlen32 = 0, lamlen64 = 0;
    hipStream_t s = nullptr;
    double *hrel2 = nullptr;  // pinned: per-problem inner targets for the device
    MvCtx<float> c32;
    MvCtx<double> c64;
    // sine-transform preconditioned inner CG (every N but 2^k + 1, when every
    // problem has a positive symbol on the sine modes): z = M^{-1} r in FP32
    bool tau = false;
    int iters_per_chunk = kGraphIters;
    float *z32 = nullptr;
    double *partC = nullptr;
    void *mu32 = nullptr;
    MvCtx<float> c32t;
};

}  // namespace fl

struct fl_batch_s {
    int d = 2, count = 0;
    std::vector<fl::BatchClass> cls;
    // one graph holding a chunk of inner iterations of every class, each class
    // on its own branch (captured from the class streams forked off `main`)
    hipStream_t main = nullptr;
    hipGraphExec_t all = nullptr;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    // the last solve: host waits on the GPU, graph launches
    int host_waits = 0, graph_launches = 0;
};

namespace fl {

static void batch_free(fl_batch b) {
    if (!b) return;
    if (b->all) (void)hipGraphExecDestroy(b->all);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (hipEvent_t e : b->joins) (void)hipEventDestroy(e);
    if (b->main) (void)hipStreamDestroy(b->main);
    for (auto &c : b->cls) {
        if (c.s) (void)hipStreamDestroy(c.s);
        if (c.hrel2) (void)hipHostFree(c.hrel2);
        if (c.buf) (void)hipFree(c.buf);
        if (c.hscal) (void)hipHostFree(c.hscal);
        for (fl_op o : c.ops) fl_op_destroy(o);
    }
    delete b;
}

// carve the class's packed buffers out of one allocation
static fl_status batch_alloc(BatchClass &c, int d) {
    const long B = c.B, M = c.M;
    const int C32 = variant_desc_pd(c.P, d, FL_FP32, c.var32).c, C64 = variant_desc_pd(c.P, d, FL_FP64, c.var64).c;
    c.lamlen32 = lam_tiled_len(d, c.P, C32);
    c.lamlen64 = lam_tiled_len(d, c.P, C64);
    c.zs_t = c.ops[0]->T1_bytes;
    c.zs_t2 = c.ops[0]->T2_bytes;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_x = off; off += al(sizeof(double) * B * M);
    const size_t o_b = off; off += al(sizeof(double) * B * M);
    const size_t o_r64 = off; off += al(sizeof(double) * B * M);
    const size_t o_rel = off; off += al(sizeof(double) * B);
    const size_t o_r32 = off; off += al(sizeof(float) * B * M);
    const size_t o_p32 = off; off += al(sizeof(float) * B * M);
    const size_t o_kp32 = off; off += al(sizeof(float) * B * M);
    const size_t o_d32 = off; off += al(sizeof(float) * B * M);
    const size_t o_pa = off; off += al(sizeof(double) * B * kMaxParts);
    const size_t o_pb = off; off += al(sizeof(double) * B * kMaxParts);
    const size_t o_sc = off; off += al(sizeof(double) * B * S_COUNT);
    const size_t o_t1 = off; off += al((size_t)c.zs_t * B);
    const size_t o_t2 = off; off += al((size_t)c.zs_t2 * B);
    const size_t o_l32 = off; off += al(sizeof(float) * c.lamlen32 * B);
    const size_t o_l64 = off; off += al(sizeof(double) * c.lamlen64 * B);
    // the preconditioned path: z, (r, z) partials and the per-problem FP32 symbols
    c.tau = tau_supported(c.ops[0]);
    const size_t o_z32 = off; off += c.tau ? al(sizeof(float) * B * M) : 0;
    const size_t o_pc = off; off += c.tau ? al(sizeof(double) * B * kMaxParts) : 0;
    const size_t o_mu = off; off += c.tau ? al(sizeof(float) * c.lamlen32 * B) : 0;
    FL_HIP_TRY(hipMalloc(&c.buf, off));
    char *base = (char *)c.buf;
    c.x = (double *)(base + o_x);
    c.b = (double *)(base + o_b);
    c.r64 = (double *)(base + o_r64);
    c.rel2 = (double *)(base + o_rel);
    c.r32 = (float *)(base + o_r32);
    c.p32 = (float *)(base + o_p32);
    c.kp32 = (float *)(base + o_kp32);
    c.d32 = (float *)(base + o_d32);
    c.partA = (double *)(base + o_pa);
    c.partB = (double *)(base + o_pb);
    c.scal = (double *)(base + o_sc);
    c.T1 = base + o_t1;
    c.T2 = c.zs_t2 ? (void *)(base + o_t2) : nullptr;
    c.lam32 = base + o_l32;
    c.lam64 = base + o_l64;
    if (c.tau) {
        c.z32 = (float *)(base + o_z32);
        c.partC = (double *)(base + o_pc);
        c.mu32 = base + o_mu;
    }
    FL_HIP_TRY(hipHostMalloc((void **)&c.hscal, sizeof(double) * B * S_COUNT, hipHostMallocDefault));
    FL_HIP_TRY(hipHostMalloc((void **)&c.hrel2, sizeof(double) * B, hipHostMallocDefault));
    // per-problem lambda tiled for the class's variants
    for (int z = 0; z < c.B; ++z) {
        FL_TRY(tile_lambda(c.ops[z], FL_FP32, C32, (float *)c.lam32 + z * c.lamlen32, c.s));
        FL_TRY(tile_lambda(c.ops[z], FL_FP64, C64, (double *)c.lam64 + z * c.lamlen64, c.s));
    }
    c.c32 = single_ctx<float>(c.ops[0]);
    c.c64 = single_ctx<double>(c.ops[0]);
    for (MvCtx<float> *cx : {&c.c32}) {
        cx->T1 = c.T1; cx->T2 = c.T2; cx->lam = (const float *)c.lam32; cx->batch = c.B; cx->zs_vec = M;
        cx->zs_t1 = c.zs_t; cx->zs_t2 = c.zs_t2; cx->zs_lam = c.lamlen32; cx->zs_done = S_COUNT;
    }
    for (MvCtx<double> *cx : {&c.c64}) {
        cx->T1 = c.T1; cx->T2 = c.T2; cx->lam = (const double *)c.lam64; cx->batch = c.B; cx->zs_vec = M;
        cx->zs_t1 = c.zs_t; cx->zs_t2 = c.zs_t2; cx->zs_lam = c.lamlen64; cx->zs_done = S_COUNT;
    }
    // every problem's preconditioner symbol, or plain CG for the class if one of
    // them has no positive symbol on the sine modes
    for (int z = 0; z < c.B && c.tau; ++z) {
        fl_status st = tau_symbol(c.ops[z], 0.0, 1.0, FL_FP32, C32, (float *)c.mu32 + z * c.lamlen32, c.s);
        if (st == FL_E_BREAKDOWN) c.tau = false;
        else FL_TRY(st);
    }
    if (c.tau) {
        c.c32t = c.c32;
        c.c32t.lam = (const float *)c.mu32;
        c.c32t.odd = true;
        c.iters_per_chunk = kGraphItersTau;
    }
    return FL_OK;
}

// launches of iters_per_chunk inner FP32 (P)CG iterations of a class (captured once).
// The preconditioned iteration keeps (r, z) in the S_RR slots, so k_cg_xr takes
// alpha = (r, z) / (p, K p) and leaves the (r, r) partials for the stop test.
static fl_status batch_chunk_launches(BatchClass &c) {
    VecLayout L = layout(c.M);
    const double *done = c.scal + S_DONE;
    // (p, Kp) from the matvec's last pass when its workgroups fit the partials array
    const int np_x = xinv_parts(c.c32.d, (long)(c.M / c.n), c.P, FL_FP32, c.var32);
    const bool fused = np_x > 0 && np_x <= kMaxParts;
    Epi<float> ep;
    if (fused) {
        ep.dotw = c.p32;
        ep.dpart = c.partA;
        ep.dpart_stride = kMaxParts;
    }
    for (int i = 0; i < c.iters_per_chunk; ++i) {
        const int parity = i & 1;
        FL_TRY(matvec_ctx<float>(c.c32, c.var32, c.p32, c.kp32, ep, done, c.s));
        if (!fused)
            hipLaunchKernelGGL(k_dot<float>, dim3(L.blocks, c.B), dim3(kVecBlock), 0, c.s, c.p32, c.kp32, L.n,
                               L.chunk, c.partA, done);
        hipLaunchKernelGGL(k_cg_xr<float>, dim3(L.blocks, c.B), dim3(kVecBlock), 0, c.s, c.d32, c.r32, c.p32,
                           c.kp32, L.n, L.chunk, c.partA, fused ? np_x : L.blocks, c.partB, c.scal, parity);
        if (c.tau) {
            FL_TRY(matvec_ctx<float>(c.c32t, c.var32, c.r32, c.z32, Epi<float>{}, done, c.s));
            hipLaunchKernelGGL(k_dot<float>, dim3(L.blocks, c.B), dim3(kVecBlock), 0, c.s, c.r32, c.z32, L.n,
                               L.chunk, c.partC, done);
            hipLaunchKernelGGL(k_pcg_p<float>, dim3(L.blocks, c.B), dim3(kVecBlock), 0, c.s, c.p32, c.z32, L.n,
                               L.chunk, c.partB, c.partC, L.blocks, c.scal, parity);
        } else {
            hipLaunchKernelGGL(k_cg_p<float>, dim3(L.blocks, c.B), dim3(kVecBlock), 0, c.s, c.p32, c.r32, L.n,
                               L.chunk, c.partB, L.blocks, c.scal, parity);
        }
    }
    FL_HIP_TRY(hipGetLastError());
    return FL_OK;
}

// the all-class chunk graph: fork every class stream off `main`, capture each
// class's chunk of inner iterations on its own stream, join back into `main`
static fl_status batch_capture_all(fl_batch b) {
    hipGraph_t g = nullptr;
    FL_HIP_TRY(hipStreamBeginCapture(b->main, hipStreamCaptureModeThreadLocal));
    fl_status st = FL_OK;
    if (hipEventRecord(b->fork, b->main) != hipSuccess) st = FL_E_DEVICE;
    for (size_t ci = 0; ci < b->cls.size() && st == FL_OK; ++ci) {
        BatchClass &c = b->cls[ci];
        if (hipStreamWaitEvent(c.s, b->fork, 0) != hipSuccess) st = FL_E_DEVICE;
        if (st == FL_OK) st = batch_chunk_launches(c);
        if (st == FL_OK && (hipEventRecord(b->joins[ci], c.s) != hipSuccess ||
                            hipStreamWaitEvent(b->main, b->joins[ci], 0) != hipSuccess))
            st = FL_E_DEVICE;
    }
    hipError_t e = hipStreamEndCapture(b->main, &g);
    FL_TRY(st);
    FL_HIP_TRY(e);
    e = hipGraphInstantiate(&b->all, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    FL_HIP_TRY(e);
    return FL_OK;
}

// `to` waits for everything issued on `from` so far
static fl_status stream_after(hipStream_t to, hipStream_t from, hipEvent_t e) {
    FL_HIP_TRY(hipEventRecord(e, from));
    FL_HIP_TRY(hipStreamWaitEvent(to, e, 0));
    return FL_OK;
}

}  // namespace fl

extern "C" {

fl_status fl_batch_create(int d, int count, const int *N, const double *alpha, const double *h, fl_batch *out) {
    if (!out || !N || !alpha || !h || count < 1 || d < 1 || d > 3) {
        set_error("bad argument");
        return FL_E_INVAL;
    }
    fl_batch b = new (std::nothrow) fl_batch_s();
    if (!b) return FL_E_NOMEM;
    b->d = d;
    b->count = count;
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    fl_status st = FL_OK;
    for (int i = 0; i < count && st == FL_OK; ++i) {
        BatchClass *c = nullptr;
        for (auto &k : b->cls)
            if (k.N == N[i]) c = &k;
        if (!c) {
            b->cls.emplace_back();
            c = &b->cls.back();
            c->N = N[i];
        }
        fl_op op = nullptr;
        st = fl_coeffs(d, alpha[i], h[i], N[i], &op);
        if (st != FL_OK) break;
        if (large_op(op)) {
            fl_op_destroy(op);
            set_error("batched solves need FFT length <= %d (N = %d)", kMaxLdsP, N[i]);
            st = FL_E_UNSUPPORTED;
            break;
        }
        c->idx.push_back(i);
        c->ops.push_back(op);
    }
    for (auto &c : b->cls) {
        if (st != FL_OK) break;
        fl_op o = c.ops[0];
        c.n = o->n;
        c.P = o->P;
        c.Q = o->Q;
        c.M = o->M;
        c.B = (int)c.ops.size();
        // kernel variants of the class's FFT length from the tuning cache
        st = tuned_variant(o, FL_FP32, &c.var32);
        if (st == FL_OK) st = tuned_variant(o, FL_FP64, &c.var64);
        if (st != FL_OK) break;
        if (hipStreamCreateWithFlags(&c.s, hipStreamNonBlocking) != hipSuccess) {
            st = FL_E_DEVICE;
            break;
        }
        st = batch_alloc(c, d);
        if (st == FL_OK && hipStreamSynchronize(c.s) != hipSuccess) st = FL_E_DEVICE;
    }
    if (st == FL_OK) {
        b->joins.assign(b->cls.size(), nullptr);
        if (hipStreamCreateWithFlags(&b->main, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
            st = FL_E_DEVICE;
        for (auto &e : b->joins)
            if (st == FL_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) st = FL_E_DEVICE;
        if (st == FL_OK) st = batch_capture_all(b);
    }
    if (st != FL_OK) {
        batch_free(b);
        return st;
    }
    *out = b;
    return FL_OK;
}

fl_status fl_batch_destroy(fl_batch b) {
    batch_free(b);
    return FL_OK;
}

fl_status fl_batch_poisson_solve(fl_batch b, const double *const *f, double *const *u, double tol, int max_iter,
                                 fl_info *infos, void *stream) {
    if (!b || !f || !u || !(tol > 0.0)) { set_error("bad argument"); return FL_E_INVAL; }
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t us = (hipStream_t)stream;
    hipEvent_t ready = nullptr;
    FL_HIP_TRY(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    FL_HIP_TRY(hipEventRecord(ready, us));  // inputs written on the caller's stream
    const double inner_tol = 1e-3;
    std::vector<std::vector<double>> bn(b->cls.size()), rel(b->cls.size());
    std::vector<std::vector<int>> iters(b->cls.size()), outer(b->cls.size()), fin(b->cls.size());
    fl_status st = FL_OK;
    // gather right-hand sides, zero solutions, norms of b
    for (size_t ci = 0; ci < b->cls.size() && st == FL_OK; ++ci) {
        BatchClass &c = b->cls[ci];
        bn[ci].assign(c.B, 0.0);
        rel[ci].assign(c.B, 1.0);
        iters[ci].assign(c.B, 0);
        outer[ci].assign(c.B, 0);
        fin[ci].assign(c.B, 0);
        if (hipStreamWaitEvent(c.s, ready, 0) != hipSuccess) st = FL_E_DEVICE;
        for (int z = 0; z < c.B && st == FL_OK; ++z)
            if (hipMemcpyAsync(c.b + z * c.M, f[c.idx[z]], sizeof(double) * c.M, hipMemcpyDeviceToDevice, c.s) !=
                hipSuccess)
                st = FL_E_DEVICE;
        hipLaunchKernelGGL(k_zero<double>, dim3(ew_grid(c.B * c.M)), dim3(256), 0, c.s, c.x, c.B * c.M);
        VecLayout L = layout(c.M);
        hipLaunchKernelGGL(k_dot<double>, dim3(L.blocks, c.B), dim3(kVecBlock), 0, c.s, c.b, c.b, L.n, L.chunk,
                           c.partA, (const double *)nullptr);
        hipLaunchKernelGGL(k_finish, dim3(1, c.B), dim3(kVecBlock), 0, c.s, c.partA, L.blocks, c.scal, (int)S_DOT);
    }
    const int cap = max_iter > 0 ? max_iter : 1 << 30;
    const size_t nc = b->cls.size();
    b->host_waits = 0;
    b->graph_launches = 0;
    // every class's scalars to the host, one wait for all of them (on `main`)
    auto read_all = [&]() -> fl_status {
        for (size_t ci = 0; ci < nc; ++ci) {
            BatchClass &c = b->cls[ci];
            FL_TRY(stream_after(b->main, c.s, b->joins[ci]));
        }
        for (auto &c : b->cls)
            FL_HIP_TRY(hipMemcpyAsync(c.hscal, c.scal, sizeof(double) * c.B * S_COUNT, hipMemcpyDeviceToHost,
                                      b->main));
        FL_HIP_TRY(hipStreamSynchronize(b->main));
        b->host_waits += 1;
        return FL_OK;
    };
    if (st == FL_OK) st = read_all();
    for (size_t ci = 0; ci < nc && st == FL_OK; ++ci) {
        BatchClass &c = b->cls[ci];
        for (int z = 0; z < c.B && st == FL_OK; ++z) {
            bn[ci][z] = std::sqrt(c.hscal[z * S_COUNT + S_DOT]);
            if (!std::isfinite(bn[ci][z])) st = FL_E_BREAKDOWN;
            if (bn[ci][z] == 0.0) { fin[ci][z] = 1; rel[ci][z] = 0.0; }
        }
    }
    int rounds = 1;  // chunk replays before the next wait (grows; carried to the next step)
    for (int outer_it = 0; st == FL_OK && outer_it < 200; ++outer_it) {
        // FP64 residuals of every class
        for (size_t ci = 0; ci < nc && st == FL_OK; ++ci) {
            BatchClass &c = b->cls[ci];
            Epi<double> ep;
            ep.w1 = c.b;
            ep.a1 = 1.0;
            ep.scale = -1.0;
            st = matvec_ctx<double>(c.c64, c.var64, c.x, c.r64, ep, nullptr, c.s);
            VecLayout L = layout(c.M);
            hipLaunchKernelGGL(k_dot<double>, dim3(L.blocks, c.B), dim3(kVecBlock), 0, c.s, c.r64, c.r64, L.n,
                               L.chunk, c.partA, (const double *)nullptr);
            hipLaunchKernelGGL(k_finish, dim3(1, c.B), dim3(kVecBlock), 0, c.s, c.partA, L.blocks, c.scal,
                               (int)S_DOT);
        }
        if (st == FL_OK) st = read_all();
        bool all = true;
        for (size_t ci = 0; ci < nc && st == FL_OK; ++ci) {
            BatchClass &c = b->cls[ci];
            for (int z = 0; z < c.B; ++z) {
                double &r2 = c.hrel2[z];
                if (fin[ci][z]) { r2 = -1.0; continue; }
                const double r = std::sqrt(c.hscal[z * S_COUNT + S_DOT]) / bn[ci][z];
                rel[ci][z] = r;
                outer[ci][z] += 1;
                if (!std::isfinite(r)) { st = FL_E_BREAKDOWN; break; }
                if (r <= tol || iters[ci][z] >= cap) { fin[ci][z] = 1; r2 = -1.0; continue; }
                double want = 0.5 * tol / r;
                double itol = want > inner_tol ? want : inner_tol;
                if (itol >= 1.0) itol = 0.5;
                r2 = itol * itol;
                all = false;
            }
            // hrel2 is pinned and not written again before the next wait
            if (st == FL_OK &&
                hipMemcpyAsync(c.rel2, c.hrel2, sizeof(double) * c.B, hipMemcpyHostToDevice, c.s) != hipSuccess)
                st = FL_E_DEVICE;
        }
        if (st != FL_OK || all) break;
        // inner FP32 CG of every class: init on the class streams, then the
        // all-class chunk graph replayed on `main` until every problem is done
        for (size_t ci = 0; ci < nc; ++ci) {
            BatchClass &c = b->cls[ci];
            VecLayout L = layout(c.M);
            const long BM = (long)c.B * c.M;
            hipLaunchKernelGGL((k_copy_cast<float, double>), dim3(ew_grid(BM)), dim3(256), 0, c.s, c.r32, c.r64, BM);
            hipLaunchKernelGGL(k_zero<float>, dim3(ew_grid(BM)), dim3(256), 0, c.s, c.d32, BM);
            hipLaunchKernelGGL(k_dot<float>, dim3(L.blocks, c.B), dim3(kVecBlock), 0, c.s, c.r32, c.r32, L.n, L.chunk,
                               c.partB, (const double *)nullptr);
            if (c.tau) {
                // z = M^{-1} r, p = z, (r, z) into the S_RR slots
                if (matvec_ctx<float>(c.c32t, c.var32, c.r32, c.z32, Epi<float>{}, nullptr, c.s) != FL_OK)
                    st = FL_E_DEVICE;
                hipLaunchKernelGGL((k_copy_cast<float, float>), dim3(ew_grid(BM)), dim3(256), 0, c.s, c.p32, c.z32,
                                   BM);
                hipLaunchKernelGGL(k_dot<float>, dim3(L.blocks, c.B), dim3(kVecBlock), 0, c.s, c.r32, c.z32, L.n,
                                   L.chunk, c.partC, (const double *)nullptr);
                hipLaunchKernelGGL(k_pcg_init, dim3(1, c.B), dim3(kVecBlock), 0, c.s, c.partB, c.partC, L.blocks,
                                   c.scal, 0.0, (const double *)c.rel2);
            } else {
                hipLaunchKernelGGL((k_copy_cast<float, float>), dim3(ew_grid(BM)), dim3(256), 0, c.s, c.p32, c.r32,
                                   BM);
                hipLaunchKernelGGL(k_cg_init, dim3(1, c.B), dim3(kVecBlock), 0, c.s, c.partB, L.blocks, c.scal, 0.0,
                                   0.0, (const double *)c.rel2);
            }
            if (st == FL_OK) st = stream_after(b->main, c.s, b->joins[ci]);
        }
        int launched = 0;  // chunk replays this step
        while (st == FL_OK) {
            for (int r = 0; r < rounds && st == FL_OK; ++r)
                if (hipGraphLaunch(b->all, b->main) != hipSuccess) st = FL_E_DEVICE;
            launched += rounds;
            b->graph_launches += rounds;
            if (st == FL_OK) st = read_all();
            if (st != FL_OK) break;
            bool done = true;
            for (size_t ci = 0; ci < nc && done; ++ci) {
                BatchClass &c = b->cls[ci];
                for (int z = 0; z < c.B; ++z)
                    if (c.hscal[z * S_COUNT + S_DONE] == 0.0 &&
                        iters[ci][z] + (long)launched * c.iters_per_chunk < cap) {
                        done = false;
                        break;
                    }
            }
            if (done) break;
            if (rounds < 64) rounds *= 2;
        }
        // the class streams continue after the graph replays
        for (size_t ci = 0; ci < nc && st == FL_OK; ++ci) {
            BatchClass &c = b->cls[ci];
            st = stream_after(c.s, b->main, b->fork);
            for (int z = 0; z < c.B; ++z)
                if (!fin[ci][z]) iters[ci][z] += (int)c.hscal[z * S_COUNT + S_ITER];
            const long BM = (long)c.B * c.M;
            hipLaunchKernelGGL(k_axpy_to64<float>, dim3(ew_grid(BM)), dim3(256), 0, c.s, c.x, c.d32, BM);
        }
    }
    // scatter solutions
    fl_status worst = st;
    for (size_t ci = 0; ci < b->cls.size(); ++ci) {
        BatchClass &c = b->cls[ci];
        for (int z = 0; z < c.B && st == FL_OK; ++z)
            if (hipMemcpyAsync(u[c.idx[z]], c.x + z * c.M, sizeof(double) * c.M, hipMemcpyDeviceToDevice, c.s) !=
                hipSuccess)
                st = FL_E_DEVICE;
        (void)hipStreamSynchronize(c.s);
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int z = 0; z < c.B; ++z) {
            fl_status ps = st != FL_OK ? st : (rel[ci][z] <= tol ? FL_OK : FL_E_NOCONV);
            if (ps != FL_OK && worst == FL_OK) worst = ps;
            if (infos) {
                fl_info &in = infos[c.idx[z]];
                in = fl_info{};
                in.iters = iters[ci][z];
                in.outer_iters = outer[ci][z];
                in.relres = rel[ci][z];
                in.status = ps;
                in.seconds = secs;
            }
        }
    }
    (void)hipEventDestroy(ready);
    // the caller's stream sees the solutions
    for (auto &c : b->cls) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) {
            (void)hipEventRecord(e, c.s);
            (void)hipStreamWaitEvent(us, e, 0);
            (void)hipEventDestroy(e);
        }
    }
    if (worst == FL_E_NOCONV) set_error("some problems did not reach the tolerance");
    return worst;
}

fl_status fl_batch_stats(fl_batch b, int *host_waits, int *graph_launches, int *var32, int *var64) {
    if (!b) { set_error("NULL batch"); return FL_E_INVAL; }
    if (host_waits) *host_waits = b->host_waits;
    if (graph_launches) *graph_launches = b->graph_launches;
    for (size_t ci = 0; ci < b->cls.size(); ++ci) {
        if (var32) var32[ci] = b->cls[ci].var32;
        if (var64) var64[ci] = b->cls[ci].var64;
    }
    return FL_OK;
}

fl_status fl_batch_info(fl_batch b, int *nclasses, int *max_batch) {
    if (!b) { set_error("NULL batch"); return FL_E_INVAL; }
    int mb = 0;
    for (auto &c : b->cls) mb = c.B > mb ? c.B : mb;
    if (nclasses) *nclasses = (int)b->cls.size();
    if (max_batch) *max_batch = mb;
    return FL_OK;
}

}  // extern "C"
