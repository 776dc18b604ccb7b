// fl_coeff.hip -- FP64 coefficients of the scheme on the GPU.
//
// With splitting parameter gamma in (alpha, 2] (2 is the paper's default,
// Sec. 5) and q = d + alpha - gamma, the scheme needs (Sec. 2 for d = 2,
// Sec. 4 for d = 3 and for d = 1, the one-dimensional case of its general-d
// scheme):
//   * element integrals E_e = int_{I_e} |xi|^{-q}, I_e = prod [e_i h, (e_i+1) h];
//   * vertex weights W_v = sum of E_e over the elements having xi_v as a vertex
//     (the patch T_v, restricted to (0, L)^d, vertices 0..N per axis), plus the
//     origin-element correction of the gamma = 2 limit rule (none for
//     gamma < 2, where the limit of psi_gamma at the origin is 0): in 2D +E_0
//     on (1,0), (0,1) and -E_0 on (1,1); in 3D +5/3 E_0 on the axis unit
//     vectors and -E_0 on every other vertex of the unit cube; in 1D +E_0 on
//     vertex 1 (psi_2 tends to u'' at the origin, taken as psi_2 at xi = h);
//   * a_v = 2^{sigma(v)} W_v / (2^d |xi_v|^gamma), sigma = number of zero indices;
//   * a_0 = -sum_{v != 0} W_v / |xi_v|^gamma - 2^d D2, D2 the integral of
//     |xi|^{-(d+alpha)} over R^d_+ minus (0, L)^d, L = N h.
// Closed forms (pyramid split of the cube corner along its diagonal planes):
//   E_0 = d h^{d-q} J(q) / (d - q),   D2 = d L^{-alpha} J(d + alpha) / alpha,
//   J(p) = int_{[0,1]^{d-1}} (1 + |s|^2)^{-p/2} ds.
// Every other element integral uses tensor Gauss-Legendre quadrature whose
// order drops with the distance from the origin (the integrand is analytic on
// those elements; its nearest singularity lies at the origin).
#include <cmath>
#include <vector>

#include "fl_internal.hpp"

namespace fl {

// Gauss-Legendre rules: orders kOrders[i] stored back to back, then the
// 40-point rule for J.
constexpr int kNumRules = 6;
constexpr int kOrders[kNumRules] = {20, 14, 9, 6, 5, 40};
constexpr int kRuleTotal = 20 + 14 + 9 + 6 + 5 + 40;
__constant__ double c_glx[kRuleTotal];
__constant__ double c_glw[kRuleTotal];
__constant__ int c_gloff[kNumRules];

// Newton iteration on the Legendre polynomial from Tricomi's asymptotic
// estimate of its roots; weights 2 / ((1 - x^2) P_n'(x)^2).
static void legendre_rule(int n, double *x, double *w) {
    const long double pi = 3.14159265358979323846264338327950288L;
    for (int k = 1; k <= n; ++k) {
        long double th = pi * (4.0L * k - 1.0L) / (4.0L * n + 2.0L);
        long double z = (1.0L - 1.0L / (8.0L * n * n) + 1.0L / (8.0L * n * n * n)) * cosl(th);
        long double dp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            long double pm = 1.0L, p = z;
            for (int j = 2; j <= n; ++j) {
                long double pn = ((2.0L * j - 1.0L) * z * p - (j - 1.0L) * pm) / j;
                pm = p;
                p = pn;
            }
            if (n == 1) pm = 1.0L;
            dp = n * (pm - z * p) / (1.0L - z * z);
            long double dz = p / dp;
            z -= dz;
            if (fabsl(dz) <= 1e-20L * (1.0L + fabsl(z))) {
                // final derivative at the converged root
                pm = 1.0L;
                p = z;
                for (int j = 2; j <= n; ++j) {
                    long double pn = ((2.0L * j - 1.0L) * z * p - (j - 1.0L) * pm) / j;
                    pm = p;
                    p = pn;
                }
                if (n == 1) pm = 1.0L;
                dp = n * (pm - z * p) / (1.0L - z * z);
                break;
            }
        }
        x[k - 1] = (double)z;  // descending; symmetric rules, order irrelevant
        w[k - 1] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
    }
}

static fl_status upload_rules() {
    static bool done[64] = {false};
    int dev = 0;
    FL_HIP_TRY(hipGetDevice(&dev));
    if (dev < 64 && done[dev]) return FL_OK;
    std::vector<double> x(kRuleTotal), w(kRuleTotal);
    int off[kNumRules];
    int o = 0;
    for (int i = 0; i < kNumRules; ++i) {
        off[i] = o;
        legendre_rule(kOrders[i], x.data() + o, w.data() + o);
        o += kOrders[i];
    }
    FL_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_glx), x.data(), sizeof(double) * kRuleTotal));
    FL_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_glw), w.data(), sizeof(double) * kRuleTotal));
    FL_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_gloff), off, sizeof(off)));
    if (dev < 64) done[dev] = true;
    return FL_OK;
}

__device__ __forceinline__ int order_of(int r) {
    switch (r) {
        case 0: return 20;
        case 1: return 14;
        case 2: return 9;
        case 3: return 6;
        case 4: return 5;
        default: return 40;
    }
}

// rule index for an element whose largest index (in units of h) is m >= 1
__device__ __forceinline__ int rule_for(int m) {
    return m <= 2 ? 0 : m <= 8 ? 1 : m <= 32 ? 2 : m <= 128 ? 3 : 4;
}

// J(p1), J(p2) and the closed forms E_0, D2 -> scal[0], scal[1]
__global__ __launch_bounds__(256) void k_closed_forms(int d, double alpha, double gamma, double h, int N,
                                                      double *scal) {
    __shared__ double s1[256], s2[256];
    const int r = 5;  // 40-point rule
    const int n = order_of(r);
    const int off = c_gloff[r];
    const double q = d + alpha - gamma, p2 = d + alpha;
    double a1 = 0.0, a2 = 0.0;
    // d = 1: J = 1 (no angular integral); one thread adds it
    const int total = d == 1 ? 1 : d == 2 ? n : n * n;
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int i = t % n, j = t / n;
        double s2sum, wt;
        if (d == 1) {
            s2sum = 0.0;
            wt = 1.0;
        } else if (d == 2) {
            const double s = 0.5 * (c_glx[off + i] + 1.0);
            s2sum = s * s;
            wt = 0.5 * c_glw[off + i];
        } else {
            const double s = 0.5 * (c_glx[off + i] + 1.0), u = 0.5 * (c_glx[off + j] + 1.0);
            s2sum = s * s + u * u;
            wt = 0.25 * c_glw[off + i] * c_glw[off + j];
        }
        a1 += wt * pow(1.0 + s2sum, -0.5 * q);
        a2 += wt * pow(1.0 + s2sum, -0.5 * p2);
    }
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            s1[threadIdx.x] += s1[threadIdx.x + k];
            s2[threadIdx.x] += s2[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double L = N * h;
        scal[0] = d * pow(h, d - q) * s1[0] / (d - q);
        scal[1] = d * pow(L, -alpha) * s2[0] / alpha;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_elements(double alpha, double gamma, double h, int N, const double *scal,
                                                  double *E) {
    const long total = D == 1 ? (long)N : D == 2 ? (long)N * N : (long)N * N * N;
    const double q = D + alpha - gamma;
    const double hq = pow(h, D - q);
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        if (idx == 0) {
            E[0] = scal[0];
            continue;
        }
        int e[3] = {0, 0, 0};
        long t = idx;
        int m = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            e[k] = (int)(t % N);
            t /= N;
            m = e[k] > m ? e[k] : m;
        }
        const int r = rule_for(m);
        const int n = order_of(r), off = c_gloff[r];
        double acc = 0.0;
        if (D == 1) {
            for (int i = 0; i < n; ++i) {
                const double x = e[0] + 0.5 * (c_glx[off + i] + 1.0);
                acc += c_glw[off + i] * pow(x, -q);
            }
            E[idx] = 0.5 * hq * acc;
        } else if (D == 2) {
            for (int i = 0; i < n; ++i) {
                const double x = e[0] + 0.5 * (c_glx[off + i] + 1.0);
                double row = 0.0;
                for (int j = 0; j < n; ++j) {
                    const double y = e[1] + 0.5 * (c_glx[off + j] + 1.0);
                    row += c_glw[off + j] * pow(x * x + y * y, -0.5 * q);
                }
                acc += c_glw[off + i] * row;
            }
            E[idx] = 0.25 * hq * acc;
        } else {
            for (int i = 0; i < n; ++i) {
                const double x = e[0] + 0.5 * (c_glx[off + i] + 1.0);
                double plane = 0.0;
                for (int j = 0; j < n; ++j) {
                    const double y = e[1] + 0.5 * (c_glx[off + j] + 1.0);
                    double row = 0.0;
                    for (int k = 0; k < n; ++k) {
                        const double z = e[2] + 0.5 * (c_glx[off + k] + 1.0);
                        row += c_glw[off + k] * pow(x * x + y * y + z * z, -0.5 * q);
                    }
                    plane += c_glw[off + j] * row;
                }
                acc += c_glw[off + i] * plane;
            }
            E[idx] = 0.125 * hq * acc;
        }
    }
}

// a_v and the a_0 summand W_v / |xi_v|^gamma for every vertex v != 0
template <int D>
__global__ __launch_bounds__(256) void k_vertex(const double *__restrict__ E, int N, double h, double gamma, double *a,
                                                double *term) {
    const int V = N + 1;
    const long total = D == 1 ? (long)V : D == 2 ? (long)V * V : (long)V * V * V;
    const double E0 = E[0];
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        if (idx == 0) {
            term[0] = 0.0;
            continue;
        }
        int v[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        long t = idx;
        int nz = 0, mx = 0;
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            v[k] = (int)(t % V);
            t /= V;
            lo[k] = v[k] > 0 ? v[k] - 1 : 0;
            hi[k] = v[k] < N ? v[k] : N - 1;
            nz += v[k] == 0;
            mx = v[k] > mx ? v[k] : mx;
            r2 += (double)v[k] * v[k];
        }
        double W = 0.0;
        if (D == 1) {
            for (int i = lo[0]; i <= hi[0]; ++i) W += E[i];
        } else if (D == 2) {
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) W += E[i + (long)N * j];
        } else {
            for (int k = lo[2]; k <= hi[2]; ++k)
                for (int j = lo[1]; j <= hi[1]; ++j)
                    for (int i = lo[0]; i <= hi[0]; ++i) W += E[i + (long)N * (j + (long)N * k)];
        }
        if (mx == 1 && gamma == 2.0) {  // floor(gamma/2) = 1 only for gamma = 2
            const bool axis = (D - nz) == 1;
            W += axis ? (D == 3 ? (5.0 / 3.0) * E0 : E0) : -E0;
        }
        const double den = gamma == 2.0 ? r2 * h * h : pow(r2 * h * h, 0.5 * gamma);
        term[idx] = W / den;
        a[idx] = (double)(1 << nz) * W / ((double)(1 << D) * den);
    }
}

// deterministic two-level sum: block b adds a fixed contiguous chunk
__global__ __launch_bounds__(256) void k_sum_partial(const double *__restrict__ x, long n, long chunk, double *part) {
    __shared__ double s[256];
    const long beg = (long)blockIdx.x * chunk;
    const long end = beg + chunk < n ? beg + chunk : n;
    double acc = 0.0;
    for (long i = beg + threadIdx.x; i < end; i += 256) acc += x[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_a0_final(const double *__restrict__ part, int np, const double *scal, int d,
                                                  double *a) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) a[0] = -s[0] - (double)(1 << d) * scal[1];
}

static inline int grid_for(long total, int block = 256, int cap = 65536) {
    long g = (total + block - 1) / block;
    return (int)(g > cap ? cap : (g < 1 ? 1 : g));
}

// Fills op->a ((N+1)^d values) on stream s.
fl_status build_coeffs(fl_op op, hipStream_t s) {
    FL_TRY(upload_rules());
    const int d = op->d, N = op->N;
    long ne = 1, nv = 1;
    for (int k = 0; k < d; ++k) {
        ne *= N;
        nv *= N + 1;
    }
    const long chunk = 4096;
    const int np = (int)((nv + chunk - 1) / chunk);
    double *E = nullptr, *term = nullptr, *part = nullptr, *scal = nullptr;
    size_t bytes = sizeof(double) * (ne + nv + np + 8);
    void *buf = nullptr;
    FL_HIP_TRY(hipMalloc(&buf, bytes));
    E = (double *)buf;
    term = E + ne;
    part = term + nv;
    scal = part + np;
    const double g = op->gamma;
    hipLaunchKernelGGL(k_closed_forms, dim3(1), dim3(256), 0, s, d, op->alpha, g, op->h, N, scal);
    if (d == 1) {
        hipLaunchKernelGGL(k_elements<1>, dim3(grid_for(ne)), dim3(256), 0, s, op->alpha, g, op->h, N, scal, E);
        hipLaunchKernelGGL(k_vertex<1>, dim3(grid_for(nv)), dim3(256), 0, s, E, N, op->h, g, op->a, term);
    } else if (d == 2) {
        hipLaunchKernelGGL(k_elements<2>, dim3(grid_for(ne)), dim3(256), 0, s, op->alpha, g, op->h, N, scal, E);
        hipLaunchKernelGGL(k_vertex<2>, dim3(grid_for(nv)), dim3(256), 0, s, E, N, op->h, g, op->a, term);
    } else {
        hipLaunchKernelGGL(k_elements<3>, dim3(grid_for(ne)), dim3(256), 0, s, op->alpha, g, op->h, N, scal, E);
        hipLaunchKernelGGL(k_vertex<3>, dim3(grid_for(nv)), dim3(256), 0, s, E, N, op->h, g, op->a, term);
    }
    hipLaunchKernelGGL(k_sum_partial, dim3(np), dim3(256), 0, s, term, nv, chunk, part);
    hipLaunchKernelGGL(k_a0_final, dim3(1), dim3(256), 0, s, part, np, scal, d, op->a);
    hipError_t le = hipGetLastError();
    hipError_t se = hipStreamSynchronize(s);
    (void)hipFree(buf);
    FL_HIP_TRY(le);
    FL_HIP_TRY(se);
    return FL_OK;
}

}  // namespace fl
