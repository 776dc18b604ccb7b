// fl_fft.hip -- FFT matvec of the multilevel Toeplitz stiffness matrix.
//
// The matrix of the scheme (Sec. 2 block Toeplitz form, Sec. 4 three-level
// form) is A_ij = -c a_{|i-j|}.  Its generator is embedded in a circulant of
// length P (a power of two >= 2n-1) per axis; the circulant's eigenvalues
// lambda are the FFT of the embedded generator (real, even in every axis).
// y = A u is then: zero-pad u to P^d, FFT, multiply by lambda, inverse FFT,
// keep the first n points per axis.
//
// Passes (x fastest, kx the half-spectrum index 0..Q-1, Q = P/2+1):
//   2D: X-fwd (real rows -> half spectra) | Y fused (fwd, x lambda, inv, crop) | X-inv
//   3D: X-fwd | Y-fwd | Z fused | Y-inv | X-inv
// Row passes pack two real rows into one complex line.  Strided passes keep
// C neighbouring columns per workgroup so that every global access is a run
// of C consecutive complex values.
#include <type_traits>

#include "fl_internal.hpp"

namespace fl {

// LDS index maps: row passes store each line contiguously, strided passes
// interleave the C columns of a workgroup (column index fastest).
struct LineMajor {
    int base;
    __device__ __forceinline__ int operator()(int pos) const { return base + pos; }
};
template <int C> struct ColInterleaved {
    int c;
    __device__ __forceinline__ int operator()(int pos) const { return pos * C + c; }
};

template <int P> __device__ __forceinline__ int fold(int k) { return k <= P / 2 ? k : P - k; }

// ---------------------------------------------------------------------------
// row pass, forward: pairs of real rows (n_in values each, zero-padded to P)
// -> Q complex half-spectrum values per row.
// ---------------------------------------------------------------------------
template <typename T, int P, int LPB>
__global__ __launch_bounds__(LPB *(P / Plan<P>::E)) void k_xfwd(
    const T *__restrict__ u, C2<T> *__restrict__ out, int nrows, int n_in, long in_pitch,
    long out_pitch, const C2<T> *__restrict__ tw, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PL = Plan<P>;
    constexpr int E = PL::E, TL = P / E;
    constexpr int R1 = Front<typename PL::Fwd>::value;
    constexpr int RL = Back<typename PL::Fwd>::value;
    __shared__ C2<T> lds[LPB * P];
    const int tl = threadIdx.x % TL;
    const int c = threadIdx.x / TL;
    const long pair = (long)blockIdx.x * LPB + c;
    const long ra = 2 * pair, rb = 2 * pair + 1;
    const bool va = ra < nrows, vb = rb < nrows;
    const T *ua = u + ra * in_pitch;
    const T *ub = u + rb * in_pitch;
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int pos = slot_pos<P, E, R1>(tl, j);
        const T xa = (va && pos < n_in) ? ua[pos] : T(0);
        const T xb = (vb && pos < n_in) ? ub[pos] : T(0);
        v[j] = mk<T>(xa, xb);
    }
    LineMajor lidx{c * P};
    Stages<T, P, E, -1, 1, typename PL::Fwd>::run(v, lds, tl, tw, lidx);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) lds[lidx(slot_pos<P, E, RL>(tl, j))] = v[j];
    __syncthreads();
    if (!va) return;
    C2<T> *oa = out + ra * out_pitch;
    C2<T> *ob = out + rb * out_pitch;
    for (int k = tl; k <= P / 2; k += TL) {
        const C2<T> zk = lds[lidx(k)];
        const C2<T> zm = lds[lidx((P - k) & (P - 1))];
        oa[k] = mk<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y));
        if (vb) ob[k] = mk<T>(T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x));
    }
}

// ---------------------------------------------------------------------------
// row pass, inverse: Q half-spectrum values of two rows -> P real values each,
// first n_out kept.  With EPI, y = a1 w1 + a2 w2 + scale (A u), w1 / w2 read
// at the same position when non-null (shifted operators and residuals of the
// solvers).  A non-null `done` flag that is set makes the kernel a no-op.
// ---------------------------------------------------------------------------
template <typename T, int P, int LPB, bool EPI>
__global__ __launch_bounds__(LPB *(P / Plan<P>::E)) void k_xinv(
    const C2<T> *__restrict__ in, T *__restrict__ y, int nrows, int n_out, long in_pitch,
    long out_pitch, const C2<T> *__restrict__ tw, Epi<T> ep, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PL = Plan<P>;
    constexpr int E = PL::E, TL = P / E;
    constexpr int R1 = Front<typename PL::Inv>::value;
    constexpr int RL = Back<typename PL::Inv>::value;
    __shared__ C2<T> lds[LPB * P];
    const int tl = threadIdx.x % TL;
    const int c = threadIdx.x / TL;
    const long pair = (long)blockIdx.x * LPB + c;
    const long ra = 2 * pair, rb = 2 * pair + 1;
    const bool va = ra < nrows, vb = rb < nrows;
    const C2<T> *ia = in + ra * in_pitch;
    const C2<T> *ib = in + rb * in_pitch;
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int pos = slot_pos<P, E, R1>(tl, j);
        const int kk = pos <= P / 2 ? pos : P - pos;
        C2<T> xa = va ? ia[kk] : mk<T>(0, 0);
        C2<T> xb = vb ? ib[kk] : mk<T>(0, 0);
        if (pos > P / 2) { xa.y = -xa.y; xb.y = -xb.y; }
        if (pos == 0 || pos == P / 2) { xa.y = T(0); xb.y = T(0); }
        v[j] = mk<T>(xa.x - xb.y, xa.y + xb.x);
    }
    LineMajor lidx{c * P};
    Stages<T, P, E, +1, 1, typename PL::Inv>::run(v, lds, tl, tw, lidx);
    if (!va) return;
    T *ya = y + ra * out_pitch;
    T *yb = y + rb * out_pitch;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int pos = slot_pos<P, E, RL>(tl, j);
        if (pos < n_out) {
            T a = v[j].x, b = v[j].y;
            if constexpr (EPI) {
                const long ia2 = ra * out_pitch + pos, ib2 = rb * out_pitch + pos;
                a = ep.scale * a;
                if (ep.w1) a += ep.a1 * ep.w1[ia2];
                if (ep.w2) a += ep.a2 * ep.w2[ia2];
                if (vb) {
                    b = ep.scale * b;
                    if (ep.w1) b += ep.a1 * ep.w1[ib2];
                    if (ep.w2) b += ep.a2 * ep.w2[ib2];
                }
            }
            ya[pos] = a;
            if (vb) yb[pos] = b;
        }
    }
}

// ---------------------------------------------------------------------------
// strided pass over lines along a non-contiguous axis.  Line (o, kx) starts at
// o*outer + kx and steps by line_stride.  MODE 0: forward; 1: inverse;
// 2: forward, multiply by lambda, inverse.  n_in values are read (the rest
// taken as zero), n_out values written.  In-place use is allowed: a
// workgroup reads all of its lines before writing any of them.
// ---------------------------------------------------------------------------
template <typename T, int P, int C, int MODE>
__global__ __launch_bounds__(C *(P / Plan<P>::E)) void k_strided(
    const C2<T> *in, C2<T> *out, int ncols, int n_in, int n_out, long line_stride, long in_outer,
    long out_outer, const C2<T> *__restrict__ tw, const T *__restrict__ lam, long lam_line,
    long lam_outer, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PL = Plan<P>;
    constexpr int E = PL::E, TL = P / E;
    using First = typename std::conditional<MODE == 1, typename PL::Inv, typename PL::Fwd>::type;
    constexpr int R1 = Front<First>::value;
    static_assert(Back<typename PL::Fwd>::value == Front<typename PL::Inv>::value,
                  "inverse plan must start with the forward plan's last radix");
    __shared__ C2<T> lds[C * P];
    const int c = threadIdx.x % C;
    const int tl = threadIdx.x / C;
    const int kx = blockIdx.x * C + c;
    const bool valid = kx < ncols;
    const long o = blockIdx.y;
    const C2<T> *src = in + o * in_outer + kx;
    C2<T> *dst = out + o * out_outer + kx;
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int pos = slot_pos<P, E, R1>(tl, j);
        v[j] = (valid && pos < n_in) ? src[pos * line_stride] : mk<T>(0, 0);
    }
    ColInterleaved<C> lidx{c};
    if constexpr (MODE == 0) {
        Stages<T, P, E, -1, 1, typename PL::Fwd>::run(v, lds, tl, tw, lidx);
        constexpr int RL = Back<typename PL::Fwd>::value;
        if (!valid) return;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = slot_pos<P, E, RL>(tl, j);
            if (pos < n_out) dst[pos * line_stride] = v[j];
        }
    } else if constexpr (MODE == 1) {
        Stages<T, P, E, +1, 1, typename PL::Inv>::run(v, lds, tl, tw, lidx);
        constexpr int RL = Back<typename PL::Inv>::value;
        if (!valid) return;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = slot_pos<P, E, RL>(tl, j);
            if (pos < n_out) dst[pos * line_stride] = v[j];
        }
    } else {
        Stages<T, P, E, -1, 1, typename PL::Fwd>::run(v, lds, tl, tw, lidx);
        constexpr int RM = Back<typename PL::Fwd>::value;
        const T *lo = lam + (long)fold<P>((int)o) * lam_outer + kx;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = slot_pos<P, E, RM>(tl, j);
            const T l = valid ? lo[(long)fold<P>(pos) * lam_line] : T(0);
            v[j] = cscale<T>(v[j], l);
        }
        __syncthreads();
        Stages<T, P, E, +1, 1, typename PL::Inv>::run(v, lds, tl, tw, lidx);
        constexpr int RL = Back<typename PL::Inv>::value;
        if (!valid) return;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = slot_pos<P, E, RL>(tl, j);
            if (pos < n_out) dst[pos * line_stride] = v[j];
        }
    }
}

// ---------------------------------------------------------------------------
// launch shapes
// ---------------------------------------------------------------------------
template <typename T, int P> struct Shape {
    static constexpr int TL = P / Plan<P>::E;
    static constexpr int LPB = TL >= 256 ? 1 : 256 / TL;  // row passes: line pairs per block
    static constexpr int CB = (int)sizeof(C2<T>) * P;     // bytes per column line
    // strided passes: columns per block, at most 32, at most 512 threads
    // (1024 at P >= 2048) and at most 64 KB of LDS (128 KB at P >= 2048)
    static constexpr int thr = P >= 2048 ? 1024 : 512;
    static constexpr int cth = thr / TL < 1 ? 1 : (thr / TL > 32 ? 32 : thr / TL);
    static constexpr int clds = (P >= 2048 ? 131072 : 65536) / CB;
    static constexpr int C = cth < clds ? cth : (clds < 1 ? 1 : clds);
};

static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

template <typename T, int P>
static void launch_xfwd(const T *u, C2<T> *out, int nrows, int n_in, long in_pitch, long out_pitch,
                        const C2<T> *tw, const double *done, hipStream_t s) {
    using S = Shape<T, P>;
    const int pairs = (nrows + 1) / 2;
    hipLaunchKernelGGL((k_xfwd<T, P, S::LPB>), dim3(cdiv(pairs, S::LPB)), dim3(S::LPB * S::TL), 0, s,
                       u, out, nrows, n_in, in_pitch, out_pitch, tw, done);
}

template <typename T, int P>
static void launch_xinv(const C2<T> *in, T *y, int nrows, int n_out, long in_pitch, long out_pitch,
                        const C2<T> *tw, const Epi<T> &ep, const double *done, hipStream_t s) {
    using S = Shape<T, P>;
    const int pairs = (nrows + 1) / 2;
    if (ep.active())
        hipLaunchKernelGGL((k_xinv<T, P, S::LPB, true>), dim3(cdiv(pairs, S::LPB)), dim3(S::LPB * S::TL),
                           0, s, in, y, nrows, n_out, in_pitch, out_pitch, tw, ep, done);
    else
        hipLaunchKernelGGL((k_xinv<T, P, S::LPB, false>), dim3(cdiv(pairs, S::LPB)), dim3(S::LPB * S::TL),
                           0, s, in, y, nrows, n_out, in_pitch, out_pitch, tw, ep, done);
}

template <typename T, int P, int MODE>
static void launch_strided(const C2<T> *in, C2<T> *out, int ncols, int nouter, int n_in, int n_out,
                           long line_stride, long in_outer, long out_outer, const C2<T> *tw,
                           const T *lam, long lam_line, long lam_outer, const double *done, hipStream_t s) {
    using S = Shape<T, P>;
    hipLaunchKernelGGL((k_strided<T, P, S::C, MODE>), dim3(cdiv(ncols, S::C), nouter), dim3(S::C * S::TL),
                       0, s, in, out, ncols, n_in, n_out, line_stride, in_outer, out_outer, tw, lam,
                       lam_line, lam_outer, done);
}

// ---------------------------------------------------------------------------
// the matvec
// ---------------------------------------------------------------------------
template <typename T> static const C2<T> *twid(fl_op op);
template <> const float2 *twid<float>(fl_op op) { return op->tw32; }
template <> const double2 *twid<double>(fl_op op) { return op->tw64; }
template <typename T> static const T *lamb(fl_op op);
template <> const float *lamb<float>(fl_op op) { return op->lam32; }
template <> const double *lamb<double>(fl_op op) { return op->lam64; }

template <typename T, int P>
static void matvec_p(fl_op op, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                     hipEvent_t *ev) {
    const int n = op->n, Q = op->Q;
    const long Qp = op->Qp;
    C2<T> *T1 = (C2<T> *)op->T1;
    C2<T> *T2 = (C2<T> *)op->T2;
    const C2<T> *tw = twid<T>(op);
    const T *lam = lamb<T>(op);
    // ev (optional): ev[0] before the first pass, ev[i+1] after pass i
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], s);
    };
    mark(0);
    if (op->d == 2) {
        launch_xfwd<T, P>(u, T1, n, n, n, Qp, tw, done, s);
        mark(1);
        launch_strided<T, P, 2>(T1, T1, Q, 1, n, n, Qp, 0, 0, tw, lam, Q, 0, done, s);
        mark(2);
        launch_xinv<T, P>(T1, y, n, n, Qp, n, tw, ep, done, s);
        mark(3);
    } else {
        const long nn = (long)n * n;
        launch_xfwd<T, P>(u, T1, (int)nn, n, n, Qp, tw, done, s);
        mark(1);
        launch_strided<T, P, 0>(T1, T2, Q, n, n, P, Qp, n * Qp, (long)P * Qp, tw, nullptr, 0, 0, done, s);
        mark(2);
        launch_strided<T, P, 2>(T2, T2, Q, P, n, n, (long)P * Qp, Qp, Qp, tw, lam, (long)Q * Q, Q, done, s);
        mark(3);
        launch_strided<T, P, 1>(T2, T1, Q, n, P, n, Qp, (long)P * Qp, n * Qp, tw, nullptr, 0, 0, done, s);
        mark(4);
        launch_xinv<T, P>(T1, y, (int)nn, n, Qp, n, tw, ep, done, s);
        mark(5);
    }
}

template <typename T>
fl_status matvec_ex(fl_op op, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                    hipEvent_t *ev) {
    switch (op->P) {
        case 8: matvec_p<T, 8>(op, u, y, ep, done, s, ev); break;
        case 16: matvec_p<T, 16>(op, u, y, ep, done, s, ev); break;
        case 32: matvec_p<T, 32>(op, u, y, ep, done, s, ev); break;
        case 64: matvec_p<T, 64>(op, u, y, ep, done, s, ev); break;
        case 128: matvec_p<T, 128>(op, u, y, ep, done, s, ev); break;
        case 256: matvec_p<T, 256>(op, u, y, ep, done, s, ev); break;
        case 512: matvec_p<T, 512>(op, u, y, ep, done, s, ev); break;
        case 1024: matvec_p<T, 1024>(op, u, y, ep, done, s, ev); break;
        case 2048: matvec_p<T, 2048>(op, u, y, ep, done, s, ev); break;
        default: set_error("FFT length %d not built", op->P); return FL_E_UNSUPPORTED;
    }
    FL_HIP_TRY(hipGetLastError());
    return FL_OK;
}

template <typename T>
fl_status matvec(fl_op op, const T *u, T *y, hipStream_t s) {
    return matvec_ex<T>(op, u, y, Epi<T>{}, nullptr, s);
}
template fl_status matvec<float>(fl_op, const float *, float *, hipStream_t);
template fl_status matvec<double>(fl_op, const double *, double *, hipStream_t);
template fl_status matvec_ex<float>(fl_op, const float *, float *, const Epi<float> &, const double *, hipStream_t,
                                    hipEvent_t *);
template fl_status matvec_ex<double>(fl_op, const double *, double *, const Epi<double> &, const double *,
                                     hipStream_t, hipEvent_t *);

int kernel_p_supported(int P) { return P >= 8 && P <= 2048 && (P & (P - 1)) == 0; }

// ---------------------------------------------------------------------------
// eigenvalues of the circulant embedding (FP64)
// ---------------------------------------------------------------------------

// generator -c a_{|m|} embedded with period P per axis; zero in the gap
__global__ void k_embed(const double *__restrict__ a, double *__restrict__ cemb, int d, int N, int P,
                        double negc) {
    const long total = d == 2 ? (long)P * P : (long)P * P * P;
    const int n = N - 1, V = N + 1;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        long t = idx;
        long off = 0, mul = 1;
        bool zero = false;
        for (int k = 0; k < d; ++k) {
            int m = (int)(t % P);
            t /= P;
            int f = m <= n - 1 ? m : (m >= P - (n - 1) ? P - m : -1);
            if (f < 0) zero = true;
            off += (long)(f < 0 ? 0 : f) * mul;
            mul *= V;
        }
        cemb[idx] = zero ? 0.0 : negc * a[off];
    }
}

__global__ void k_extract(const double2 *__restrict__ spec, double *__restrict__ lam64, float *__restrict__ lam32,
                          int d, int P, int Q, long Qp, double inv) {
    const long total = d == 2 ? (long)Q * Q : (long)Q * Q * Q;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        const long kx = idx % Q;
        const long rest = idx / Q;
        long src;
        if (d == 2) src = rest * Qp + kx;
        else {
            const long ky = rest % Q, kz = rest / Q;
            src = (kz * P + ky) * Qp + kx;
        }
        const double l = spec[src].x * inv;
        lam64[idx] = l;
        lam32[idx] = (float)l;
    }
}

template <int P>
static void symbol_fft(double *cemb, double2 *T, int d, const double2 *tw, hipStream_t s) {
    const int Q = P / 2 + 1;
    const long Qp = ((Q + 15) / 16) * 16;
    if (d == 2) {
        launch_xfwd<double, P>(cemb, T, P, P, P, Qp, tw, nullptr, s);
        launch_strided<double, P, 0>(T, T, Q, 1, P, P, Qp, 0, 0, tw, nullptr, 0, 0, nullptr, s);
    } else {
        launch_xfwd<double, P>(cemb, T, P * P, P, P, Qp, tw, nullptr, s);
        launch_strided<double, P, 0>(T, T, Q, P, P, P, Qp, (long)P * Qp, (long)P * Qp, tw, nullptr, 0, 0, nullptr, s);
        launch_strided<double, P, 0>(T, T, Q, P, P, P, (long)P * Qp, Qp, Qp, tw, nullptr, 0, 0, nullptr, s);
    }
}

fl_status build_symbol(fl_op op, hipStream_t s) {
    const int d = op->d, P = op->P, Q = op->Q;
    const long Qp = op->Qp;
    const long total = d == 2 ? (long)P * P : (long)P * P * P;
    const long rows = total / P;
    double *cemb = nullptr;
    double2 *T = nullptr;
    FL_HIP_TRY(hipMalloc((void **)&cemb, sizeof(double) * total));
    hipError_t e = hipMalloc((void **)&T, sizeof(double2) * rows * Qp);
    if (e != hipSuccess) {
        (void)hipFree(cemb);
        set_error("workspace for the symbol: %s", hipGetErrorString(e));
        return FL_E_NOMEM;
    }
    hipLaunchKernelGGL(k_embed, dim3(cdiv(total, 256) > 65536 ? 65536 : cdiv(total, 256)), dim3(256), 0, s,
                       op->a, cemb, d, op->N, P, -op->c);
    switch (P) {
        case 8: symbol_fft<8>(cemb, T, d, op->tw64, s); break;
        case 16: symbol_fft<16>(cemb, T, d, op->tw64, s); break;
        case 32: symbol_fft<32>(cemb, T, d, op->tw64, s); break;
        case 64: symbol_fft<64>(cemb, T, d, op->tw64, s); break;
        case 128: symbol_fft<128>(cemb, T, d, op->tw64, s); break;
        case 256: symbol_fft<256>(cemb, T, d, op->tw64, s); break;
        case 512: symbol_fft<512>(cemb, T, d, op->tw64, s); break;
        case 1024: symbol_fft<1024>(cemb, T, d, op->tw64, s); break;
        case 2048: symbol_fft<2048>(cemb, T, d, op->tw64, s); break;
        default: break;
    }
    const long ql = d == 2 ? (long)Q * Q : (long)Q * Q * Q;
    const double inv = 1.0 / (double)total;
    hipLaunchKernelGGL(k_extract, dim3(cdiv(ql, 256) > 65536 ? 65536 : cdiv(ql, 256)), dim3(256), 0, s, T,
                       op->lam64, op->lam32, d, P, Q, Qp, inv);
    hipError_t le = hipGetLastError();
    hipError_t se = hipStreamSynchronize(s);
    (void)hipFree(cemb);
    (void)hipFree(T);
    FL_HIP_TRY(le);
    FL_HIP_TRY(se);
    return FL_OK;
}

}  // namespace fl
