// fl_internal.hpp -- shared internals of the gfx950 fractional Laplacian library:
// complex helpers, the in-register DFT butterflies, the Stockham stage
// helpers, the operator object and error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/fl.h"

namespace fl {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const char *fmt, ...);

#define FL_HIP_TRY(expr)                                                              \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ::fl::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                            __FILE__, __LINE__);                                      \
            return e_ == hipErrorOutOfMemory ? FL_E_NOMEM : FL_E_DEVICE;              \
        }                                                                             \
    } while (0)

#define FL_TRY(expr)                                                                  \
    do {                                                                              \
        fl_status s_ = (expr);                                                        \
        if (s_ != FL_OK) return s_;                                                   \
    } while (0)

// ---------------------------------------------------------------------------
// complex values: float2 / double2 with the arithmetic the FFT needs
// ---------------------------------------------------------------------------
template <typename T> struct cvec;
template <> struct cvec<float> { using type = float2; };
template <> struct cvec<double> { using type = double2; };
template <typename T> using C2 = typename cvec<T>::type;

template <typename T> __device__ __forceinline__ C2<T> mk(T x, T y) { C2<T> r; r.x = x; r.y = y; return r; }
template <typename T> __device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// x where b holds, else zero, as two scalar selects: a conditional over the
// vector type compiles to a branch around the load that produced x, and one
// such branch per element serialises a thread's loads behind exec-mask jumps
template <typename T> __device__ __forceinline__ C2<T> keep(bool b, C2<T> x) {
    return mk<T>(b ? x.x : T(0), b ? x.y : T(0));
}
template <typename T> __device__ __forceinline__ C2<T> cconj(C2<T> a) { return mk<T>(a.x, -a.y); }
// multiply by s*i, s = +1 or -1 (exact)
template <typename T, int S> __device__ __forceinline__ C2<T> cmuli(C2<T> a) {
    return S > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// cos(2 pi k / 32), k = 0..8 (the first-quadrant 32nd roots the butterflies need)
constexpr double kCos32[9] = {1.0,
                              0.98078528040323044913, 0.92387953251128675613, 0.83146961230254523708,
                              0.70710678118654752440, 0.55557023301960222474, 0.38268343236508977173,
                              0.19509032201612826785, 0.0};

// w = exp(DIR * 2 pi i k / R) as an exact constant, k < R <= 32
template <typename T, int R, int DIR, int K>
__device__ __forceinline__ C2<T> root() {
    static_assert(R <= 32 && 32 % R == 0, "roots up to the 32nd");
    constexpr int m = (K * 32 / R) & 31;  // in 32nds of a turn
    // cos(2 pi m/32), sin(2 pi m/32) from the first-quadrant table
    constexpr int q = m / 8, r = m % 8;
    constexpr double c0 = kCos32[r], s0 = kCos32[8 - r];
    constexpr double c = q == 0 ? c0 : q == 1 ? -s0 : q == 2 ? -c0 : s0;
    constexpr double s = q == 0 ? s0 : q == 1 ? c0 : q == 2 ? -s0 : -c0;
    return mk<T>((T)c, (T)(DIR * s));
}

// v * exp(DIR 2 pi i K / R) with the trivial rotations done exactly
template <typename T, int R, int DIR, int K>
__device__ __forceinline__ C2<T> rot(C2<T> v) {
    constexpr int m = (K * 32 / R) & 31;
    if constexpr (m == 0) return v;
    else if constexpr (m == 8) return cmuli<T, DIR>(v);
    else if constexpr (m == 16) return mk<T>(-v.x, -v.y);
    else if constexpr (m == 24) return cmuli<T, -DIR>(v);
    else return cmul<T>(v, root<T, R, DIR, K>());
}

// ---------------------------------------------------------------------------
// in-register DFT of length R (R = 1, 2, 4, 8, 16, 32), natural order in and out:
//   v[k] <- sum_r v[r] exp(DIR 2 pi i r k / R)
// radix-2 decimation in time, fully unrolled.
// ---------------------------------------------------------------------------
template <typename T, int R, int DIR> struct Dft {
    template <int K>
    __device__ __forceinline__ static void combine(C2<T> *v, const C2<T> *e, const C2<T> *o) {
        if constexpr (K < R / 2) {
            C2<T> t = rot<T, R, DIR, K>(o[K]);
            v[K] = cadd<T>(e[K], t);
            v[K + R / 2] = csub<T>(e[K], t);
            combine<K + 1>(v, e, o);
        }
    }
    __device__ __forceinline__ static void run(C2<T> *v) {
        C2<T> e[R / 2], o[R / 2];
#pragma unroll
        for (int r = 0; r < R / 2; ++r) { e[r] = v[2 * r]; o[r] = v[2 * r + 1]; }
        Dft<T, R / 2, DIR>::run(e);
        Dft<T, R / 2, DIR>::run(o);
        combine<0>(v, e, o);
    }
};
template <typename T, int DIR> struct Dft<T, 1, DIR> {
    __device__ __forceinline__ static void run(C2<T> *) {}
};
template <typename T, int DIR> struct Dft<T, 2, DIR> {
    __device__ __forceinline__ static void run(C2<T> *v) {
        C2<T> a = v[0], b = v[1];
        v[0] = cadd<T>(a, b);
        v[1] = csub<T>(a, b);
    }
};

// ---------------------------------------------------------------------------
// streaming stores of pass outputs: the next pass reads them on other XCDs,
// so they bypass this XCD's L2 (non-temporal), which also keeps the end of
// the kernel from waiting on dirty L2 lines
// ---------------------------------------------------------------------------
typedef float fvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_stream(float *p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(double *p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(float2 *p, float2 v) {
    fvec2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, (fvec2 *)p);
}
__device__ __forceinline__ void st_stream(double2 *p, double2 v) {
    dvec2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, (dvec2 *)p);
}

// ---------------------------------------------------------------------------
// FFT plans: length P (a power of two), E points per thread (TL = P / E
// threads per line).  Radices greedily as large as E: R[0..L-1], product P.
// ---------------------------------------------------------------------------
template <int P, int E_> struct Plan {
    static_assert((P & (P - 1)) == 0 && (E_ & (E_ - 1)) == 0 && E_ <= P && E_ >= 2, "bad plan");
    static constexpr int E = E_;
    static constexpr int count() {
        int l = 0;
        for (int rem = P; rem > 1; rem /= (rem < E ? rem : E)) ++l;
        return l;
    }
    static constexpr int L = count();
    static constexpr int radix(int s) {
        int rem = P;
        for (int i = 0; i < s; ++i) rem /= (rem < E ? rem : E);
        return rem < E ? rem : E;
    }
    static constexpr int R[6] = {radix(0), L > 1 ? radix(1) : 1, L > 2 ? radix(2) : 1,
                                 L > 3 ? radix(3) : 1, L > 4 ? radix(4) : 1, L > 5 ? radix(5) : 1};
    static_assert(L <= 6, "plan too long");
};

// product of the radices before stage s
template <typename PL> constexpr int stage_ns(int s) {
    int ns = 1;
    for (int i = 0; i < s; ++i) ns *= PL::R[i];
    return ns;
}
// offset of stage s's twiddles in a thread's twiddle registers (stage 0 has none)
template <typename PL> constexpr int stage_tw(int s) {
    int o = 0;
    for (int i = 1; i < s; ++i) o += PL::E - PL::E / PL::R[i];
    return o;
}
template <typename PL> constexpr int num_tw() { return stage_tw<PL>(PL::L) > 0 ? stage_tw<PL>(PL::L) : 1; }

// Stage s of the Stockham (decimation-in-time) forward transform, thread tl,
// register slot j = i*R + r for butterfly b = tl + i*TL:
//   reads x[b + r*(P/R)], multiplies by w^{(b mod Ns) r}, w = exp(-2 pi i/(Ns R)),
//   takes the R-point DFT, writes position (b/Ns)*Ns*R + (b mod Ns) + r*Ns.
template <int P, typename PL, int S> __device__ __forceinline__ int in_pos(int tl, int j) {
    constexpr int R = PL::R[S], TL = P / PL::E;
    return tl + (j / R) * TL + (j % R) * (P / R);
}
template <int P, typename PL, int S> __device__ __forceinline__ int out_pos(int tl, int j) {
    constexpr int R = PL::R[S], TL = P / PL::E, Ns = stage_ns<PL>(S);
    const int b = tl + (j / R) * TL;
    return (b / Ns) * Ns * R + (b % Ns) + (j % R) * Ns;
}

// First-stage inputs v[j] (positions in_pos<0>) of a forward transform: a line
// of stored values extended to period P, ld(i) returning stored value i (i is
// always a valid index).  A thread's slot j lies below P/2 exactly when
// j mod R[0] < R[0]/2, so the half a slot falls in is known at compile time.
//   n_in > P/2        zero past n_in;
//   0 <= n_in <= P/2  zero-padded: the upper half is zero and is not loaded;
//   n_in < 0          odd extension about -1, over the P/2 - 1 points of the
//                     sine basis, of n = -n_in <= P/2 - 1 stored values:
//                     x[p] for p < n, -x[P - 2 - p] where P - 2 - p < n,
//                     zero elsewhere.  Its transform holds only the sine modes
//                     (the Dirichlet sine basis of P/2 - 1 points).
template <typename T, int P, typename PL, typename Ld>
__device__ __forceinline__ void load_line(C2<T> *v, int tl, int n_in, Ld ld) {
    constexpr int R = PL::R[0], E = PL::E;
    static_assert(R >= 2 && R % 2 == 0, "first radix must be even");
    const C2<T> zero = mk<T>(T(0), T(0));
    if (n_in < 0) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = in_pos<P, PL, 0>(tl, j);
            if ((j % R) < R / 2) {
                const bool ok = pos < -n_in;
                v[j] = keep<T>(ok, ld(ok ? pos : 0));
            } else {
                const int src = P - 2 - pos;
                const bool ok = src >= 0 && src < -n_in;
                const C2<T> x = ld(ok ? src : 0);
                v[j] = keep<T>(ok, mk<T>(-x.x, -x.y));
            }
        }
    } else if (n_in <= P / 2) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            if ((j % R) < R / 2) {
                const int pos = in_pos<P, PL, 0>(tl, j);
                const bool ok = pos < n_in;
                v[j] = keep<T>(ok, ld(ok ? pos : 0));
            } else {
                v[j] = zero;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = in_pos<P, PL, 0>(tl, j);
            const bool ok = pos < n_in;
            v[j] = keep<T>(ok, ld(ok ? pos : 0));
        }
    }
}

// every twiddle a thread uses, loaded once from the table exp(-2 pi i m / P)
template <typename T, int P, typename PL, int S = 1>
__device__ __forceinline__ void load_twiddles(C2<T> *tws, const C2<T> *__restrict__ table, int tl) {
    if constexpr (S < PL::L) {
        constexpr int R = PL::R[S], E = PL::E, TL = P / E, Ns = stage_ns<PL>(S), TW = stage_tw<PL>(S);
#pragma unroll
        for (int i = 0; i < E / R; ++i) {
            const int k = (tl + i * TL) % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) tws[TW + i * (R - 1) + r - 1] = table[k * r * (P / (Ns * R))];
        }
        load_twiddles<T, P, PL, S + 1>(tws, table, tl);
    }
}

// Lane-ordered twiddles.  For the plan of length P with E points per thread
// (TL = P / E threads per line), entry k * TL + tl of the plan's table holds the
// k-th twiddle thread tl needs, in the order load_twiddles gathers them; a
// wavefront's k-th twiddle load then reads consecutive entries.  One buffer
// holds the tables of every E = 2, 4, ..., 32 (E <= P), at sched_off(P, E).
constexpr int plan_stages(int P, int E) {
    int l = 0;
    for (int rem = P; rem > 1; rem /= (rem < E ? rem : E)) ++l;
    return l;
}
constexpr int plan_radix(int P, int E, int s) {
    int rem = P;
    for (int i = 0; i < s; ++i) rem /= (rem < E ? rem : E);
    return rem < E ? rem : E;
}
constexpr int plan_tw(int P, int E) {
    int o = 0;
    for (int s = 1; s < plan_stages(P, E); ++s) o += E - E / plan_radix(P, E, s);
    return o > 0 ? o : 1;
}
// the plans the kernels instantiate: at most 6 stages, at most 32 points per thread
constexpr bool plan_ok(int P, int E) { return E >= 2 && E <= P && E <= 32 && plan_stages(P, E) <= 6; }
constexpr long sched_off(int P, int E) {
    long off = 0;
    for (int e = 2; e < E; e *= 2)
        if (plan_ok(P, e)) off += (long)plan_tw(P, e) * (P / e);
    return off;
}
constexpr long sched_len(int P) { return sched_off(P, 64); }

template <typename T, int P, typename PL>
__device__ __forceinline__ void load_twiddles_lanes(C2<T> *tws, const C2<T> *__restrict__ sched, int tl) {
    static_assert(plan_tw(P, PL::E) == num_tw<PL>() && plan_stages(P, PL::E) == PL::L, "plan tables");
    constexpr int TL = P / PL::E;
    if constexpr (PL::L > 1) {
#pragma unroll
        for (int k = 0; k < num_tw<PL>(); ++k) tws[k] = sched[k * TL + tl];
    }
}

// LDS padding: one slot per 16 positions breaks the stride-R bank pattern of
// the early stages' stores
__device__ __forceinline__ int padpos(int pos) { return pos + (pos >> 4); }
template <int P> constexpr int padded_len() { return P + P / 16; }

// A stage position split as a + k: a from the thread index, k constant once
// the register slot j is (the slot loops unroll).  When a or k is a multiple
// of 16, padpos(a + k) = padpos(a) + padpos(k), so every slot's LDS address
// is one per-thread base plus an immediate offset.
struct SplitPos {
    int a, k;
    bool exact;
    __device__ operator int() const { return a + k; }
};
__device__ __forceinline__ int padpos(SplitPos p) { return p.exact ? padpos(p.a) + padpos(p.k) : padpos(p.a + p.k); }
template <int P, typename PL, int S> __device__ __forceinline__ SplitPos in_split(int tl, int j) {
    constexpr int R = PL::R[S], TL = P / PL::E;
    const int k = (j / R) * TL + (j % R) * (P / R);
    return SplitPos{tl, k, k % 16 == 0};
}
template <int P, typename PL, int S> __device__ __forceinline__ SplitPos out_split(int tl, int j) {
    constexpr int R = PL::R[S], TL = P / PL::E, Ns = stage_ns<PL>(S), NB = PL::E / R;
    const int i = j / R, r = j % R;
    if constexpr (TL % Ns == 0) {
        // b = tl + i TL: b / Ns = tl / Ns + i TL / Ns, b mod Ns = tl mod Ns
        const int k = i * TL * R + r * Ns;
        constexpr bool a16 = Ns == 1 && R % 16 == 0;  // a = tl R
        return SplitPos{(tl / Ns) * Ns * R + tl % Ns, k, a16 || k % 16 == 0};
    } else if constexpr (Ns % TL == 0 && NB * TL <= Ns) {
        // b = tl + i TL < Ns: the position is b + r Ns
        const int k = i * TL + r * Ns;
        return SplitPos{tl, k, k % 16 == 0};
    } else {
        return SplitPos{out_pos<P, PL, S>(tl, j), 0, true};
    }
}

// forward butterflies of stage S (twiddle, then DFT with exp(-2 pi i ...))
template <typename T, typename PL, int S>
__device__ __forceinline__ void fwd_bfly(C2<T> *v, const C2<T> *tws) {
    constexpr int R = PL::R[S], E = PL::E, TW = stage_tw<PL>(S);
#pragma unroll
    for (int i = 0; i < E / R; ++i) {
        if constexpr (S > 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[i * R + r] = cmul<T>(v[i * R + r], tws[TW + i * (R - 1) + r - 1]);
        }
        Dft<T, R, -1>::run(v + i * R);
    }
}
// adjoint of stage S (DFT with exp(+2 pi i ...), then conjugate twiddle): applying
// the adjoints of stages L-1..0 gives the unnormalised inverse DFT
template <typename T, typename PL, int S>
__device__ __forceinline__ void adj_bfly(C2<T> *v, const C2<T> *tws) {
    constexpr int R = PL::R[S], E = PL::E, TW = stage_tw<PL>(S);
#pragma unroll
    for (int i = 0; i < E / R; ++i) {
        Dft<T, R, +1>::run(v + i * R);
        if constexpr (S > 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[i * R + r] = cmul<T>(v[i * R + r], cconj<T>(tws[TW + i * (R - 1) + r - 1]));
        }
    }
}

// forward transform: v enters at in_pos<0>, leaves at out_pos<L-1> = natural
// positions b + r*(P/R_last)
template <typename T, int P, typename PL, int S, typename Lidx>
__device__ __forceinline__ void fwd_stages(C2<T> *v, C2<T> *lds, int tl, const C2<T> *tws, Lidx lidx) {
    fwd_bfly<T, PL, S>(v, tws);
    if constexpr (S + 1 < PL::L) {
        constexpr int E = PL::E;
#pragma unroll
        for (int j = 0; j < E; ++j) lds[lidx(out_split<P, PL, S>(tl, j))] = v[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = lds[lidx(in_split<P, PL, S + 1>(tl, j))];
        __syncthreads();
        fwd_stages<T, P, PL, S + 1>(v, lds, tl, tws, lidx);
    }
}
// inverse transform (adjoint stages L-1..0): v enters at out_pos<L-1>, leaves at in_pos<0>
template <typename T, int P, typename PL, int S, typename Lidx>
__device__ __forceinline__ void adj_stages(C2<T> *v, C2<T> *lds, int tl, const C2<T> *tws, Lidx lidx) {
    adj_bfly<T, PL, S>(v, tws);
    if constexpr (S > 0) {
        constexpr int E = PL::E;
#pragma unroll
        for (int j = 0; j < E; ++j) lds[lidx(in_split<P, PL, S>(tl, j))] = v[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = lds[lidx(out_split<P, PL, S - 1>(tl, j))];
        __syncthreads();
        adj_stages<T, P, PL, S - 1>(v, lds, tl, tws, lidx);
    }
}


}  // namespace fl

// ---------------------------------------------------------------------------
// operator object
// ---------------------------------------------------------------------------
struct fl_op_s {
    int d = 0, N = 0, n = 0, P = 0, Q = 0, Qp = 0;
    int nk[3] = {0, 0, 0};        // interior nodes per axis (x first; 1 past d); n each on the square
    int64_t M = 0;
    double alpha = 0, h = 0, c = 0, a0 = 0;
    double gamma = 2.0;           // splitting parameter of the scheme, in (alpha, 2]
    int device = 0;
    double *a = nullptr;          // (N+1)^d coefficients, a[0] = a_0
    double *lam64 = nullptr;      // Q^d eigenvalues / P^d, natural order
    double *lam64t = nullptr;     // the same, tiled for the FP64 fused pass
    float *lam32t = nullptr;      // FP32 copy, tiled for the FP32 fused pass
    int var32 = 0, var64 = 0;     // selected kernel variants (0 = default)
    double2 *tw64 = nullptr;      // exp(-2 pi i m / P), m < P
    float2 *tw32 = nullptr;
    double2 *sch64 = nullptr;     // lane-ordered twiddles of every plan (sched_len(P) entries)
    float2 *sch32 = nullptr;
    void *T1 = nullptr;           // spectra workspaces (sized for FP64)
    void *T2 = nullptr;
    size_t T1_bytes = 0, T2_bytes = 0;
    // solver workspace (allocated on first use)
    void *sw = nullptr;
    size_t sw_bytes = 0;
    double *scal = nullptr;       // device scalars of the solvers
    double *hscal = nullptr;      // pinned host mirror
    fl_unet net = nullptr;        // learned preconditioner (not owned)
    // sine-transform preconditioner of s0 I + s1 A: its symbol, tiled like lam64t
    // for FP64 variant mu_var (allocated on first use)
    double *mu64t = nullptr;
    double mu_s0 = 0.0, mu_s1 = 0.0;
    int mu_var = -1;
    // the same symbol in FP32 for FP32 variant mu32_var (the FP32 inner solves)
    float *mu32t = nullptr;
    double mu32_s0 = 0.0, mu32_s1 = 0.0;
    int mu32_var = -1;
};

namespace fl {
// epilogue of the last matvec pass: y = a1 w1 + a2 w2 + scale (A u); a null
// w1 / w2 drops its term; the default is y = A u.
template <typename T> struct Epi {
    const T *w1 = nullptr;
    T a1 = T(0);
    const T *w2 = nullptr;
    T a2 = T(0);
    T scale = T(1);
    // with dpart: each X-inverse workgroup b writes sum (dotw, y) over its rows,
    // in FP64 and a fixed order, to dpart[z * dpart_stride + b] (z = problem)
    const T *dotw = nullptr;
    double *dpart = nullptr;
    long dpart_stride = 0;
    bool active() const { return w1 != nullptr || w2 != nullptr || scale != T(1) || dpart != nullptr; }
};
// number of X-inverse workgroups of a matvec (the partial sums an epilogue
// dot writes): d, rows of the x pass (M / nk[0]), P, precision, kernel variant
int xinv_parts(int d, long rows, int P, int prec, int variant);
template <typename T>
fl_status matvec(fl_op op, const T *u, T *y, hipStream_t s);
// `done`: optional device flag; when it holds a nonzero value every pass returns at once
// ev (optional): 2 events per pass, recorded at each kernel's start and stop
template <typename T>
fl_status matvec_ex(fl_op op, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                    hipEvent_t *ev = nullptr);

// what a matvec launch needs: sizes, workspaces, twiddles, tiled lambda, and for
// a batch of same-size problems (blockIdx.z = problem) the per-problem strides
template <typename T> struct MvCtx {
    int d = 2, n = 0, P = 0, Q = 0;
    int nk[3] = {0, 0, 0};     // interior nodes per axis, x first
    void *T1 = nullptr, *T2 = nullptr;
    const C2<T> *tw = nullptr;   // exp(-2 pi i m / P)
    const C2<T> *tws = nullptr;  // lane-ordered twiddles of every plan
    const T *lam = nullptr;
    bool odd = false;          // forward loads take the odd extension (sine-transform preconditioner)
    int batch = 1;
    long zs_vec = 0;           // elements between problems' vectors
    long zs_t1 = 0, zs_t2 = 0; // bytes between problems' workspaces
    long zs_lam = 0;           // elements between problems' tiled lambda
    int zs_done = 0;           // doubles between problems' done flags
};
template <typename T> MvCtx<T> single_ctx(fl_op op);
template <typename T>
fl_status matvec_ctx(const MvCtx<T> &cx, int variant, const T *u, T *y, const Epi<T> &ep, const double *done,
                     hipStream_t s, hipEvent_t *ev = nullptr);
fl_status build_symbol(fl_op op, hipStream_t s);
// the lane-ordered twiddle tables of op's FFT length (LDS path) from tw64 / tw32
fl_status make_schedules(fl_op op, hipStream_t s);
int kernel_p_supported(int P);
fl_status unet_apply(fl_unet u, const double *r, int n, double alpha, double *z, const double *rr_dev,
                     hipStream_t s);
int unet_size(fl_unet u);
// kernel variants of a matvec: points per thread in the row / strided passes,
// spectrum tile width, line pairs per row block
// kind 0: workgroup-per-tile kernels; kind 1 (2D only): one wavefront per FFT
// line, four rows per row-pass workgroup (ex, ey: points per lane)
struct VariantDesc {
    int ex, ey, c, lpb, kind;
};
int variant_count(fl_op op, int prec);
VariantDesc variant_desc(fl_op op, int prec, int k);
VariantDesc variant_desc_pd(int P, int d, int prec, int k);
fl_status tile_lambda(fl_op op, int prec, int C, void *lt, hipStream_t s);
// spectral x-columns kept by the matvec: P/2 in 2D (DC and Nyquist packed in
// column 0), P/2 + 1 in 1D and 3D
inline int spec_cols(int d, int P) { return d == 2 ? P / 2 : P / 2 + 1; }
// elements of a tiled lambda of tile width C (2D: tiles plus one packed column)
// entries of lambda laid out for a variant of tile width C (1D: Q in natural order)
inline long lam_tiled_len(int d, int P, int C) {
    const long Q = P / 2 + 1, nt = (spec_cols(d, P) + C - 1) / C;
    return d == 1 ? Q : d == 2 ? nt * C * Q + Q : nt * C * Q * Q;
}
fl_status select_variant(fl_op op, int prec, int k, hipStream_t s);
// the variant for (op's d and FFT length, prec) from the on-disk tuning cache
// (timed and recorded on a miss), selected on op
fl_status tuned_variant(fl_op op, int prec, int *k);
// sine-transform preconditioner of s0 I + s1 A (operators whose every axis has
// at most P/2 - 1 nodes, the large 2D ones included; on power-of-two squares and cubes the tau
// matrix itself, elsewhere the inverse of the tau matrix on the embedding's
// P/2 - 1 nodes restricted to the operator's): tau_prepare builds its FP64 symbol for the selected
// FP64 variant (FL_E_BREAKDOWN when s0 + s1 lambda is not positive on a sine
// mode); tau_apply computes z = M^{-1} r in FP64 (a set `done` flag skips it)
bool tau_supported(const fl_op_s *op);
// the preconditioner's symbol tiled to width C in FP32 or FP64 into lt (lam_tiled_len entries)
fl_status tau_symbol(fl_op op, double s0, double s1, int prec, int C, void *lt, hipStream_t s);
fl_status tau_prepare(fl_op op, double s0, double s1, hipStream_t s);
fl_status tau_apply(fl_op op, const double *r, double *z, const double *done, hipStream_t s);
// FP32 counterparts for the selected FP32 variant
fl_status tau_prepare32(fl_op op, double s0, double s1, hipStream_t s);
fl_status tau_apply32(fl_op op, const float *r, float *z, const double *done, hipStream_t s);
constexpr int kMaxTile = 16;  // largest tile width of any variant
// longest FFT whose line a workgroup keeps in LDS; longer 2D embeddings (up to
// 16384) take the global-memory passes of the large-operator path
constexpr int kMaxLdsP = 2048;
inline bool large_op(const fl_op_s *op) { return op->P > kMaxLdsP; }
// large-operator path (2D): symbol and matvec with the solver epilogue and done
// flag (no fused dot partials)
fl_status large_symbol(fl_op op, hipStream_t s);
template <typename T>
fl_status large_matvec(fl_op op, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                       const T *sym = nullptr, bool odd = false);
}  // namespace fl
