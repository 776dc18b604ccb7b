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
template <typename T> __device__ __forceinline__ C2<T> cconj(C2<T> a) { return mk<T>(a.x, -a.y); }
// multiply by s*i, s = +1 or -1 (exact)
template <typename T, int S> __device__ __forceinline__ C2<T> cmuli(C2<T> a) {
    return S > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// cos / sin of 2 pi k / 16, k = 0..4 (the 16th roots the butterflies need)
constexpr double kCos16[5] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                                         0.38268343236508977173, 0.0};

// w = exp(DIR * 2 pi i k / R) as an exact constant, k < R <= 16
template <typename T, int R, int DIR, int K>
__device__ __forceinline__ C2<T> root() {
    constexpr int m = (K * 16 / R) & 15;  // in 16ths of a turn
    // cos(2 pi m/16), sin(2 pi m/16) from the first-quadrant table
    constexpr int q = m / 4, r = m % 4;
    constexpr double c0 = kCos16[r], s0 = kCos16[4 - r];
    constexpr double c = q == 0 ? c0 : q == 1 ? -s0 : q == 2 ? -c0 : s0;
    constexpr double s = q == 0 ? s0 : q == 1 ? c0 : q == 2 ? -s0 : -c0;
    return mk<T>((T)c, (T)(DIR * s));
}

// v * exp(DIR 2 pi i K / R) with the trivial rotations done exactly
template <typename T, int R, int DIR, int K>
__device__ __forceinline__ C2<T> rot(C2<T> v) {
    constexpr int m = (K * 16 / R) & 15;
    if constexpr (m == 0) return v;
    else if constexpr (m == 4) return cmuli<T, DIR>(v);
    else if constexpr (m == 8) return mk<T>(-v.x, -v.y);
    else if constexpr (m == 12) return cmuli<T, -DIR>(v);
    else return cmul<T>(v, root<T, R, DIR, K>());
}

// ---------------------------------------------------------------------------
// in-register DFT of length R (R = 1, 2, 4, 8, 16), natural order in and out:
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
// FFT plans: radix sequence per power-of-two length P.  E = registers (points)
// per thread, TL = P / E threads per line.  Every radix divides E.
// ---------------------------------------------------------------------------
template <int... Rs> struct Radices {};

template <int P> struct Plan;
template <> struct Plan<8>    { static constexpr int E = 8;  using Fwd = Radices<8>;          using Inv = Radices<8>; };
template <> struct Plan<16>   { static constexpr int E = 16; using Fwd = Radices<16>;         using Inv = Radices<16>; };
template <> struct Plan<32>   { static constexpr int E = 8;  using Fwd = Radices<8, 4>;       using Inv = Radices<4, 8>; };
template <> struct Plan<64>   { static constexpr int E = 8;  using Fwd = Radices<8, 8>;       using Inv = Radices<8, 8>; };
template <> struct Plan<128>  { static constexpr int E = 16; using Fwd = Radices<16, 8>;      using Inv = Radices<8, 16>; };
template <> struct Plan<256>  { static constexpr int E = 16; using Fwd = Radices<16, 16>;     using Inv = Radices<16, 16>; };
template <> struct Plan<512>  { static constexpr int E = 16; using Fwd = Radices<16, 8, 4>;   using Inv = Radices<4, 8, 16>; };
template <> struct Plan<1024> { static constexpr int E = 16; using Fwd = Radices<16, 16, 4>;  using Inv = Radices<4, 16, 16>; };
template <> struct Plan<2048> { static constexpr int E = 16; using Fwd = Radices<16, 16, 8>;  using Inv = Radices<8, 16, 16>; };

template <int First, int... Rest> struct FirstOf { static constexpr int value = First; };
template <typename L> struct Front;
template <int... Rs> struct Front<Radices<Rs...>> { static constexpr int value = FirstOf<Rs...>::value; };
template <typename L> struct Back;
template <int R> struct Back<Radices<R>> { static constexpr int value = R; };
template <int R, int R2, int... Rs> struct Back<Radices<R, R2, Rs...>> { static constexpr int value = Back<Radices<R2, Rs...>>::value; };

// ---------------------------------------------------------------------------
// Stockham stages over one line of P points held E per thread.
// Before a radix-R stage, thread tl holds v[i*R + r] = x[b + r*(P/R)],
// b = tl + i*TL, i < E/R.  After the butterfly the value belongs at position
// (b/Ns)*Ns*R + b%Ns + r*Ns.  Exchanges go through LDS with the index
// functor Lidx(pos).
// ---------------------------------------------------------------------------
template <typename T, int P, int E, int DIR, int Ns, int R>
__device__ __forceinline__ void butterflies(C2<T> *v, int tl, const C2<T> *__restrict__ tw) {
    constexpr int TL = P / E;
#pragma unroll
    for (int i = 0; i < E / R; ++i) {
        const int b = tl + i * TL;
        if constexpr (Ns > 1) {
            const int k = b % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C2<T> w = tw[k * r * (P / (Ns * R))];
                if (DIR > 0) w.y = -w.y;
                v[i * R + r] = cmul<T>(v[i * R + r], w);
            }
        }
        Dft<T, R, DIR>::run(v + i * R);
    }
}

template <typename T, int P, int E, int Ns, int R, typename Lidx>
__device__ __forceinline__ void stage_store(const C2<T> *v, C2<T> *lds, int tl, Lidx lidx) {
    constexpr int TL = P / E;
#pragma unroll
    for (int i = 0; i < E / R; ++i) {
        const int b = tl + i * TL;
        const int base = (b / Ns) * Ns * R + (b % Ns);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lidx(base + r * Ns)] = v[i * R + r];
    }
}

template <typename T, int P, int E, int R, typename Lidx>
__device__ __forceinline__ void stage_load(C2<T> *v, const C2<T> *lds, int tl, Lidx lidx) {
    constexpr int TL = P / E;
#pragma unroll
    for (int i = 0; i < E / R; ++i) {
        const int b = tl + i * TL;
#pragma unroll
        for (int r = 0; r < R; ++r) v[i * R + r] = lds[lidx(b + r * (P / R))];
    }
}

// position of register slot j (= i*R + r) for a layout "ready for radix R"
template <int P, int E, int R>
__device__ __forceinline__ int slot_pos(int tl, int j) {
    constexpr int TL = P / E;
    return tl + (j / R) * TL + (j % R) * (P / R);
}

template <typename T, int P, int E, int DIR, int Ns, typename L> struct Stages;
template <typename T, int P, int E, int DIR, int Ns, int R, int... Rest>
struct Stages<T, P, E, DIR, Ns, Radices<R, Rest...>> {
    template <typename Lidx>
    __device__ __forceinline__ static void run(C2<T> *v, C2<T> *lds, int tl, const C2<T> *tw, Lidx lidx) {
        butterflies<T, P, E, DIR, Ns, R>(v, tl, tw);
        if constexpr (sizeof...(Rest) > 0) {
            constexpr int R2 = FirstOf<Rest...>::value;
            stage_store<T, P, E, Ns, R>(v, lds, tl, lidx);
            __syncthreads();
            stage_load<T, P, E, R2>(v, lds, tl, lidx);
            __syncthreads();
            Stages<T, P, E, DIR, Ns * R, Radices<Rest...>>::run(v, lds, tl, tw, lidx);
        }
    }
};

}  // namespace fl

// ---------------------------------------------------------------------------
// operator object
// ---------------------------------------------------------------------------
struct fl_op_s {
    int d = 0, N = 0, n = 0, P = 0, Q = 0, Qp = 0;
    int64_t M = 0;
    double alpha = 0, h = 0, c = 0, a0 = 0;
    int device = 0;
    double *a = nullptr;          // (N+1)^d coefficients, a[0] = a_0
    double *lam64 = nullptr;      // Q^d eigenvalues / P^d
    float *lam32 = nullptr;
    double2 *tw64 = nullptr;      // exp(-2 pi i m / P), m < P
    float2 *tw32 = nullptr;
    void *T1 = nullptr;           // spectra workspaces (sized for FP64)
    void *T2 = nullptr;
    size_t T1_bytes = 0, T2_bytes = 0;
    // solver workspace (allocated on first use)
    void *sw = nullptr;
    size_t sw_bytes = 0;
    double *scal = nullptr;       // device scalars of the solvers
    double *hscal = nullptr;      // pinned host mirror
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
    bool active() const { return w1 != nullptr || w2 != nullptr || scale != T(1); }
};
template <typename T>
fl_status matvec(fl_op op, const T *u, T *y, hipStream_t s);
// `done`: optional device flag; when it holds a nonzero value every pass returns at once
template <typename T>
fl_status matvec_ex(fl_op op, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                    hipEvent_t *ev = nullptr);
fl_status build_symbol(fl_op op, hipStream_t s);
int kernel_p_supported(int P);
}  // namespace fl
