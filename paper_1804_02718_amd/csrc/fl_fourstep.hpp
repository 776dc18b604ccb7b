// Large 2D operators (FFT length P = 4096 ... 16384).  Included inside
// namespace fl by fl_fft.hip, after the plan, stage and twiddle helpers.
//
// y = A u in five passes over HBM:
//   xrow  one real row per workgroup, whole in LDS: the P/2-point complex
//         transform of z[m] = x[2m] + i x[2m+1] and the split into the row's
//         half spectrum X[0..P/2], written in natural column order
//   ya    y step 1 over the Q half-spectrum columns, twiddle
//   ymid  y step 2, lambda, the inverse of y step 2 (in place)
//   yai   conjugate twiddle, inverse y step 1, the ny rows kept
//   xrowi one row per workgroup: the inverse of xrow and the solver epilogue
// A column of P values does not fit a workgroup's LDS (the y passes carry
// kFsLines adjacent columns to keep every access contiguous), so the y
// transform is split by the four-step factorisation P = P1 P2 (P1, P2 in
// {64, 128}): with n = P2 n1 + n2 and k = k1 + P1 k2,
//   X[k1 + P1 k2] = sum_n2 W_P2^(n2 k2) W_P^(n2 k1) sum_n1 x[P2 n1 + n2] W_P1^(n1 k1),
// one pass of P1-point transforms over n1 with the twiddle W_P^(n2 k1), one of
// P2-point transforms over n2, and the inverse the same steps backwards with
// conjugate twiddles; between them the spectrum stays in that transposed
// order.  A row's P/2-point transform is the same factorisation inside one
// workgroup's LDS, P/2 = M1 x 128.

// the y passes' short transforms: 16 points per thread at L = 128 (one LDS
// exchange), except in the FP64 middle pass (MID), whose registers would then
// halve its resident waves; 8 points below L = 128
template <int L, bool MID = false, typename T = float> struct FsPlan {
    static constexpr int E = L == 128 && !(MID && sizeof(T) == 8) ? 16 : 8;
    using PN = Plan<L, E>;
};
// short column transforms per workgroup of the y passes (lines); P1, P2 are multiples of it
constexpr int kFsLines = 32;
template <int L, bool MID = false, typename T = float> constexpr int fs_threads() {
    return kFsLines * (L / FsPlan<L, MID, T>::PN::E);
}
// the short transforms' twiddle tables exp(-2 pi i m / L), L = 128, 64, 32, 16, in one buffer
constexpr int fs_tw_off(int L) { return L == 128 ? 0 : L == 64 ? 128 : L == 32 ? 192 : 224; }
constexpr int kFsTwLen = 240;

// ---------------------------------------------------------------------------
// x passes: a real row of the P-periodic line (zero-padded, or for ODD its odd
// extension: e[p] = x[p] for p < nx, -x[P - 2 - p] where P - 2 - p < nx) as
// z[m] = e[2m] + i e[2m+1], m < M = P/2.  With Z = FFT_M(z), E and O the
// transforms of the even and odd samples, Z = E + i O and
//   E[k] = (Z[k] + conj Z[M - k]) / 2,  O[k] = (Z[k] - conj Z[M - k]) / (2i),
//   X[k] = E[k] + W_P^k O[k],  k = 0 .. M   (Z of period M).
// The inverse forms Z'[k] = (X[k] + conj X[M - k]) + i W_P^-k (X[k] - conj X[M - k]),
// k < M, whose unnormalised inverse M-point transform is e[2m] + i e[2m+1].
// LDS holds z as M1 lines of 128 (index m = 128 a + b at xr_addr(a, b));
// step A transforms the lines b over a (M1 points), step B the lines a over b.
// ---------------------------------------------------------------------------
template <int M1> constexpr int xr_threads() { return M1 >= 32 ? 512 : 256; }
// line stride: one more than the padded line, so consecutive lines start on
// different banks (the split reads the lines k mod M1 for consecutive k)
constexpr int kXrLS = padded_len<128>() + 1;
__device__ __forceinline__ int xr_addr(int a, int b) { return a * kXrLS + padpos(b); }

// the row kernels' twiddles, copied to LDS once per workgroup: the short
// transforms' tables exp(-2 pi i m / L) at fs_tw_off(L), then W_M^e and W_P^e
// for e < 128; a twiddle of the M- or P-point transform is the product of two
// entries, so no global load is left between a row's loads and its stores
constexpr int kXrTw = kFsTwLen + 256;
template <typename T>
__device__ __forceinline__ void xr_load_tw(C2<T> *twl, const C2<T> *__restrict__ tw, const C2<T> *__restrict__ subtw) {
    for (int i = threadIdx.x; i < kXrTw; i += blockDim.x)
        twl[i] = i < kFsTwLen ? subtw[i] : (i < kFsTwLen + 128 ? tw[2 * (i - kFsTwLen)] : tw[i - kFsTwLen - 128]);
}
// W_M^e, e < M = 128 M1: W_M1^(e / 128) W_M^(e mod 128)
template <typename T, int M1> __device__ __forceinline__ C2<T> xr_wm(const C2<T> *twl, int e) {
    return cmul<T>(twl[fs_tw_off(M1) + (e >> 7)], twl[kFsTwLen + (e & 127)]);
}
// W_P^k, k <= M = P / 2: W_(2 M1)^(k / 128) W_P^(k mod 128)
template <typename T, int M1> __device__ __forceinline__ C2<T> xr_wp(const C2<T> *twl, int k) {
    return cmul<T>(twl[fs_tw_off(2 * M1) + (k >> 7)], twl[kFsTwLen + 128 + (k & 127)]);
}

// Step A's layout of a row in registers: thread (c, tl) = (threadIdx.x mod LPA,
// threadIdx.x / LPA) holds, in slot rr * EA + j, the point m = 128 a + b of
// line b = rr * LPA + c at a = in_pos<M1, PA, 0>(tl, j) -- the inputs of its
// step-A butterflies going forward and their outputs coming back.
// At M1 = 64 (512 threads) both steps take 16 points per thread: one round of
// 128 (64) lines and one LDS exchange per step; shorter rows take 8.
template <int M1, int NTH> struct XrShape {
    using PA = Plan<M1, M1 == 64 ? 16 : 8>;
    using PB = Plan<128, M1 == 64 ? 16 : 8>;
    static constexpr int EA = PA::E, TLA = M1 / EA, LA = PA::L, EB = PB::E, TLB = 128 / EB, LB = PB::L;
    static constexpr int LPA = NTH / TLA, RA = 128 / LPA, LPB = NTH / TLB, RB = M1 / LPB;
    static constexpr int NR = RA * EA;  // register slots of a row
    static_assert(RA >= 1 && RB >= 1 && RA * LPA == 128 && RB * LPB == M1, "rounds");
    // point of slot (rr, j); only slots with j mod R0 < R0 / 2 lie below M / 2
    static __device__ __forceinline__ int point(int rr, int j) {
        const int c = threadIdx.x % LPA, tl = threadIdx.x / LPA;
        return 128 * in_pos<M1, PA, 0>(tl, j) + rr * LPA + c;
    }
    static constexpr bool low(int j) { return (j % PA::R[0]) < PA::R[0] / 2; }
};

// z of one row (zero-padded, or its odd extension, to P) into step A's
// registers, in two parts: xr_load_za issues the loads (clamped addresses, the
// raw values), xr_fix_za zeroes or negates what lies outside the stored values.
// Split so that a prefetch's loads are not waited for where they are issued.
template <typename T, int M1, int NTH, bool ODD>
__device__ __forceinline__ void xr_load_za(C2<T> *zl, const T *__restrict__ ur, int nx) {
    using S = XrShape<M1, NTH>;
    constexpr int P = 256 * M1;
#pragma unroll
    for (int rr = 0; rr < S::RA; ++rr)
#pragma unroll
        for (int j = 0; j < S::EA; ++j) {
            if (!ODD && !S::low(j)) continue;  // m >= P/4: past every stored value
            const int m = S::point(rr, j);
            T e2[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int p = 2 * m + h;
                if constexpr (!ODD) {
                    e2[h] = ur[p < nx ? p : 0];
                } else {
                    const int q = P - 2 - p;
                    e2[h] = ur[p < nx ? p : (q >= 0 && q < nx ? q : 0)];
                }
            }
            zl[rr * S::EA + j] = mk<T>(e2[0], e2[1]);
        }
}
template <typename T, int M1, int NTH, bool ODD>
__device__ __forceinline__ void xr_fix_za(C2<T> *zl, int nx) {
    using S = XrShape<M1, NTH>;
    constexpr int P = 256 * M1;
#pragma unroll
    for (int rr = 0; rr < S::RA; ++rr)
#pragma unroll
        for (int j = 0; j < S::EA; ++j) {
            C2<T> &z = zl[rr * S::EA + j];
            if (!ODD && !S::low(j)) {
                z = mk<T>(T(0), T(0));
                continue;
            }
            const int m = S::point(rr, j);
            T e2[2] = {z.x, z.y};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int p = 2 * m + h;
                if constexpr (!ODD) {
                    e2[h] = p < nx ? e2[h] : T(0);
                } else {
                    const int q = P - 2 - p;
                    e2[h] = p < nx ? e2[h] : (q >= 0 && q < nx ? -e2[h] : T(0));
                }
            }
            z = mk<T>(e2[0], e2[1]);
        }
}

// The LDS transform of both row kernels.  Forward: step A (M1-point
// transforms over a of the lines b, from the registers zr, then
// W_M^(b k1) = W_P^(2 b k1)), mid(), step B (128-point transforms over b of
// the lines k1); leaves Z[k1 + M1 k2] at xr_addr(k1, k2).  INV: the adjoint
// steps in reverse order (B', the conjugate twiddle, mid(), A') from Z' at
// xr_addr(k1, k2) to z in the registers zr.  Callers barrier before it (buf
// free, or Z' complete) and after it.
template <typename T, int M1, int NTH, bool INV, typename Mid>
__device__ __forceinline__ void xr_transform(C2<T> *buf, const C2<T> *twl, C2<T> *zr, Mid mid) {
    using S = XrShape<M1, NTH>;
    using PA = typename S::PA;
    using PB = typename S::PB;
    constexpr int M2 = 128, EA = S::EA, LA = S::LA, EB = S::EB, LB = S::LB, LPA = S::LPA, RA = S::RA;
    constexpr int LPB = S::LPB, RB = S::RB, TLB = S::TLB;
    auto step_a = [&]() {
        const int c = threadIdx.x % LPA, tl = threadIdx.x / LPA;
        C2<T> tws[num_tw<PA>()];
        load_twiddles<T, M1, PA>(tws, twl + fs_tw_off(M1), tl);
#pragma unroll
        for (int rr = 0; rr < RA; ++rr) {
            const int b = rr * LPA + c;
            C2<T> v[EA];
            auto lidx = [b](int pos) { return xr_addr(pos, b); };
            if constexpr (!INV) {
#pragma unroll
                for (int j = 0; j < EA; ++j) v[j] = zr[rr * EA + j];
                fwd_stages<T, M1, PA, 0>(v, buf, tl, tws, lidx);
#pragma unroll
                for (int j = 0; j < EA; ++j) {
                    const int k1 = out_pos<M1, PA, LA - 1>(tl, j);
                    buf[lidx(k1)] = cmul<T>(v[j], xr_wm<T, M1>(twl, b * k1));
                }
            } else {
#pragma unroll
                for (int j = 0; j < EA; ++j) v[j] = buf[lidx(out_pos<M1, PA, LA - 1>(tl, j))];
                __syncthreads();  // in registers before the line's exchanges overwrite it
                adj_stages<T, M1, PA, LA - 1>(v, buf, tl, tws, lidx);
#pragma unroll
                for (int j = 0; j < EA; ++j) zr[rr * EA + j] = v[j];
            }
        }
    };
    auto step_b = [&]() {
        const int tl = threadIdx.x % TLB, c = threadIdx.x / TLB;
        C2<T> tws[num_tw<PB>()];
        load_twiddles<T, M2, PB>(tws, twl + fs_tw_off(M2), tl);
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
            const int k1 = rr * LPB + c;
            C2<T> v[EB];
            auto lidx = [k1](auto pos) { return k1 * kXrLS + padpos(pos); };
            if constexpr (!INV) {
#pragma unroll
                for (int j = 0; j < EB; ++j) v[j] = buf[lidx(in_split<M2, PB, 0>(tl, j))];
                __syncthreads();
                fwd_stages<T, M2, PB, 0>(v, buf, tl, tws, lidx);
#pragma unroll
                for (int j = 0; j < EB; ++j) buf[lidx(out_split<M2, PB, LB - 1>(tl, j))] = v[j];
            } else {
#pragma unroll
                for (int j = 0; j < EB; ++j) v[j] = buf[lidx(out_split<M2, PB, LB - 1>(tl, j))];
                __syncthreads();
                adj_stages<T, M2, PB, LB - 1>(v, buf, tl, tws, lidx);
#pragma unroll
                for (int j = 0; j < EB; ++j) {
                    const int b = in_pos<M2, PB, 0>(tl, j);
                    buf[lidx(in_split<M2, PB, 0>(tl, j))] = cmul<T>(v[j], cconj<T>(xr_wm<T, M1>(twl, b * k1)));
                }
            }
        }
    };
    if constexpr (!INV) {
        step_a();
        mid();
        __syncthreads();
        step_b();
    } else {
        step_b();
        mid();
        __syncthreads();
        step_a();
    }
}

// PF: the forward row kernel's workgroups take rows b, b + gridDim.x, ...
// (FP64 at P = 16384, zero-padded rows: one 145 KB workgroup per CU) and the
// next row's loads are issued once step A has consumed the current row's
// registers, arriving during step B and the split; the transform reads its
// twiddles from LDS, so no other global load waits behind them.  Otherwise
// (two or more workgroups per CU overlap instead, or the odd extension's
// loads would not fit the registers) a workgroup takes one row, as the
// inverse always does (a prefetch of its spectra would not fit either).
template <typename T, int M1, bool ODD> constexpr bool xr_prefetch() { return sizeof(T) == 8 && M1 == 64 && !ODD; }

// x forward: z of the row into step A's registers, the transform, the split
// into X[0..M].  Split twiddles: for k = t + NTH i (t = threadIdx.x),
// W_P^k = W_P^t W_(P/NTH)^i.
template <typename T, int M1, bool ODD>
__global__ __launch_bounds__(xr_threads<M1>()) void k_fs_xrow(
    const T *__restrict__ u, C2<T> *__restrict__ S, int nx, int ny, int Qs, const C2<T> *__restrict__ tw,
    const C2<T> *__restrict__ subtw, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    constexpr int NTH = xr_threads<M1>(), M = M1 * 128, P = 2 * M, NR = XrShape<M1, NTH>::NR;
    constexpr int NS = (M + 1 + NTH - 1) / NTH;  // split outputs X[0..M] per thread
    constexpr bool PF = xr_prefetch<T, M1, ODD>();
    static_assert(NR * NTH == M && P / NTH <= 32, "whole rows per thread set");
    __shared__ C2<T> buf[M1 * kXrLS];
    __shared__ C2<T> twl[kXrTw];
    xr_load_tw<T>(twl, tw, subtw);
    __syncthreads();
    const C2<T> wt = xr_wp<T, M1>(twl, threadIdx.x);
    C2<T> zl[NR];
    auto body = [&](int row, auto mid) {
        xr_fix_za<T, M1, NTH, ODD>(zl, nx);
        xr_transform<T, M1, NTH, false>(buf, twl, zl, mid);
        __syncthreads();
        C2<T> *srow = S + (long)row * Qs;
#pragma unroll 1
        for (int i = 0; i < NS; ++i) {
            const int k = threadIdx.x + NTH * i;
            if (k <= M) {
                const int kk = k == M ? 0 : k, km = k == 0 ? 0 : M - k;
                const C2<T> zk = buf[xr_addr(kk % M1, kk / M1)];
                const C2<T> zm = buf[xr_addr(km % M1, km / M1)];
                const C2<T> ev = mk<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y));
                const C2<T> od = mk<T>(T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x));
                const C2<T> w = cmul<T>(wt, twl[fs_tw_off(P / NTH) + i]);
                st_stream(srow + k, cadd<T>(ev, cmul<T>(od, w)));
            }
        }
    };
    if constexpr (!PF) {
        xr_load_za<T, M1, NTH, ODD>(zl, u + (long)blockIdx.x * nx, nx);
        body(blockIdx.x, [] {});
    } else {
        int row = blockIdx.x;
        if (row < ny) xr_load_za<T, M1, NTH, ODD>(zl, u + (long)row * nx, nx);
        for (; row < ny; row += gridDim.x) {
            // keeps the LDS twiddle reads inside the loop (hoisted, they would
            // hold registers across rows)
            asm volatile("" ::: "memory");
            const int next = row + gridDim.x;
            body(row, [&] {
                if (next < ny) xr_load_za<T, M1, NTH, ODD>(zl, u + (long)next * nx, nx);
            });
            __syncthreads();  // the split's reads before the next row's transform
        }
    }
}

// x inverse: X[0..M] of the row -> Z' -> the inverse transform into step A's
// registers -> y[2m] = Re z[m], y[2m + 1] = Im z[m] below nx, with the
// epilogue (its reads issued before the last step).  A thread reads X[k] and
// X[M - k] (k < M/2) once for both of
//   Z'[k]     = (X[k] + conj X[M-k]) + i W_P^-k (X[k] - conj X[M-k]),
//   Z'[M - k] = (X[M-k] + conj X[k]) - i W_P^k (X[M-k] - conj X[k])   (k > 0),
// since W_P^-(M-k) = -W_P^k; thread 0 also takes k = M/2.
template <typename T, int M1, bool EPI>
__global__ __launch_bounds__(xr_threads<M1>()) void k_fs_xrowi(
    const C2<T> *__restrict__ S, T *__restrict__ y, int nx, int ny, int Qs, const C2<T> *__restrict__ tw,
    const C2<T> *__restrict__ subtw, Epi<T> ep, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    constexpr int NTH = xr_threads<M1>(), M = M1 * 128, P = 2 * M;
    using SH = XrShape<M1, NTH>;
    constexpr int NR = SH::NR, NP = NR / 2;
    constexpr int RA = SH::RA, EA = SH::EA;
    static_assert(NR * NTH == M && P / NTH <= 32, "whole rows per thread set");
    __shared__ C2<T> buf[M1 * kXrLS];
    __shared__ C2<T> twl[kXrTw];
    xr_load_tw<T>(twl, tw, subtw);
    const int row = blockIdx.x;
    const C2<T> *srow = S + (long)row * Qs;
    C2<T> xa[NP], xb[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int k = threadIdx.x + NTH * i;
        xa[i] = srow[k];
        xb[i] = srow[M - k];
    }
    const C2<T> xh = srow[M / 2];
    __syncthreads();  // twl complete
    const C2<T> wt = xr_wp<T, M1>(twl, threadIdx.x);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int k = threadIdx.x + NTH * i;
        const C2<T> a = xa[i], b = xb[i], w = cmul<T>(wt, twl[fs_tw_off(P / NTH) + i]);
        const C2<T> wd = cmul<T>(mk<T>(a.x - b.x, a.y + b.y), cconj<T>(w));
        buf[xr_addr(k % M1, k / M1)] = mk<T>(a.x + b.x - wd.y, a.y - b.y + wd.x);
        if (k > 0) {
            const C2<T> we = cmul<T>(mk<T>(b.x - a.x, b.y + a.y), w);
            const int km = M - k;
            buf[xr_addr(km % M1, km / M1)] = mk<T>(b.x + a.x + we.y, b.y - a.y - we.x);
        }
    }
    if (threadIdx.x == 0) {
        const C2<T> wd = cmul<T>(mk<T>(T(0), xh.y + xh.y), cconj<T>(xr_wp<T, M1>(twl, M / 2)));
        buf[xr_addr((M / 2) % M1, (M / 2) / M1)] = mk<T>(xh.x + xh.x - wd.y, wd.x);
    }
    __syncthreads();
    // epilogue reads at the thread's output positions (slots below M/2 only)
    const long r0 = (long)row * nx;
    T e1[RA][EA][2], e2[RA][EA][2];
    auto epi_loads = [&] {
        if constexpr (EPI) {
#pragma unroll
            for (int rr = 0; rr < RA; ++rr)
#pragma unroll
                for (int j = 0; j < EA; ++j) {
                    if (!SH::low(j)) continue;
                    const int m = SH::point(rr, j);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int p = 2 * m + h;
                        const bool ok = p < nx;
                        e1[rr][j][h] = ep.w1 ? ep.w1[r0 + (ok ? p : 0)] : T(0);
                        e2[rr][j][h] = ep.w2 ? ep.w2[r0 + (ok ? p : 0)] : T(0);
                    }
                }
        }
    };
    C2<T> zo[NR];
    xr_transform<T, M1, NTH, true>(buf, twl, zo, epi_loads);
    T *yr = y + r0;
#pragma unroll
    for (int rr = 0; rr < RA; ++rr)
#pragma unroll
        for (int j = 0; j < EA; ++j) {
            if (!SH::low(j)) continue;  // m >= M/2: past nx
            const int m = SH::point(rr, j);
            const C2<T> z = zo[rr * EA + j];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int p = 2 * m + h;
                if (p < nx) {
                    T v = h ? z.y : z.x;
                    if constexpr (EPI) v = v * ep.scale + ep.a1 * e1[rr][j][h] + ep.a2 * e2[rr][j][h];
                    yr[p] = v;
                }
            }
        }
}

// ya: y step 1 over the columns (a workgroup: kFsLines adjacent columns and one
// n2): rows P2 n1 + n2 of S (ny rows; ODD: the odd extensions of the columns),
// P1-point transforms over n1, times W_P^(n2 k1), to row P2 k1 + n2 of Tb
template <typename T, int P1, int P2, bool ODD>
__global__ __launch_bounds__(fs_threads<P1>()) void k_fs_ya(
    const C2<T> *__restrict__ S, C2<T> *__restrict__ Tb, int ny, int Qs, const C2<T> *__restrict__ tw,
    const C2<T> *__restrict__ subtw, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PN = typename FsPlan<P1>::PN;
    constexpr int E = PN::E, L = PN::L, NL = kFsLines, R0 = PN::R[0], P = P1 * P2;
    __shared__ C2<T> lds[NL * padded_len<P1>()];
    const int c = threadIdx.x % NL, tl = threadIdx.x / NL;
    const int col = blockIdx.x * NL + c;  // < Qs (the row stride), a multiple of kFsLines
    const int n2 = blockIdx.y;
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int p = P2 * in_pos<P1, PN, 0>(tl, j) + n2;
        if constexpr (!ODD) {
            if ((j % R0) < R0 / 2) {
                const bool ok = p < ny;
                v[j] = keep<T>(ok, S[(long)(ok ? p : 0) * Qs + col]);
            } else {
                v[j] = mk<T>(T(0), T(0));
            }
        } else {
            const int q = P - 2 - p;
            const bool lo = p < ny, hi = q >= 0 && q < ny;
            const C2<T> x = S[(long)(lo ? p : (hi ? q : 0)) * Qs + col];
            v[j] = keep<T>(lo || hi, lo ? x : mk<T>(-x.x, -x.y));
        }
    }
    C2<T> tws[num_tw<PN>()];
    load_twiddles<T, P1, PN>(tws, subtw + fs_tw_off(P1), tl);
    auto lidx = [c](auto pos) { return padpos(pos) * NL + c; };
    fwd_stages<T, P1, PN, 0>(v, lds, tl, tws, lidx);
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int k1 = out_pos<P1, PN, L - 1>(tl, j);
        st_stream(Tb + (long)(P2 * k1 + n2) * Qs + col, cmul<T>(v[j], tw[n2 * k1]));
    }
}

// ymid: for one k1 and kFsLines adjacent columns, y step 2 over rows
// P2 k1 + n2 (P2-point), lambda at ky = k1 + P1 k2 (row fold(ky) of lam,
// natural columns, row stride Q), and the inverse of y step 2, in place
template <typename T, int P1, int P2>
__global__ __launch_bounds__((fs_threads<P2, true, T>())) void k_fs_ymid(
    C2<T> *__restrict__ Tb, int Q, int Qs, const T *__restrict__ lam, const C2<T> *__restrict__ subtw,
    const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PN = typename FsPlan<P2, true, T>::PN;
    constexpr int E = PN::E, L = PN::L, NL = kFsLines, P = P1 * P2;
    __shared__ C2<T> lds[NL * padded_len<P2>()];
    const int c = threadIdx.x % NL, tl = threadIdx.x / NL;
    const int col = blockIdx.x * NL + c;
    // k1 in the order 0, P1/2, 1, P1 - 1, 2, P1 - 2, ...: k1 and P1 - k1 read the
    // same rows of lambda, and launched one after the other the second finds
    // them in the last-level cache
    const int q = blockIdx.y, qj = q >> 1;
    const int k1 = q == 0 ? 0 : (q == 1 ? P1 / 2 : ((q & 1) ? P1 - qj : qj));
    C2<T> *base = Tb + (long)P2 * k1 * Qs + col;
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = base[(long)in_pos<P2, PN, 0>(tl, j) * Qs];
    C2<T> tws[num_tw<PN>()];
    load_twiddles<T, P2, PN>(tws, subtw + fs_tw_off(P2), tl);
    // lambda with the data: the padding columns past Q read column Q - 1
    T lv[E];
    const T *lc = lam + (col < Q ? col : Q - 1);
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int ky = k1 + P1 * out_pos<P2, PN, L - 1>(tl, j);
        lv[j] = lc[(long)(ky <= P / 2 ? ky : P - ky) * Q];
    }
    auto lidx = [c](auto pos) { return padpos(pos) * NL + c; };
    fwd_stages<T, P2, PN, 0>(v, lds, tl, tws, lidx);
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = cscale<T>(v[j], lv[j]);
    adj_stages<T, P2, PN, L - 1>(v, lds, tl, tws, lidx);
#pragma unroll
    for (int j = 0; j < E; ++j) st_stream(base + (long)in_pos<P2, PN, 0>(tl, j) * Qs, v[j]);
}

// yai: rows P2 k1 + n2 of Tb times W_P^(-n2 k1), inverse P1-point transforms
// over k1, rows P2 n1 + n2 < ny to S
template <typename T, int P1, int P2>
__global__ __launch_bounds__(fs_threads<P1>()) void k_fs_yai(
    const C2<T> *__restrict__ Tb, C2<T> *__restrict__ S, int ny, int Qs, const C2<T> *__restrict__ tw,
    const C2<T> *__restrict__ subtw, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PN = typename FsPlan<P1>::PN;
    constexpr int E = PN::E, L = PN::L, NL = kFsLines, R0 = PN::R[0];
    __shared__ C2<T> lds[NL * padded_len<P1>()];
    const int c = threadIdx.x % NL, tl = threadIdx.x / NL;
    const int col = blockIdx.x * NL + c;
    const int n2 = blockIdx.y;
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int k1 = out_pos<P1, PN, L - 1>(tl, j);
        v[j] = cmul<T>(Tb[(long)(P2 * k1 + n2) * Qs + col], cconj<T>(tw[n2 * k1]));
    }
    C2<T> tws[num_tw<PN>()];
    load_twiddles<T, P1, PN>(tws, subtw + fs_tw_off(P1), tl);
    auto lidx = [c](auto pos) { return padpos(pos) * NL + c; };
    adj_stages<T, P1, PN, L - 1>(v, lds, tl, tws, lidx);
#pragma unroll
    for (int j = 0; j < E; ++j) {
        if ((j % R0) < R0 / 2) {  // n1 >= P1/2 lies past every kept row
            const int p = P2 * in_pos<P1, PN, 0>(tl, j) + n2;
            if (p < ny) st_stream(S + (long)p * Qs + col, v[j]);
        }
    }
}

// lambda (or the preconditioner's symbol) of a large operator in natural order,
// Q x Q (kx fastest), as the y passes read it
template <typename T>
__global__ void k_large_symbol(const double *__restrict__ lam64, T *__restrict__ out, int Q, SymMap m) {
    const long total = (long)Q * Q;
    const int N2 = Q - 1;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x)
        out[idx] = (T)sym_at(lam64, idx, (int)(idx % Q), (int)(idx / Q), 0, 2, N2, m);
}

inline void fs_split(int P, int &P1, int &P2) {
    P2 = P >= 8192 ? 128 : 64;
    P1 = P / P2;
}

// workgroups of a persistent launch over `items`: as many as the device keeps
// resident (from the occupancy calculator, cached per device), at most items
template <auto K> static int fs_grid(int threads, int items) {
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cache[dev] == 0) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, K, threads, 0) != hipSuccess || cus * per <= 0)
            return items;  // one workgroup per item: correct at any grid
        cache[dev] = cus * per;
    }
    return cache[dev] < items ? cache[dev] : items;
}

template <typename T, int P1, int P2>
static fl_status fs_matvec(fl_op op, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                           const T *lam, bool odd, const C2<T> *tw, const C2<T> *subtw) {
    const int Q = op->Q, Qs = op->Qp, nx = op->nk[0], ny = op->nk[1];
    constexpr int P = P1 * P2, M1 = P / 256;
    static_assert(P1 % kFsLines == 0 && P2 % kFsLines == 0, "whole workgroups of lines");
    if (Qs % kFsLines != 0 || Qs < Q) {  // the row stride covers whole column groups (set at creation)
        set_error("row stride %d of the large-operator spectra is not a multiple of %d", Qs, kFsLines);
        return FL_E_UNSUPPORTED;
    }
    C2<T> *Tb = (C2<T> *)op->T1;  // P x Qs: the y passes' transposed-order spectra
    C2<T> *S = (C2<T> *)op->T2;   // ny x Qs: the rows' half spectra
    const dim3 b1(fs_threads<P1>()), b2(fs_threads<P2, true, T>()), bx(xr_threads<M1>());
    // row kernels with prefetch: as many workgroups as stay resident, each
    // looping over rows; without it one row per workgroup
    if (odd) {
        const int g = xr_prefetch<T, M1, true>() ? fs_grid<k_fs_xrow<T, M1, true>>(xr_threads<M1>(), ny) : ny;
        hipLaunchKernelGGL((k_fs_xrow<T, M1, true>), dim3(g), bx, 0, s, u, S, nx, ny, Qs, tw, subtw, done);
    } else {
        const int g = xr_prefetch<T, M1, false>() ? fs_grid<k_fs_xrow<T, M1, false>>(xr_threads<M1>(), ny) : ny;
        hipLaunchKernelGGL((k_fs_xrow<T, M1, false>), dim3(g), bx, 0, s, u, S, nx, ny, Qs, tw, subtw, done);
    }
    if (odd)
        hipLaunchKernelGGL((k_fs_ya<T, P1, P2, true>), dim3(Qs / kFsLines, P2), b1, 0, s, S, Tb, ny, Qs, tw, subtw,
                           done);
    else
        hipLaunchKernelGGL((k_fs_ya<T, P1, P2, false>), dim3(Qs / kFsLines, P2), b1, 0, s, S, Tb, ny, Qs, tw, subtw,
                           done);
    hipLaunchKernelGGL((k_fs_ymid<T, P1, P2>), dim3(Qs / kFsLines, P1), b2, 0, s, Tb, Q, Qs, lam, subtw, done);
    hipLaunchKernelGGL((k_fs_yai<T, P1, P2>), dim3(Qs / kFsLines, P2), b1, 0, s, Tb, S, ny, Qs, tw, subtw, done);
    if (ep.active())
        hipLaunchKernelGGL((k_fs_xrowi<T, M1, true>), dim3(ny), bx, 0, s, S, y, nx, ny, Qs, tw, subtw, ep, done);
    else
        hipLaunchKernelGGL((k_fs_xrowi<T, M1, false>), dim3(ny), bx, 0, s, S, y, nx, ny, Qs, tw, subtw, ep, done);
    return FL_OK;
}
