// fl_fft.hip -- FFT matvec of the multilevel Toeplitz stiffness matrix.
//
// The matrix of the scheme (Sec. 2 block Toeplitz form, Sec. 4 three-level
// form) is A_ij = -c a_{|i-j|}.  Its generator is embedded in a circulant of
// length P (a power of two >= 2n-1) per axis; the circulant's eigenvalues
// lambda are the FFT of the embedded generator (real, even in every axis).
// y = A u is then: zero-pad u to P^d, FFT, multiply by lambda, inverse FFT,
// keep the first n points per axis.
//
// Passes (x fastest; kx the half-spectrum index 0..Q-1, Q = P/2+1):
//   1D: one fused pass (fwd, x lambda, inv, crop) per pair of vectors
//   2D: X-fwd (real rows -> half spectra) | Y fused (fwd, x lambda, inv, crop) | X-inv
//   3D: X-fwd | Y-fwd | Z fused | Y-inv | X-inv
// Half spectra are stored in tiles of C consecutive kx: element (slab k,
// tile t, line position j, column c) sits at ((k*ntiles + t)*nj + j)*C + c, so a
// strided pass reads each tile as one contiguous block and a row pass writes
// runs of C values for each of its rows.  Row passes pack two real rows into
// one complex line.  The inverse transforms are the adjoints of the forward
// stages in reverse order, so every pass loads its twiddles once.
#include <hip/hip_ext.h>

#include "fl_internal.hpp"

namespace fl {

template <int P> __device__ __forceinline__ int fold(int k) { return k <= P / 2 ? k : P - k; }

// default launch shape of each (precision, length, dimension); the autotuner
// can replace it by one of the variants listed further down
template <typename T, int P, int D> struct Shape {
    static constexpr int E = P >= 128 ? 16 : (P >= 16 ? 8 : P);
    static constexpr int TL = P / E;
    static constexpr int SZ = (int)sizeof(C2<T>);
    // tile width: columns per strided workgroup
    static constexpr int C32 = D == 3 ? (P >= 1024 ? 8 : 16) : (P >= 1024 ? 4 : (P >= 256 ? 8 : 16));
    static constexpr int C = sizeof(T) == 8 ? (C32 / 2 < 2 ? 2 : C32 / 2) : C32;
    // row passes: line pairs per block (>= 128-byte runs per tile, ~256 threads)
    static constexpr int lp_bytes = (128 + 2 * C * SZ - 1) / (2 * C * SZ);
    static constexpr int lp_thr = TL >= 256 ? 1 : 256 / TL;
    static constexpr int lp_max = TL >= 512 ? 1 : 512 / TL;
    static constexpr int LPB0 = lp_bytes > lp_thr ? lp_bytes : lp_thr;
    static constexpr int LPB = LPB0 > lp_max ? lp_max : LPB0;
};

// per-problem offsets of a batched launch (blockIdx.z = problem): input and
// output elements, lambda entries, and done-flag slots
struct BatchStrides {
    long in = 0, out = 0, lam = 0;
    int done = 0;
};

// tiled layout: row r of slab k = r / nj, line j = r mod nj, column kx = t*C + c
// at ((k*ntiles + t)*nj + j)*C + c = rowbase(r) + t*(nj*C) + c (element offsets
// stay below 2^31 for every supported size)
// Workgroups are dispatched to the 8 XCDs round-robin (hardware id h runs on
// XCD h mod 8), and each XCD has its own L2.  The row passes map h to a
// logical block so that every XCD takes one contiguous run of row groups:
// neighbouring rows of the tiled spectra share cache lines, which are then
// fetched and written once per line instead of once per XCD.
__device__ __forceinline__ int xcd_block(int h, int G) {
    const int base = G >> 3, r = G & 7, x = h & 7;
    return x * base + (x < r ? x : r) + (h >> 3);
}

__device__ __forceinline__ int tiled_rowbase(int r, int nj, int ntiles, int C) {
    const int k = r / nj, j = r - k * nj;
    return (k * ntiles * nj + j) * C;
}

// ---------------------------------------------------------------------------
// row pass, forward: pairs of real rows (n_in values each, zero-padded to P)
// -> Q half-spectrum values per row, written tiled.  With PACK the real DC and
// Nyquist values of a row share column 0 as (X_0, X_{P/2}), leaving P/2
// columns (the 2D path: P/2 columns fill whole tiles).
// ---------------------------------------------------------------------------
template <typename T, int P, int E, int C, int LPB, bool PACK>
__global__ __launch_bounds__(LPB * (P / E)) void k_xfwd(
    const T *__restrict__ u, C2<T> *__restrict__ out, int nrows, int n_in, long in_pitch, int nj, int ntiles,
    const C2<T> *__restrict__ table, const double *__restrict__ done, BatchStrides bz) {
    const int z = blockIdx.z;  // problem of a batch
    if (done && done[z * bz.done] != 0.0) return;
    u += z * bz.in;
    out += z * bz.out;
    using PN = Plan<P, E>;
    constexpr int TL = P / E, L = PN::L;
    constexpr int PL = padded_len<P>();
    __shared__ C2<T> lds[LPB * PL];
    const int tl = threadIdx.x % TL;
    const int lp = threadIdx.x / TL;
    const int bx = xcd_block(blockIdx.x, gridDim.x);
    const int ra = 2 * (bx * LPB + lp), rb = ra + 1;
    const bool va = ra < nrows, vb = rb < nrows;
    // twiddles first: the waits for the data below (each value is masked as
    // it arrives) then cover their latency too
    C2<T> tws[num_tw<PN>()];
    load_twiddles_lanes<T, P, PN>(tws, table, tl);
    C2<T> v[E];
    // loads from clamped, always valid addresses; rows past nrows read as 0
    const T *ua = u + (long)(va ? ra : 0) * in_pitch, *ub = u + (long)(vb ? rb : 0) * in_pitch;
    load_line<T, P, PN>(v, tl, n_in, [&](int i) {
        const T xa = ua[i], xb = ub[i];
        return mk<T>(va ? xa : T(0), vb ? xb : T(0));
    });
    const int base = lp * PL;
    auto lidx = [base](auto pos) { return base + padpos(pos); };
    fwd_stages<T, P, PN, 0>(v, lds, tl, tws, lidx);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) lds[lidx(out_split<P, PN, L - 1>(tl, j))] = v[j];
    __syncthreads();
    // Hermitian split, written tile by tile: consecutive threads cover the
    // block's rows of one tile, which are contiguous in the tiled layout
    constexpr int RW = 2 * LPB, NTH = LPB * TL;
    const int r0 = 2 * bx * LPB;
    const int tstride = nj * C;
    if constexpr (NTH % (C * RW) == 0) {
        // a thread keeps one (row, column) and walks the tiles
        const int c = threadIdx.x % C, rr = (threadIdx.x / C) % RW;
        const int row = r0 + rr;
        if (row >= nrows) return;
        const int pb = (rr >> 1) * PL;
        C2<T> *orow = out + tiled_rowbase(row, nj, ntiles, C) + c;
        // tile count and walk are compile-time: the loop unrolls to constant offsets
        constexpr int NT = ((PACK ? P / 2 : P / 2 + 1) + C - 1) / C, ST = NTH / (C * RW);
        const int t0 = threadIdx.x / (C * RW);
#pragma unroll
        for (int it = 0; it < (NT + ST - 1) / ST; ++it) {
            const int t = t0 + it * ST;
            const int kx = t * C + c;
            if (t >= NT || kx > P / 2 || (PACK && kx == P / 2)) continue;
            const C2<T> zk = lds[pb + padpos(kx)];
            const C2<T> zm = lds[pb + padpos((P - kx) & (P - 1))];
            if (PACK && kx == 0) {
                // X_0 and X_{P/2} of a real row are real: (Re or Im of Z_0, of Z_{P/2})
                const C2<T> zn = lds[pb + padpos(P / 2)];
                st_stream(orow, (rr & 1) ? mk<T>(zk.y, zn.y) : mk<T>(zk.x, zn.x));
                continue;
            }
            st_stream(orow + t * tstride, (rr & 1) ? mk<T>(T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x))
                                                   : mk<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)));
        }
    } else {
        for (int idx = threadIdx.x; idx < ntiles * RW * C; idx += NTH) {
            const int c = idx % C, rr = (idx / C) % RW, t = idx / (C * RW);
            const int kx = t * C + c, row = r0 + rr;
            if (kx > P / 2 || (PACK && kx == P / 2) || row >= nrows) continue;
            const int pb = (rr >> 1) * PL;
            const C2<T> zk = lds[pb + padpos(kx)];
            const C2<T> zm = lds[pb + padpos((P - kx) & (P - 1))];
            C2<T> o = (rr & 1) ? mk<T>(T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x))
                               : mk<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y));
            if (PACK && kx == 0) {
                const C2<T> zn = lds[pb + padpos(P / 2)];
                o = (rr & 1) ? mk<T>(zk.y, zn.y) : mk<T>(zk.x, zn.x);
            }
            st_stream(out + tiled_rowbase(row, nj, ntiles, C) + t * tstride + c, o);
        }
    }
}

// ---------------------------------------------------------------------------
// row pass, inverse: Q half-spectrum values of two rows -> P real values each,
// first n_out kept.  With EPI, y = a1 w1 + a2 w2 + scale (A u), w1 / w2 read
// at the same position when non-null (shifted operators and residuals of the
// solvers).  A non-null `done` flag that is set makes the kernel a no-op.
// PACK: column 0 holds (X_0, X_{P/2}) as written by k_xfwd<PACK>.
// ---------------------------------------------------------------------------
template <typename T, int P, int E, int C, int LPB, bool EPI, bool PACK>
__global__ __launch_bounds__(LPB * (P / E)) void k_xinv(
    const C2<T> *__restrict__ in, T *__restrict__ y, int nrows, int n_out, long out_pitch, int nj, int ntiles,
    const C2<T> *__restrict__ table, Epi<T> ep, const double *__restrict__ done, BatchStrides bz) {
    const int z = blockIdx.z;
    if (done && done[z * bz.done] != 0.0) return;
    in += z * bz.in;
    y += z * bz.out;
    if (ep.w1) ep.w1 += z * bz.out;
    if (ep.w2) ep.w2 += z * bz.out;
    if (ep.dotw) ep.dotw += z * bz.out;
    using PN = Plan<P, E>;
    constexpr int TL = P / E, L = PN::L;
    constexpr int PL = padded_len<P>();
    constexpr int Q = P / 2 + 1;
    constexpr int LL = PL > 2 * Q ? PL : 2 * Q;  // LDS per line pair
    __shared__ C2<T> lds[LPB * LL];
    const int tl = threadIdx.x % TL;
    const int lp = threadIdx.x / TL;
    const int bx = xcd_block(blockIdx.x, gridDim.x);
    const int ra = 2 * (bx * LPB + lp), rb = ra + 1;
    const bool va = ra < nrows, vb = rb < nrows;
    C2<T> tws[num_tw<PN>()];
    load_twiddles_lanes<T, P, PN>(tws, table, tl);
    // the block's rows, tile by tile (contiguous runs), into LDS: row pair p,
    // member w at p*LL + w*Q + kx
    constexpr int RW = 2 * LPB, NTH = LPB * TL;
    {
        const int r0 = 2 * bx * LPB;
        const int tstride = nj * C;
        if constexpr (NTH % (C * RW) == 0) {
            const int c = threadIdx.x % C, rr = (threadIdx.x / C) % RW;
            const int row = r0 + rr;
            const bool rv = row < nrows;
            const C2<T> *irow = in + tiled_rowbase(rv ? row : 0, nj, ntiles, C) + c;
            C2<T> *lrow = lds + (rr >> 1) * LL + (rr & 1) * Q;
            constexpr int NT = ((PACK ? P / 2 : P / 2 + 1) + C - 1) / C, ST = NTH / (C * RW);
            const int t0 = threadIdx.x / (C * RW);
            // every load issued (clamped addresses) before the first is used
            constexpr int NIT = (NT + ST - 1) / ST;
            C2<T> xs[NIT];
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int t = t0 + it * ST;
                const bool ok = t < NT && t * C + c < (PACK ? P / 2 : Q);
                xs[it] = irow[(ok ? t : 0) * tstride];
            }
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int t = t0 + it * ST;
                const int kx = t * C + c;
                if (t >= NT || kx >= (PACK ? P / 2 : Q)) continue;
                const C2<T> x = keep<T>(rv, xs[it]);
                if (PACK && kx == 0) {
                    lrow[0] = mk<T>(x.x, 0);
                    lrow[P / 2] = mk<T>(x.y, 0);
                } else {
                    lrow[kx] = x;
                }
            }
        } else {
            for (int idx = threadIdx.x; idx < ntiles * RW * C; idx += NTH) {
                const int c = idx % C, rr = (idx / C) % RW, t = idx / (C * RW);
                const int kx = t * C + c, row = r0 + rr;
                if (kx >= (PACK ? P / 2 : Q)) continue;
                const bool rv = row < nrows;
                const C2<T> x = keep<T>(rv, in[tiled_rowbase(rv ? row : 0, nj, ntiles, C) + t * tstride + c]);
                C2<T> *lrow = lds + (rr >> 1) * LL + (rr & 1) * Q;
                if (PACK && kx == 0) {
                    lrow[0] = mk<T>(x.x, 0);
                    lrow[P / 2] = mk<T>(x.y, 0);
                } else {
                    lrow[kx] = x;
                }
            }
        }
    }
    __syncthreads();
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int pos = out_pos<P, PN, L - 1>(tl, j);
        const int kk = fold<P>(pos);
        C2<T> xa = lds[lp * LL + kk];
        C2<T> xb = lds[lp * LL + Q + kk];
        if (pos > P / 2) { xa.y = -xa.y; xb.y = -xb.y; }
        if (pos == 0 || pos == P / 2) { xa.y = T(0); xb.y = T(0); }
        v[j] = mk<T>(xa.x - xb.y, xa.y + xb.x);
    }
    __syncthreads();
    const int base = lp * LL;
    auto lidx = [base](auto pos) { return base + padpos(pos); };
    adj_stages<T, P, PN, L - 1>(v, lds, tl, tws, lidx);
    double acc = 0.0;  // epilogue dot (dotw, y) over this thread's outputs
    if (va) {
        T *ya = y + (long)ra * out_pitch, *yb = y + (long)rb * out_pitch;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = in_pos<P, PN, 0>(tl, j);
            if (pos < n_out) {
                T a = v[j].x, b = v[j].y;
                if constexpr (EPI) {
                    const long ia2 = (long)ra * out_pitch + pos, ib2 = (long)rb * out_pitch + pos;
                    a = ep.scale * a;
                    if (ep.w1) a += ep.a1 * ep.w1[ia2];
                    if (ep.w2) a += ep.a2 * ep.w2[ia2];
                    if (vb) {
                        b = ep.scale * b;
                        if (ep.w1) b += ep.a1 * ep.w1[ib2];
                        if (ep.w2) b += ep.a2 * ep.w2[ib2];
                    }
                    if (ep.dpart) {
                        acc += (double)a * (double)ep.dotw[ia2];
                        if (vb) acc += (double)b * (double)ep.dotw[ib2];
                    }
                }
                st_stream(ya + pos, a);
                if (vb) st_stream(yb + pos, b);
            }
        }
    }
    if constexpr (EPI) {
        if (ep.dpart) {  // block-uniform
            __shared__ double wsum[(LPB * (P / E) + 63) / 64];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
            if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int w = 0; w < (NTH + 63) / 64; ++w) t += wsum[w];
                ep.dpart[z * ep.dpart_stride + bx] = t;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// d = 1: the whole matvec in one pass.  Two real vectors share one complex
// line z = a + i b; lambda is real and even, so the inverse transform of
// lambda * FFT(z) is (A a) + i (A b): forward transform, multiply, inverse and
// crop, all in LDS.  Rows are the vectors of a batch along blockIdx.x (one
// vector per problem along blockIdx.z for a batch of operators).  Epilogue as
// in k_xinv: y = a1 w1 + a2 w2 + scale (A u), and the workgroup's (dotw, y).
// ---------------------------------------------------------------------------
template <typename T, int P, int E, int LPB, bool EPI>
__global__ __launch_bounds__(LPB * (P / E)) void k_conv1d(
    const T *__restrict__ u, T *__restrict__ y, int nrows, int n, int n_in, const T *__restrict__ lam,
    const C2<T> *__restrict__ table, Epi<T> ep, const double *__restrict__ done, BatchStrides bz) {
    const int z = blockIdx.z;
    if (done && done[z * bz.done] != 0.0) return;
    u += z * bz.in;
    y += z * bz.out;
    lam += z * bz.lam;
    if (ep.w1) ep.w1 += z * bz.out;
    if (ep.w2) ep.w2 += z * bz.out;
    if (ep.dotw) ep.dotw += z * bz.out;
    using PN = Plan<P, E>;
    constexpr int TL = P / E, L = PN::L;
    constexpr int PL = padded_len<P>();
    __shared__ C2<T> lds[LPB * PL];
    const int tl = threadIdx.x % TL;
    const int lp = threadIdx.x / TL;
    const int bx = blockIdx.x;
    const int ra = 2 * (bx * LPB + lp), rb = ra + 1;
    const bool va = ra < nrows, vb = rb < nrows;
    // twiddles and lambda first: the waits for the data below (each value is
    // masked as it arrives) then cover their latency too
    C2<T> tws[num_tw<PN>()];
    load_twiddles_lanes<T, P, PN>(tws, table, tl);
    T lv[E];
#pragma unroll
    for (int j = 0; j < E; ++j) lv[j] = lam[fold<P>(out_pos<P, PN, L - 1>(tl, j))];
    C2<T> v[E];
    // loads from clamped, always valid addresses; out-of-range values replaced by 0
    const T *ua = u + (long)(va ? ra : 0) * n, *ub = u + (long)(vb ? rb : 0) * n;
    load_line<T, P, PN>(v, tl, n_in, [&](int i) {
        const T xa = ua[i], xb = ub[i];
        return mk<T>(va ? xa : T(0), vb ? xb : T(0));
    });
    const int base = lp * PL;
    auto lidx = [base](auto pos) { return base + padpos(pos); };
    fwd_stages<T, P, PN, 0>(v, lds, tl, tws, lidx);
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = cscale<T>(v[j], lv[j]);
    adj_stages<T, P, PN, L - 1>(v, lds, tl, tws, lidx);
    double acc = 0.0;  // epilogue dot (dotw, y) over this thread's outputs
    if (va) {
        T *ya = y + (long)ra * n, *yb = y + (long)rb * n;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = in_pos<P, PN, 0>(tl, j);
            if (pos < n) {
                T a = v[j].x, b = v[j].y;
                if constexpr (EPI) {
                    const long ia2 = (long)ra * n + pos, ib2 = (long)rb * n + pos;
                    a = ep.scale * a;
                    if (ep.w1) a += ep.a1 * ep.w1[ia2];
                    if (ep.w2) a += ep.a2 * ep.w2[ia2];
                    if (vb) {
                        b = ep.scale * b;
                        if (ep.w1) b += ep.a1 * ep.w1[ib2];
                        if (ep.w2) b += ep.a2 * ep.w2[ib2];
                    }
                    if (ep.dpart) {
                        acc += (double)a * (double)ep.dotw[ia2];
                        if (vb) acc += (double)b * (double)ep.dotw[ib2];
                    }
                }
                st_stream(ya + pos, a);
                if (vb) st_stream(yb + pos, b);
            }
        }
    }
    if constexpr (EPI) {
        if (ep.dpart) {  // block-uniform
            constexpr int NTH = LPB * TL;
            if constexpr (NTH >= 64) {  // whole wavefronts: shuffles see only active lanes
                __shared__ double wsum[NTH / 64];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
                if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
                __syncthreads();
                if (threadIdx.x == 0) {
                    double t = 0.0;
                    for (int w = 0; w < NTH / 64; ++w) t += wsum[w];
                    ep.dpart[z * ep.dpart_stride + bx] = t;
                }
            } else {  // a partial wavefront: through LDS, in thread order
                __shared__ double wsum[NTH];
                wsum[threadIdx.x] = acc;
                __syncthreads();
                if (threadIdx.x == 0) {
                    double t = 0.0;
                    for (int w = 0; w < NTH; ++w) t += wsum[w];
                    ep.dpart[z * ep.dpart_stride + bx] = t;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// strided pass: the C lines of tile t for outer index o, line position p at
// o*outer + t*tile + p*line + c.  MODE 0: forward; 1: inverse; 2: forward,
// multiply by lambda (tiled: t*lam_tile + fold(o)*lam_outer + fold(p)*C + c),
// inverse.  n_in values read (the rest zero), n_out written; in place allowed.
// ---------------------------------------------------------------------------
struct Strides {  // element offsets (below 2^31 for every supported size)
    int in_outer, in_tile, out_outer, out_tile, line;
    int lam_tile, lam_outer;
    int lam_pack = 0;  // PACK: offset of the (lambda_0 - lambda_{P/2}) / 2 column
};

// occupancy target of the strided pass (waves per SIMD): enough resident
// workgroups that one launch of all tiles runs in a single round (2D P=2048:
// 512 tiles of 8 waves, two per CU)
template <typename T, int P, int E, int C, bool PACK> constexpr int strided_waves() {
    if (sizeof(T) != 4 || C * (P / E) != 512 || E != 8) return 1;
    return P == 512 ? (PACK ? 1 : 6) : (P == 2048 ? 4 : 1);
}

// PACK (2D fused pass): column 0 of tile 0 carries two real columns, z = a + i b
// with a = DC and b = Nyquist column of the row transform.  Their spectra
// A, B are the even and odd parts of Z: A(k) = (Z(k) + conj Z(-k)) / 2 and
// i B(k) = (Z(k) - conj Z(-k)) / 2, so lambda_0 A + i lambda_N B =
// s(k) Z(k) + d(k) conj Z(-k) with s = (lambda_0 + lambda_N) / 2 (stored in
// the tile) and d = (lambda_0 - lambda_N) / 2 (at lam_pack).  Both products
// stay Hermitian, so the inverse again gives two real columns.
template <typename T, int P, int E, int C, int MODE, bool PACK = false>
__global__ __launch_bounds__(C * (P / E)) __attribute__((amdgpu_waves_per_eu(strided_waves<T, P, E, C, PACK>())))
void k_strided(
    const C2<T> *in, C2<T> *out, int ncols, int n_in, int n_out, Strides st, const C2<T> *__restrict__ table,
    const T *__restrict__ lam, const double *__restrict__ done, BatchStrides bz) {
    const int zb = blockIdx.z;
    if (done && done[zb * bz.done] != 0.0) return;
    in += zb * bz.in;
    out += zb * bz.out;
    if (lam) lam += zb * bz.lam;
    using PN = Plan<P, E>;
    constexpr int L = PN::L;
    constexpr int PL = padded_len<P>();
    __shared__ C2<T> lds[C * PL];
    const int c = threadIdx.x % C;
    const int tl = threadIdx.x / C;
    // 3D: (tile, outer) from the XCD-aware order with the outer index fastest,
    // since the C-wide chunks of neighbouring outer indices share cache lines
    // (Z pass); a single outer index (2D) keeps the launch order
    const int G = gridDim.x * gridDim.y;
    int t = blockIdx.x, o = 0;
    if (gridDim.y > 1) {
        const int lb = xcd_block(blockIdx.x + gridDim.x * blockIdx.y, G);
        t = lb / gridDim.y;
        o = lb - t * gridDim.y;
    }
    const bool valid = t * C + c < ncols;
    // columns past ncols still lie inside the tile; their loads are discarded
    const C2<T> *src = in + (o * st.in_outer + t * st.in_tile + c);
    C2<T> *dst = out + (o * st.out_outer + t * st.out_tile + c);
    C2<T> tws[num_tw<PN>()];
    C2<T> v[E];
    auto lidx = [c](auto pos) { return padpos(pos) * C + c; };
    if constexpr (MODE == 1) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = out_pos<P, PN, L - 1>(tl, j);
            const bool in = pos < n_in;
            v[j] = keep<T>(valid && in, src[(in ? pos : 0) * st.line]);
        }
        load_twiddles_lanes<T, P, PN>(tws, table, tl);
        adj_stages<T, P, PN, L - 1>(v, lds, tl, tws, lidx);
    } else {
        // twiddles and (MODE 2) lambda first: the waits for the data below
        // (each value is masked as it arrives) then cover their latency too
        load_twiddles_lanes<T, P, PN>(tws, table, tl);
        T lv[E], ldv[E];
        if constexpr (MODE == 2) {
            // lambda at this thread's spectral positions
            const T *lo = lam + (t * st.lam_tile + fold<P>(o) * st.lam_outer + c);
#pragma unroll
            for (int j = 0; j < E; ++j) lv[j] = lo[fold<P>(out_pos<P, PN, L - 1>(tl, j)) * C];
            // the packed column's second symbol d (applied on column 0 only)
            if (PACK && t == 0) {
#pragma unroll
                for (int j = 0; j < E; ++j) ldv[j] = lam[st.lam_pack + fold<P>(out_pos<P, PN, L - 1>(tl, j))];
            }
        }
        load_line<T, P, PN>(v, tl, n_in, [&](int i) { return keep<T>(valid, src[i * st.line]); });
        if constexpr (MODE == 2) {
            fwd_stages<T, P, PN, 0>(v, lds, tl, tws, lidx);
            if (PACK && t == 0) {  // block-uniform: the tile holding the packed column
                // every lane exchanges and applies s Z(k) + d conj Z(-k) without a
                // branch (d = 0 off column 0); the forward stages end with all of
                // their LDS reads behind a barrier, so the writes need none before
#pragma unroll
                for (int j = 0; j < E; ++j) lds[lidx(out_split<P, PN, L - 1>(tl, j))] = v[j];
                __syncthreads();
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    const int pos = out_pos<P, PN, L - 1>(tl, j);
                    const C2<T> zm = lds[lidx((P - pos) & (P - 1))];
                    const T d = c == 0 ? ldv[j] : T(0);
                    v[j] = mk<T>(lv[j] * v[j].x + d * zm.x, lv[j] * v[j].y - d * zm.y);
                }
                __syncthreads();
            } else {
#pragma unroll
                for (int j = 0; j < E; ++j) v[j] = cscale<T>(v[j], lv[j]);
            }
            adj_stages<T, P, PN, L - 1>(v, lds, tl, tws, lidx);
        } else {
            fwd_stages<T, P, PN, 0>(v, lds, tl, tws, lidx);
        }
    }
    if (!valid) return;
    if constexpr (MODE == 0) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = out_pos<P, PN, L - 1>(tl, j);
            if (pos < n_out) st_stream(dst + pos * st.line, v[j]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = in_pos<P, PN, 0>(tl, j);
            if (pos < n_out) st_stream(dst + pos * st.line, v[j]);
        }
    }
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// ev (optional): kernel start / stop events
template <typename K, typename... Args>
static void launch(K kernel, dim3 g, dim3 b, hipStream_t s, const hipEvent_t *ev, Args... args) {
    if (ev)
        hipExtLaunchKernelGGL(kernel, g, b, 0, s, ev[0], ev[1], 0, args...);
    else
        hipLaunchKernelGGL(kernel, g, b, 0, s, args...);
}

template <typename T, int P, int E, int C, int LPB, bool PACK = false>
static void launch_xfwd(const T *u, C2<T> *out, int nrows, int n_in, long in_pitch, int nj, int ntiles,
                        const C2<T> *tw, const double *done, hipStream_t s, const hipEvent_t *ev, int nb = 1,
                        BatchStrides bz = BatchStrides{}) {
    const int pairs = (nrows + 1) / 2;
    launch(k_xfwd<T, P, E, C, LPB, PACK>, dim3(cdiv(pairs, LPB), 1, nb), dim3(LPB * (P / E)), s, ev, u, out, nrows, n_in,
           in_pitch, nj, ntiles, tw + sched_off(P, E), done, bz);
}

template <typename T, int P, int E, int C, int LPB, bool PACK = false>
static void launch_xinv(const C2<T> *in, T *y, int nrows, int n_out, long out_pitch, int nj, int ntiles,
                        const C2<T> *tw, const Epi<T> &ep, const double *done, hipStream_t s, const hipEvent_t *ev,
                        int nb = 1, BatchStrides bz = BatchStrides{}) {
    const int pairs = (nrows + 1) / 2;
    if (ep.active())
        launch(k_xinv<T, P, E, C, LPB, true, PACK>, dim3(cdiv(pairs, LPB), 1, nb), dim3(LPB * (P / E)), s, ev, in,
               y, nrows, n_out, out_pitch, nj, ntiles, tw + sched_off(P, E), ep, done, bz);
    else
        launch(k_xinv<T, P, E, C, LPB, false, PACK>, dim3(cdiv(pairs, LPB), 1, nb), dim3(LPB * (P / E)), s, ev, in,
               y, nrows, n_out, out_pitch, nj, ntiles, tw + sched_off(P, E), ep, done, bz);
}

template <typename T, int P, int E, int C, int MODE, bool PACK = false>
static void launch_strided(const C2<T> *in, C2<T> *out, int ncols, int nouter, int n_in, int n_out,
                           const Strides &st, const C2<T> *tw, const T *lam, const double *done, hipStream_t s,
                           const hipEvent_t *ev, int nb = 1, BatchStrides bz = BatchStrides{}) {
    launch(k_strided<T, P, E, C, MODE, PACK>, dim3(cdiv(ncols, C), nouter, nb), dim3(C * (P / E)), s, ev, in, out, ncols,
           n_in, n_out, st, tw + sched_off(P, E), lam, done, bz);
}

template <typename T, int P, int E, int LPB>
static void launch_conv1d(const T *u, T *y, int nrows, int n, int n_in, const T *lam, const C2<T> *tw,
                          const Epi<T> &ep, const double *done, hipStream_t s, const hipEvent_t *ev, int nb,
                          BatchStrides bz) {
    const int pairs = (nrows + 1) / 2;
    if (ep.active())
        launch(k_conv1d<T, P, E, LPB, true>, dim3(cdiv(pairs, LPB), 1, nb), dim3(LPB * (P / E)), s, ev, u, y, nrows,
               n, n_in, lam, tw + sched_off(P, E), ep, done, bz);
    else
        launch(k_conv1d<T, P, E, LPB, false>, dim3(cdiv(pairs, LPB), 1, nb), dim3(LPB * (P / E)), s, ev, u, y,
               nrows, n, n_in, lam, tw + sched_off(P, E), ep, done, bz);
}

// ---------------------------------------------------------------------------
// the matvec: one variant = (EX points per thread in the row passes, EY in
// the strided passes, tile width C, line pairs per row block LPB)
// ---------------------------------------------------------------------------
template <typename T> static const C2<T> *twid(fl_op op);
template <> const float2 *twid<float>(fl_op op) { return op->tw32; }
template <> const double2 *twid<double>(fl_op op) { return op->tw64; }
template <typename T> static const C2<T> *scht(fl_op op);
template <> const float2 *scht<float>(fl_op op) { return op->sch32; }
template <> const double2 *scht<double>(fl_op op) { return op->sch64; }
template <typename T> static const T *lamt(fl_op op);
template <> const float *lamt<float>(fl_op op) { return op->lam32t; }
template <> const double *lamt<double>(fl_op op) { return op->lam64t; }

template <typename T> MvCtx<T> single_ctx(fl_op op) {
    MvCtx<T> c;
    c.d = op->d;
    c.n = op->n;
    for (int k = 0; k < 3; ++k) c.nk[k] = op->nk[k];
    c.P = op->P;
    c.Q = op->Q;
    c.T1 = op->T1;
    c.T2 = op->T2;
    c.tw = twid<T>(op);
    c.tws = scht<T>(op);
    c.lam = lamt<T>(op);
    return c;
}
template MvCtx<float> single_ctx<float>(fl_op);
template MvCtx<double> single_ctx<double>(fl_op);

template <typename T, int P, int D, int EX, int EY, int C, int LPB>
static void matvec_v(const MvCtx<T> &cx, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                     const hipEvent_t *ev) {
    // interior nodes per axis: the box's own sizes, all below P / 2 + 1, so the
    // same embedding (period P per axis) holds every pair of nodes of the box
    const int nx = cx.nk[0], ny = cx.nk[1], nz = cx.nk[2], Q = cx.Q;
    const int nt = cdiv(spec_cols(D, P), C);
    C2<T> *T1 = (C2<T> *)cx.T1;
    C2<T> *T2 = (C2<T> *)cx.T2;
    const C2<T> *tw = cx.tws;  // the launchers take each plan's lane-ordered table from here
    const T *lam = cx.lam;
    const int nb = cx.batch;
    // element strides between problems: vectors, tiled spectra (in complex values), lambda
    const long zt1 = cx.zs_t1 / (long)sizeof(C2<T>), zt2 = cx.zs_t2 / (long)sizeof(C2<T>);
    auto E = [&](int i) { return ev ? ev + 2 * i : nullptr; };
    BatchStrides b_in{cx.zs_vec, zt1, 0, cx.zs_done};
    // values read per line by the forward passes: zero-padded, or (odd) the odd
    // extension of the sine-transform preconditioner
    const int ix = cx.odd ? -nx : nx, iy = cx.odd ? -ny : ny, iz = cx.odd ? -nz : nz;
    if constexpr (D == 1) {
        (void)T1; (void)T2; (void)nt; (void)ny; (void)nz; (void)Q; (void)zt2; (void)b_in; (void)iy; (void)iz;
        launch_conv1d<T, P, EX, LPB>(u, y, 1, nx, ix, lam, tw, ep, done, s, E(0), nb,
                                     BatchStrides{cx.zs_vec, cx.zs_vec, cx.zs_lam, cx.zs_done});
    } else if constexpr (D == 2) {
        (void)iz;
        launch_xfwd<T, P, EX, C, LPB, true>(u, T1, ny, ix, nx, ny, nt, tw, done, s, E(0), nb, b_in);
        Strides sy{0, ny * C, 0, ny * C, C, Q * C, 0, nt * Q * C};
        launch_strided<T, P, EY, C, 2, true>(T1, T1, P / 2, 1, iy, ny, sy, tw, lam, done, s, E(1), nb,
                                             BatchStrides{zt1, zt1, cx.zs_lam, cx.zs_done});
        launch_xinv<T, P, EX, C, LPB, true>(T1, y, ny, nx, nx, ny, nt, tw, ep, done, s, E(2), nb,
                                            BatchStrides{zt1, cx.zs_vec, 0, cx.zs_done});
    } else {
        const long rows = (long)ny * nz;
        launch_xfwd<T, P, EX, C, LPB>(u, T1, (int)rows, ix, nx, ny, nt, tw, done, s, E(0), nb, b_in);
        Strides s1{nt * ny * C, ny * C, nt * P * C, P * C, C, 0, 0};
        launch_strided<T, P, EY, C, 0>(T1, T2, Q, nz, iy, P, s1, tw, nullptr, done, s, E(1), nb,
                                       BatchStrides{zt1, zt2, 0, cx.zs_done});
        Strides s2{C, P * C, C, P * C, nt * P * C, Q * Q * C, Q * C};
        launch_strided<T, P, EY, C, 2>(T2, T2, Q, P, iz, nz, s2, tw, lam, done, s, E(2), nb,
                                       BatchStrides{zt2, zt2, cx.zs_lam, cx.zs_done});
        Strides s3{nt * P * C, P * C, nt * ny * C, ny * C, C, 0, 0};
        launch_strided<T, P, EY, C, 1>(T2, T1, Q, nz, P, ny, s3, tw, nullptr, done, s, E(3), nb,
                                       BatchStrides{zt2, zt1, 0, cx.zs_done});
        launch_xinv<T, P, EX, C, LPB>(T1, y, (int)rows, nx, nx, ny, nt, tw, ep, done, s, E(4), nb,
                                      BatchStrides{zt1, cx.zs_vec, 0, cx.zs_done});
    }
}

#include "fl_wave2d.hpp"

// the 2D matvec with one wavefront per FFT line (fl_wave2d.hpp): X forward,
// Y fused, X inverse over the same tiled spectra (tiles of C columns)
template <typename T, int P, int C>
static void matvec_w2(const MvCtx<T> &cx, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                      const hipEvent_t *ev) {
    const int nx = cx.nk[0], ny = cx.nk[1], Q = cx.Q;
    const int nt = cdiv(spec_cols(2, P), C);
    C2<T> *T1 = (C2<T> *)cx.T1;
    const long zt1 = cx.zs_t1 / (long)sizeof(C2<T>);
    const int nb = cx.batch;
    auto E = [&](int i) { return ev ? ev + 2 * i : nullptr; };
    const int ix = cx.odd ? -nx : nx, iy = cx.odd ? -ny : ny;
    const int blocks = cdiv(ny, 4);
    launch(k_w2_xfwd<T, P, C>, dim3(blocks, 1, nb), dim3(256), s, E(0), u, T1, ny, ix, (long)nx, ny, nt, cx.tw,
           done, BatchStrides{cx.zs_vec, zt1, 0, cx.zs_done});
    launch(k_w2_yfused<T, P, C, true>, dim3(nt, 1, nb), dim3(64 * C), s, E(1), T1, iy, ny, ny, cx.tw, cx.lam,
           Q * C, nt * Q * C, done, BatchStrides{zt1, zt1, cx.zs_lam, cx.zs_done});
    if (ep.active())
        launch(k_w2_xinv<T, P, C, true>, dim3(blocks, 1, nb), dim3(256), s, E(2), T1, y, ny, nx, (long)nx, ny, nt,
               cx.tw, ep, done, BatchStrides{zt1, cx.zs_vec, 0, cx.zs_done});
    else
        launch(k_w2_xinv<T, P, C, false>, dim3(blocks, 1, nb), dim3(256), s, E(2), T1, y, ny, nx, (long)nx, ny,
               nt, cx.tw, ep, done, BatchStrides{zt1, cx.zs_vec, 0, cx.zs_done});
}

template <typename T> struct Variant {
    VariantDesc desc;
    void (*fn)(const MvCtx<T> &, const T *, T *, const Epi<T> &, const double *, hipStream_t, const hipEvent_t *);
};

#define FL_VAR(T, P, D, EX, EY, C, LPB) \
    { {EX, EY, C, LPB}, &matvec_v<T, P, D, EX, EY, C, LPB> }
#define FL_VARW(T, P, C) \
    { {P / 128, P / 64, C, 2, 1}, &matvec_w2<T, P, C> }
#define FL_DEF(T, P, D)                                                                      \
    FL_VAR(T, P, D, (Shape<T, P, D>::E), (Shape<T, P, D>::E), (Shape<T, P, D>::C), (Shape<T, P, D>::LPB))

// candidate variants per (precision, P, d); the first is the default (for the
// sizes measured so far, the fastest one)
template <typename T> static const Variant<T> *variants(int P, int d, int *count);

template <> const Variant<float> *variants<float>(int P, int d, int *count) {
    using T = float;
    // 1D: one fused pass, one vector pair per workgroup
    static const Variant<T> v1_8[] = {FL_VAR(T, 8, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_16[] = {FL_VAR(T, 16, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_32[] = {FL_VAR(T, 32, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_64[] = {FL_VAR(T, 64, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_128[] = {FL_VAR(T, 128, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_256[] = {FL_VAR(T, 256, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_512[] = {FL_VAR(T, 512, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_1024[] = {FL_VAR(T, 1024, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_2048[] = {FL_VAR(T, 2048, 1, 8, 8, 1, 1)};
    static const Variant<T> v2_8[] = {FL_DEF(T, 8, 2)};
    static const Variant<T> v2_16[] = {FL_DEF(T, 16, 2)};
    static const Variant<T> v2_32[] = {FL_DEF(T, 32, 2)};
    static const Variant<T> v2_64[] = {FL_DEF(T, 64, 2)};
    static const Variant<T> v2_128[] = {FL_DEF(T, 128, 2), FL_VAR(T, 128, 2, 8, 8, 8, 4)};
    static const Variant<T> v2_256[] = {FL_DEF(T, 256, 2), FL_VAR(T, 256, 2, 8, 8, 8, 2),
                                        FL_VAR(T, 256, 2, 8, 8, 4, 2)};
    static const Variant<T> v2_512[] = {FL_DEF(T, 512, 2), FL_VAR(T, 512, 2, 8, 8, 8, 2),
                                        FL_VAR(T, 512, 2, 8, 8, 4, 2), FL_VAR(T, 512, 2, 4, 4, 4, 1)};
    static const Variant<T> v2_1024[] = {FL_DEF(T, 1024, 2), FL_VAR(T, 1024, 2, 8, 8, 4, 2),
                                         FL_VAR(T, 1024, 2, 8, 8, 2, 2), FL_VAR(T, 1024, 2, 4, 4, 2, 1),
                                         FL_VAR(T, 1024, 2, 8, 16, 4, 2)};
    // measured fastest first (MI355X, 2D N=1024): 8 points per thread in the row
    // passes, 16 in the fused pass over 256 tiles of 4 columns (one per CU)
    static const Variant<T> v2_2048[] = {FL_VAR(T, 2048, 2, 8, 16, 4, 1), FL_VARW(T, 2048, 4), FL_VAR(T, 2048, 2, 8, 8, 2, 1),
                                         FL_DEF(T, 2048, 2),             FL_VAR(T, 2048, 2, 8, 8, 4, 1),
                                         FL_VAR(T, 2048, 2, 8, 8, 2, 4), FL_VAR(T, 2048, 2, 4, 4, 2, 1),
                                         FL_VAR(T, 2048, 2, 4, 8, 2, 1), FL_VAR(T, 2048, 2, 16, 8, 2, 2)};
    static const Variant<T> v3_8[] = {FL_DEF(T, 8, 3)};
    static const Variant<T> v3_16[] = {FL_DEF(T, 16, 3)};
    static const Variant<T> v3_32[] = {FL_DEF(T, 32, 3)};
    static const Variant<T> v3_64[] = {FL_DEF(T, 64, 3)};
    static const Variant<T> v3_128[] = {FL_DEF(T, 128, 3)};
    static const Variant<T> v3_256[] = {FL_DEF(T, 256, 3), FL_VAR(T, 256, 3, 8, 8, 16, 2)};
    // measured fastest first (MI355X, 3D N=256: 16 points per thread in every pass,
    // tiles of 8 columns)
    static const Variant<T> v3_512[] = {FL_VAR(T, 512, 3, 16, 16, 8, 4), FL_VAR(T, 512, 3, 8, 16, 8, 4),
                                        FL_VAR(T, 512, 3, 8, 8, 8, 4), FL_DEF(T, 512, 3),
                                        FL_VAR(T, 512, 3, 8, 8, 16, 4), FL_VAR(T, 512, 3, 16, 8, 16, 8),
                                        FL_VAR(T, 512, 3, 8, 16, 16, 4)};
    static const Variant<T> v3_1024[] = {FL_DEF(T, 1024, 3)};
#define FL_PICK(arr)                                  \
    do {                                              \
        *count = (int)(sizeof(arr) / sizeof(arr[0])); \
        return arr;                                   \
    } while (0)
    if (d == 1) {
        switch (P) {
            case 8: FL_PICK(v1_8); case 16: FL_PICK(v1_16); case 32: FL_PICK(v1_32); case 64: FL_PICK(v1_64);
            case 128: FL_PICK(v1_128); case 256: FL_PICK(v1_256); case 512: FL_PICK(v1_512);
            case 1024: FL_PICK(v1_1024); case 2048: FL_PICK(v1_2048);
        }
    } else if (d == 2) {
        switch (P) {
            case 8: FL_PICK(v2_8); case 16: FL_PICK(v2_16); case 32: FL_PICK(v2_32); case 64: FL_PICK(v2_64);
            case 128: FL_PICK(v2_128); case 256: FL_PICK(v2_256); case 512: FL_PICK(v2_512);
            case 1024: FL_PICK(v2_1024); case 2048: FL_PICK(v2_2048);
        }
    } else {
        switch (P) {
            case 8: FL_PICK(v3_8); case 16: FL_PICK(v3_16); case 32: FL_PICK(v3_32); case 64: FL_PICK(v3_64);
            case 128: FL_PICK(v3_128); case 256: FL_PICK(v3_256); case 512: FL_PICK(v3_512);
            case 1024: FL_PICK(v3_1024);
        }
    }
    *count = 0;
    return nullptr;
}

template <> const Variant<double> *variants<double>(int P, int d, int *count) {
    using T = double;
    // 1D: one fused pass, one vector pair per workgroup
    static const Variant<T> v1_8[] = {FL_VAR(T, 8, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_16[] = {FL_VAR(T, 16, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_32[] = {FL_VAR(T, 32, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_64[] = {FL_VAR(T, 64, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_128[] = {FL_VAR(T, 128, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_256[] = {FL_VAR(T, 256, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_512[] = {FL_VAR(T, 512, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_1024[] = {FL_VAR(T, 1024, 1, 8, 8, 1, 1)};
    static const Variant<T> v1_2048[] = {FL_VAR(T, 2048, 1, 8, 8, 1, 1)};
    static const Variant<T> v2_8[] = {FL_DEF(T, 8, 2)};
    static const Variant<T> v2_16[] = {FL_DEF(T, 16, 2)};
    static const Variant<T> v2_32[] = {FL_DEF(T, 32, 2)};
    static const Variant<T> v2_64[] = {FL_DEF(T, 64, 2)};
    static const Variant<T> v2_128[] = {FL_DEF(T, 128, 2)};
    static const Variant<T> v2_256[] = {FL_DEF(T, 256, 2), FL_VAR(T, 256, 2, 8, 8, 4, 2)};
    static const Variant<T> v2_512[] = {FL_DEF(T, 512, 2), FL_VAR(T, 512, 2, 8, 8, 4, 2),
                                        FL_VAR(T, 512, 2, 8, 8, 2, 2)};
    static const Variant<T> v2_1024[] = {FL_DEF(T, 1024, 2), FL_VAR(T, 1024, 2, 8, 8, 2, 2),
                                         FL_VAR(T, 1024, 2, 4, 4, 2, 1)};
    // measured fastest first (MI355X, 2D N=1024): 8 points per thread in every
    // pass, tiles of 2 columns
    static const Variant<T> v2_2048[] = {FL_VAR(T, 2048, 2, 8, 8, 2, 1), FL_VARW(T, 2048, 2), FL_DEF(T, 2048, 2),
                                         FL_VAR(T, 2048, 2, 8, 16, 2, 1), FL_VAR(T, 2048, 2, 8, 8, 2, 2),
                                         FL_VAR(T, 2048, 2, 4, 4, 2, 1)};
    static const Variant<T> v3_8[] = {FL_DEF(T, 8, 3)};
    static const Variant<T> v3_16[] = {FL_DEF(T, 16, 3)};
    static const Variant<T> v3_32[] = {FL_DEF(T, 32, 3)};
    static const Variant<T> v3_64[] = {FL_DEF(T, 64, 3)};
    static const Variant<T> v3_128[] = {FL_DEF(T, 128, 3)};
    static const Variant<T> v3_256[] = {FL_DEF(T, 256, 3)};
    // measured fastest first (MI355X, 3D N=256: the default shape, 16 points per
    // thread in every pass over tiles of 8 columns)
    static const Variant<T> v3_512[] = {FL_DEF(T, 512, 3), FL_VAR(T, 512, 3, 8, 16, 4, 2),
                                        FL_VAR(T, 512, 3, 8, 8, 4, 2), FL_VAR(T, 512, 3, 8, 16, 8, 2),
                                        FL_VAR(T, 512, 3, 8, 8, 8, 2)};
    static const Variant<T> v3_1024[] = {FL_DEF(T, 1024, 3)};
    if (d == 1) {
        switch (P) {
            case 8: FL_PICK(v1_8); case 16: FL_PICK(v1_16); case 32: FL_PICK(v1_32); case 64: FL_PICK(v1_64);
            case 128: FL_PICK(v1_128); case 256: FL_PICK(v1_256); case 512: FL_PICK(v1_512);
            case 1024: FL_PICK(v1_1024); case 2048: FL_PICK(v1_2048);
        }
    } else if (d == 2) {
        switch (P) {
            case 8: FL_PICK(v2_8); case 16: FL_PICK(v2_16); case 32: FL_PICK(v2_32); case 64: FL_PICK(v2_64);
            case 128: FL_PICK(v2_128); case 256: FL_PICK(v2_256); case 512: FL_PICK(v2_512);
            case 1024: FL_PICK(v2_1024); case 2048: FL_PICK(v2_2048);
        }
    } else {
        switch (P) {
            case 8: FL_PICK(v3_8); case 16: FL_PICK(v3_16); case 32: FL_PICK(v3_32); case 64: FL_PICK(v3_64);
            case 128: FL_PICK(v3_128); case 256: FL_PICK(v3_256); case 512: FL_PICK(v3_512);
            case 1024: FL_PICK(v3_1024);
        }
    }
#undef FL_PICK
    *count = 0;
    return nullptr;
}

template <typename T> static int &chosen(fl_op op);
template <> int &chosen<float>(fl_op op) { return op->var32; }
template <> int &chosen<double>(fl_op op) { return op->var64; }

template <typename T>
fl_status matvec_ctx(const MvCtx<T> &cx, int k, const T *u, T *y, const Epi<T> &ep, const double *done,
                     hipStream_t s, hipEvent_t *ev) {
    int count = 0;
    const Variant<T> *vs = variants<T>(cx.P, cx.d, &count);
    if (!vs || k < 0 || k >= count) {
        set_error("no kernel variant %d for FFT length %d, d=%d", k, cx.P, cx.d);
        return FL_E_UNSUPPORTED;
    }
    vs[k].fn(cx, u, y, ep, done, s, ev);
    FL_HIP_TRY(hipGetLastError());
    return FL_OK;
}
template fl_status matvec_ctx<float>(const MvCtx<float> &, int, const float *, float *, const Epi<float> &,
                                     const double *, hipStream_t, hipEvent_t *);
template fl_status matvec_ctx<double>(const MvCtx<double> &, int, const double *, double *, const Epi<double> &,
                                      const double *, hipStream_t, hipEvent_t *);

template <typename T>
fl_status matvec_ex(fl_op op, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                    hipEvent_t *ev) {
    if (large_op(op)) {
        // no fused dot partials (xinv_parts is 0 above the LDS lengths) and no per-pass events
        if (ep.dpart || ev) {
            set_error("operators with FFT length above %d take no fused dot or per-pass events", kMaxLdsP);
            return FL_E_UNSUPPORTED;
        }
        return large_matvec<T>(op, u, y, ep, done, s);
    }
    return matvec_ctx<T>(single_ctx<T>(op), chosen<T>(op), u, y, ep, done, s, ev);
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

int xinv_parts(int d, long rows, int P, int prec, int variant) {
    const VariantDesc vd = variant_desc_pd(P, d, prec, variant);
    return vd.lpb > 0 ? cdiv((rows + 1) / 2, vd.lpb) : 0;
}

int variant_count(fl_op op, int prec) {
    int n = 0;
    if (prec == FL_FP32) variants<float>(op->P, op->d, &n);
    else variants<double>(op->P, op->d, &n);
    return n;
}

VariantDesc variant_desc_pd(int P, int d, int prec, int k) {
    int n = 0;
    if (prec == FL_FP32) {
        const Variant<float> *v = variants<float>(P, d, &n);
        return k >= 0 && k < n ? v[k].desc : VariantDesc{0, 0, 0, 0};
    }
    const Variant<double> *v = variants<double>(P, d, &n);
    return k >= 0 && k < n ? v[k].desc : VariantDesc{0, 0, 0, 0};
}

VariantDesc variant_desc(fl_op op, int prec, int k) {
    int n = 0;
    if (prec == FL_FP32) {
        const Variant<float> *v = variants<float>(op->P, op->d, &n);
        return k >= 0 && k < n ? v[k].desc : VariantDesc{0, 0, 0, 0};
    }
    const Variant<double> *v = variants<double>(op->P, op->d, &n);
    return k >= 0 && k < n ? v[k].desc : VariantDesc{0, 0, 0, 0};
}

// value of the tiled symbol at natural-order entry i (frequency kx, ky, kz):
// lambda itself, or (tau) the sine-transform preconditioner's 1 / (s0 + s1 lambda)
// on the sine modes (no index 0 or P/2 on any axis) and 0 elsewhere, both with
// the inverse transform's 1 / P^d
struct SymMap {
    int tau = 0;
    double s0 = 0.0, s1 = 1.0;
    double Pd = 1.0;  // P^d
};
__device__ __forceinline__ double sym_at(const double *__restrict__ lam64, long i, int kx, int ky, int kz, int d,
                                         int N2, const SymMap &m) {
    const double l = lam64[i];
    if (!m.tau) return l;
    const bool sine = kx != 0 && kx != N2 && (d < 2 || (ky != 0 && ky != N2)) && (d < 3 || (kz != 0 && kz != N2));
    return sine ? 1.0 / ((m.s0 + m.s1 * (l * m.Pd)) * m.Pd) : 0.0;
}

// tiled symbol for the fused pass: 1D natural order, 2D [t][ky][c], 3D [t][ky][kz][c]; zero past
// the stored columns.  2D (packed columns): column 0 holds (s_0 + s_{P/2}) / 2
// and Q more entries after the tiles hold (s_0 - s_{P/2}) / 2, per ky.
template <typename T>
__global__ void k_tile_lambda(const double *__restrict__ lam64, T *__restrict__ lt, int d, int Q, int C, int ntiles,
                              SymMap m) {
    const long tiles = d == 1 ? (long)Q : d == 2 ? (long)ntiles * Q * C : (long)ntiles * Q * Q * C;
    const long total = d == 2 ? tiles + Q : tiles;
    const int N2 = Q - 1;  // P / 2
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        const int c = (int)(idx % C);
        long rest = idx / C;
        double v = 0.0;
        if (d == 1) {
            v = sym_at(lam64, idx, (int)idx, 0, 0, 1, N2, m);
        } else if (d == 2 && idx >= tiles) {
            const int ky = (int)(idx - tiles);
            v = 0.5 * (sym_at(lam64, (long)ky * Q, 0, ky, 0, 2, N2, m) -
                       sym_at(lam64, (long)ky * Q + N2, N2, ky, 0, 2, N2, m));
        } else if (d == 2) {
            const int ky = (int)(rest % Q), t = (int)(rest / Q);
            const int kx = t * C + c;
            if (kx == 0)
                v = 0.5 * (sym_at(lam64, (long)ky * Q, 0, ky, 0, 2, N2, m) +
                           sym_at(lam64, (long)ky * Q + N2, N2, ky, 0, 2, N2, m));
            else if (kx < N2)
                v = sym_at(lam64, (long)ky * Q + kx, kx, ky, 0, 2, N2, m);
        } else {
            const int kz = (int)(rest % Q);
            rest /= Q;
            const int ky = (int)(rest % Q), t = (int)(rest / Q);
            const int kx = t * C + c;
            if (kx < Q) v = sym_at(lam64, ((long)kz * Q + ky) * Q + kx, kx, ky, kz, 3, N2, m);
        }
        lt[idx] = (T)v;
    }
}

#include "fl_fourstep.hpp"

// bad <- 1 where s0 + s1 lambda is not positive and finite on a sine mode
__global__ void k_tau_check(const double *__restrict__ lam64, int d, int Q, SymMap m, int *bad) {
    const long total = d == 1 ? (long)Q : d == 2 ? (long)Q * Q : (long)Q * Q * Q;
    const int N2 = Q - 1;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        const int kx = (int)(idx % Q), ky = d > 1 ? (int)((idx / Q) % Q) : 1, kz = d > 2 ? (int)(idx / Q / Q) : 1;
        const bool sine = kx != 0 && kx != N2 && ky != 0 && ky != N2 && kz != 0 && kz != N2;
        if (!sine) continue;
        const double den = m.s0 + m.s1 * (lam64[idx] * m.Pd);
        if (!(den > 0.0) || !std::isfinite(den)) *bad = 1;
    }
}

__global__ void k_set_int(int *p, int v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

// lambda of one operator tiled to width C into lt (FP32 or FP64)
fl_status tile_lambda(fl_op op, int prec, int C, void *lt, hipStream_t s) {
    const int Q = op->Q, nt = cdiv(spec_cols(op->d, op->P), C);
    const long len = lam_tiled_len(op->d, op->P, C);
    const int g = cdiv(len, 256) > 65536 ? 65536 : cdiv(len, 256);
    if (prec == FL_FP32)
        hipLaunchKernelGGL(k_tile_lambda<float>, dim3(g), dim3(256), 0, s, op->lam64, (float *)lt, op->d, Q, C, nt,
                           SymMap{});
    else
        hipLaunchKernelGGL(k_tile_lambda<double>, dim3(g), dim3(256), 0, s, op->lam64, (double *)lt, op->d, Q, C, nt,
                           SymMap{});
    FL_HIP_TRY(hipGetLastError());
    return FL_OK;
}

// select variant k for a precision: re-tile lambda to the variant's tile width
fl_status select_variant(fl_op op, int prec, int k, hipStream_t s) {
    const int n = variant_count(op, prec);
    if (k < 0 || k >= n) {
        set_error("variant %d out of range (%d available)", k, n);
        return FL_E_INVAL;
    }
    const VariantDesc vd = variant_desc(op, prec, k);
    const int Q = op->Q, nt = cdiv(spec_cols(op->d, op->P), vd.c);
    const long len = lam_tiled_len(op->d, op->P, vd.c);
    const int g = cdiv(len, 256) > 65536 ? 65536 : cdiv(len, 256);
    if (prec == FL_FP32)
        hipLaunchKernelGGL(k_tile_lambda<float>, dim3(g), dim3(256), 0, s, op->lam64, op->lam32t, op->d, Q, vd.c, nt,
                           SymMap{});
    else
        hipLaunchKernelGGL(k_tile_lambda<double>, dim3(g), dim3(256), 0, s, op->lam64, op->lam64t, op->d, Q, vd.c,
                           nt, SymMap{});
    FL_HIP_TRY(hipGetLastError());
    if (prec == FL_FP32) op->var32 = k;
    else op->var64 = k;
    return FL_OK;
}

// ---------------------------------------------------------------------------
// sine-transform (tau) preconditioner of K = s0 I + s1 A.  On n' = P/2 - 1
// nodes per axis the sine vectors sin(pi j k / (n' + 1)) are eigenvectors of
// every matrix S diag(mu) S; with mu the circulant symbol of K at the sine
// frequencies this is the tau-class matrix of the n'-node K (K minus its two
// Hankel corrections).  Its inverse applied to r is the circulant of symbol
// 1 / mu on the odd extension of r, cropped: the matvec's passes with the
// odd loads and the inverted symbol.  On power-of-two squares and cubes
// n' = n; otherwise r is zero-extended to the n' grid and the result
// restricted to the operator's nodes, which needs n_k <= n' on every axis.
// ---------------------------------------------------------------------------
bool tau_supported(const fl_op_s *op) {
    for (int k = 0; k < op->d; ++k)
        if (op->nk[k] > op->P / 2 - 1) return false;
    return true;
}

fl_status tau_symbol(fl_op op, double s0, double s1, int prec, int C, void *lt, hipStream_t s) {
    if (!tau_supported(op)) {
        set_error("the sine-transform preconditioner needs at most P/2 - 1 nodes per axis (N not 2^k + 1)");
        return FL_E_UNSUPPORTED;
    }
    if (!(s0 >= 0.0) || !(s1 >= 0.0) || !(s0 + s1 > 0.0) || !std::isfinite(s0) || !std::isfinite(s1)) {
        set_error("preconditioner of s0 I + s1 A needs s0, s1 >= 0, not both 0");
        return FL_E_INVAL;
    }
    const int d = op->d, Q = op->Q;
    SymMap m;
    m.tau = 1;
    m.s0 = s0;
    m.s1 = s1;
    m.Pd = std::pow((double)op->P, d);
    // positivity on the sine modes (the workspace T1 holds the flag)
    int *bad = (int *)op->T1;
    const long ql = d == 1 ? (long)Q : d == 2 ? (long)Q * Q : (long)Q * Q * Q;
    const int g = cdiv(ql, 256) > 65536 ? 65536 : cdiv(ql, 256);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, bad, 0);
    hipLaunchKernelGGL(k_tau_check, dim3(g), dim3(256), 0, s, op->lam64, d, Q, m, bad);
    int hbad = 0;
    FL_HIP_TRY(hipGetLastError());
    FL_HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    FL_HIP_TRY(hipStreamSynchronize(s));
    if (hbad) {
        set_error("s0 + s1 lambda is not positive on every sine mode: no sine-transform preconditioner");
        return FL_E_BREAKDOWN;
    }
    if (large_op(op)) {  // natural order, as the large-operator passes read lambda
        const int gn = cdiv(ql, 256) > 65536 ? 65536 : cdiv(ql, 256);
        if (prec == FL_FP32)
            hipLaunchKernelGGL(k_large_symbol<float>, dim3(gn), dim3(256), 0, s, op->lam64, (float *)lt, Q, m);
        else
            hipLaunchKernelGGL(k_large_symbol<double>, dim3(gn), dim3(256), 0, s, op->lam64, (double *)lt, Q, m);
        FL_HIP_TRY(hipGetLastError());
        return FL_OK;
    }
    const int nt = cdiv(spec_cols(d, op->P), C);
    const long len = lam_tiled_len(d, op->P, C);
    const int gt = cdiv(len, 256) > 65536 ? 65536 : cdiv(len, 256);
    if (prec == FL_FP32)
        hipLaunchKernelGGL(k_tile_lambda<float>, dim3(gt), dim3(256), 0, s, op->lam64, (float *)lt, d, Q, C, nt, m);
    else
        hipLaunchKernelGGL(k_tile_lambda<double>, dim3(gt), dim3(256), 0, s, op->lam64, (double *)lt, d, Q, C, nt,
                           m);
    FL_HIP_TRY(hipGetLastError());
    return FL_OK;
}

fl_status tau_prepare(fl_op op, double s0, double s1, hipStream_t s) {
    if (!tau_supported(op)) return tau_symbol(op, s0, s1, FL_FP64, 1, nullptr, s);  // sets the error
    if (op->mu64t && op->mu_var == op->var64 && op->mu_s0 == s0 && op->mu_s1 == s1) return FL_OK;
    if (!op->mu64t) {
        long qrest = 1;
        for (int k = 1; k < op->d; ++k) qrest *= op->Q;
        const long len = qrest * (op->Q + kMaxTile - 1);
        hipError_t e = hipMalloc((void **)&op->mu64t, sizeof(double) * len);
        if (e != hipSuccess) {
            op->mu64t = nullptr;
            set_error("preconditioner symbol: %s", hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? FL_E_NOMEM : FL_E_DEVICE;
        }
    }
    op->mu_var = -1;
    FL_TRY(tau_symbol(op, s0, s1, FL_FP64, variant_desc(op, FL_FP64, op->var64).c, op->mu64t, s));
    op->mu_var = op->var64;
    op->mu_s0 = s0;
    op->mu_s1 = s1;
    return FL_OK;
}

fl_status tau_prepare32(fl_op op, double s0, double s1, hipStream_t s) {
    if (!tau_supported(op)) return tau_symbol(op, s0, s1, FL_FP32, 1, nullptr, s);  // sets the error
    if (op->mu32t && op->mu32_var == op->var32 && op->mu32_s0 == s0 && op->mu32_s1 == s1) return FL_OK;
    if (!op->mu32t) {
        long qrest = 1;
        for (int k = 1; k < op->d; ++k) qrest *= op->Q;
        const long len = qrest * (op->Q + kMaxTile - 1);
        hipError_t e = hipMalloc((void **)&op->mu32t, sizeof(float) * len);
        if (e != hipSuccess) {
            op->mu32t = nullptr;
            set_error("preconditioner symbol: %s", hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? FL_E_NOMEM : FL_E_DEVICE;
        }
    }
    op->mu32_var = -1;
    FL_TRY(tau_symbol(op, s0, s1, FL_FP32, variant_desc(op, FL_FP32, op->var32).c, op->mu32t, s));
    op->mu32_var = op->var32;
    op->mu32_s0 = s0;
    op->mu32_s1 = s1;
    return FL_OK;
}

fl_status tau_apply32(fl_op op, const float *r, float *z, const double *done, hipStream_t s) {
    if (!op->mu32t || op->mu32_var != op->var32) {
        set_error("sine-transform preconditioner not prepared for the selected FP32 kernel variant");
        return FL_E_INVAL;
    }
    if (large_op(op)) return large_matvec<float>(op, r, z, Epi<float>{}, done, s, op->mu32t, true);
    MvCtx<float> cx = single_ctx<float>(op);
    cx.lam = op->mu32t;
    cx.odd = true;
    return matvec_ctx<float>(cx, op->var32, r, z, Epi<float>{}, done, s);
}

fl_status tau_apply(fl_op op, const double *r, double *z, const double *done, hipStream_t s) {
    if (!op->mu64t || op->mu_var != op->var64) {
        set_error("sine-transform preconditioner not prepared for the selected kernel variant");
        return FL_E_INVAL;
    }
    if (large_op(op)) return large_matvec<double>(op, r, z, Epi<double>{}, done, s, op->mu64t, true);
    MvCtx<double> cx = single_ctx<double>(op);
    cx.lam = op->mu64t;
    cx.odd = true;
    return matvec_ctx<double>(cx, op->var64, r, z, Epi<double>{}, done, s);
}

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

// natural-order lambda (x fastest, Q^d) from the tiled spectrum of width C
__global__ void k_extract(const double2 *__restrict__ spec, double *__restrict__ lam64, int d, int P, int Q,
                          int C, int ntiles, double inv) {
    const long total = d == 2 ? (long)Q * Q : (long)Q * Q * Q;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long)gridDim.x * blockDim.x) {
        const int kx = (int)(idx % Q);
        const long rest = idx / Q;
        long src;
        if (d == 2) src = ((long)(kx / C) * P + rest) * C + kx % C;
        else {
            const long ky = rest % Q, kz = rest / Q;
            src = (((kz * ntiles + kx / C) * P) + ky) * C + kx % C;
        }
        lam64[idx] = spec[src].x * inv;
    }
}

template <int P, int D>
static void symbol_fft(double *cemb, double2 *T, const double2 *tw, hipStream_t s) {
    using S = Shape<double, P, D>;
    constexpr int E = S::E, C = S::C, LPB = S::LPB;
    const int Q = P / 2 + 1, nt = cdiv(Q, C);
    if constexpr (D == 2) {
        launch_xfwd<double, P, E, C, LPB>(cemb, T, P, P, P, P, nt, tw, nullptr, s, nullptr);
        Strides sy{0, P * C, 0, P * C, C, 0, 0};
        launch_strided<double, P, E, C, 0>(T, T, Q, 1, P, P, sy, tw, nullptr, nullptr, s, nullptr);
    } else {
        launch_xfwd<double, P, E, C, LPB>(cemb, T, P * P, P, P, P, nt, tw, nullptr, s, nullptr);
        Strides sy{nt * P * C, P * C, nt * P * C, P * C, C, 0, 0};
        launch_strided<double, P, E, C, 0>(T, T, Q, P, P, P, sy, tw, nullptr, nullptr, s, nullptr);
        Strides sz{C, P * C, C, P * C, nt * P * C, 0, 0};
        launch_strided<double, P, E, C, 0>(T, T, Q, P, P, P, sz, tw, nullptr, nullptr, s, nullptr);
    }
}

// 1D symbol: lambda(k) / P = (t_0 + 2 sum_{m=1}^{n-1} t_m cos(2 pi k m / P)) / P for
// the even generator t_m = -c a_m (zero in the gap), k < Q; a direct cosine sum
// (n <= 1024 terms per k) with the FP64 twiddle table and a compensated sum
__global__ __launch_bounds__(256) void k_symbol1d(const double *__restrict__ a, const double2 *__restrict__ tw,
                                                  double *__restrict__ lam64, int n, int P, double negc) {
    const int Q = P / 2 + 1;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < Q; k += gridDim.x * blockDim.x) {
        double s = 0.0, comp = 0.0;
        for (int m = 1; m <= n - 1; ++m) {
            const double t = 2.0 * negc * a[m] * tw[(long)k * m % P].x;
            const double y = s + t;
            comp += fabs(s) >= fabs(t) ? (s - y) + t : (t - y) + s;
            s = y;
        }
        lam64[k] = (negc * a[0] + (s + comp)) / (double)P;
    }
}

// ---------------------------------------------------------------------------
// lane-ordered twiddle tables: thread tl of plan (P, E) gathers its twiddles
// from the natural-order table exactly as load_twiddles does and stores them
// at k * TL + tl
// ---------------------------------------------------------------------------
template <typename T, int P, int E>
__global__ __launch_bounds__(256) void k_make_sched(const C2<T> *__restrict__ table, C2<T> *__restrict__ sched) {
    using PN = Plan<P, E>;
    constexpr int TL = P / E;
    const int tl = blockIdx.x * blockDim.x + threadIdx.x;
    if (tl >= TL) return;
    if constexpr (PN::L > 1) {
        C2<T> tws[num_tw<PN>()];
        load_twiddles<T, P, PN>(tws, table, tl);
        C2<T> *out = sched + sched_off(P, E);
#pragma unroll
        for (int k = 0; k < num_tw<PN>(); ++k) out[(long)k * TL + tl] = tws[k];
    }
}

template <typename T, int P, int E = 2>
static void make_sched_all(const C2<T> *table, C2<T> *sched, hipStream_t s) {
    if constexpr (E <= 32) {
        if constexpr (plan_ok(P, E)) {
            constexpr int TL = P / E;
            hipLaunchKernelGGL((k_make_sched<T, P, E>), dim3(cdiv(TL, 256)), dim3(256), 0, s, table, sched);
        }
        make_sched_all<T, P, 2 * E>(table, sched, s);
    }
}

// twiddles exp(-2 pi i m / L) of the large-operator passes' short transforms
// (L = 16 ... 128 at fs_tw_off(L)), taken from the length-P table
template <typename T>
__global__ void k_fs_subtw(const C2<T> *__restrict__ tw, C2<T> *__restrict__ sub, int P) {
    const int i = threadIdx.x;
    for (int L = 16; L <= 128; L *= 2)
        if (i < L) sub[fs_tw_off(L) + i] = tw[i * (P / L)];
}

fl_status make_schedules(fl_op op, hipStream_t s) {
    if (large_op(op)) {
        FL_HIP_TRY(hipMalloc((void **)&op->sch64, sizeof(double2) * kFsTwLen));
        FL_HIP_TRY(hipMalloc((void **)&op->sch32, sizeof(float2) * kFsTwLen));
        hipLaunchKernelGGL(k_fs_subtw<double>, dim3(1), dim3(128), 0, s, op->tw64, op->sch64, op->P);
        hipLaunchKernelGGL(k_fs_subtw<float>, dim3(1), dim3(128), 0, s, op->tw32, op->sch32, op->P);
        FL_HIP_TRY(hipGetLastError());
        return FL_OK;
    }
    switch (op->P) {
#define FL_SCHED(PP)                                                  \
    case PP:                                                          \
        make_sched_all<double, PP>(op->tw64, op->sch64, s);           \
        make_sched_all<float, PP>(op->tw32, op->sch32, s);            \
        break;
        FL_SCHED(8) FL_SCHED(16) FL_SCHED(32) FL_SCHED(64) FL_SCHED(128) FL_SCHED(256) FL_SCHED(512)
        FL_SCHED(1024) FL_SCHED(2048)
#undef FL_SCHED
        default:
            set_error("no twiddle tables for FFT length %d", op->P);
            return FL_E_UNSUPPORTED;
    }
    FL_HIP_TRY(hipGetLastError());
    return FL_OK;
}

// ---------------------------------------------------------------------------
// Symbol of a large 2D operator (FFT length P = 4096 ... 16384), built once:
// the generator embedded in P x P, transformed along x (P/2 row pairs packed
// as complex lines, then split into half spectra) and along y over the Q
// columns, every radix pass a kernel over the whole buffer in HBM (Stockham
// autosort, out of place, radix 16 as 4 x 4 in registers, then radix 4 or 2
// for the rest of log2 P; the indexing of Govindaraju et al., SC 2008).  The
// matvec itself runs the four-step passes of fl_fourstep.hpp.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_big_pack(const T *__restrict__ u, C2<T> *__restrict__ lines, int nx, int ny,
                                                  int P) {
    const int nl = (ny + 1) / 2;
    const long total = (long)nl * nx;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const long r = idx / nx;
        const int p = (int)(idx - r * nx);
        const T a = u[2 * r * nx + p];
        const T b = 2 * r + 1 < ny ? u[(2 * r + 1) * nx + p] : T(0);
        lines[r * P + p] = mk<T>(a, b);
    }
}

// forward radix-4 DFT in place: X1 = t1 - i t3, X3 = t1 + i t3
template <typename T>
__device__ __forceinline__ void big_dft4(C2<T> &a, C2<T> &b, C2<T> &c, C2<T> &d) {
    const C2<T> t0 = cadd<T>(a, c), t1 = csub<T>(a, c), t2 = cadd<T>(b, d), t3 = csub<T>(b, d);
    const C2<T> it3 = cmuli<T, -1>(t3);
    a = cadd<T>(t0, t2);
    c = csub<T>(t0, t2);
    b = cadd<T>(t1, it3);
    d = csub<T>(t1, it3);
}

// one forward Stockham pass of radix R over nlines transforms of length P: line
// l, position q at l*lstride + q*pstride.  LINE_FAST: consecutive threads take
// consecutive lines (the column passes, whose lines are adjacent in memory).
template <typename T, int R, bool LINE_FAST>
__global__ __launch_bounds__(256) void k_big_pass(const C2<T> *__restrict__ in, C2<T> *__restrict__ out, int P, int Ns,
                                                  int nlines, long lstride, long pstride, const C2<T> *__restrict__ tw) {
    const int PR = P / R;
    const long total = (long)nlines * PR;
    for (long g = (long)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (long)gridDim.x * blockDim.x) {
        long line;
        int j;
        if (LINE_FAST) {
            line = g % nlines;
            j = (int)(g / nlines);
        } else {
            line = g / PR;
            j = (int)(g - line * PR);
        }
        const C2<T> *src = in + line * lstride;
        C2<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[(long)(j + r * PR) * pstride];
        // twiddles W^{r m}, W = exp(-2 pi i / (Ns R)): table index r m P / (Ns R) < P
        const int m = j % Ns, step = P / (Ns * R);
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul<T>(v[r], tw[r * m * step]);
        if constexpr (R == 2) {
            const C2<T> a = v[0];
            v[0] = cadd<T>(a, v[1]);
            v[1] = csub<T>(a, v[1]);
        } else if constexpr (R == 4) {
            big_dft4<T>(v[0], v[1], v[2], v[3]);
        } else {
            // 16 = 4 x 4: DFT4 over n1 of x[4 n1 + n2] for each n2, twiddle W16^(n2 k1),
            // DFT4 over n2 for each k1; X[k1 + 4 k2] lands in v[4 n2 + k1] transposed below
#pragma unroll
            for (int n2 = 0; n2 < 4; ++n2) big_dft4<T>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
#pragma unroll
            for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
                for (int k1 = 1; k1 < 4; ++k1) v[4 * k1 + n2] = cmul<T>(v[4 * k1 + n2], tw[n2 * k1 * (P / 16)]);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) big_dft4<T>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
            // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 index
            C2<T> w[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) w[k] = v[k];
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
                for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = w[4 * k1 + k2];
        }
        C2<T> *dst = out + line * lstride;
        const int base = (j / Ns) * Ns * R + m;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[(long)(base + r * Ns) * pstride] = v[r];
    }
}

// half spectra of the two real rows in each line: X_a = (Z(k) + conj Z(-k)) / 2
// to row 2r, X_b = (Z(k) - conj Z(-k)) / (2i) to row 2r + 1, k < Q
template <typename T>
__global__ __launch_bounds__(256) void k_big_split(const C2<T> *__restrict__ Z, C2<T> *__restrict__ S, int nrows, int P,
                                                   int Q, int Qs) {
    const int nl = (nrows + 1) / 2;
    const long total = (long)nl * Q;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const long r = idx / Q;
        const int k = (int)(idx - r * Q);
        const C2<T> zk = Z[r * P + k];
        const C2<T> zm = cconj<T>(Z[r * P + ((P - k) & (P - 1))]);
        S[2 * r * Qs + k] = cscale<T>(cadd<T>(zk, zm), T(0.5));
        if (2 * r + 1 < nrows) {
            const C2<T> w = csub<T>(zk, zm);
            S[(2 * r + 1) * Qs + k] = mk<T>(T(0.5) * w.y, T(-0.5) * w.x);
        }
    }
}

// lambda / P^2 in natural order (ky, kx < Q) from the forward spectrum of the generator
__global__ __launch_bounds__(256) void k_big_extract(const double2 *__restrict__ F, double *__restrict__ lam64, int P,
                                                     int Q, int Qs) {
    const long total = (long)Q * Q;
    const double inv = 1.0 / ((double)P * (double)P);
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const long ky = idx / Q, kx = idx - ky * Q;
        lam64[idx] = F[ky * Qs + kx].x * inv;
    }
}

static int big_grid(long total) {
    const long g = (total + 255) / 256;
    return (int)(g > (1L << 20) ? (1L << 20) : (g < 1 ? 1 : g));
}

// the forward passes of one set of transforms (radix 16 while it divides, then
// 4 or 2), ping-ponging between a and b; returns the buffer that holds the result
template <typename T, bool LINE_FAST>
static C2<T> *big_fft(C2<T> *a, C2<T> *b, int P, int nlines, long lstride, long pstride, const C2<T> *tw,
                      hipStream_t s) {
    for (int Ns = 1; Ns < P;) {
        const int R = (P / Ns) % 16 == 0 ? 16 : ((P / Ns) % 4 == 0 ? 4 : 2);
        const int g = big_grid((long)nlines * (P / R));
        if (R == 16)
            hipLaunchKernelGGL((k_big_pass<T, 16, LINE_FAST>), dim3(g), dim3(256), 0, s, a, b, P, Ns, nlines, lstride,
                               pstride, tw);
        else if (R == 4)
            hipLaunchKernelGGL((k_big_pass<T, 4, LINE_FAST>), dim3(g), dim3(256), 0, s, a, b, P, Ns, nlines, lstride,
                               pstride, tw);
        else
            hipLaunchKernelGGL((k_big_pass<T, 2, LINE_FAST>), dim3(g), dim3(256), 0, s, a, b, P, Ns, nlines, lstride,
                               pstride, tw);
        Ns *= R;
        C2<T> *t = a;
        a = b;
        b = t;
    }
    return a;
}

template <typename T> static const T *big_lam(fl_op op);
template <> const float *big_lam<float>(fl_op op) { return op->lam32t; }
template <> const double *big_lam<double>(fl_op op) { return op->lam64; }
template <typename T> static const C2<T> *fs_subtw(fl_op op);
template <> const float2 *fs_subtw<float>(fl_op op) { return op->sch32; }
template <> const double2 *fs_subtw<double>(fl_op op) { return op->sch64; }

// sym (optional) replaces lambda (Q x Q, natural order); odd: the forward
// passes read the odd extensions (the sine-transform preconditioner)
template <typename T>
fl_status large_matvec(fl_op op, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                       const T *sym, bool odd) {
    const T *lam = sym ? sym : big_lam<T>(op);
    const C2<T> *tw = twid<T>(op), *sub = fs_subtw<T>(op);
    fl_status st = FL_E_UNSUPPORTED;
    switch (op->P) {
        case 4096: st = fs_matvec<T, 64, 64>(op, u, y, ep, done, s, lam, odd, tw, sub); break;
        case 8192: st = fs_matvec<T, 64, 128>(op, u, y, ep, done, s, lam, odd, tw, sub); break;
        case 16384: st = fs_matvec<T, 128, 128>(op, u, y, ep, done, s, lam, odd, tw, sub); break;
        default: set_error("no four-step plan for FFT length %d", op->P);
    }
    if (st != FL_OK) return st;
    FL_HIP_TRY(hipGetLastError());
    return FL_OK;
}
template fl_status large_matvec<float>(fl_op, const float *, float *, const Epi<float> &, const double *,
                                       hipStream_t, const float *, bool);
template fl_status large_matvec<double>(fl_op, const double *, double *, const Epi<double> &, const double *,
                                        hipStream_t, const double *, bool);

// lambda of a large operator: the generator -c a_{|m|} embedded in P x P
// (the same embedding as the LDS path), transformed along x (P rows) and y
// (Q columns) in FP64; the real part / P^2 at ky, kx < Q
fl_status large_symbol(fl_op op, hipStream_t s) {
    const int P = op->P, Q = op->Q, Qs = op->Qp;
    const long total = (long)P * P;
    double *cemb = nullptr;
    FL_HIP_TRY(hipMalloc((void **)&cemb, sizeof(double) * total));
    double2 *B0 = (double2 *)op->T1, *B1 = (double2 *)op->T2;
    hipLaunchKernelGGL(k_embed, dim3(big_grid(total)), dim3(256), 0, s, op->a, cemb, 2, op->N, P, -op->c);
    hipLaunchKernelGGL(k_big_pack<double>, dim3(big_grid(total / 2)), dim3(256), 0, s, cemb, B0, P, P, P);
    double2 *X = big_fft<double, false>(B0, B1, P, P / 2, P, 1, op->tw64, s);
    double2 *S = X == B0 ? B1 : B0;
    hipLaunchKernelGGL(k_big_split<double>, dim3(big_grid((long)(P / 2) * Q)), dim3(256), 0, s, X, S, P, P, Q, Qs);
    double2 *F = big_fft<double, true>(S, X, P, Q, 1, Qs, op->tw64, s);
    hipLaunchKernelGGL(k_big_extract, dim3(big_grid((long)Q * Q)), dim3(256), 0, s, F, op->lam64, P, Q, Qs);
    // the FP32 copy the FP32 passes read (the FP64 passes read lam64 itself)
    hipLaunchKernelGGL(k_large_symbol<float>, dim3(big_grid((long)Q * Q)), dim3(256), 0, s, op->lam64, op->lam32t, Q,
                       SymMap{});
    hipError_t le = hipGetLastError();
    hipError_t se = hipStreamSynchronize(s);
    (void)hipFree(cemb);
    FL_HIP_TRY(le);
    FL_HIP_TRY(se);
    // the persistent row kernel's grid from the occupancy calculator, cached now
    // so that no matvec (possibly under a caller's graph capture) queries it
    if (P == 16384) (void)fs_grid<k_fs_xrow<double, 64, false>>(xr_threads<64>(), 1);
    return FL_OK;
}

template <int P, int D> constexpr int sym_c() { return Shape<double, P, D>::C; }

fl_status build_symbol(fl_op op, hipStream_t s) {
    const int d = op->d, P = op->P, Q = op->Q;
    if (large_op(op)) return large_symbol(op, s);
    if (d == 1) {
        hipLaunchKernelGGL(k_symbol1d, dim3(cdiv(Q, 256)), dim3(256), 0, s, op->a, op->tw64, op->lam64, op->n, P,
                           -op->c);
        fl_status st = select_variant(op, FL_FP32, op->var32, s);
        if (st == FL_OK) st = select_variant(op, FL_FP64, op->var64, s);
        FL_TRY(st);
        FL_HIP_TRY(hipGetLastError());
        FL_HIP_TRY(hipStreamSynchronize(s));
        return FL_OK;
    }
    int C = 0;
#define FL_SYC(PP)                                           \
    case PP: C = d == 2 ? sym_c<PP, 2>() : sym_c<PP, 3>(); break;
    switch (P) {
        FL_SYC(8) FL_SYC(16) FL_SYC(32) FL_SYC(64) FL_SYC(128) FL_SYC(256) FL_SYC(512) FL_SYC(1024)
        case 2048: C = sym_c<2048, 2>(); break;
        default: set_error("FFT length %d not built", P); return FL_E_UNSUPPORTED;
    }
#undef FL_SYC
    const int nt = cdiv(Q, C);
    const long total = d == 2 ? (long)P * P : (long)P * P * P;
    const long rows = total / P;
    double *cemb = nullptr;
    double2 *T = nullptr;
    FL_HIP_TRY(hipMalloc((void **)&cemb, sizeof(double) * total));
    hipError_t e = hipMalloc((void **)&T, sizeof(double2) * rows * nt * C);
    if (e != hipSuccess) {
        (void)hipFree(cemb);
        set_error("workspace for the symbol: %s", hipGetErrorString(e));
        return FL_E_NOMEM;
    }
    auto grid = [](long n) { return cdiv(n, 256) > 65536 ? 65536 : cdiv(n, 256); };
    hipLaunchKernelGGL(k_embed, dim3(grid(total)), dim3(256), 0, s, op->a, cemb, d, op->N, P, -op->c);
#define FL_SY(PP)                                                          \
    case PP:                                                               \
        if (d == 2) symbol_fft<PP, 2>(cemb, T, op->sch64, s);              \
        else symbol_fft<PP, 3>(cemb, T, op->sch64, s);                     \
        break;
    switch (P) {
        FL_SY(8) FL_SY(16) FL_SY(32) FL_SY(64) FL_SY(128) FL_SY(256) FL_SY(512) FL_SY(1024)
        case 2048: symbol_fft<2048, 2>(cemb, T, op->sch64, s); break;
    }
#undef FL_SY
    const long ql = d == 2 ? (long)Q * Q : (long)Q * Q * Q;
    hipLaunchKernelGGL(k_extract, dim3(grid(ql)), dim3(256), 0, s, T, op->lam64, d, P, Q, C, nt,
                       1.0 / (double)total);
    fl_status st = select_variant(op, FL_FP32, op->var32, s);
    if (st == FL_OK) st = select_variant(op, FL_FP64, op->var64, s);
    hipError_t le = hipGetLastError();
    hipError_t se = hipStreamSynchronize(s);
    (void)hipFree(cemb);
    (void)hipFree(T);
    FL_TRY(st);
    FL_HIP_TRY(le);
    FL_HIP_TRY(se);
    return FL_OK;
}

}  // namespace fl
