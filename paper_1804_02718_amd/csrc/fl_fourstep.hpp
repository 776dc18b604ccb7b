// Large 2D operators (FFT length P = 4096 ... 16384) by the four-step
// factorisation P = P1 * P2 (P1, P2 in {64, 128}).  Included inside namespace
// fl by fl_fft.hip, after the plan, stage and twiddle helpers.
//
// A line of P values no longer fits a workgroup's LDS, but its transform splits
// into short transforms that do.  With n = P2 n1 + n2 and k = k1 + P1 k2,
//   X[k1 + P1 k2] = sum_n2 W_P2^(n2 k2) W_P^(n2 k1) sum_n1 x[P2 n1 + n2] W_P1^(n1 k1),
// so a transform is one pass of P1-point transforms over n1 (a stride of P2)
// with the twiddle W_P^(n2 k1), then one pass of P2-point transforms over the
// contiguous n2, and the inverse runs the same steps backwards with conjugate
// twiddles.  The spectrum stays in that transposed order (k1 major).
//
// y = A u takes seven passes over HBM, each a set of short transforms in LDS:
//   xa   row pairs packed as complex lines, x step 1 (P1-point), twiddle
//   xb   x step 2 (P2-point) and the Hermitian split into the half spectra of
//        the two rows; lines k1 and P1 - k1 share a workgroup, so each finds
//        its mirror Z(-k) in LDS
//   ya   y step 1 over the Q half-spectrum columns, twiddle
//   ymid y step 2, lambda, the inverse of y step 2 (in place)
//   yai  conjugate twiddle, inverse y step 1, the ny rows kept
//   xbi  unsplit and inverse x step 2, conjugate twiddle
//   xai  inverse x step 1, unpack to the two rows, solver epilogue
// The half-spectrum columns are stored in the permuted order fs_col below
// (k1-major, mirror lines adjacent), which keeps every access of every pass a
// run of consecutive addresses; lambda is stored in the same column order.

template <int L> struct FsPlan;
template <> struct FsPlan<128> { using PN = Plan<128, 8>; };
template <> struct FsPlan<64> { using PN = Plan<64, 8>; };
// short transforms per workgroup (lines); P1 and P2 are multiples of it
constexpr int kFsLines = 32;
template <int L> constexpr int fs_threads() { return kFsLines * (L / FsPlan<L>::PN::E); }
// the short transforms' twiddle tables exp(-2 pi i m / L) in one buffer
constexpr int fs_tw_off(int L) { return L == 128 ? 0 : 128; }
constexpr int kFsTwLen = 192;

// column of half-spectrum frequency kx = k1 + P1 k2 (kx <= P / 2):
//   k1 = 0:       k2 in [0, P2/2]      -> columns [0, P2/2]
//   k1 = P1/2:    k2 in [0, P2/2)      -> columns (P2/2, P2]
//   the pair p = min(k1, P1 - k1) in [1, P1/2): line p, then line P1 - p,
//                 P2/2 columns each from P2 + 1 + (p - 1) P2
__host__ __device__ inline int fs_col(int P1, int P2, int k1, int k2) {
    if (k1 == 0) return k2;
    if (k1 == P1 / 2) return P2 / 2 + 1 + k2;
    const bool lo = k1 < P1 / 2;
    const int p = lo ? k1 : P1 - k1;
    return P2 + 1 + (2 * (p - 1) + (lo ? 0 : 1)) * (P2 / 2) + k2;
}
// the frequency kx of a column (the inverse of fs_col)
__host__ __device__ inline int fs_kx(int P1, int P2, int col) {
    if (col <= P2 / 2) return P1 * col;
    if (col <= P2) return P1 / 2 + P1 * (col - (P2 / 2 + 1));
    const int c = col - (P2 + 1), g = c / (P2 / 2), k2 = c - g * (P2 / 2);
    const int p = g / 2 + 1;
    return ((g & 1) ? P1 - p : p) + P1 * k2;
}
// line of a workgroup of xb / xbi: pair pi = 0 holds the self-mirrored lines
// k1 = 0 and P1/2, pair pi > 0 the lines pi and P1 - pi
__device__ __forceinline__ int fs_pair_line(int P1, int pi, int which) {
    return pi == 0 ? (which ? P1 / 2 : 0) : (which ? P1 - pi : pi);
}

// xa: row pair r of u (ny rows of nx values) as the complex line
// u[2r] + i u[2r+1], zero-padded (ODD: the odd extensions of the rows);
// P1-point transforms over n1 for the workgroup's kFsLines values of n2, times
// W_P^(n2 k1), to line r of Lb at P2 k1 + n2
template <typename T, int P1, int P2, bool ODD>
__global__ __launch_bounds__(fs_threads<P1>()) void k_fs_xa(
    const T *__restrict__ u, C2<T> *__restrict__ Lb, int nx, int ny, const C2<T> *__restrict__ tw,
    const C2<T> *__restrict__ subtw, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PN = typename FsPlan<P1>::PN;
    constexpr int E = PN::E, L = PN::L, NL = kFsLines, R0 = PN::R[0], P = P1 * P2;
    __shared__ C2<T> lds[NL * padded_len<P1>()];
    const int c = threadIdx.x % NL, tl = threadIdx.x / NL;
    const int n2 = blockIdx.x * NL + c;
    const long r = blockIdx.y;
    const bool hb = 2 * r + 1 < ny;
    const T *ua = u + 2 * r * nx, *ub = u + (hb ? 2 * r + 1 : 2 * r) * nx;
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int p = P2 * in_pos<P1, PN, 0>(tl, j) + n2;
        if constexpr (!ODD) {
            // n1 >= P1/2 (p >= P/2 >= nx) is the zero padding: known per slot
            if ((j % R0) < R0 / 2) {
                const bool ok = p < nx;
                const T a = ua[ok ? p : 0], b = ub[ok ? p : 0];
                v[j] = mk<T>(ok ? a : T(0), (ok && hb) ? b : T(0));
            } else {
                v[j] = mk<T>(T(0), T(0));
            }
        } else {
            // x[p] for p < nx, -x[P - 2 - p] where P - 2 - p < nx, zero elsewhere
            const int q = P - 2 - p;
            const bool lo = p < nx, hi = q >= 0 && q < nx;
            const int s = lo ? p : (hi ? q : 0);
            const T a = ua[s], b = ub[s];
            const T sg = lo ? T(1) : (hi ? T(-1) : T(0));
            v[j] = mk<T>(sg * a, hb ? sg * b : T(0));
        }
    }
    C2<T> tws[num_tw<PN>()];
    load_twiddles<T, P1, PN>(tws, subtw + fs_tw_off(P1), tl);
    auto lidx = [c](int pos) { return padpos(pos) * NL + c; };
    fwd_stages<T, P1, PN, 0>(v, lds, tl, tws, lidx);
    C2<T> *dst = Lb + r * P + n2;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int k1 = out_pos<P1, PN, L - 1>(tl, j);
        st_stream(dst + P2 * k1, cmul<T>(v[j], tw[n2 * k1]));
    }
}

// xb: P2-point transforms over the contiguous n2 of lines k1 (pairs k1, P1 - k1
// in one workgroup), then the half spectra of rows 2r and 2r + 1:
// X_a = (Z(k) + conj Z(-k)) / 2, X_b = (Z(k) - conj Z(-k)) / (2i), k <= P/2,
// to columns fs_col of S (row stride Qs)
template <typename T, int P1, int P2>
__global__ __launch_bounds__(fs_threads<P2>()) void k_fs_xb(
    const C2<T> *__restrict__ Lb, C2<T> *__restrict__ S, int ny, int Qs, const C2<T> *__restrict__ subtw,
    const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PN = typename FsPlan<P2>::PN;
    constexpr int E = PN::E, TL = P2 / E, L = PN::L, NL = kFsLines, H = NL / 2, PLL = padded_len<P2>();
    constexpr int P = P1 * P2;
    __shared__ C2<T> lds[NL * PLL];
    const int tl = threadIdx.x % TL, c = threadIdx.x / TL;
    const int pi = blockIdx.x * H + c % H;
    const int k1 = fs_pair_line(P1, pi, c / H);
    const long r = blockIdx.y;
    const C2<T> *src = Lb + r * P + P2 * k1;
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = src[in_pos<P2, PN, 0>(tl, j)];
    C2<T> tws[num_tw<PN>()];
    load_twiddles<T, P2, PN>(tws, subtw + fs_tw_off(P2), tl);
    auto lidx = [c](int pos) { return c * PLL + padpos(pos); };
    fwd_stages<T, P2, PN, 0>(v, lds, tl, tws, lidx);
    // the forward stages end with their LDS reads behind a barrier
#pragma unroll
    for (int j = 0; j < E; ++j) lds[lidx(out_pos<P2, PN, L - 1>(tl, j))] = v[j];
    __syncthreads();
    const int cm = pi == 0 ? c : (c + H) % NL;  // the line holding Z(-k)
    const int cnt = k1 == 0 ? P2 / 2 + 1 : P2 / 2;
    const bool hb = 2 * r + 1 < ny;
    C2<T> *sa = S + 2 * r * Qs, *sb = S + (2 * r + 1) * Qs;
    for (int k2 = tl; k2 < cnt; k2 += TL) {
        const int m2 = k1 == 0 ? (P2 - k2) & (P2 - 1) : P2 - 1 - k2;
        const C2<T> zk = lds[lidx(k2)];
        const C2<T> zq = lds[cm * PLL + padpos(m2)];  // Z(-k) = zq; conj Z(-k) = (zq.x, -zq.y)
        const int col = fs_col(P1, P2, k1, k2);
        // plain stores: a line's threads write TL consecutive columns per
        // step, and the L2 merges the steps' runs before they reach HBM (measured
        // 1.5x faster here than streaming stores)
        sa[col] = mk<T>(T(0.5) * (zk.x + zq.x), T(0.5) * (zk.y - zq.y));
        if (hb) sb[col] = mk<T>(T(0.5) * (zk.y + zq.y), T(-0.5) * (zk.x - zq.x));
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
    auto lidx = [c](int pos) { return padpos(pos) * NL + c; };
    fwd_stages<T, P1, PN, 0>(v, lds, tl, tws, lidx);
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int k1 = out_pos<P1, PN, L - 1>(tl, j);
        st_stream(Tb + (long)(P2 * k1 + n2) * Qs + col, cmul<T>(v[j], tw[n2 * k1]));
    }
}

// ymid: for one k1 and kFsLines adjacent columns, y step 2 over rows
// P2 k1 + n2 (P2-point), lambda at ky = k1 + P1 k2 (row fold(ky) of lam,
// columns in fs_col order, row stride Q), and the inverse of y step 2, in place
template <typename T, int P1, int P2>
__global__ __launch_bounds__(fs_threads<P2>()) void k_fs_ymid(
    C2<T> *__restrict__ Tb, int Q, int Qs, const T *__restrict__ lam, const C2<T> *__restrict__ subtw,
    const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PN = typename FsPlan<P2>::PN;
    constexpr int E = PN::E, L = PN::L, NL = kFsLines, P = P1 * P2;
    __shared__ C2<T> lds[NL * padded_len<P2>()];
    const int c = threadIdx.x % NL, tl = threadIdx.x / NL;
    const int col = blockIdx.x * NL + c;
    const int k1 = blockIdx.y;
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
    auto lidx = [c](int pos) { return padpos(pos) * NL + c; };
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
    auto lidx = [c](int pos) { return padpos(pos) * NL + c; };
    adj_stages<T, P1, PN, L - 1>(v, lds, tl, tws, lidx);
#pragma unroll
    for (int j = 0; j < E; ++j) {
        if ((j % R0) < R0 / 2) {  // n1 >= P1/2 lies past every kept row
            const int p = P2 * in_pos<P1, PN, 0>(tl, j) + n2;
            if (p < ny) st_stream(S + (long)p * Qs + col, v[j]);
        }
    }
}

// xbi: the full spectrum Z(k) = X_a(k) + i X_b(k) of lines k1 (pairs k1, P1 - k1
// in one workgroup) from the half spectra of rows 2r and 2r + 1 (k > P/2 from
// the mirror: Z(k) = conj X_a(P - k) + i conj X_b(P - k)), inverse P2-point
// transforms over k2, times W_P^(-n2 k1), to line r of Lb at P2 k1 + n2
template <typename T, int P1, int P2>
__global__ __launch_bounds__(fs_threads<P2>()) void k_fs_xbi(
    const C2<T> *__restrict__ S, C2<T> *__restrict__ Lb, int ny, int Qs, const C2<T> *__restrict__ tw,
    const C2<T> *__restrict__ subtw, const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PN = typename FsPlan<P2>::PN;
    constexpr int E = PN::E, TL = P2 / E, L = PN::L, NL = kFsLines, H = NL / 2, PLL = padded_len<P2>();
    constexpr int P = P1 * P2;
    __shared__ C2<T> lds[NL * PLL];
    const int tl = threadIdx.x % TL, c = threadIdx.x / TL;
    const int pi = blockIdx.x * H + c % H;
    const int k1 = fs_pair_line(P1, pi, c / H);
    const long r = blockIdx.y;
    const bool hb = 2 * r + 1 < ny;
    const C2<T> *sa = S + 2 * r * Qs, *sb = S + (hb ? 2 * r + 1 : 2 * r) * Qs;
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int k2 = out_pos<P2, PN, L - 1>(tl, j);
        const bool dir = k1 == 0 ? k2 <= P2 / 2 : k2 < P2 / 2;
        const int m1 = dir ? k1 : (P1 - k1) & (P1 - 1);
        const int m2 = dir ? k2 : (k1 == 0 ? P2 - k2 : P2 - 1 - k2);
        const int col = fs_col(P1, P2, m1, m2);
        const C2<T> A = sa[col];
        const C2<T> B = keep<T>(hb, sb[col]);
        v[j] = dir ? mk<T>(A.x - B.y, A.y + B.x) : mk<T>(A.x + B.y, B.x - A.y);
    }
    C2<T> tws[num_tw<PN>()];
    load_twiddles<T, P2, PN>(tws, subtw + fs_tw_off(P2), tl);
    auto lidx = [c](int pos) { return c * PLL + padpos(pos); };
    adj_stages<T, P2, PN, L - 1>(v, lds, tl, tws, lidx);
    C2<T> *dst = Lb + r * P + P2 * k1;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int n2 = in_pos<P2, PN, 0>(tl, j);
        st_stream(dst + n2, cmul<T>(v[j], cconj<T>(tw[n2 * k1])));
    }
}

// xai: inverse P1-point transforms over k1 of line r (kFsLines values of n2),
// positions P2 n1 + n2 < nx unpacked to rows 2r (real part) and 2r + 1
// (imaginary part) of y, with the solver epilogue y = a1 w1 + a2 w2 + scale (A u)
template <typename T, int P1, int P2, bool EPI>
__global__ __launch_bounds__(fs_threads<P1>()) void k_fs_xai(
    const C2<T> *__restrict__ Lb, T *__restrict__ y, int nx, int ny, const C2<T> *__restrict__ subtw, Epi<T> ep,
    const double *__restrict__ done) {
    if (done && *done != 0.0) return;
    using PN = typename FsPlan<P1>::PN;
    constexpr int E = PN::E, L = PN::L, NL = kFsLines, R0 = PN::R[0], P = P1 * P2;
    __shared__ C2<T> lds[NL * padded_len<P1>()];
    const int c = threadIdx.x % NL, tl = threadIdx.x / NL;
    const int n2 = blockIdx.x * NL + c;
    const long r = blockIdx.y;
    const C2<T> *src = Lb + r * P + n2;
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = src[P2 * out_pos<P1, PN, L - 1>(tl, j)];
    C2<T> tws[num_tw<PN>()];
    load_twiddles<T, P1, PN>(tws, subtw + fs_tw_off(P1), tl);
    auto lidx = [c](int pos) { return padpos(pos) * NL + c; };
    adj_stages<T, P1, PN, L - 1>(v, lds, tl, tws, lidx);
    const bool hb = 2 * r + 1 < ny;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        if ((j % R0) < R0 / 2) {  // n1 >= P1/2 lies past nx
            const int p = P2 * in_pos<P1, PN, 0>(tl, j) + n2;
            if (p < nx) {
                const long ia = 2 * r * nx + p, ib = ia + nx;
                T a = v[j].x, b = v[j].y;
                if constexpr (EPI) {
                    a *= ep.scale;
                    b *= ep.scale;
                    if (ep.w1) {
                        a += ep.a1 * ep.w1[ia];
                        if (hb) b += ep.a1 * ep.w1[ib];
                    }
                    if (ep.w2) {
                        a += ep.a2 * ep.w2[ia];
                        if (hb) b += ep.a2 * ep.w2[ib];
                    }
                }
                y[ia] = a;
                if (hb) y[ib] = b;
            }
        }
    }
}

// lambda (and the preconditioner's symbol) of a large operator in the fs_col
// column order: out[ky * Q + col] = f(lam64[ky * Q + fs_kx(col)]) for ky, col < Q
template <typename T>
__global__ void k_fs_permute(const double *__restrict__ lam64, T *__restrict__ out, int Q, int P1, int P2, SymMap m) {
    const long total = (long)Q * Q;
    const int N2 = Q - 1;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        const int ky = (int)(idx / Q), col = (int)(idx - (long)ky * Q);
        const int kx = fs_kx(P1, P2, col);
        out[idx] = (T)sym_at(lam64, (long)ky * Q + kx, kx, ky, 0, 2, N2, m);
    }
}

inline void fs_split(int P, int &P1, int &P2) {
    P2 = P >= 8192 ? 128 : 64;
    P1 = P / P2;
}

template <typename T, int P1, int P2>
static fl_status fs_matvec(fl_op op, const T *u, T *y, const Epi<T> &ep, const double *done, hipStream_t s,
                      const T *lam, bool odd, const C2<T> *tw, const C2<T> *subtw) {
    const int Q = op->Q, Qs = op->Qp, nx = op->nk[0], ny = op->nk[1], P = P1 * P2;
    static_assert(P1 % kFsLines == 0 && P2 % kFsLines == 0, "whole workgroups of lines");
    if (Qs % kFsLines != 0 || Qs < Q) {  // the row stride covers whole column groups (set at creation)
        set_error("row stride %d of the large-operator spectra is not a multiple of %d", Qs, kFsLines);
        return FL_E_UNSUPPORTED;
    }
    const int nl = (ny + 1) / 2;
    C2<T> *Tb = (C2<T> *)op->T1;
    C2<T> *Lb = (C2<T> *)op->T2;
    C2<T> *S = Lb + (long)nl * P;  // nl P + ny Qs <= P Qs complex values
    const dim3 b1(fs_threads<P1>()), b2(fs_threads<P2>());
    if (odd)
        hipLaunchKernelGGL((k_fs_xa<T, P1, P2, true>), dim3(P2 / kFsLines, nl), b1, 0, s, u, Lb, nx, ny, tw, subtw,
                           done);
    else
        hipLaunchKernelGGL((k_fs_xa<T, P1, P2, false>), dim3(P2 / kFsLines, nl), b1, 0, s, u, Lb, nx, ny, tw, subtw,
                           done);
    hipLaunchKernelGGL((k_fs_xb<T, P1, P2>), dim3(P1 / kFsLines, nl), b2, 0, s, Lb, S, ny, Qs, subtw, done);
    if (odd)
        hipLaunchKernelGGL((k_fs_ya<T, P1, P2, true>), dim3(Qs / kFsLines, P2), b1, 0, s, S, Tb, ny, Qs, tw, subtw,
                           done);
    else
        hipLaunchKernelGGL((k_fs_ya<T, P1, P2, false>), dim3(Qs / kFsLines, P2), b1, 0, s, S, Tb, ny, Qs, tw, subtw,
                           done);
    hipLaunchKernelGGL((k_fs_ymid<T, P1, P2>), dim3(Qs / kFsLines, P1), b2, 0, s, Tb, Q, Qs, lam, subtw, done);
    hipLaunchKernelGGL((k_fs_yai<T, P1, P2>), dim3(Qs / kFsLines, P2), b1, 0, s, Tb, S, ny, Qs, tw, subtw, done);
    hipLaunchKernelGGL((k_fs_xbi<T, P1, P2>), dim3(P1 / kFsLines, nl), b2, 0, s, S, Lb, ny, Qs, tw, subtw, done);
    if (ep.active())
        hipLaunchKernelGGL((k_fs_xai<T, P1, P2, true>), dim3(P2 / kFsLines, nl), b1, 0, s, Lb, y, nx, ny, subtw, ep,
                           done);
    else
        hipLaunchKernelGGL((k_fs_xai<T, P1, P2, false>), dim3(P2 / kFsLines, nl), b1, 0, s, Lb, y, nx, ny, subtw,
                           ep, done);
    return FL_OK;
}
