// fl_wave2d.hpp -- the 2D matvec passes with one wavefront per FFT line
// (included by fl_fft.hip; same spectra layout, lambda tiles, epilogue, done
// flags and batch strides as the workgroup-per-tile kernels there).
//
// Every FFT here belongs to one wavefront: lane tl (0..63) holds E = L/64
// points of a line of length L, and the Stockham stages exchange values
// through the wavefront's own LDS region.  A wavefront's LDS instructions
// complete in order, so an exchange needs only a wait for its own writes,
// never a workgroup barrier; workgroup barriers remain only around the
// cooperative, fully coalesced global loads and stores of a tile.
//
//   X forward  (k_w2_xfwd): one real row per wavefront, four rows per
//     workgroup.  The row (zero-padded to P) is transformed as the complex
//     sequence z[m] = x[2m] + i x[2m+1] of length P/2, then split into its
//     half spectrum X[k] = (Z[k] + conj Z[-k])/2 - (i/2) w^k (Z[k] - conj Z[-k]),
//     w = exp(-2 pi i / P), k = 0..P/2.  The four rows of a tile chunk are
//     stored as one contiguous run.
//   Y fused    (k_w2_yfused): one spectral column per wavefront, the C columns
//     of a tile per workgroup: forward FFT of length P, times lambda, inverse,
//     crop.
//   X inverse  (k_w2_xinv): one row per wavefront: Z[k] = (X[k] + conj X[P/2-k])
//     + i w^-k (X[k] - conj X[P/2-k]) and the inverse FFT of length P/2 give
//     z[m] = y[2m] + i y[2m+1]; the solver epilogue follows.
#pragma once

// (this file is included inside namespace fl)

// Order a wavefront's LDS writes before its following LDS reads (and reads
// before later writes): the compiler may not move LDS accesses across this
// point, and the wait makes the wavefront's own writes complete first.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// LDS position of line entry pos: one pad slot per RP entries, RP the first
// radix, which makes the first stage's stride-RP writes conflict-free
template <int RP> __device__ __forceinline__ int wpad(int pos) { return pos + pos / RP; }
template <int L, int RP> constexpr int wpad_len() { return L + L / RP; }

// twiddles of a length-L plan read from the length-P table exp(-2 pi i m / P)
// (entry m * P / L is exp(-2 pi i m / L))
template <typename T, int L, typename PL, int TS, int S = 1>
__device__ __forceinline__ void wave_twiddles(C2<T> *tws, const C2<T> *__restrict__ table, int tl) {
    if constexpr (S < PL::L) {
        constexpr int R = PL::R[S], E = PL::E, TL = L / E, Ns = stage_ns<PL>(S), TW = stage_tw<PL>(S);
#pragma unroll
        for (int i = 0; i < E / R; ++i) {
            const int k = (tl + i * TL) % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) tws[TW + i * (R - 1) + r - 1] = table[k * r * (L / (Ns * R)) * TS];
        }
        wave_twiddles<T, L, PL, TS, S + 1>(tws, table, tl);
    }
}

// The Stockham positions of a wavefront's line (TL = 64 lanes, first radix
// R0 = E) split into a lane part and a slot part, pos = a(tl) + b(j), such that
// the padded LDS index is wpad(a) + b + b / E: the slot part becomes an
// immediate offset of the LDS instruction.  (b is a multiple of E, or b < E
// with a a multiple of E; wave_pos_ok checks every (tl, j) at compile time.)
template <int L, typename PL, int S> struct WPos {
    static constexpr int R = PL::R[S], E = PL::E, TL = L / E, Ns = stage_ns<PL>(S);
    static constexpr int in_a(int tl) { return tl; }
    static constexpr int in_b(int j) { return (j / R) * TL + (j % R) * (L / R); }
    static constexpr int out_a(int tl) { return Ns >= TL ? tl : (tl / Ns) * Ns * R + tl % Ns; }
    static constexpr int out_b(int j) {
        return Ns >= TL ? ((j / R) * TL / Ns) * Ns * R + ((j / R) * TL) % Ns + (j % R) * Ns
                        : (j / R) * TL * R + (j % R) * Ns;
    }
    // the reference index maps (the workgroup kernels' in_pos / out_pos)
    static constexpr int in_ref(int tl, int j) { return tl + (j / R) * TL + (j % R) * (L / R); }
    static constexpr int out_ref(int tl, int j) {
        const int b = tl + (j / R) * TL;
        return (b / Ns) * Ns * R + (b % Ns) + (j % R) * Ns;
    }
};
template <int E> constexpr int wpad_c(int pos) { return pos + pos / E; }
template <int L, typename PL, int S> constexpr bool wave_pos_ok() {
    using W = WPos<L, PL, S>;
    constexpr int E = PL::E;
    for (int tl = 0; tl < W::TL; ++tl)
        for (int j = 0; j < E; ++j) {
            if (W::in_a(tl) + W::in_b(j) != W::in_ref(tl, j)) return false;
            if (W::out_a(tl) + W::out_b(j) != W::out_ref(tl, j)) return false;
            if (wpad_c<E>(W::in_ref(tl, j)) != wpad_c<E>(W::in_a(tl)) + W::in_b(j) + W::in_b(j) / E) return false;
            if (wpad_c<E>(W::out_ref(tl, j)) != wpad_c<E>(W::out_a(tl)) + W::out_b(j) + W::out_b(j) / E)
                return false;
        }
    return true;
}

// forward stages S.. of a wavefront's line in its LDS region `lds` (padded by
// one slot per E entries): v enters at in_pos<S>, leaves at out_pos<last>
template <typename T, int L, typename PL, int S>
__device__ __forceinline__ void wave_fwd(C2<T> *v, C2<T> *lds, int tl, const C2<T> *tws) {
    fwd_bfly<T, PL, S>(v, tws);
    if constexpr (S + 1 < PL::L) {
        constexpr int E = PL::E;
        using WO = WPos<L, PL, S>;
        using WI = WPos<L, PL, S + 1>;
        static_assert(wave_pos_ok<L, PL, S>() && wave_pos_ok<L, PL, S + 1>(), "position split");
        C2<T> *wo = lds + wpad_c<E>(WO::out_a(tl));
#pragma unroll
        for (int j = 0; j < E; ++j) wo[WO::out_b(j) + WO::out_b(j) / E] = v[j];
        wave_lds_sync();
        const C2<T> *wi = lds + wpad_c<E>(WI::in_a(tl));
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = wi[WI::in_b(j) + WI::in_b(j) / E];
        wave_lds_sync();
        wave_fwd<T, L, PL, S + 1>(v, lds, tl, tws);
    }
}
// adjoint stages S..0 (the unnormalised inverse): v enters at out_pos<S>, leaves at in_pos<0>
template <typename T, int L, typename PL, int S>
__device__ __forceinline__ void wave_adj(C2<T> *v, C2<T> *lds, int tl, const C2<T> *tws) {
    adj_bfly<T, PL, S>(v, tws);
    if constexpr (S > 0) {
        constexpr int E = PL::E;
        using WI = WPos<L, PL, S>;
        using WO = WPos<L, PL, S - 1>;
        static_assert(wave_pos_ok<L, PL, S>() && wave_pos_ok<L, PL, S - 1>(), "position split");
        C2<T> *wi = lds + wpad_c<E>(WI::in_a(tl));
#pragma unroll
        for (int j = 0; j < E; ++j) wi[WI::in_b(j) + WI::in_b(j) / E] = v[j];
        wave_lds_sync();
        const C2<T> *wo = lds + wpad_c<E>(WO::out_a(tl));
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = wo[WO::out_b(j) + WO::out_b(j) / E];
        wave_lds_sync();
        wave_adj<T, L, PL, S - 1>(v, lds, tl, tws);
    }
}
// v[j] <- region[pos] or region[pos] = v[j] at the positions in_pos<0> / out_pos<last>
template <typename T, int L, typename PL>
__device__ __forceinline__ const C2<T> *wave_in0(const C2<T> *lds, int tl) {
    return lds + wpad_c<PL::E>(WPos<L, PL, 0>::in_a(tl));
}
template <typename T, int L, typename PL>
__device__ __forceinline__ C2<T> *wave_outl(C2<T> *lds, int tl) {
    return lds + wpad_c<PL::E>(WPos<L, PL, PL::L - 1>::out_a(tl));
}
template <int L, typename PL> constexpr int wave_in0_off(int j) {
    return WPos<L, PL, 0>::in_b(j) + WPos<L, PL, 0>::in_b(j) / PL::E;
}
template <int L, typename PL> constexpr int wave_outl_off(int j) {
    return WPos<L, PL, PL::L - 1>::out_b(j) + WPos<L, PL, PL::L - 1>::out_b(j) / PL::E;
}

// a pair of consecutive complex values: 16 bytes in FP32 (one dwordx4 access);
// an FP64 value is already 16 bytes
template <typename T> struct Pair2 {
    C2<T> a, b;
};

__device__ __forceinline__ void st_stream(Pair2<float> *p, Pair2<float> v) {
    fvec4 t = {v.a.x, v.a.y, v.b.x, v.b.y};
    __builtin_nontemporal_store(t, (fvec4 *)p);
}

// 4-byte-aligned float2: rows of odd length start at odd float offsets
typedef float float2_a4 __attribute__((ext_vector_type(2), aligned(4)));

// ---------------------------------------------------------------------------
// X forward: rows r = 4 * block + wave of u (row pitch in_pitch, n_in values,
// or with n_in < 0 the odd extension of -n_in values), half spectra written
// tiled (ntiles tiles of C columns, nj rows per slab), DC and Nyquist packed in
// column 0.  256 threads.
// ---------------------------------------------------------------------------
template <typename T, int P, int C>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1))) void k_w2_xfwd(
    const T *__restrict__ u, C2<T> *__restrict__ out, int nrows, int n_in, long in_pitch, int nj, int ntiles,
    const C2<T> *__restrict__ table, const double *__restrict__ done, BatchStrides bz) {
    const int z = blockIdx.z;
    if (done && done[z * bz.done] != 0.0) return;
    u += z * bz.in;
    out += z * bz.out;
    constexpr int L = P / 2, E = L / 64, RP = E;
    using PN = Plan<L, E>;
    constexpr int LL = wpad_len<L, RP>();
    __shared__ C2<T> lds[4 * LL];
    const int w = threadIdx.x >> 6, tl = threadIdx.x & 63;
    const int bx = xcd_block(blockIdx.x, gridDim.x);
    const int row = 4 * bx + w;
    const bool rv = row < nrows;
    C2<T> *wl = lds + w * LL;
    C2<T> tws[num_tw<PN>()];
    wave_twiddles<T, L, PN, 2>(tws, table, tl);
    // the split's twiddles w^k for the columns this thread stores (fetched early)
    constexpr int CPT = sizeof(T) == 4 ? 2 : 1;  // columns per thread
    constexpr int SLOTS = 4 * C / CPT;             // threads per tile chunk
    constexpr int TPS = 256 / SLOTS;               // tiles per sweep
    constexpr int NT = L / C;                      // tiles (the P/2 packed columns)
    static_assert(NT % TPS == 0, "whole sweeps");
    const int slot = threadIdx.x % SLOTS, tsub = threadIdx.x / SLOTS;
    const int rr = slot / (C / CPT), c0 = (slot % (C / CPT)) * CPT;
    C2<T> wsp[NT / TPS][CPT];
#pragma unroll
    for (int it = 0; it < NT / TPS; ++it)
#pragma unroll
        for (int q = 0; q < CPT; ++q) wsp[it][q] = table[(tsub + it * TPS) * C + c0 + q];
    C2<T> v[E];
    const T *ur = u + (long)(rv ? row : 0) * in_pitch;
    if (n_in >= 0) {
        // z[m] = x[2m] + i x[2m+1], zero at and past n_in
        const int nc = (n_in + 1) / 2;  // complex entries with a nonzero part
        load_line<T, L, PN>(v, tl, nc <= L / 2 ? nc : L, [&](int m) {
            C2<T> x;
            if constexpr (sizeof(T) == 4) {
                if (2 * m + 1 < n_in) {
                    const float2_a4 t = *(const float2_a4 *)(ur + 2 * m);
                    x = mk<T>(t.x, t.y);
                } else {
                    x = mk<T>(ur[2 * m], T(0));
                }
            } else {
                x = mk<T>(ur[2 * m], 2 * m + 1 < n_in ? ur[2 * m + 1] : T(0));
            }
            return keep<T>(rv, x);
        });
    } else {
        // odd extension e[p] about -1 of n = -n_in values: x[p] for p < n,
        // -x[P-2-p] where P-2-p < n, zero elsewhere; z[m] = e[2m] + i e[2m+1]
        const int n = -n_in;
        auto e = [&](int p) {
            const int q = P - 2 - p;
            const bool lo = p < n, hi = q >= 0 && q < n;
            const T x = ur[lo ? p : (hi ? q : 0)];
            return (rv && lo) ? x : ((rv && hi) ? -x : T(0));
        };
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int m = in_pos<L, PN, 0>(tl, j);
            v[j] = mk<T>(e(2 * m), e(2 * m + 1));
        }
    }
    // FFT of length L in the wavefront's region, then Z in natural order (padded)
    wave_fwd<T, L, PN, 0>(v, wl, tl, tws);
    {
        C2<T> *wo = wave_outl<T, L, PN>(wl, tl);
#pragma unroll
        for (int j = 0; j < E; ++j) wo[wave_outl_off<L, PN>(j)] = v[j];
    }
    __syncthreads();
    // split and store: per tile, the 4 rows x C columns are one contiguous run;
    // a thread takes two consecutive columns (16 bytes in FP32) or one (FP64)
    const int srow = 4 * bx + rr;
    if (srow >= nrows) return;
    const C2<T> *zl = lds + rr * LL;
    auto zat = [&](int k) { return zl[wpad<RP>(k)]; };
    C2<T> *orow = out + tiled_rowbase(srow, nj, ntiles, C) + c0;
    const int tstride = nj * C;
    const T half = T(0.5);
    (void)ntiles;
#pragma unroll
    for (int it = 0; it < NT / TPS; ++it) {
        const int t = tsub + it * TPS;
        C2<T> o[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int k = t * C + c0 + q;
            const C2<T> zk = zat(k), zm = zat(L - k);  // Z[-k] = Z[L-k]
            if (k == 0) {
                // X_0 = Re Z0 + Im Z0, X_{P/2} = Re Z0 - Im Z0 (both real), packed
                o[q] = mk<T>(zk.x + zk.y, zk.x - zk.y);
            } else {
                // a = (Z[k] + conj Z[-k]) / 2, b = (Z[k] - conj Z[-k]) / 2; X = a - i w^k b
                const C2<T> a = mk<T>(half * (zk.x + zm.x), half * (zk.y - zm.y));
                const C2<T> b = mk<T>(half * (zk.x - zm.x), half * (zk.y + zm.y));
                const C2<T> wb = cmul<T>(wsp[it][q], b);
                o[q] = mk<T>(a.x + wb.y, a.y - wb.x);
            }
        }
        if constexpr (CPT == 2) {
            st_stream((Pair2<T> *)(orow + t * tstride), Pair2<T>{o[0], o[1]});
        } else {
            st_stream(orow + t * tstride, o[0]);
        }
    }
}

// ---------------------------------------------------------------------------
// Y fused: tile t (columns t*C .. t*C+C-1, one per wavefront) of the tiled half
// spectra, in place: n_in rows read (n_in < 0: the odd extension of -n_in),
// forward FFT of length P, times lambda (tiled), inverse, n_out rows written.
// PACK: column 0 of tile 0 holds the packed DC / Nyquist columns.
// ---------------------------------------------------------------------------
template <typename T, int P, int C, bool PACK>
__global__ __launch_bounds__(64 * C) __attribute__((amdgpu_waves_per_eu(1))) void k_w2_yfused(
    C2<T> *buf, int n_in, int n_out, int nj, const C2<T> *__restrict__ table, const T *__restrict__ lam,
    int lam_tile, int lam_pack, const double *__restrict__ done, BatchStrides bz) {
    const int zb = blockIdx.z;
    if (done && done[zb * bz.done] != 0.0) return;
    buf += zb * bz.in;
    lam += zb * bz.lam;
    constexpr int E = P / 64, RP = E;
    using PN = Plan<P, E>;
    constexpr int L = PN::L;
    constexpr int LL = wpad_len<P, RP>();
    __shared__ C2<T> lds[C * LL];
    const int c = threadIdx.x >> 6, tl = threadIdx.x & 63;
    const int t = blockIdx.x;
    C2<T> *tile = buf + (long)t * nj * C;
    C2<T> *wl = lds + c * LL;
    auto li = [](int pos) { return wpad<RP>(pos); };
    // the tile's rows (nj x C contiguous) into the column regions, coalesced
    const int nrd = n_in >= 0 ? n_in : -n_in;  // stored rows the loads need
    constexpr int CPT = sizeof(T) == 4 ? 2 : 1;
    constexpr int SPR = C / CPT;  // threads per row
    constexpr int NIT = (P / 2 * SPR) / (64 * C);  // sweeps for up to P/2 rows
    static_assert((P / 2 * SPR) % (64 * C) == 0, "whole sweeps");
    {
        Pair2<T> xs[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = threadIdx.x + it * 64 * C;
            const int j = i / SPR, c0 = (i % SPR) * CPT;
            const long off = (long)(j < nrd ? j : 0) * C + c0;
            if constexpr (CPT == 2) xs[it] = *(const Pair2<T> *)(tile + off);
            else xs[it].a = tile[off];
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int i = threadIdx.x + it * 64 * C;
            const int j = i / SPR, c0 = (i % SPR) * CPT;
            if (j < nrd) {
                lds[c0 * LL + li(j)] = xs[it].a;
                if constexpr (CPT == 2) lds[(c0 + 1) * LL + li(j)] = xs[it].b;
            }
        }
    }
    C2<T> tws[num_tw<PN>()];
    wave_twiddles<T, P, PN, 1>(tws, table, tl);
    // lambda at this lane's spectral positions
    T lv[E], ldv[E];
    const T *lo = lam + (t * lam_tile + c);
#pragma unroll
    for (int j = 0; j < E; ++j) lv[j] = lo[fold<P>(out_pos<P, PN, L - 1>(tl, j)) * C];
    if (PACK && t == 0 && c == 0) {  // the packed column's second symbol, fetched early
#pragma unroll
        for (int j = 0; j < E; ++j) ldv[j] = lam[lam_pack + fold<P>(out_pos<P, PN, L - 1>(tl, j))];
    }
    __syncthreads();
    C2<T> v[E];
    load_line<T, P, PN>(v, tl, n_in, [&](int i) { return wl[li(i)]; });
    wave_lds_sync();
    wave_fwd<T, P, PN, 0>(v, wl, tl, tws);
    if (PACK && t == 0 && c == 0) {  // wavefront-uniform: the packed DC / Nyquist column
#pragma unroll
        for (int j = 0; j < E; ++j) wl[li(out_pos<P, PN, L - 1>(tl, j))] = v[j];
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = out_pos<P, PN, L - 1>(tl, j);
            const C2<T> zm = wl[li((P - pos) & (P - 1))];
            v[j] = mk<T>(lv[j] * v[j].x + ldv[j] * zm.x, lv[j] * v[j].y - ldv[j] * zm.y);
        }
        wave_lds_sync();
    } else {
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = cscale<T>(v[j], lv[j]);
    }
    wave_adj<T, P, PN, L - 1>(v, wl, tl, tws);
    // results into the column region, then the tile's rows out, coalesced
    {
        C2<T> *wo = (C2<T> *)wave_in0<T, P, PN>(wl, tl);
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int pos = in_pos<P, PN, 0>(tl, j);
            if (pos < n_out) wo[wave_in0_off<P, PN>(j)] = v[j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int i = threadIdx.x + it * 64 * C;
        const int j = i / SPR, c0 = (i % SPR) * CPT;
        if (j < n_out) {
            if constexpr (CPT == 2) {
                st_stream((Pair2<T> *)(tile + (long)j * C + c0),
                          Pair2<T>{lds[c0 * LL + li(j)], lds[(c0 + 1) * LL + li(j)]});
            } else {
                st_stream(tile + (long)j * C + c0, lds[c0 * LL + li(j)]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// X inverse: rows r = 4 * block + wave; the half spectra (tiled, DC/Nyquist
// packed) of the block's four rows are read as contiguous runs, each row is
// inverted as a complex line of length P/2, and y = a1 w1 + a2 w2 + scale (A u)
// is written for the first n_out entries (row pitch out_pitch).  With dpart
// the block writes its sum (dotw, y) in FP64 to dpart[z * stride + block].
// ---------------------------------------------------------------------------
template <typename T, int P, int C, bool EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1))) void k_w2_xinv(
    const C2<T> *__restrict__ in, T *__restrict__ y, int nrows, int n_out, long out_pitch, int nj, int ntiles,
    const C2<T> *__restrict__ table, Epi<T> ep, const double *__restrict__ done, BatchStrides bz) {
    const int z = blockIdx.z;
    if (done && done[z * bz.done] != 0.0) return;
    in += z * bz.in;
    y += z * bz.out;
    if (ep.w1) ep.w1 += z * bz.out;
    if (ep.w2) ep.w2 += z * bz.out;
    if (ep.dotw) ep.dotw += z * bz.out;
    constexpr int L = P / 2, E = L / 64, RP = E;
    using PN = Plan<L, E>;
    constexpr int LX = L + 1;                           // X[0..L] per row, natural order
    constexpr int LL = wpad_len<L, RP>() > LX ? wpad_len<L, RP>() : LX;
    __shared__ C2<T> lds[4 * LL];
    const int w = threadIdx.x >> 6, tl = threadIdx.x & 63;
    const int bx = xcd_block(blockIdx.x, gridDim.x);
    C2<T> tws[num_tw<PN>()];
    wave_twiddles<T, L, PN, 2>(tws, table, tl);
    // w^k at this lane's first inverse positions (fetched early)
    C2<T> wz[E];
#pragma unroll
    for (int j = 0; j < E; ++j) wz[j] = table[out_pos<L, PN, PN::L - 1>(tl, j)];
    // the block's four rows of half spectra, tile by tile, into LDS (natural order)
    {
        constexpr int CPT = sizeof(T) == 4 ? 2 : 1;
        constexpr int SLOTS = 4 * C / CPT, TPS = 256 / SLOTS;
        const int slot = threadIdx.x % SLOTS, tsub = threadIdx.x / SLOTS;
        const int rr = slot / (C / CPT), c0 = (slot % (C / CPT)) * CPT;
        const int srow = 4 * bx + rr;
        const bool sv = srow < nrows;
        const C2<T> *irow = in + tiled_rowbase(sv ? srow : 0, nj, ntiles, C) + c0;
        C2<T> *xl = lds + rr * LL;
        const int tstride = nj * C;
        constexpr int NT = L / C, NIT = NT / TPS;
        static_assert(NT % TPS == 0, "whole sweeps");
        (void)ntiles;
        Pair2<T> xs[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int t = tsub + it * TPS;
            if constexpr (CPT == 2) xs[it] = *(const Pair2<T> *)(irow + t * tstride);
            else xs[it].a = irow[t * tstride];
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int t = tsub + it * TPS;
            const C2<T> xv[2] = {xs[it].a, xs[it].b};
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const int k = t * C + c0 + q;
                const C2<T> x = sv ? xv[q] : mk<T>(T(0), T(0));
                if (k == 0) {
                    xl[0] = mk<T>(x.x, T(0));
                    xl[L] = mk<T>(x.y, T(0));
                } else {
                    xl[k] = x;
                }
            }
        }
    }
    __syncthreads();
    const int row = 4 * bx + w;
    C2<T> *xl = lds + w * LL;
    // Z[k] = (X[k] + conj X[L-k]) + i w^-k (X[k] - conj X[L-k]) at this lane's
    // first inverse positions
    C2<T> v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int k = out_pos<L, PN, PN::L - 1>(tl, j);
        const C2<T> xk = xl[k], xm = xl[L - k];
        const C2<T> s = mk<T>(xk.x + xm.x, xk.y - xm.y);
        const C2<T> d = mk<T>(xk.x - xm.x, xk.y + xm.y);
        const C2<T> wd = cmul<T>(cconj<T>(wz[j]), d);  // w^-k d
        v[j] = mk<T>(s.x - wd.y, s.y + wd.x);
    }
    // the wavefront's region is reused for the exchanges once every lane has read
    wave_lds_sync();
    wave_adj<T, L, PN, PN::L - 1>(v, xl, tl, tws);
    double acc = 0.0;
    if (row < nrows) {
        T *yr = y + (long)row * out_pitch;
        const long rb = (long)row * out_pitch;
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int m = in_pos<L, PN, 0>(tl, j);
            T o[2] = {v[j].x, v[j].y};
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int p = 2 * m + q;
                if (p < n_out) {
                    T a = o[q];
                    if constexpr (EPI) {
                        a = ep.scale * a;
                        if (ep.w1) a += ep.a1 * ep.w1[rb + p];
                        if (ep.w2) a += ep.a2 * ep.w2[rb + p];
                        if (ep.dpart) acc += (double)a * (double)ep.dotw[rb + p];
                    }
                    o[q] = a;
                }
            }
            if constexpr (sizeof(T) == 4) {
                if (2 * m + 1 < n_out) {
                    st_stream(yr + 2 * m, o[0]);
                    st_stream(yr + 2 * m + 1, o[1]);
                } else if (2 * m < n_out) {
                    st_stream(yr + 2 * m, o[0]);
                }
            } else {
                if (2 * m < n_out) st_stream(yr + 2 * m, o[0]);
                if (2 * m + 1 < n_out) st_stream(yr + 2 * m + 1, o[1]);
            }
        }
    }
    if constexpr (EPI) {
        if (ep.dpart) {  // block-uniform
            __shared__ double wsum[4];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
            if (tl == 0) wsum[w] = acc;
            __syncthreads();
            if (threadIdx.x == 0) ep.dpart[z * ep.dpart_stride + bx] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
        }
    }
}
