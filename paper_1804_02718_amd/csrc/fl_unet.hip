// fl_unet.hip -- the learned preconditioner: a small convolutional U-Net with
// hand-written forward, backward and Adam kernels; the convolutions run as
// implicit GEMMs on bf16 MFMA (16x16x16) with FP32 accumulation.
//
// Network (all 3x3 convolutions bias-free, ReLU after every one but the last):
//   level 1 @ H x W:      2 -> 16 -> 16            (skip s1)
//   avg-pool 2x2, level 2 @ H/2: 16 -> 32 -> 32    (skip s2)
//   avg-pool 2x2, level 3 @ H/4: 32 -> 64 -> 64
//   nearest up x2, concat s2 (96), 96 -> 32 -> 32 @ H/2
//   nearest up x2, concat s1 (48), 48 -> 16 -> 16 @ H
//   1x1 convolution 16 -> 1
// Input channels: the normalised residual and a constant alpha channel.
// Activations are NHWC in FP32; GEMM operands are rounded to bf16.
//
// GEMM convention (every product below): C[m][n] = sum_k A[m][k] * B[n][k],
// A and B bf16 with k contiguous ("NT").  Forward conv: A = im2row(X)
// ([pixel][k], k = (ky*3 + kx)*Cin + ci), B = W ([cout][k]).  Backward data:
// A = dY ([pixel][cout]), B = W^T ([k][cout]), then a gather col2im.  Weight
// gradient: A = dY^T ([cout][pixel]), B = im2row(X)^T ([k][pixel]), split
// over pixels with a fixed-order reduction of the partial products.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <random>
#include <type_traits>
#include <vector>

#include "fl_internal.hpp"

namespace fl {

using bf16 = unsigned short;
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16 to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)(u >> 16);  // inf / nan kept
    u += 0x7fffu + ((u >> 16) & 1u);                               // round to nearest even
    return (bf16)(u >> 16);
}
__device__ __forceinline__ float from_bf16(bf16 b) { return __uint_as_float(((unsigned)b) << 16); }

// GEMM operand storage: bf16 (production) or fp32 (verification mode)
template <typename T> __device__ __forceinline__ T to_op(float f);
template <> __device__ __forceinline__ bf16 to_op<bf16>(float f) { return to_bf16(f); }
template <> __device__ __forceinline__ float to_op<float>(float f) { return f; }
template <typename T> __device__ __forceinline__ float op_to_f(T v);
template <> __device__ __forceinline__ float op_to_f<bf16>(bf16 v) { return from_bf16(v); }
template <> __device__ __forceinline__ float op_to_f<float>(float v) { return v; }

static inline int cdiv_i(long a, long b) { return (int)((a + b - 1) / b); }
static inline int grid1(long n) {
    long g = (n + 255) / 256;
    return (int)(g > 65535 ? 65535 : (g < 1 ? 1 : g));
}

// ---------------------------------------------------------------------------
// NT GEMM on MFMA.  Block 256 threads = 4 waves in a 2 x 2 arrangement, block
// tile 64 (m) x 64 (n), each wave 32 x 32 = 2 x 2 MFMA tiles of 16 x 16, k in
// steps of 16.  Lane l = 16 q + r loads A[m0 + r][k0 + 4q .. 4q + 3] and
// B[n0 + r][k0 + 4q .. 4q + 3].
//  bf16: one v_mfma_f32_16x16x16_bf16 per tile, whose operand layout is
//        exactly that (lane (r, q) supplies row r, k = 4q + i);
//  fp32: four v_mfma_f32_16x16x4_f32, the j-th taking element j of every
//        lane's 4-vector (lane (r, q) supplies row r, k = 4q + j), so the
//        four products together cover the 16 k of the step.
// Result layout of both: lane (r, q) holds D[4q + t][r], t = 0..3.
// M, N, K multiples of 16 (callers pad).  Split-K: blockIdx.z = split s takes
// k in [s*kchunk, (s+1)*kchunk) and, with PART, writes its partial product to
// C + s*M*ldc.  RELU applies max(0, .); ACC adds to C.
// ---------------------------------------------------------------------------
template <typename T, bool RELU, bool ACC, bool PART>
__global__ __launch_bounds__(256) void k_gemm_nt(const T *__restrict__ A, int lda, const T *__restrict__ B, int ldb,
                                                 float *__restrict__ C, int ldc, int M, int N, int K, int kchunk) {
    using V = typename std::conditional<sizeof(T) == 2, v4s, v4f>::type;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int n0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int kb = blockIdx.z * kchunk;
    const int ke = kb + kchunk < K ? kb + kchunk : K;
    const int r = lane & 15, q = lane >> 4;
    v4f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    const bool mv[2] = {m0 < M, m0 + 16 < M};
    const bool nv[2] = {n0 < N, n0 + 16 < N};
    if ((mv[0] || mv[1]) && (nv[0] || nv[1])) {
        const T *ap[2], *bp[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int mm = mv[i] ? m0 + 16 * i + r : r;
            const int nn = nv[i] ? n0 + 16 * i + r : r;
            ap[i] = A + (long)mm * lda + 4 * q;
            bp[i] = B + (long)nn * ldb + 4 * q;
        }
        for (int k0 = kb; k0 < ke; k0 += 16) {
            V a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *(const V *)(ap[i] + k0);
                b[i] = *(const V *)(bp[i] + k0);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if constexpr (sizeof(T) == 2) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][e], b[j][e], acc[i][j], 0, 0, 0);
                    }
                }
        }
    }
    float *Cb = PART ? C + (long)blockIdx.z * M * ldc : C;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        if (!mv[i]) continue;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (!nv[j]) continue;
            const int col = n0 + 16 * j + r;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int row = m0 + 16 * i + 4 * q + t;
                float v = acc[i][j][t];
                float *dst = Cb + (long)row * ldc + col;
                if (ACC) v += *dst;
                if (RELU) v = v > 0.f ? v : 0.f;
                *dst = v;
            }
        }
    }
}

// C[i] (+)= sum over s of part[s*stride + i], fixed order
__global__ void k_splitk_reduce(const float *__restrict__ part, int splits, long stride, long count,
                                float *__restrict__ C, int acc) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
        float s = acc ? C[i] : 0.f;
        for (int k = 0; k < splits; ++k) s += part[k * stride + i];
        C[i] = s;
    }
}

template <typename T>
__global__ void k_cvt(const float *__restrict__ src, long n, T *__restrict__ dst) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        dst[i] = to_op<T>(src[i]);
}

// im2row: X NHWC fp32 [b][y][x][cin] (channel pitch cs) -> R [pixel][Kp] operands,
// k = (ky*ks + kx)*cin + ci for a ks x ks window centred on the pixel, zero outside
template <typename T>
__global__ void k_im2row(const float *__restrict__ X, int cs, int cin, int H, int W, int nb, int ks,
                         T *__restrict__ R, int Kp) {
    const long total = (long)nb * H * W * Kp;
    const int hk = ks / 2;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int k = (int)(i % Kp);
        const long p = i / Kp;
        float v = 0.f;
        if (k < ks * ks * cin) {
            const int ci = k % cin, tap = k / cin, kx = tap % ks, ky = tap / ks;
            const int x = (int)(p % W), y = (int)((p / W) % H);
            const long b = p / ((long)W * H);
            const int yy = y + ky - hk, xx = x + kx - hk;
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = X[((b * H + yy) * W + xx) * cs + ci];
        }
        R[i] = to_op<T>(v);
    }
}

// gather col2im: dX[b][y][x][ci] (+)= sum over taps of G[pixel y - ky + hk, x - kx + hk][k]
__global__ void k_col2im(const float *__restrict__ G, int Kp, int cin, int H, int W, int nb, int ks,
                         float *__restrict__ dX, int cs, int acc) {
    const long total = (long)nb * H * W * cin;
    const int hk = ks / 2;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int ci = (int)(i % cin);
        const long p = i / cin;
        const int x = (int)(p % W), y = (int)((p / W) % H);
        const long b = p / ((long)W * H);
        float s = 0.f;
        for (int ky = 0; ky < ks; ++ky)
            for (int kx = 0; kx < ks; ++kx) {
                const int yy = y - ky + hk, xx = x - kx + hk;
                if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                s += G[((b * H + yy) * W + xx) * Kp + (ky * ks + kx) * cin + ci];
            }
        float *d = dX + p * cs + ci;
        *d = acc ? *d + s : s;
    }
}

// transpose to operands: src [R][C] (row pitch sp, first `cols` columns) -> dst [C][R]
template <typename S, typename T>
__global__ void k_transpose_op(const S *__restrict__ src, long rows, int cols, int sp, T *__restrict__ dst) {
    __shared__ float tile[32][33];
    const long r0 = (long)blockIdx.x * 32;
    const int c0 = blockIdx.y * 32;
    for (int yy = threadIdx.y; yy < 32; yy += blockDim.y) {
        const long r = r0 + yy;
        const int c = c0 + threadIdx.x;
        float v = 0.f;
        if (r < rows && c < cols) {
            if constexpr (std::is_same<S, float>::value) v = src[r * sp + c];
            else v = op_to_f<S>(src[r * sp + c]);
        }
        tile[yy][threadIdx.x] = v;
    }
    __syncthreads();
    for (int yy = threadIdx.y; yy < 32; yy += blockDim.y) {
        const int c = c0 + yy;
        const long r = r0 + threadIdx.x;
        if (c < cols && r < rows) dst[(long)c * rows + r] = to_op<T>(tile[threadIdx.x][yy]);
    }
}

// dY <- dY * (Y > 0) over the first c channels of pitch cs
__global__ void k_relu_bwd(float *__restrict__ dY, const float *__restrict__ Y, long pix, int c, int cs) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < pix * c; i += (long)gridDim.x * blockDim.x) {
        const long p = i / c;
        const int ch = (int)(i % c);
        if (!(Y[p * cs + ch] > 0.f)) dY[p * cs + ch] = 0.f;
    }
}

// 2x2 average pool, NHWC: Y[b][y][x][c] = mean of X[b][2y+i][2x+j][c]
__global__ void k_pool_fwd(const float *__restrict__ X, int H, int W, int c, int nb, float *__restrict__ Y) {
    const int h = H / 2, w = W / 2;
    const long total = (long)nb * h * w * c;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        const long p = i / c;
        const int x = (int)(p % w), y = (int)((p / w) % h);
        const long b = p / ((long)w * h);
        const float *s = X + ((b * H + 2 * y) * W + 2 * x) * c + ch;
        Y[i] = 0.25f * (s[0] + s[c] + s[(long)W * c] + s[(long)W * c + c]);
    }
}
// dX (+)= 1/4 dY spread over each 2x2 window
__global__ void k_pool_bwd(const float *__restrict__ dY, int H, int W, int c, int nb, float *__restrict__ dX,
                           int acc) {
    const long total = (long)nb * H * W * c;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        const long p = i / c;
        const int x = (int)(p % W), y = (int)((p / W) % H);
        const long b = p / ((long)W * H);
        const float g = 0.25f * dY[((b * (H / 2) + y / 2) * (W / 2) + x / 2) * c + ch];
        dX[i] = acc ? dX[i] + g : g;
    }
}
// nearest x2 upsample of X (h x w, c channels) into channels [0, c) of Y (pitch cs)
__global__ void k_up_fwd(const float *__restrict__ X, int h, int w, int c, int nb, float *__restrict__ Y, int cs) {
    const int H = 2 * h, W = 2 * w;
    const long total = (long)nb * H * W * c;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        const long p = i / c;
        const int x = (int)(p % W), y = (int)((p / W) % H);
        const long b = p / ((long)W * H);
        Y[p * cs + ch] = X[((b * h + y / 2) * w + x / 2) * c + ch];
    }
}
// dX = sum of the 2x2 block of dY channels [0, c) (pitch cs)
__global__ void k_up_bwd(const float *__restrict__ dY, int h, int w, int c, int cs, int nb, float *__restrict__ dX) {
    const long total = (long)nb * h * w * c;
    const int W = 2 * w;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        const long p = i / c;
        const int x = (int)(p % w), y = (int)((p / w) % h);
        const long b = p / ((long)w * h);
        const float *s = dY + ((b * 2 * h + 2 * y) * W + 2 * x) * cs + ch;
        dX[i] = s[0] + s[cs] + s[(long)W * cs] + s[(long)W * cs + cs];
    }
}
// copy channels: dst[p][doff + ch] (pitch ds) (+)= src[p][soff + ch] (pitch ss), ch < c
__global__ void k_copy_ch(const float *__restrict__ src, int ss, int soff, float *__restrict__ dst, int ds, int doff,
                          long pix, int c, int acc) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < pix * c; i += (long)gridDim.x * blockDim.x) {
        const long p = i / c;
        const int ch = (int)(i % c);
        const float v = src[p * ss + soff + ch];
        float *d = dst + p * ds + doff + ch;
        *d = acc ? *d + v : v;
    }
}

// per-sample sums of (y - t)^2 and t^2 over channel 0 of y (pitch ys): block b, sample z
__global__ __launch_bounds__(256) void k_loss_sums(const float *__restrict__ Y, int ys, const float *__restrict__ T,
                                                   long pix, float *__restrict__ part) {
    __shared__ double s1[256], s2[256];
    const int z = blockIdx.y;
    double a = 0.0, b = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < pix; i += (long)gridDim.x * 256) {
        const double y = Y[(z * pix + i) * ys], t = T[z * pix + i];
        a += (y - t) * (y - t);
        b += t * t;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            s1[threadIdx.x] += s1[threadIdx.x + k];
            s2[threadIdx.x] += s2[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * (z * gridDim.x + blockIdx.x)] = (float)s1[0];
        part[2 * (z * gridDim.x + blockIdx.x) + 1] = (float)s2[0];
    }
}
// per-sample totals: tot[2z] = sum (y-t)^2, tot[2z+1] = sum t^2, loss[z] = ratio
__global__ void k_loss_total(const float *__restrict__ part, int nblk, int nb, float *__restrict__ tot,
                             float *__restrict__ loss) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= nb) return;
    float e = 0.f, t2 = 0.f;
    for (int k = 0; k < nblk; ++k) {
        e += part[2 * (z * nblk + k)];
        t2 += part[2 * (z * nblk + k) + 1];
    }
    tot[2 * z] = e;
    tot[2 * z + 1] = t2;
    loss[z] = e / t2;
}
// gradient of the mean over the batch of the relative squared errors:
// dY = 2 (y - t) / (sum t^2 * nb) in channel 0, 0 in the other channels
__global__ void k_loss_grad(const float *__restrict__ Y, int ys, const float *__restrict__ T, long pix, int nb,
                            const float *__restrict__ tot, float *__restrict__ dY) {
    const long total = (long)nb * pix * ys;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % ys);
        const long p = i / ys;
        dY[i] = ch == 0 ? 2.f * (Y[i] - T[p]) / (tot[2 * (p / pix) + 1] * nb) : 0.f;
    }
}
// squared norm of x[0..n): kSqParts workgroups sum contiguous chunks into
// part[], then one workgroup adds the partials in order (fixed order)
constexpr int kSqParts = 64;
__global__ __launch_bounds__(256) void k_sumsq_part(const double *__restrict__ x, long n, double *__restrict__ part) {
    __shared__ double sh[256];
    const long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long beg = (long)blockIdx.x * chunk, end = beg + chunk < n ? beg + chunk : n;
    double a = 0.0;
    for (long i = beg + threadIdx.x; i < end; i += 256) a += x[i] * x[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_sumsq_final(const double *__restrict__ part, int np, double *__restrict__ out) {
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < np; ++i) t += part[i];
        out[0] = t;
    }
}

// Adam on FP32 master weights; refreshes the operand copies W [cout][Kp] and W^T [Kp][coutp]
template <typename T>
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v, const float *__restrict__ g,
                       int cout, int K, int Kp, int coutp, float lr, float b1, float b2, float eps, float c1, float c2,
                       T *__restrict__ wb, T *__restrict__ wt) {
    const long total = (long)cout * K;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const int co = (int)(i / K), k = (int)(i % K);
        const long gi = (long)co * Kp + k;
        if (lr > 0.f) {
            const float gg = g[gi];
            const float mm = b1 * m[i] + (1.f - b1) * gg;
            const float vv = b2 * v[i] + (1.f - b2) * gg * gg;
            m[i] = mm;
            v[i] = vv;
            w[i] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
        }
        const T b = to_op<T>(w[i]);
        wb[(long)co * Kp + k] = b;
        wt[(long)k * coutp + co] = b;
    }
}

// training sample from a (residual, solution) pair: x = (r / rms(r), alpha) and
// t = sol / rms(r) on the top-left n x n of the H x W grid, zero elsewhere
__global__ void k_pack_sample(const double *__restrict__ r, const double *__restrict__ sol, int n, int H, int W,
                              float alpha, const double *nrm, float *__restrict__ X, float *__restrict__ T) {
    const double s = nrm[0] > 0.0 ? (double)n / sqrt(nrm[0]) : 1.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (long)H * W; i += (long)gridDim.x * blockDim.x) {
        const int x = (int)(i % W), y = (int)(i / W);
        const bool in = x < n && y < n;
        X[2 * i] = in ? (float)(s * r[(long)y * n + x]) : 0.f;
        X[2 * i + 1] = alpha;
        if (T) T[i] = in && sol ? (float)(s * sol[(long)y * n + x]) : 0.f;
    }
}
// energy-norm loss, step 1: d = y - t on the n x n interior (compact, row-major)
__global__ void k_energy_diff(const float *__restrict__ Y, int ys, const float *__restrict__ T, int n, int W,
                              float *__restrict__ d) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (long)n * n; i += (long)gridDim.x * blockDim.x) {
        const long p = (i / n) * W + i % n;
        d[i] = Y[p * ys] - T[p];
    }
}
// step 2 (one block): loss = (d, A d) / (t, x0) with x0 = channel 0 of the input;
// since A t = x0 for an exact pair, the denominator is ||t||_A^2
__global__ __launch_bounds__(256) void k_energy_loss(const float *__restrict__ d, const float *__restrict__ Ad,
                                                     const float *__restrict__ T, const float *__restrict__ X, int n,
                                                     int W, float *__restrict__ loss, float *__restrict__ den) {
    __shared__ double s1[256], s2[256];
    double a = 0.0, b = 0.0;
    for (long i = threadIdx.x; i < (long)n * n; i += 256) {
        const long p = (i / n) * W + i % n;
        a += (double)d[i] * (double)Ad[i];
        b += (double)T[p] * (double)X[2 * p];
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            s1[threadIdx.x] += s1[threadIdx.x + k];
            s2[threadIdx.x] += s2[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        loss[0] = (float)(s1[0] / s2[0]);
        den[0] = (float)s2[0];
    }
}
// step 3: dY = 2 A d / (den * nb) in channel 0 of the interior, 0 elsewhere
__global__ void k_energy_grad(const float *__restrict__ Ad, const float *__restrict__ den, int n, int H, int W, int nb,
                              float *__restrict__ dY, int ys) {
    const float sc = 2.f / (den[0] * nb);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (long)H * W * ys; i += (long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % ys);
        const long p = i / ys;
        const int x = (int)(p % W), y = (int)(p / W);
        dY[i] = (ch == 0 && x < n && y < n) ? sc * Ad[(long)y * n + x] : 0.f;
    }
}

// residual loss ||A y - x0||^2 / ||x0||^2 on the n x n interior (x0 = channel 0
// of the input, the scaled residual): the preconditioner's own criterion, A M
// close to the identity on the residuals it is shown.  step 1: y compacted.
__global__ void k_res_compact(const float *__restrict__ Y, int ys, int n, int W, float *__restrict__ yc) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (long)n * n; i += (long)gridDim.x * blockDim.x) {
        const long p = (i / n) * W + i % n;
        yc[i] = Y[p * ys];
    }
}
// step 2 (one block, after q = A y): q <- e = q - x0 in place; loss = (e, e) / (x0, x0)
__global__ __launch_bounds__(256) void k_res_loss(float *__restrict__ q, const float *__restrict__ X, int n, int W,
                                                  float *__restrict__ loss, float *__restrict__ den) {
    __shared__ double s1[256], s2[256];
    double a = 0.0, b = 0.0;
    for (long i = threadIdx.x; i < (long)n * n; i += 256) {
        const long p = (i / n) * W + i % n;
        const float x0 = X[2 * p];
        const float e = q[i] - x0;
        q[i] = e;
        a += (double)e * (double)e;
        b += (double)x0 * (double)x0;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            s1[threadIdx.x] += s1[threadIdx.x + k];
            s2[threadIdx.x] += s2[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        loss[0] = (float)(s1[0] / s2[0]);
        den[0] = (float)s2[0];
    }
}
// step 3 is A e by a matvec; step 4 is k_energy_grad on A e: dY = 2 A e / (den nb)

// minibatch gather: dst[j] = src[idx[j]] for blocks of `len` floats
__global__ void k_gather(const float *__restrict__ src, const long *__restrict__ idx, int nb, long len,
                         float *__restrict__ dst) {
    const long total = (long)nb * len;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        const long j = i / len, e = i % len;
        dst[i] = src[idx[j] * len + e];
    }
}

// ---------------------------------------------------------------------------
// Fused convolution for inference: implicit GEMM straight from the NHWC
// activations.  A workgroup (4 waves) owns an 8 x 8 tile of output pixels of
// one sample and all output channels.  It stages the input halo
// (8+KS-1)^2 x cin in LDS as GEMM operands, forming the input on the fly:
//   SRC_PLAIN  X[y][x][ci]
//   SRC_POOL   the 2 x 2 average of a source at twice the resolution
//   SRC_CATUP  channels [0, ca) from a source at half the resolution (nearest
//              upsampling), channels [ca, cin) from a source at this one.
// Wave w computes pixels 16w..16w+15 against every output channel with the
// same MFMA tiles and k order (k = tap*cin + ci, steps of 16) as k_gemm_nt on
// im2row rows.  cin is a multiple of 16, except the 2-channel first layer
// (GENERIC), whose k steps cross taps.
// ---------------------------------------------------------------------------
enum { SRC_PLAIN = 0, SRC_POOL = 1, SRC_CATUP = 2 };

struct ConvSrc {
    const float *a = nullptr, *b = nullptr;  // sources (b: the second one of SRC_CATUP)
    int csa = 0, csb = 0;                    // channel pitches
    int ca = 0;                              // SRC_CATUP: channels taken from a
};

// NS > 1 splits the output channels over NS workgroups per tile (blockIdx.z =
// sample * NS + split), for the coarse levels whose grids are small.
template <typename T, int MODE, int KS, int CIN, int COUTP, int NS>
__global__ __launch_bounds__(256) void k_conv_fused(ConvSrc src, int H, int W, const T *__restrict__ Wb,
                                                    float *__restrict__ Y, int relu) {
    constexpr int TS = 8, HH = TS + KS - 1, HK = KS / 2;
    constexpr bool GENERIC = CIN % 16 != 0;  // the 2-channel first layer
    constexpr int K = KS * KS * CIN, Kp = (K + 15) / 16 * 16, NTN = COUTP / 16 / NS;
    static_assert(COUTP % (16 * NS) == 0, "channel split");
    constexpr int CV = CIN % 4 == 0 ? 4 : 1;  // channels staged per thread and step
    __shared__ T tile[HH * HH * CIN];
    const int b = blockIdx.z / NS, n0 = (blockIdx.z % NS) * NTN * 16;  // first output channel
    const int tx0 = blockIdx.x * TS, ty0 = blockIdx.y * TS;
    // stage the halo, CV channels at a time
    for (int e = threadIdx.x; e < HH * HH * (CIN / CV); e += 256) {
        const int cg = e % (CIN / CV), pix = e / (CIN / CV);
        const int hx = pix % HH, hy = pix / HH;
        const int y = ty0 + hy - HK, x = tx0 + hx - HK;
        float v[CV];
#pragma unroll
        for (int i = 0; i < CV; ++i) v[i] = 0.f;
        if (y >= 0 && y < H && x >= 0 && x < W) {
            const int ci = cg * CV;
            if (MODE == SRC_PLAIN) {
                const float *q = src.a + (((long)b * H + y) * W + x) * src.csa + ci;
#pragma unroll
                for (int i = 0; i < CV; ++i) v[i] = q[i];
            } else if (MODE == SRC_POOL) {
                const int W2 = 2 * W;
                const float *q = src.a + (((long)b * 2 * H + 2 * y) * W2 + 2 * x) * src.csa + ci;
                const long dy = (long)W2 * src.csa;
#pragma unroll
                for (int i = 0; i < CV; ++i) v[i] = 0.25f * (q[i] + q[src.csa + i] + q[dy + i] + q[dy + src.csa + i]);
            } else {
                const float *q = ci < src.ca
                                     ? src.a + (((long)b * (H / 2) + y / 2) * (W / 2) + x / 2) * src.csa + ci
                                     : src.b + (((long)b * H + y) * W + x) * src.csb + (ci - src.ca);
#pragma unroll
                for (int i = 0; i < CV; ++i) v[i] = q[i];
            }
        }
#pragma unroll
        for (int i = 0; i < CV; ++i) tile[pix * CIN + cg * CV + i] = to_op<T>(v[i]);
    }
    __syncthreads();
    using V = typename std::conditional<sizeof(T) == 2, v4s, v4f>::type;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int m = 16 * wave + r;  // this lane's pixel for the A operand
    const int pbase = ((m / TS) * HH + (m % TS)) * CIN;
    v4f acc[NTN];
#pragma unroll
    for (int j = 0; j < NTN; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 6
    for (int k0 = 0; k0 < Kp; k0 += 16) {
        V bv[NTN];
#pragma unroll
        for (int j = 0; j < NTN; ++j) bv[j] = *(const V *)(Wb + (n0 + 16 * j + r) * Kp + k0 + 4 * q);
        V a;
        if constexpr (GENERIC) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = k0 + 4 * q + i;
                T t = to_op<T>(0.f);
                if (k < K) {
                    const int tap = k / CIN, ci = k % CIN;
                    t = tile[pbase + ((tap / KS) * HH + (tap % KS)) * CIN + ci];
                }
                if constexpr (sizeof(T) == 2) a[i] = (short)t;
                else a[i] = t;
            }
        } else {
            const int tap = k0 / CIN;
            a = *(const V *)(tile + pbase + ((tap / KS) * HH + (tap % KS)) * CIN + (k0 - tap * CIN) + 4 * q);
        }
#pragma unroll
        for (int j = 0; j < NTN; ++j) {
            if constexpr (sizeof(T) == 2) {
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv[j], acc[j], 0, 0, 0);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], bv[j][e], acc[j], 0, 0, 0);
            }
        }
    }
    // D rows 4q+i are pixels 16w+4q+i, column r is channel 16j+r
#pragma unroll
    for (int j = 0; j < NTN; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int mm = 16 * wave + 4 * q + i;
            const int y = ty0 + mm / TS, x = tx0 + mm % TS;
            if (y >= H || x >= W) continue;
            float v = acc[j][i];
            if (relu) v = v > 0.f ? v : 0.f;
            Y[(((long)b * H + y) * W + x) * COUTP + n0 + 16 * j + r] = v;
        }
}

// ---------------------------------------------------------------------------
// Two 3x3 convolutions of one U-Net level in one launch (inference).  A
// workgroup owns a TS x TS output tile.  It stages the (TS+4)^2 input halo in
// LDS (formed on the fly as in k_conv_fused, or from the residual: channel 0
// = r / rms(r) on the interior n x n, channel 1 = alpha), computes the first
// convolution + ReLU on the (TS+2)^2 ring the second one reads into LDS (zero
// outside the image: the second convolution's padding), then the second
// convolution + ReLU on the tile.  LAST also applies the final 1x1 convolution
// and writes z = rms(r) * Net at the interior.  Operands: gfx950's
// v_mfma_f32_16x16x32_bf16 (fp32 mode: eight v_mfma_f32_16x16x4_f32 per k
// step), lane (r, q) supplying row r and k = 8q .. 8q+7 of each 32-wide step,
// with k = tap * cin + ci as in k_conv_fused.
// ---------------------------------------------------------------------------
enum { SRC_RESID = 3 };
struct PairSrc {
    ConvSrc c;
    const double *r = nullptr;    // SRC_RESID: the residual (n x n, row-major) ...
    const double *nrm = nullptr;  // ... and its squared norm (device)
    int n = 0;
    float alpha = 0.f;
    double *z = nullptr;          // LAST: the preconditioned residual (n x n)
};
typedef short v8s __attribute__((ext_vector_type(8)));
typedef float v8f __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// acc[j] (output channels 16j + r of M-tile mt, pixels 16 mt + 4q + i) of the
// 3x3 convolution of the LDS tile `in` (IW x IW pixels of CIN channels, pixel
// pitch CP) over an
// OW x OW output region whose pixel (oy, ox) reads in at (oy + ty, ox + tx);
// weights W [cout][ldw] (global or LDS), k past Kw reads as zero
template <typename T, int CIN, int CP, int COUT, int IW, int OW>
__device__ __forceinline__ void conv3_tile(const T *in, const T *W, int ldw, int Kw, int mt, int lane, v4f *acc) {
    constexpr int K = 9 * CIN, K32 = (K + 31) / 32 * 32, NTN = COUT / 16;
    using V = typename std::conditional<sizeof(T) == 2, v8s, v8f>::type;
    const int r = lane & 15, q = lane >> 4;
    const int m0 = 16 * mt + r;
    const int m = m0 < OW * OW ? m0 : OW * OW - 1;  // rows past the region: any pixel, results unused
    const int pbase = ((m / OW) * IW + (m % OW)) * CP;
#pragma unroll
    for (int j = 0; j < NTN; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
    for (int k0 = 0; k0 < K32; k0 += 32) {
        const int k = k0 + 8 * q;
        V a;
        if constexpr (CIN % 8 == 0) {
            // k .. k+7 lie in one tap; past K (zero weights) any tap in range is read
            const int kk = k < K ? k : 0;
            const int tap = kk / CIN;
            a = *(const V *)(in + pbase + ((tap / 3) * IW + tap % 3) * CP + (kk - tap * CIN));
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int kk = k + i < K ? k + i : 0;
                const int tap = kk / CIN;
                const T t = in[pbase + ((tap / 3) * IW + tap % 3) * CP + (kk - tap * CIN)];
                if constexpr (sizeof(T) == 2) a[i] = (short)t;
                else a[i] = t;
            }
        }
        const bool wk = k < Kw;  // 8-aligned and Kw a multiple of 16: all 8 or none
        V b[NTN];
#pragma unroll
        for (int j = 0; j < NTN; ++j) {
            const V w = *(const V *)(W + (16 * j + r) * ldw + (wk ? k : 0));
            b[j] = wk ? w : V{};
        }
#pragma unroll
        for (int j = 0; j < NTN; ++j) {
            if constexpr (sizeof(T) == 2) {
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                                 __builtin_bit_cast(v8bf, b[j]), acc[j], 0, 0, 0);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[j][e], acc[j], 0, 0, 0);
            }
        }
    }
}

// LDS row stride of a staged weight matrix with rows of Kw operands: a multiple
// of 8 operands whose byte length is 16 mod 128, so the 16 rows one k step reads
// (16 bytes each) spread over the LDS banks
template <typename T> constexpr int wstride(int Kw) {
    const int b = Kw * (int)sizeof(T);
    return (Kw * (int)sizeof(T) + ((16 - b % 128) + 128) % 128) / (int)sizeof(T);
}

// threads of a k_conv_pair workgroup (8 waves)
constexpr int kPairThreads = 512;

// copy a [ROWS][K] bf16 matrix from global memory into LDS rows of stride S,
// in 16-byte chunks, a thread's loads all issued before its stores
template <int ROWS, int K, int S>
__device__ __forceinline__ void stage_rows(const bf16 *__restrict__ src, bf16 *dst) {
    constexpr int NC = ROWS * (K / 8), NIT = (NC + kPairThreads - 1) / kPairThreads;
    v8s c[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = threadIdx.x + kPairThreads * it, ec = e < NC ? e : 0;
        c[it] = *(const v8s *)(src + (long)(ec / (K / 8)) * K + 8 * (ec % (K / 8)));
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = threadIdx.x + kPairThreads * it;
        if (e < NC) *(v8s *)(dst + (e / (K / 8)) * S + 8 * (e % (K / 8))) = c[it];
    }
}

template <typename T, int MODE, int CIN, int CMID, int COUT, int TS, bool LAST>
__global__ __launch_bounds__(kPairThreads) void k_conv_pair(PairSrc ps, int H, const T *__restrict__ WA,
                                                   const T *__restrict__ WB, const T *__restrict__ WL,
                                                   float *__restrict__ Y) {
    constexpr int IW = TS + 4, MW = TS + 2, CV = CIN % 4 == 0 ? 4 : 1;
    // pixel pitches in LDS: 16 bytes past the channels, so the 16 pixels of a
    // k step's A operand (16 bytes each) fall on distinct banks
    constexpr int CPI = CIN % 8 == 0 ? CIN + 8 : CIN, CPM = CMID + 8;
    static_assert(!LAST || COUT == 16, "the final 1x1 convolution reads 16 channels");
    // bf16 operands: both weight matrices staged in LDS once (fp32 mode reads them from global)
    constexpr bool WL_LDS = sizeof(T) == 2;
    constexpr int KA = (9 * CIN + 15) / 16 * 16, KB = (9 * CMID + 15) / 16 * 16;
    constexpr int SA = wstride<T>(KA), SB = wstride<T>(KB);
    __shared__ __attribute__((aligned(32))) T tin[IW * IW * CPI > TS * TS * 16 ? IW * IW * CPI : TS * TS * 16];
    __shared__ __attribute__((aligned(32))) T tmid[MW * MW * CPM];
    __shared__ __attribute__((aligned(32))) T wla[WL_LDS ? CMID * SA : 1];
    __shared__ __attribute__((aligned(32))) T wlb[WL_LDS ? COUT * SB : 1];
    if constexpr (WL_LDS) {
        // 16-byte chunks, every load of a thread issued before its first LDS store;
        // KA, KB are multiples of 16 operands (the host's padding)
        stage_rows<CMID, KA, SA>(WA, wla);
        stage_rows<COUT, KB, SB>(WB, wlb);
    }
    const T *wa = WL_LDS ? (const T *)wla : WA;
    const T *wb = WL_LDS ? (const T *)wlb : WB;
    const int lda = WL_LDS ? SA : KA, ldb = WL_LDS ? SB : KB;
    const int W = H;
    const int b = blockIdx.z;
    const int tx0 = blockIdx.x * TS, ty0 = blockIdx.y * TS;
    const ConvSrc &src = ps.c;
    double s_in = 1.0;
    if constexpr (MODE == SRC_RESID) s_in = (ps.nrm && ps.nrm[0] > 0.0) ? (double)ps.n / sqrt(ps.nrm[0]) : 1.0;
    // stage the input halo, CV channels per task: all of a thread's loads (from
    // clamped, always valid addresses) before its LDS stores
    constexpr int NE = IW * IW * (CIN / CV), NIT = (NE + kPairThreads - 1) / kPairThreads;
    float v[NIT][CV];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = threadIdx.x + kPairThreads * it;
        const int cg = e % (CIN / CV), pix = (e < NE ? e : 0) / (CIN / CV);
        const int y = ty0 + pix / IW - 2, x = tx0 + pix % IW - 2;
        const bool ok = e < NE && y >= 0 && y < H && x >= 0 && x < W;
        const int yc = ok ? y : 0, xc = ok ? x : 0;
        const int ci = cg * CV;
        if constexpr (MODE == SRC_RESID) {
            // CIN = 2, CV = 1: r / rms(r) on the interior n x n, alpha elsewhere in the image
            const bool inr = ok && ci == 0 && yc < ps.n && xc < ps.n;
            const double rv = ps.r[inr ? (long)yc * ps.n + xc : 0];
            v[it][0] = !ok ? 0.f : (ci == 0 ? (inr ? (float)(s_in * rv) : 0.f) : ps.alpha);
        } else if constexpr (MODE == SRC_PLAIN) {
            const float *q = src.a + (((long)b * H + yc) * W + xc) * src.csa + ci;
#pragma unroll
            for (int i = 0; i < CV; ++i) v[it][i] = ok ? q[i] : 0.f;
        } else if constexpr (MODE == SRC_POOL) {
            const int W2 = 2 * W;
            const float *q = src.a + (((long)b * 2 * H + 2 * yc) * W2 + 2 * xc) * src.csa + ci;
            const long dy = (long)W2 * src.csa;
#pragma unroll
            for (int i = 0; i < CV; ++i) {
                const float t = 0.25f * (q[i] + q[src.csa + i] + q[dy + i] + q[dy + src.csa + i]);
                v[it][i] = ok ? t : 0.f;
            }
        } else {
            const float *q = ci < src.ca
                                 ? src.a + (((long)b * (H / 2) + yc / 2) * (W / 2) + xc / 2) * src.csa + ci
                                 : src.b + (((long)b * H + yc) * W + xc) * src.csb + (ci - src.ca);
#pragma unroll
            for (int i = 0; i < CV; ++i) v[it][i] = ok ? q[i] : 0.f;
        }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = threadIdx.x + kPairThreads * it;
        if (e < NE) {
            const int cg = e % (CIN / CV), pix = e / (CIN / CV);
            if constexpr (CV == 4) {  // one 4-operand store (8 or 16 bytes, aligned)
                typedef T T4 __attribute__((ext_vector_type(4)));
                T4 w;
#pragma unroll
                for (int i = 0; i < 4; ++i) w[i] = to_op<T>(v[it][i]);
                *(T4 *)(tin + pix * CPI + cg * 4) = w;
            } else {
                tin[pix * CPI + cg] = to_op<T>(v[it][0]);
            }
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    // first convolution on the MW x MW ring, ReLU, zero outside the image
    {
        constexpr int NMT = (MW * MW + 15) / 16, NTN = CMID / 16;
        for (int mt = wave; mt < NMT; mt += kPairThreads / 64) {
            v4f acc[NTN];
            conv3_tile<T, CIN, CPI, CMID, IW, MW>(tin, wa, lda, KA, mt, lane, acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 16 * mt + 4 * q + i;
                if (m >= MW * MW) continue;
                const int gy = ty0 - 1 + m / MW, gx = tx0 - 1 + m % MW;
                const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
#pragma unroll
                for (int j = 0; j < NTN; ++j) {
                    const float v = acc[j][i];
                    tmid[m * CPM + 16 * j + r] = to_op<T>(in && v > 0.f ? v : 0.f);
                }
            }
        }
    }
    __syncthreads();
    // second convolution on the tile, ReLU
    {
        constexpr int NMT = TS * TS / 16, NTN = COUT / 16;
        for (int mt = wave; mt < NMT; mt += kPairThreads / 64) {
            v4f acc[NTN];
            conv3_tile<T, CMID, CPM, COUT, MW, TS>(tmid, wb, ldb, KB, mt, lane, acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 16 * mt + 4 * q + i;
                const int oy = m / TS, ox = m % TS;
#pragma unroll
                for (int j = 0; j < NTN; ++j) {
                    const float v = acc[j][i] > 0.f ? acc[j][i] : 0.f;
                    if constexpr (LAST) {
                        tin[m * 16 + r] = to_op<T>(v);  // the input tile is no longer read
                    } else {
                        const int y = ty0 + oy, x = tx0 + ox;
                        if (y < H && x < W) Y[(((long)b * H + y) * W + x) * COUT + 16 * j + r] = v;
                    }
                }
            }
        }
    }
    if constexpr (LAST) {
        __syncthreads();
        // final 1x1 convolution (one output channel) and z = rms(r) * y at the interior
        const double s_out = (ps.nrm && ps.nrm[0] > 0.0) ? sqrt(ps.nrm[0]) / (double)ps.n : 1.0;
        for (int m = threadIdx.x; m < TS * TS; m += kPairThreads) {
            const int y = ty0 + m / TS, x = tx0 + m % TS;
            if (y >= ps.n || x >= ps.n) continue;
            float t = 0.f;
#pragma unroll
            for (int c = 0; c < 16; ++c) t += op_to_f<T>(WL[c]) * op_to_f<T>(tin[m * 16 + c]);
            ps.z[(long)b * ps.n * ps.n + (long)y * ps.n + x] = s_out * (double)t;
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Conv {
    int cin, cout, ks, K, Kp, coutp;   // K = ks*ks*cin, Kp padded to 16, coutp padded to 16
    long woff;                          // offset of this layer in the parameter arrays
};

}  // namespace fl

struct fl_unet_s {
    int H = 0, W = 0, nb = 0;           // image size, batch capacity
    std::vector<fl::Conv> conv;         // 11 layers
    long nparam = 0;                    // sum cout*K
    long nparam_pad = 0;                // sum cout*Kp (gradient layout)
    int fp32 = 0;                       // GEMM operands in fp32 (verification mode) instead of bf16
    size_t osz = 2;                     // bytes per GEMM operand
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // fp32 master, Adam, gradient (padded)
    void *wb = nullptr, *wt = nullptr;                             // operand copies W, W^T
    long wb_len = 0, wt_len = 0;
    std::vector<long> wb_off, wt_off;
    int step = 0;
    // activations and gradients (fp32 NHWC, batch nb)
    float *act = nullptr;
    size_t act_bytes = 0;
    std::vector<float *> A, G;          // per tensor
    void *rowbuf = nullptr, *tbuf = nullptr, *tbuf2 = nullptr;        // operand staging
    float *colbuf = nullptr, *part = nullptr, *lossbuf = nullptr, *lpart = nullptr, *ltot = nullptr;
    size_t row_elems = 0, col_elems = 0, part_elems = 0;
    double *nrm = nullptr;
    double *sqpart = nullptr;           // partial sums of squared norms
    hipEvent_t ev = nullptr;            // joins the caller's stream and the network's
    long *idx = nullptr;                // minibatch indices (device)
    float *ebuf = nullptr;              // energy loss: d and A d (2 x H*W floats)
    hipStream_t s = nullptr;
};

namespace fl {

// tensor ids
enum {
    T_X0, T_A1, T_S1, T_P1, T_A2, T_S2, T_P2, T_A3, T_B3, T_C2, T_A4, T_B4, T_C1, T_A5, T_B5, T_Y, T_TGT, T_COUNT
};

struct TShape {
    int h, c;  // side length (h = H, H/2, H/4) and channels
};

static TShape tshape(const fl_unet_s *u, int t) {
    const int H = u->H;
    switch (t) {
        case T_X0: return {H, 2};
        case T_A1: case T_S1: case T_A5: case T_B5: return {H, 16};
        case T_P1: return {H / 2, 16};
        case T_A2: case T_S2: case T_A4: case T_B4: return {H / 2, 32};
        case T_P2: return {H / 4, 32};
        case T_A3: case T_B3: return {H / 4, 64};
        case T_C2: return {H / 2, 96};
        case T_C1: return {H, 48};
        case T_Y: return {H, 16};
        case T_TGT: return {H, 1};
    }
    return {0, 0};
}

template <typename T>
static void launch_gemm(bool relu, bool acc, const T *A, int lda, const T *B, int ldb, float *C, int ldc, int M, int N,
                        int K, hipStream_t s) {
    dim3 g(cdiv_i(M, 64), cdiv_i(N, 64), 1);
    if (relu)
        hipLaunchKernelGGL((k_gemm_nt<T, true, false, false>), g, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, K);
    else if (acc)
        hipLaunchKernelGGL((k_gemm_nt<T, false, true, false>), g, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, K);
    else
        hipLaunchKernelGGL((k_gemm_nt<T, false, false, false>), g, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, K);
}
template <typename T> static T *wb_of(fl_unet u, int li) { return (T *)u->wb + u->wb_off[li]; }
template <typename T> static T *wt_of(fl_unet u, int li) { return (T *)u->wt + u->wt_off[li]; }

// conv forward: Y[pix][cout] (pitch coutp) = relu?(im2row(X) W^T)
template <typename T>
static void conv_fwd(fl_unet u, int li, const float *X, int xcs, int h, int nb, float *Y, bool relu) {
    const Conv &c = u->conv[li];
    const long pix = (long)nb * h * h;
    T *row = (T *)u->rowbuf;
    hipLaunchKernelGGL(k_im2row<T>, dim3(grid1(pix * c.Kp)), dim3(256), 0, u->s, X, xcs, c.cin, h, h, nb, c.ks, row,
                       c.Kp);
    launch_gemm<T>(relu, false, row, c.Kp, wb_of<T>(u, li), c.Kp, Y, c.coutp, (int)pix, c.coutp, c.Kp, u->s);
}

// conv backward: dY (pitch coutp, already masked by the ReLU) -> gradient of the
// weights (into u->g) and, if dX, the input gradient (+= when accx)
template <typename T>
static void conv_bwd(fl_unet u, int li, const float *X, int xcs, int h, int nb, const float *dY, float *dX, int dxcs,
                     bool accx) {
    const Conv &c = u->conv[li];
    const long pix = (long)nb * h * h;
    hipStream_t s = u->s;
    T *row = (T *)u->rowbuf, *tb = (T *)u->tbuf, *tb2 = (T *)u->tbuf2;
    // weight gradient: dW[cout][k] = sum_pix dY[pix][cout] R[pix][k]
    hipLaunchKernelGGL(k_im2row<T>, dim3(grid1(pix * c.Kp)), dim3(256), 0, s, X, xcs, c.cin, h, h, nb, c.ks, row, c.Kp);
    hipLaunchKernelGGL((k_transpose_op<T, T>), dim3(cdiv_i(pix, 32), cdiv_i(c.Kp, 32)), dim3(32, 8), 0, s, row, pix,
                       c.Kp, c.Kp, tb);  // [Kp][pix]
    hipLaunchKernelGGL((k_transpose_op<float, T>), dim3(cdiv_i(pix, 32), cdiv_i(c.coutp, 32)), dim3(32, 8), 0, s, dY,
                       pix, c.coutp, c.coutp, tb2);  // [coutp][pix]
    const int kchunk = 2048;
    const int splits = cdiv_i(pix, kchunk);
    dim3 g(cdiv_i(c.coutp, 64), cdiv_i(c.Kp, 64), splits);
    hipLaunchKernelGGL((k_gemm_nt<T, false, false, true>), g, dim3(256), 0, s, tb2, (int)pix, tb, (int)pix, u->part,
                       c.Kp, c.coutp, c.Kp, (int)pix, kchunk);
    // partial products are [coutp][Kp]; the first cout rows are the real gradient
    hipLaunchKernelGGL(k_splitk_reduce, dim3(grid1((long)c.cout * c.Kp)), dim3(256), 0, s, u->part, splits,
                       (long)c.coutp * c.Kp, (long)c.cout * c.Kp, u->g + u->wb_off[li], 0);
    if (!dX) return;
    // input gradient: G[pix][k] = sum_cout dY[pix][cout] W[cout][k], then col2im
    hipLaunchKernelGGL(k_cvt<T>, dim3(grid1(pix * c.coutp)), dim3(256), 0, s, dY, pix * c.coutp, tb);
    launch_gemm<T>(false, false, tb, c.coutp, wt_of<T>(u, li), c.coutp, u->colbuf, c.Kp, (int)pix, c.Kp, c.coutp, s);
    hipLaunchKernelGGL(k_col2im, dim3(grid1(pix * c.cin)), dim3(256), 0, s, u->colbuf, c.Kp, c.cin, h, h, nb, c.ks,
                       dX, dxcs, accx ? 1 : 0);
}

template <typename T>
static void net_forward_t(fl_unet u, int nb) {
    const int H = u->H;
    auto *A = u->A.data();
    hipStream_t s = u->s;
    conv_fwd<T>(u, 0, A[T_X0], 2, H, nb, A[T_A1], true);
    conv_fwd<T>(u, 1, A[T_A1], 16, H, nb, A[T_S1], true);
    hipLaunchKernelGGL(k_pool_fwd, dim3(grid1((long)nb * H * H / 4 * 16)), dim3(256), 0, s, A[T_S1], H, H, 16, nb,
                       A[T_P1]);
    conv_fwd<T>(u, 2, A[T_P1], 16, H / 2, nb, A[T_A2], true);
    conv_fwd<T>(u, 3, A[T_A2], 32, H / 2, nb, A[T_S2], true);
    hipLaunchKernelGGL(k_pool_fwd, dim3(grid1((long)nb * H * H / 16 * 32)), dim3(256), 0, s, A[T_S2], H / 2, H / 2, 32,
                       nb, A[T_P2]);
    conv_fwd<T>(u, 4, A[T_P2], 32, H / 4, nb, A[T_A3], true);
    conv_fwd<T>(u, 5, A[T_A3], 64, H / 4, nb, A[T_B3], true);
    const long p2 = (long)nb * (H / 2) * (H / 2), p1 = (long)nb * H * H;
    hipLaunchKernelGGL(k_up_fwd, dim3(grid1(p2 * 64)), dim3(256), 0, s, A[T_B3], H / 4, H / 4, 64, nb, A[T_C2], 96);
    hipLaunchKernelGGL(k_copy_ch, dim3(grid1(p2 * 32)), dim3(256), 0, s, A[T_S2], 32, 0, A[T_C2], 96, 64, p2, 32, 0);
    conv_fwd<T>(u, 6, A[T_C2], 96, H / 2, nb, A[T_A4], true);
    conv_fwd<T>(u, 7, A[T_A4], 32, H / 2, nb, A[T_B4], true);
    hipLaunchKernelGGL(k_up_fwd, dim3(grid1(p1 * 32)), dim3(256), 0, s, A[T_B4], H / 2, H / 2, 32, nb, A[T_C1], 48);
    hipLaunchKernelGGL(k_copy_ch, dim3(grid1(p1 * 16)), dim3(256), 0, s, A[T_S1], 16, 0, A[T_C1], 48, 32, p1, 16, 0);
    conv_fwd<T>(u, 8, A[T_C1], 48, H, nb, A[T_A5], true);
    conv_fwd<T>(u, 9, A[T_A5], 16, H, nb, A[T_B5], true);
    conv_fwd<T>(u, 10, A[T_B5], 16, H, nb, A[T_Y], false);
}

// gradients of every weight from dY (in G[T_Y], pitch 16)
template <typename T>
static void net_backward_t(fl_unet u, int nb) {
    const int H = u->H;
    auto *A = u->A.data();
    auto *G = u->G.data();
    hipStream_t s = u->s;
    const long p1 = (long)nb * H * H, p2 = p1 / 4, p3 = p1 / 16;
    conv_bwd<T>(u, 10, A[T_B5], 16, H, nb, G[T_Y], G[T_B5], 16, false);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(p1 * 16)), dim3(256), 0, s, G[T_B5], A[T_B5], p1, 16, 16);
    conv_bwd<T>(u, 9, A[T_A5], 16, H, nb, G[T_B5], G[T_A5], 16, false);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(p1 * 16)), dim3(256), 0, s, G[T_A5], A[T_A5], p1, 16, 16);
    conv_bwd<T>(u, 8, A[T_C1], 48, H, nb, G[T_A5], G[T_C1], 48, false);
    // concat 1: channels [0,32) from up(B4), [32,48) to S1
    hipLaunchKernelGGL(k_up_bwd, dim3(grid1(p2 * 32)), dim3(256), 0, s, G[T_C1], H / 2, H / 2, 32, 48, nb, G[T_B4]);
    hipLaunchKernelGGL(k_copy_ch, dim3(grid1(p1 * 16)), dim3(256), 0, s, G[T_C1], 48, 32, G[T_S1], 16, 0, p1, 16, 0);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(p2 * 32)), dim3(256), 0, s, G[T_B4], A[T_B4], p2, 32, 32);
    conv_bwd<T>(u, 7, A[T_A4], 32, H / 2, nb, G[T_B4], G[T_A4], 32, false);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(p2 * 32)), dim3(256), 0, s, G[T_A4], A[T_A4], p2, 32, 32);
    conv_bwd<T>(u, 6, A[T_C2], 96, H / 2, nb, G[T_A4], G[T_C2], 96, false);
    hipLaunchKernelGGL(k_up_bwd, dim3(grid1(p3 * 64)), dim3(256), 0, s, G[T_C2], H / 4, H / 4, 64, 96, nb, G[T_B3]);
    hipLaunchKernelGGL(k_copy_ch, dim3(grid1(p2 * 32)), dim3(256), 0, s, G[T_C2], 96, 64, G[T_S2], 32, 0, p2, 32, 0);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(p3 * 64)), dim3(256), 0, s, G[T_B3], A[T_B3], p3, 64, 64);
    conv_bwd<T>(u, 5, A[T_A3], 64, H / 4, nb, G[T_B3], G[T_A3], 64, false);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(p3 * 64)), dim3(256), 0, s, G[T_A3], A[T_A3], p3, 64, 64);
    conv_bwd<T>(u, 4, A[T_P2], 32, H / 4, nb, G[T_A3], G[T_P2], 32, false);
    // pool 2 feeds S2, which also went to concat 2
    hipLaunchKernelGGL(k_pool_bwd, dim3(grid1(p2 * 32)), dim3(256), 0, s, G[T_P2], H / 2, H / 2, 32, nb, G[T_S2], 1);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(p2 * 32)), dim3(256), 0, s, G[T_S2], A[T_S2], p2, 32, 32);
    conv_bwd<T>(u, 3, A[T_A2], 32, H / 2, nb, G[T_S2], G[T_A2], 32, false);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(p2 * 32)), dim3(256), 0, s, G[T_A2], A[T_A2], p2, 32, 32);
    conv_bwd<T>(u, 2, A[T_P1], 16, H / 2, nb, G[T_A2], G[T_P1], 16, false);
    hipLaunchKernelGGL(k_pool_bwd, dim3(grid1(p1 * 16)), dim3(256), 0, s, G[T_P1], H, H, 16, nb, G[T_S1], 1);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(p1 * 16)), dim3(256), 0, s, G[T_S1], A[T_S1], p1, 16, 16);
    conv_bwd<T>(u, 1, A[T_A1], 16, H, nb, G[T_S1], G[T_A1], 16, false);
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(p1 * 16)), dim3(256), 0, s, G[T_A1], A[T_A1], p1, 16, 16);
    conv_bwd<T>(u, 0, A[T_X0], 2, H, nb, G[T_A1], nullptr, 0, false);
}

template <typename T>
static void refresh_t(fl_unet u, float lr) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)u->step), c2 = 1.f - powf(b2, (float)u->step);
    long off = 0;
    for (size_t li = 0; li < u->conv.size(); ++li) {
        const Conv &c = u->conv[li];
        const long n = (long)c.cout * c.K;
        hipLaunchKernelGGL(k_adam<T>, dim3(grid1(n)), dim3(256), 0, u->s, u->w + off, u->m + off, u->v + off,
                           u->g + u->wb_off[li], c.cout, c.K, c.Kp, c.coutp, lr, b1, b2, 1e-8f,
                           c1 > 0.f ? c1 : 1.f, c2 > 0.f ? c2 : 1.f, wb_of<T>(u, li), wt_of<T>(u, li));
        off += n;
    }
}
// one workgroup per 8 x 8 tile of output pixels and sample; grids of fewer
// than 512 tiles also split the output channels, one 16-channel tile each
template <typename T, int MODE, int KS, int CIN, int COUTP>
static void conv_fused_launch(fl_unet u, int li, const ConvSrc &src, int h, int nb, float *Y, bool relu) {
    const int tiles = ((h + 7) / 8) * ((h + 7) / 8) * nb;
    constexpr int NS = COUTP / 16;
    if (NS > 1 && tiles < 512) {
        dim3 g((h + 7) / 8, (h + 7) / 8, nb * NS);
        hipLaunchKernelGGL((k_conv_fused<T, MODE, KS, CIN, COUTP, NS>), g, dim3(256), 0, u->s, src, h, h,
                           wb_of<T>(u, li), Y, relu ? 1 : 0);
    } else {
        dim3 g((h + 7) / 8, (h + 7) / 8, nb);
        hipLaunchKernelGGL((k_conv_fused<T, MODE, KS, CIN, COUTP, 1>), g, dim3(256), 0, u->s, src, h, h,
                           wb_of<T>(u, li), Y, relu ? 1 : 0);
    }
}

// forward for inference: one fused convolution per layer (pooling, upsampling
// and concatenation folded into the operand staging); same results as the
// im2row path (same bf16 operands, same MFMA k order)
template <typename T>
static void net_forward_fused_t(fl_unet u, int nb) {
    const int H = u->H;
    auto *A = u->A.data();
    auto plain = [](const float *a, int cs) { ConvSrc s; s.a = a; s.csa = cs; return s; };
    auto catup = [](const float *a, int csa, const float *b, int csb) {
        ConvSrc s; s.a = a; s.csa = csa; s.ca = csa; s.b = b; s.csb = csb; return s;
    };
    conv_fused_launch<T, SRC_PLAIN, 3, 2, 16>(u, 0, plain(A[T_X0], 2), H, nb, A[T_A1], true);
    conv_fused_launch<T, SRC_PLAIN, 3, 16, 16>(u, 1, plain(A[T_A1], 16), H, nb, A[T_S1], true);
    conv_fused_launch<T, SRC_POOL, 3, 16, 32>(u, 2, plain(A[T_S1], 16), H / 2, nb, A[T_A2], true);
    conv_fused_launch<T, SRC_PLAIN, 3, 32, 32>(u, 3, plain(A[T_A2], 32), H / 2, nb, A[T_S2], true);
    conv_fused_launch<T, SRC_POOL, 3, 32, 64>(u, 4, plain(A[T_S2], 32), H / 4, nb, A[T_A3], true);
    conv_fused_launch<T, SRC_PLAIN, 3, 64, 64>(u, 5, plain(A[T_A3], 64), H / 4, nb, A[T_B3], true);
    conv_fused_launch<T, SRC_CATUP, 3, 96, 32>(u, 6, catup(A[T_B3], 64, A[T_S2], 32), H / 2, nb, A[T_A4], true);
    conv_fused_launch<T, SRC_PLAIN, 3, 32, 32>(u, 7, plain(A[T_A4], 32), H / 2, nb, A[T_B4], true);
    conv_fused_launch<T, SRC_CATUP, 3, 48, 16>(u, 8, catup(A[T_B4], 32, A[T_S1], 16), H, nb, A[T_A5], true);
    conv_fused_launch<T, SRC_PLAIN, 3, 16, 16>(u, 9, plain(A[T_A5], 16), H, nb, A[T_B5], true);
    conv_fused_launch<T, SRC_PLAIN, 1, 16, 16>(u, 10, plain(A[T_B5], 16), H, nb, A[T_Y], false);
}
static void net_forward_fused(fl_unet u, int nb) {
    if (u->fp32) net_forward_fused_t<float>(u, nb);
    else net_forward_fused_t<bf16>(u, nb);
}

// the preconditioner action z = rms(r) * Net(r / rms(r), alpha) for one
// sample in five launches, two convolutions each (the last also the 1x1 head):
// level 0 down, 1 down, 2, 1 up, 0 up; only S1, S2, B3 and B4 go through HBM.
// The kernels take each weight row length (k padded to 16) from the layer shape,
// as fl_unet_create lays the operand copies out.
template <typename T>
static void net_apply_pairs_t(fl_unet u, const PairSrc &io, hipStream_t s) {
    const int H = u->H;
    auto *A = u->A.data();
    auto Wt = [&](int li) { return (const T *)wb_of<T>(u, li); };
    auto grid = [](int h, int ts) { return dim3((h + ts - 1) / ts, (h + ts - 1) / ts, 1); };
    PairSrc p = io;
    hipLaunchKernelGGL((k_conv_pair<T, SRC_RESID, 2, 16, 16, 16, false>), grid(H, 16), dim3(kPairThreads), 0, s, p, H, Wt(0),
                       Wt(1), (const T *)nullptr, A[T_S1]);
    p.c = ConvSrc{};
    p.c.a = A[T_S1];
    p.c.csa = 16;
    hipLaunchKernelGGL((k_conv_pair<T, SRC_POOL, 16, 32, 32, 8, false>), grid(H / 2, 8), dim3(kPairThreads), 0, s, p, H / 2,
                       Wt(2), Wt(3), (const T *)nullptr, A[T_S2]);
    p.c.a = A[T_S2];
    p.c.csa = 32;
    hipLaunchKernelGGL((k_conv_pair<T, SRC_POOL, 32, 64, 64, 8, false>), grid(H / 4, 8), dim3(kPairThreads), 0, s, p, H / 4,
                       Wt(4), Wt(5), (const T *)nullptr, A[T_B3]);
    p.c.a = A[T_B3];
    p.c.csa = 64;
    p.c.ca = 64;
    p.c.b = A[T_S2];
    p.c.csb = 32;
    hipLaunchKernelGGL((k_conv_pair<T, SRC_CATUP, 96, 32, 32, 8, false>), grid(H / 2, 8), dim3(kPairThreads), 0, s, p, H / 2,
                       Wt(6), Wt(7), (const T *)nullptr, A[T_B4]);
    p.c.a = A[T_B4];
    p.c.csa = 32;
    p.c.ca = 32;
    p.c.b = A[T_S1];
    p.c.csb = 16;
    hipLaunchKernelGGL((k_conv_pair<T, SRC_CATUP, 48, 16, 16, 16, true>), grid(H, 16), dim3(kPairThreads), 0, s, p, H, Wt(8),
                       Wt(9), Wt(10), (float *)nullptr);
}

static void net_forward(fl_unet u, int nb) {
    if (u->fp32) net_forward_t<float>(u, nb);
    else net_forward_t<bf16>(u, nb);
}
static void net_backward(fl_unet u, int nb) {
    if (u->fp32) net_backward_t<float>(u, nb);
    else net_backward_t<bf16>(u, nb);
}
static void refresh_bf16(fl_unet u, float lr) {
    if (u->fp32) refresh_t<float>(u, lr);
    else refresh_t<bf16>(u, lr);
}

// forward on A[T_X0] (nb samples); with targets in A[T_TGT]: loss, backward and,
// for lr > 0, one Adam step.  ops (per sample, may be NULL) selects the
// energy-norm loss ||y - t||_A^2 / ||t||_A^2 instead of the relative L2 loss,
// or with `residual` the target-free loss ||A y - x0||^2 / ||x0||^2.
static fl_status train_step(fl_unet u, int nb, bool with_target, float lr, const fl_op *ops = nullptr,
                            bool residual = false) {
    const long pix = (long)u->H * u->W;
    hipStream_t s = u->s;
    if (!with_target) {  // inference: fused convolutions
        net_forward_fused(u, nb);
        return FL_OK;
    }
    net_forward(u, nb);
    if (ops && residual) {
        float *b0 = u->ebuf, *b1 = u->ebuf + pix;
        for (int z = 0; z < nb; ++z) {
            const int n = ops[z]->n;
            const float *Yz = u->A[T_Y] + z * pix * 16, *Xz = u->A[T_X0] + z * pix * 2;
            hipLaunchKernelGGL(k_res_compact, dim3(grid1((long)n * n)), dim3(256), 0, s, Yz, 16, n, u->W, b0);
            FL_TRY(matvec<float>(ops[z], b0, b1, s));
            hipLaunchKernelGGL(k_res_loss, dim3(1), dim3(256), 0, s, b1, Xz, n, u->W, u->lossbuf + z,
                               u->ltot + 2 * z + 1);
            FL_TRY(matvec<float>(ops[z], b1, b0, s));
            hipLaunchKernelGGL(k_energy_grad, dim3(grid1(pix * 16)), dim3(256), 0, s, b0, u->ltot + 2 * z + 1, n,
                               u->H, u->W, nb, u->G[T_Y] + z * pix * 16, 16);
        }
    } else if (ops) {
        float *d = u->ebuf, *Ad = u->ebuf + pix;
        for (int z = 0; z < nb; ++z) {
            const int n = ops[z]->n;
            const float *Yz = u->A[T_Y] + z * pix * 16, *Tz = u->A[T_TGT] + z * pix, *Xz = u->A[T_X0] + z * pix * 2;
            hipLaunchKernelGGL(k_energy_diff, dim3(grid1((long)n * n)), dim3(256), 0, s, Yz, 16, Tz, n, u->W, d);
            FL_TRY(matvec<float>(ops[z], d, Ad, s));
            hipLaunchKernelGGL(k_energy_loss, dim3(1), dim3(256), 0, s, d, Ad, Tz, Xz, n, u->W, u->lossbuf + z,
                               u->ltot + 2 * z + 1);
            hipLaunchKernelGGL(k_energy_grad, dim3(grid1(pix * 16)), dim3(256), 0, s, Ad, u->ltot + 2 * z + 1, n,
                               u->H, u->W, nb, u->G[T_Y] + z * pix * 16, 16);
        }
    } else {
        const int nblk = 64;
        hipLaunchKernelGGL(k_loss_sums, dim3(nblk, nb), dim3(256), 0, s, u->A[T_Y], 16, u->A[T_TGT], pix, u->lpart);
        hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, u->lpart, nblk, nb, u->ltot, u->lossbuf);
        hipLaunchKernelGGL(k_loss_grad, dim3(grid1(nb * pix * 16)), dim3(256), 0, s, u->A[T_Y], 16, u->A[T_TGT], pix,
                           nb, u->ltot, u->G[T_Y]);
    }
    net_backward(u, nb);
    if (lr > 0.f) {
        u->step += 1;
        refresh_bf16(u, lr);
    }
    return FL_OK;
}

}  // namespace fl

using namespace fl;

extern "C" {

fl_status fl_unet_create(int H, int max_batch, unsigned long long seed, int fp32_operands, fl_unet *out) {
    if (!out || H < 16 || H % 16 != 0 || H > 2048 || max_batch < 1 || max_batch > 256) {
        set_error("fl_unet_create: H must be a multiple of 16 in [16, 2048] and max_batch in [1, 256]");
        return FL_E_INVAL;
    }
    fl_unet u = new (std::nothrow) fl_unet_s();
    if (!u) return FL_E_NOMEM;
    u->H = u->W = H;
    u->nb = max_batch;
    u->fp32 = fp32_operands ? 1 : 0;
    u->osz = u->fp32 ? sizeof(float) : sizeof(bf16);
    const int spec[11][3] = {{2, 16, 3},  {16, 16, 3}, {16, 32, 3}, {32, 32, 3}, {32, 64, 3}, {64, 64, 3},
                             {96, 32, 3}, {32, 32, 3}, {48, 16, 3}, {16, 16, 3}, {16, 1, 1}};
    long wbo = 0, wto = 0;
    for (auto &sp : spec) {
        Conv c;
        c.cin = sp[0];
        c.cout = sp[1];
        c.ks = sp[2];
        c.K = c.ks * c.ks * c.cin;
        c.Kp = (c.K + 15) / 16 * 16;
        c.coutp = (c.cout + 15) / 16 * 16;
        c.woff = u->nparam;
        u->nparam += (long)c.cout * c.K;
        u->wb_off.push_back(wbo);
        u->wt_off.push_back(wto);
        wbo += (long)c.coutp * c.Kp;
        wto += (long)c.Kp * c.coutp;
        u->conv.push_back(c);
    }
    u->wb_len = wbo;
    u->wt_len = wto;
    // He-style initialisation (seeded, host), kept in FP32 master copies
    std::vector<float> w(u->nparam);
    std::mt19937_64 rng(seed);
    for (auto &c : u->conv) {
        std::normal_distribution<float> nd(0.f, sqrtf(2.f / (float)c.K) * (c.ks == 1 ? 0.02f : 1.f));
        for (long i = 0; i < (long)c.cout * c.K; ++i) w[c.woff + i] = nd(rng);
    }
    // activations
    const long p1 = (long)max_batch * H * H;
    size_t total = 0;
    std::vector<size_t> sizes(T_COUNT);
    for (int t = 0; t < T_COUNT; ++t) {
        TShape sh = tshape(u, t);
        sizes[t] = (size_t)max_batch * sh.h * sh.h * sh.c;
        total += sizes[t];
    }
    u->act_bytes = sizeof(float) * total * 2;
    size_t maxrow = 0, maxcol = 0, maxpart = 0;
    for (size_t li = 0; li < u->conv.size(); ++li) {
        const int h = li < 2 || li >= 8 ? H : (li < 4 || (li >= 6 && li < 8) ? H / 2 : H / 4);
        const long pix = (long)max_batch * h * h;
        const Conv &c = u->conv[li];
        maxrow = std::max(maxrow, (size_t)(pix * c.Kp));
        maxcol = std::max(maxcol, (size_t)(pix * c.Kp));
        maxpart = std::max(maxpart, (size_t)(cdiv_i(pix, 2048)) * c.coutp * c.Kp);
    }
    u->row_elems = maxrow;
    u->col_elems = maxcol;
    u->part_elems = maxpart;
    hipError_t e = hipSuccess;
    auto AL = [&](void **p, size_t b) {
        if (e == hipSuccess) e = hipMalloc(p, b);
    };
    AL((void **)&u->w, sizeof(float) * u->nparam);
    AL((void **)&u->m, sizeof(float) * u->nparam);
    AL((void **)&u->v, sizeof(float) * u->nparam);
    AL((void **)&u->g, sizeof(float) * u->wb_len);
    AL(&u->wb, u->osz * u->wb_len);
    AL(&u->wt, u->osz * u->wt_len);
    AL((void **)&u->act, u->act_bytes);
    AL(&u->rowbuf, u->osz * maxrow);
    AL(&u->tbuf, u->osz * std::max(maxrow, (size_t)p1 * 16));
    AL(&u->tbuf2, u->osz * (size_t)p1 * 64);
    AL((void **)&u->colbuf, sizeof(float) * maxcol);
    AL((void **)&u->part, sizeof(float) * maxpart);
    AL((void **)&u->lossbuf, sizeof(float) * max_batch);
    AL((void **)&u->lpart, sizeof(float) * 2 * 64 * max_batch);
    AL((void **)&u->ltot, sizeof(float) * 2 * max_batch);
    AL((void **)&u->nrm, sizeof(double) * 8);
    AL((void **)&u->sqpart, sizeof(double) * kSqParts);
    AL((void **)&u->idx, sizeof(long) * max_batch);
    AL((void **)&u->ebuf, sizeof(float) * 2 * (size_t)H * H);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&u->s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&u->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        set_error("fl_unet_create: %s", hipGetErrorString(e));
        fl_unet_destroy(u);
        return FL_E_NOMEM;
    }
    float *base = u->act;
    for (int t = 0; t < T_COUNT; ++t) {
        u->A.push_back(base);
        base += sizes[t];
    }
    for (int t = 0; t < T_COUNT; ++t) {
        u->G.push_back(base);
        base += sizes[t];
    }
    if (hipMemcpy(u->w, w.data(), sizeof(float) * u->nparam, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemsetAsync(u->m, 0, sizeof(float) * u->nparam, u->s) != hipSuccess ||
        hipMemsetAsync(u->v, 0, sizeof(float) * u->nparam, u->s) != hipSuccess ||
        hipMemsetAsync(u->g, 0, sizeof(float) * u->wb_len, u->s) != hipSuccess ||
        hipMemsetAsync(u->wb, 0, u->osz * u->wb_len, u->s) != hipSuccess ||
        hipMemsetAsync(u->wt, 0, u->osz * u->wt_len, u->s) != hipSuccess ||
        hipMemsetAsync(u->act, 0, u->act_bytes, u->s) != hipSuccess) {
        fl_unet_destroy(u);
        set_error("fl_unet_create: initialisation failed");
        return FL_E_DEVICE;
    }
    refresh_bf16(u, 0.f);
    if (hipStreamSynchronize(u->s) != hipSuccess) {
        fl_unet_destroy(u);
        return FL_E_DEVICE;
    }
    *out = u;
    return FL_OK;
}

fl_status fl_unet_destroy(fl_unet u) {
    if (!u) return FL_OK;
    for (void *p : {(void *)u->w, (void *)u->m, (void *)u->v, (void *)u->g, (void *)u->wb, (void *)u->wt,
                    (void *)u->act, (void *)u->rowbuf, (void *)u->tbuf, (void *)u->tbuf2, (void *)u->colbuf,
                    (void *)u->part, (void *)u->lossbuf, (void *)u->lpart, (void *)u->ltot, (void *)u->nrm, (void *)u->sqpart, (void *)u->idx, (void *)u->ebuf})
        if (p) (void)hipFree(p);
    if (u->s) (void)hipStreamDestroy(u->s);
    if (u->ev) (void)hipEventDestroy(u->ev);
    delete u;
    return FL_OK;
}

fl_status fl_unet_num_params(fl_unet u, long long *n) {
    if (!u || !n) return FL_E_INVAL;
    *n = u->nparam;
    return FL_OK;
}

// weights (fp32 master, layer by layer, each [cout][K] with k = (ky*ks + kx)*cin + ci)
fl_status fl_unet_get_weights(fl_unet u, float *w_host) {
    if (!u || !w_host) return FL_E_INVAL;
    FL_HIP_TRY(hipStreamSynchronize(u->s));
    FL_HIP_TRY(hipMemcpy(w_host, u->w, sizeof(float) * u->nparam, hipMemcpyDeviceToHost));
    return FL_OK;
}

fl_status fl_unet_set_weights(fl_unet u, const float *w_host) {
    if (!u || !w_host) return FL_E_INVAL;
    FL_HIP_TRY(hipStreamSynchronize(u->s));
    FL_HIP_TRY(hipMemcpy(u->w, w_host, sizeof(float) * u->nparam, hipMemcpyHostToDevice));
    refresh_bf16(u, 0.f);
    FL_HIP_TRY(hipStreamSynchronize(u->s));
    return FL_OK;
}

// forward (and optionally backward) on nb samples: x [nb][H][W][2] fp32 NHWC
// device input, y out [nb][H][W] (channel 0), t (may be NULL) targets
// [nb][H][W]; with t: loss per sample to loss_host (may be NULL) and weight
// gradients (fp32, layer by layer as the weights) to grad_host (may be NULL);
// lr > 0 additionally takes one Adam step.
fl_status fl_unet_step(fl_unet u, int nb, const float *x, const float *t, float *y, float lr, float *loss_host,
                       float *grad_host) {
    if (!u || !x || nb < 1 || nb > u->nb) { set_error("fl_unet_step: bad argument"); return FL_E_INVAL; }
    const int H = u->H;
    const long pix = (long)H * H;
    hipStream_t s = u->s;
    FL_HIP_TRY(hipMemcpyAsync(u->A[T_X0], x, sizeof(float) * nb * pix * 2, hipMemcpyDeviceToDevice, s));
    if (t) FL_HIP_TRY(hipMemcpyAsync(u->A[T_TGT], t, sizeof(float) * nb * pix, hipMemcpyDeviceToDevice, s));
    FL_TRY(train_step(u, nb, t != nullptr, lr));
    if (y)
        hipLaunchKernelGGL(k_copy_ch, dim3(grid1(nb * pix)), dim3(256), 0, s, u->A[T_Y], 16, 0, y, 1, 0, nb * pix, 1, 0);
    FL_HIP_TRY(hipGetLastError());
    FL_HIP_TRY(hipStreamSynchronize(s));
    if (t && loss_host) FL_HIP_TRY(hipMemcpy(loss_host, u->lossbuf, sizeof(float) * nb, hipMemcpyDeviceToHost));
    if (t && grad_host) {
        std::vector<float> gp(u->wb_len);
        FL_HIP_TRY(hipMemcpy(gp.data(), u->g, sizeof(float) * u->wb_len, hipMemcpyDeviceToHost));
        for (size_t li = 0; li < u->conv.size(); ++li) {
            const Conv &c = u->conv[li];
            for (int co = 0; co < c.cout; ++co)
                for (int k = 0; k < c.K; ++k) grad_host[c.woff + (long)co * c.K + k] = gp[u->wb_off[li] + (long)co * c.Kp + k];
        }
    }
    return FL_OK;
}

fl_status fl_unet_pack(fl_unet u, int count, const double *const *r, const double *const *sol, const double *alpha,
                       int n, float *x, float *t) {
    if (!u || count < 0 || (count > 0 && (!r || !alpha || !x)) || n < 1 || n > u->H) {
        set_error("fl_unet_pack: bad argument");
        return FL_E_INVAL;
    }
    const long pix = (long)u->H * u->W;
    for (int z = 0; z < count; ++z) {
        if (!r[z]) { set_error("fl_unet_pack: NULL residual"); return FL_E_INVAL; }
        hipLaunchKernelGGL(k_sumsq_part, dim3(kSqParts), dim3(256), 0, u->s, r[z], (long)n * n, u->sqpart);
        hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(64), 0, u->s, u->sqpart, kSqParts, u->nrm);
        hipLaunchKernelGGL(k_pack_sample, dim3(grid1(pix)), dim3(256), 0, u->s, r[z], sol ? sol[z] : nullptr, n, u->H,
                           u->W, (float)alpha[z], u->nrm, x + z * pix * 2, t ? t + z * pix : nullptr);
    }
    FL_HIP_TRY(hipGetLastError());
    FL_HIP_TRY(hipStreamSynchronize(u->s));
    return FL_OK;
}

fl_status fl_unet_train(fl_unet u, long count, const float *x, const float *t, const fl_op *ops, int epochs,
                        int batch, float lr, float lr_final, unsigned long long seed, float *epoch_loss) {
    if (!u || !x || (!t && !ops) || count < 1 || epochs < 1 || batch < 1 || batch > u->nb || !(lr > 0.f) ||
        lr_final < 0.f) {
        set_error("fl_unet_train: bad argument");
        return FL_E_INVAL;
    }
    if (ops)
        for (long i = 0; i < count; ++i)
            if (!ops[i] || ops[i]->d != 2 || ops[i]->n > u->H) {
                set_error("fl_unet_train: sample %ld needs a 2D operator with n <= %d", i, u->H);
                return FL_E_INVAL;
            }
    std::vector<fl_op> bops(batch);
    const long pix = (long)u->H * u->W;
    const long steps_per_epoch = count / batch;  // the ragged remainder of a shuffled epoch is dropped
    if (steps_per_epoch < 1) { set_error("fl_unet_train: fewer samples than one batch"); return FL_E_INVAL; }
    std::mt19937_64 rng(seed);
    std::vector<long> order(count);
    std::vector<float> lossh(batch);
    const long total_steps = steps_per_epoch * epochs;
    long done = 0;
    for (int e = 0; e < epochs; ++e) {
        for (long i = 0; i < count; ++i) order[i] = i;
        for (long i = count - 1; i > 0; --i) std::swap(order[i], order[(long)(rng() % (unsigned long long)(i + 1))]);
        double acc = 0.0;
        for (long b = 0; b < steps_per_epoch; ++b, ++done) {
            // cosine decay from lr to lr_final over all steps
            const double ph = (double)done / (double)total_steps;
            const float lr_k = (float)(lr_final + 0.5 * (lr - lr_final) * (1.0 + std::cos(M_PI * ph)));
            FL_HIP_TRY(hipMemcpyAsync(u->idx, order.data() + b * batch, sizeof(long) * batch, hipMemcpyHostToDevice,
                                      u->s));
            hipLaunchKernelGGL(k_gather, dim3(grid1(batch * pix * 2)), dim3(256), 0, u->s, x, u->idx, batch, pix * 2,
                               u->A[T_X0]);
            if (t)
                hipLaunchKernelGGL(k_gather, dim3(grid1(batch * pix)), dim3(256), 0, u->s, t, u->idx, batch, pix,
                                   u->A[T_TGT]);
            if (ops)
                for (int z = 0; z < batch; ++z) bops[z] = ops[order[b * batch + z]];
            FL_TRY(train_step(u, batch, true, lr_k, ops ? bops.data() : nullptr, t == nullptr));
            FL_HIP_TRY(hipMemcpyAsync(lossh.data(), u->lossbuf, sizeof(float) * batch, hipMemcpyDeviceToHost, u->s));
            FL_HIP_TRY(hipStreamSynchronize(u->s));
            for (int z = 0; z < batch; ++z) acc += lossh[z];
        }
        if (epoch_loss) epoch_loss[e] = (float)(acc / (double)(steps_per_epoch * batch));
        if (!std::isfinite(acc)) { set_error("fl_unet_train: loss is not finite"); return FL_E_BREAKDOWN; }
    }
    FL_HIP_TRY(hipGetLastError());
    return FL_OK;
}

}  // extern "C"

namespace fl {
int unet_size(fl_unet u) { return u->H; }
// z = rms(r) * Net(r / rms(r), alpha) on the stream s (r, z: n x n, n <= H), with
// rr_dev the squared norm of r on the device.  Used inside flexible PCG.
fl_status unet_apply(fl_unet u, const double *r, int n, double alpha, double *z, const double *rr_dev,
                     hipStream_t s) {
    PairSrc io;
    io.r = r;
    io.nrm = rr_dev;
    io.n = n;
    io.alpha = (float)alpha;
    io.z = z;
    // on the caller's stream: the action is ordered with the solver's own work
    if (u->fp32) net_apply_pairs_t<float>(u, io, s);
    else net_apply_pairs_t<bf16>(u, io, s);
    FL_HIP_TRY(hipGetLastError());
    return FL_OK;
}
}  // namespace fl

namespace fl {
// GEMM check: C[M][N] = A[M][K] B[N][K]^T with operands rounded to the
// operand type; kchunk < K runs the split-K path with its fixed-order reduction
template <typename T>
static fl_status gemm_test(int M, int N, int K, int kchunk, const float *A_host, const float *B_host, float *C_host) {
    float *a = nullptr, *b = nullptr, *c = nullptr, *part = nullptr;
    T *ab = nullptr, *bb = nullptr;
    const int splits = (K + kchunk - 1) / kchunk;
    hipError_t e = hipSuccess;
    auto AL = [&](void **p, size_t n) {
        if (e == hipSuccess) e = hipMalloc(p, n);
    };
    AL((void **)&a, sizeof(float) * M * K);
    AL((void **)&b, sizeof(float) * N * K);
    AL((void **)&c, sizeof(float) * M * N);
    AL((void **)&part, sizeof(float) * M * N * splits);
    AL((void **)&ab, sizeof(T) * M * K);
    AL((void **)&bb, sizeof(T) * N * K);
    if (e == hipSuccess) e = hipMemcpy(a, A_host, sizeof(float) * M * K, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b, B_host, sizeof(float) * N * K, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_cvt<T>, dim3(grid1((long)M * K)), dim3(256), 0, 0, a, (long)M * K, ab);
        hipLaunchKernelGGL(k_cvt<T>, dim3(grid1((long)N * K)), dim3(256), 0, 0, b, (long)N * K, bb);
        if (splits == 1) {
            launch_gemm<T>(false, false, ab, K, bb, K, c, N, M, N, K, 0);
        } else {
            dim3 g(cdiv_i(M, 64), cdiv_i(N, 64), splits);
            hipLaunchKernelGGL((k_gemm_nt<T, false, false, true>), g, dim3(256), 0, 0, ab, K, bb, K, part, N, M, N, K,
                               kchunk);
            hipLaunchKernelGGL(k_splitk_reduce, dim3(grid1((long)M * N)), dim3(256), 0, 0, part, splits, (long)M * N,
                               (long)M * N, c, 0);
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(C_host, c, sizeof(float) * M * N, hipMemcpyDeviceToHost);
    for (void *p : {(void *)a, (void *)b, (void *)c, (void *)part, (void *)ab, (void *)bb})
        if (p) (void)hipFree(p);
    if (e != hipSuccess) {
        set_error("fl_gemm_test: %s", hipGetErrorString(e));
        return FL_E_DEVICE;
    }
    return FL_OK;
}

}  // namespace fl

extern "C" {

fl_status fl_unet_apply(fl_unet u, const double *r, int n, double alpha, double *z, void *stream) {
    if (!u || !r || !z || n < 1 || n > u->H) { set_error("fl_unet_apply: bad argument"); return FL_E_INVAL; }
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_sumsq_part, dim3(kSqParts), dim3(256), 0, s, r, (long)n * n, u->sqpart);
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(64), 0, s, u->sqpart, kSqParts, u->nrm);
    FL_TRY(unet_apply(u, r, n, alpha, z, u->nrm, s));
    return FL_OK;
}

fl_status fl_gemm_test(int M, int N, int K, int kchunk, int fp32_operands, const float *A_host, const float *B_host,
                       float *C_host) {
    if (M % 16 || N % 16 || K % 16 || M <= 0 || N <= 0 || K <= 0 || kchunk <= 0 || kchunk % 16 || !A_host ||
        !B_host || !C_host || (long)M * K > (1L << 26) || (long)N * K > (1L << 26) || (long)M * N > (1L << 26)) {
        set_error("fl_gemm_test: sizes must be positive multiples of 16 (at most 2^26 elements per matrix)");
        return FL_E_INVAL;
    }
    return fp32_operands ? gemm_test<float>(M, N, K, kchunk, A_host, B_host, C_host)
                         : gemm_test<bf16>(M, N, K, kchunk, A_host, B_host, C_host);
}

}  // extern "C"
