// fl_noalloc.hip -- the matvec y = A u for callers that cannot allocate device
// memory: the same passes and kernel variant as fl_apply, with the spectra
// workspaces taken from one statically sized device array per GPU instead of
// the operator's own.
//
// The array is a file-scope __device__ variable.  Its device address is
// looked up once per GPU (hipGetSymbolAddress, with that GPU current) on the
// first call there, and only that looked-up address is handed to kernels.
// Every call on a GPU shares that GPU's array: calls that overlap in time on
// one GPU (different streams, or different host threads) race on it.  The
// matvec writes every workspace entry it later reads, so nothing is cleared
// between calls.
#include <mutex>

#include "fl_internal.hpp"

namespace fl {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static void *g_scratch_dev[kMaxDevices];  // device address of `scratch`, per GPU
static std::mutex g_scratch_mu;

// device address of this GPU's copy of `scratch` (looked up on first use)
static fl_status scratch_address(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d outside the %d devices the static workspace serves", dev, kMaxDevices);
        return FL_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int prev = 0;
        FL_HIP_TRY(hipGetDevice(&prev));
        if (prev != dev) FL_HIP_TRY(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != dev) (void)hipSetDevice(prev);
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            return FL_E_DEVICE;
        }
        g_scratch_dev[dev] = p;
    }
    *out = (unsigned char *)g_scratch_dev[dev];
    return FL_OK;
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// the spectra workspaces of one matvec of the selected variant: T1 holds the
// row pass's tiled half spectra (rows = ny nz lines), T2 (3D) the y pass's
// (nz lines of P y frequencies), each nt tiles of C columns per line
template <typename T>
static fl_status workspace_bytes(fl_op op, int prec, int variant, size_t *t1, size_t *t2) {
    const VariantDesc v = variant_desc(op, prec, variant);
    if (v.c < 1) {
        set_error("no kernel variant %d for FFT length %d, d=%d", variant, op->P, op->d);
        return FL_E_UNSUPPORTED;
    }
    const size_t cols = (size_t)((spec_cols(op->d, op->P) + v.c - 1) / v.c) * v.c;
    const size_t es = sizeof(C2<T>);
    *t1 = op->d == 1 ? 0 : es * cols * op->nk[1] * op->nk[2];
    *t2 = op->d == 3 ? es * cols * op->nk[2] * op->P : 0;
    return FL_OK;
}

template <typename T>
static fl_status apply_static(fl_op op, const T *u, T *y, int prec, hipStream_t s) {
    const int variant = prec == FL_FP64 ? op->var64 : op->var32;
    size_t t1 = 0, t2 = 0;
    FL_TRY(workspace_bytes<T>(op, prec, variant, &t1, &t2));
    const size_t need = round256(t1) + t2;
    if (need > kScratchBytes) {
        set_error("this matvec needs %zu bytes of workspace; the static workspace holds %zu (64 MiB)", need,
                  kScratchBytes);
        return FL_E_INVAL;
    }
    unsigned char *base = nullptr;
    FL_TRY(scratch_address(op->device, &base));
    MvCtx<T> cx = single_ctx<T>(op);
    cx.T1 = t1 ? base : nullptr;
    cx.T2 = t2 ? base + round256(t1) : nullptr;
    return matvec_ctx<T>(cx, variant, u, y, Epi<T>{}, nullptr, s);
}

}  // namespace fl

using namespace fl;

extern "C" fl_status fl_apply_noalloc(fl_op op, const void *u, void *y, int prec, void *stream) {
    if (!op || !u || !y) { set_error("NULL argument"); return FL_E_INVAL; }
    if (prec != FL_FP64 && prec != FL_FP32) { set_error("prec must be FL_FP64 or FL_FP32"); return FL_E_INVAL; }
    const size_t es = prec == FL_FP64 ? sizeof(double) : sizeof(float);
    const char *a = (const char *)u, *b = (const char *)y;
    if (a < b + es * op->M && b < a + es * op->M) { set_error("u and y overlap"); return FL_E_INVAL; }
    if (large_op(op)) {
        set_error("the static workspace serves FFT lengths up to %d (this operator's is %d)", kMaxLdsP, op->P);
        return FL_E_UNSUPPORTED;
    }
    hipStream_t s = (hipStream_t)stream;
    if (prec == FL_FP64) return apply_static<double>(op, (const double *)u, (double *)y, prec, s);
    return apply_static<float>(op, (const float *)u, (float *)y, prec, s);
}
