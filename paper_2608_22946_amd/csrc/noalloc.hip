// Allocation-free variant of the Krylov multi-dot (helm_vec_dots_static).
//
// The reduction kernel of helm_vec_dots needs device memory beyond its inputs
// and outputs: one slot of partial sums per block and a completion ticket.
// Here that memory is a file-scope static device array, so the call performs
// no hipMalloc / hipFree and allocates nothing else (callers under HIP graph
// capture, tight serving loops, harnesses that forbid allocation).  Each GPU
// holds its own copy of the array until the process ends; its address on a
// device is taken once, with that device current, by hipGetSymbolAddress, and
// only that address is handed to kernels (the array's name is a host-side
// stand-in in host code).
#include <mutex>

#include "helm_internal.h"

namespace {

// partial sums of at most kRedMaxBlocks reduction blocks x kRedSlots complex slots, then the ticket
constexpr size_t kPartialBytes = (size_t)helm::kRedMaxBlocks * 2 * helm::kRedSlots * sizeof(double);
constexpr size_t kCounterOffset = (kPartialBytes + 255) & ~(size_t)255;
constexpr size_t kScratchBytes = kCounterOffset + 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static_assert(kScratchBytes <= 192 * 1024, "the static scratch array stays at most 192 KiB per GPU");

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_ptr[kMaxDevices];          // device address of `scratch` on each device (null until first use)

helm_status fail(helm_status st, const char *msg) { return helm::thread_error(st, msg); }

// address of this device's copy of the array (looked up once per device, with the device current)
hipError_t scratch_ptr(int dev, void **out) {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

template <typename T>
hipError_t run(void *base, int k, const void *const *V, const void *w, long long n, double *out, hipStream_t s) {
    helm::RedBuf rb;
    rb.partials = static_cast<double *>(base);
    rb.counter = reinterpret_cast<unsigned *>(static_cast<char *>(base) + kCounterOffset);
    // the ticket must start at zero: cleared by a fill kernel (no memset node under capture)
    hipError_t e = helm::launch_fill_zero<helm::c32>(reinterpret_cast<helm::c32 *>(rb.counter), 256 / sizeof(helm::c32), s);
    if (e != hipSuccess) return e;
    return helm::launch_dots<T>(reinterpret_cast<const T *const *>(V), k, static_cast<const T *>(w), true, n,
                                helm::EPI_STORE, nullptr, 0, out, rb, s);
}

}  // namespace

extern "C" {

helm_status helm_vec_dots_static(int precision, long long n, int k, const void *const *V, const void *w,
                                 double *out, void *stream) {
    if (precision != HELM_FP32 && precision != HELM_FP64) return fail(HELM_EINVAL, "precision must be HELM_FP32 or HELM_FP64");
    if (n < 1 || n > (1LL << 40)) return fail(HELM_EINVAL, "n must be in 1..2^40");
    if (k < 0 || k > helm::kMMax) return fail(HELM_EINVAL, "k must be in 0..12");
    if ((k > 0 && !V) || !w || !out) return fail(HELM_EINVAL, "V (for k > 0), w and out must not be NULL");
    for (int j = 0; j < k; ++j)
        if (!V[j]) return fail(HELM_EINVAL, "V holds a NULL pointer");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(HELM_EHIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(HELM_EINVAL, "device index beyond 63");
    void *base = nullptr;
    if ((e = scratch_ptr(dev, &base)) != hipSuccess) return fail(HELM_EHIP, hipGetErrorString(e));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    e = (precision == HELM_FP64) ? run<helm::c64>(base, k, V, w, n, out, s) : run<helm::c32>(base, k, V, w, n, out, s);
    if (e != hipSuccess) return fail(HELM_EHIP, hipGetErrorString(e));
    return HELM_OK;
}

}  // extern "C"
