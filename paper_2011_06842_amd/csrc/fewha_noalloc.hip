// fewha_apply_A_noalloc (include/fewha.h): y = M x for callers that cannot allocate device
// memory.  The operator's intermediates live in one file-scope device array per GPU instead of
// the context's workspace; the kernels are the operator's own (they take the array's address
// as they take the workspace buffers in fewha_apply_A).
#include <hip/hip_runtime.h>

#include <mutex>

#include "fewha_internal.h"

namespace fewha {

namespace {

// The operator intermediates of fewha_apply_A_noalloc: one fixed array per GPU, held until the
// process ends.  On the host this name only stands for the symbol (a kernel given it would
// fault), so its device address is taken once per device (scratch_init) and used instead.
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` per device (null: not taken yet)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

fewha_status scratch_init(const char** err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *err = "no current HIP device (or more than 64 devices)";
        return FEWHA_E_HIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return FEWHA_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        *err = "hipGetSymbolAddress of the static scratch array failed";
        return FEWHA_E_HIP;
    }
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
    return FEWHA_OK;
}

}  // namespace fewha

namespace {

// Errors of the entry point carry static messages: nothing is allocated on any of its paths.
fewha_status fail_static(fewha_ctx* ctx, fewha_status st, const char* msg) {
    if (ctx) ctx->c.err_lit = msg;
    return st;
}

}  // namespace

extern "C" {

fewha_status fewha_apply_A_noalloc(fewha_ctx* ctx, const void* d_x, void* d_y, void* stream) {
    using namespace fewha;
    if (!ctx || !d_x || !d_y) return fail_static(ctx, FEWHA_E_INVAL, "NULL argument");
    if (d_x == d_y) return fail_static(ctx, FEWHA_E_INVAL, "d_y must not alias d_x");
    const Ctx& c = ctx->c;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail_static(ctx, FEWHA_E_HIP, "no current HIP device");
    char* base;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch_ptr[dev];
    }
    if (!base)
        return fail_static(ctx, FEWHA_E_STATE,
                           "the static scratch array of the current device has no address: set up a context on it");
    // nodal image, two wavelet ping-pong buffers and the layer adjoint (N each), sensor nodes
    // (V), weighted slopes of tip/tilt-filtered sensors (S)
    const size_t vN = align256(c.esz * size_t(c.N)), vV = align256(c.esz * size_t(c.V));
    const size_t vS = align256(c.esz * size_t(c.S));
    if (4 * vN + vV + vS > kScratchBytes)
        return fail_static(ctx, FEWHA_E_NOMEM,
                           "the operator's intermediates exceed the 16 MiB static scratch array of "
                           "fewha_apply_A_noalloc (use fewha_apply_A)");
    const OpBufs ob{base, base + vN, base + 2 * vN, base + 3 * vN, base + 3 * vN + vV, base + 4 * vN + vV};
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (c.prec == FEWHA_FP64)
        launch_apply_M<double>(c, static_cast<const double*>(d_x), static_cast<double*>(d_y), nullptr, s, &ob);
    else
        launch_apply_M<float>(c, static_cast<const float*>(d_x), static_cast<float*>(d_y), nullptr, s, &ob);
    if (hipGetLastError() != hipSuccess) return fail_static(ctx, FEWHA_E_HIP, "kernel launch failed");
    return FEWHA_OK;
}

}  // extern "C"
