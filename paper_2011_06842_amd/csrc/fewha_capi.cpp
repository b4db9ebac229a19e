// C ABI entry points of the augmented-FEWHA library (declared in include/fewha.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>

#include "fewha_internal.h"
#include "../../include/fewha_unet.h"

namespace {

thread_local std::string g_setup_err;
constexpr uint64_t kStateMagic = 0x46455748415354ULL;   // "FEWHAST"

fewha_status fail(fewha_ctx* ctx, fewha_status st, const std::string& msg) {
    if (ctx) {
        ctx->c.err = msg;
        ctx->c.err_lit = nullptr;
    }
    return st;
}


fewha_status check_launch(fewha_ctx* ctx, hipStream_t s) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, FEWHA_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    if (ctx->c.prof.on) {
        const hipError_t p = fewha::profiler_collect(ctx->c, s);
        if (p != hipSuccess) return fail(ctx, FEWHA_E_HIP, std::string("profiler: ") + hipGetErrorString(p));
    }
    return FEWHA_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Status of a frame call whose frame was enqueued: FEWHA_E_BREAKDOWN once for every frame of
// the context found broken down (the end of such a frame writes its number into the pinned
// report word; a frame still running is reported by a later call), else FEWHA_OK.
fewha_status solve_status(fewha_ctx* ctx) {
    fewha::Ctx& c = ctx->c;
    const int64_t seen = *reinterpret_cast<volatile int64_t*>(c.brk_host);
    if (seen > c.brk_reported) {
        c.brk_reported = seen;
        return fail(ctx, FEWHA_E_BREAKDOWN,
                    "frame " + std::to_string(seen) + " of this context broke down (its info flags tell how); "
                    "the carried state kept its last finite values and this call's frame was enqueued");
    }
    return FEWHA_OK;
}

}  // namespace

extern "C" {

fewha_status fewha_workspace_size_batch(const fewha_config* cfgs, int32_t n, size_t* bytes) {
    std::string err;
    const fewha_status st = fewha::validate_batch(cfgs, n, err);
    if (st != FEWHA_OK) {
        g_setup_err = err;
        return st;
    }
    if (!bytes) return FEWHA_E_INVAL;
    *bytes = fewha::compute_layout(cfgs, n).total;
    return FEWHA_OK;
}

fewha_status fewha_workspace_size(const fewha_config* cfg, size_t* bytes) {
    return fewha_workspace_size_batch(cfg, 1, bytes);
}

fewha_status fewha_setup_batch(const fewha_config* cfgs, int32_t n, void* d_workspace, size_t bytes, void* stream,
                               fewha_ctx** out) {
    if (!out) return FEWHA_E_INVAL;
    *out = nullptr;
    std::string err;
    fewha_status st = fewha::validate_batch(cfgs, n, err);
    if (st != FEWHA_OK) {
        g_setup_err = err;
        return st;
    }
    const fewha::Layout lo = fewha::compute_layout(cfgs, n);
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255)) {
        g_setup_err = "workspace must be a 256-byte aligned device pointer";
        return FEWHA_E_INVAL;
    }
    if (bytes < lo.total) {
        g_setup_err = "workspace too small: need " + std::to_string(lo.total) + " bytes";
        return FEWHA_E_NOMEM;
    }
    fewha_ctx* ctx = new (std::nothrow) fewha_ctx();
    if (!ctx) return FEWHA_E_NOMEM;
    fewha::Ctx& c = ctx->c;
    const fewha_config* cfg = &cfgs[0];
    c.prec = cfg->precision;
    c.esz = cfg->precision == FEWHA_FP64 ? 8 : 4;
    c.max_iter = cfg->max_iter;
    c.k = cfg->recycle_k;
    c.mode = cfg->recycle_mode;
    c.project_all = cfg->project_all;
    c.rel_tol = cfg->rel_tol;
    c.ws = static_cast<char*>(d_workspace);
    c.ws_bytes = bytes;
    c.lay = lo;
    hipStream_t s = as_stream(stream);
    // zero the carried state and the scratch vectors
    if (hipMemsetAsync(c.ws + lo.nodal, 0, lo.total - lo.nodal, s) != hipSuccess) {
        g_setup_err = "hipMemsetAsync failed";
        delete ctx;
        return FEWHA_E_HIP;
    }
    st = fewha::build_tables(c, cfgs, n, s);
    if (st != FEWHA_OK) {
        g_setup_err = c.err;
        delete ctx;
        return st;
    }
    // the breakdown report word (pinned host memory the device writes; see solve_status)
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, 256, hipHostMallocMapped) != hipSuccess || hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        if (h) (void)hipHostFree(h);
        g_setup_err = "hipHostMalloc of the breakdown report word failed";
        delete ctx;
        return FEWHA_E_HIP;
    }
    std::memset(h, 0, 256);
    c.brk_host = static_cast<int64_t*>(h);
    c.brk_dev = static_cast<int64_t*>(d);
    // the device address of fewha_apply_A_noalloc's static scratch array on this device
    const char* serr = nullptr;
    if (fewha::scratch_init(&serr) != FEWHA_OK) {
        g_setup_err = serr;
        (void)hipHostFree(h);
        delete ctx;
        return FEWHA_E_HIP;
    }
    *out = ctx;
    return FEWHA_OK;
}

fewha_status fewha_setup(const fewha_config* cfg, void* d_workspace, size_t bytes, void* stream, fewha_ctx** out) {
    return fewha_setup_batch(cfg, 1, d_workspace, bytes, stream, out);
}

fewha_status fewha_instances(const fewha_ctx* ctx, int64_t* coeff_offsets, int64_t* slope_offsets, int32_t n,
                             int32_t* n_out) {
    if (!ctx) return FEWHA_E_INVAL;
    const fewha::Ctx& c = ctx->c;
    for (int i = 0; i <= c.B && i < n; ++i) {
        if (coeff_offsets) coeff_offsets[i] = i < c.B ? c.insts[i].off : c.N;
        if (slope_offsets) slope_offsets[i] = c.s_offs[i];
    }
    if (n_out) *n_out = c.B;
    return FEWHA_OK;
}

fewha_status fewha_sizes(const fewha_ctx* ctx, int64_t* n_coeff, int64_t* n_slopes) {
    if (!ctx) return FEWHA_E_INVAL;
    if (n_coeff) *n_coeff = ctx->c.N;
    if (n_slopes) *n_slopes = ctx->c.S;
    return FEWHA_OK;
}

fewha_status fewha_apply_A(fewha_ctx* ctx, const void* d_x, void* d_y, void* stream) {
    if (!ctx || !d_x || !d_y) return fail(ctx, FEWHA_E_INVAL, "NULL argument");
    if (d_x == d_y) return fail(ctx, FEWHA_E_INVAL, "d_y must not alias d_x");
    const fewha::Ctx& c = ctx->c;
    if (c.prec == FEWHA_FP64)
        fewha::launch_apply_M<double>(c, static_cast<const double*>(d_x), static_cast<double*>(d_y), nullptr,
                                      as_stream(stream));
    else
        fewha::launch_apply_M<float>(c, static_cast<const float*>(d_x), static_cast<float*>(d_y), nullptr,
                                     as_stream(stream));
    return check_launch(ctx, as_stream(stream));
}

fewha_status fewha_rhs(fewha_ctx* ctx, const void* d_s, void* d_b, void* stream) {
    if (!ctx || !d_s || !d_b) return fail(ctx, FEWHA_E_INVAL, "NULL argument");
    const fewha::Ctx& c = ctx->c;
    if (c.prec == FEWHA_FP64)
        fewha::launch_rhs<double>(c, static_cast<const double*>(d_s), static_cast<double*>(d_b), as_stream(stream));
    else
        fewha::launch_rhs<float>(c, static_cast<const float*>(d_s), static_cast<float*>(d_b), as_stream(stream));
    return check_launch(ctx, as_stream(stream));
}

fewha_status fewha_solve_aug(fewha_ctx* ctx, const void* d_s, void* d_c, void* d_info, void* stream) {
    if (!ctx || !d_s) return fail(ctx, FEWHA_E_INVAL, "NULL argument");
    fewha::Ctx& c = ctx->c;
    auto* info = static_cast<fewha_solve_info*>(d_info);
    hipError_t e;
    if (c.prec == FEWHA_FP64)
        e = fewha::launch_solve_frame<double>(c, static_cast<const double*>(d_s), static_cast<double*>(d_c), info,
                                              as_stream(stream));
    else
        e = fewha::launch_solve_frame<float>(c, static_cast<const float*>(d_s), static_cast<float*>(d_c), info,
                                             as_stream(stream));
    if (e != hipSuccess) return fail(ctx, FEWHA_E_HIP, std::string("frame launch failed: ") + hipGetErrorString(e));
    const fewha_status st = check_launch(ctx, as_stream(stream));
    return st != FEWHA_OK ? st : solve_status(ctx);
}

fewha_status fewha_solve_aug_ws(fewha_ctx* ctx, fewha_unet* net, const fewha_warmstart* ws, const void* d_s,
                                void* d_c, void* d_info, void* stream) {
    if (!ctx || !net || !ws || !d_s) return fail(ctx, FEWHA_E_INVAL, "NULL argument");
    fewha::Ctx& c = ctx->c;
    if (c.B != 1) return fail(ctx, FEWHA_E_INVAL, "the warm start needs a single-instance context");
    if (!(ws->scale_c > 0) || !(ws->scale_r > 0) || !std::isfinite(ws->scale_out))
        return fail(ctx, FEWHA_E_INVAL, "bad warm-start scales");
    int32_t images[FEWHA_UNET_MAX_GROUPS], size[FEWHA_UNET_MAX_GROUPS], G = 0;
    fewha_unet_groups(net, images, size, &G);
    int l = 0;
    for (int g = 0; g < G; ++g)
        for (int k = 0; k < images[g]; ++k, ++l)
            if (l >= c.L || c.layers_n[l] != size[g])
                return fail(ctx, FEWHA_E_INVAL, "the network's images do not match the layers");
    if (l != c.L) return fail(ctx, FEWHA_E_INVAL, "the network's images do not match the layers");
    const fewha::WarmStart w{net, ws->scale_c, ws->scale_r, ws->scale_out};
    auto* info = static_cast<fewha_solve_info*>(d_info);
    hipError_t e;
    if (c.prec == FEWHA_FP64)
        e = fewha::launch_solve_frame_ws<double>(c, w, static_cast<const double*>(d_s), static_cast<double*>(d_c), info,
                                                 as_stream(stream));
    else
        e = fewha::launch_solve_frame_ws<float>(c, w, static_cast<const float*>(d_s), static_cast<float*>(d_c), info,
                                                as_stream(stream));
    if (e != hipSuccess) return fail(ctx, FEWHA_E_HIP, std::string("frame launch failed: ") + hipGetErrorString(e));
    const fewha_status st = check_launch(ctx, as_stream(stream));
    return st != FEWHA_OK ? st : solve_status(ctx);
}

fewha_status fewha_warmstart_input(fewha_ctx* ctx, const fewha_warmstart* ws, const void* d_c, const void* d_s,
                                   float* d_in, void* stream) {
    if (!ctx || !ws || !d_c || !d_s || !d_in) return fail(ctx, FEWHA_E_INVAL, "NULL argument");
    const fewha::Ctx& c = ctx->c;
    if (c.B != 1) return fail(ctx, FEWHA_E_INVAL, "the warm start needs a single-instance context");
    if (!(ws->scale_c > 0) || !(ws->scale_r > 0) || !std::isfinite(ws->scale_c) || !std::isfinite(ws->scale_r))
        return fail(ctx, FEWHA_E_INVAL, "bad warm-start scales");
    if (reinterpret_cast<uintptr_t>(d_in) & 15) return fail(ctx, FEWHA_E_INVAL, "d_in must be 16-byte aligned");
    const fewha::WarmStart w{nullptr, ws->scale_c, ws->scale_r, ws->scale_out};
    hipError_t e;
    if (c.prec == FEWHA_FP64)
        e = fewha::launch_ws_input<double>(c, w, static_cast<const double*>(d_c), static_cast<const double*>(d_s), d_in,
                                           as_stream(stream));
    else
        e = fewha::launch_ws_input<float>(c, w, static_cast<const float*>(d_c), static_cast<const float*>(d_s), d_in,
                                          as_stream(stream));
    if (e != hipSuccess) return fail(ctx, FEWHA_E_HIP, std::string("launch failed: ") + hipGetErrorString(e));
    return check_launch(ctx, as_stream(stream));
}

fewha_status fewha_frame_iterations(const fewha_ctx* ctx, int32_t* iters) {
    if (!ctx || !iters) return FEWHA_E_INVAL;
    *iters = ctx->c.frame_iters;
    return FEWHA_OK;
}

fewha_status fewha_reset(fewha_ctx* ctx) {
    if (!ctx) return FEWHA_E_INVAL;
    ctx->c.first = true;
    ctx->c.count = 0;
    ctx->c.last_iters = 0;
    return FEWHA_OK;
}

fewha_status fewha_apply_piece(fewha_ctx* ctx, int32_t piece, const void* d_in, void* d_out, void* stream) {
    if (!ctx || !d_in || !d_out) return fail(ctx, FEWHA_E_INVAL, "NULL argument");
    if (d_in == d_out) return fail(ctx, FEWHA_E_INVAL, "d_out must not alias d_in");
    if ((reinterpret_cast<uintptr_t>(d_in) | reinterpret_cast<uintptr_t>(d_out)) & 15)
        return fail(ctx, FEWHA_E_INVAL, "d_in and d_out must be 16-byte aligned");
    const fewha::Ctx& c = ctx->c;
    hipStream_t s = as_stream(stream);
    auto run = [&](auto tag) {
        using T = decltype(tag);
        const T* in = static_cast<const T*>(d_in);
        T* out = static_cast<T*>(d_out);
        T* psi_n = c.at<T>(c.lay.psi_nodes);
        switch (piece) {
            case FEWHA_PIECE_WINV: fewha::launch_winv<T>(c, in, out, s); break;
            case FEWHA_PIECE_WINVT:
                fewha::launch_winvt<T>(c, in, out, static_cast<const T*>(nullptr), nullptr, s);
                break;
            case FEWHA_PIECE_A: fewha::launch_fwd_slopes<T>(c, in, out, s); break;
            case FEWHA_PIECE_AT:
                fewha::launch_slopes_adj<T>(c, in, psi_n, 0, s);
                fewha::launch_adj_gather<T>(c, psi_n, out, s);
                break;
        }
    };
    if (piece < FEWHA_PIECE_WINV || piece > FEWHA_PIECE_AT) return fail(ctx, FEWHA_E_INVAL, "unknown piece");
    if (c.prec == FEWHA_FP64)
        run(double{});
    else
        run(float{});
    return check_launch(ctx, as_stream(stream));
}

fewha_status fewha_get_vector(fewha_ctx* ctx, int32_t which, void* d_out, void* stream) {
    if (!ctx || !d_out) return fail(ctx, FEWHA_E_INVAL, "NULL argument");
    const fewha::Ctx& c = ctx->c;
    size_t off;
    if (which == 0)
        off = c.lay.prior_a;
    else if (which == 1)
        off = c.lay.jinv;
    else
        return fail(ctx, FEWHA_E_INVAL, "which must be 0 (alpha D) or 1 (J^-1)");
    if (hipMemcpyAsync(d_out, c.ws + off, c.esz * c.N, hipMemcpyDeviceToDevice, as_stream(stream)) != hipSuccess)
        return fail(ctx, FEWHA_E_HIP, "hipMemcpyAsync failed");
    return FEWHA_OK;
}

fewha_status fewha_state_size(const fewha_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return FEWHA_E_INVAL;
    *bytes = ctx->c.lay.state_bytes;
    return FEWHA_OK;
}

// State buffer: [256-byte header][instances x (slots doubles (p_j, q_j), 1 double: real recycled
// directions)][c][r][b_prev][U slots][Q slots]
fewha_status fewha_get_state(fewha_ctx* ctx, void* d_dst, void* stream) {
    if (!ctx || !d_dst) return fail(ctx, FEWHA_E_INVAL, "NULL argument");
    const fewha::Ctx& c = ctx->c;
    hipStream_t s = as_stream(stream);
    uint64_t* h = ctx->state_header;
    std::memset(h, 0, sizeof(ctx->state_header));
    h[0] = kStateMagic;
    h[1] = uint64_t(c.N);
    h[2] = uint64_t(c.slots);
    h[3] = uint64_t(c.esz);
    h[4] = uint64_t(c.head);
    h[5] = uint64_t(c.count);
    h[6] = uint64_t(c.last_iters);
    h[7] = uint64_t(c.first ? 1 : 0);
    h[8] = uint64_t(c.B);
    char* dst = static_cast<char*>(d_dst);
    const size_t vb = c.esz * c.N;
    bool ok = hipMemcpyAsync(dst, h, 256, hipMemcpyHostToDevice, s) == hipSuccess;
    // per instance: (p_j, q_j) of every slot, then the count of real recycled directions
    // (tolerance mode), as a double
    const size_t pib = sizeof(double) * (c.slots + 1);
    if (ok) ok = fewha::launch_state_avail(c, dst + 256, pib, true, s) == hipSuccess;
    for (int i = 0; i < c.B; ++i)
        ok = ok && hipMemcpyAsync(dst + 256 + pib * i,
                                  c.ws + c.lay.scalars + sizeof(fewha::Scalars) * i + offsetof(fewha::Scalars, gam),
                                  sizeof(double) * c.slots, hipMemcpyDeviceToDevice, s) == hipSuccess;
    size_t o = 256 + pib * c.B;
    for (size_t src : {c.lay.c, c.lay.r, c.lay.b_prev}) {
        ok = ok && hipMemcpyAsync(dst + o, c.ws + src, vb, hipMemcpyDeviceToDevice, s) == hipSuccess;
        o += vb;
    }
    ok = ok && hipMemcpyAsync(dst + o, c.ws + c.lay.ring_u, vb * c.slots, hipMemcpyDeviceToDevice, s) == hipSuccess;
    o += vb * c.slots;
    ok = ok && hipMemcpyAsync(dst + o, c.ws + c.lay.ring_q, vb * c.slots, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (ok) ok = hipStreamSynchronize(s) == hipSuccess;   // the header is host memory
    return ok ? FEWHA_OK : fail(ctx, FEWHA_E_HIP, "state copy failed");
}

fewha_status fewha_set_state(fewha_ctx* ctx, const void* d_src, void* stream) {
    if (!ctx || !d_src) return fail(ctx, FEWHA_E_INVAL, "NULL argument");
    fewha::Ctx& c = ctx->c;
    hipStream_t s = as_stream(stream);
    uint64_t h[32];
    if (hipMemcpyAsync(h, d_src, 256, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail(ctx, FEWHA_E_HIP, "state header copy failed");
    if (h[0] != kStateMagic || h[1] != uint64_t(c.N) || h[2] != uint64_t(c.slots) || h[3] != uint64_t(c.esz) ||
        h[4] >= uint64_t(c.slots) || h[5] > uint64_t(c.slots) || h[8] != uint64_t(c.B))
        return fail(ctx, FEWHA_E_STATE, "state buffer does not match this configuration");
    const char* src = static_cast<const char*>(d_src);
    const size_t vb = c.esz * c.N;
    bool ok = true;
    const size_t pib = sizeof(double) * (c.slots + 1);
    for (int i = 0; i < c.B; ++i)
        ok = ok && hipMemcpyAsync(c.ws + c.lay.scalars + sizeof(fewha::Scalars) * i + offsetof(fewha::Scalars, gam),
                                  src + 256 + pib * i, sizeof(double) * c.slots, hipMemcpyDeviceToDevice,
                                  s) == hipSuccess;
    if (ok) ok = fewha::launch_state_avail(c, const_cast<char*>(src) + 256, pib, false, s) == hipSuccess;
    size_t o = 256 + pib * c.B;
    for (size_t dst : {c.lay.c, c.lay.r, c.lay.b_prev}) {
        ok = ok && hipMemcpyAsync(c.ws + dst, src + o, vb, hipMemcpyDeviceToDevice, s) == hipSuccess;
        o += vb;
    }
    ok = ok && hipMemcpyAsync(c.ws + c.lay.ring_u, src + o, vb * c.slots, hipMemcpyDeviceToDevice, s) == hipSuccess;
    o += vb * c.slots;
    ok = ok && hipMemcpyAsync(c.ws + c.lay.ring_q, src + o, vb * c.slots, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (!ok) return fail(ctx, FEWHA_E_HIP, "state copy failed");
    c.head = int(h[4]);
    c.count = int(h[5]);
    c.last_iters = int(h[6]);
    c.first = h[7] != 0;
    return FEWHA_OK;
}

fewha_status fewha_profile(fewha_ctx* ctx, int32_t enable) {
    if (!ctx) return FEWHA_E_INVAL;
    fewha::Profiler& p = ctx->c.prof;
    p.on = enable != 0;
    p.pending.clear();
    for (int i = 0; i < fewha::KID_COUNT; ++i) {
        p.ms[i] = 0;
        p.launches[i] = 0;
    }
    return FEWHA_OK;
}

fewha_status fewha_profile_read(const fewha_ctx* ctx, double* ms, int64_t* launches, int32_t n, int32_t* n_out) {
    if (!ctx) return FEWHA_E_INVAL;
    const fewha::Profiler& p = ctx->c.prof;
    for (int i = 0; i < n && i < fewha::KID_COUNT; ++i) {
        if (ms) ms[i] = p.ms[i];
        if (launches) launches[i] = p.launches[i];
    }
    if (n_out) *n_out = fewha::KID_COUNT;
    return FEWHA_OK;
}

fewha_status fewha_time_kernel(fewha_ctx* ctx, int32_t kernel, int32_t step, int32_t reps, void* stream,
                               float* avg_ms) {
    if (!ctx || !avg_ms) return FEWHA_E_INVAL;
    fewha::Ctx& c = ctx->c;
    hipError_t e = c.prec == FEWHA_FP64
                       ? fewha::time_operator_kernel<double>(c, kernel, step, reps, as_stream(stream), avg_ms)
                       : fewha::time_operator_kernel<float>(c, kernel, step, reps, as_stream(stream), avg_ms);
    if (e == hipErrorInvalidValue) return fail(ctx, FEWHA_E_INVAL, "kernel is not an operator kernel or bad step");
    if (e != hipSuccess) return fail(ctx, FEWHA_E_HIP, std::string("kernel timing failed: ") + hipGetErrorString(e));
    return FEWHA_OK;
}

fewha_status fewha_get_tuning(const fewha_ctx* ctx, fewha_tuning* t) {
    if (!ctx || !t) return FEWHA_E_INVAL;
    std::memset(t, 0, sizeof(*t));
    const fewha::Ctx& c = ctx->c;
    t->syn_tile = c.syn_tile ? c.syn_tile : (c.syn_large < fewha::kSmallTileBelow ? fewha::kSynTile / 2 : fewha::kSynTile);
    t->gather_rows = c.gather_rows;
    return FEWHA_OK;
}

fewha_status fewha_set_tuning(fewha_ctx* ctx, const fewha_tuning* t) {
    if (!ctx || !t) return FEWHA_E_INVAL;
    const bool big_ok = ctx->c.prec != FEWHA_FP64;   // 64 x 64 tiles need FP32 (LDS)
    if (t->syn_tile != 0 && t->syn_tile != fewha::kSynTile / 2 && t->syn_tile != fewha::kSynTile &&
        !(big_ok && t->syn_tile == 2 * fewha::kSynTile))
        return fail(ctx, FEWHA_E_INVAL, "syn_tile must be 0, 16, 32 or (FP32) 64");
    if (t->gather_rows != 1 && t->gather_rows != 4) return fail(ctx, FEWHA_E_INVAL, "gather_rows must be 1 or 4");
    fewha::Ctx& c = ctx->c;
    if (c.syn_tile != t->syn_tile || c.gather_rows != t->gather_rows) {
        c.syn_tile = t->syn_tile;
        c.gather_rows = t->gather_rows;
        fewha::release_graphs(c);   // the captured frames hold the old launches
    }
    return FEWHA_OK;
}

fewha_status fewha_autotune(fewha_ctx* ctx, int32_t reps, void* stream, fewha_tuning* best, float* ms, int32_t n,
                            int32_t* n_out) {
    if (!ctx || reps < 1) return FEWHA_E_INVAL;
    fewha::Ctx& c = ctx->c;
    const int nsyn = c.prec == FEWHA_FP64 ? 2 : 3;
    const int syn[3] = {fewha::kSynTile / 2, fewha::kSynTile, 2 * fewha::kSynTile}, rows[2] = {1, 4};
    fewha_tuning cand[6] = {}, keep = {};
    (void)fewha_get_tuning(ctx, &keep);
    float tm[6] = {};
    int k = 0, b = -1;
    for (int i = 0; i < nsyn; ++i)
        for (int j = 0; j < 2; ++j, ++k) {
            cand[k].syn_tile = syn[i];
            cand[k].gather_rows = rows[j];
            (void)fewha_set_tuning(ctx, &cand[k]);
            hipError_t e = c.prec == FEWHA_FP64
                               ? fewha::time_operator_kernel<double>(c, fewha::KID_APPLY, 0, reps, as_stream(stream), &tm[k])
                               : fewha::time_operator_kernel<float>(c, fewha::KID_APPLY, 0, reps, as_stream(stream), &tm[k]);
            if (e != hipSuccess) {
                (void)fewha_set_tuning(ctx, &keep);
                return fail(ctx, FEWHA_E_HIP, std::string("autotune timing failed: ") + hipGetErrorString(e));
            }
            if (b < 0 || tm[k] < tm[b]) b = k;
        }
    (void)fewha_set_tuning(ctx, &cand[b]);
    if (best) *best = cand[b];
    for (int i = 0; i < n && i < k; ++i) ms[i] = tm[i];
    if (n_out) *n_out = k;
    return FEWHA_OK;
}

fewha_status fewha_wavelet_steps(const fewha_ctx* ctx, int32_t* block_sizes, int32_t* layer_counts, int32_t n,
                                 int32_t* n_out) {
    if (!ctx) return FEWHA_E_INVAL;
    const auto& st = ctx->c.steps;
    for (int i = 0; i < n && i < int(st.size()); ++i) {
        if (block_sizes) block_sizes[i] = st[i].nb;
        if (layer_counts) layer_counts[i] = int32_t(st[i].nl);
    }
    if (n_out) *n_out = int32_t(st.size());
    return FEWHA_OK;
}

const char* fewha_kernel_name(int32_t i) {
    return (i >= 0 && i < fewha::KID_COUNT) ? fewha::kKernelNames[i] : nullptr;
}

fewha_status fewha_use_graphs(fewha_ctx* ctx, int32_t enable) {
    if (!ctx) return FEWHA_E_INVAL;
    ctx->c.use_graphs = enable != 0;
    return FEWHA_OK;
}

fewha_status fewha_destroy(fewha_ctx* ctx) {
    if (ctx) {
        for (hipEvent_t e : ctx->c.prof.pool) (void)hipEventDestroy(e);
        fewha::release_graphs(ctx->c);
        if (ctx->c.brk_host) (void)hipHostFree(ctx->c.brk_host);
    }
    delete ctx;
    return FEWHA_OK;
}

const char* fewha_last_error(const fewha_ctx* ctx) {
    if (!ctx) return g_setup_err.c_str();
    return ctx->c.err_lit ? ctx->c.err_lit : ctx->c.err.c_str();
}

}  // extern "C"
