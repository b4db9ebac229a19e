// Learned warm start (declared in include/fewha_unet.h): U-Net forward, backward and Adam on
// the bfloat16 matrix cores of gfx950 (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
//   k_conv3x3      implicit GEMM of a same-size 3x3 convolution over NHWC bf16 activations:
//                  out[p][co] = sum_{tap, ci} in[p + tap][ci] w[tap][co][ci]; 64 pixels x 32
//                  output channels per wavefront (4 x 2 MFMA tiles of 16 x 16), the weights as
//                  the A operand; the reduction over taps and channel blocks optionally split
//                  over the wavefronts of a workgroup (KS = 2 or 4); zero padding reads a zero
//                  row stored after every image, not masks; the decoder's 2x nearest upsampling
//                  and skip concatenation are folded into the operand addresses; the input
//                  gradient is the same kernel on the ReLU-masked output gradient with
//                  flipped, transposed weights.
//   k_conv_wgrad   weight gradient sum_p x[p + tap][ci] dy[p][co] of all nine taps and the
//                  bias gradient sum_p dy[p][co]: tiles of 64 pixels are transposed through LDS
//                  so that every MFMA operand is one 16-byte read; per-chunk FP32 partials,
//                  summed in a fixed order by k_reduce_table (one launch for the network).
//   small kernels  input packing, pooling and its adjoint, the upsample/concat adjoint, the
//                  1x1 head with the MSE loss, ReLU', bias gradients, Adam, layouts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fewha_unet.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16_t;   // bfloat16 storage

constexpr int kT = 256;            // threads of every kernel
constexpr int kConvPix = 256;      // pixels per convolution workgroup (without a reduction split)
constexpr int kWBlocks = 768;      // weight-gradient workgroups aimed at per convolution (3 per CU)
constexpr int kLevels = 4;
constexpr int kCh[kLevels] = {32, 64, 128, 256};
constexpr int kInCh = 32;          // padded input channels
constexpr int kInputs = 4;         // used input channels
constexpr int kConvs = 14;

__host__ __device__ inline float bf2f(bf16_t h) {
    const uint32_t u = uint32_t(h) << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// Round to nearest even (finite inputs).
__host__ __device__ inline bf16_t f2bf(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return bf16_t(u >> 16);
}

__device__ inline bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ inline uint4 and_mask(uint4 v, uint32_t m) { return make_uint4(v.x & m, v.y & m, v.z & m, v.w & m); }

// ------------------------------------------------------------------ convolution (implicit GEMM)

enum { CONV_DIRECT = 0, CONV_CONCAT_UP = 1 };

// MODE CONV_DIRECT: in0 [N][H][W][Cin].  MODE CONV_CONCAT_UP: channels [0, C1) come from the
// 2x nearest upsampling of in0 [N][H/2][W/2][C1], channels [C1, Cin) from in1 [N][H][W][Cin-C1].
// Every input tensor carries one extra pixel of zeros after its last pixel (the zero row):
// operands outside the image read it, so the zero padding costs no masking.
// OUT_BF16: out = bf16(relu?(acc + bias)) [P][Cout]; else out = acc (FP32) [P][Cout].
// One launch covers several image groups (square images, per-group tensors).
// Cin, C1, Cout multiples of 32.  A wavefront computes 64 pixels x 32 output channels (4 x 2
// MFMA tiles of 16 x 16, K = 32 channels of one tap per reduction position).  KS (1, 2 or 4)
// splits the reduction over the wavefronts of a workgroup: the workgroup covers 256 / KS
// pixels, wavefront w the 64 pixels w mod (4 / KS) and every KS-th reduction position from
// w / (4 / KS); the KS partial tiles are summed in a fixed order through LDS.  Requires
// 9 Cin / 32 to be a multiple of 3 KS.  Byte offsets into the inputs must fit in 32 bits
// (with at most 2^25 pixels per level and 64 bytes per full-resolution pixel they do).
// The image groups of one launch: group g covers workgroups [block0[g], block0[g + 1]).
struct ConvGroup {
    const bf16_t* in0;
    const bf16_t* in1;
    void* out;
    int N, H, block0;
};
struct ConvGroups {
    ConvGroup g[FEWHA_UNET_MAX_GROUPS + 1];   // entry `count` holds the end block
    int count;
};

template <int MODE, bool OUT_BF16, int KS>
__global__ void __launch_bounds__(kT) k_conv3x3(ConvGroups cg, int C1, int Cin, const bf16_t* __restrict__ wt,
                                                 const float* __restrict__ bias, int relu, int Cout) {
    constexpr int PG = 4 / KS;            // 64-pixel groups per workgroup
    constexpr int MT = 4;                 // 16-pixel MFMA tiles per wavefront
    int gi = 0;
    while (gi + 1 < cg.count && int(blockIdx.x) >= cg.g[gi + 1].block0) ++gi;
    const bf16_t* __restrict__ in0 = cg.g[gi].in0;
    const bf16_t* __restrict__ in1 = cg.g[gi].in1;
    void* __restrict__ out = cg.g[gi].out;
    const int N = cg.g[gi].N, H = cg.g[gi].H, W = H;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar position counters
    const int r16 = lane & 15, kg = lane >> 4;
    const int pg = wv % PG, ks = wv / PG;
    const int P = N * H * W;
    const int co0 = blockIdx.y * 32;
    const int pb = (int(blockIdx.x) - cg.g[gi].block0) * (64 * PG) + pg * 64;
    const int C2 = Cin - C1, Hh = H >> 1, Wh = W >> 1, Ph = N * Hh * Wh;
    const int lh = __builtin_ctz(H), lw = __builtin_ctz(W);   // H, W powers of two
    // per MFMA row tile: the in-image bits of the lane's nine taps, the element offset of its
    // pixel in the full-resolution input (in0, or in1 when concatenating), and for the
    // upsampled input its half-resolution pixel and the parities of its coordinates
    const int Cf = MODE == CONV_DIRECT ? Cin : C2;
    uint32_t okbits[MT], oc[MT], hc[MT], par[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int p = pb + 16 * mt + r16;
        const bool pin = p < P;
        const int pc = pin ? p : 0;
        const int pn = pc >> (lh + lw), py = (pc >> lw) & (H - 1), px = pc & (W - 1);
        uint32_t bits = 0;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ys = py + t / 3 - 1, xs = px + t % 3 - 1;
            bits |= uint32_t(pin & (unsigned(ys) < unsigned(H)) & (unsigned(xs) < unsigned(W))) << t;
        }
        okbits[mt] = bits;
        oc[mt] = (uint32_t(pc) * Cf + 8 * kg) * 2u;                // byte offsets from here on
        hc[mt] = uint32_t((pn * Hh + (py >> 1)) * Wh + (px >> 1));
        par[mt] = uint32_t((py & 1) | ((px & 1) << 1));
    }
    const uint32_t oz = (uint32_t(P) * Cf + 8 * kg) * 2u;          // the zero row
    const uint32_t ozh = (uint32_t(Ph) * C1 + 8 * kg) * 2u;
    // weight offsets (elements) of the lane's two output-channel rows, relative to a tap's
    // [Cout][Cin] block
    uint32_t ob[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) ob[nt] = (uint32_t(co0 + 16 * nt + r16) * Cin + 8 * kg) * 2u;

    f32x4 acc[MT][2];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    // The reduction runs over (tap, 32-channel block) positions.  Operands are fetched two
    // positions ahead into a ring of three register sets, so that every MFMA waits only for
    // loads issued two positions earlier; fetches past the wavefront's last position repeat
    // the last tap (valid addresses, unused values).
    int ftap = 0, fcb = 32 * ks;          // Cin / 32 >= KS, so the first position is in tap 0
    auto fetch = [&](uint4 (&a)[MT], uint4 (&b)[2]) {
        const int dy = ftap / 3 - 1, dx = ftap - 3 * (ftap / 3) - 1;
        const uint32_t shift = uint32_t((dy * W + dx) * Cf) * 2u;   // uniform
        const bool upsampled = MODE == CONV_CONCAT_UP && fcb < C1;
        const char* base = reinterpret_cast<const char*>(MODE == CONV_DIRECT ? in0 + fcb
                                                         : upsampled         ? in0 + fcb
                                                                             : in1 + (fcb - C1));
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const bool ok = (okbits[mt] >> ftap) & 1u;
            uint32_t off;
            if (upsampled) {
                // half-resolution pixel of the shifted full-resolution pixel: floor((2y' + e + d) / 2)
                const int sy = (int(par[mt] & 1u) + dy) >> 1, sx = (int(par[mt] >> 1) + dx) >> 1;
                off = ok ? ((hc[mt] + uint32_t(sy * Wh + sx)) * uint32_t(C1) + 8 * kg) * 2u : ozh;
            } else {
                off = ok ? oc[mt] + shift : oz;
            }
            a[mt] = *reinterpret_cast<const uint4*>(base + off);
        }
        const char* wtap = reinterpret_cast<const char*>(wt + (size_t(ftap) * Cout * Cin + fcb));
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) b[nt] = *reinterpret_cast<const uint4*>(wtap + ob[nt]);
        // next position of this wavefront (32 KS <= Cin: at most one tap carry)
        fcb += 32 * KS;
        if (fcb >= Cin) {
            fcb -= Cin;
            ftap = ftap < 8 ? ftap + 1 : 8;
        }
    };
    // weights as the A operand and pixels as B: the tile is C[co][pixel], so that a lane's
    // four results are four consecutive output channels of one pixel (one vector store)
    auto mma = [&](const uint4 (&a)[MT], const uint4 (&b)[2]) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(b[nt]), as_bf16x8(a[mt]), acc[mt][nt],
                                                                      0, 0, 0);
    };
    uint4 a0[MT], b0[2], a1[MT], b1[2], a2[MT], b2[2];
    fetch(a0, b0);
    fetch(a1, b1);
    const int iters = 9 * (Cin >> 5) / KS;
    for (int it = 0; it < iters; it += 3) {
        fetch(a2, b2);
        mma(a0, b0);
        fetch(a0, b0);
        mma(a1, b1);
        fetch(a1, b1);
        mma(a2, b2);
    }
    if constexpr (KS > 1) {   // fixed-order sum of the KS partial tiles into wavefronts with ks == 0
        __shared__ f32x4 red[KS - 1][PG][MT * 2][64];
        if (ks > 0) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) red[ks - 1][pg][2 * mt + nt][lane] = acc[mt][nt];
        }
        __syncthreads();
        if (ks > 0) return;
#pragma unroll
        for (int j = 0; j < KS - 1; ++j)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) acc[mt][nt] += red[j][pg][2 * mt + nt][lane];
    }
    // lane l, register v: output channel 4 (l / 16) + v, pixel l mod 16 of the tile
    float bv[2][4] = {};
    if (OUT_BF16 && bias) {
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) bv[nt][v] = bias[co0 + 16 * nt + 4 * kg + v];
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int p = pb + 16 * mt + r16;
        if (p >= P) continue;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const size_t o = size_t(p) * Cout + co0 + 16 * nt + 4 * kg;
            if (OUT_BF16) {
                uint32_t h[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float val = acc[mt][nt][v] + bv[nt][v];
                    if (relu) val = fmaxf(val, 0.f);
                    h[v] = f2bf(val);
                }
                *reinterpret_cast<uint2*>(static_cast<bf16_t*>(out) + o) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
            } else {
                *reinterpret_cast<float4*>(static_cast<float*>(out) + o) =
                    make_float4(acc[mt][nt][0], acc[mt][nt][1], acc[mt][nt][2], acc[mt][nt][3]);
            }
        }
    }
}

// ------------------------------------------------------------------ weight gradient

// Weight and bias gradient partials of the pixels of chunk blockIdx.x (chunk_px pixels, a
// multiple of 64; one launch covers every image group) for
// the (co tile of 32, ci tile of 32) pair blockIdx.y, all nine taps at once:
//   part[chunk][tap][co][ci] = sum_p dy[p][co] x[p + tap][ci],
//   part[chunk][9 Cout Cin + co] = sum_p dy[p][co]   (written by the ci-tile-0 blocks).
// Per step of 64 pixels the block stages dy[64][32 co] and the nine shifted inputs
// x[64 (+ tap)][32 ci] into LDS transposed (channel rows, pixel columns), so that every
// MFMA operand (8 consecutive pixels of one channel) is one 16-byte LDS read; wavefront w
// accumulates the 16 x 16 sub-tile (w / 2, w % 2) of every tap (2 MFMAs of K = 32 per tap
// and step).  Staging: thread t moves pixels 2 (t mod 32) and 2 (t mod 32) + 1 of the 8
// channels 8 ((t / 32) mod 4) .. +7 of five of the ten sources (dy and the nine taps), as
// packed pixel pairs (one 4-byte LDS write per channel).
// The image groups of one launch: group g's chunks are workgroups [block0[g], block0[g + 1])
// along x, and partial rows of the same indices.
struct WgradGroup {
    const bf16_t* dy;
    const bf16_t* in0;
    const bf16_t* in1;
    int N, H, block0;
};
struct WgradGroups {
    WgradGroup g[FEWHA_UNET_MAX_GROUPS + 1];   // entry `count` holds the end block
    int count;
};

template <int MODE>
__global__ void __launch_bounds__(kT) k_conv_wgrad(WgradGroups wg, int C1, int Cin, int Cout, int chunk_px,
                                                    float* __restrict__ part) {
    int gi = 0;
    while (gi + 1 < wg.count && int(blockIdx.x) >= wg.g[gi + 1].block0) ++gi;
    const bf16_t* __restrict__ dy = wg.g[gi].dy;
    const bf16_t* __restrict__ in0 = wg.g[gi].in0;
    const bf16_t* __restrict__ in1 = wg.g[gi].in1;
    const int N = wg.g[gi].N, H = wg.g[gi].H, W = H;
    constexpr int SP = 64;                     // pixels per step
    constexpr int LD = SP + 8;                 // padded row (bf16): 36 dwords, 16-byte aligned rows
    __shared__ __align__(16) bf16_t st[10][32][LD];   // source 0: dy [co][px]; 1 + tap: x [ci][px]
    __shared__ float bsh[2][32];                      // bias partials of waves 0 and 1
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform
    const int r16 = lane & 15, kg = lane >> 4;
    const int nci = Cin / 32;
    const int co0 = (blockIdx.y / nci) * 32, ci0 = (blockIdx.y % nci) * 32;
    const bool with_bias = ci0 == 0;
    const int P = N * H * W, C2 = Cin - C1, Hh = H >> 1, Wh = W >> 1;
    const int lh = __builtin_ctz(H), lw = __builtin_ctz(W);   // H, W powers of two
    const int p_begin = (int(blockIdx.x) - wg.g[gi].block0) * chunk_px;
    const int p_end = min(P, p_begin + chunk_px);
    // staging role: pixel pair (2 pair, 2 pair + 1) of the step and channel group grp, so that
    // the lanes of one load cover whole 64-byte pixel rows; sources 2 j + half
    const int pair = (threadIdx.x & 127) >> 2, grp = threadIdx.x & 3, half = wv >> 1;
    // LDS rows hold 32 dwords of pixel pairs; the dword column of a row of channel group g
    // is rotated by 8 g (mod 32), which spreads the four groups of a store over the banks
    auto col = [](int dw, int g) { return ((dw + 8 * g) & 31); };
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) bsum[i] = 0.f;
    const int mt = wv >> 1, nt = wv & 1;
    // the thread's ten 16-byte loads of the step starting at pixel p0 (issued together; the
    // bias sums take the dy values as they are staged)
    // Inputs outside the image and pixels past the chunk read the zero row of their tensor
    // (one pixel of zeros after the last), so no masking is needed; byte offsets fit in 32 bits.
    const int Cf = MODE == CONV_DIRECT ? Cin : C2;           // channels of the full-resolution input
    const bool up = MODE == CONV_CONCAT_UP && ci0 < C1;     // this ci tile comes from the upsampling
    const char* xbase = reinterpret_cast<const char*>(up ? in0 + ci0 : MODE == CONV_DIRECT ? in0 + ci0 : in1 + (ci0 - C1));
    const char* dbase = reinterpret_cast<const char*>(dy + co0);
    const uint32_t xC = up ? C1 : Cf;                          // channels per pixel of that input
    const uint32_t Ph = uint32_t(N) * Hh * Wh;
    const uint32_t xzero = ((up ? Ph : uint32_t(P)) * xC + 8 * grp) * 2u;
    const uint32_t dzero = (uint32_t(P) * Cout + 8 * grp) * 2u;
    uint4 v[5][2];
    auto load_step = [&](int p0) {
        uint32_t okb[2], xo[2], dofs[2], hc[2], par[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int p = p0 + 2 * pair + e;
            const bool pin = p < p_end;
            const int pc = pin ? p : p_begin;
            const int pn = pc >> (lh + lw), py = (pc >> lw) & (H - 1), px = pc & (W - 1);
            uint32_t bits = 0;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int ys = py + t / 3 - 1, xs = px + t % 3 - 1;
                bits |= uint32_t(pin & (unsigned(ys) < unsigned(H)) & (unsigned(xs) < unsigned(W))) << t;
            }
            okb[e] = bits;
            xo[e] = (uint32_t(pc) * xC + 8 * grp) * 2u;
            dofs[e] = pin ? (uint32_t(pc) * Cout + 8 * grp) * 2u : dzero;
            hc[e] = uint32_t((pn * Hh + (py >> 1)) * Wh + (px >> 1));
            par[e] = uint32_t((py & 1) | ((px & 1) << 1));
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int src_id = 2 * j + half;        // 0: dy, 1 + tap: shifted input (uniform)
            const int tap = src_id > 0 ? src_id - 1 : 4;
            const int dyy = tap / 3 - 1, dxx = tap - 3 * (tap / 3) - 1;
            const uint32_t shift = uint32_t((dyy * W + dxx) * int(xC)) * 2u;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const char* src;
                if (src_id == 0) {
                    src = dbase + dofs[e];
                } else {
                    const bool ok = (okb[e] >> tap) & 1u;
                    uint32_t off;
                    if (up) {
                        const int sy = (int(par[e] & 1u) + dyy) >> 1, sx = (int(par[e] >> 1) + dxx) >> 1;
                        off = ok ? ((hc[e] + uint32_t(sy * Wh + sx)) * xC + 8 * grp) * 2u : xzero;
                    } else {
                        off = ok ? xo[e] + shift : xzero;
                    }
                    src = xbase + off;
                }
                v[j][e] = *reinterpret_cast<const uint4*>(src);
            }
        }
    };
    load_step(p_begin);
    for (int p0 = p_begin; p0 < p_end; p0 += SP) {
        if (with_bias && half == 0) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const bf16_t* h = reinterpret_cast<const bf16_t*>(&v[0][e]);
#pragma unroll
                for (int i = 0; i < 8; ++i) bsum[i] += bf2f(h[i]);
            }
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int src_id = 2 * j + half;
            const uint32_t* w0 = reinterpret_cast<const uint32_t*>(&v[j][0]);
            const uint32_t* w1 = reinterpret_cast<const uint32_t*>(&v[j][1]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {      // channels 2i, 2i + 1 of the group: (pixel 0, pixel 1) pairs
                const uint32_t lo = (w0[i] & 0xFFFFu) | (w1[i] << 16);
                const uint32_t hi = (w0[i] >> 16) | (w1[i] & 0xFFFF0000u);
                *reinterpret_cast<uint32_t*>(&st[src_id][8 * grp + 2 * i][2 * col(pair, grp)]) = lo;
                *reinterpret_cast<uint32_t*>(&st[src_id][8 * grp + 2 * i + 1][2 * col(pair, grp)]) = hi;
            }
        }
        __syncthreads();
        // the next step's loads fly while this step's MFMAs run (the last step reloads itself)
        load_step(p0 + SP < p_end ? p0 + SP : p0);
#pragma unroll
        for (int kk = 0; kk < SP / 32; ++kk) {
            // all operands of the K step first, then the nine MFMAs
            // rows 16 mt + r16 (dy) and 16 nt + r16 (x) belong to channel groups 2 mt + r16 / 8
            // and 2 nt + r16 / 8; the lane's 4 dwords start at logical dword 16 kk + 4 kg
            const int ra = 16 * mt + r16, rb = 16 * nt + r16;
            const uint4 a = *reinterpret_cast<const uint4*>(&st[0][ra][2 * col(16 * kk + 4 * kg, ra >> 3)]);
            uint4 b[9];
#pragma unroll
            for (int t = 0; t < 9; ++t)
                b[t] = *reinterpret_cast<const uint4*>(&st[1 + t][rb][2 * col(16 * kk + 4 * kg, rb >> 3)]);
            // x as the A operand and dy as B: the tile is C[ci][co], a lane's four results are
            // four consecutive input channels (one vector store)
#pragma unroll
            for (int t = 0; t < 9; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(b[t]), as_bf16x8(a), acc[t], 0, 0, 0);
        }
        __syncthreads();
    }
    const size_t row = size_t(9) * Cout * Cin + Cout;
    float* dst = part + size_t(blockIdx.x) * row;
    // lane l, register v: ci row 4 (l / 16) + v, co column l mod 16 of the sub-tile
    {
        const int co = co0 + 16 * mt + r16, ci = ci0 + 16 * nt + 4 * kg;
#pragma unroll
        for (int t = 0; t < 9; ++t)
            *reinterpret_cast<float4*>(dst + (size_t(t) * Cout + co) * Cin + ci) =
                make_float4(acc[t][0], acc[t][1], acc[t][2], acc[t][3]);
    }
    if (with_bias) {
        // waves 0 and 1 hold the dy values: sum over the 16 lanes of each channel group (lane
        // mod 4), then wave 0 adds wave 1's sums
        if (half == 0) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                float v = bsum[i];
#pragma unroll
                for (int o = 4; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
                bsum[i] = v;
            }
            if (wv == 1 && lane < 4) {
#pragma unroll
                for (int i = 0; i < 8; ++i) bsh[1][8 * grp + i] = bsum[i];
            }
        }
        __syncthreads();
        if (wv == 0 && lane < 4) {
#pragma unroll
            for (int i = 0; i < 8; ++i) dst[size_t(9) * Cout * Cin + co0 + 8 * grp + i] = bsum[i] + bsh[1][8 * grp + i];
        }
    }
}

// Fixed-order sums of chunk partials for several tensors in one launch.  Every element is the
// sum of its chunks in eight running sums (sum j takes the chunks c with c mod 8 = j, in
// increasing order), combined as ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7)).  Tensor k
// owns blocks [block0[k], block0[k + 1]) and splits the eight sums of an element over
// stripes[k] threads (1, 2, 4 or 8; thread u of an element keeps the sums u, u + S, ...), so
// that tensors with many chunks keep more loads in flight; the split leaves every bit of the
// result unchanged.
struct ReduceTable {
    const float* part[16];
    float* out[16];
    int64_t n[16];
    int chunks[16];
    int stripes[16];
    int block0[17];
    int count;
};

// The running sums u + S q (q < 8 / S) of one element over C chunks of stride n, S groups of
// eight chunks per step with every load issued before the additions.
template <int S>
__device__ inline void stripe_sums(const float* __restrict__ p, int64_t n, int C, int u, float* s) {
    constexpr int J = 8 / S;
    int c = 0;
    for (; c + 8 * S <= C; c += 8 * S) {
        float v[S][J];
#pragma unroll
        for (int g = 0; g < S; ++g)
#pragma unroll
            for (int q = 0; q < J; ++q) v[g][q] = p[size_t(c + 8 * g + u + S * q) * n];
#pragma unroll
        for (int g = 0; g < S; ++g)
#pragma unroll
            for (int q = 0; q < J; ++q) s[q] += v[g][q];
    }
    for (; c < C; c += 8) {
#pragma unroll
        for (int q = 0; q < J; ++q)
            if (c + u + S * q < C) s[q] += p[size_t(c + u + S * q) * n];
    }
}

__global__ void __launch_bounds__(kT) k_reduce_table(ReduceTable tb) {
    __shared__ float sm[8][kT];
    int k = 0;
    while (k + 1 < tb.count && int(blockIdx.x) >= tb.block0[k + 1]) ++k;
    const int S = tb.stripes[k];
    const int E = kT / S;   // elements per block
    const int u = int(threadIdx.x) / E, e = int(threadIdx.x) - u * E;
    const int64_t i = int64_t(blockIdx.x - tb.block0[k]) * E + e;
    const int64_t n = tb.n[k];
    const bool live = i < n;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (live) {
        const float* __restrict__ p = tb.part[k] + i;
        const int C = tb.chunks[k];
        switch (S) {
            case 1: stripe_sums<1>(p, n, C, u, s); break;
            case 2: stripe_sums<2>(p, n, C, u, s); break;
            case 4: stripe_sums<4>(p, n, C, u, s); break;
            default: stripe_sums<8>(p, n, C, u, s); break;
        }
    }
    for (int q = 0; q < 8 / S; ++q) sm[u + S * q][e] = s[q];
    __syncthreads();
    if (int(threadIdx.x) < E && live) {
        const int t = int(threadIdx.x);
        tb.out[k][i] = ((sm[0][t] + sm[1][t]) + (sm[2][t] + sm[3][t])) + ((sm[4][t] + sm[5][t]) + (sm[6][t] + sm[7][t]));
    }
}

// ------------------------------------------------------------------ small kernels

// in [P][4] FP32 -> x [P][32] bf16 (channels 4..31 zero)
__global__ void __launch_bounds__(kT) k_pack_input(const float* __restrict__ in, int64_t P, bf16_t* __restrict__ x) {
    const int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (e >= P * kInCh) return;
    const int64_t p = e / kInCh;
    const int c = int(e - p * kInCh);
    x[e] = c < kInputs ? f2bf(in[p * kInputs + c]) : bf16_t(0);
}

// 2x2 average pooling, bf16 -> bf16 (sum in FP32)
__global__ void __launch_bounds__(kT) k_pool2(const bf16_t* __restrict__ x, int N, int H, int W, int C,
                                               bf16_t* __restrict__ y) {
    const int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x;
    const int Ho = H / 2, Wo = W / 2;
    if (e >= int64_t(N) * Ho * Wo * C) return;
    const int c = int(e % C);
    const int64_t q = e / C;
    const int xo = int(q % Wo), yo = int((q / Wo) % Ho), n = int(q / (int64_t(Wo) * Ho));
    const size_t b = (size_t(n * H + 2 * yo) * W + 2 * xo) * C + c;
    const float s = (bf2f(x[b]) + bf2f(x[b + C])) + (bf2f(x[b + size_t(W) * C]) + bf2f(x[b + size_t(W) * C + C]));
    y[e] = f2bf(0.25f * s);
}

// g_full[n][y][x][c] += 0.25 g_low[n][y/2][x/2][c]   (adjoint of the pooling)
__global__ void __launch_bounds__(kT) k_pool2_grad_add(const float* __restrict__ gl, int N, int H, int W, int C,
                                                        float* __restrict__ gf) {
    const int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (e >= int64_t(N) * H * W * C) return;
    const int c = int(e % C);
    const int64_t q = e / C;
    const int x = int(q % W), y = int((q / W) % H), n = int(q / (int64_t(W) * H));
    gf[e] += 0.25f * gl[(size_t(n * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c];
}

// Adjoint of [upsample(low), skip]: g_low[q][c] = sum of the 2x2 window of gcat[..][c < C1];
// g_skip[p][c] = gcat[p][C1 + c] (written, the first gradient of the skip tensor).
__global__ void __launch_bounds__(kT) k_split_concat_grad(const float* __restrict__ gcat, int N, int H, int W, int C1,
                                                           int C2, float* __restrict__ glow,
                                                           float* __restrict__ gskip) {
    const int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x;
    const int64_t nl = int64_t(N) * (H / 2) * (W / 2) * C1, ns = int64_t(N) * H * W * C2;
    const int Cc = C1 + C2;
    if (e < nl) {
        const int c = int(e % C1);
        const int64_t q = e / C1;
        const int xo = int(q % (W / 2)), yo = int((q / (W / 2)) % (H / 2)), n = int(q / (int64_t(W / 2) * (H / 2)));
        const size_t b = (size_t(n * H + 2 * yo) * W + 2 * xo) * Cc + c;
        glow[e] = (gcat[b] + gcat[b + Cc]) + (gcat[b + size_t(W) * Cc] + gcat[b + size_t(W) * Cc + Cc]);
    } else if (e < nl + ns) {
        const int64_t f = e - nl;
        const int c = int(f % C2);
        const int64_t p = f / C2;
        gskip[f] = gcat[p * Cc + C1 + c];
    }
}

// dpre = bf16(g * (act > 0)) for the n = P C entries, then the zero row (C zeros) that the
// input-gradient convolution reads for its zero padding
__global__ void __launch_bounds__(kT) k_relu_grad(const float* __restrict__ g, const bf16_t* __restrict__ act,
                                                   int64_t n, int C, bf16_t* __restrict__ dpre) {
    const int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (e >= n + C) return;
    dpre[e] = e < n ? f2bf(bf2f(act[e]) > 0.f ? g[e] : 0.f) : bf16_t(0);
}

// out[p] = sum_c x[p][c] w[c] + b
__global__ void __launch_bounds__(kT) k_head(const bf16_t* __restrict__ x, const float* __restrict__ w,
                                              const float* __restrict__ b, int64_t P, float* __restrict__ out) {
    const int64_t p = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (p >= P) return;
    float s = 0.f;
#pragma unroll 8
    for (int c = 0; c < kCh[0]; ++c) s += bf2f(x[p * kCh[0] + c]) * bf2f(f2bf(w[c]));
    out[p] = s + b[0];
}

// MSE: dout = 2 (out - t) / total; gx[p][c] = dout w_bf16[c]; per-block partials of the loss
// sum, of the head weight gradient and of the head bias gradient
// (part row: [loss, gw[0..31], gb]).
__global__ void __launch_bounds__(kT) k_head_back(const float* __restrict__ out, const float* __restrict__ t,
                                                   const bf16_t* __restrict__ x, const float* __restrict__ w,
                                                   int64_t P, double total, float* __restrict__ gx,
                                                   float* __restrict__ part, int block0) {
    constexpr int C = kCh[0];
    __shared__ float sh[kT / 64][C + 2];
    const int64_t p = int64_t(blockIdx.x) * kT + threadIdx.x;
    float l = 0.f, gb = 0.f, gw[C];
#pragma unroll
    for (int c = 0; c < C; ++c) gw[c] = 0.f;
    if (p < P) {
        const float d = out[p] - t[p];
        const float dout = float(2.0 * double(d) / total);
        l = d * d;
        gb = dout;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            gw[c] = bf2f(x[p * C + c]) * dout;
            gx[p * C + c] = dout * bf2f(f2bf(w[c]));
        }
    }
    auto wsum = [](float v) {
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        return v;
    };
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    l = wsum(l);
    gb = wsum(gb);
#pragma unroll
    for (int c = 0; c < C; ++c) gw[c] = wsum(gw[c]);
    if (lane == 0) {
        sh[wv][0] = l;
#pragma unroll
        for (int c = 0; c < C; ++c) sh[wv][1 + c] = gw[c];
        sh[wv][C + 1] = gb;
    }
    __syncthreads();
    if (threadIdx.x < C + 2) {
        const int k = threadIdx.x;
        part[size_t(block0 + blockIdx.x) * (C + 2) + k] = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
    }
}

// Adam over all n master entries in one launch; the entries of conv k's weights
// [w_off[k], w_off[k] + nw[k]) (internal layout [9][Cout][Cin]) also refresh their bf16
// forward copy and the flipped, transposed copy wd[8 - tap][ci][co] of the input gradient.
struct AdamTable {
    int64_t w_off[kConvs], nw[kConvs];
    bf16_t* wt[kConvs];
    bf16_t* wd[kConvs];
    int cout[kConvs], cin[kConvs];
};

__global__ void __launch_bounds__(kT) k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                                              float eps, float c1, float c2, AdamTable tb) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    int k = 0;
    while (k + 1 < kConvs && i >= tb.w_off[k + 1]) ++k;
    const int64_t j = i - tb.w_off[k];
    if (j < tb.nw[k]) {
        const bf16_t h = f2bf(wi);
        tb.wt[k][j] = h;
        const int Cout = tb.cout[k], Cin = tb.cin[k];
        const int64_t per = int64_t(Cout) * Cin;
        const int tap = int(j / per);
        const int64_t r = j - tap * per;
        const int co = int(r / Cin), ci = int(r - int64_t(co) * Cin);
        tb.wd[k][(size_t(8 - tap) * Cin + ci) * Cout + co] = h;
    }
}

// Network-order parameters <-> internal layout.  dir 0: ext -> master (+ bf16 copies);
// dir 1: master -> ext.  Conv weights: ext [3][3][Cin][Cout], internal [9][Cout][Cin].
__global__ void __launch_bounds__(kT) k_conv_layout(float* __restrict__ ext, float* __restrict__ w, int Cin, int Cout,
                                                     int dir, bf16_t* __restrict__ wt, bf16_t* __restrict__ wd) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    const int64_t n = int64_t(9) * Cin * Cout;
    if (i >= n) return;
    const int tap = int(i / (int64_t(Cin) * Cout));
    const int64_t r = i - tap * int64_t(Cin) * Cout;
    const int ci = int(r / Cout), co = int(r - int64_t(ci) * Cout);
    const size_t j = (size_t(tap) * Cout + co) * Cin + ci;
    if (dir == 0) {
        const float x = ext[i];
        w[j] = x;
        const bf16_t h = f2bf(x);
        wt[j] = h;
        wd[(size_t(8 - tap) * Cin + ci) * Cout + co] = h;
    } else {
        ext[i] = w[j];
    }
}

__global__ void __launch_bounds__(kT) k_copy(float* __restrict__ dst, const float* __restrict__ src, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void __launch_bounds__(kT) k_zero(float* __restrict__ x, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
    if (i < n) x[i] = 0.f;
}

// reduced head row -> loss (mean) and the head gradients
__global__ void k_head_finish(const float* __restrict__ hred, double total, float* __restrict__ loss,
                              float* __restrict__ gw, float* __restrict__ gb) {
    const int k = threadIdx.x;
    if (k == 0 && loss) loss[0] = float(double(hred[0]) / total);
    if (k < kCh[0]) gw[k] = hred[1 + k];
    if (k == 0) gb[0] = hred[kCh[0] + 1];
}

inline unsigned blocks(int64_t n, int per = kT) { return unsigned((n + per - 1) / per); }

// ------------------------------------------------------------------ host network

struct ConvSpec {
    const char* name;
    int cin, cout;
    int level;       // resolution level of its output
    bool concat;     // decoder first convolution: [upsample(coarser), skip]
};

const ConvSpec kSpecs[kConvs] = {
    {"e0a", kInCh, 32, 0, false},   {"e0b", 32, 32, 0, false},    {"e1a", 32, 64, 1, false},
    {"e1b", 64, 64, 1, false},      {"e2a", 64, 128, 2, false},   {"e2b", 128, 128, 2, false},
    {"e3a", 128, 256, 3, false},    {"e3b", 256, 256, 3, false},  {"d2a", 384, 128, 2, true},
    {"d2b", 128, 128, 2, false},    {"d1a", 192, 64, 1, true},    {"d1b", 64, 64, 1, false},
    {"d0a", 96, 32, 0, true},       {"d0b", 32, 32, 0, false}};

enum { E0A, E0B, E1A, E1B, E2A, E2B, E3A, E3B, D2A, D2B, D1A, D1B, D0A, D0B };

}  // namespace

struct fewha_unet {
    // configuration
    int G = 0;
    int images[FEWHA_UNET_MAX_GROUPS] = {}, size[FEWHA_UNET_MAX_GROUPS] = {};
    float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    int64_t nodes = 0, n_params = 0;
    int step = 0;
    std::string err;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t used = 0;
    // parameters (internal layout), FP32 master/m/v/grad share offsets
    int64_t w_off[kConvs] = {}, b_off[kConvs] = {}, hw_off = 0, hb_off = 0, n_master = 0;
    int64_t ext_w[kConvs] = {}, ext_b[kConvs] = {}, ext_hw = 0, ext_hb = 0;
    float *master = nullptr, *mom1 = nullptr, *mom2 = nullptr, *grad = nullptr;
    bf16_t* wt[kConvs] = {};
    bf16_t* wd[kConvs] = {};
    // activations per group: x, conv outputs, pooled inputs
    bf16_t* x[FEWHA_UNET_MAX_GROUPS] = {};
    bf16_t* act[FEWHA_UNET_MAX_GROUPS][kConvs] = {};
    bf16_t* pool[FEWHA_UNET_MAX_GROUPS][3] = {};
    float* out[FEWHA_UNET_MAX_GROUPS] = {};
    // gradient buffers (largest sizes over groups; groups are processed one after the other)
    // gradient buffers per group (every group's backward runs in the same launches)
    float* gact[FEWHA_UNET_MAX_GROUPS][kConvs] = {};   // gradient of each conv output
    float* gcat[FEWHA_UNET_MAX_GROUPS][3] = {};        // of the concatenated decoder inputs (levels 2, 1, 0)
    float* gpool[FEWHA_UNET_MAX_GROUPS][3] = {};       // of the pooled inputs of levels 1, 2, 3
    bf16_t* dpre[FEWHA_UNET_MAX_GROUPS] = {};          // bf16 ReLU-masked gradient of the current conv
    float* wpart[kConvs] = {};      // gradient partials [chunks][9 Cout Cin + Cout] (weights, bias)
    int wchunks[kConvs] = {};
    int chunk_px[kConvs] = {};      // pixels per weight-gradient chunk
    float* hpart = nullptr;         // head partials [blocks][34]
    int hblocks = 0;
    float* hred = nullptr;          // reduced head row [loss sum, gw[32], gb]

    int64_t P(int g, int level) const {
        const int s = size[g] >> level;
        return int64_t(images[g]) * s * s;
    }

    // bump allocation on the workspace (or size counting when ws is null)
    template <typename Tp>
    Tp* take(int64_t count) {
        const size_t off = used;
        used = (used + size_t(count) * sizeof(Tp) + 255) & ~size_t(255);
        return ws ? reinterpret_cast<Tp*>(ws + off) : nullptr;
    }

    void layout() {
        used = 0;
        // parameters
        int64_t o = 0, e = 0;
        for (int k = 0; k < kConvs; ++k) {
            const int64_t nw = int64_t(9) * kSpecs[k].cin * kSpecs[k].cout;
            w_off[k] = o;
            o += nw;
            b_off[k] = o;
            o += kSpecs[k].cout;
            ext_w[k] = e;
            e += nw;
            ext_b[k] = e;
            e += kSpecs[k].cout;
        }
        hw_off = o;
        o += kCh[0];
        hb_off = o;
        o += 1;
        ext_hw = e;
        e += kCh[0];
        ext_hb = e;
        e += 1;
        n_master = o;
        n_params = e;
        master = take<float>(o);
        mom1 = take<float>(o);
        mom2 = take<float>(o);
        grad = take<float>(o);
        for (int k = 0; k < kConvs; ++k) {
            wt[k] = take<bf16_t>(int64_t(9) * kSpecs[k].cin * kSpecs[k].cout);
            wd[k] = take<bf16_t>(int64_t(9) * kSpecs[k].cin * kSpecs[k].cout);
        }
        // activations
        nodes = 0;
        for (int g = 0; g < G; ++g) {
            nodes += P(g, 0);
            // every convolution input carries a zero row (one pixel of zeros after the last)
            x[g] = take<bf16_t>((P(g, 0) + 1) * kInCh);
            for (int k = 0; k < kConvs; ++k) act[g][k] = take<bf16_t>((P(g, kSpecs[k].level) + 1) * kSpecs[k].cout);
            for (int l = 0; l < 3; ++l) pool[g][l] = take<bf16_t>((P(g, l + 1) + 1) * kCh[l]);
            out[g] = take<float>(P(g, 0));
        }
        // gradients, per group
        for (int g = 0; g < G; ++g) {
            int64_t maxpc = 0;
            for (int k = 0; k < kConvs; ++k) {
                gact[g][k] = take<float>(P(g, kSpecs[k].level) * kSpecs[k].cout);
                maxpc = std::max(maxpc, P(g, kSpecs[k].level) * kSpecs[k].cout);
            }
            for (int l = 0; l < 3; ++l) {
                gcat[g][l] = take<float>(P(g, 2 - l) * kSpecs[D2A + 2 * l].cin);
                gpool[g][l] = take<float>(P(g, l + 1) * kCh[l]);
            }
            dpre[g] = take<bf16_t>(maxpc + 256);   // + a zero row of up to 256 channels
        }
        for (int k = 0; k < kConvs; ++k) {
            // chunks sized so that a convolution's launches add up to about kWBlocks workgroups
            const int64_t tiles = int64_t(kSpecs[k].cout / 32) * (kSpecs[k].cin / 32);
            int64_t pk = 0;
            for (int g = 0; g < G; ++g) pk += P(g, kSpecs[k].level);
            const int64_t want = (pk * tiles + kWBlocks - 1) / kWBlocks;
            chunk_px[k] = int(std::min<int64_t>(4096, std::max<int64_t>(64, (want + 63) / 64 * 64)));
            wchunks[k] = 0;
            for (int g = 0; g < G; ++g) wchunks[k] += int((P(g, kSpecs[k].level) + chunk_px[k] - 1) / chunk_px[k]);
            wpart[k] = take<float>(int64_t(wchunks[k]) * grad_row(k));
        }
        hblocks = 0;
        for (int g = 0; g < G; ++g) hblocks += int(blocks(P(g, 0)));
        hpart = take<float>(int64_t(hblocks) * (kCh[0] + 2));
        hred = take<float>(kCh[0] + 2);
    }

    // gradient entries of conv k: weights [9][Cout][Cin], then bias [Cout]
    static int64_t grad_row(int k) { return int64_t(9) * kSpecs[k].cin * kSpecs[k].cout + kSpecs[k].cout; }

    // ---- launches
    // upsampled channels of a decoder concatenation: the coarser level's channel count
    static int concat_c1(int k) { return kSpecs[k].cin - kSpecs[k].cout; }

    const bf16_t* conv_in0(int k, int g) const {
        switch (k) {
            case E0A: return x[g];
            case E1A: return pool[g][0];
            case E2A: return pool[g][1];
            case E3A: return pool[g][2];
            case D2A: return act[g][E3B];
            case D1A: return act[g][D2B];
            case D0A: return act[g][D1B];
            default: return act[g][k - 1];
        }
    }
    const bf16_t* conv_in1(int k, int g) const {
        switch (k) {
            case D2A: return act[g][E2B];
            case D1A: return act[g][E1B];
            case D0A: return act[g][E0B];
            default: return nullptr;
        }
    }

    // 3x3 convolution launch over the groups of `cg` (their N and H set): the reduction is
    // split over the wavefronts of a workgroup (KS = 2 or 4) when the output alone gives fewer
    // than 768 workgroups of 256 pixels
    template <int MODE, bool OUT>
    static void conv(ConvGroups cg, int C1, int Cin, const bf16_t* w, const float* bias, int relu, int Cout,
                     hipStream_t s) {
        int64_t b1 = 0;
        for (int g = 0; g < cg.count; ++g) b1 += int64_t(blocks(int64_t(cg.g[g].N) * cg.g[g].H * cg.g[g].H, kConvPix));
        b1 *= Cout / 32;
        const int ks = b1 >= 768 ? 1 : Cin % 128 == 0 ? 4 : Cin % 64 == 0 ? 2 : 1;
        int nb = 0;
        for (int g = 0; g < cg.count; ++g) {
            cg.g[g].block0 = nb;
            nb += int(blocks(int64_t(cg.g[g].N) * cg.g[g].H * cg.g[g].H, kConvPix / ks));
        }
        cg.g[cg.count].block0 = nb;
        const dim3 grid(nb, Cout / 32);
        if (ks == 4)
            k_conv3x3<MODE, OUT, 4><<<grid, kT, 0, s>>>(cg, C1, Cin, w, bias, relu, Cout);
        else if (ks == 2)
            k_conv3x3<MODE, OUT, 2><<<grid, kT, 0, s>>>(cg, C1, Cin, w, bias, relu, Cout);
        else
            k_conv3x3<MODE, OUT, 1><<<grid, kT, 0, s>>>(cg, C1, Cin, w, bias, relu, Cout);
    }

    static ConvGroups one_group(const bf16_t* in0, const bf16_t* in1, void* out, int N, int H) {
        ConvGroups cg{};
        cg.g[0] = ConvGroup{in0, in1, out, N, H, 0};
        cg.count = 1;
        return cg;
    }

    // forward pass of every group, each convolution one launch over all groups
    void forward_all(const float* in, hipStream_t s) {
        int64_t o = 0;
        for (int g = 0; g < G; ++g) {
            const int64_t P0 = P(g, 0);
            k_pack_input<<<blocks(P0 * kInCh), kT, 0, s>>>(in + o * kInputs, P0, x[g]);
            o += P0;
        }
        for (int k = 0; k < kConvs; ++k) {
            const ConvSpec& c = kSpecs[k];
            ConvGroups cg{};
            cg.count = G;
            for (int g = 0; g < G; ++g) {
                if (k == E1A || k == E2A || k == E3A) {   // pool the previous level's output
                    const int l = c.level - 1, Hs = size[g] >> l;
                    k_pool2<<<blocks(P(g, l + 1) * kCh[l]), kT, 0, s>>>(act[g][k - 1], images[g], Hs, Hs, kCh[l],
                                                                        pool[g][l]);
                }
                cg.g[g] = ConvGroup{conv_in0(k, g), conv_in1(k, g), act[g][k], images[g], size[g] >> c.level, 0};
            }
            const float* bias = master + b_off[k];
            if (c.concat)
                conv<CONV_CONCAT_UP, true>(cg, concat_c1(k), c.cin, wt[k], bias, 1, c.cout, s);
            else
                conv<CONV_DIRECT, true>(cg, 0, c.cin, wt[k], bias, 1, c.cout, s);
        }
        for (int g = 0; g < G; ++g) {
            const int64_t P0 = P(g, 0);
            k_head<<<blocks(P0), kT, 0, s>>>(act[g][D0B], master + hw_off, master + hb_off, P0, out[g]);
        }
    }

    // gradient of conv k's output is in gact[g][k] for every group: ReLU' per group, then the
    // weight/bias partials and (unless k == E0A) the input gradient into gin[g] (FP32), each
    // one launch over all groups
    void conv_back(int k, float* const* gin, hipStream_t s) {
        const ConvSpec& c = kSpecs[k];
        WgradGroups wg{};
        ConvGroups cg{};
        wg.count = cg.count = G;
        int nb = 0;
        for (int g = 0; g < G; ++g) {
            const int H = size[g] >> c.level;
            const int64_t Pn = P(g, c.level);
            k_relu_grad<<<blocks((Pn + 1) * c.cout), kT, 0, s>>>(gact[g][k], act[g][k], Pn * c.cout, c.cout, dpre[g]);
            wg.g[g] = WgradGroup{dpre[g], conv_in0(k, g), conv_in1(k, g), images[g], H, nb};
            nb += int(blocks(Pn, chunk_px[k]));
            if (gin) cg.g[g] = ConvGroup{dpre[g], nullptr, gin[g], images[g], H, 0};
        }
        wg.g[G].block0 = nb;
        const dim3 grid(nb, (c.cout / 32) * (c.cin / 32));
        if (c.concat)
            k_conv_wgrad<CONV_CONCAT_UP><<<grid, kT, 0, s>>>(wg, concat_c1(k), c.cin, c.cout, chunk_px[k], wpart[k]);
        else
            k_conv_wgrad<CONV_DIRECT><<<grid, kT, 0, s>>>(wg, 0, c.cin, c.cout, chunk_px[k], wpart[k]);
        if (gin) conv<CONV_DIRECT, false>(cg, 0, c.cout, wd[k], nullptr, 0, c.cin, s);
    }

    void backward_all(const float* target, double total, hipStream_t s) {
        int64_t o = 0;
        int hb = 0;
        for (int g = 0; g < G; ++g) {
            const int64_t P0 = P(g, 0);
            k_head_back<<<blocks(P0), kT, 0, s>>>(out[g], target + o, act[g][D0B], master + hw_off, P0, total,
                                                  gact[g][D0B], hpart, hb);
            o += P0;
            hb += int(blocks(P0));
        }
        float* gin[FEWHA_UNET_MAX_GROUPS];
        auto back = [&](int k, auto target_of) {
            for (int g = 0; g < G; ++g) gin[g] = target_of(g);
            conv_back(k, target_of(0) ? gin : nullptr, s);
        };
        auto split = [&](int lvl_out, int l, int klow, int kskip, int c1, int c2) {
            for (int g = 0; g < G; ++g) {
                const int H = size[g] >> lvl_out;
                const int64_t n = P(g, lvl_out + 1) * c1 + P(g, lvl_out) * c2;
                k_split_concat_grad<<<blocks(n), kT, 0, s>>>(gcat[g][l], images[g], H, H, c1, c2, gact[g][klow],
                                                             gact[g][kskip]);
            }
        };
        auto pool_add = [&](int lvl, int kf, int C) {
            for (int g = 0; g < G; ++g) {
                const int H = size[g] >> lvl;
                k_pool2_grad_add<<<blocks(P(g, lvl) * C), kT, 0, s>>>(gpool[g][lvl], images[g], H, H, C, gact[g][kf]);
            }
        };
        auto ga = [&](int k) { return [this, k](int g) { return gact[g][k]; }; };
        auto gc = [&](int l) { return [this, l](int g) { return gcat[g][l]; }; };
        auto gp = [&](int l) { return [this, l](int g) { return gpool[g][l]; }; };
        // decoder
        back(D0B, ga(D0A));
        back(D0A, gc(2));
        split(0, 2, D1B, E0B, kCh[1], kCh[0]);
        back(D1B, ga(D1A));
        back(D1A, gc(1));
        split(1, 1, D2B, E1B, kCh[2], kCh[1]);
        back(D2B, ga(D2A));
        back(D2A, gc(0));
        split(2, 0, E3B, E2B, kCh[3], kCh[2]);
        // encoder
        back(E3B, ga(E3A));
        back(E3A, gp(2));
        pool_add(2, E2B, kCh[2]);
        back(E2B, ga(E2A));
        back(E2A, gp(1));
        pool_add(1, E1B, kCh[1]);
        back(E1B, ga(E1A));
        back(E1A, gp(0));
        pool_add(0, E0B, kCh[0]);
        back(E0B, ga(E0A));
        back(E0A, [](int) { return static_cast<float*>(nullptr); });
    }
};

namespace {

thread_local std::string g_unet_err;

fewha_status ufail(fewha_unet* n, fewha_status st, const std::string& m) {
    if (n) n->err = m;
    else g_unet_err = m;
    return st;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

fewha_status validate(const fewha_unet_config* c, std::string& err) {
    if (!c) { err = "config is NULL"; return FEWHA_E_INVAL; }
    if (c->abi_version != FEWHA_ABI_VERSION) { err = "abi_version mismatch"; return FEWHA_E_INVAL; }
    if (c->n_groups < 1 || c->n_groups > FEWHA_UNET_MAX_GROUPS) { err = "n_groups out of range"; return FEWHA_E_INVAL; }
    for (int g = 0; g < c->n_groups; ++g) {
        const int s = c->size[g];
        if (s < 16 || s > 4096 || (s & (s - 1))) { err = "image size must be a power of two in [16, 4096]"; return FEWHA_E_INVAL; }
        if (c->images[g] < 1) { err = "images per group must be >= 1"; return FEWHA_E_INVAL; }
        if (int64_t(c->images[g]) * s * s > (int64_t(1) << 25)) { err = "group too large (at most 2^25 nodes)"; return FEWHA_E_INVAL; }
    }
    if (!(c->lr > 0) || !(c->beta1 >= 0 && c->beta1 < 1) || !(c->beta2 >= 0 && c->beta2 < 1) || !(c->eps > 0)) {
        err = "bad Adam settings";
        return FEWHA_E_INVAL;
    }
    return FEWHA_OK;
}

void configure(fewha_unet& n, const fewha_unet_config* c) {
    n.G = c->n_groups;
    for (int g = 0; g < n.G; ++g) {
        n.images[g] = c->images[g];
        n.size[g] = c->size[g];
    }
    n.lr = c->lr;
    n.b1 = c->beta1;
    n.b2 = c->beta2;
    n.eps = c->eps;
}

fewha_status check(fewha_unet* n) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ufail(n, FEWHA_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return FEWHA_OK;
}

}  // namespace

extern "C" {

fewha_status fewha_unet_workspace_size(const fewha_unet_config* cfg, size_t* bytes) {
    std::string err;
    const fewha_status st = validate(cfg, err);
    if (st != FEWHA_OK) return ufail(nullptr, st, err);
    if (!bytes) return FEWHA_E_INVAL;
    fewha_unet n;
    configure(n, cfg);
    n.layout();
    *bytes = n.used;
    return FEWHA_OK;
}

fewha_status fewha_unet_setup(const fewha_unet_config* cfg, void* d_workspace, size_t bytes, void* stream,
                              fewha_unet** out) {
    if (!out) return FEWHA_E_INVAL;
    *out = nullptr;
    std::string err;
    fewha_status st = validate(cfg, err);
    if (st != FEWHA_OK) return ufail(nullptr, st, err);
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255))
        return ufail(nullptr, FEWHA_E_INVAL, "workspace must be a 256-byte aligned device pointer");
    fewha_unet* n = new (std::nothrow) fewha_unet();
    if (!n) return FEWHA_E_NOMEM;
    configure(*n, cfg);
    n->layout();
    if (bytes < n->used) {
        const size_t need = n->used;
        delete n;
        return ufail(nullptr, FEWHA_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    }
    n->ws = static_cast<char*>(d_workspace);
    n->ws_bytes = bytes;
    n->layout();
    hipStream_t s = as_stream(stream);
    if (hipMemsetAsync(n->ws, 0, n->used, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        delete n;
        return ufail(nullptr, FEWHA_E_HIP, "workspace initialisation failed");
    }
    *out = n;
    return FEWHA_OK;
}

fewha_status fewha_unet_num_params(const fewha_unet* net, int64_t* n) {
    if (!net || !n) return FEWHA_E_INVAL;
    *n = net->n_params;
    return FEWHA_OK;
}

fewha_status fewha_unet_num_nodes(const fewha_unet* net, int64_t* n) {
    if (!net || !n) return FEWHA_E_INVAL;
    *n = net->nodes;
    return FEWHA_OK;
}

fewha_status fewha_unet_set_params(fewha_unet* net, const float* d_params, void* stream) {
    if (!net || !d_params) return ufail(net, FEWHA_E_INVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    float* ext = const_cast<float*>(d_params);   // read only (direction 0)
    for (int k = 0; k < kConvs; ++k) {
        const int64_t nw = int64_t(9) * kSpecs[k].cin * kSpecs[k].cout;
        k_conv_layout<<<blocks(nw), kT, 0, s>>>(ext + net->ext_w[k], net->master + net->w_off[k], kSpecs[k].cin,
                                                kSpecs[k].cout, 0, net->wt[k], net->wd[k]);
        k_copy<<<blocks(kSpecs[k].cout), kT, 0, s>>>(net->master + net->b_off[k], d_params + net->ext_b[k],
                                                     kSpecs[k].cout);
    }
    k_copy<<<1, kT, 0, s>>>(net->master + net->hw_off, d_params + net->ext_hw, kCh[0]);
    k_copy<<<1, kT, 0, s>>>(net->master + net->hb_off, d_params + net->ext_hb, 1);
    k_zero<<<blocks(net->n_master), kT, 0, s>>>(net->mom1, net->n_master);
    k_zero<<<blocks(net->n_master), kT, 0, s>>>(net->mom2, net->n_master);
    net->step = 0;
    return check(net);
}

static fewha_status export_vec(fewha_unet* net, const float* src, float* d_out, hipStream_t s) {
    for (int k = 0; k < kConvs; ++k) {
        const int64_t nw = int64_t(9) * kSpecs[k].cin * kSpecs[k].cout;
        k_conv_layout<<<blocks(nw), kT, 0, s>>>(d_out + net->ext_w[k], const_cast<float*>(src) + net->w_off[k],
                                                kSpecs[k].cin, kSpecs[k].cout, 1, nullptr, nullptr);
        k_copy<<<blocks(kSpecs[k].cout), kT, 0, s>>>(d_out + net->ext_b[k], src + net->b_off[k], kSpecs[k].cout);
    }
    k_copy<<<1, kT, 0, s>>>(d_out + net->ext_hw, src + net->hw_off, kCh[0]);
    k_copy<<<1, kT, 0, s>>>(d_out + net->ext_hb, src + net->hb_off, 1);
    return check(net);
}

fewha_status fewha_unet_get_params(fewha_unet* net, float* d_params, void* stream) {
    if (!net || !d_params) return ufail(net, FEWHA_E_INVAL, "NULL argument");
    return export_vec(net, net->master, d_params, as_stream(stream));
}

fewha_status fewha_unet_get_grads(fewha_unet* net, float* d_grads, void* stream) {
    if (!net || !d_grads) return ufail(net, FEWHA_E_INVAL, "NULL argument");
    return export_vec(net, net->grad, d_grads, as_stream(stream));
}

fewha_status fewha_unet_forward(fewha_unet* net, const float* d_in, float* d_out, void* stream) {
    if (!net || !d_in || !d_out) return ufail(net, FEWHA_E_INVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    net->forward_all(d_in, s);
    int64_t o = 0;
    for (int g = 0; g < net->G; ++g) {
        const int64_t P0 = net->P(g, 0);
        k_copy<<<blocks(P0), kT, 0, s>>>(d_out + o, net->out[g], P0);
        o += P0;
    }
    return check(net);
}

fewha_status fewha_unet_backward(fewha_unet* net, const float* d_in, const float* d_target, float* d_loss,
                                 void* stream) {
    if (!net || !d_in || !d_target) return ufail(net, FEWHA_E_INVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    const double total = double(net->nodes);
    net->forward_all(d_in, s);
    net->backward_all(d_target, total, s);
    // fixed-order reduction of every partial into the gradient vector (conv weights and bias
    // rows, then the head row [loss sum, gw[32], gb]), one launch
    // the tensors with the most chunks (the longest workgroups) are dispatched first
    int order[kConvs + 1];
    for (int k = 0; k <= kConvs; ++k) order[k] = k;
    auto chunks_of = [&](int k) { return k == kConvs ? net->hblocks : net->wchunks[k]; };
    std::stable_sort(order, order + kConvs + 1, [&](int a, int b) { return chunks_of(a) > chunks_of(b); });
    ReduceTable tb{};
    int nb = 0;
    for (int t = 0; t <= kConvs; ++t) {
        const int k = order[t];
        const bool head = k == kConvs;
        tb.part[t] = head ? net->hpart : net->wpart[k];
        tb.out[t] = head ? net->hred : net->grad + net->w_off[k];
        tb.n[t] = head ? kCh[0] + 2 : fewha_unet::grad_row(k);
        tb.chunks[t] = chunks_of(k);
        // at most 32 chunks per thread, at most eight threads per element
        int S = 1;
        while (S < 8 && tb.chunks[t] > 32 * S) S *= 2;
        tb.stripes[t] = S;
        tb.block0[t] = nb;
        nb += int((tb.n[t] + kT / S - 1) / (kT / S));
    }
    tb.count = kConvs + 1;
    tb.block0[kConvs + 1] = nb;
    k_reduce_table<<<nb, kT, 0, s>>>(tb);
    k_head_finish<<<1, 64, 0, s>>>(net->hred, total, d_loss, net->grad + net->hw_off, net->grad + net->hb_off);
    return check(net);
}

fewha_status fewha_unet_adam_step(fewha_unet* net, void* stream) {
    if (!net) return FEWHA_E_INVAL;
    hipStream_t s = as_stream(stream);
    net->step += 1;
    const float c1 = float(1.0 - std::pow(double(net->b1), net->step));
    const float c2 = float(1.0 - std::pow(double(net->b2), net->step));
    AdamTable tb{};
    for (int k = 0; k < kConvs; ++k) {
        tb.w_off[k] = net->w_off[k];
        tb.nw[k] = int64_t(9) * kSpecs[k].cin * kSpecs[k].cout;
        tb.wt[k] = net->wt[k];
        tb.wd[k] = net->wd[k];
        tb.cout[k] = kSpecs[k].cout;
        tb.cin[k] = kSpecs[k].cin;
    }
    k_adam<<<blocks(net->n_master), kT, 0, s>>>(net->master, net->mom1, net->mom2, net->grad, net->n_master, net->lr,
                                                net->b1, net->b2, net->eps, c1, c2, tb);
    return check(net);
}

fewha_status fewha_unet_groups(const fewha_unet* net, int32_t* images, int32_t* size, int32_t* n_groups) {
    if (!net) return FEWHA_E_INVAL;
    for (int g = 0; g < net->G; ++g) {
        if (images) images[g] = net->images[g];
        if (size) size[g] = net->size[g];
    }
    if (n_groups) *n_groups = net->G;
    return FEWHA_OK;
}

fewha_status fewha_unet_destroy(fewha_unet* net) {
    delete net;
    return FEWHA_OK;
}

const char* fewha_unet_last_error(const fewha_unet* net) { return net ? net->err.c_str() : g_unet_err.c_str(); }

}  // extern "C"
