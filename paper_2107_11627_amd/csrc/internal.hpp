// Internal declarations of libp2s: handle layouts, kernel launchers and the
// small device helpers the kernels share.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "p2s.h"

namespace p2s {

// ------------------------------------------------------------------ types
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef float floatx8 __attribute__((ext_vector_type(8)));

// Device copy of a PSF basis, laid out as MFMA A-operands (rows = basis
// functions in blocks of 16, reduction = PSF taps).  Taps are stored in
// correlation order: the operand for tap offset (dy, dx) multiplies the image
// sample at (y + dy, x + dx) and holds phi_k[R - dy][R - dx].
struct Basis {
    int K, P, R;
    int nmb;              // ceil(K / 16)
    // FP32: [t4][nmb][64] floats, lane L of step t -> basis 16 mb + L%16,
    // tap u = 4 t + L/16 in row-major (dy + R, dx + R) order (zero past P*P).
    int t4;
    float* f32;
    // BF16: [t32][nmb][64][8] bf16, chunk c = 4 t + L/16 of 8 taps:
    //   c <  P*A8          row chunk: dy = c / A8 - R, taps dx = (c % A8) * 8 - R + e
    //   c <  P*A8 + ncol   column chunk q: taps (dy = -R + 8 q + e, dx = R)
    //   otherwise          zero
    // with A8 = P / 8 and ncol = ceil(P / 8); only P = 8 A8 + 1 is laid out.
    int t32;
    int bf16_ok;
    uint16_t* bf16;
    // FP8 E4M3 (v_mfma_scale_f32_16x16x128_f8f6f4): [t128][nmb][64][32] bytes;
    // lane L of step t supplies chunks 16 t + 4 (L/16) + j, j = 0..3, as bytes
    // 8 j .. 8 j + 7 (same chunk numbering as BF16).  Basis k is stored as
    // E4M3(phi_k * 2^e_k); fp8_scale[k] = 127 - e_k is the E8M0 code of
    // 2^-e_k that the MFMA applies to row k (127, i.e. 1, for padding rows).
    int t128;
    uint8_t* fp8;
    int* fp8_scale;       // [16 nmb]
};

struct Mlp {
    int L;
    int dims[P2S_MAX_LAYERS + 1];
    int mb;               // every layer's output padded to mb blocks of 16
    // FP32 A-operands (v_mfma_f32_16x16x4f32): per layer [mb][nkc][64]
    //   layer 0 chunk kc: lane group g -> input feature 4 kc + g
    //   layer l > 0 chunk kc = 4 mb' + i: lane group g -> feature 16 mb' + 4 g + i
    float* w32;
    size_t off32[P2S_MAX_LAYERS];
    int nkc32[P2S_MAX_LAYERS];
    size_t bytes32;
    // BF16 A-operands (v_mfma_f32_16x16x32_bf16): per layer [mb][nkc][64][8]
    //   layer 0 chunk kc (2 chunks): lane group g, element e -> feature 32 kc + 8 g + e
    //   layer l > 0 chunk kc: element e -> feature 16 (2 kc + e / 4) + 4 g + e % 4
    uint16_t* w16;
    size_t off16[P2S_MAX_LAYERS];
    int nkc16[P2S_MAX_LAYERS];
    size_t bytes16;
    float* bias;          // per layer, padded to 16 * mb
    int boff[P2S_MAX_LAYERS];
};

// Device copy of the anchor-grid field model: the lower Cholesky factors of
// the anchor correlation matrix (FP32 [Gp][ld], row-major, zero above the
// diagonal and in the padding rows and columns; Gp = G^2 rounded up to 32, and
// the row stride ld = Gp + 32 so that the rows of a tile, read together, do
// not all fall on a power-of-two stride) and of the mode covariance per
// (D/r0)^(5/3) (FP32 [n][n], zero above the diagonal).  nct = ceil(n / 16)
// column tiles of the product.
struct Anchor {
    int G, n, Gp, ld, nct;
    float* Ls;
    float* Lz;
};

// Packed network weights are staged in the LDS of one workgroup.
constexpr size_t kMlpLdsBytes = 160 * 1024;

// ------------------------------------------------------------- launchers
struct FieldPlan {
    int H, W, Nfy, Nfx, nplanes, npairs;
    uint32_t k0, k1;
    float corr_len;
    float norm;                      // 1 / (sqrt(mean S_y mean S_x) sqrt(Nfy Nfx))
    int kcx, kcy;                    // band half-widths (filter >= 1e-9 of its peak)
    int Mx, My;                      // band sizes, min(N, 2 kc + 1)
    int nrad_x, nrad_y;
    int rad_x[12], rad_y[12];        // radix passes, product = Nfx / Nfy
    float sigma[P2S_MAX_ZERNIKE];    // per-plane standard deviation
};

// ------------------------------------------------------------- batches
// One frame of a batch as the batched kernels see it (device memory).
struct FrameDesc {
    const float* image;
    float* out;
    float* fields;                   // [nz][H][W]
    float* w;                        // [H*W][K]
    float* blurred;                  // [C][H][W]
    float2* V;                       // field intermediate [pairs][Mx][H]
    float2* twx;                     // [Nfx] row twiddles
    int C, H, W;
    int tiles_x, tiles_y;            // blur tiles
    int lg_cpb, lg_rpb;              // field transforms per workgroup item (log2)
    int ncol_chunks, nrow_chunks;    // field items per plane pair
    int mlp_groups;                  // network pixel groups
    int warp_tiles_x, warp_tiles;    // warp items
    FieldPlan fp;
};

enum { ST_COLS = 0, ST_ROWS, ST_MLP, ST_BLUR, ST_WARP, ST_N };

// Launch description of a planned batch: device pointers to the frame table
// and to the per-stage prefix sums of work items (first[stage][n + 1]), plus
// per-stage grid and LDS sizes.
struct BatchLaunch {
    const FrameDesc* frames;
    const int* first;
    int n;
    int items[ST_N];
    int grid[ST_N];
    size_t lds[ST_N];
    int blur_rows;                   // 16 or 8 rows per blur tile
};

// Index of the frame whose items contain `item` (first[0] = 0, first[n] = total).
__device__ __forceinline__ int find_frame(const int* __restrict__ first, int n, int item) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

constexpr size_t kColsLdsBudget = 48 * 1024;
constexpr size_t kRowsLdsBudget = 48 * 1024;
size_t fields_cols_lds(int N, int nb);
size_t fields_rows_lds(int N, int nb);
int fields_pick_lg(int N, size_t budget, bool cols);
hipError_t launch_fields_batch(const BatchLaunch& bl, hipStream_t s);
hipError_t launch_mlp_batch(const Mlp& m, const BatchLaunch& bl, p2s_precision prec, hipStream_t s);
hipError_t launch_blur_batch(const Basis& b, const BatchLaunch& bl, p2s_precision prec, hipStream_t s);
hipError_t launch_warp_batch(const BatchLaunch& bl, double scale, hipStream_t s);
int mlp_pixels_per_group();
int blur_tile_rows(p2s_precision prec, int nmb, int preferred);
// Workgroups of each batched kernel the whole device holds at once.
int fields_batch_resident(bool cols, size_t lds);
int mlp_batch_resident(const Mlp& m, p2s_precision prec);
int blur_batch_resident(const Basis& b, p2s_precision prec, int rows);
int warp_batch_resident();

int num_cus();
inline int resident_workgroups(const void* fn, int threads, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, lds) != hipSuccess || nb < 1) nb = 1;
    return nb * num_cus();
}

int factor_radices(int n, int* rad);   // -> number of passes, 0 if not 5-smooth
hipError_t launch_fields(const FieldPlan& fp, float* V, float* F, hipStream_t s);
hipError_t launch_debug_noise(int Nfy, int Nfx, int pair, uint32_t k0, uint32_t k1,
                              uint32_t* raw, float* normals, hipStream_t s);
hipError_t launch_mlp(const Mlp& m, const float* fields, int H, int W, p2s_precision prec,
                      float* w, hipStream_t s);
hipError_t launch_blur(const Basis& b, const float* img, int C, int H, int W, const float* w,
                       p2s_precision prec, float* out, hipStream_t s);
hipError_t launch_warp(const float* in, int C, int H, int W, const float* tilt, double scale,
                       float* out, hipStream_t s);
// Network fused into the blur (BF16 network, BF16 or FP8 blur); `fields` is
// the frame's full [nz][H][W] array.
bool blur_mlp_supported(const Basis& b, const Mlp& m, p2s_precision prec);
size_t network_lds_bytes(const Mlp& m);               // packed BF16 weights + biases
int blur_mlp_tile_rows(p2s_precision prec, int nmb);   // output rows per fused work item
int blur_mlp_batch_resident(const Basis& b, const Mlp& m, p2s_precision prec);
hipError_t launch_blur_mlp(const Basis& b, const Mlp& m, p2s_precision prec, const float* img, int C, int H, int W,
                           const float* fields, float* out, hipStream_t s);
hipError_t launch_blur_mlp_batch(const Basis& b, const Mlp& m, const BatchLaunch& bl, p2s_precision prec,
                                 hipStream_t s);

// Anchor-grid fields: noise, triangular product and interpolation on stream s;
// ws holds anchor_ws_bytes.  anchor_window_cols: anchor columns one segment of
// seg pixels of a W-wide image touches (its LDS window is 2 rows of them).
int anchor_window_cols(int G, int W, int seg);
size_t anchor_ws_bytes(const Anchor& an);
hipError_t launch_anchor_fields(const Anchor& an, int H, int W, double D_over_r0, uint32_t k0, uint32_t k1,
                                float* fields, void* ws, hipStream_t s);

// --------------------------------------------------------- host helpers
uint16_t f32_to_bf16_rne(float x);
uint8_t f32_to_e4m3_rne(float x);     // OCP E4M3, ties to even, |x| clamped to 448
int e4m3_scale_exponent(float amax);  // largest e with amax 2^e <= 448 (0 for 0), within +-127

// ------------------------------------------------------- device helpers
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 bit
// products on words 0 and 2, key advanced by the Weyl constants between
// rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t lo0 = 0xD2511F53u * c0;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Box-Muller pair from two Philox outputs: u_a = ((o0 >> 8) + 1) 2^-24 in
// (0, 1], u_b = (o1 >> 8) 2^-24 in [0, 1) (both exact in FP32);
// returns sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b).
__device__ __forceinline__ float2 box_muller(uint32_t o0, uint32_t o1) {
    const float two24 = 5.9604644775390625e-08f;   // 2^-24
    const float ua = (float)((o0 >> 8) + 1u) * two24, ub = (float)(o1 >> 8) * two24;
    const float r = sqrtf(-2.0f * logf(ua));
    float s, c;
    sincospif(2.0f * ub, &s, &c);
    return make_float2(r * c, r * s);
}

__device__ __forceinline__ uint32_t bf16_bits_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }
// Eight float32 values to bfloat16, round to nearest even (one conversion
// instruction per pair on gfx950); bit-identical to bf16_bits_rne for finite
// values.
__device__ __forceinline__ bf16x8 to_bf16x8(floatx8 v) { return __builtin_convertvector(v, bf16x8); }
__device__ __forceinline__ floatx8 from_bf16x8(bf16x8 v) { return __builtin_convertvector(v, floatx8); }

}  // namespace p2s
