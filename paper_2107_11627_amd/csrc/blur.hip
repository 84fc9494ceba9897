// Stage 3 of the hot path: the spatially varying blur of Sec. 3.1 in its
// basis form (Eq. 4-5),
//
//   out_c(x) = sum_k w_k(x) * sum_u phi_k(u) I_c(clamp(x - u)),
//
// computed per output tile as one GEMM on MFMA followed by a row dot:
//   conv[k][pixel] = sum_taps basis[k][tap] * patch[tap][pixel]  (MFMA, FP32 acc)
//   out[pixel]     = sum_k conv[k][pixel] * w[pixel][k]           (epilogue)
// The K convolution results live only in accumulator registers.
//
// A operand = basis (rows: 16 basis functions per block), B operand = image
// patches (columns: 16 consecutive pixels of one image row), reduction over
// PSF taps.  The accumulator lane layout (basis 16 mb + 4 (L/16) + i, pixel
// L%16) lets each lane fold its 4 basis rows per block against w with one
// float4 load, leaving a 4-way cross-lane sum.
//
// Tile: 16 x 32 pixels of one channel per workgroup (4 waves, each 4 rows x
// 32 pixels = 8 pixel blocks), or 8 x 32 with 4 pixel blocks per wave when
// K > 112; grid = tiles x channels.
#include "mlp_block.hpp"

namespace p2s {
namespace {

constexpr int kTX = 32;
constexpr int kMaxR = (P2S_MAX_P - 1) / 2;

__device__ __forceinline__ float wave_sum4(float v) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// Epilogue shared by both precisions: dot the accumulators with w and store.
// The w loads of GB pixel blocks are all issued before any is used (address
// clamped in bounds, out-of-range terms masked), so one memory round trip
// serves GB * NMB loads instead of one each.
template <int NMB, int NBLK>
__device__ __forceinline__ void epilogue(const floatx4 (&acc)[NBLK][NMB], const float* __restrict__ w, int K,
                                         int yw, int x0, int H, int W, int g, int m, float* __restrict__ out_c) {
    constexpr int GB = NBLK < 4 ? NBLK : 4;
#pragma unroll
    for (int b0 = 0; b0 < NBLK; b0 += GB) {
        __builtin_amdgcn_sched_barrier(0);   // keep each batch's loads and sums together
        float wv[GB][NMB][4];
#pragma unroll
        for (int bb = 0; bb < GB; ++bb) {
            const int b = b0 + bb;
            const int y = yw + (b >> 1), x = x0 + (b & 1) * 16 + m;
            const size_t pix = (y < H && x < W) ? (size_t)y * W + x : 0;
            const float* wp = w + pix * K;
            if ((K & 3) == 0) {
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb) {
                    const int k = 16 * mb + 4 * g;
                    const float4 v = *reinterpret_cast<const float4*>(wp + (k < K ? k : 0));
                    wv[bb][mb][0] = v.x;
                    wv[bb][mb][1] = v.y;
                    wv[bb][mb][2] = v.z;
                    wv[bb][mb][3] = v.w;
                }
            } else {
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int k = 16 * mb + 4 * g + i;
                        wv[bb][mb][i] = wp[k < K ? k : 0];
                    }
            }
        }
#pragma unroll
        for (int bb = 0; bb < GB; ++bb) {
            const int b = b0 + bb;
            const int y = yw + (b >> 1), x = x0 + (b & 1) * 16 + m;
            float part = 0.0f;
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = 16 * mb + 4 * g + i;
                    if (k < K) part = fmaf(acc[b][mb][i], wv[bb][mb][i], part);
                }
            part = wave_sum4(part);
            if (y < H && x < W && g == 0) out_c[(size_t)y * W + x] = part;
        }
    }
}

// Epilogue sources for the low-precision tiles (called with the accumulators,
// the wave's first output row, the tile's first column, the lane's (g, m) and
// the channel).  WFromMemory reads w from the [H*W][K] array; WFromNetwork
// evaluates the P2S network for each pair of pixel blocks from the field
// planes (weights in LDS), so that w never exists in memory.  Both produce the
// same values: the network arithmetic does not depend on which pixels share
// an MFMA.
template <int NMB, int NBLK>
struct WFromMemory {
    const float* w;
    int K, H, W;
    float* out;
    __device__ __forceinline__ void prefetch(int, int, int) {}
    __device__ __forceinline__ void settle() {}
    __device__ __forceinline__ void begin(int, int, int, int) {}
    __device__ __forceinline__ void operator()(const floatx4 (&acc)[NBLK][NMB], int yw, int x0, int g, int m,
                                               int c) const {
        epilogue<NMB, NBLK>(acc, w, K, yw, x0, H, W, g, m, out + (size_t)c * H * W);
    }
};

template <int NMB, int NBLK, bool EVAL, bool LO = true>
struct WFromNetwork {
    const MlpArgs* a;
    const uint4* lds_w16;
    const float* bias;
    const float* fields2;             // plane 2 (alpha_4) of the frame's fields
    int H, W;
    float* out;
    float in[NBLK][2][8];             // the network inputs of the wave's pixel blocks
    float wv[NBLK][NMB][4];           // the tile's weights (EVAL: computed before the convolutions)

    __device__ __forceinline__ int pixel(int b, int yw, int x0, int m, bool& ok) const {
        const int y = yw + (b >> 1), x = x0 + (b & 1) * 16 + m;
        ok = y < H && x < W;
        return ok ? y * W + x : 0;
    }

    // At the start of a tile: the field loads, in flight while the image is
    // staged.
    __device__ __forceinline__ void prefetch(int yw, int x0, int m) {
        if constexpr (!EVAL) return;
        int pixc[NBLK];
        bool ok;
#pragma unroll
        for (int b = 0; b < NBLK; ++b) pixc[b] = pixel(b, yw, x0, m, ok);
        mlp_load_inputs<NBLK>(*a, fields2, H * W, pixc, in);
    }

    // Take delivery of the field loads here, before the next window's copy is
    // started: the compiler waits for every outstanding memory operation
    // when a register loaded before a global_load_lds is first used, so a
    // first use after the copy would wait for the copy as well.
    __device__ __forceinline__ void settle() {
        if constexpr (!EVAL) return;
#pragma unroll
        for (int b = 0; b < NBLK; ++b)
#pragma unroll
            for (int kc = 0; kc < 2; ++kc)
#pragma unroll
                for (int e = 0; e < 8; ++e) asm volatile("" : "+v"(in[b][kc][e]));
    }

    // Before the convolutions, while no accumulator is live: the network for
    // the wave's pixel blocks, two at a time with bf16 hi + lo activations
    // (every weight read from LDS serves both; more at once would need two
    // full activation sets of registers for each), four at a time with bf16
    // activations alone (half the registers per block).
    __device__ __forceinline__ void begin(int, int, int, int) {
        if constexpr (!EVAL) return;
        constexpr int GB = !LO && NBLK >= 4 ? 4 : (NBLK >= 2 ? 2 : NBLK);
#pragma unroll
        for (int b0 = 0; b0 < NBLK; b0 += GB) {
            const float (&ig)[GB][2][8] = *reinterpret_cast<const float (*)[GB][2][8]>(&in[b0]);
            float (&og)[GB][NMB][4] = *reinterpret_cast<float (*)[GB][NMB][4]>(&wv[b0]);
            mlp_bf16_eval<NMB, GB, LO>(*a, lds_w16, bias, ig, og);
        }
    }

    __device__ __forceinline__ void operator()(const floatx4 (&acc)[NBLK][NMB], int yw, int x0, int g, int m,
                                               int c) const {
        float* out_c = out + (size_t)c * H * W;
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            bool ok;
            const int pix = pixel(b, yw, x0, m, ok);
            // Rows k >= K: basis and last-layer weights and biases are
            // zero-padded, so both factors are exactly 0 there and their
            // fused multiply-add leaves part as it is (part is never -0): the
            // same sum, bit for bit, as the memory-reading epilogue's, which
            // skips those rows.
            float part = 0.0f;
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) part = fmaf(acc[b][mb][i], wv[b][mb][i], part);
            part = wave_sum4(part);
            if (ok && g == 0) out_c[pix] = part;
        }
    }
};

// A tile buffer in LDS, one per (type, size, tag) and kernel: the fused
// kernel instantiates a tile function twice (channel 0 with the network, the
// other channels without), and both instances share these buffers.
template <class T, int N, int TAG>
__device__ __forceinline__ T* lds_buffer() {
    __shared__ __attribute__((aligned(16))) T buf[N];
    return buf;
}

constexpr int kBlurThreads = 256;   // every blur kernel runs 256-thread workgroups

// f(idx) for idx = threadIdx.x + 256 i < N.  ALL: unrolled, so that the LDS
// reads of all items are in flight together (costs registers: the fused
// kernels have them free here, the others would spill).
template <int N, bool ALL, class F>
__device__ __forceinline__ void for_block_items(F&& f) {
    if constexpr (ALL) {
        constexpr int IT = (N + kBlurThreads - 1) / kBlurThreads;
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int idx = (int)threadIdx.x + kBlurThreads * i;
            if (N % kBlurThreads == 0 || i + 1 < IT || idx < N) f(idx);
        }
    } else {
#pragma unroll 1
        for (int idx = threadIdx.x; idx < N; idx += kBlurThreads) f(idx);
    }
}

// Copy a clamped (replicate-border) window of image rows y_lo.. and columns
// x_lo.. into LDS, nr x nc floats at pitch ld; loads are issued in batches of
// kBatch per thread before any store.
template <int kBatch>
__device__ __forceinline__ void stage_window(float* __restrict__ dst, int ld, const float* __restrict__ ic, int H,
                                             int W, int y_lo, int x_lo, int nr, int nc) {
    const int n = nr * nc;
    for (int base = 0; base < n; base += kBatch * (int)blockDim.x) {
        float v[kBatch];
        int at[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int idx = base + i * (int)blockDim.x + (int)threadIdx.x;
            const int r = idx / nc, q = idx - r * nc;
            const int yy = min(max(y_lo + r, 0), H - 1);
            const int xx = min(max(x_lo + q, 0), W - 1);
            at[i] = idx < n ? r * ld + q : -1;
            v[i] = ic[(size_t)yy * W + xx];
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i)
            if (at[i] >= 0) dst[at[i]] = v[i];
    }
}

// Rows of the staged fp32 window of a low-precision tile (P taps, 2 NBLK
// output rows); the stage has a pitch of 64 floats (kTX + 2 R <= 64), one
// row per wave-wide copy instruction.
// Staged rows start 68 floats apart: 17 x 16 bytes, an odd number of 16-byte
// units, so that 16-byte reads of the same columns of consecutive rows fall
// on different LDS banks (the chunk packing reads rows that way).
constexpr int kStagePitch = 68;
template <int P, int NBLK>
struct TileGeom {
    static constexpr int R = (P - 1) / 2;
    static constexpr int TY = NBLK * 2;
    static constexpr int PH = TY + 2 * R;                 // rows of the row-chunk layout
    static constexpr int QH = TY + 8 * ((P + 7) / 8 - 1); // rows of the column-chunk layout
    static constexpr int SH = QH + 7 > PH ? QH + 7 : PH;  // staged rows
    static_assert(kTX + 2 * R <= kStagePitch, "stage pitch");
};

template <int P, int NBLK>
__device__ __forceinline__ float* stage_lds() {
    return lds_buffer<float, TileGeom<P, NBLK>::SH * kStagePitch, 2>();
}

// Entries of the FP8 row- and column-chunk layouts, eight at a time: from a
// run of 16 consecutive staged values v (a row run or a column run) entry k
// holds values k .. k+7, i.e. bytes k .. k+7 of the run's E4M3 codes; v[15]
// falls in no window.  Every value is converted once (the conversion is
// elementwise, so an entry equals converting its 8 values directly) and the
// windows are byte alignments of neighbouring code words.  The codes are
// those of the values clamped to +-448 (one med3), rounded to nearest even.
__device__ __forceinline__ void e4m3_windows8(const float (&v)[16], uint2 (&e)[8]) {
    uint32_t d[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float c[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = __builtin_amdgcn_fmed3f(v[4 * i + j], -448.0f, 448.0f);
        d[i] = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0, false);
        d[i] = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], (int)d[i], true);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int m = k >> 2, sh = k & 3;
        e[k] = sh ? make_uint2(__builtin_amdgcn_alignbyte(d[m + 1], d[m], sh), __builtin_amdgcn_alignbyte(d[m + 2], d[m + 1], sh))
                  : make_uint2(d[m], d[m + 1]);
    }
}

// Both FP8 chunk layouts of a staged window.  Row units: entries p0 .. p0+7 of
// one layout row r (row r of the stage, 4 reads of 16 bytes), taken
// row-fastest, so that with an odd entry pitch (and the odd 16-byte pitch
// of the stage) the lanes' reads and writes spread over the LDS banks.
// Column units: entries r0 .. r0+7 of one column (15 values down staged
// column q + 2R), column-fastest.  ALL: fully unrolled (the fused kernels
// have the registers free here).
template <int P, int NBLK, bool ALL, class E, class Conv>
__device__ __forceinline__ void pack_chunks(const float* __restrict__ stage, E* __restrict__ rowpk, int rpitch,
                                            E* __restrict__ colpk, int cpitch, Conv&& conv) {
    using G = TileGeom<P, NBLK>;
    constexpr int R = G::R, PH = G::PH, QH = G::QH, SH = G::SH;
    constexpr int RG = (kTX + 8 * (P / 8 - 1)) / 8;   // 8-entry groups per layout row
    constexpr int CG = (QH + 7) / 8;
    constexpr int UR = PH * RG, U = UR + CG * kTX;
    auto unit = [&](int u) {
        float v[16];
        E e[8];
        if (u < UR) {
            const int r = u % PH, p0 = (u / PH) * 8;
            const float4* src = reinterpret_cast<const float4*>(stage + r * kStagePitch + p0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float4 x = src[i];
                v[4 * i] = x.x;
                v[4 * i + 1] = x.y;
                v[4 * i + 2] = x.z;
                v[4 * i + 3] = x.w;
            }
            conv(v, e);
            E* dst = rowpk + r * rpitch + p0;
#pragma unroll
            for (int k = 0; k < 8; ++k) dst[k] = e[k];
        } else {
            const int uc = u - UR;
            const int q = uc % kTX, r0 = (uc / kTX) * 8;
            const float* src = stage + r0 * kStagePitch + q + 2 * R;
#pragma unroll
            for (int i = 0; i < 15; ++i) v[i] = (QH % 8 == 0 || r0 + i < SH) ? src[i * kStagePitch] : 0.0f;
            v[15] = 0.0f;
            conv(v, e);
            E* dst = colpk + r0 * cpitch + q;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (QH % 8 == 0 || r0 + k < QH) dst[k * cpitch] = e[k];
        }
    };
    for_block_items<U, ALL>(unit);
}

// The image window a tile item stages: rows y_lo.., columns x_lo.. of
// channel plane ic (clamped to the image).
struct Window {
    const float* ic;
    int H, W, y_lo, x_lo;
};

// Start the copy of a window into the stage without registers: one
// global_load_lds per row and wave (lane l copies column x_lo + l, clamped),
// completed by s_waitcnt vmcnt(0) and a barrier before the stage is read.
// Every wave issues the same compile-time number of copies (the last wave
// repeats the last row: the same bytes to the same place), so the compiler
// knows how many memory operations are younger than the loads issued before
// the copy and waits for those alone, not for the copy.  w.ic must be valid.
template <int SH>
__device__ __forceinline__ void window_dma(float* stage, const Window& w) {
    constexpr int kWaves = kBlurThreads / 64;
    constexpr int kRows = (SH + kWaves - 1) / kWaves;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int xx = min(max(w.x_lo + lane, 0), w.W - 1);
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
        const int r = min(wave + kWaves * i, SH - 1);
        const int yy = min(max(w.y_lo + r, 0), w.H - 1);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(w.ic + (size_t)yy * w.W + xx),
                                         (__attribute__((address_space(3))) void*)(stage + r * kStagePitch), 4, 0, 0);
    }
}

// s_waitcnt immediate for vmcnt(0) alone (expcnt and lgkmcnt at their
// maximum, no wait): vmcnt bits 3:0 and 15:14 zero, expcnt 6:4 = 7,
// lgkmcnt 11:8 = 15.
constexpr int kVmcnt0 = 0x0F70;

__device__ __forceinline__ void wait_window() {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}

// ------------------------------------------------------------------ FP32
// LDS tile of the image with a halo of R on every side (replicate border),
// pitch padded by one float.  Tap u = 4 t + L/16 in row-major (dy, dx) order.
template <int NMB, int NBLK>
__device__ __forceinline__ void blur_f32_tile(const float* __restrict__ img, int H, int W, int P, const float* __restrict__ bp,
                              int t4, int K, const float* __restrict__ w, float* __restrict__ out, int tiles_x,
                              int tile, int c) {
    constexpr int TY = NBLK * 2;                  // rows per workgroup: 4 waves x (NBLK/2) rows
    constexpr int LW = kTX + 2 * kMaxR;
    constexpr int PITCH = LW + 1;
    constexpr int LH = TY + 2 * kMaxR;
    __shared__ float tile_lds[LH * PITCH];
    const int R = (P - 1) / 2;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int x0 = tx * kTX, y0 = ty * TY;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, m = lane & 15;
    constexpr int RPW = NBLK / 2;                 // rows per wave
    const int lyw = wave * RPW;
    const size_t HW = (size_t)H * W;
    const int th = TY + 2 * R, twd = kTX + 2 * R;

    {
        const float* ic = img + c * HW;
        __syncthreads();                          // previous item of a persistent workgroup done with LDS
        stage_window<12>(tile_lds, PITCH, ic, H, W, y0 - R, x0 - R, th, twd);
        __syncthreads();
        floatx4 acc[NBLK][NMB];
#pragma unroll
        for (int b = 0; b < NBLK; ++b)
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) acc[b][mb] = floatx4{0.f, 0.f, 0.f, 0.f};
        // pixel (lyw + b/2, 16 (b%2) + m) sits at tile (.. + R, .. + R)
        const int base = (lyw + R) * PITCH + m + R;
        int dy = g / P - R, dx = g % P - R;
        // Same two-set operand pipeline as the BF16 kernel.
        float a0[NMB], p0[NBLK], a1[NMB], p1[NBLK];
        auto fetch = [&](int t, float* av, float* pv) {
            const int off = (dy <= R) ? dy * PITCH + dx : 0;
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) av[mb] = bp[((size_t)t * NMB + mb) * 64 + lane];
#pragma unroll
            for (int b = 0; b < NBLK; ++b) pv[b] = tile_lds[base + (b >> 1) * PITCH + (b & 1) * 16 + off];
            dx += 4;
            while (dx > R) {
                dx -= P;
                dy += 1;
            }
        };
        auto mma = [&](const float* av, const float* pv) {
#pragma unroll
            for (int b = 0; b < NBLK; ++b)
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb)
                    acc[b][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb], pv[b], acc[b][mb], 0, 0, 0);
        };
        fetch(0, a0, p0);
#pragma unroll 1
        for (int t = 0; t + 1 < t4; t += 2) {
            fetch(t + 1, a1, p1);
            mma(a0, p0);
            fetch(t + 2, a0, p0);
            mma(a1, p1);
        }
        if (t4 & 1) mma(a0, p0);
        epilogue<NMB, NBLK>(acc, w, K, y0 + lyw, x0, H, W, g, m, out + c * HW);
    }
}

// ------------------------------------------------------------------ BF16
// Two pre-packed LDS layouts, each entry 8 bf16 (16 bytes), so every B
// operand is a single aligned ds_read_b128:
//   RowPk[r][p] = I(y0 - R + r, x0 - R + p + e), e = 0..7   (row chunks)
//   ColPk[r][q] = I(y0 - R + r + e, x0 + q + R), e = 0..7   (the last tap column)
// A pixel (ly, lx) reads row chunk (dy, dx0) at RowPk[ly + R + dy][lx + R + dx0]
// and column chunk q at ColPk[ly + 8 q][lx].  RowPk rows hold kTX + 8 (A8 - 1)
// entries, ColPk rows kTX; a lane's per-pixel-block row step is the pitch of
// the kind its chunk of the current step comes from.
template <int P, int NMB, int NBLK, bool DMA = false, class Epi>
__device__ __forceinline__ void blur_bf16_tile(const float* __restrict__ img, int H, int W,
                                               const uint4* __restrict__ bp, int tiles_x, int tile, int c, Epi&& epi,
                                               const Window& next = Window{}) {
    constexpr int R = (P - 1) / 2;
    constexpr int A8 = P / 8;                    // row chunks per PSF row
    constexpr int NROW = P * A8;
    constexpr int NCOL = (P + 7) / 8;
    constexpr int T32 = (NROW + NCOL + 3) / 4;
    constexpr int TY = NBLK * 2;
    constexpr int PITCH = kTX + 8 * (A8 - 1);    // row-chunk positions per row
    constexpr int CPITCH = kTX;                  // column-chunk positions per row
    constexpr int PH = TY + 2 * R;               // rows of RowPk
    constexpr int QH = TY + 8 * (NCOL - 1);      // rows of ColPk
    constexpr int SW = kStagePitch;              // fp32 staging tile pitch
    constexpr int SH = TileGeom<P, NBLK>::SH;
    static_assert(P == 8 * A8 + 1, "bf16 layout needs P = 8a + 1");
    uint4* const rowpk = lds_buffer<uint4, PH * PITCH, 0>();
    uint4* const colpk = lds_buffer<uint4, QH * CPITCH, 1>();
    float* const stage = stage_lds<P, NBLK>();

    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int x0 = tx * kTX, y0 = ty * TY;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, m = lane & 15;
    constexpr int RPW = NBLK / 2;
    const int lyw = wave * RPW;
    const size_t HW = (size_t)H * W;

    {
        if constexpr (DMA) {
            // the window was started earlier (kernel prologue or previous
            // item); the barrier also retires the previous item's LDS reads
            wait_window();
            epi.prefetch(y0 + lyw, x0, m);
        } else {
            const float* ic = img + c * HW;
            epi.prefetch(y0 + lyw, x0, m);
            __syncthreads();                      // previous item of a persistent workgroup done with LDS
            stage_window<14>(stage, SW, ic, H, W, y0 - R, x0 - R, SH, kTX + 2 * R);
            __syncthreads();
        }
        for_block_items<PH * PITCH, DMA>([&](int idx) {
            const int r = idx / PITCH, p = idx - r * PITCH;
            const float* s = stage + r * SW + p;
            const floatx8 v = {s[0], s[1], s[2], s[3], s[4], s[5], s[6], s[7]};
            rowpk[idx] = __builtin_bit_cast(uint4, to_bf16x8(v));
        });
        for_block_items<QH * kTX, DMA>([&](int idx) {
            const int r = idx / kTX, q = idx - r * kTX;
            const float* s = stage + r * SW + q + 2 * R;
            const floatx8 v = {s[0], s[SW], s[2 * SW], s[3 * SW], s[4 * SW], s[5 * SW], s[6 * SW], s[7 * SW]};
            colpk[r * CPITCH + q] = __builtin_bit_cast(uint4, to_bf16x8(v));
        });
        __syncthreads();
        if constexpr (DMA) {
            epi.settle();
            window_dma<SH>(stage, next);          // stage free until the next item
        }
        floatx4 acc[NBLK][NMB];
        // B-operand source of chunk 4 t + g for this lane's pixel block 0, and
        // the row step of that kind of chunk
        auto chunk_src = [&](int t, int& step) -> const uint4* {
            const int ch = 4 * t + g;
            if (ch < NROW) {
                const int dy = ch / A8 - R, dx0 = (ch % A8) * 8 - R;
                step = PITCH;
                return rowpk + (lyw + dy + R) * PITCH + m + dx0 + R;
            }
            int q = ch - NROW;
            if (q >= NCOL) q = 0;                 // zero chunk: any valid entry
            step = CPITCH;
            return colpk + (lyw + 8 * q) * CPITCH + m;
        };
        // Two operand sets alternate: the loads of one step are in flight while
        // the MFMAs of the other run.  Loads one step past the end read a
        // zero basis step and a valid LDS entry.
        uint4 a0[NMB], p0[NBLK], a1[NMB], p1[NBLK];
        auto fetch = [&](int t, uint4* av, uint4* pv) {
            int step;
            const uint4* src = chunk_src(t, step);
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) av[mb] = bp[((size_t)t * NMB + mb) * 64 + lane];
#pragma unroll
            for (int b = 0; b < NBLK; ++b) pv[b] = src[(b >> 1) * step + (b & 1) * 16];
        };
        auto mma = [&](const uint4* av, const uint4* pv) {
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                const bf16x8 px = __builtin_bit_cast(bf16x8, pv[b]);
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb)
                    acc[b][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[mb]), px,
                                                                        acc[b][mb], 0, 0, 0);
            }
        };
        fetch(0, a0, p0);                         // in flight during the network
        epi.begin(y0 + lyw, x0, g, m);           // before the accumulators are live
        // The window copy and the first operands have long landed; saying so
        // (vmcnt(0) through the builtin, which the compiler's wait analysis
        // sees) keeps it from treating the copy as pending inside the loop,
        // where it would otherwise wait for every load at each step.
        if constexpr (DMA) __builtin_amdgcn_s_waitcnt(kVmcnt0);
#pragma unroll
        for (int b = 0; b < NBLK; ++b)
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb) acc[b][mb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
        for (int t = 0; t + 1 < T32; t += 2) {
            fetch(t + 1, a1, p1);
            mma(a0, p0);
            fetch(t + 2, a0, p0);
            mma(a1, p1);
        }
        if constexpr (T32 & 1) mma(a0, p0);
        epi(acc, y0 + lyw, x0, g, m, c);
    }
}

// ------------------------------------------------------------------- FP8
// E4M3 operands on v_mfma_scale_f32_16x16x128_f8f6f4.  The LDS holds the same
// RowPk / ColPk arrangement as BF16 with 8 E4M3 values (8 bytes) per entry.
// One step covers 16 chunks (128 taps): lane group g supplies chunks
// 16 t + 4 g + j, j = 0..3, as the 32 bytes of its B operand, and the packed
// basis supplies the same chunks of its row.  The MFMA multiplies row k by
// the E8M0 scale 2^-e_k of that basis function, so the accumulators hold the
// unscaled convolutions and the epilogue is the one of the other precisions.
// The image is rounded to E4M3 (ties to even) after clamping to +-448.
template <int P, int NMB, int NBLK, bool DMA = false, class Epi>
__device__ __forceinline__ void blur_fp8_tile(const float* __restrict__ img, int H, int W,
                                              const uint4* __restrict__ bp, const int* __restrict__ scale,
                                              int tiles_x, int tile, int c, Epi&& epi, const Window& next = Window{}) {
    constexpr int R = (P - 1) / 2;
    constexpr int A8 = P / 8;
    constexpr int NROW = P * A8;
    constexpr int NCOL = (P + 7) / 8;
    constexpr int T128 = (NROW + NCOL + 15) / 16;
    constexpr int TY = NBLK * 2;
    constexpr int PITCH = (kTX + 8 * (A8 - 1)) | 1;   // odd: see pack_chunks
    constexpr int PH = TY + 2 * R;
    constexpr int QH = TY + 8 * (NCOL - 1);
    constexpr int NR = PH > QH ? PH : QH;
    constexpr int SW = kStagePitch;
    constexpr int SH = TileGeom<P, NBLK>::SH;
    static_assert(P == 8 * A8 + 1, "fp8 layout needs P = 8a + 1");
    uint2* const rowpk8 = lds_buffer<uint2, NR * PITCH, 3>();
    uint2* const colpk8 = lds_buffer<uint2, NR * PITCH, 4>();
    float* const stage8 = stage_lds<P, NBLK>();

    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int x0 = tx * kTX, y0 = ty * TY;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, m = lane & 15;
    constexpr int RPW = NBLK / 2;
    const int lyw = wave * RPW;
    const size_t HW = (size_t)H * W;

    if constexpr (DMA) {
        wait_window();                            // started earlier; also retires the previous item's LDS reads
        epi.prefetch(y0 + lyw, x0, m);
    } else {
        const float* ic = img + c * HW;
        epi.prefetch(y0 + lyw, x0, m);
        __syncthreads();                          // previous item of a persistent workgroup done with LDS
        stage_window<14>(stage8, SW, ic, H, W, y0 - R, x0 - R, SH, kTX + 2 * R);
        __syncthreads();
    }
    pack_chunks<P, NBLK, DMA>(stage8, rowpk8, PITCH, colpk8, PITCH,
                              [](const float (&v)[16], uint2 (&e)[8]) { e4m3_windows8(v, e); });
    __syncthreads();
    if constexpr (DMA) {
        epi.settle();
        window_dma<SH>(stage8, next);             // stage free until the next item
    }
    int sc[NMB];
#pragma unroll
    for (int mb = 0; mb < NMB; ++mb) sc[mb] = scale[16 * mb + m];
    floatx4 acc[NBLK][NMB];
    const int pbase = lyw * PITCH + m;
    auto chunk_src = [&](int ch) -> const uint2* {
        if (ch < NROW) {
            const int dy = ch / A8 - R, dx0 = (ch % A8) * 8 - R;
            return rowpk8 + pbase + (dy + R) * PITCH + (dx0 + R);
        }
        int q = ch - NROW;
        if (q >= NCOL) q = 0;                     // zero chunk: any valid entry
        return colpk8 + pbase + 8 * q * PITCH;
    };
    // Register budget: the A operands (8 registers per basis block) of the
    // next step are loaded at the start of a step into the second of two
    // sets; the B operands are streamed per pixel block, the LDS reads of
    // block b + 1 issued before the MFMAs of block b (sched barriers keep the
    // compiler from hoisting all of a step's reads).  Loads past the last step
    // read a zero basis step and a valid LDS entry.
    const intx8* bp8 = reinterpret_cast<const intx8*>(bp);
    intx8 a0[NMB], a1[NMB];
    auto load_a = [&](int t, intx8* av) {
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) av[mb] = bp8[((size_t)t * NMB + mb) * 64 + lane];
    };
    auto load_b = [&](const uint2* const* src, int b, intx8& pv) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint2 v = src[j][(b >> 1) * PITCH + (b & 1) * 16];
            pv[2 * j] = (int)v.x;
            pv[2 * j + 1] = (int)v.y;
        }
    };
    auto step = [&](int t, const intx8* av, intx8* an) {
        load_a(t + 1, an);
        const uint2* src[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) src[j] = chunk_src(16 * t + 4 * g + j);
        intx8 pb[2];
        load_b(src, 0, pb[0]);
#pragma unroll
        for (int b = 0; b < NBLK; ++b) {
            if (b + 1 < NBLK) load_b(src, b + 1, pb[(b + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int mb = 0; mb < NMB; ++mb)
                acc[b][mb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av[mb], pb[b & 1], acc[b][mb], 0, 0, 0,
                                                                             sc[mb], 0, 127);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    load_a(0, a0);                                // in flight during the network
    epi.begin(y0 + lyw, x0, g, m);               // before the accumulators are live
    if constexpr (DMA) __builtin_amdgcn_s_waitcnt(kVmcnt0);   // as in the BF16 tile
#pragma unroll
    for (int b = 0; b < NBLK; ++b)
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb) acc[b][mb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int t = 0; t + 1 < T128; t += 2) {
        step(t, a0, a1);
        step(t + 1, a1, a0);
    }
    if constexpr (T128 & 1) step(T128 - 1, a0, a1);
    epi(acc, y0 + lyw, x0, g, m, c);
}

template <int NMB, int NBLK>
__global__ void __launch_bounds__(256) blur_f32_kernel(const float* __restrict__ img, int H, int W, int P,
                                                       const float* __restrict__ bp, int t4, int K,
                                                       const float* __restrict__ w, float* __restrict__ out,
                                                       int tiles_x) {
    blur_f32_tile<NMB, NBLK>(img, H, W, P, bp, t4, K, w, out, tiles_x, blockIdx.x, blockIdx.y);
}

template <int P, int NMB, int NBLK>
__global__ void __launch_bounds__(256) blur_bf16_kernel(const float* __restrict__ img, int H, int W,
                                                        const uint4* __restrict__ bp, int K,
                                                        const float* __restrict__ w, float* __restrict__ out,
                                                        int tiles_x) {
    blur_bf16_tile<P, NMB, NBLK>(img, H, W, bp, tiles_x, blockIdx.x, blockIdx.y, WFromMemory<NMB, NBLK>{w, K, H, W, out});
}

template <int P, int NMB, int NBLK>
__global__ void __launch_bounds__(256) blur_fp8_kernel(const float* __restrict__ img, int H, int W,
                                                       const uint4* __restrict__ bp, const int* __restrict__ scale,
                                                       int K, const float* __restrict__ w, float* __restrict__ out,
                                                       int tiles_x) {
    blur_fp8_tile<P, NMB, NBLK>(img, H, W, bp, scale, tiles_x, blockIdx.x, blockIdx.y,
                                WFromMemory<NMB, NBLK>{w, K, H, W, out});
}

// Batched, persistent forms over the (frame, channel, tile) list.
template <int NMB, int NBLK>
__global__ void __launch_bounds__(256) blur_f32_batch(const FrameDesc* __restrict__ fr, const int* __restrict__ first,
                                                      int n, int P, const float* __restrict__ bp, int t4, int K) {
    const int total = first[n];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int f = find_frame(first, n, item);
        const FrameDesc& d = fr[f];
        const int l = item - first[f];
        const int nt = d.tiles_x * d.tiles_y;
        const int c = l / nt;
        blur_f32_tile<NMB, NBLK>(d.image, d.H, d.W, P, bp, t4, K, d.w, d.blurred, d.tiles_x, l - c * nt, c);
    }
}

template <int P, int NMB, int NBLK>
__global__ void __launch_bounds__(256) blur_bf16_batch(const FrameDesc* __restrict__ fr, const int* __restrict__ first,
                                                       int n, const uint4* __restrict__ bp, int K) {
    const int total = first[n];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int f = find_frame(first, n, item);
        const FrameDesc& d = fr[f];
        const int l = item - first[f];
        const int nt = d.tiles_x * d.tiles_y;
        const int c = l / nt;
        blur_bf16_tile<P, NMB, NBLK>(d.image, d.H, d.W, bp, d.tiles_x, l - c * nt, c,
                                     WFromMemory<NMB, NBLK>{d.w, K, d.H, d.W, d.blurred});
    }
}

template <int P, int NMB, int NBLK>
__global__ void __launch_bounds__(256) blur_fp8_batch(const FrameDesc* __restrict__ fr, const int* __restrict__ first,
                                                      int n, const uint4* __restrict__ bp,
                                                      const int* __restrict__ scale, int K) {
    const int total = first[n];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int f = find_frame(first, n, item);
        const FrameDesc& d = fr[f];
        const int l = item - first[f];
        const int nt = d.tiles_x * d.tiles_y;
        const int c = l / nt;
        blur_fp8_tile<P, NMB, NBLK>(d.image, d.H, d.W, bp, scale, d.tiles_x, l - c * nt, c,
                                    WFromMemory<NMB, NBLK>{d.w, K, d.H, d.W, d.blurred});
    }
}

// Network fused into the blur (BF16 network; BF16 or FP8 blur): persistent
// workgroups stage the packed network weights into dynamic LDS once, then
// stride over the tiles of one frame, or over the (frame, tile) list of a
// batch.  An item blurs every channel of its tile with the weights the
// network produced once for the tile's pixels.  The image window of the next
// (channel or item) is copied into the stage while the current one computes.
template <int P, int NBLK>
__device__ __forceinline__ Window tile_window(const float* plane, int H, int W, int tiles_x, int tile) {
    constexpr int R = TileGeom<P, NBLK>::R, TY = TileGeom<P, NBLK>::TY;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    return Window{plane, H, W, ty * TY - R, tx * kTX - R};
}

template <int P, int NMB, int NBLK, bool FP8>
__device__ __forceinline__ void fused_item(const float* img, int C, int H, int W, const uint4* bp, const int* scale,
                                           const MlpArgs& a, const uint4* lds_w16, const float* bias,
                                           const float* fields2, float* out, int tiles_x, int tile,
                                           const Window& after) {
    const size_t HW = (size_t)H * W;
    auto next_of = [&](int c) {
        return c + 1 < C ? tile_window<P, NBLK>(img + (c + 1) * HW, H, W, tiles_x, tile) : after;
    };
    // channel 0 runs the network; the other channels reuse its weights (a
    // separate instance of the tile code, so that the network's registers
    // are not held across the channel loop)
    // the FP8 blur's network takes bf16 activations alone (as p2s_mlp does
    // for that precision), the BF16 blur's a bf16 hi + lo pair
    WFromNetwork<NMB, NBLK, true, !FP8> first{&a, lds_w16, bias, fields2, H, W, out, {}, {}};
    if constexpr (FP8)
        blur_fp8_tile<P, NMB, NBLK, true>(img, H, W, bp, scale, tiles_x, tile, 0, first, next_of(0));
    else
        blur_bf16_tile<P, NMB, NBLK, true>(img, H, W, bp, tiles_x, tile, 0, first, next_of(0));
    if (C == 1) return;
    WFromNetwork<NMB, NBLK, false, !FP8> rest{&a, lds_w16, bias, fields2, H, W, out, {}, {}};
#pragma unroll
    for (int b = 0; b < NBLK; ++b)
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) rest.wv[b][mb][i] = first.wv[b][mb][i];
    for (int c = 1; c < C; ++c) {
        if constexpr (FP8)
            blur_fp8_tile<P, NMB, NBLK, true>(img, H, W, bp, scale, tiles_x, tile, c, rest, next_of(c));
        else
            blur_bf16_tile<P, NMB, NBLK, true>(img, H, W, bp, tiles_x, tile, c, rest, next_of(c));
    }
}

template <int P, int NMB, int NBLK, bool FP8>
__global__ void __launch_bounds__(256) blur_mlp_kernel(const float* __restrict__ img, int C, int H, int W,
                                                       const uint4* __restrict__ bp, const int* __restrict__ scale,
                                                       MlpArgs a, const uint4* __restrict__ wg16,
                                                       const float* __restrict__ bias,
                                                       const float* __restrict__ fields2, float* __restrict__ out,
                                                       int tiles_x, int tiles_y) {
    extern __shared__ uint4 lds_w16[];
    constexpr int SH = TileGeom<P, NBLK>::SH;
    const int nt = tiles_x * tiles_y;
    if ((int)blockIdx.x < nt) window_dma<SH>(stage_lds<P, NBLK>(), tile_window<P, NBLK>(img, H, W, tiles_x, blockIdx.x));
    const float* lds_bias = stage_bf16_network(lds_w16, a, wg16, bias);   // the tile's first barrier publishes them
    for (int item = blockIdx.x; item < nt; item += gridDim.x) {
        // the window copied after this item's last channel: the next item's,
        // or (for the last item) this one's again, which nothing reads
        const int nx = item + (int)gridDim.x;
        const Window after = tile_window<P, NBLK>(img, H, W, tiles_x, nx < nt ? nx : item);
        fused_item<P, NMB, NBLK, FP8>(img, C, H, W, bp, scale, a, lds_w16, lds_bias, fields2, out, tiles_x, item,
                                      after);
    }
}

template <int P, int NMB, int NBLK, bool FP8>
__device__ __forceinline__ Window batch_window(const FrameDesc* fr, const int* first, int n, int item) {
    const int f = find_frame(first, n, item);
    const FrameDesc& d = fr[f];
    return tile_window<P, NBLK>(d.image, d.H, d.W, d.tiles_x, item - first[f]);
}

template <int P, int NMB, int NBLK, bool FP8>
__global__ void __launch_bounds__(256) blur_mlp_batch(const FrameDesc* __restrict__ fr, const int* __restrict__ first,
                                                      int n, const uint4* __restrict__ bp,
                                                      const int* __restrict__ scale, MlpArgs a,
                                                      const uint4* __restrict__ wg16, const float* __restrict__ bias) {
    extern __shared__ uint4 lds_w16[];
    constexpr int SH = TileGeom<P, NBLK>::SH;
    const int total = first[n];
    if ((int)blockIdx.x < total)
        window_dma<SH>(stage_lds<P, NBLK>(), batch_window<P, NMB, NBLK, FP8>(fr, first, n, blockIdx.x));
    const float* lds_bias = stage_bf16_network(lds_w16, a, wg16, bias);
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int f = find_frame(first, n, item);
        const FrameDesc& d = fr[f];
        const int nx = item + (int)gridDim.x;
        const Window after = batch_window<P, NMB, NBLK, FP8>(fr, first, n, nx < total ? nx : item);
        fused_item<P, NMB, NBLK, FP8>(d.image, d.C, d.H, d.W, bp, scale, a, lds_w16, lds_bias,
                                      d.fields + 2 * (size_t)d.H * d.W, d.blurred, d.tiles_x, item - first[f], after);
    }
}

template <int NMB>
hipError_t launch_f32(const Basis& b, const float* img, int C, int H, int W, const float* w, float* out,
                      hipStream_t s) {
    constexpr int NBLK = NMB <= 7 ? 8 : 4;
    constexpr int TY = NBLK * 2;
    const int tiles_x = (W + kTX - 1) / kTX, tiles_y = (H + TY - 1) / TY;
    hipLaunchKernelGGL((blur_f32_kernel<NMB, NBLK>), dim3(tiles_x * tiles_y, C), dim3(kBlurThreads), 0, s, img, H, W, b.P,
                       b.f32, b.t4, b.K, w, out, tiles_x);
    return hipGetLastError();
}

// BF16 and FP8 share the chunk layout, the tile shapes and the dispatch.
template <int P, int NMB>
hipError_t launch_lowp(const Basis& b, p2s_precision prec, const float* img, int C, int H, int W, const float* w,
                       float* out, hipStream_t s) {
    const int TY = blur_tile_rows(prec, NMB, 16);
    const int tiles_x = (W + kTX - 1) / kTX, tiles_y = (H + TY - 1) / TY;
    const dim3 grid(tiles_x * tiles_y, C);
    if (prec == P2S_BF16) {
        constexpr int NBLK = NMB <= 7 ? 8 : 4;
        hipLaunchKernelGGL((blur_bf16_kernel<P, NMB, NBLK>), grid, dim3(kBlurThreads), 0, s, img, H, W,
                           reinterpret_cast<const uint4*>(b.bf16), b.K, w, out, tiles_x);
    } else {
        hipLaunchKernelGGL((blur_fp8_kernel<P, NMB, 4>), grid, dim3(kBlurThreads), 0, s, img, H, W,
                           reinterpret_cast<const uint4*>(b.fp8), b.fp8_scale, b.K, w, out, tiles_x);
    }
    return hipGetLastError();
}

template <int P>
hipError_t dispatch_lowp(const Basis& b, p2s_precision prec, const float* img, int C, int H, int W, const float* w,
                         float* out, hipStream_t s) {
    switch (b.nmb) {
        case 1: return launch_lowp<P, 1>(b, prec, img, C, H, W, w, out, s);
        case 2: return launch_lowp<P, 2>(b, prec, img, C, H, W, w, out, s);
        case 3: return launch_lowp<P, 3>(b, prec, img, C, H, W, w, out, s);
        case 4: return launch_lowp<P, 4>(b, prec, img, C, H, W, w, out, s);
        case 5: return launch_lowp<P, 5>(b, prec, img, C, H, W, w, out, s);
        case 6: return launch_lowp<P, 6>(b, prec, img, C, H, W, w, out, s);
        case 7: return launch_lowp<P, 7>(b, prec, img, C, H, W, w, out, s);
        case 8: return launch_lowp<P, 8>(b, prec, img, C, H, W, w, out, s);
        default: return hipErrorInvalidValue;
    }
}

// Batched kernel instance for a basis, precision and tile height (nullptr if
// there is none).  16-row tiles (8 pixel blocks per wave) need NMB <= 7.
template <int NMB>
const void* f32_batch_fn(int rows) {
    if constexpr (NMB <= 7) {
        if (rows == 16) return (const void*)blur_f32_batch<NMB, 8>;
    }
    return (const void*)blur_f32_batch<NMB, 4>;
}

template <int P, int NMB>
const void* lowp_batch_fn(p2s_precision prec, int rows) {
    if (prec == P2S_FP8E4M3) return (const void*)blur_fp8_batch<P, NMB, 4>;
    if constexpr (NMB <= 7) {
        if (rows == 16) return (const void*)blur_bf16_batch<P, NMB, 8>;
    }
    return (const void*)blur_bf16_batch<P, NMB, 4>;
}

template <int P>
const void* lowp_batch_fn_p(p2s_precision prec, int nmb, int rows) {
    switch (nmb) {
        case 1: return lowp_batch_fn<P, 1>(prec, rows);
        case 2: return lowp_batch_fn<P, 2>(prec, rows);
        case 3: return lowp_batch_fn<P, 3>(prec, rows);
        case 4: return lowp_batch_fn<P, 4>(prec, rows);
        case 5: return lowp_batch_fn<P, 5>(prec, rows);
        case 6: return lowp_batch_fn<P, 6>(prec, rows);
        case 7: return lowp_batch_fn<P, 7>(prec, rows);
        case 8: return lowp_batch_fn<P, 8>(prec, rows);
        default: return nullptr;
    }
}

const void* blur_batch_fn(const Basis& b, p2s_precision prec, int rows) {
    if (prec == P2S_FP32) {
        switch (b.nmb) {
            case 1: return f32_batch_fn<1>(rows);
            case 2: return f32_batch_fn<2>(rows);
            case 3: return f32_batch_fn<3>(rows);
            case 4: return f32_batch_fn<4>(rows);
            case 5: return f32_batch_fn<5>(rows);
            case 6: return f32_batch_fn<6>(rows);
            case 7: return f32_batch_fn<7>(rows);
            case 8: return f32_batch_fn<8>(rows);
            default: return nullptr;
        }
    }
    if (!b.bf16_ok || (prec != P2S_BF16 && prec != P2S_FP8E4M3)) return nullptr;
    switch (b.P) {
        case 9: return lowp_batch_fn_p<9>(prec, b.nmb, rows);
        case 17: return lowp_batch_fn_p<17>(prec, b.nmb, rows);
        case 25: return lowp_batch_fn_p<25>(prec, b.nmb, rows);
        case 33: return lowp_batch_fn_p<33>(prec, b.nmb, rows);
        default: return nullptr;
    }
}

}  // namespace

// Output rows per blur work item: 16 (8 pixel blocks per wave) unless the
// accumulators and operands of a wave would not fit its registers: K > 112
// in FP32 and BF16, and always in FP8 (its operands are twice as wide).
int blur_tile_rows(p2s_precision prec, int nmb, int preferred) {
    if (prec == P2S_FP8E4M3) return 8;
    return (nmb <= 7 && preferred == 16) ? 16 : 8;
}

int blur_batch_resident(const Basis& b, p2s_precision prec, int rows) {
    const void* fn = blur_batch_fn(b, prec, blur_tile_rows(prec, b.nmb, rows));
    return fn ? resident_workgroups(fn, 256, 0) : 0;
}

hipError_t launch_blur_batch(const Basis& b, const BatchLaunch& bl, p2s_precision prec, hipStream_t s) {
    if (bl.items[ST_BLUR] == 0) return hipSuccess;
    const void* fn = blur_batch_fn(b, prec, bl.blur_rows);
    if (!fn) return hipErrorInvalidValue;
    const FrameDesc* fr = bl.frames;
    const int* first = bl.first + ST_BLUR * (bl.n + 1);
    int n = bl.n, P = b.P, t4 = b.t4, K = b.K;
    const float* bp32 = b.f32;
    const uint4* bp16 = reinterpret_cast<const uint4*>(b.bf16);
    const uint4* bp8 = reinterpret_cast<const uint4*>(b.fp8);
    const int* sc8 = b.fp8_scale;
    if (prec == P2S_FP32) {
        void* args[] = {&fr, &first, &n, &P, &bp32, &t4, &K};
        return hipLaunchKernel(fn, dim3(bl.grid[ST_BLUR]), dim3(kBlurThreads), args, 0, s);
    }
    if (prec == P2S_BF16) {
        void* args[] = {&fr, &first, &n, &bp16, &K};
        return hipLaunchKernel(fn, dim3(bl.grid[ST_BLUR]), dim3(kBlurThreads), args, 0, s);
    }
    void* args[] = {&fr, &first, &n, &bp8, &sc8, &K};
    return hipLaunchKernel(fn, dim3(bl.grid[ST_BLUR]), dim3(kBlurThreads), args, 0, s);
}

namespace {

// Pixel blocks per wave of the fused kernels: the blur accumulators
// (4 NBLK NMB registers), the network outputs they are dotted with (as many)
// and the operands in flight share the wave's 512 registers, so wide bases
// take 8-row or 4-row tiles.  Each basis operand a wave loads feeds NBLK
// MFMAs, and these loads are what the convolution loop waits on (every wave
// reads the basis from the L1 cache, whose bandwidth per CU is about what
// 4 waves need at NBLK = 4), so FP8 keeps NBLK = 4 up to K = 112 as well
// (at K = 112 a few network values spill to scratch, off the convolution
// loop).
constexpr int fused_nblk_bf16(int nmb) { return nmb >= 8 ? 2 : (nmb >= 4 ? 4 : 8); }
constexpr int fused_nblk_fp8(int nmb) { return nmb >= 8 ? 2 : 4; }
// FP8 instances whose registers fit (the others use the
// network kernel and the w-reading blur)
constexpr bool fused_fp8_fits(int P, int nmb) { return nmb <= 7 && !(P == 17 && nmb >= 4); }

template <int P, int NMB>
const void* fused_fn_nmb(p2s_precision prec, bool batch) {
    // (the discarded branches are not instantiated)
    if constexpr (16 * (NMB - 1) + 1 > P * P) {
        return nullptr;                          // more basis functions than taps: not a basis
    } else {
        if (prec == P2S_FP8E4M3) {
            if constexpr (!fused_fp8_fits(P, NMB)) {
                return nullptr;
            } else {
                constexpr int NBLK = fused_nblk_fp8(NMB);
                return batch ? (const void*)blur_mlp_batch<P, NMB, NBLK, true>
                             : (const void*)blur_mlp_kernel<P, NMB, NBLK, true>;
            }
        }
        constexpr int NBLK = fused_nblk_bf16(NMB);
        return batch ? (const void*)blur_mlp_batch<P, NMB, NBLK, false>
                     : (const void*)blur_mlp_kernel<P, NMB, NBLK, false>;
    }
}

template <int P>
const void* fused_fn_p(p2s_precision prec, int nmb, bool batch) {
    switch (nmb) {
        case 1: return fused_fn_nmb<P, 1>(prec, batch);
        case 2: return fused_fn_nmb<P, 2>(prec, batch);
        case 3: return fused_fn_nmb<P, 3>(prec, batch);
        case 4: return fused_fn_nmb<P, 4>(prec, batch);
        case 5: return fused_fn_nmb<P, 5>(prec, batch);
        case 6: return fused_fn_nmb<P, 6>(prec, batch);
        case 7: return fused_fn_nmb<P, 7>(prec, batch);
        case 8: return fused_fn_nmb<P, 8>(prec, batch);
        default: return nullptr;
    }
}

// The fused kernel for this basis, network and precision, or nullptr when the
// fused form does not apply: FP32, a PSF side without the low-precision
// layout, network output blocks other than the basis blocks, or packed BF16
// network weights that do not fit the LDS left beside the blur tile.
const void* fused_fn(const Basis& b, const Mlp& m, p2s_precision prec, bool batch) {
    if (prec == P2S_FP32 || !b.bf16_ok || m.mb != b.nmb || m.dims[m.L] != b.K) return nullptr;
    const void* fn = nullptr;
    switch (b.P) {
        case 9: fn = fused_fn_p<9>(prec, b.nmb, batch); break;
        case 17: fn = fused_fn_p<17>(prec, b.nmb, batch); break;
        case 25: fn = fused_fn_p<25>(prec, b.nmb, batch); break;
        case 33: fn = fused_fn_p<33>(prec, b.nmb, batch); break;
        default: return nullptr;
    }
    if (!fn) return nullptr;
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, fn) != hipSuccess) return nullptr;
    if (attr.sharedSizeBytes + network_lds_bytes(m) > kMlpLdsBytes) return nullptr;
    return fn;
}

}  // namespace

size_t network_lds_bytes(const Mlp& m) { return m.bytes16 + sizeof(float) * (size_t)m.L * 16 * m.mb; }

namespace {

hipError_t prepare_fused(const void* fn) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, fn);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kMlpLdsBytes - attr.sharedSizeBytes));
}

}  // namespace

int blur_mlp_tile_rows(p2s_precision prec, int nmb) {
    return 2 * (prec == P2S_FP8E4M3 ? fused_nblk_fp8(nmb) : fused_nblk_bf16(nmb));
}

bool blur_mlp_supported(const Basis& b, const Mlp& m, p2s_precision prec) {
    return fused_fn(b, m, prec, false) != nullptr && fused_fn(b, m, prec, true) != nullptr;
}

int blur_mlp_batch_resident(const Basis& b, const Mlp& m, p2s_precision prec) {
    const void* fn = fused_fn(b, m, prec, true);
    if (!fn || prepare_fused(fn) != hipSuccess) return 0;
    return resident_workgroups(fn, 256, network_lds_bytes(m));
}

hipError_t launch_blur_mlp(const Basis& b, const Mlp& m, p2s_precision prec, const float* img, int C, int H, int W,
                           const float* fields, float* out, hipStream_t s) {
    const void* fn = fused_fn(b, m, prec, false);
    if (!fn) return hipErrorInvalidValue;
    hipError_t e = prepare_fused(fn);
    if (e != hipSuccess) return e;
    MlpArgs a{};
    a.L = m.L;
    a.n_in = m.dims[0];
    a.K = m.dims[m.L];
    for (int l = 0; l < m.L; ++l) a.boff[l] = m.boff[l];
    fill_weight_args(m, P2S_BF16, a);
    const int TY = blur_mlp_tile_rows(prec, b.nmb);
    int tiles_x = (W + kTX - 1) / kTX, tiles_y = (H + TY - 1) / TY;
    const int items = tiles_x * tiles_y;            // each covers all channels of its tile
    const int grid = std::min(items, resident_workgroups(fn, 256, network_lds_bytes(m)));
    const uint4* bp = reinterpret_cast<const uint4*>(prec == P2S_BF16 ? (const void*)b.bf16 : (const void*)b.fp8);
    const int* scale = b.fp8_scale;
    const uint4* wg16 = reinterpret_cast<const uint4*>(m.w16);
    const float* bias = m.bias;
    const float* fields2 = fields + 2 * (size_t)H * W;
    void* args[] = {&img, &C, &H, &W, &bp, &scale, &a, &wg16, &bias, &fields2, &out, &tiles_x, &tiles_y};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlurThreads), args, network_lds_bytes(m), s);
}

hipError_t launch_blur_mlp_batch(const Basis& b, const Mlp& m, const BatchLaunch& bl, p2s_precision prec,
                                 hipStream_t s) {
    if (bl.items[ST_BLUR] == 0) return hipSuccess;
    const void* fn = fused_fn(b, m, prec, true);
    if (!fn) return hipErrorInvalidValue;
    hipError_t e = prepare_fused(fn);
    if (e != hipSuccess) return e;
    MlpArgs a{};
    a.L = m.L;
    a.n_in = m.dims[0];
    a.K = m.dims[m.L];
    for (int l = 0; l < m.L; ++l) a.boff[l] = m.boff[l];
    fill_weight_args(m, P2S_BF16, a);
    const FrameDesc* fr = bl.frames;
    const int* first = bl.first + ST_BLUR * (bl.n + 1);
    int n = bl.n;
    const uint4* bp = reinterpret_cast<const uint4*>(prec == P2S_BF16 ? (const void*)b.bf16 : (const void*)b.fp8);
    const int* scale = b.fp8_scale;
    const uint4* wg16 = reinterpret_cast<const uint4*>(m.w16);
    const float* bias = m.bias;
    void* args[] = {&fr, &first, &n, &bp, &scale, &a, &wg16, &bias};
    return hipLaunchKernel(fn, dim3(bl.grid[ST_BLUR]), dim3(kBlurThreads), args, network_lds_bytes(m), s);
}

hipError_t launch_blur(const Basis& b, const float* img, int C, int H, int W, const float* w, p2s_precision prec,
                       float* out, hipStream_t s) {
    if (prec == P2S_FP32) {
        switch (b.nmb) {
            case 1: return launch_f32<1>(b, img, C, H, W, w, out, s);
            case 2: return launch_f32<2>(b, img, C, H, W, w, out, s);
            case 3: return launch_f32<3>(b, img, C, H, W, w, out, s);
            case 4: return launch_f32<4>(b, img, C, H, W, w, out, s);
            case 5: return launch_f32<5>(b, img, C, H, W, w, out, s);
            case 6: return launch_f32<6>(b, img, C, H, W, w, out, s);
            case 7: return launch_f32<7>(b, img, C, H, W, w, out, s);
            case 8: return launch_f32<8>(b, img, C, H, W, w, out, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (b.P) {
        case 9: return dispatch_lowp<9>(b, prec, img, C, H, W, w, out, s);
        case 17: return dispatch_lowp<17>(b, prec, img, C, H, W, w, out, s);
        case 25: return dispatch_lowp<25>(b, prec, img, C, H, W, w, out, s);
        case 33: return dispatch_lowp<33>(b, prec, img, C, H, W, w, out, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace p2s
