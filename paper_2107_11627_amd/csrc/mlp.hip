// Stage 2 of the hot path: the P2S network (Sec. 3.3), fully connected layers
// applied independently at every pixel, y = W x + b, ReLU between layers.
//
// The product is computed transposed, H^T[feature][pixel] = W H_prev^T, so
// that MFMA rows are output features (blocks of 16) and columns are pixels
// (blocks of 16).  The accumulator of one layer then already sits in the
// lanes that feed the next layer's B operand: lane L holds features
// 16 mb + 4 (L/16) + i of pixel L%16, and the packed weights of the next
// layer use exactly that feature order along the reduction.  Activations
// never leave registers between layers.
//
// Every hidden and output layer is padded to the same MB blocks of 16 (zero
// weights and biases), so all loops over blocks are compile-time and the code
// has no per-element branches.  Weights sit in LDS (staged once per
// workgroup, which then loops over pixel groups).
//
// FP32 path: v_mfma_f32_16x16x4f32.  BF16 path: v_mfma_f32_16x16x32_bf16
// with every activation split as bf16 hi + bf16 lo (two MFMAs), bf16 weights
// and FP32 accumulation, so only the weights are rounded.
#include <algorithm>

#include "mlp_block.hpp"

namespace p2s {
namespace {

constexpr int kWaves = 8;
constexpr int kNb = 2;                       // pixel blocks of 16 per wave
constexpr int kPixPerGroup = kWaves * kNb * 16;

// bias, ReLU (hidden layers) and the move into the next layer's inputs
template <int MB>
__device__ __forceinline__ void finish_layer(const floatx4 (&acc)[kNb][MB], float (&act)[kNb][MB][4],
                                             const float* __restrict__ bias, int g, bool last) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float b = bias[16 * mb + 4 * g + i];
#pragma unroll
            for (int nb = 0; nb < kNb; ++nb) {
                const float v = acc[nb][mb][i] + b;
                act[nb][mb][i] = last ? v : fmaxf(v, 0.0f);
            }
        }
}

// store w[pix][16 mb + 4 g + i] for the valid pixels and basis indices
template <int MB>
__device__ __forceinline__ void store_w(const float (&act)[kNb][MB][4], float* __restrict__ wout, int pix0, int m,
                                        int g, int HW, int K) {
#pragma unroll
    for (int nb = 0; nb < kNb; ++nb) {
        const int pix = pix0 + nb * 16 + m;
        if (pix >= HW) continue;
        float* dst = wout + (size_t)pix * K;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int k = 16 * mb + 4 * g;
            if ((K & 3) == 0) {
                if (k < K)
                    *reinterpret_cast<float4*>(dst + k) =
                        make_float4(act[nb][mb][0], act[nb][mb][1], act[nb][mb][2], act[nb][mb][3]);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (k + i < K) dst[k + i] = act[nb][mb][i];
            }
        }
    }
}

// ------------------------------------------------------------------ FP32
// One group of kPixPerGroup pixels starting at pixel grp * kPixPerGroup of a
// frame with HW pixels; `fields` points at plane 2 (alpha_4) of the frame.
template <int MB>
__device__ __forceinline__ void mlp_f32_group(const MlpArgs& a, const float* __restrict__ lds_w, const float* __restrict__ bias,
                              const float* __restrict__ fields, float* __restrict__ wout, int HW, int grp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, m = lane & 15;
    const int pix0 = grp * kPixPerGroup + wave * kNb * 16;
    int pixc[kNb];
#pragma unroll
    for (int nb = 0; nb < kNb; ++nb) pixc[nb] = min(pix0 + nb * 16 + m, HW - 1);
    float act[kNb][MB][4];
    floatx4 acc[kNb][MB];
#pragma unroll
    for (int nb = 0; nb < kNb; ++nb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[nb][mb] = floatx4{0.f, 0.f, 0.f, 0.f};
    // layer 0: B operand straight from the field planes (feature 4 kc + g)
    const float* w0 = lds_w + a.woff[0];
    for (int kc = 0; kc < a.nkc0; ++kc) {
        const int f = min(4 * kc + g, a.n_in - 1);
        const float fmask = (4 * kc + g < a.n_in) ? 1.0f : 0.0f;
        float x[kNb];
#pragma unroll
        for (int nb = 0; nb < kNb; ++nb) x[nb] = fields[(size_t)f * HW + pixc[nb]] * fmask;
        float wa[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) wa[mb] = w0[(mb * a.nkc0 + kc) * 64 + lane];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < kNb; ++nb)
                acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[mb], x[nb], acc[nb][mb], 0, 0, 0);
    }
    finish_layer<MB>(acc, act, bias + a.boff[0], g, a.L == 1);
    for (int l = 1; l < a.L; ++l) {
        const float* wl = lds_w + a.woff[l];
        constexpr int NKC = 4 * MB;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            float wa[NKC];
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) wa[kc] = wl[(mb * NKC + kc) * 64 + lane];
            floatx4 c[kNb];
#pragma unroll
            for (int nb = 0; nb < kNb; ++nb) c[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
                for (int nb = 0; nb < kNb; ++nb)
                    c[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[kc], act[nb][kc >> 2][kc & 3], c[nb], 0, 0, 0);
#pragma unroll
            for (int nb = 0; nb < kNb; ++nb) acc[nb][mb] = c[nb];
            __builtin_amdgcn_sched_barrier(0);
        }
        finish_layer<MB>(acc, act, bias + a.boff[l], g, l == a.L - 1);
    }
    store_w<MB>(act, wout, pix0, m, g, HW, a.K);
}

template <int MB>
__global__ void __launch_bounds__(kWaves * 64) mlp_f32_kernel(MlpArgs a, const float* __restrict__ fields,
                                                              const float* __restrict__ wg,
                                                              const float* __restrict__ bias,
                                                              float* __restrict__ wout) {
    extern __shared__ float lds_w[];
    stage_weights(lds_w, wg, a.wtotal);
    __syncthreads();
    for (int grp = blockIdx.x; grp < a.ngroups; grp += gridDim.x)
        mlp_f32_group<MB>(a, lds_w, bias, fields, wout, a.HW, grp);
}

template <int MB>
__global__ void __launch_bounds__(kWaves * 64) mlp_f32_batch(MlpArgs a, const FrameDesc* __restrict__ fr,
                                                             const int* __restrict__ first, int n,
                                                             const float* __restrict__ wg,
                                                             const float* __restrict__ bias) {
    extern __shared__ float lds_w[];
    stage_weights(lds_w, wg, a.wtotal);
    __syncthreads();
    const int total = first[n];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int f = find_frame(first, n, item);
        const int HW = fr[f].H * fr[f].W;
        mlp_f32_group<MB>(a, lds_w, bias, fr[f].fields + 2 * (size_t)HW, fr[f].w, HW, item - first[f]);
    }
}

// ------------------------------------------------------------------ BF16
// One wave per SIMD, 4 pixel blocks per wave (the same 256-pixel groups as
// FP32): the evaluation interleaves its own VALU work with its MFMAs, so it
// needs no second wave to hide latency, and the next group's inputs are
// loaded before the current group is evaluated.
constexpr int kWaves16 = 4;
constexpr int kNb16 = kPixPerGroup / (kWaves16 * 16);

template <int MB>
__device__ __forceinline__ void store_w16(const float (&act)[kNb16][MB][4], float* __restrict__ wout, int pix0,
                                          int m, int g, int HW, int K) {
#pragma unroll
    for (int nb = 0; nb < kNb16; ++nb) {
        const int pix = pix0 + nb * 16 + m;
        if (pix >= HW) continue;
        float* dst = wout + (size_t)pix * K;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int k = 16 * mb + 4 * g;
            if ((K & 3) == 0) {
                if (k < K)
                    *reinterpret_cast<float4*>(dst + k) =
                        make_float4(act[nb][mb][0], act[nb][mb][1], act[nb][mb][2], act[nb][mb][3]);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (k + i < K) dst[k + i] = act[nb][mb][i];
            }
        }
    }
}

// The wave's blocks two at a time: two blocks need about half the registers
// of a SIMD (two activation sets), four would need all of them.
template <int MB, bool LO>
__device__ __forceinline__ void eval_halves(const MlpArgs& a, const uint4* __restrict__ lds_w16,
                                            const float* __restrict__ bias, const float (&in)[kNb16][2][8],
                                            float (&out)[kNb16][MB][4]) {
#pragma unroll
    for (int b0 = 0; b0 < kNb16; b0 += 2) {
        const float (&ig)[2][2][8] = *reinterpret_cast<const float (*)[2][2][8]>(&in[b0]);
        float (&og)[2][MB][4] = *reinterpret_cast<float (*)[2][MB][4]>(&out[b0]);
        mlp_bf16_eval<MB, 2, LO>(a, lds_w16, bias, ig, og);
    }
}

__device__ __forceinline__ void bf16_group_pixels(int grp, int HW, int (&pixc)[kNb16], int& pix0) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    pix0 = grp * kPixPerGroup + wave * kNb16 * 16;
#pragma unroll
    for (int nb = 0; nb < kNb16; ++nb) pixc[nb] = min(pix0 + nb * 16 + (lane & 15), HW - 1);
}

// LO: activations as bf16 hi + lo (P2S_BF16); without: bf16 alone (the
// network of P2S_FP8E4M3).
template <int MB, bool LO>
__global__ void __launch_bounds__(kWaves16 * 64) mlp_bf16_kernel(MlpArgs a, const float* __restrict__ fields,
                                                                 const uint4* __restrict__ wg,
                                                                 const float* __restrict__ bias,
                                                                 float* __restrict__ wout) {
    extern __shared__ uint4 lds_w16[];
    const float* lds_bias = stage_bf16_network(lds_w16, a, wg, bias);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    int pixc[kNb16], pix0;
    float in[kNb16][2][8];
    int grp = blockIdx.x;
    if (grp < a.ngroups) {
        bf16_group_pixels(grp, a.HW, pixc, pix0);
        mlp_load_inputs<kNb16>(a, fields, a.HW, pixc, in);
    }
    for (; grp < a.ngroups; grp += gridDim.x) {
        float cur[kNb16][2][8];
#pragma unroll
        for (int nb = 0; nb < kNb16; ++nb)
#pragma unroll
            for (int kc = 0; kc < 2; ++kc)
#pragma unroll
                for (int e = 0; e < 8; ++e) cur[nb][kc][e] = in[nb][kc][e];
        const int cur0 = pix0;
        if (grp + (int)gridDim.x < a.ngroups) {
            bf16_group_pixels(grp + gridDim.x, a.HW, pixc, pix0);
            mlp_load_inputs<kNb16>(a, fields, a.HW, pixc, in);
        }
        float outv[kNb16][MB][4];
        eval_halves<MB, LO>(a, lds_w16, lds_bias, cur, outv);
        store_w16<MB>(outv, wout, cur0, lane & 15, lane >> 4, a.HW, a.K);
    }
}

template <int MB, bool LO>
__global__ void __launch_bounds__(kWaves16 * 64) mlp_bf16_batch(MlpArgs a, const FrameDesc* __restrict__ fr,
                                                                const int* __restrict__ first, int n,
                                                                const uint4* __restrict__ wg,
                                                                const float* __restrict__ bias) {
    extern __shared__ uint4 lds_w16[];
    const float* lds_bias = stage_bf16_network(lds_w16, a, wg, bias);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int total = first[n];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int f = find_frame(first, n, item);
        const int HW = fr[f].H * fr[f].W;
        int pixc[kNb16], pix0;
        bf16_group_pixels(item - first[f], HW, pixc, pix0);
        float in[kNb16][2][8], outv[kNb16][MB][4];
        mlp_load_inputs<kNb16>(a, fr[f].fields + 2 * (size_t)HW, HW, pixc, in);
        eval_halves<MB, LO>(a, lds_w16, lds_bias, in, outv);
        store_w16<MB>(outv, fr[f].w, pix0, lane & 15, lane >> 4, HW, a.K);
    }
}


template <int MB>
hipError_t set_attrs() {
    static bool attr = false;
    if (!attr) {
        const void* ks[] = {(const void*)mlp_f32_kernel<MB>,        (const void*)mlp_bf16_kernel<MB, true>,
                            (const void*)mlp_bf16_kernel<MB, false>, (const void*)mlp_f32_batch<MB>,
                            (const void*)mlp_bf16_batch<MB, true>,   (const void*)mlp_bf16_batch<MB, false>};
        for (const void* k : ks) {
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
        }
        attr = true;
    }
    return hipSuccess;
}

}  // namespace

void fill_weight_args(const Mlp& mm, p2s_precision prec, MlpArgs& a) {
    if (prec == P2S_FP32) {
        for (int l = 0; l < mm.L; ++l) a.woff[l] = (int)(mm.off32[l] / sizeof(float));
        a.nkc0 = mm.nkc32[0];
        a.wtotal = (int)(mm.bytes32 / sizeof(float));
    } else {
        for (int l = 0; l < mm.L; ++l) a.woff[l] = (int)(mm.off16[l] / 16);
        a.nkc0 = mm.nkc16[0];
        a.wtotal = (int)(mm.bytes16 / 16);
    }
    a.nbias = mm.L * 16 * mm.mb;
}

namespace {

template <int MB>
hipError_t launch_mb_batch(const Mlp& mm, const MlpArgs& a0, const BatchLaunch& bl, p2s_precision prec,
                           hipStream_t s) {
    hipError_t e = set_attrs<MB>();
    if (e != hipSuccess) return e;
    MlpArgs a = a0;
    fill_weight_args(mm, prec, a);
    const int* first = bl.first + ST_MLP * (bl.n + 1);
    if (prec == P2S_FP32)
        hipLaunchKernelGGL(mlp_f32_batch<MB>, dim3(bl.grid[ST_MLP]), dim3(kWaves * 64), mm.bytes32, s, a, bl.frames,
                           first, bl.n, mm.w32, mm.bias);
    else if (prec == P2S_BF16)
        hipLaunchKernelGGL((mlp_bf16_batch<MB, true>), dim3(bl.grid[ST_MLP]), dim3(kWaves16 * 64),
                           mm.bytes16 + 4 * (size_t)a.nbias, s, a, bl.frames,
                           first, bl.n, reinterpret_cast<const uint4*>(mm.w16), mm.bias);
    else
        hipLaunchKernelGGL((mlp_bf16_batch<MB, false>), dim3(bl.grid[ST_MLP]), dim3(kWaves16 * 64),
                           mm.bytes16 + 4 * (size_t)a.nbias, s, a, bl.frames,
                           first, bl.n, reinterpret_cast<const uint4*>(mm.w16), mm.bias);
    return hipGetLastError();
}

template <int MB>
hipError_t launch_mb(const Mlp& mm, const MlpArgs& a0, const float* fields, p2s_precision prec, float* w,
                     hipStream_t s) {
    hipError_t e0 = set_attrs<MB>();
    if (e0 != hipSuccess) return e0;
    MlpArgs a = a0;
    const int grid = std::min(a.ngroups, mlp_batch_resident(mm, prec));
    if (prec == P2S_FP32) {
        for (int l = 0; l < mm.L; ++l) a.woff[l] = (int)(mm.off32[l] / sizeof(float));
        a.nkc0 = mm.nkc32[0];
        a.wtotal = (int)(mm.bytes32 / sizeof(float));
        hipLaunchKernelGGL(mlp_f32_kernel<MB>, dim3(grid), dim3(kWaves * 64), mm.bytes32, s, a, fields, mm.w32,
                           mm.bias, w);
    } else {
        fill_weight_args(mm, prec, a);
        if (prec == P2S_BF16)
            hipLaunchKernelGGL((mlp_bf16_kernel<MB, true>), dim3(grid), dim3(kWaves16 * 64),
                               mm.bytes16 + 4 * (size_t)a.nbias, s, a, fields, reinterpret_cast<const uint4*>(mm.w16),
                               mm.bias, w);
        else
            hipLaunchKernelGGL((mlp_bf16_kernel<MB, false>), dim3(grid), dim3(kWaves16 * 64),
                               mm.bytes16 + 4 * (size_t)a.nbias, s, a, fields, reinterpret_cast<const uint4*>(mm.w16),
                               mm.bias, w);
    }
    return hipGetLastError();
}

}  // namespace

int num_cus() {
    static int n = 0;
    if (n == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
    }
    return n;
}

int mlp_pixels_per_group() { return kPixPerGroup; }

int mlp_batch_resident(const Mlp& mm, p2s_precision prec) {
    (void)mm;
    // weights staged once per workgroup; FP32: LDS allows two per CU, BF16:
    // one (its waves need the whole register file of their SIMD)
    return prec == P2S_FP32 ? 2 * num_cus() : num_cus();
}

hipError_t launch_mlp_batch(const Mlp& mm, const BatchLaunch& bl, p2s_precision prec, hipStream_t s) {
    if (bl.items[ST_MLP] == 0) return hipSuccess;
    MlpArgs a{};
    a.L = mm.L;
    a.n_in = mm.dims[0];
    a.K = mm.dims[mm.L];
    for (int l = 0; l < mm.L; ++l) a.boff[l] = mm.boff[l];
    switch (mm.mb) {
        case 1: return launch_mb_batch<1>(mm, a, bl, prec, s);
        case 2: return launch_mb_batch<2>(mm, a, bl, prec, s);
        case 3: return launch_mb_batch<3>(mm, a, bl, prec, s);
        case 4: return launch_mb_batch<4>(mm, a, bl, prec, s);
        case 5: return launch_mb_batch<5>(mm, a, bl, prec, s);
        case 6: return launch_mb_batch<6>(mm, a, bl, prec, s);
        case 7: return launch_mb_batch<7>(mm, a, bl, prec, s);
        case 8: return launch_mb_batch<8>(mm, a, bl, prec, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_mlp(const Mlp& mm, const float* fields, int H, int W, p2s_precision prec, float* w,
                      hipStream_t s) {
    MlpArgs a{};
    a.L = mm.L;
    a.n_in = mm.dims[0];
    a.HW = H * W;
    a.K = mm.dims[mm.L];
    a.ngroups = (a.HW + kPixPerGroup - 1) / kPixPerGroup;
    for (int l = 0; l < mm.L; ++l) a.boff[l] = mm.boff[l];
    switch (mm.mb) {
        case 1: return launch_mb<1>(mm, a, fields, prec, w, s);
        case 2: return launch_mb<2>(mm, a, fields, prec, w, s);
        case 3: return launch_mb<3>(mm, a, fields, prec, w, s);
        case 4: return launch_mb<4>(mm, a, fields, prec, w, s);
        case 5: return launch_mb<5>(mm, a, fields, prec, w, s);
        case 6: return launch_mb<6>(mm, a, fields, prec, w, s);
        case 7: return launch_mb<7>(mm, a, fields, prec, w, s);
        case 8: return launch_mb<8>(mm, a, fields, prec, w, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace p2s
