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
// FP32 path: v_mfma_f32_16x16x4f32.  BF16 path: v_mfma_f32_16x16x32_bf16
// with every activation split as bf16 hi + bf16 lo (two MFMAs), bf16 weights
// and FP32 accumulation, so only the weights are rounded.
#include "internal.hpp"

namespace p2s {
namespace {

constexpr int kMaxMb = P2S_MAX_WIDTH / 16;   // 8
constexpr int kWaves = 8;
constexpr int kNb = 2;                       // pixel blocks of 16 per wave
constexpr int kPixPerGroup = kWaves * kNb * 16;
constexpr int kMaxIn = P2S_MAX_ZERNIKE;      // layer-0 width bound (64)

struct MlpArgs {
    int L;
    int dims[P2S_MAX_LAYERS + 1];
    int nkc[P2S_MAX_LAYERS];
    int woff[P2S_MAX_LAYERS];       // element offsets into the packed weights
    int boff[P2S_MAX_LAYERS];
    int HW;
    int K;
    int ngroups;
    int stage;                      // weights copied to LDS
    int wtotal;                     // packed weight elements (floats or uint4 / 8)
};

__device__ __forceinline__ int nmb_of(int n) { return (n + 15) >> 4; }

template <typename T>
__device__ void stage_weights(T* lds, const T* __restrict__ g, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = g[i];
}

// ------------------------------------------------------------------ FP32
template <bool STAGE>
__global__ void __launch_bounds__(kWaves * 64) mlp_f32_kernel(MlpArgs a, const float* __restrict__ fields,
                                                              const float* __restrict__ wg,
                                                              const float* __restrict__ bias,
                                                              float* __restrict__ wout) {
    extern __shared__ float lds_w[];
    if constexpr (STAGE) {
        stage_weights(lds_w, wg, a.wtotal);
        __syncthreads();
    }
    // weights from LDS when staged (ds_read), else from global memory
    auto wsrc = [&](int i) -> float {
        if constexpr (STAGE) return lds_w[i];
        else return wg[i];
    };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, m = lane & 15;
    const int n_in = a.dims[0];
    const int nkc0 = a.nkc[0];
    for (int grp = blockIdx.x; grp < a.ngroups; grp += gridDim.x) {
        const int pix0 = grp * kPixPerGroup + wave * kNb * 16;
        float act[kNb][kMaxMb][4];
        floatx4 acc[kNb][kMaxMb];
        // layer 0: B operand straight from the field planes (feature 4 kc + g)
        {
            const int nmo = nmb_of(a.dims[1]);
            float x0[kNb][kMaxIn / 4];
#pragma unroll
            for (int nb = 0; nb < kNb; ++nb) {
                const int pix = pix0 + nb * 16 + m;
#pragma unroll
                for (int kc = 0; kc < kMaxIn / 4; ++kc) {
                    const int f = 4 * kc + g;
                    x0[nb][kc] = (kc < nkc0 && f < n_in && pix < a.HW) ? fields[(size_t)f * a.HW + pix] : 0.0f;
                }
            }
#pragma unroll
            for (int mb = 0; mb < kMaxMb; ++mb) {
                if (mb < nmo) {
#pragma unroll
                    for (int nb = 0; nb < kNb; ++nb) acc[nb][mb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kc = 0; kc < kMaxIn / 4; ++kc) {
                        if (kc < nkc0) {
                            const float wa = wsrc(a.woff[0] + (mb * nkc0 + kc) * 64 + lane);
#pragma unroll
                            for (int nb = 0; nb < kNb; ++nb)
                                acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa, x0[nb][kc], acc[nb][mb], 0, 0, 0);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        // bias, ReLU, then the remaining layers
        for (int l = 0; l < a.L; ++l) {
            const int nmo = nmb_of(a.dims[l + 1]);
            const bool last = (l == a.L - 1);
            if (l > 0) {
                const int nkc = a.nkc[l];
#pragma unroll
                for (int mb = 0; mb < kMaxMb; ++mb) {
                    if (mb < nmo) {
#pragma unroll
                        for (int nb = 0; nb < kNb; ++nb) acc[nb][mb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int mbi = 0; mbi < kMaxMb; ++mbi) {
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const int kc = 4 * mbi + i;
                                if (kc < nkc) {
                                    const float wa = wsrc(a.woff[l] + (mb * nkc + kc) * 64 + lane);
#pragma unroll
                                    for (int nb = 0; nb < kNb; ++nb)
                                        acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa, act[nb][mbi][i], acc[nb][mb], 0, 0, 0);
                                }
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
#pragma unroll
            for (int mb = 0; mb < kMaxMb; ++mb) {
                if (mb < nmo) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float b = bias[a.boff[l] + 16 * mb + 4 * g + i];
#pragma unroll
                        for (int nb = 0; nb < kNb; ++nb) {
                            float v = acc[nb][mb][i] + b;
                            act[nb][mb][i] = last ? v : fmaxf(v, 0.0f);
                        }
                    }
                } else {
#pragma unroll
                    for (int nb = 0; nb < kNb; ++nb)
#pragma unroll
                        for (int i = 0; i < 4; ++i) act[nb][mb][i] = 0.0f;
                }
            }
        }
        // store w[pix][16 mb + 4 g + i]
        const int K = a.K;
        const int nmo = nmb_of(K);
#pragma unroll
        for (int nb = 0; nb < kNb; ++nb) {
            const int pix = pix0 + nb * 16 + m;
            if (pix < a.HW) {
                float* dst = wout + (size_t)pix * K;
#pragma unroll
                for (int mb = 0; mb < kMaxMb; ++mb) {
                    if (mb < nmo) {
                        const int k = 16 * mb + 4 * g;
                        if ((K & 3) == 0 && k + 3 < K) {
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
        }
    }
}

// ------------------------------------------------------------------ BF16
__device__ __forceinline__ void split8(const float v[8], bf16x8& hi, bf16x8& lo) {
    uint32_t h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = bf16_bits_rne(v[e]);
        l[e] = bf16_bits_rne(v[e] - bf16_bits_to_f32(h[e]));
    }
    uint4 ph = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
    uint4 pl = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16), l[6] | (l[7] << 16));
    hi = __builtin_bit_cast(bf16x8, ph);
    lo = __builtin_bit_cast(bf16x8, pl);
}

template <bool STAGE>
__global__ void __launch_bounds__(kWaves * 64) mlp_bf16_kernel(MlpArgs a, const float* __restrict__ fields,
                                                               const uint4* __restrict__ wg,
                                                               const float* __restrict__ bias,
                                                               float* __restrict__ wout) {
    extern __shared__ uint4 lds_w16[];
    if constexpr (STAGE) {
        stage_weights(lds_w16, wg, a.wtotal);
        __syncthreads();
    }
    auto wsrc = [&](int i) -> uint4 {
        if constexpr (STAGE) return lds_w16[i];
        else return wg[i];
    };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, m = lane & 15;
    const int n_in = a.dims[0];
    const int nkc0 = a.nkc[0];
    constexpr int kMaxKc0 = kMaxIn / 32;   // 2
    constexpr int kMaxKc = kMaxMb / 2;     // 4
    for (int grp = blockIdx.x; grp < a.ngroups; grp += gridDim.x) {
        const int pix0 = grp * kPixPerGroup + wave * kNb * 16;
        float act[kNb][kMaxMb][4];
        floatx4 acc[kNb][kMaxMb];
        {
            const int nmo = nmb_of(a.dims[1]);
            bf16x8 xh[kNb][kMaxKc0], xl[kNb][kMaxKc0];
#pragma unroll
            for (int nb = 0; nb < kNb; ++nb) {
                const int pix = pix0 + nb * 16 + m;
#pragma unroll
                for (int kc = 0; kc < kMaxKc0; ++kc) {
                    float v[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int f = 32 * kc + 8 * g + e;
                        v[e] = (kc < nkc0 && f < n_in && pix < a.HW) ? fields[(size_t)f * a.HW + pix] : 0.0f;
                    }
                    split8(v, xh[nb][kc], xl[nb][kc]);
                }
            }
#pragma unroll
            for (int mb = 0; mb < kMaxMb; ++mb) {
                if (mb < nmo) {
#pragma unroll
                    for (int nb = 0; nb < kNb; ++nb) acc[nb][mb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kc = 0; kc < kMaxKc0; ++kc) {
                        if (kc < nkc0) {
                            const bf16x8 wa = __builtin_bit_cast(bf16x8, wsrc(a.woff[0] + (mb * nkc0 + kc) * 64 + lane));
#pragma unroll
                            for (int nb = 0; nb < kNb; ++nb) {
                                acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, xh[nb][kc], acc[nb][mb], 0, 0, 0);
                                acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, xl[nb][kc], acc[nb][mb], 0, 0, 0);
                            }
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        for (int l = 0; l < a.L; ++l) {
            const int nmo = nmb_of(a.dims[l + 1]);
            const bool last = (l == a.L - 1);
            if (l > 0) {
                const int nkc = a.nkc[l];
                bf16x8 xh[kNb][kMaxKc], xl[kNb][kMaxKc];
#pragma unroll
                for (int nb = 0; nb < kNb; ++nb)
#pragma unroll
                    for (int kc = 0; kc < kMaxKc; ++kc) {
                        float v[8];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            v[e] = act[nb][2 * kc][e];
                            v[4 + e] = act[nb][2 * kc + 1][e];
                        }
                        split8(v, xh[nb][kc], xl[nb][kc]);
                    }
#pragma unroll
                for (int mb = 0; mb < kMaxMb; ++mb) {
                    if (mb < nmo) {
#pragma unroll
                        for (int nb = 0; nb < kNb; ++nb) acc[nb][mb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                        for (int kc = 0; kc < kMaxKc; ++kc) {
                            if (kc < nkc) {
                                const bf16x8 wa = __builtin_bit_cast(bf16x8, wsrc(a.woff[l] + (mb * nkc + kc) * 64 + lane));
#pragma unroll
                                for (int nb = 0; nb < kNb; ++nb) {
                                    acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, xh[nb][kc], acc[nb][mb], 0, 0, 0);
                                    acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa, xl[nb][kc], acc[nb][mb], 0, 0, 0);
                                }
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
#pragma unroll
            for (int mb = 0; mb < kMaxMb; ++mb) {
                if (mb < nmo) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float b = bias[a.boff[l] + 16 * mb + 4 * g + i];
#pragma unroll
                        for (int nb = 0; nb < kNb; ++nb) {
                            float v = acc[nb][mb][i] + b;
                            act[nb][mb][i] = last ? v : fmaxf(v, 0.0f);
                        }
                    }
                } else {
#pragma unroll
                    for (int nb = 0; nb < kNb; ++nb)
#pragma unroll
                        for (int i = 0; i < 4; ++i) act[nb][mb][i] = 0.0f;
                }
            }
        }
        const int K = a.K;
        const int nmo = nmb_of(K);
#pragma unroll
        for (int nb = 0; nb < kNb; ++nb) {
            const int pix = pix0 + nb * 16 + m;
            if (pix < a.HW) {
                float* dst = wout + (size_t)pix * K;
#pragma unroll
                for (int mb = 0; mb < kMaxMb; ++mb) {
                    if (mb < nmo) {
                        const int k = 16 * mb + 4 * g;
                        if ((K & 3) == 0 && k + 3 < K) {
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
        }
    }
}

int num_cus() {
    static int n = 0;
    if (n == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
    }
    return n;
}

}  // namespace

hipError_t launch_mlp(const Mlp& mm, const float* fields, int H, int W, p2s_precision prec, float* w,
                      hipStream_t s) {
    const size_t kMaxLds = 160 * 1024;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)mlp_f32_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)mlp_bf16_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    MlpArgs a{};
    a.L = mm.L;
    for (int i = 0; i <= mm.L; ++i) a.dims[i] = mm.dims[i];
    a.HW = H * W;
    a.K = mm.dims[mm.L];
    a.ngroups = (a.HW + kPixPerGroup - 1) / kPixPerGroup;
    const int grid = std::min(a.ngroups, num_cus() * 2);
    for (int l = 0; l < mm.L; ++l) a.boff[l] = mm.boff[l];
    if (prec == P2S_FP32) {
        for (int l = 0; l < mm.L; ++l) {
            a.nkc[l] = mm.nkc32[l];
            a.woff[l] = (int)(mm.off32[l] / sizeof(float));
        }
        a.wtotal = (int)(mm.bytes32 / sizeof(float));
        a.stage = mm.bytes32 <= 128 * 1024;
        if (a.stage)
            hipLaunchKernelGGL(mlp_f32_kernel<true>, dim3(grid), dim3(kWaves * 64), mm.bytes32, s, a, fields, mm.w32, mm.bias, w);
        else
            hipLaunchKernelGGL(mlp_f32_kernel<false>, dim3(grid), dim3(kWaves * 64), 0, s, a, fields, mm.w32, mm.bias, w);
    } else {
        for (int l = 0; l < mm.L; ++l) {
            a.nkc[l] = mm.nkc16[l];
            a.woff[l] = (int)(mm.off16[l] / 16);
        }
        a.wtotal = (int)(mm.bytes16 / 16);
        a.stage = mm.bytes16 <= 128 * 1024;
        const uint4* w16 = reinterpret_cast<const uint4*>(mm.w16);
        if (a.stage)
            hipLaunchKernelGGL(mlp_bf16_kernel<true>, dim3(grid), dim3(kWaves * 64), mm.bytes16, s, a, fields, w16, mm.bias, w);
        else
            hipLaunchKernelGGL(mlp_bf16_kernel<false>, dim3(grid), dim3(kWaves * 64), 0, s, a, fields, w16, mm.bias, w);
    }
    return hipGetLastError();
}

}  // namespace p2s
