// The P2S network (Sec. 3.3) on BF16 MFMA for a few blocks of 16 pixels,
// shared by the network kernel and the blur kernel with the network fused
// into its epilogue.  Layout conventions are those of mlp.hip: the product is
// computed transposed (rows = output features in blocks of 16, columns =
// pixels), so lane (g = L/16, m = L%16) ends holding features 16 mb + 4 g + i
// of its pixel, which is also the accumulator layout of the blur.
#pragma once

#include "internal.hpp"

namespace p2s {

template <typename T>
__device__ void stage_weights(T* lds, const T* __restrict__ g, int n) {
    constexpr int kB = 8;
    for (int base = 0; base < n; base += kB * (int)blockDim.x) {
        T v[kB];
#pragma unroll
        for (int i = 0; i < kB; ++i) {
            const int idx = base + i * (int)blockDim.x + (int)threadIdx.x;
            v[i] = g[idx < n ? idx : 0];
        }
#pragma unroll
        for (int i = 0; i < kB; ++i) {
            const int idx = base + i * (int)blockDim.x + (int)threadIdx.x;
            if (idx < n) lds[idx] = v[i];
        }
    }
}

struct MlpArgs {
    int L;
    int n_in;
    int nkc0;                       // layer-0 reduction chunks
    int woff[P2S_MAX_LAYERS];       // element offsets into the packed weights
    int boff[P2S_MAX_LAYERS];
    int HW;
    int K;
    int ngroups;
    int wtotal;                     // packed weight elements (floats, or uint4 for BF16)
    int nbias;                      // biases (floats): L layers of 16 MB
};

// BF16 kernels stage the packed weights and then the biases into LDS.
__device__ __forceinline__ const float* stage_bf16_network(uint4* lds, const MlpArgs& a, const uint4* __restrict__ wg,
                                                           const float* __restrict__ bias) {
    stage_weights(lds, wg, a.wtotal);
    float* lb = reinterpret_cast<float*>(lds + a.wtotal);
    stage_weights(lb, bias, a.nbias);
    return lb;
}



// Host: weight offsets, layer-0 chunks and packed size for a precision.
void fill_weight_args(const Mlp& mm, p2s_precision prec, MlpArgs& a);

// v = hi + lo with hi = bf16(v) and lo = bf16(v - hi), both rounded to
// nearest even.
__device__ __forceinline__ void split8(const float v[8], bf16x8& hi, bf16x8& lo) {
    const floatx8 f = {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
    hi = to_bf16x8(f);
    lo = to_bf16x8(f - from_bf16x8(hi));
}

// One layer on MFMA: acc[nb][mb] = b_mb + W_mb x_nb for the NB pixel blocks,
// reduction over NKC chunks of 32 features, each input a bf16 hi + lo pair.
// Every (output block, pixel block) is one accumulation chain that starts
// from the bias and adds the hi and then the lo product of each chunk.
// Output blocks go in pairs, so 2 NB chains are interleaved and a chain's
// next MFMA issues 2 NB MFMAs after its previous one; the weights of the next
// pair are read from LDS while the current pair's MFMAs run.
template <int MB, int NB, int NKC>
__device__ __forceinline__ void layer_mfma(const uint4* __restrict__ wl, const float* __restrict__ lbias,
                                           const bf16x8 (&xh)[NB][NKC], const bf16x8 (&xl)[NB][NKC],
                                           floatx4 (&acc)[NB][MB], int lane) {
    const int g = lane >> 4;
    constexpr int J = 2;
    constexpr int NP = (MB + J - 1) / J;
    bf16x8 w[2][J][NKC];
    auto load = [&](int p, bf16x8 (&dst)[J][NKC]) {
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc)
                if (p * J + j < MB)
                    dst[j][kc] = __builtin_bit_cast(bf16x8, wl[((p * J + j) * NKC + kc) * 64 + lane]);
    };
    load(0, w[0]);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (p + 1 < NP) load(p + 1, w[(p + 1) & 1]);
        floatx4 c[J][NB];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int mb = p * J + j < MB ? p * J + j : MB - 1;
            const floatx4 bv = *reinterpret_cast<const floatx4*>(lbias + 16 * mb + 4 * g);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) c[j][nb] = bv;
        }
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
#pragma unroll
            for (int j = 0; j < J; ++j)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    if (p * J + j < MB)
                        c[j][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[p & 1][j][kc], xh[nb][kc], c[j][nb], 0, 0, 0);
#pragma unroll
            for (int j = 0; j < J; ++j)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    if (p * J + j < MB)
                        c[j][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[p & 1][j][kc], xl[nb][kc], c[j][nb], 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (p * J + j < MB)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[nb][p * J + j] = c[j][nb];
    }
}

// The network inputs of NB pixel blocks for this lane: features 32 kc + 8 g + e
// of pixel pixc[nb] (zero past the input width) into in[nb][kc][e].  Separate
// from the evaluation so that a caller can issue the loads of the next blocks
// before evaluating the current ones.
template <int NB>
__device__ __forceinline__ void mlp_load_inputs(const MlpArgs& a, const float* __restrict__ fields, int HW,
                                                const int (&pixc)[NB], float (&in)[NB][2][8]) {
    const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int kc = 0; kc < 2; ++kc)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int f = 32 * kc + 8 * g + e;
            const int fc = min(f, a.n_in - 1);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) in[nb][kc][e] = fields[(size_t)fc * HW + pixc[nb]];
        }
}

template <int MB, int NB>
__device__ __forceinline__ void mlp_bf16_eval(const MlpArgs& a, const uint4* __restrict__ lds_w16,
                                              const float* __restrict__ bias, const float (&in)[NB][2][8],
                                              float (&out)[NB][MB][4]) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4;
    constexpr int MBE = (MB + 1) & ~1;      // even block count: chunks pair blocks
    constexpr int NKC = MBE / 2;
    float act[NB][MBE][4];
    floatx4 acc[NB][MB];
    // layer 0: chunk kc covers features 32 kc + 8 g + e
    {
        bf16x8 xh[NB][2], xl[NB][2];
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
            float v[NB][8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float fm = 32 * kc + 8 * g + e < a.n_in ? 1.0f : 0.0f;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) v[nb][e] = in[nb][kc][e] * fm;
            }
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) split8(v[nb], xh[nb][kc], xl[nb][kc]);
        }
        layer_mfma<MB, NB, 2>(lds_w16 + a.woff[0], bias + a.boff[0], xh, xl, acc, lane);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i) act[nb][MBE - 1][i] = 0.0f;   // padding block when MB is odd
    // act holds each layer's output with its bias; the ReLU of hidden layers
    // is applied where the next layer reads its inputs
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) act[nb][mb][i] = acc[nb][mb][i];
    for (int l = 1; l < a.L; ++l) {
        bf16x8 xh[NB][NKC], xl[NB][NKC];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc) {
                float v[8];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = fmaxf(act[nb][2 * kc][e], 0.0f);
                    v[4 + e] = fmaxf(act[nb][2 * kc + 1][e], 0.0f);
                }
                split8(v, xh[nb][kc], xl[nb][kc]);
            }
        layer_mfma<MB, NB, NKC>(lds_w16 + a.woff[l], bias + a.boff[l], xh, xl, acc, lane);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) act[nb][mb][i] = acc[nb][mb][i];
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[nb][mb][i] = act[nb][mb][i];
}

template <int MB, int NB>
__device__ __forceinline__ void mlp_bf16_blocks(const MlpArgs& a, const uint4* __restrict__ lds_w16,
                                                const float* __restrict__ bias, const float* __restrict__ fields,
                                                int HW, const int (&pixc)[NB], float (&out)[NB][MB][4]) {
    float in[NB][2][8];
    mlp_load_inputs<NB>(a, fields, HW, pixc, in);
    mlp_bf16_eval<MB, NB>(a, lds_w16, bias, in, out);
}

}  // namespace p2s
