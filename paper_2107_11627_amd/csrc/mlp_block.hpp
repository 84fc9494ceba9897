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

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two floats to a packed bf16 pair (first in the low half), round to nearest
// even: one v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(floatx2{a, b}, bf16x2));
}

// ReLU as an integer max on the bit pattern: every float with the sign bit
// set is a negative int32, every other one keeps its value, so this is
// max(x, +0) for every non-NaN x in one v_max_i32 (a float max in IEEE mode
// costs a second instruction that quiets its operand first).
__device__ __forceinline__ float relu(float x) {
    const int b = __builtin_bit_cast(int, x);
    return __builtin_bit_cast(float, b > 0 ? b : 0);
}

// Weights (chunks of 32 inputs) and biases of one output pair, blocks 2p and
// 2p + 1, of a layer with NKC input chunks.
template <int NKC>
struct PairW {
    bf16x8 w[2][NKC];
    floatx4 b[2];
};

template <int MB, int NKC>
__device__ __forceinline__ void load_pair(PairW<NKC>& d, const uint4* __restrict__ wl, const float* __restrict__ lb,
                                          int p, int lane) {
    const int g = lane >> 4;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (2 * p + j >= MB) continue;           // second block of an odd last pair
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc)
            d.w[j][kc] = __builtin_bit_cast(bf16x8, wl[((2 * p + j) * NKC + kc) * 64 + lane]);
        d.b[j] = *reinterpret_cast<const floatx4*>(lb + 16 * (2 * p + j) + 4 * g);
    }
}

// Turning 8 values per pixel block into one input chunk of the next layer:
// v -> (ReLU) -> hi = bf16(v), lo = bf16(v - hi), both round to nearest even,
// packed as 4 dwords of 2 values (dword d holds values 2d, 2d + 1; value e
// is v[e / 4][nb][e % 4]).  Each dword is two slices of 4 VALU instructions,
// so that slices can sit between MFMAs without holding them up:
//   A: ReLU both values (in place), pack hi, widen its low half into lo
//   B: widen its high half, both differences, pack lo.
// The values are overwritten and lo holds a temporary between the slices,
// so the split needs no registers beyond its source and destination.
// Dwords d with 2 d >= zero_from hold a padding block: constant zero.
//
// LO = false: the activations enter as bf16 alone (no lo part): only the
// first slice of each dword does work.
template <int NB, int NC, bool RELU, bool LO = true>
__device__ __forceinline__ void split_slice(int s, floatx4 (&v)[2][NB], int zero_from, u32x4 (&hi)[NB][NC],
                                            u32x4 (&lo)[NB][NC], int col) {
    const int nb = s >> 3, d = (s >> 1) & 3;
    const int j = d >> 1, i = 2 * (d & 1);
    if (2 * d >= zero_from) {
        if ((s & 1) == 0) {
            hi[nb][col][d] = 0u;
            if constexpr (LO) lo[nb][col][d] = 0u;
        }
        return;
    }
    if ((s & 1) == 0) {
        if constexpr (RELU) {
            v[j][nb][i] = relu(v[j][nb][i]);
            v[j][nb][i + 1] = relu(v[j][nb][i + 1]);
        }
        hi[nb][col][d] = pk_bf16(v[j][nb][i], v[j][nb][i + 1]);
        if constexpr (LO) lo[nb][col][d] = hi[nb][col][d] << 16;
    } else if constexpr (LO) {
        // (the elements are copied out first: __builtin_bit_cast applied to
        // a vector element lvalue reads element 0)
        const uint32_t t0 = lo[nb][col][d], t1 = hi[nb][col][d] & 0xFFFF0000u;
        const float h0 = __builtin_bit_cast(float, t0);
        const float h1 = __builtin_bit_cast(float, t1);
        lo[nb][col][d] = pk_bf16(v[j][nb][i] - h0, v[j][nb][i + 1] - h1);
    }
}

// The MFMAs of one output pair (JP = 1 or 2 blocks):
// c[j][nb] = b_j + sum_kc W_j,kc (xh + xl)[nb][kc], each chain starting from
// the bias.  Order: chunk, then hi/lo, then block, then pixel block, so two
// MFMAs of one chain are JP NB instructions apart.  After every second MFMA
// the caller's slot(k, kc) runs its VALU work for slot k; a scheduling
// barrier after each MFMA keeps the interleave as written (the hardware
// issues in order, so VALU placed after a run of MFMAs would leave the matrix
// pipe idle while it issues).
//
// LO = false: the bf16 activations alone, one MFMA per (chunk, block, pixel
// block), and the caller's slot after every MFMA (the same slot numbering).
template <int NB, int NKC, int JP, bool LO, class Slot>
__device__ __forceinline__ void pair_mfma(const PairW<NKC>& w, const u32x4 (&xh)[NB][NKC], const u32x4 (&xl)[NB][NKC],
                                          floatx4 (&c)[2][NB], Slot&& slot) {
    constexpr int NH = LO ? 2 : 1;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int j = 0; j < JP; ++j)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int t = ((kc * NH + h) * JP + j) * NB + nb;
                    const bf16x8 x = __builtin_bit_cast(bf16x8, h ? xl[nb][kc] : xh[nb][kc]);
                    c[j][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.w[j][kc], x, (kc == 0 && h == 0) ? w.b[j]
                                                                                                          : c[j][nb],
                                                                        0, 0, 0);
                    if (LO ? (t & 1) != 0 : true) slot(LO ? t >> 1 : t, kc);
                    __builtin_amdgcn_sched_barrier(0);
                }
}

// Spread NS slices over the slots k < nslots: slot k runs slices
// [k ceil(NS / nslots), (k + 1) ceil(NS / nslots)).
template <int NS>
__device__ __forceinline__ void slices_of_slot(int k, int nslots, int& s0, int& s1) {
    const int per = (NS + nslots - 1) / nslots;
    s0 = k * per;
    s1 = s0 + per < NS ? s0 + per : NS;
}

// One layer of MB output blocks over NKC input chunks.  Pair 0's weights
// arrive preloaded in w0; during the last pair the next layer's pair-0
// weights are loaded into wn0 (unless LAST).  With PEND, input chunk NKC-1
// is the previous layer's last pair (pin, its blocks from zero_in on are
// padding), split during this layer's pair-0 MFMAs of the earlier chunks.
// The ReLU + split of pair p - 1 runs between the MFMAs of pair p; the last
// pair's accumulators leave in pout for the next layer.  LAST: the pairs go
// to out, no activation.
template <int MB, int NB, int NKC, int NKCN, bool PEND, bool LAST, bool LO>
__device__ __forceinline__ void layer_bf16(const uint4* __restrict__ wl, const float* __restrict__ lb,
                                           const PairW<NKC>& w0, const uint4* __restrict__ wln,
                                           const float* __restrict__ lbn, PairW<NKCN>& wn0,
                                           u32x4 (&xh)[NB][NKC], u32x4 (&xl)[NB][NKC], floatx4 (&pin)[2][NB],
                                           u32x4 (&nh)[NB][NKCN], u32x4 (&nl)[NB][NKCN], floatx4 (&pout)[2][NB],
                                           floatx4 (&out)[NB][MB], int lane) {
    constexpr int NP = (MB + 1) / 2;
    constexpr int NS = 8 * NB;                   // slices of one split
    constexpr int ZERO_IN = MB & 1 ? 4 : 8;      // real values of the previous layer's last pair
    PairW<NKC> wb[2];
    wb[0] = w0;
    floatx4 c[2][2][NB];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (p + 1 < NP)
            load_pair<MB, NKC>(wb[(p + 1) & 1], wl, lb, p + 1, lane);
        else if constexpr (!LAST)
            load_pair<MB, NKCN>(wn0, wln, lbn, 0, lane);
        const bool two = 2 * p + 1 < MB;
        if constexpr (PEND && NKC == 1) {
            if (p == 0) {                        // no earlier chunk to hide the split behind
#pragma unroll
                for (int s = 0; s < NS; ++s) split_slice<NB, NKC, true, LO>(s, pin, ZERO_IN, xh, xl, 0);
            }
        }
        // VALU work between this pair's MFMAs: in pair 0 the split of the
        // previous layer's last pair (before the MFMAs of chunk NKC - 1 need
        // it), in pair p > 0 the split of pair p - 1
        auto slot = [&](int k, int kc) {
            if (p == 0) {
                if constexpr (PEND && NKC > 1) {
                    if (kc >= NKC - 1) return;
                    int s0, s1;
                    slices_of_slot<NS>(k, (two ? 2 : 1) * NB * (NKC - 1), s0, s1);
#pragma unroll
                    for (int s = s0; s < s1; ++s) split_slice<NB, NKC, true, LO>(s, pin, ZERO_IN, xh, xl, NKC - 1);
                }
            } else if constexpr (!LAST) {
                int s0, s1;
                slices_of_slot<NS>(k, (two ? 2 : 1) * NB * NKC, s0, s1);
#pragma unroll
                for (int s = s0; s < s1; ++s) split_slice<NB, NKCN, true, LO>(s, c[(p - 1) & 1], 8, nh, nl, p - 1);
            }
        };
        if (two)
            pair_mfma<NB, NKC, 2, LO>(wb[p & 1], xh, xl, c[p & 1], slot);
        else
            pair_mfma<NB, NKC, 1, LO>(wb[p & 1], xh, xl, c[p & 1], slot);
        if constexpr (LAST) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
                if (2 * p + j < MB)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) out[nb][2 * p + j] = c[p & 1][j][nb];
        }
    }
    if constexpr (!LAST)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) pout[j][nb] = c[(NP - 1) & 1][j][nb];
}

// The network inputs of NB pixel blocks for this lane: features 32 kc + 8 g + e
// of pixel pixc[nb], zero past the input width, into in[nb][kc][e].  Separate
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
            for (int nb = 0; nb < NB; ++nb) {
                const float v = fields[(size_t)fc * HW + pixc[nb]];
                in[nb][kc][e] = f < a.n_in ? v : 0.0f;
            }
        }
}

// Hidden layers l0 .. L-2 alternate between the two activation sets, so the
// loop runs two layers per iteration; the last layer reads whichever set the
// parity of L leaves.
//
// LO: activations as a bf16 hi + lo pair (about 16 significant bits, the
// BF16 precision); without it bf16 alone (the FP8 precision, whose blur
// error is far larger than what the lo part removes).
template <int MB, int NB, bool LO = true>
__device__ __forceinline__ void mlp_bf16_eval(const MlpArgs& a, const uint4* __restrict__ lds_w16,
                                              const float* __restrict__ bias, const float (&in)[NB][2][8],
                                              float (&out)[NB][MB][4]) {
    const int lane = threadIdx.x & 63;
    constexpr int NKC = (MB + 1) / 2;            // chunks of 32 features: pairs of 16-blocks
    constexpr int NS = 8 * NB;
    floatx4 o[NB][MB];
    u32x4 x0h[NB][2], x0l[NB][2];
    u32x4 ah[NB][NKC], al[NB][NKC], bh[NB][NKC], bl[NB][NKC];
    floatx4 pa[2][NB], pb[2][NB];
    PairW<2> w00;
    PairW<NKC> wa, wb;
    load_pair<MB, 2>(w00, lds_w16 + a.woff[0], bias + a.boff[0], 0, lane);
    // layer-0 inputs (no ReLU)
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
        floatx4 v[2][NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e >> 2][nb][e & 3] = in[nb][kc][e];
#pragma unroll
        for (int s = 0; s < NS; ++s) split_slice<NB, 2, false, LO>(s, v, 8, x0h, x0l, kc);
    }
    if (a.L == 1) {
        layer_bf16<MB, NB, 2, NKC, false, true, LO>(lds_w16 + a.woff[0], bias + a.boff[0], w00, nullptr, nullptr, wa, x0h,
                                                x0l, pa, ah, al, pb, o, lane);
    } else {
        layer_bf16<MB, NB, 2, NKC, false, false, LO>(lds_w16 + a.woff[0], bias + a.boff[0], w00, lds_w16 + a.woff[1],
                                                 bias + a.boff[1], wa, x0h, x0l, pb, ah, al, pa, o, lane);
        int l = 1;
        for (; l + 2 < a.L; l += 2) {
            layer_bf16<MB, NB, NKC, NKC, true, false, LO>(lds_w16 + a.woff[l], bias + a.boff[l], wa, lds_w16 + a.woff[l + 1],
                                                      bias + a.boff[l + 1], wb, ah, al, pa, bh, bl, pb, o, lane);
            layer_bf16<MB, NB, NKC, NKC, true, false, LO>(lds_w16 + a.woff[l + 1], bias + a.boff[l + 1], wb,
                                                      lds_w16 + a.woff[l + 2], bias + a.boff[l + 2], wa, bh, bl, pb, ah,
                                                      al, pa, o, lane);
        }
        if (l + 1 < a.L) {                       // one hidden layer left, then the last
            layer_bf16<MB, NB, NKC, NKC, true, false, LO>(lds_w16 + a.woff[l], bias + a.boff[l], wa, lds_w16 + a.woff[l + 1],
                                                      bias + a.boff[l + 1], wb, ah, al, pa, bh, bl, pb, o, lane);
            layer_bf16<MB, NB, NKC, NKC, true, true, LO>(lds_w16 + a.woff[l + 1], bias + a.boff[l + 1], wb, nullptr, nullptr,
                                                     wa, bh, bl, pb, ah, al, pa, o, lane);
        } else {
            layer_bf16<MB, NB, NKC, NKC, true, true, LO>(lds_w16 + a.woff[l], bias + a.boff[l], wa, nullptr, nullptr, wb, ah,
                                                     al, pa, bh, bl, pb, o, lane);
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) out[nb][mb][i] = o[nb][mb][i];
}

}  // namespace p2s
