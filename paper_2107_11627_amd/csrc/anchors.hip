// The paper's own field model (Sec. 3.4, "Interpolation across the grid"):
// Zernike coefficients drawn jointly on a G x G grid of anchor points from a
// precomputed correlation matrix, then bilinearly interpolated (in the phase
// domain) to every pixel.  With L_s the lower Cholesky factor of the anchor
// correlation matrix and L_Z that of Noll's mode covariance R_Z (Sec. 2.2),
//
//   A = L_s (E L_Z^T (D/r0)^(5/6)),   E [G^2][n] standard normals,
//
// so Cov(A_pj, A_qk) = R_s[p][q] R_Z[j][k] (D/r0)^(5/3).  Three kernels:
//   noise:  Philox4x32-10 counter (p, i >> 1, 0, 1) and Box-Muller per anchor
//           p and plane pair, times L_Z^T (D/r0)^(5/6) -> Bt [KP][ld]
//           (transposed, so a lane's four consecutive k are one 16-byte load);
//   gemm:   the triangular product L_s Bt^T on v_mfma_f32_16x16x4f32.  Row
//           tiles of 16 anchors are paired (t, T-1-t) so every pair carries
//           the same number of 32-wide k chunks; S workgroups of 8 waves
//           share a pair, chunks dealt round-robin to the 8 S waves, and each
//           workgroup writes its partial sum -> P [S][Gp][KP];
//   interp: one workgroup per (anchor cell row, 64-pixel column segment,
//           group of 16 planes): the two anchor rows of the cell and the
//           columns the segment needs are summed over the S partials into
//           LDS, then every pixel row of the cell is written, plane by plane,
//           with coalesced stores.
// The matrix product is the only dense contraction (G^4 / 2 n multiply-adds;
// 0.29 G MACs for G = 64, n = 35 padded to 48); the interpolation is bound by
// the HBM writes of the n planes.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace p2s {
namespace {

constexpr int kNoiseThreads = 256;
constexpr int kNoiseAnchors = 16;     // anchors per noise workgroup (Gp is a multiple)
constexpr int kGemmWaves = 8;
constexpr int kInterpThreads = 256;
constexpr int kPlaneGroup = 2;        // planes per interpolation workgroup
constexpr int kInterpSeg = 1024;      // pixels per interpolation column segment

// 16 anchors per workgroup of 256 threads: the normals of all of them go to
// LDS first (one Philox call per anchor and plane pair), then thread
// (anchor a, lane l) forms the outputs c = l, l + 16, ... as dot products of
// row c of L_Z (zero above the diagonal) with the anchor's normals.
template <int NCT>
__global__ __launch_bounds__(kNoiseThreads) void anchor_noise_kernel(const float* __restrict__ Lz, int n, int G2,
                                                                     int ld, uint32_t k0, uint32_t k1, float scale,
                                                                     float* __restrict__ Bt) {
    constexpr int KP = 16 * NCT;
    __shared__ float lz[KP * KP];     // L_Z padded with zeros to KP x KP
    __shared__ float e[kNoiseAnchors][KP + 1];
    for (int i = threadIdx.x; i < KP * KP; i += kNoiseThreads) {
        const int r = i / KP, c = i % KP;
        lz[i] = r < n && c < n ? Lz[r * n + c] : 0.0f;
    }
    const int p0 = blockIdx.x * kNoiseAnchors;
    for (int i = threadIdx.x; i < kNoiseAnchors * KP / 2; i += kNoiseThreads) {
        const int a = i % kNoiseAnchors, q = i / kNoiseAnchors, p = p0 + a;
        float2 z = make_float2(0.0f, 0.0f);
        if (p < G2 && 2 * q < n) {
            uint32_t c0 = (uint32_t)p, c1 = (uint32_t)q, c2 = 0u, c3 = 1u;
            philox4x32_10(c0, c1, c2, c3, k0, k1);
            z = box_muller(c0, c1);
        }
        e[a][2 * q] = z.x;
        e[a][2 * q + 1] = z.y;
    }
    __syncthreads();
    const int a = threadIdx.x / 16, l = threadIdx.x % 16;
    float x[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) x[k] = e[a][k];
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
        const int c = l + 16 * t;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < KP; ++k) acc = fmaf(lz[c * KP + k], x[k], acc);
        Bt[(size_t)c * ld + p0 + a] = acc * scale;
    }
}

// Pair `blockIdx.x / S` of row tiles, split `blockIdx.x % S`.  Lane (g, i) of
// a wave supplies A = L_s[16 t + i][32 c + 16 h + 4 g + s] and
// B = Bt[16 ct + i][32 c + 16 h + 4 g + s] for k-step (h, s): the same
// permutation of k on both operands, so the sum is unchanged.
template <int NCT>
__global__ __launch_bounds__(kGemmWaves * 64) void anchor_gemm_kernel(const float* __restrict__ Ls,
                                                                      const float* __restrict__ Bt, int Gp, int ld,
                                                                      int S, float* __restrict__ Pout) {
    constexpr int KP = 16 * NCT;
    __shared__ float red[kGemmWaves][2][16][KP];
    const int T = Gp / 16;
    const int pair = blockIdx.x / S, split = blockIdx.x % S;
    const int t1 = pair, t2 = T - 1 - pair;            // T is even: t1 < t2
    const int n1 = (t1 >> 1) + 1, n2 = (t2 >> 1) + 1;  // 32-wide chunks up to the diagonal
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, i = lane & 15;
    const int nw = S * kGemmWaves;
    const float* r1 = Ls + (size_t)(16 * t1 + i) * ld + 4 * g;
    const float* r2 = Ls + (size_t)(16 * t2 + i) * ld + 4 * g;
    const float* bc = Bt + (size_t)i * ld + 4 * g;
    floatx4 acc1[NCT], acc2[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
        acc1[ct] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        acc2[ct] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    // Operands of one 32-wide chunk.  Three sets rotate so that two chunks'
    // loads are in flight while the MFMAs of the third run.
    struct Ops {
        floatx4 b[NCT][2], a1[2], a2[2];
    };
    auto load = [&](Ops& o, int c) {
        if (c >= n2) return;
        const int k = 32 * c;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
                o.b[ct][h] = *reinterpret_cast<const floatx4*>(bc + (size_t)16 * ct * ld + k + 16 * h);
            o.a2[h] = *reinterpret_cast<const floatx4*>(r2 + k + 16 * h);
            o.a1[h] = c < n1 ? *reinterpret_cast<const floatx4*>(r1 + k + 16 * h) : floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    };
    auto compute = [&](const Ops& o, int c) {
        if (c >= n2) return;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int ct = 0; ct < NCT; ++ct)
                    acc2[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a2[h][s], o.b[ct][h][s], acc2[ct], 0, 0, 0);
        if (c < n1) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int ct = 0; ct < NCT; ++ct)
                        acc1[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a1[h][s], o.b[ct][h][s], acc1[ct], 0, 0, 0);
        }
    };
    const int c0 = split * kGemmWaves + wave;
    Ops o0, o1, o2;
    load(o0, c0);
    load(o1, c0 + nw);
    load(o2, c0 + 2 * nw);
    for (int c = c0; c < n2; c += 3 * nw) {
        compute(o0, c);
        load(o0, c + 3 * nw);
        compute(o1, c + nw);
        load(o1, c + 4 * nw);
        compute(o2, c + 2 * nw);
        load(o2, c + 5 * nw);
    }
    // lane (g, i) holds rows 4 g + v, column 16 ct + i of each tile
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            red[wave][0][4 * g + v][16 * ct + i] = acc1[ct][v];
            red[wave][1][4 * g + v][16 * ct + i] = acc2[ct][v];
        }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 2 * 16 * KP; idx += kGemmWaves * 64) {
        const int tile = idx / (16 * KP), r = (idx / KP) % 16, col = idx % KP;
        float s = 0.0f;
#pragma unroll
        for (int w = 0; w < kGemmWaves; ++w) s += red[w][tile][r][col];
        const int row = 16 * (tile ? t2 : t1) + r;
        Pout[((size_t)split * Gp + row) * KP + col] = s;
    }
}

__device__ __forceinline__ int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Anchor cell of a pixel coordinate and the position inside it, exactly:
// cell = min(floor(y (G-1) / (N-1)), G-2), fraction = (y (G-1) - cell (N-1)) / (N-1).
__device__ __forceinline__ int cell_of(int y, int N, int G) {
    return N == 1 ? 0 : min(y * (G - 1) / (N - 1), G - 2);
}
__device__ __forceinline__ float frac_of(int y, int cell, int N, int G) {
    return N == 1 ? 0.0f : (float)(y * (G - 1) - cell * (N - 1)) / (float)(N - 1);
}

// Workgroup (cell row a, column segment of segw pixels, group of up to pg
// planes).  64 threads across, each V = 4 adjacent pixels (one 16-byte store
// per row and plane; W a multiple of 4 and 16-byte aligned planes) or V = 1;
// 4 rows at a time.  Wide segments give long contiguous runs of every output
// row.
template <int V>
__global__ __launch_bounds__(kInterpThreads) void anchor_interp_kernel(const float* __restrict__ P, int S, int Gp,
                                                                       int KP, int G, int n, int H, int W, int segw,
                                                                       int nseg, int pg, int npg,
                                                                       float* __restrict__ F) {
    constexpr int TX = 64, RG = kInterpThreads / TX;
    extern __shared__ float win[];    // [2][ncw][m], m planes of this group
    const int a = blockIdx.x / (nseg * npg), rest = blockIdx.x % (nseg * npg);
    const int seg = rest / npg, j0 = (rest % npg) * pg, m = min(pg, n - j0);
    int ylo, yhi;
    if (H == 1) {
        if (a != 0) return;
        ylo = yhi = 0;
    } else {
        ylo = ceil_div(a * (H - 1), G - 1);
        yhi = a == G - 2 ? H - 1 : ceil_div((a + 1) * (H - 1), G - 1) - 1;
        if (ylo > yhi) return;        // anchors denser than pixel rows: no row lies in this cell
    }
    const int x0 = seg * segw, x1 = min(W, x0 + segw) - 1;
    const int b0 = cell_of(x0, W, G), ncw = cell_of(x1, W, G) + 2 - b0;
    for (int idx = threadIdx.x; idx < 2 * ncw * m; idx += kInterpThreads) {
        const int r = idx / (ncw * m), rem = idx % (ncw * m);
        const size_t p = (size_t)(a + r) * G + b0 + rem / m;
        float s = 0.0f;
        for (int sp = 0; sp < S; ++sp) s += P[((size_t)sp * Gp + p) * KP + j0 + rem % m];
        win[idx] = s;
    }
    __syncthreads();
    const size_t plane = (size_t)H * W;
    for (int xs = x0 + (int)(threadIdx.x % TX) * V; xs <= x1; xs += TX * V) {
        const float* w0[V];
        const float* w1[V];
        float tx[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int x = xs + v, bx = cell_of(x, W, G);  // V = 4: x <= x1 since W is a multiple of 4
            tx[v] = frac_of(x, bx, W, G);
            w0[v] = win + (bx - b0) * m;                  // anchor row a, columns bx, bx + 1
            w1[v] = win + (ncw + bx - b0) * m;            // anchor row a + 1
        }
        float* base = F + (size_t)j0 * plane + xs;
        for (int y = ylo + (int)(threadIdx.x / TX); y <= yhi; y += RG) {
            const float ty = frac_of(y, a, H, G);
            float* o = base + (size_t)y * W;
            for (int j = 0; j < m; ++j) {
                float val[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const float top = (1.0f - tx[v]) * w0[v][j] + tx[v] * w0[v][m + j];
                    const float bot = (1.0f - tx[v]) * w1[v][j] + tx[v] * w1[v][m + j];
                    val[v] = (1.0f - ty) * top + ty * bot;
                }
                if constexpr (V == 4)
                    *reinterpret_cast<floatx4*>(o + j * plane) = floatx4{val[0], val[1], val[2], val[3]};
                else
                    o[j * plane] = val[0];
            }
        }
    }
}

// Workgroups per pair of row tiles: about one per CU in all.
int gemm_splits(int Gp) {
    const int pairs = Gp / 32;
    return std::max(1, std::min(8, (num_cus() + pairs - 1) / pairs));
}

template <int NCT>
hipError_t launch_nct(const Anchor& an, int H, int W, float scale, uint32_t k0, uint32_t k1, float* fields,
                      float* ws, hipStream_t s) {
    const int KP = 16 * NCT, Gp = an.Gp, S = gemm_splits(Gp);
    float* Bt = ws;
    float* P = ws + (size_t)KP * an.ld;
    anchor_noise_kernel<NCT><<<Gp / kNoiseAnchors, kNoiseThreads, 0, s>>>(
        an.Lz, an.n, an.G * an.G, an.ld, k0, k1, scale, Bt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    anchor_gemm_kernel<NCT><<<(Gp / 32) * S, kGemmWaves * 64, 0, s>>>(an.Ls, Bt, Gp, an.ld, S, P);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const bool v4 = W % 4 == 0 && reinterpret_cast<uintptr_t>(fields) % 16 == 0;
    const int segw = std::min(W, kInterpSeg), nseg = (W + segw - 1) / segw;
    const int pg = std::min(an.n, kPlaneGroup), npg = (an.n + pg - 1) / pg;
    const size_t lds = (size_t)2 * anchor_window_cols(an.G, W, segw) * pg * sizeof(float);
    const int grid = (an.G - 1) * nseg * npg;
    if (v4)
        anchor_interp_kernel<4><<<grid, kInterpThreads, lds, s>>>(P, S, Gp, KP, an.G, an.n, H, W, segw, nseg, pg, npg,
                                                                  fields);
    else
        anchor_interp_kernel<1><<<grid, kInterpThreads, lds, s>>>(P, S, Gp, KP, an.G, an.n, H, W, segw, nseg, pg, npg,
                                                                  fields);
    return hipGetLastError();
}

}  // namespace

int anchor_window_cols(int G, int W, int seg) {
    if (W == 1) return 2;
    // a segment of seg pixels spans at most ceil((seg-1) (G-1) / (W-1)) cells past its first
    return std::min(G, (int)(((long)(seg - 1) * (G - 1) + W - 2) / (W - 1)) + 2);
}

size_t anchor_ws_bytes(const Anchor& an) {
    const size_t KP = 16 * (size_t)an.nct;
    return (KP * an.ld + (size_t)gemm_splits(an.Gp) * an.Gp * KP) * sizeof(float);
}

hipError_t launch_anchor_fields(const Anchor& an, int H, int W, double D_over_r0, uint32_t k0, uint32_t k1,
                                float* fields, void* ws, hipStream_t s) {
    const float scale = (float)std::pow(D_over_r0, 5.0 / 6.0);
    float* w = static_cast<float*>(ws);
    switch (an.nct) {
        case 1: return launch_nct<1>(an, H, W, scale, k0, k1, fields, w, s);
        case 2: return launch_nct<2>(an, H, W, scale, k0, k1, fields, w, s);
        case 3: return launch_nct<3>(an, H, W, scale, k0, k1, fields, w, s);
        default: return launch_nct<4>(an, H, W, scale, k0, k1, fields, w, s);
    }
}

}  // namespace p2s
