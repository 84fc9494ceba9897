// Stage 1 of the hot path: spatially correlated Zernike coefficient planes
// (the per-pixel alpha_j of Sec. 2.2 Eq. 1, correlated in space as Sec. 3.4
// requires), made by filtering seeded white noise with a Gaussian power
// spectral density and inverse FFTs.
//
// The white noise is drawn directly in the frequency domain as i.i.d.
// complex normals N_q(k) per plane pair q, so that
//
//   G_q(y, x) = (1/sqrt(Nfy Nfx)) sum_k sqrt(S_y(ky) S_x(kx)) N_q(k) e^{+2 pi i k.(y,x)/Nf}
//
// and plane 2q = sigma Re G_q, plane 2q+1 = sigma Im G_q (two independent
// fields per transform).  The Gaussian PSD is negligible away from DC: only
// the band where the 1-D filter is >= 1e-9 of its peak is kept (the dropped
// part changes a unit-variance field by < 1.5e-9 rms).  Two kernels:
//   columns: for each band column kx: noise * filter on the band rows, zero
//            elsewhere -> inverse FFT along y -> V[q][y][j] for y < H
//   rows:    for each output row y: V scattered into the band bins -> inverse
//            FFT along x -> planes 2q, 2q+1 for x < W
// FFTs: Stockham auto-sort in LDS, radix 9/8/4/2/3/5 passes, FP64-evaluated
// twiddle table, thread -> (transform, butterfly) mapping by shifts; the
// 576-point grid of 512-pixel sides runs on a fixed 9 x 8 x 8 plan with one
// butterfly per thread and pass (same arithmetic, same bits).
#include <algorithm>

#include "internal.hpp"

namespace p2s {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 mul_i(float2 a, float sgn) {   // sgn * i * a
    return make_float2(-sgn * a.y, sgn * a.x);
}

// Complex standard normal of bin (ky, kx) of plane pair q: counter
// (kx, ky, q, 0), Box-Muller on outputs 0 and 1.
__device__ __forceinline__ float2 bin_noise(int kx, int ky, int q, uint32_t k0, uint32_t k1,
                                            uint32_t* raw_out = nullptr) {
    uint32_t c0 = (uint32_t)kx, c1 = (uint32_t)ky, c2 = (uint32_t)q, c3 = 0u;
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    if (raw_out) {
        raw_out[0] = c0;
        raw_out[1] = c1;
        raw_out[2] = c2;
        raw_out[3] = c3;
    }
    return box_muller(c0, c1);
}

// Band index of an FFT bin (bins 0..kc and N-(M-1-kc)..N-1 hold band
// entries 0..M-1), or -1 outside the band.
__device__ __forceinline__ int bin_to_band(int b, int kc, int N, int M) {
    if (b <= kc) return b < M ? b : -1;
    const int j = b - (N - M);
    return j > kc && j < M ? j : -1;
}
__device__ __forceinline__ int band_to_bin(int j, int kc, int N, int M) { return j <= kc ? j : j + (N - M); }

// Inverse (sgn = +1) or forward (sgn = -1) DFTs of 2, 3, 4, 5, 8 and 9
// points in registers: X[k] = sum_n x[n] exp(sgn 2 pi i n k / R).
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

__device__ __forceinline__ void dft3(float2& a, float2& b, float2& c, float sgn) {
    const float s3 = 0.86602540378443864676f;
    const float2 t1 = cadd(b, c);
    const float2 t2 = make_float2(a.x - 0.5f * t1.x, a.y - 0.5f * t1.y);
    const float2 t3 = mul_i(make_float2(s3 * (b.x - c.x), s3 * (b.y - c.y)), sgn);
    a = cadd(a, t1);
    b = cadd(t2, t3);
    c = csub(t2, t3);
}

__device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d, float sgn) {
    const float2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d);
    const float2 d1 = mul_i(csub(b, d), sgn);
    a = cadd(s0, s1);
    c = csub(s0, s1);
    b = cadd(d0, d1);
    d = csub(d0, d1);
}

template <int R>
__device__ __forceinline__ void dft(float2 (&v)[R], float sgn) {
    if constexpr (R == 2) {
        const float2 t = v[0];
        v[0] = cadd(t, v[1]);
        v[1] = csub(t, v[1]);
    } else if constexpr (R == 3) {
        dft3(v[0], v[1], v[2], sgn);
    } else if constexpr (R == 4) {
        dft4(v[0], v[1], v[2], v[3], sgn);
    } else if constexpr (R == 5) {
        const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
        const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
        const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
        const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
        const float2 x0 = v[0];
        v[0] = cadd(x0, cadd(a1, a2));
        const float2 p1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
        const float2 p2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
        const float2 q1 = mul_i(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y), sgn);
        const float2 q2 = mul_i(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y), sgn);
        v[1] = cadd(p1, q1);
        v[4] = csub(p1, q1);
        v[2] = cadd(p2, q2);
        v[3] = csub(p2, q2);
    } else if constexpr (R == 8) {
        // even and odd halves, then W8^k on the odd one
        float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4(e0, e1, e2, e3, sgn);
        dft4(o0, o1, o2, o3, sgn);
        const float h = 0.70710678118654752440f;
        o1 = make_float2(h * (o1.x - sgn * o1.y), h * (o1.y + sgn * o1.x));     // * (1 + sgn i) / sqrt 2
        o2 = mul_i(o2, sgn);                                                      // * sgn i
        o3 = make_float2(-h * (o3.x + sgn * o3.y), h * (sgn * o3.x - o3.y));    // * (-1 + sgn i) / sqrt 2
        v[0] = cadd(e0, o0);
        v[4] = csub(e0, o0);
        v[1] = cadd(e1, o1);
        v[5] = csub(e1, o1);
        v[2] = cadd(e2, o2);
        v[6] = csub(e2, o2);
        v[3] = cadd(e3, o3);
        v[7] = csub(e3, o3);
    } else {                                     // R == 9: 3 x 3
        // X[k2 + 3 k1] = sum_n1 W3^(n1 k1) W9^(n1 k2) sum_n2 x[n1 + 3 n2] W3^(n2 k2)
        dft3(v[0], v[3], v[6], sgn);
        dft3(v[1], v[4], v[7], sgn);
        dft3(v[2], v[5], v[8], sgn);
        const float c1 = 0.76604444311897803520f, s1 = 0.64278760968653932632f;   // cos, sin 2 pi / 9
        const float c2 = 0.17364817766693034885f, s2 = 0.98480775301220805936f;   // 4 pi / 9
        const float c4 = -0.93969262078590838405f, s4 = 0.34202014332566873304f;  // 8 pi / 9
        auto rot = [&](float2 x, float c, float sn) {
            return make_float2(c * x.x - sgn * sn * x.y, c * x.y + sgn * sn * x.x);
        };
        v[4] = rot(v[4], c1, s1);                // n1 = 1, k2 = 1
        v[7] = rot(v[7], c2, s2);                // n1 = 1, k2 = 2
        v[5] = rot(v[5], c2, s2);                // n1 = 2, k2 = 1
        v[8] = rot(v[8], c4, s4);                // n1 = 2, k2 = 2
        dft3(v[0], v[1], v[2], sgn);             // k2 = 0 -> X0, X3, X6
        dft3(v[3], v[4], v[5], sgn);             // k2 = 1 -> X1, X4, X7
        dft3(v[6], v[7], v[8], sgn);             // k2 = 2 -> X2, X5, X8
        const float2 x0 = v[0], x3 = v[1], x6 = v[2], x1 = v[3], x4 = v[4], x7 = v[5], x2 = v[6], x5 = v[7],
                     x8 = v[8];
        v[0] = x0; v[1] = x1; v[2] = x2; v[3] = x3; v[4] = x4; v[5] = x5; v[6] = x6; v[7] = x7; v[8] = x8;
    }
}

// w^r for r = 1 .. R-1 from w (|w| = 1), by products in a shallow tree
// (w^2 = w w, w^3 = w^2 w, w^4 = w^2 w^2, ...): at most three roundings deep,
// so each power is within a few ulp of the exact root, and one table read
// replaces R - 1.
template <int R>
__device__ __forceinline__ void twiddle_powers(float2 w, float2 (&p)[R]) {
    p[1] = w;
    if constexpr (R > 2) p[2] = cmul(w, w);
    if constexpr (R > 3) p[3] = cmul(p[2], w);
    if constexpr (R > 4) p[4] = cmul(p[2], p[2]);
    if constexpr (R > 5) p[5] = cmul(p[4], w);
    if constexpr (R > 6) p[6] = cmul(p[4], p[2]);
    if constexpr (R > 7) p[7] = cmul(p[4], p[3]);
    if constexpr (R > 8) p[8] = cmul(p[4], p[4]);
}

// One Stockham pass of radix R over the transforms of one work item, each of
// length N with tpf = 2^lg_tpf threads; Ns = product of the radices already
// applied.  Butterfly j reads x[j + r N/R] (src(f, index)), multiplies by
// the twiddles W_N^(r k N/(Ns R)) (k = j mod Ns; the table gives r = 1, the
// other powers follow by products; none in the first pass, where
// Ns = 1) and writes X[(j / Ns) Ns R + k + q Ns] (dst(f, index, value)).
// j / Ns is formed as floor((j + 0.5) / Ns) in FP32, exact for these sizes.
// tw[q] = exp(-2 pi i q / N); the inverse (sgn = +1) conjugates it.
template <int R, bool FIRST, class Src, class Dst>
__device__ __forceinline__ void stockham(int N, int Ns, int lg_tpf, const float2* __restrict__ tw, float sgn,
                                         Src&& src, Dst&& dst) {
    const int nb = N / R;
    const int f = threadIdx.x >> lg_tpf;
    const int tpf = 1 << lg_tpf;
    const int step = nb / Ns;
    const float inv_ns = 1.0f / (float)Ns;
    for (int j = threadIdx.x & (tpf - 1); j < nb; j += tpf) {
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src(f, j + r * nb);
        int base = j * R;
        if constexpr (!FIRST) {
            const int qj = __float2int_rd(((float)j + 0.5f) * inv_ns);
            const int k = j - qj * Ns;
            float2 w = tw[k * step];
            w.y *= -sgn;
            float2 wp[R];
            twiddle_powers<R>(w, wp);
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], wp[r]);
            base = qj * Ns * R + k;
        }
        dft<R>(v, sgn);
#pragma unroll
        for (int q = 0; q < R; ++q) dst(f, base + q * Ns, v[q]);
    }
}

// The same pass in place, for a transform that lives in one wave and whose
// butterflies take at most MAXIT rounds of its threads: every thread reads
// the inputs of all its butterflies before any thread writes, and a wave's
// LDS operations complete in the order it issues them, so the pass may
// overwrite its own input (one LDS buffer per transform instead of two).
template <int R, int MAXIT, class Src, class Dst>
__device__ __forceinline__ void stockham_inplace(int N, int Ns, int lg_tpf, const float2* __restrict__ tw, float sgn,
                                                 Src&& src, Dst&& dst) {
    const int nb = N / R;
    const int f = threadIdx.x >> lg_tpf;
    const int tpf = 1 << lg_tpf;
    const int step = nb / Ns;
    const float inv_ns = 1.0f / (float)Ns;
    const int j0 = threadIdx.x & (tpf - 1);
    float2 v[MAXIT][R];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int j = j0 + it * tpf;
        if (j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = src(f, j + r * nb);
        }
    }
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int j = j0 + it * tpf;
        if (j >= nb) continue;
        const int qj = __float2int_rd(((float)j + 0.5f) * inv_ns);
        const int k = j - qj * Ns;
        float2 w = tw[k * step];
        w.y *= -sgn;
        float2 wp[R];
        twiddle_powers<R>(w, wp);
#pragma unroll
        for (int r = 1; r < R; ++r) v[it][r] = cmul(v[it][r], wp[r]);
        dft<R>(v[it], sgn);
        const int base = qj * Ns * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) dst(f, base + q * Ns, v[it][q]);
    }
}

template <class Src, class Dst>
__device__ __forceinline__ void stockham_inplace_r(int R, int N, int Ns, int lg_tpf, const float2* tw, float sgn,
                                                   Src&& src, Dst&& dst) {
    switch (R) {
        case 2: stockham_inplace<2, 2>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
        case 3: stockham_inplace<3, 2>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
        case 4: stockham_inplace<4, 2>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
        case 5: stockham_inplace<5, 2>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
        case 8: stockham_inplace<8, 2>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
        default: stockham_inplace<9, 2>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
    }
}

template <bool FIRST, class Src, class Dst>
__device__ __forceinline__ void stockham_r(int R, int N, int Ns, int lg_tpf, const float2* tw, float sgn, Src&& src,
                                           Dst&& dst) {
    switch (R) {
        case 2: stockham<2, FIRST>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
        case 3: stockham<3, FIRST>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
        case 4: stockham<4, FIRST>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
        case 5: stockham<5, FIRST>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
        case 8: stockham<8, FIRST>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
        default: stockham<9, FIRST>(N, Ns, lg_tpf, tw, sgn, src, dst); break;
    }
}

// First pass of an inverse transform whose nonzero inputs all lie in
// x[0 .. nb) and x[N - nb .. N) (nb = N / R): only inputs r = 0 and r = R - 1
// of a butterfly can be nonzero, so X[k] = x[j] + x[j + N - nb] e^{-2 pi i k / R}
// (twiddles from the table, tw[k N / R]); no other input is read.
template <int R, class Src, class Dst>
__device__ __forceinline__ void first_pass_sparse(int N, int lg_tpf, const float2* __restrict__ tw, Src&& src,
                                                  Dst&& dst) {
    const int nb = N / R;
    const int f = threadIdx.x >> lg_tpf;
    const int tpf = 1 << lg_tpf;
    float2 w[R];
#pragma unroll
    for (int k = 0; k < R; ++k) w[k] = tw[k * nb];
    for (int j = threadIdx.x & (tpf - 1); j < nb; j += tpf) {
        const float2 a = src(f, j), b = src(f, j + N - nb);
#pragma unroll
        for (int k = 0; k < R; ++k)
            dst(f, j * R + k, make_float2(a.x + b.x * w[k].x - b.y * w[k].y, a.y + b.x * w[k].y + b.y * w[k].x));
    }
}

template <class Src, class Dst>
__device__ __forceinline__ void first_pass_sparse_r(int R, int N, int lg_tpf, const float2* tw, Src&& src, Dst&& dst) {
    switch (R) {
        case 2: first_pass_sparse<2>(N, lg_tpf, tw, src, dst); break;
        case 3: first_pass_sparse<3>(N, lg_tpf, tw, src, dst); break;
        case 4: first_pass_sparse<4>(N, lg_tpf, tw, src, dst); break;
        case 5: first_pass_sparse<5>(N, lg_tpf, tw, src, dst); break;
        case 8: first_pass_sparse<8>(N, lg_tpf, tw, src, dst); break;
        default: first_pass_sparse<9>(N, lg_tpf, tw, src, dst); break;
    }
}

// Between passes: a transform handled by at most 64 threads lives in one
// wave (its LDS rows are that wave's alone), so the wave's own LDS order is
// enough; wider transforms need the workgroup barrier.
__device__ __forceinline__ void pass_sync(int lg_tpf) {
    if (lg_tpf <= 6) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Whether the middle passes of an N-point transform on 2^lg_tpf threads may
// run in place: the transform lives in one wave (at most 64 threads) and no
// middle pass needs more than two rounds of its threads.
__host__ __device__ inline bool ifft_inplace_ok(int N, int lg_tpf, const int* rad, int nrad) {
    if (lg_tpf > 6) return false;
    for (int i = 1; i + 1 < nrad; ++i)
        if (N / rad[i] > (2 << lg_tpf)) return false;
    return true;
}

// Whole inverse transforms of one item: the first pass gathers its inputs
// with src (band entries or zero), the middle passes run LDS to LDS at
// stride ld, the last pass hands every output to out(f, index, value).
// At least two passes (N >= 72 > the largest radix).  band_lo / band_hi:
// the nonzero inputs lie in [0, band_lo] and [N - band_hi, N); when both
// parts fit in one first-pass stride the sparse first pass is used.
//
// inplace: the middle passes overwrite their input (ifft_inplace_ok holds
// for this transform), and b is not used.
template <class Src, class Out>
__device__ __forceinline__ void ifft_item(int N, int ld, int lg_tpf, const int* rad, int nrad, const float2* tw,
                                          float2* a, float2* b, int band_lo, int band_hi, bool inplace, Src&& src,
                                          Out&& out) {
    auto to_lds = [&](float2* buf) {
        return [buf, ld](int f, int i, float2 v) { buf[f * ld + i] = v; };
    };
    auto from_lds = [&](const float2* buf) {
        return [buf, ld](int f, int i) { return buf[f * ld + i]; };
    };
    const int nb0 = N / rad[0];
    if (band_lo < nb0 && band_hi <= nb0)
        first_pass_sparse_r(rad[0], N, lg_tpf, tw, src, to_lds(a));
    else
        stockham_r<true>(rad[0], N, 1, lg_tpf, tw, 1.0f, src, to_lds(a));
    pass_sync(lg_tpf);
    int Ns = rad[0];
    for (int i = 1; i + 1 < nrad; ++i) {
        if (inplace) {
            stockham_inplace_r(rad[i], N, Ns, lg_tpf, tw, 1.0f, from_lds(a), to_lds(a));
        } else {
            stockham_r<false>(rad[i], N, Ns, lg_tpf, tw, 1.0f, from_lds(a), to_lds(b));
            float2* t = a;
            a = b;
            b = t;
        }
        pass_sync(lg_tpf);
        Ns *= rad[i];
    }
    stockham_r<false>(rad[nrad - 1], N, Ns, lg_tpf, tw, 1.0f, from_lds(a), out);
}

// tw[q] = exp(-2 pi i q / N) for q < N, each rounded once from FP64.  For
// N divisible by 4 only the first quarter is evaluated: adding N/4 to q
// multiplies by -i, (c, s) -> (s, -c), an exact move of the rounded values.
__device__ void fill_twiddles(float2* tw, int N) {
    const bool quarter = (N & 3) == 0;
    const int n = quarter ? N >> 2 : N;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)q / (double)N, &s, &c);
        const float fc = (float)c, fs = (float)s;
        tw[q] = make_float2(fc, fs);
        if (quarter) {
            tw[q + n] = make_float2(fs, -fc);
            tw[q + 2 * n] = make_float2(-fc, -fs);
            tw[q + 3 * n] = make_float2(-fs, fc);
        }
    }
}

// exp(-pi^2 l^2 f^2), f = k/N wrapped to [-1/2, 1/2): the 1-D factor of sqrt(S)
__device__ __forceinline__ float gauss_filter(int k, int N, float corr_len) {
    const double a = 3.14159265358979323846 * 3.14159265358979323846 * (double)corr_len * (double)corr_len;
    const int kk = (k < (N + 1) / 2) ? k : k - N;
    const double f = (double)kk / (double)N;
    return (float)exp(-a * f * f);
}

__device__ __forceinline__ int ld_of(int N) { return N | 1; }   // odd stride spreads LDS banks

// Column work item: plane pair q, band columns j0 .. j0 + 2^lg_cpb - 1.  The
// first pass draws the noise of the band rows times the separable filter
// (zero elsewhere), the transform runs along y, the last pass writes
// V[q][j][y] for y < H (column-major, so consecutive threads write
// consecutive y).  Item (q=0, j0=0) also publishes the row transforms'
// twiddle table.
__device__ __forceinline__ void fields_cols_item(const FieldPlan& fp, float2* __restrict__ V, float2* __restrict__ twx_out,
                                 int lg_cpb, int q, int j0, float2* smem, bool fresh) {
    const int cpb = 1 << lg_cpb;
    const int N = fp.Nfy, ld = ld_of(N);
    const bool inplace = ifft_inplace_ok(N, 8 - lg_cpb, fp.rad_y, fp.nrad_y);
    float2* buf0 = smem;
    float2* buf1 = smem + cpb * ld;
    float2* tw = smem + (inplace ? 1 : 2) * cpb * ld;
    float* filt = reinterpret_cast<float*>(tw + N);
    if (q == 0 && j0 == 0) fill_twiddles(twx_out, fp.Nfx);
    const int lg_tpf = 8 - lg_cpb;             // 256 threads
    if (fresh) {                               // first item of this frame in the workgroup
        __syncthreads();                       // every wave done with the previous frame's tables
        fill_twiddles(tw, N);
        // only the band rows' factors are ever read (bins |k| <= kcy)
        for (int i = threadIdx.x; i <= 2 * fp.kcy; i += blockDim.x) {
            const int k = i <= fp.kcy ? i : N - (i - fp.kcy);
            filt[k] = gauss_filter(k, N, fp.corr_len);
        }
        __syncthreads();
    }
    // this thread's column: its bin and its filter factor, once per item
    const int jme = j0 + (int)(threadIdx.x >> lg_tpf);
    const bool col_ok = jme < fp.Mx;
    const int kx = band_to_bin(jme, fp.kcx, fp.Nfx, fp.Mx);
    const float hx = col_ok ? gauss_filter(kx, fp.Nfx, fp.corr_len) * fp.norm : 0.0f;
    auto noise = [&](int, int ky) -> float2 {
        const int kyw = ky < (N + 1) / 2 ? ky : N - ky;
        if (!col_ok || kyw > fp.kcy) return make_float2(0.f, 0.f);
        const float h = hx * filt[ky];
        const float2 z = bin_noise(kx, ky, q, fp.k0, fp.k1);
        return make_float2(h * z.x, h * z.y);
    };
    const int H = fp.H, Mx = fp.Mx;
    float2* Vq = V + (size_t)q * Mx * H;
    auto out = [&](int c, int y, float2 v) {
        const int j = j0 + c;
        if (y < H && j < Mx) Vq[(size_t)j * H + y] = v;
    };
    ifft_item(N, ld, lg_tpf, fp.rad_y, fp.nrad_y, tw, buf0, buf1, fp.kcy, fp.kcy, inplace, noise, out);
    if (lg_tpf > 6) __syncthreads();           // LDS free for the next item (shared rows)
}

// Row work item: plane pair q, output rows y0 .. y0 + 2^lg_rpb - 1.  The first
// pass gathers the band entries of V (zero elsewhere), the transform runs
// along x, the last pass writes planes 2q, 2q+1 for x < W.
__device__ __forceinline__ void fields_rows_item(const FieldPlan& fp, const float2* __restrict__ V, float* __restrict__ F,
                                 const float2* __restrict__ twx, int lg_rpb, int q, int y0, float2* smem, bool fresh) {
    const int rpb = 1 << lg_rpb;
    const int N = fp.Nfx, ld = ld_of(N);
    const bool inplace = ifft_inplace_ok(N, 8 - lg_rpb, fp.rad_x, fp.nrad_x);
    float2* buf0 = smem;
    float2* buf1 = smem + rpb * ld;
    float2* tw = smem + (inplace ? 1 : 2) * rpb * ld;
    const int H = fp.H, W = fp.W, Mx = fp.Mx, kcx = fp.kcx;
    if (fresh) {                               // first item of this frame in the workgroup
        __syncthreads();                       // every wave done with the previous frame's table
        for (int k = threadIdx.x; k < N; k += blockDim.x) tw[k] = twx[k];
        __syncthreads();
    }
    const float2* Vq = V + (size_t)q * Mx * H;
    auto band = [&](int r, int b) -> float2 {
        const int y = y0 + r;
        const int j = bin_to_band(b, kcx, N, Mx);
        return (y < H && j >= 0) ? Vq[(size_t)j * H + y] : make_float2(0.f, 0.f);
    };
    const int p0 = 2 * q, p1 = 2 * q + 1;
    const float s0 = fp.sigma[p0];
    const bool has1 = p1 < fp.nplanes;
    const float s1 = has1 ? fp.sigma[p1] : 0.0f;
    float* F0 = F + (size_t)p0 * H * W;
    float* F1 = F + (size_t)p1 * H * W;
    // this thread's output row (the last pass hands it only its own row)
    const int ry = y0 + (int)(threadIdx.x >> (8 - lg_rpb));
    float* const row0 = F0 + (size_t)ry * W;
    float* const row1 = F1 + (size_t)ry * W;
    auto out = [&](int, int x, float2 v) {
        if (ry >= H || x >= W) return;
        row0[x] = s0 * v.x;
        if (has1) row1[x] = s1 * v.y;
    };
    ifft_item(N, ld, 8 - lg_rpb, fp.rad_x, fp.nrad_x, tw, buf0, buf1, kcx, Mx - 1 - kcx, inplace, band, out);
    if (lg_rpb < 2) __syncthreads();           // LDS free for the next item (shared rows)
}

// Single frame: persistent workgroups stride over the (pair, chunk) items, so
// the twiddle table (and the column filter) is built once per workgroup.
__global__ void __launch_bounds__(kThreads) fields_cols_kernel(FieldPlan fp, float2* __restrict__ V, int lg_cpb,
                                                               float2* __restrict__ twx_out, int nchunks) {
    extern __shared__ float2 smem[];
    const int total = nchunks * fp.npairs;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int q = item / nchunks;
        fields_cols_item(fp, V, twx_out, lg_cpb, q, (item - q * nchunks) << lg_cpb, smem, item == (int)blockIdx.x);
    }
}

// Row items in XCD order: workgroups go to the 8 XCDs round-robin (b on XCD
// b % 8), so in each block of 32 slots of the persistent loop the 4 slots of
// one XCD take 4 consecutive items; their 4 x 4 rows fill whole 128-byte
// lines of the column-major V, which then come from that XCD's L2 instead of
// being fetched by 4 XCDs.
__device__ __forceinline__ int xcd_row_item(int k) { return (k & ~31) | ((k & 7) << 2) | ((k >> 3) & 3); }

__global__ void __launch_bounds__(kThreads) fields_rows_kernel(FieldPlan fp, const float2* __restrict__ V,
                                                               float* __restrict__ F, int lg_rpb,
                                                               const float2* __restrict__ twx, int nchunks) {
    extern __shared__ float2 smem[];
    const int total = nchunks * fp.npairs;
    const int slots = (total + 31) & ~31;
    bool fresh = true;
    for (int k = blockIdx.x; k < slots; k += gridDim.x) {
        const int item = xcd_row_item(k);
        if (item >= total) continue;
        const int q = item / nchunks;
        fields_rows_item(fp, V, F, twx, lg_rpb, q, (item - q * nchunks) << lg_rpb, smem, fresh);
        fresh = false;
    }
}

// Batched, persistent forms: workgroups stride over the (frame, item) list.
__global__ void __launch_bounds__(kThreads) fields_cols_batch(const FrameDesc* __restrict__ fr,
                                                              const int* __restrict__ first, int n) {
    extern __shared__ float2 smem[];
    const int total = first[n];
    int prev = -1;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int f = find_frame(first, n, item);
        const FrameDesc& d = fr[f];
        const int l = item - first[f];
        const int q = l / d.ncol_chunks;
        fields_cols_item(d.fp, d.V, d.twx, d.lg_cpb, q, (l - q * d.ncol_chunks) << d.lg_cpb, smem, f != prev);
        prev = f;
    }
}

__global__ void __launch_bounds__(kThreads) fields_rows_batch(const FrameDesc* __restrict__ fr,
                                                              const int* __restrict__ first, int n) {
    extern __shared__ float2 smem[];
    const int total = first[n];
    const int slots = (total + 31) & ~31;
    int prev = -1;
    for (int k = blockIdx.x; k < slots; k += gridDim.x) {
        const int item = xcd_row_item(k);
        if (item >= total) continue;
        const int f = find_frame(first, n, item);
        const FrameDesc& d = fr[f];
        const int l = item - first[f];
        const int q = l / d.nrow_chunks;
        fields_rows_item(d.fp, d.V, d.fields, d.twx, d.lg_rpb, q, (l - q * d.nrow_chunks) << d.lg_rpb, smem,
                         f != prev);
        prev = f;
    }
}

// ---------------------------------------------------------- fixed plans
// Transforms whose length N = R0 R1 R2 is known at compile time, with one
// butterfly per thread and pass: TPF = max(N / R) threads per transform, T
// transforms per workgroup.  In the runtime-sized passes above a 576-point
// transform (9 x 8 x 8) on 64 threads runs each radix-8 pass as two rounds,
// the second with 8 of 64 lanes busy, and forms every index at run time;
// here every lane of a round has a butterfly (except in the 64-butterfly
// radix-9 pass) and the index arithmetic folds into constants.  The
// arithmetic of every butterfly is the runtime path's (same twiddle table
// entry, same powers by products, same DFT), so both give the same bits.
//
// Passes: the sparse first pass (inputs x[j], x[j + N - N/R0]) writes the
// LDS row of its transform; the middle pass reads its R1 inputs, waits for
// the whole workgroup, and overwrites them in place; the last pass reads
// and hands its R2 outputs to the caller's store.

// Entry m of the table fill_twiddles writes for an N-point transform, bit
// for bit (the same FP64 evaluation and the same exact quarter moves).
__device__ __forceinline__ float2 twiddle_entry(int m, int N) {
    const bool quarter = (N & 3) == 0;
    const int n = quarter ? N >> 2 : N;
    const int quad = m / n, q = m - quad * n;
    double sn, cs;
    sincospi(-2.0 * (double)q / (double)N, &sn, &cs);
    const float fc = (float)cs, fs = (float)sn;
    switch (quad) {
        case 0: return make_float2(fc, fs);
        case 1: return make_float2(fs, -fc);
        case 2: return make_float2(-fc, -fs);
        default: return make_float2(-fs, fc);
    }
}

template <int R0, int R1, int R2, int T>
struct FixedPlan {
    static constexpr int N = R0 * R1 * R2;
    static constexpr int NB0 = N / R0, NB1 = N / R1, NB2 = N / R2;
    static constexpr int TPF = NB0 > NB1 ? (NB0 > NB2 ? NB0 : NB2) : (NB1 > NB2 ? NB1 : NB2);
    static constexpr int NT = T * TPF;
    static constexpr int LD = N | 1;
    // the twiddles the passes use: entries 0 .. NB2-1 of the table (the last
    // pass, and the middle pass's k R2 < NB2), then k NB0 for k < R0 (the
    // first pass) at NB2 + k
    static constexpr int NTW = NB2 + R0;
    static_assert((R0 - 1) * R2 < NB2, "middle-pass twiddles inside the first NB2 entries");
    static constexpr size_t lds_bytes = (size_t)(T * LD + NTW) * 8;
    __device__ static void fill_table(float2* ct) {
        for (int i = threadIdx.x; i < NTW; i += NT) ct[i] = twiddle_entry(i < NB2 ? i : (i - NB2) * NB0, N);
    }
};

// The first pass's butterfly of this thread: transform t % T, butterfly
// t / T (consecutive threads take consecutive transforms, so that a
// column-major source is read in runs of T), valid for t < T N / R0.
template <int R0, int R1, int R2, int T>
__device__ __forceinline__ bool fixed_first(int& f, int& j) {
    using P = FixedPlan<R0, R1, R2, T>;
    const int t = threadIdx.x;
    f = t % T;
    j = t / T;
    return t < T * P::NB0;
}

// The transforms of one workgroup; a = x[j], b = x[j + N - N/R0] are the
// inputs of this thread's first-pass butterfly (fixed_first), the compact
// twiddle table tw (FixedPlan::fill_table) is in place and a barrier has
// passed since it was written.  out(f, j, v) takes the last-pass butterfly j
// of transform f: outputs j + s N/R2 in v[s] (s < R2), so that the caller
// forms one address per butterfly and stores at constant offsets from it.
template <int R0, int R1, int R2, int T, class Out>
__device__ __forceinline__ void fixed_ifft(float2* __restrict__ buf, const float2* __restrict__ tw, float2 a,
                                           float2 b, Out&& out) {
    using P = FixedPlan<R0, R1, R2, T>;
    constexpr int LD = P::LD;
    int f1, j1;
    if (fixed_first<R0, R1, R2, T>(f1, j1)) {    // sparse radix-R0 pass
        const int f = f1, j = j1;
        float2 w[R0];
#pragma unroll
        for (int k = 0; k < R0; ++k) w[k] = tw[P::NB2 + k];
        float2* row = buf + f * LD + j * R0;
#pragma unroll
        for (int k = 0; k < R0; ++k)
            row[k] = make_float2(a.x + b.x * w[k].x - b.y * w[k].y, a.y + b.x * w[k].y + b.y * w[k].x);
    }
    __syncthreads();
    const int f = threadIdx.x / P::TPF, j = threadIdx.x - f * P::TPF;
    float2* const row = buf + f * LD;
    {                                            // radix-R1 pass, in place, Ns = R0
        constexpr int Ns = R0, step = P::NB1 / Ns;
        float2 v[R1];
        const bool act = j < P::NB1;
        if (act) {
#pragma unroll
            for (int r = 0; r < R1; ++r) v[r] = row[j + r * P::NB1];
        }
        __syncthreads();                         // every input read before any is overwritten
        if (act) {
            const int qj = j / Ns, k = j - qj * Ns;
            float2 w = tw[k * step];
            w.y *= -1.0f;
            float2 wp[R1];
            twiddle_powers<R1>(w, wp);
#pragma unroll
            for (int r = 1; r < R1; ++r) v[r] = cmul(v[r], wp[r]);
            dft<R1>(v, 1.0f);
            const int base = qj * Ns * R1 + k;
#pragma unroll
            for (int q = 0; q < R1; ++q) row[base + q * Ns] = v[q];
        }
    }
    __syncthreads();
    if (j < P::NB2) {                            // last pass, radix R2, Ns = N / R2
        constexpr int Ns = P::NB2;
        float2 v[R2];
#pragma unroll
        for (int r = 0; r < R2; ++r) v[r] = row[j + r * P::NB2];
        float2 w = tw[j];
        w.y *= -1.0f;
        float2 wp[R2];
        twiddle_powers<R2>(w, wp);
#pragma unroll
        for (int r = 1; r < R2; ++r) v[r] = cmul(v[r], wp[r]);
        dft<R2>(v, 1.0f);
        out(f, j, v);
    }
}

// Column items of a fixed plan: T band columns of one plane pair per
// workgroup (the runtime path's fields_cols_item, one butterfly per thread).
template <int R0, int R1, int R2, int T>
__global__ void __launch_bounds__((FixedPlan<R0, R1, R2, T>::NT))
    fields_cols_fixed(FieldPlan fp, float2* __restrict__ V, float2* __restrict__ twx_out, int nchunks) {
    using P = FixedPlan<R0, R1, R2, T>;
    constexpr int N = P::N;
    extern __shared__ float2 smem[];
    float2* buf = smem;
    float2* tw = smem + T * P::LD;
    float* filt = reinterpret_cast<float*>(tw + P::NTW);   // band rows: |ky| at |ky|, -|ky| at kcy + |ky|
    const int item = blockIdx.x;
    const int q = item / nchunks, j0 = (item - q * nchunks) * T;
    if (item == 0) fill_twiddles(twx_out, fp.Nfx);
    P::fill_table(tw);
    for (int i = threadIdx.x; i <= 2 * fp.kcy; i += P::NT) {
        const int k = i <= fp.kcy ? i : N - (i - fp.kcy);
        filt[i] = gauss_filter(k, N, fp.corr_len);
    }
    __syncthreads();
    int f1, j1;
    const bool first = fixed_first<R0, R1, R2, T>(f1, j1);
    const int jme = j0 + f1;
    const bool col_ok = jme < fp.Mx;
    const int kx = band_to_bin(jme, fp.kcx, fp.Nfx, fp.Mx);
    const float hx = col_ok ? gauss_filter(kx, fp.Nfx, fp.corr_len) * fp.norm : 0.0f;
    auto noise = [&](int, int ky) -> float2 {
        const int kyw = ky < (N + 1) / 2 ? ky : N - ky;
        if (!col_ok || kyw > fp.kcy) return make_float2(0.f, 0.f);
        const float h = hx * filt[ky < (N + 1) / 2 ? kyw : fp.kcy + kyw];
        const float2 z = bin_noise(kx, ky, q, fp.k0, fp.k1);
        return make_float2(h * z.x, h * z.y);
    };
    const int H = fp.H, Mx = fp.Mx;
    float2* Vq = V + (size_t)q * Mx * H;
    auto out = [&](int c, int y, const float2 (&v)[R2]) {
        if (j0 + c >= Mx) return;
        float2* col = Vq + (size_t)(j0 + c) * H + y;
#pragma unroll
        for (int s = 0; s < R2; ++s)
            if (y + s * P::NB2 < H) col[s * P::NB2] = v[s];
    };
    float2 a = make_float2(0.f, 0.f), b = a;
    if (first) {
        a = noise(f1, j1);
        b = noise(f1, j1 + N - P::NB0);
    }
    fixed_ifft<R0, R1, R2, T>(buf, tw, a, b, out);
}

// Row items of a fixed plan: T output rows of one plane pair per workgroup,
// in the XCD order of fields_rows_kernel.
template <int R0, int R1, int R2, int T>
__global__ void __launch_bounds__((FixedPlan<R0, R1, R2, T>::NT))
    fields_rows_fixed(FieldPlan fp, const float2* __restrict__ V, float* __restrict__ F, int nchunks) {
    using P = FixedPlan<R0, R1, R2, T>;
    constexpr int N = P::N;
    extern __shared__ float2 smem[];
    float2* buf = smem;
    float2* tw = smem + T * P::LD;
    const int item = xcd_row_item(blockIdx.x);
    if (item >= nchunks * fp.npairs) return;
    const int q = item / nchunks, y0 = (item - q * nchunks) * T;
    const int H = fp.H, W = fp.W, Mx = fp.Mx, kcx = fp.kcx;
    const float2* Vq = V + (size_t)q * Mx * H;
    auto band = [&](int r, int b) -> float2 {
        const int y = y0 + r;
        const int j = bin_to_band(b, kcx, N, Mx);
        return (y < H && j >= 0) ? Vq[(size_t)j * H + y] : make_float2(0.f, 0.f);
    };
    int f1, j1;
    float2 a = make_float2(0.f, 0.f), b = a;
    if (fixed_first<R0, R1, R2, T>(f1, j1)) {     // inputs in flight while the table is evaluated
        a = band(f1, j1);
        b = band(f1, j1 + N - P::NB0);
    }
    P::fill_table(tw);
    __syncthreads();
    const int p0 = 2 * q, p1 = 2 * q + 1;
    const float s0 = fp.sigma[p0];
    const bool has1 = p1 < fp.nplanes;
    const float s1 = has1 ? fp.sigma[p1] : 0.0f;
    float* F0 = F + (size_t)p0 * H * W;
    float* F1 = F + (size_t)p1 * H * W;
    auto out = [&](int r, int x, const float2 (&v)[R2]) {
        const int y = y0 + r;
        if (y >= H) return;
        float* o0 = F0 + (size_t)y * W + x;
        float* o1 = F1 + (size_t)y * W + x;
#pragma unroll
        for (int s = 0; s < R2; ++s) {
            if (x + s * P::NB2 >= W) continue;
            o0[s * P::NB2] = s0 * v[s].x;
            if (has1) o1[s * P::NB2] = s1 * v[s].y;
        }
    };
    fixed_ifft<R0, R1, R2, T>(buf, tw, a, b, out);
}

__global__ void debug_noise_kernel(int Nfy, int Nfx, int pair, uint32_t k0, uint32_t k1, uint32_t* raw,
                                   float* normals) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Nfy * Nfx) return;
    const int ky = idx / Nfx, kx = idx - ky * Nfx;
    uint32_t o[4];
    const float2 z = bin_noise(kx, ky, pair, k0, k1, o);
#pragma unroll
    for (int e = 0; e < 4; ++e) raw[(size_t)idx * 4 + e] = o[e];
    if (normals) {
        normals[(size_t)idx * 2] = z.x;
        normals[(size_t)idx * 2 + 1] = z.y;
    }
}

}  // namespace

// LDS buffers per transform: one when the middle passes run in place.
static int lds_buffers(int N, int nb) {
    int rad[12];
    const int n = factor_radices(N, rad);
    return n && ifft_inplace_ok(N, 8 - __builtin_ctz((unsigned)nb), rad, n) ? 1 : 2;
}
size_t fields_cols_lds(int N, int nb) {
    return (size_t)(lds_buffers(N, nb) * nb * (N | 1) + N) * 8 + (size_t)N * 4;
}
size_t fields_rows_lds(int N, int nb) { return (size_t)(lds_buffers(N, nb) * nb * (N | 1) + N) * 8; }

int fields_pick_lg(int N, size_t budget, bool cols) {
    int lg = 3;
    while (lg > 0 && (cols ? fields_cols_lds(N, 1 << lg) : fields_rows_lds(N, 1 << lg)) > budget) --lg;
    return lg;
}

int fields_batch_resident(bool cols, size_t lds) {
    return resident_workgroups(cols ? (const void*)fields_cols_batch : (const void*)fields_rows_batch, kThreads, lds);
}

hipError_t launch_fields_batch(const BatchLaunch& bl, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)fields_cols_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)fields_rows_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (bl.items[ST_COLS] > 0) {
        hipLaunchKernelGGL(fields_cols_batch, dim3(bl.grid[ST_COLS]), dim3(kThreads), bl.lds[ST_COLS], s, bl.frames,
                           bl.first + ST_COLS * (bl.n + 1), bl.n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (bl.items[ST_ROWS] > 0)
        hipLaunchKernelGGL(fields_rows_batch, dim3(bl.grid[ST_ROWS]), dim3(kThreads), bl.lds[ST_ROWS], s, bl.frames,
                           bl.first + ST_ROWS * (bl.n + 1), bl.n);
    return hipGetLastError();
}

// Radix passes for a 5-smooth length: 9s and 8s first (fewest passes), then
// 4, 2, 3, 5 for what is left.
int factor_radices(int n, int* rad) {
    int k = 0;
    while (n % 9 == 0) { rad[k++] = 9; n /= 9; }
    while (n % 8 == 0) { rad[k++] = 8; n /= 8; }
    while (n % 4 == 0) { rad[k++] = 4; n /= 4; }
    while (n % 2 == 0) { rad[k++] = 2; n /= 2; }
    while (n % 3 == 0) { rad[k++] = 3; n /= 3; }
    while (n % 5 == 0) { rad[k++] = 5; n /= 5; }
    return n == 1 ? k : 0;
}

// Whether a transform runs on the fixed 576-point plan (9 x 8 x 8, the grid
// of 512-pixel sides at the default correlation length): its radices are
// those and its band lies inside the sparse first pass.
static bool fixed_576(int N, const int* rad, int nrad, int band_lo, int band_hi) {
    return N == 576 && nrad == 3 && rad[0] == 9 && rad[1] == 8 && rad[2] == 8 && band_lo < 64 && band_hi <= 64;
}
constexpr size_t kFixedBandRows = 128;             // filter factors of the band rows (2 kcy + 1 <= 127)
constexpr int kFixedColsT = 4, kFixedRowsT = 4;   // transforms per workgroup

hipError_t launch_fields(const FieldPlan& fp, float* V, float* F, hipStream_t s) {
    const size_t kMaxLds = 160 * 1024;
    const int lc = fields_pick_lg(fp.Nfy, kColsLdsBudget, true);
    const int lr = fields_pick_lg(fp.Nfx, kRowsLdsBudget, false);
    const size_t bc = fields_cols_lds(fp.Nfy, 1 << lc), br = fields_rows_lds(fp.Nfx, 1 << lr);
    if (bc > kMaxLds || br > kMaxLds) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)fields_cols_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)fields_rows_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kMaxLds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    float2* V2 = reinterpret_cast<float2*>(V);
    float2* twx = V2 + (size_t)fp.npairs * fp.H * fp.Mx;   // Nfx twiddles after the intermediate
    static int res_c = 0, res_r = 0;
    static size_t res_c_lds = 0, res_r_lds = 0;
    if (res_c_lds != bc) {
        res_c = resident_workgroups((const void*)fields_cols_kernel, kThreads, bc);
        res_c_lds = bc;
    }
    if (res_r_lds != br) {
        res_r = resident_workgroups((const void*)fields_rows_kernel, kThreads, br);
        res_r_lds = br;
    }
    const int nc = (fp.Mx + (1 << lc) - 1) >> lc, nr = (fp.H + (1 << lr) - 1) >> lr;
    if (fixed_576(fp.Nfy, fp.rad_y, fp.nrad_y, fp.kcy, fp.kcy)) {
        using P = FixedPlan<9, 8, 8, kFixedColsT>;
        const int chunks = (fp.Mx + kFixedColsT - 1) / kFixedColsT;
        hipLaunchKernelGGL((fields_cols_fixed<9, 8, 8, kFixedColsT>), dim3(chunks * fp.npairs), dim3(P::NT),
                           P::lds_bytes + kFixedBandRows * 4, s, fp, V2, twx, chunks);
    } else {
        hipLaunchKernelGGL(fields_cols_kernel, dim3(std::min(nc * fp.npairs, res_c)), dim3(kThreads), bc, s, fp, V2,
                           lc, twx, nc);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (fixed_576(fp.Nfx, fp.rad_x, fp.nrad_x, fp.kcx, fp.Mx - 1 - fp.kcx)) {
        using P = FixedPlan<9, 8, 8, kFixedRowsT>;
        const int chunks = (fp.H + kFixedRowsT - 1) / kFixedRowsT;
        hipLaunchKernelGGL((fields_rows_fixed<9, 8, 8, kFixedRowsT>), dim3((chunks * fp.npairs + 31) & ~31),
                           dim3(P::NT), P::lds_bytes, s, fp, (const float2*)V2, F, chunks);
    } else {
        hipLaunchKernelGGL(fields_rows_kernel, dim3(std::min(nr * fp.npairs, res_r)), dim3(kThreads), br, s, fp,
                           (const float2*)V2, F, lr, (const float2*)twx, nr);
    }
    return hipGetLastError();
}

hipError_t launch_debug_noise(int Nfy, int Nfx, int pair, uint32_t k0, uint32_t k1, uint32_t* raw,
                              float* normals, hipStream_t s) {
    const int n = Nfy * Nfx;
    hipLaunchKernelGGL(debug_noise_kernel, dim3((n + 255) / 256), dim3(256), 0, s, Nfy, Nfx, pair, k0, k1, raw,
                       normals);
    return hipGetLastError();
}

}  // namespace p2s
