// Stage 1 of the hot path: spatially correlated Zernike coefficient planes
// (the per-pixel alpha_j of Sec. 2.2 Eq. 1, correlated in space as Sec. 3.4
// requires), made by colouring seeded white noise with a separable Gaussian
// power spectral density:
//
//   field_p = crop_HxW( IDFT2( sqrt(S_y) sqrt(S_x) DFT2(noise_p) ) ) * sigma_p
//
// Two passes, each a batch of 1-D complex FFTs held in LDS:
//   rows:    Philox noise for two grid rows packed as one complex row
//            (real = row 2q, imag = row 2q+1) -> FFT -> * sqrt(S_x) -> IFFT
//            -> keep the first W columns -> T[p][r][0..W)
//   columns: two columns of T packed as one complex column -> FFT ->
//            * sqrt(S_y) sigma_p -> IFFT -> keep the first H rows -> F[p]
// The filters are real and even, so the packed real and imaginary parts stay
// separate exactly.  FFT: Stockham auto-sort, radix 4/2/3/5 passes, twiddles
// from an FP64-evaluated table in LDS.
#include "internal.hpp"

namespace p2s {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by +i (inv) or -i (forward): the sign of the DFT exponent
__device__ __forceinline__ float2 mul_i(float2 a, float sgn) {   // sgn * i * a
    return make_float2(-sgn * a.y, sgn * a.x);
}

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

// Four normals for cells 4g .. 4g+3 of grid row r of plane p.
__device__ __forceinline__ void noise4(int g, int r, int p, uint32_t k0, uint32_t k1, float z[4],
                                       uint32_t* raw_out = nullptr) {
    uint32_t c0 = (uint32_t)g, c1 = (uint32_t)r, c2 = (uint32_t)p, c3 = 0u;
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    if (raw_out) {
        raw_out[0] = c0;
        raw_out[1] = c1;
        raw_out[2] = c2;
        raw_out[3] = c3;
    }
    const float two24 = 5.9604644775390625e-08f;   // 2^-24
    const float ua0 = (float)((c0 >> 8) + 1u) * two24, ub0 = (float)(c1 >> 8) * two24;
    const float ua1 = (float)((c2 >> 8) + 1u) * two24, ub1 = (float)(c3 >> 8) * two24;
    const float r0 = sqrtf(-2.0f * logf(ua0)), r1 = sqrtf(-2.0f * logf(ua1));
    float s0, co0, s1, co1;
    sincospif(2.0f * ub0, &s0, &co0);
    sincospif(2.0f * ub1, &s1, &co1);
    z[0] = r0 * co0;
    z[1] = r0 * s0;
    z[2] = r1 * co1;
    z[3] = r1 * s1;
}

// One Stockham pass of radix R over `nfft` transforms of length N stored at
// stride ld.  Ns = product of the radices already applied.  tw[q] =
// exp(-2 pi i q / N); sgn = -1 forward, +1 inverse.
template <int R>
__device__ __forceinline__ void stockham_pass(const float2* __restrict__ src, float2* __restrict__ dst,
                                              int N, int ld, int nfft, int Ns, const float2* __restrict__ tw,
                                              float sgn) {
    const int nb = N / R;
    const int step = N / (Ns * R);
    for (int idx = threadIdx.x; idx < nfft * nb; idx += blockDim.x) {
        const int f = idx / nb;
        const int j = idx - f * nb;
        const float2* s = src + f * ld;
        float2* d = dst + f * ld;
        const int k = j % Ns;
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float2 x = s[j + r * nb];
            if (r > 0) {
                float2 w = tw[r * k * step];
                w.y *= -sgn;   // table holds exp(-i..); inverse uses the conjugate
                x = cmul(x, w);
            }
            v[r] = x;
        }
        float2 o[R];
        if constexpr (R == 2) {
            o[0] = make_float2(v[0].x + v[1].x, v[0].y + v[1].y);
            o[1] = make_float2(v[0].x - v[1].x, v[0].y - v[1].y);
        } else if constexpr (R == 4) {
            const float2 a = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
            const float2 b = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
            const float2 c = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
            const float2 dd = mul_i(make_float2(v[1].x - v[3].x, v[1].y - v[3].y), sgn);
            o[0] = make_float2(a.x + c.x, a.y + c.y);
            o[2] = make_float2(a.x - c.x, a.y - c.y);
            o[1] = make_float2(b.x + dd.x, b.y + dd.y);
            o[3] = make_float2(b.x - dd.x, b.y - dd.y);
        } else if constexpr (R == 3) {
            const float s3 = 0.86602540378443864676f;
            const float2 t1 = make_float2(v[1].x + v[2].x, v[1].y + v[2].y);
            const float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
            const float2 t3 = mul_i(make_float2(s3 * (v[1].x - v[2].x), s3 * (v[1].y - v[2].y)), sgn);
            o[0] = make_float2(v[0].x + t1.x, v[0].y + t1.y);
            o[1] = make_float2(t2.x + t3.x, t2.y + t3.y);
            o[2] = make_float2(t2.x - t3.x, t2.y - t3.y);
        } else {   // R == 5
            const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
            const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
            const float2 a1 = make_float2(v[1].x + v[4].x, v[1].y + v[4].y);
            const float2 b1 = make_float2(v[1].x - v[4].x, v[1].y - v[4].y);
            const float2 a2 = make_float2(v[2].x + v[3].x, v[2].y + v[3].y);
            const float2 b2 = make_float2(v[2].x - v[3].x, v[2].y - v[3].y);
            o[0] = make_float2(v[0].x + a1.x + a2.x, v[0].y + a1.y + a2.y);
            const float2 p1 = make_float2(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
            const float2 p2 = make_float2(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
            const float2 q1 = mul_i(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y), sgn);
            const float2 q2 = mul_i(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y), sgn);
            o[1] = make_float2(p1.x + q1.x, p1.y + q1.y);
            o[4] = make_float2(p1.x - q1.x, p1.y - q1.y);
            o[2] = make_float2(p2.x + q2.x, p2.y + q2.y);
            o[3] = make_float2(p2.x - q2.x, p2.y - q2.y);
        }
        const int base = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) d[base + q * Ns] = o[q];
    }
}

// Full transform; returns the buffer holding the result.
__device__ float2* fft_batch(float2* a, float2* b, int N, int ld, int nfft, const int* rad, int nrad,
                             const float2* tw, float sgn) {
    int Ns = 1;
    for (int i = 0; i < nrad; ++i) {
        const int R = rad[i];
        if (R == 4) stockham_pass<4>(a, b, N, ld, nfft, Ns, tw, sgn);
        else if (R == 2) stockham_pass<2>(a, b, N, ld, nfft, Ns, tw, sgn);
        else if (R == 3) stockham_pass<3>(a, b, N, ld, nfft, Ns, tw, sgn);
        else stockham_pass<5>(a, b, N, ld, nfft, Ns, tw, sgn);
        __syncthreads();
        float2* t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

// Twiddle table exp(-2 pi i q / N) (FP64 evaluation) and the real even filter
// h[k] = exp(-pi^2 l^2 f_k^2) * scale, f_k = k/N wrapped to [-1/2, 1/2).
__device__ void fill_tables(float2* tw, float* filt, int N, float corr_len, float scale) {
    const double a = 3.14159265358979323846 * 3.14159265358979323846 * (double)corr_len * (double)corr_len;
    for (int q = threadIdx.x; q < N; q += blockDim.x) {
        double s, c;
        sincospi(-2.0 * (double)q / (double)N, &s, &c);
        tw[q] = make_float2((float)c, (float)s);
        const int kk = (q < (N + 1) / 2) ? q : q - N;
        const double f = (double)kk / (double)N;
        filt[q] = (float)(exp(-a * f * f) * (double)scale);
    }
}

__device__ __forceinline__ int ld_of(int N) { return N | 1; }   // odd stride spreads LDS banks

__global__ void __launch_bounds__(kThreads) fields_rows_kernel(FieldPlan fp, float* __restrict__ T, int fpb) {
    extern __shared__ float2 smem[];
    const int N = fp.Nfx, ld = ld_of(N);
    float2* buf0 = smem;
    float2* buf1 = smem + fpb * ld;
    float2* tw = smem + 2 * fpb * ld;
    float* filt = reinterpret_cast<float*>(tw + N);
    const int plane = blockIdx.y;
    const int pair0 = blockIdx.x * fpb;
    const int npairs = (fp.Nfy + 1) / 2;
    fill_tables(tw, filt, N, fp.corr_len, fp.scale_x);

    const int ng = (N + 3) / 4;
    for (int idx = threadIdx.x; idx < fpb * 2 * ng; idx += blockDim.x) {
        const int f = idx / (2 * ng);
        const int rem = idx - f * 2 * ng;
        const int half = rem / ng;
        const int g = rem - half * ng;
        const int r = 2 * (pair0 + f) + half;
        float z[4] = {0.f, 0.f, 0.f, 0.f};
        if (r < fp.Nfy) noise4(g, r, plane, fp.k0, fp.k1, z);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = 4 * g + e;
            if (c < N) {
                float* dst = reinterpret_cast<float*>(&buf0[f * ld + c]);
                dst[half] = z[e];
            }
        }
    }
    __syncthreads();
    float2* X = fft_batch(buf0, buf1, N, ld, fpb, fp.rad_x, fp.nrad_x, tw, -1.0f);
    float2* Y = (X == buf0) ? buf1 : buf0;
    for (int idx = threadIdx.x; idx < fpb * N; idx += blockDim.x) {
        const int f = idx / N, k = idx - f * N;
        const float h = filt[k];
        float2 v = X[f * ld + k];
        X[f * ld + k] = make_float2(v.x * h, v.y * h);
    }
    __syncthreads();
    X = fft_batch(X, Y, N, ld, fpb, fp.rad_x, fp.nrad_x, tw, 1.0f);
    const int W = fp.W;
    for (int idx = threadIdx.x; idx < fpb * 2 * W; idx += blockDim.x) {
        const int f = idx / (2 * W);
        const int rem = idx - f * 2 * W;
        const int half = rem / W;
        const int c = rem - half * W;
        const int pair = pair0 + f;
        const int r = 2 * pair + half;
        if (pair < npairs && r < fp.Nfy) {
            const float2 v = X[f * ld + c];
            T[((size_t)plane * fp.Nfy + r) * W + c] = half ? v.y : v.x;
        }
    }
}

__global__ void __launch_bounds__(kThreads) fields_cols_kernel(FieldPlan fp, const float* __restrict__ T,
                                                               float* __restrict__ F, int fpb) {
    extern __shared__ float2 smem[];
    const int N = fp.Nfy, ld = ld_of(N);
    float2* buf0 = smem;
    float2* buf1 = smem + fpb * ld;
    float2* tw = smem + 2 * fpb * ld;
    float* filt = reinterpret_cast<float*>(tw + N);
    const int plane = blockIdx.y;
    const int c0 = blockIdx.x * 2 * fpb;
    const int W = fp.W, H = fp.H;
    fill_tables(tw, filt, N, fp.corr_len, fp.scale_y * fp.sigma[plane]);
    const int ncol = 2 * fpb;
    const float* Tp = T + (size_t)plane * N * W;
    for (int idx = threadIdx.x; idx < N * ncol; idx += blockDim.x) {
        const int r = idx / ncol;
        const int j = idx - r * ncol;
        const int c = c0 + j;
        const float v = (c < W) ? Tp[(size_t)r * W + c] : 0.0f;
        float* dst = reinterpret_cast<float*>(&buf0[(j >> 1) * ld + r]);
        dst[j & 1] = v;
    }
    __syncthreads();
    float2* X = fft_batch(buf0, buf1, N, ld, fpb, fp.rad_y, fp.nrad_y, tw, -1.0f);
    float2* Y = (X == buf0) ? buf1 : buf0;
    for (int idx = threadIdx.x; idx < fpb * N; idx += blockDim.x) {
        const int f = idx / N, k = idx - f * N;
        const float h = filt[k];
        float2 v = X[f * ld + k];
        X[f * ld + k] = make_float2(v.x * h, v.y * h);
    }
    __syncthreads();
    X = fft_batch(X, Y, N, ld, fpb, fp.rad_y, fp.nrad_y, tw, 1.0f);
    float* Fp = F + (size_t)plane * H * W;
    for (int idx = threadIdx.x; idx < H * ncol; idx += blockDim.x) {
        const int r = idx / ncol;
        const int j = idx - r * ncol;
        const int c = c0 + j;
        if (c < W) {
            const float2 v = X[(j >> 1) * ld + r];
            Fp[(size_t)r * W + c] = (j & 1) ? v.y : v.x;
        }
    }
}

__global__ void debug_noise_kernel(int Nfy, int Nfx, int plane, uint32_t k0, uint32_t k1, uint32_t* raw,
                                   float* normals) {
    const int ng = (Nfx + 3) / 4;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Nfy * ng) return;
    const int r = idx / ng, g = idx - r * ng;
    float z[4];
    uint32_t o[4];
    noise4(g, r, plane, k0, k1, z, o);
#pragma unroll
    for (int e = 0; e < 4; ++e) raw[(size_t)idx * 4 + e] = o[e];
    if (normals) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (4 * g + e < Nfx) normals[(size_t)r * Nfx + 4 * g + e] = z[e];
    }
}

size_t fft_lds_bytes(int N, int fpb) { return (size_t)(2 * fpb * (N | 1) + N) * 8 + (size_t)N * 4; }

int pick_fpb(int N, size_t budget) {
    int f = 8;
    while (f > 1 && fft_lds_bytes(N, f) > budget) f >>= 1;
    return f;
}

}  // namespace

int factor_radices(int n, int* rad) {
    int k = 0;
    while (n % 4 == 0) { rad[k++] = 4; n /= 4; }
    while (n % 2 == 0) { rad[k++] = 2; n /= 2; }
    while (n % 3 == 0) { rad[k++] = 3; n /= 3; }
    while (n % 5 == 0) { rad[k++] = 5; n /= 5; }
    return n == 1 ? k : 0;
}

hipError_t launch_fields(const FieldPlan& fp, float* T, float* F, hipStream_t s) {
    const size_t kMaxLds = 160 * 1024;
    const int fr = pick_fpb(fp.Nfx, 48 * 1024);
    const int fc = pick_fpb(fp.Nfy, 80 * 1024);
    const size_t lr = fft_lds_bytes(fp.Nfx, fr), lc = fft_lds_bytes(fp.Nfy, fc);
    if (lr > kMaxLds || lc > kMaxLds) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)fields_rows_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)fields_cols_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kMaxLds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int npairs = (fp.Nfy + 1) / 2;
    dim3 gr((npairs + fr - 1) / fr, fp.nplanes);
    hipLaunchKernelGGL(fields_rows_kernel, gr, dim3(kThreads), lr, s, fp, T, fr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 gc((fp.W + 2 * fc - 1) / (2 * fc), fp.nplanes);
    hipLaunchKernelGGL(fields_cols_kernel, gc, dim3(kThreads), lc, s, fp, (const float*)T, F, fc);
    return hipGetLastError();
}

hipError_t launch_debug_noise(int Nfy, int Nfx, int plane, uint32_t k0, uint32_t k1, uint32_t* raw,
                              float* normals, hipStream_t s) {
    const int n = Nfy * ((Nfx + 3) / 4);
    hipLaunchKernelGGL(debug_noise_kernel, dim3((n + 255) / 256), dim3(256), 0, s, Nfy, Nfx, plane, k0, k1,
                       raw, normals);
    return hipGetLastError();
}

}  // namespace p2s
