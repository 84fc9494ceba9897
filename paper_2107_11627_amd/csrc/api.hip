// Host side of libp2s: argument validation, handle creation (basis and
// network packed into MFMA operand layouts), workspace carving and the chain
// of launches behind each public call.  See include/p2s.h for the contract.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

struct p2s_basis_s {
    p2s::Basis b;
};
struct p2s_mlp_s {
    p2s::Mlp m;
};
struct p2s_anchor_s {
    p2s::Anchor a;
};


namespace p2s {
namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return P2S_OK;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(P2S_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// -------------------------------------------------------------- Noll R_Z
// (n+1) Gamma(n - 5/6) / (Gamma(17/6)^2 Gamma(n + 23/6)) for radial order n.
double noll_shape(int n) {
    return (n + 1) * std::exp(std::lgamma(n - 5.0 / 6.0) - 2.0 * std::lgamma(17.0 / 6.0) - std::lgamma(n + 23.0 / 6.0));
}

// Constant fixing sum_{j>=2} V_j to Noll's piston-removed variance 1.0299.
double noll_constant() {
    static const double kc = [] {
        double s = 0.0;
        for (int n = 199999; n >= 1; --n) s += (n + 1) * noll_shape(n);   // small terms first
        return 1.0299 / s;
    }();
    return kc;
}

int radial_order(int j) {
    int n = 0;
    while ((n + 1) * (n + 2) / 2 < j) ++n;
    return n;
}

double noll_var(int j) { return noll_constant() * noll_shape(radial_order(j)); }

// ---------------------------------------------------------------- fields
bool smooth5(int n) {
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

int grid_of(int n, float corr_len) {
    long v = (long)n + (long)std::ceil(4.0 * (double)corr_len);
    while (!smooth5((int)v)) ++v;
    return (int)v;
}

struct Params {
    float corr_len = 16.0f;
    float q = 2.0f;
};

int read_params(const p2s_params* p, Params* out) {
    Params r;
    if (p) {
        r.corr_len = p->corr_len_px;
        r.q = p->q_sampling;
    }
    if (!(std::isfinite(r.corr_len) && r.corr_len > 0.0f && r.corr_len <= 1024.0f))
        return fail(P2S_EINVAL, "corr_len_px must be in (0, 1024], got %g", (double)r.corr_len);
    if (!(std::isfinite(r.q) && r.q > 0.0f && r.q <= 64.0f))
        return fail(P2S_EINVAL, "q_sampling must be in (0, 64], got %g", (double)r.q);
    *out = r;
    return P2S_OK;
}

// Largest FFT length the LDS of one workgroup holds (one transform, ping-pong
// buffers, twiddles and filter): 16 (N|1) + 12 N bytes <= 160 KiB.
constexpr int kMaxFftLen = 5800;

// Band half-width: the largest k <= N/2 whose 1-D filter factor
// exp(-pi^2 l^2 (k/N)^2) is still >= 1e-9 of its peak.
int band_half(int N, double corr_len) {
    const double a = M_PI * M_PI * corr_len * corr_len;
    int kc = 0;
    for (int k = 1; k <= N / 2; ++k) {
        const double f = (double)k / N;
        if (std::exp(-a * f * f) >= 1e-9) kc = k;
        else break;
    }
    return kc;
}

int band_size(int N, double corr_len) { return std::min(N, 2 * band_half(N, corr_len) + 1); }

// Intermediate of the field generator: complex [pairs][band columns][H],
// followed by the Nfx twiddle factors of the row transforms.
size_t fields_ws(int H, int W, int nz, const Params& pr) {
    const int Nfx = grid_of(W, pr.corr_len);
    const int Mx = band_size(Nfx, pr.corr_len);
    return align256(((size_t)((nz + 1) / 2) * H * Mx + Nfx) * 8);
}

int check_frame(int C, int H, int W) {
    if (C < 1 || C > P2S_MAX_CHANNELS) return fail(P2S_EINVAL, "C must be in [1, %d], got %d", P2S_MAX_CHANNELS, C);
    if (H < 1 || W < 1 || H > P2S_MAX_SIDE || W > P2S_MAX_SIDE)
        return fail(P2S_EINVAL, "H, W must be in [1, %d], got %d x %d", P2S_MAX_SIDE, H, W);
    return P2S_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + nb && pb < pa + na;
}

// Plan of the field generator for one frame (validated; no device work).
int build_field_plan(int H, int W, double d, int nz, uint64_t seed, const Params& pr, FieldPlan* out) {
    if (H < 1 || W < 1 || H > P2S_MAX_SIDE || W > P2S_MAX_SIDE)
        return fail(P2S_EINVAL, "H, W must be in [1, %d], got %d x %d", P2S_MAX_SIDE, H, W);
    if (nz < 1 || nz > P2S_MAX_ZERNIKE) return fail(P2S_EINVAL, "n_zernike must be in [1, %d], got %d", P2S_MAX_ZERNIKE, nz);
    if (!(std::isfinite(d) && d >= 0.0)) return fail(P2S_EINVAL, "D/r0 must be finite and >= 0, got %g", d);
    FieldPlan fp{};
    fp.H = H;
    fp.W = W;
    fp.Nfy = grid_of(H, pr.corr_len);
    fp.Nfx = grid_of(W, pr.corr_len);
    if (fp.Nfy > kMaxFftLen || fp.Nfx > kMaxFftLen)
        return fail(P2S_EUNSUPPORTED, "noise grid %d x %d exceeds the single-workgroup FFT limit %d", fp.Nfy, fp.Nfx,
                    kMaxFftLen);
    fp.nrad_x = factor_radices(fp.Nfx, fp.rad_x);
    fp.nrad_y = factor_radices(fp.Nfy, fp.rad_y);
    if (!fp.nrad_x || !fp.nrad_y) return fail(P2S_EINVAL, "internal: grid not 5-smooth");
    fp.nplanes = nz;
    fp.npairs = (nz + 1) / 2;
    fp.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    fp.k1 = (uint32_t)(seed >> 32);
    fp.corr_len = pr.corr_len;
    fp.kcx = band_half(fp.Nfx, pr.corr_len);
    fp.kcy = band_half(fp.Nfy, pr.corr_len);
    fp.Mx = std::min(fp.Nfx, 2 * fp.kcx + 1);
    fp.My = std::min(fp.Nfy, 2 * fp.kcy + 1);
    const double a = 2.0 * M_PI * M_PI * (double)pr.corr_len * (double)pr.corr_len;
    auto mean_s = [&](int N) {
        double m = 0.0;
        for (int k = 0; k < N; ++k) {
            const int kk = (k < (N + 1) / 2) ? k : k - N;
            const double f = (double)kk / N;
            m += std::exp(-a * f * f);
        }
        return m / N;
    };
    fp.norm = (float)(1.0 / (std::sqrt(mean_s(fp.Nfx) * mean_s(fp.Nfy)) * std::sqrt((double)fp.Nfx * fp.Nfy)));
    const double d53 = std::pow(d, 5.0 / 3.0);
    for (int p = 0; p < nz; ++p) fp.sigma[p] = (float)std::sqrt(noll_var(p + 2) * d53);
    *out = fp;
    return P2S_OK;
}

int make_fields_impl(int H, int W, double d, int nz, uint64_t seed, const Params& pr, float* F, void* ws,
                     size_t ws_bytes, hipStream_t s) {
    FieldPlan fp;
    int rc = build_field_plan(H, W, d, nz, seed, pr, &fp);
    if (rc) return rc;
    if (!F) return fail(P2S_EINVAL, "fields is NULL");
    if (!ws) return fail(P2S_EINVAL, "workspace is NULL");
    const size_t need = fields_ws(H, W, nz, pr);
    if (ws_bytes < need) return fail(P2S_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    hipError_t e = launch_fields(fp, (float*)ws, F, s);
    if (e != hipSuccess) return hip_fail(e, "field kernels");
    return P2S_OK;
}

int anchor_fields_impl(const Anchor& an, int H, int W, double d, uint64_t seed, float* F, void* ws,
                       size_t ws_bytes, hipStream_t s) {
    if (H < 1 || W < 1 || H > P2S_MAX_SIDE || W > P2S_MAX_SIDE)
        return fail(P2S_EINVAL, "H, W must be in [1, %d], got %d x %d", P2S_MAX_SIDE, H, W);
    if (!(std::isfinite(d) && d >= 0.0)) return fail(P2S_EINVAL, "D/r0 must be finite and >= 0");
    if (!F) return fail(P2S_EINVAL, "fields is NULL");
    if (!ws) return fail(P2S_EINVAL, "workspace is NULL");
    const size_t need = anchor_ws_bytes(an);
    if (ws_bytes < need) return fail(P2S_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    if (overlap(ws, need, F, (size_t)an.n * H * W * 4)) return fail(P2S_EINVAL, "workspace and fields overlap");
    hipError_t e = launch_anchor_fields(an, H, W, d, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), F, ws, s);
    if (e != hipSuccess) return hip_fail(e, "anchor field kernels");
    return P2S_OK;
}

int pack_anchor(int G, int n, const double* Ls, const double* Lz, Anchor* out) {
    Anchor an;
    an.G = G;
    an.n = n;
    an.Gp = (G * G + 31) / 32 * 32;
    an.ld = an.Gp + 32;
    an.nct = (n + 15) / 16;
    an.Ls = nullptr;
    an.Lz = nullptr;
    const size_t G2 = (size_t)G * G, Gp = an.Gp, ld = an.ld;
    std::vector<float> hs(Gp * ld, 0.0f), hz((size_t)n * n, 0.0f);
    for (size_t r = 0; r < G2; ++r)
        for (size_t c = 0; c <= r; ++c) hs[r * ld + c] = (float)Ls[r * G2 + c];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c <= r; ++c) hz[(size_t)r * n + c] = (float)Lz[(size_t)r * n + c];
    hipError_t e = hipMalloc((void**)&an.Ls, hs.size() * 4);
    if (e != hipSuccess) return fail(P2S_ENOMEM, "device allocation of %zu bytes failed", hs.size() * 4);
    e = hipMalloc((void**)&an.Lz, hz.size() * 4);
    if (e != hipSuccess) {
        (void)hipFree(an.Ls);
        return fail(P2S_ENOMEM, "device allocation failed");
    }
    e = hipMemcpy(an.Ls, hs.data(), hs.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(an.Lz, hz.data(), hz.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(an.Ls);
        (void)hipFree(an.Lz);
        return hip_fail(e, "upload of the anchor factors");
    }
    *out = an;
    return P2S_OK;
}

// ----------------------------------------------------------------- basis
int pack_basis(const double* hb, int K, int P, Basis* B) {
    const int R = (P - 1) / 2;
    const int U = P * P;
    B->K = K;
    B->P = P;
    B->R = R;
    B->nmb = (K + 15) / 16;
    B->t4 = (U + 3) / 4;
    auto tap = [&](int k, int dy, int dx) -> double {   // correlation-order tap
        if (k >= K || dy < -R || dy > R || dx < -R || dx > R) return 0.0;
        return hb[((size_t)k * P + (R - dy)) * P + (R - dx)];
    };
    std::vector<float> f32((size_t)(B->t4 + 2) * B->nmb * 64, 0.0f);   // two zero steps: prefetch slack
    for (int t = 0; t < B->t4; ++t)
        for (int mb = 0; mb < B->nmb; ++mb)
            for (int L = 0; L < 64; ++L) {
                const int u = 4 * t + L / 16, k = 16 * mb + L % 16;
                double v = 0.0;
                if (u < U) v = tap(k, u / P - R, u % P - R);
                f32[((size_t)t * B->nmb + mb) * 64 + L] = (float)v;
            }
    B->bf16_ok = (P % 8 == 1 && P >= 9);
    std::vector<uint16_t> h16;
    std::vector<uint8_t> h8;
    std::vector<int> sc;
    if (B->bf16_ok) {
        const int A8 = P / 8, NROW = P * A8, NCOL = (P + 7) / 8;
        // tap of chunk ch, element e (row chunks, then the last tap column, then zero)
        auto chunk_tap = [&](int k, int ch, int e) -> double {
            if (ch < NROW) return tap(k, ch / A8 - R, (ch % A8) * 8 - R + e);
            if (ch < NROW + NCOL) return tap(k, -R + 8 * (ch - NROW) + e, R);
            return 0.0;
        };
        B->t32 = (NROW + NCOL + 3) / 4;
        h16.assign((size_t)(B->t32 + 2) * B->nmb * 64 * 8, 0);   // two zero steps: prefetch slack
        for (int t = 0; t < B->t32; ++t)
            for (int mb = 0; mb < B->nmb; ++mb)
                for (int L = 0; L < 64; ++L)
                    for (int e = 0; e < 8; ++e)
                        h16[(((size_t)t * B->nmb + mb) * 64 + L) * 8 + e] =
                            f32_to_bf16_rne((float)chunk_tap(16 * mb + L % 16, 4 * t + L / 16, e));
        // FP8: per-basis power-of-two scale from the float32 taps
        sc.assign((size_t)16 * B->nmb, 127);
        std::vector<int> ex(K, 0);
        for (int k = 0; k < K; ++k) {
            float amax = 0.0f;
            for (int u = 0; u < U; ++u) amax = std::max(amax, std::fabs((float)hb[(size_t)k * U + u]));
            ex[k] = e4m3_scale_exponent(amax);
            sc[k] = 127 - ex[k];
        }
        B->t128 = (NROW + NCOL + 15) / 16;
        h8.assign((size_t)(B->t128 + 2) * B->nmb * 64 * 32, 0);  // two zero steps: prefetch slack
        for (int t = 0; t < B->t128; ++t)
            for (int mb = 0; mb < B->nmb; ++mb)
                for (int L = 0; L < 64; ++L) {
                    const int k = 16 * mb + L % 16;
                    for (int j = 0; j < 4; ++j)
                        for (int e = 0; e < 8; ++e) {
                            const float v = (float)chunk_tap(k, 16 * t + 4 * (L / 16) + j, e);
                            h8[(((size_t)t * B->nmb + mb) * 64 + L) * 32 + 8 * j + e] =
                                k < K ? f32_to_e4m3_rne(std::ldexp(v, ex[k])) : 0;
                        }
                }
    }
    B->f32 = nullptr;
    B->bf16 = nullptr;
    B->fp8 = nullptr;
    B->fp8_scale = nullptr;
    auto release = [&] {
        (void)hipFree(B->f32);
        (void)hipFree(B->bf16);
        (void)hipFree(B->fp8);
        (void)hipFree(B->fp8_scale);
    };
    auto upload = [&](void** dst, const void* src, size_t bytes) -> int {
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) {
            *dst = nullptr;
            release();
            return fail(P2S_ENOMEM, "hipMalloc basis: %s", hipGetErrorString(e));
        }
        e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            release();
            return hip_fail(e, "upload basis");
        }
        return P2S_OK;
    };
    int rc = upload((void**)&B->f32, f32.data(), f32.size() * sizeof(float));
    if (rc) return rc;
    if (B->bf16_ok) {
        if ((rc = upload((void**)&B->bf16, h16.data(), h16.size() * sizeof(uint16_t))) ||
            (rc = upload((void**)&B->fp8, h8.data(), h8.size())) ||
            (rc = upload((void**)&B->fp8_scale, sc.data(), sc.size() * sizeof(int))))
            return rc;
    }
    return P2S_OK;
}

// ------------------------------------------------------------------- mlp
int pack_mlp(int L, const int* dims, const float* const* W, const float* const* b, Mlp* M) {
    M->L = L;
    for (int i = 0; i <= L; ++i) M->dims[i] = dims[i];
    int mb = 1;
    for (int l = 1; l <= L; ++l) mb = std::max(mb, (dims[l] + 15) / 16);
    M->mb = mb;
    const int mbe = (mb + 1) & ~1;
    std::vector<float> w32, bias;
    std::vector<uint16_t> w16;
    for (int l = 0; l < L; ++l) {
        const int in = dims[l], out = dims[l + 1];
        const float* Wl = W[l];
        auto wat = [&](int r, int f) -> float { return (r < out && f < in) ? Wl[(size_t)r * in + f] : 0.0f; };
        // FP32
        const int nkc = (l == 0) ? (in + 3) / 4 : 4 * mb;
        M->nkc32[l] = nkc;
        M->off32[l] = w32.size() * sizeof(float);
        for (int ob = 0; ob < mb; ++ob)
            for (int kc = 0; kc < nkc; ++kc)
                for (int Ln = 0; Ln < 64; ++Ln) {
                    const int g = Ln / 16, r = 16 * ob + Ln % 16;
                    const int f = (l == 0) ? 4 * kc + g : 16 * (kc / 4) + 4 * g + kc % 4;
                    w32.push_back(wat(r, f));
                }
        // BF16
        const int nk16 = (l == 0) ? 2 : mbe / 2;
        M->nkc16[l] = (l == 0) ? (in + 31) / 32 : nk16;
        M->off16[l] = w16.size() * sizeof(uint16_t);
        for (int ob = 0; ob < mb; ++ob)
            for (int kc = 0; kc < nk16; ++kc)
                for (int Ln = 0; Ln < 64; ++Ln)
                    for (int e = 0; e < 8; ++e) {
                        const int g = Ln / 16, r = 16 * ob + Ln % 16;
                        const int f = (l == 0) ? 32 * kc + 8 * g + e : 16 * (2 * kc + e / 4) + 4 * g + e % 4;
                        w16.push_back(f32_to_bf16_rne(wat(r, f)));
                    }
        M->boff[l] = (int)bias.size();
        for (int r = 0; r < 16 * mb; ++r) bias.push_back((b && b[l] && r < out) ? b[l][r] : 0.0f);
    }
    M->bytes32 = w32.size() * sizeof(float);
    M->bytes16 = w16.size() * sizeof(uint16_t);
    M->w32 = nullptr;
    M->w16 = nullptr;
    M->bias = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&M->w32, M->bytes32)) != hipSuccess || (e = hipMalloc(&M->w16, M->bytes16)) != hipSuccess ||
        (e = hipMalloc(&M->bias, bias.size() * sizeof(float))) != hipSuccess) {
        (void)hipFree(M->w32);
        (void)hipFree(M->w16);
        (void)hipFree(M->bias);
        return fail(P2S_ENOMEM, "hipMalloc network: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(M->w32, w32.data(), M->bytes32, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(M->w16, w16.data(), M->bytes16, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(M->bias, bias.data(), bias.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(M->w32);
        (void)hipFree(M->w16);
        (void)hipFree(M->bias);
        return hip_fail(e, "upload network");
    }
    return P2S_OK;
}

int check_prec(p2s_precision prec) {
    if (prec == P2S_FP32 || prec == P2S_BF16 || prec == P2S_FP8E4M3) return P2S_OK;
    return fail(P2S_EINVAL, "unknown precision %d", (int)prec);
}

int mlp_impl(const Mlp& m, const float* F, int nz, int H, int W, p2s_precision prec, float* w, hipStream_t s) {
    if (H < 1 || W < 1 || H > P2S_MAX_SIDE || W > P2S_MAX_SIDE)
        return fail(P2S_EINVAL, "H, W must be in [1, %d], got %d x %d", P2S_MAX_SIDE, H, W);
    if (nz - 2 != m.dims[0])
        return fail(P2S_EINVAL, "n_zernike - 2 = %d does not match the network input width %d", nz - 2, m.dims[0]);
    if (!F || !w) return fail(P2S_EINVAL, "fields or w is NULL");
    int rc = check_prec(prec);
    if (rc) return rc;
    const size_t wbytes = prec == P2S_FP32 ? m.bytes32 : network_lds_bytes(m);
    if (wbytes > kMlpLdsBytes)
        return fail(P2S_EUNSUPPORTED, "packed network weights (%zu bytes) exceed the %zu-byte LDS of one workgroup "
                    "in this precision", wbytes, kMlpLdsBytes);
    const size_t HW = (size_t)H * W;
    if (overlap(F, (size_t)nz * HW * 4, w, HW * m.dims[m.L] * 4)) return fail(P2S_EINVAL, "fields and w overlap");
    // the kernel reads planes 2.. : pass a pointer to plane 2
    hipError_t e = launch_mlp(m, F + 2 * HW, H, W, prec, w, s);
    if (e != hipSuccess) return hip_fail(e, "network kernel");
    return P2S_OK;
}

int blur_impl(const float* img, int C, int H, int W, const Basis& b, const float* w, p2s_precision prec, float* out,
              hipStream_t s) {
    int rc = check_frame(C, H, W);
    if (rc) return rc;
    rc = check_prec(prec);
    if (rc) return rc;
    if (!img || !w || !out) return fail(P2S_EINVAL, "image, w or out is NULL");
    const size_t n = (size_t)C * H * W * 4;
    if (overlap(img, n, out, n)) return fail(P2S_EINVAL, "image and out overlap");
    if (overlap(w, (size_t)H * W * b.K * 4, out, n)) return fail(P2S_EINVAL, "w and out overlap");
    if (prec != P2S_FP32 && !b.bf16_ok)
        return fail(P2S_EUNSUPPORTED, "BF16 and FP8 blur need a PSF side P = 8a + 1 (9, 17, 25, 33); got %d", b.P);
    hipError_t e = launch_blur(b, img, C, H, W, w, prec, out, s);
    if (e != hipSuccess) return hip_fail(e, "blur kernel");
    return P2S_OK;
}

int warp_impl(const float* in, int C, int H, int W, const float* tilt, const Params& pr, float* out, hipStream_t s) {
    int rc = check_frame(C, H, W);
    if (rc) return rc;
    if (!in || !tilt || !out) return fail(P2S_EINVAL, "in, tilt or out is NULL");
    const size_t n = (size_t)C * H * W * 4;
    if (overlap(in, n, out, n)) return fail(P2S_EINVAL, "in and out overlap");
    if (overlap(tilt, (size_t)2 * H * W * 4, out, n)) return fail(P2S_EINVAL, "tilt and out overlap");
    const double scale = 2.0 * (double)pr.q / M_PI;
    hipError_t e = launch_warp(in, C, H, W, tilt, scale, out, s);
    if (e != hipSuccess) return hip_fail(e, "warp kernel");
    return P2S_OK;
}

struct SimLayout {
    size_t fields, region2, blurred, total;
};

// with_w: the second region also holds the network output w (the path that
// runs the network and the blur as two kernels); without it, only the field
// generator's intermediate.
SimLayout sim_layout_fws(int C, int H, int W, int nz, int K, size_t fws, bool with_w) {
    SimLayout L;
    const size_t HW = (size_t)H * W;
    L.fields = 0;
    const size_t fb = align256((size_t)nz * HW * 4);
    const size_t r2 = with_w ? std::max(align256(fws), align256(HW * K * 4)) : align256(fws);
    L.region2 = fb;
    L.blurred = fb + r2;
    L.total = L.blurred + align256((size_t)C * HW * 4);
    return L;
}

SimLayout sim_layout(int C, int H, int W, int nz, int K, const Params& pr, bool with_w = true) {
    return sim_layout_fws(C, H, W, nz, K, fields_ws(H, W, nz, pr), with_w);
}

// ---------------------------------------------------------------- batches
// Workspace of a batch: the device plan (frame table, then the per-stage item
// prefix sums), then every frame's fields | field intermediate or weights |
// blurred image, as in a single frame.
struct BatchLayout {
    size_t table, first, frames0, total;
    std::vector<size_t> frame_off;
};

int batch_layout(const p2s_frame* fr, int n, int nz, int K, const Params& pr, BatchLayout* L) {
    L->table = 0;
    L->first = align256((size_t)n * sizeof(FrameDesc));
    L->frames0 = L->first + align256((size_t)ST_N * (n + 1) * sizeof(int));
    L->frame_off.resize(n);
    size_t off = L->frames0;
    for (int i = 0; i < n; ++i) {
        int rc = check_frame(fr[i].C, fr[i].H, fr[i].W);
        if (rc) return fail(rc, "frame %d: %s", i, g_err.c_str());
        L->frame_off[i] = off;
        off += sim_layout(fr[i].C, fr[i].H, fr[i].W, nz, K, pr).total;
    }
    L->total = n ? off : 0;
    return P2S_OK;
}

struct BatchHost {
    int n = 0;
    p2s_precision prec = P2S_FP32;
    double scale = 0.0;
    const Basis* basis = nullptr;
    const Mlp* mlp = nullptr;
    void* pinned = nullptr;         // host copy of the device plan
    size_t plan_bytes = 0;
    void* plan_dev = nullptr;       // start of the workspace
    hipEvent_t uploaded = nullptr;  // recorded after the last upload
    bool upload_pending = false;
    bool fused = false;             // network evaluated inside the blur kernel
    BatchLaunch bl{};
};

void batch_free(BatchHost* h) {
    if (h->uploaded) {
        if (h->upload_pending) (void)hipEventSynchronize(h->uploaded);
        (void)hipEventDestroy(h->uploaded);
    }
    if (h->pinned) (void)hipHostFree(h->pinned);
    delete h;
}

int batch_create(const p2s_frame* frames, int n, int nz, const Basis& B, const Mlp& M, p2s_precision prec,
                 const Params& pr, const p2s_batch_options* opt, void* ws, size_t ws_bytes, BatchHost** out) {
    if (n < 0) return fail(P2S_EINVAL, "n must be >= 0, got %d", n);
    if (n > 0 && !frames) return fail(P2S_EINVAL, "frames is NULL");
    int rc = check_prec(prec);
    if (rc) return rc;
    if (nz < 3 || nz > P2S_MAX_ZERNIKE) return fail(P2S_EINVAL, "n_zernike must be in [3, %d], got %d", P2S_MAX_ZERNIKE, nz);
    if (M.dims[0] != nz - 2)
        return fail(P2S_EINVAL, "n_zernike - 2 = %d does not match the network input width %d", nz - 2, M.dims[0]);
    if (M.dims[M.L] != B.K)
        return fail(P2S_EINVAL, "network output width %d does not match the basis size K = %d", M.dims[M.L], B.K);
    if (prec != P2S_FP32 && !B.bf16_ok)
        return fail(P2S_EUNSUPPORTED, "BF16 and FP8 blur need a PSF side P = 8a + 1 (9, 17, 25, 33); got %d", B.P);
    const size_t wbytes = prec == P2S_FP32 ? M.bytes32 : network_lds_bytes(M);
    if (wbytes > kMlpLdsBytes)
        return fail(P2S_EUNSUPPORTED, "packed network weights (%zu bytes) exceed the %zu-byte LDS of one workgroup "
                    "in this precision", wbytes, kMlpLdsBytes);
    int rows = 16, persistent = 1;
    if (opt) {
        if (opt->blur_tile_rows != 16 && opt->blur_tile_rows != 8)
            return fail(P2S_EINVAL, "blur_tile_rows must be 16 or 8, got %d", opt->blur_tile_rows);
        if (opt->persistent != 0 && opt->persistent != 1)
            return fail(P2S_EINVAL, "persistent must be 0 or 1, got %d", opt->persistent);
        rows = opt->blur_tile_rows;
        persistent = opt->persistent;
    }
    // The network runs inside the blur unless the caller chose another tile height.
    const bool fused = blur_mlp_supported(B, M, prec) && rows == 16;
    rows = fused ? blur_mlp_tile_rows(prec, B.nmb) : blur_tile_rows(prec, B.nmb, rows);
    BatchLayout L;
    rc = batch_layout(frames, n, nz, B.K, pr, &L);
    if (rc) return rc;
    if (n > 0 && !ws) return fail(P2S_EINVAL, "workspace is NULL");
    if (ws_bytes < L.total) return fail(P2S_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    // Per-frame checks and descriptors.
    std::vector<FrameDesc> desc(n);
    std::vector<int> first((size_t)ST_N * (n + 1), 0);
    std::vector<std::pair<const char*, const char*>> outs(n);
    size_t lds_cols = 0, lds_rows = 0;
    long long tot[ST_N] = {0, 0, 0, 0, 0};
    char* base = (char*)ws;
    for (int i = 0; i < n; ++i) {
        const p2s_frame& f = frames[i];
        FieldPlan fp;
        rc = build_field_plan(f.H, f.W, f.D_over_r0, nz, f.seed, pr, &fp);
        if (rc) return fail(rc, "frame %d: %s", i, g_err.c_str());
        if (!f.image || !f.out) return fail(P2S_EINVAL, "frame %d: image or out is NULL", i);
        const size_t HW = (size_t)f.H * f.W, nb = (size_t)f.C * HW * 4;
        if (overlap(ws, L.total, f.image, nb) || overlap(ws, L.total, f.out, nb))
            return fail(P2S_EINVAL, "frame %d: workspace overlaps image or out", i);
        outs[i] = {(const char*)f.out, (const char*)f.out + nb};
        const SimLayout S = sim_layout(f.C, f.H, f.W, nz, B.K, pr);
        FrameDesc& d = desc[i];
        d.image = f.image;
        d.out = f.out;
        char* fb = base + L.frame_off[i];
        d.fields = (float*)(fb + S.fields);
        d.w = (float*)(fb + S.region2);
        d.blurred = (float*)(fb + S.blurred);
        d.V = (float2*)(fb + S.region2);
        d.twx = d.V + (size_t)fp.npairs * f.H * fp.Mx;
        d.C = f.C;
        d.H = f.H;
        d.W = f.W;
        d.tiles_x = (f.W + 31) / 32;
        d.tiles_y = (f.H + rows - 1) / rows;
        d.lg_cpb = fields_pick_lg(fp.Nfy, kColsLdsBudget, true);
        d.lg_rpb = fields_pick_lg(fp.Nfx, kRowsLdsBudget, false);
        d.ncol_chunks = (fp.Mx + (1 << d.lg_cpb) - 1) >> d.lg_cpb;
        d.nrow_chunks = (f.H + (1 << d.lg_rpb) - 1) >> d.lg_rpb;
        d.mlp_groups = (int)((HW + mlp_pixels_per_group() - 1) / mlp_pixels_per_group());
        d.warp_tiles_x = (f.W + 63) / 64;
        d.warp_tiles = d.warp_tiles_x * ((f.H + 3) / 4);
        d.fp = fp;
        lds_cols = std::max(lds_cols, fields_cols_lds(fp.Nfy, 1 << d.lg_cpb));
        lds_rows = std::max(lds_rows, fields_rows_lds(fp.Nfx, 1 << d.lg_rpb));
        const long long items[ST_N] = {(long long)fp.npairs * d.ncol_chunks, (long long)fp.npairs * d.nrow_chunks,
                                       d.mlp_groups, (long long)(fused ? 1 : f.C) * d.tiles_x * d.tiles_y,
                                       d.warp_tiles};   // a fused item covers every channel of its tile
        for (int st = 0; st < ST_N; ++st) {
            tot[st] += items[st];
            if (tot[st] > std::numeric_limits<int>::max()) return fail(P2S_EINVAL, "batch too large");
            first[(size_t)st * (n + 1) + i + 1] = (int)tot[st];
        }
    }
    std::sort(outs.begin(), outs.end());
    for (int i = 1; i < n; ++i)
        if (outs[i].first < outs[i - 1].second) return fail(P2S_EINVAL, "output buffers of two frames overlap");
    if (lds_cols > kMlpLdsBytes || lds_rows > kMlpLdsBytes)
        return fail(P2S_EUNSUPPORTED, "field transforms need %zu / %zu bytes of LDS", lds_cols, lds_rows);
    auto* h = new (std::nothrow) BatchHost();
    if (!h) return fail(P2S_ENOMEM, "host allocation failed");
    h->n = n;
    h->prec = prec;
    h->scale = 2.0 * (double)pr.q / M_PI;
    h->basis = &B;
    h->mlp = &M;
    h->plan_bytes = L.frames0;
    h->plan_dev = ws;
    BatchLaunch& bl = h->bl;
    bl.frames = (const FrameDesc*)(base + L.table);
    bl.first = (const int*)(base + L.first);
    bl.n = n;
    bl.blur_rows = rows;
    bl.lds[ST_COLS] = lds_cols;
    bl.lds[ST_ROWS] = lds_rows;
    for (int st = 0; st < ST_N; ++st) bl.items[st] = (int)tot[st];
    h->fused = fused;
    if (n > 0) {
        const int res[ST_N] = {fields_batch_resident(true, lds_cols), fields_batch_resident(false, lds_rows),
                               mlp_batch_resident(M, prec),
                               h->fused ? blur_mlp_batch_resident(B, M, prec) : blur_batch_resident(B, prec, rows),
                               warp_batch_resident()};
        for (int st = 0; st < ST_N; ++st) bl.grid[st] = persistent ? std::min(bl.items[st], res[st]) : bl.items[st];
        hipError_t e = hipHostMalloc(&h->pinned, h->plan_bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            h->pinned = nullptr;
            batch_free(h);
            return fail(P2S_ENOMEM, "pinned plan buffer: %s", hipGetErrorString(e));
        }
        std::memset(h->pinned, 0, h->plan_bytes);
        std::memcpy((char*)h->pinned + L.table, desc.data(), (size_t)n * sizeof(FrameDesc));
        std::memcpy((char*)h->pinned + L.first, first.data(), first.size() * sizeof(int));
        e = hipEventCreateWithFlags(&h->uploaded, hipEventDisableTiming);
        if (e != hipSuccess) {
            h->uploaded = nullptr;
            batch_free(h);
            return hip_fail(e, "event");
        }
    }
    *out = h;
    return P2S_OK;
}

int batch_upload(BatchHost* h, hipStream_t s) {
    if (h->n == 0) return P2S_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return hip_fail(e, "stream query");
    if (cs != hipStreamCaptureStatusNone)
        return fail(P2S_EUNSUPPORTED, "upload the plan outside stream capture; capture p2s_batch_launch only");
    e = hipMemcpyAsync(h->plan_dev, h->pinned, h->plan_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "plan upload");
    e = hipEventRecord(h->uploaded, s);
    if (e != hipSuccess) return hip_fail(e, "event record");
    h->upload_pending = true;
    return P2S_OK;
}

int batch_launch(const BatchHost* h, hipStream_t s) {
    if (h->n == 0) return P2S_OK;
    hipError_t e = launch_fields_batch(h->bl, s);
    if (e != hipSuccess) return hip_fail(e, "batched field kernels");
    if (h->fused) {
        e = launch_blur_mlp_batch(*h->basis, *h->mlp, h->bl, h->prec, s);
        if (e != hipSuccess) return hip_fail(e, "batched fused network and blur kernel");
    } else {
        e = launch_mlp_batch(*h->mlp, h->bl, h->prec, s);
        if (e != hipSuccess) return hip_fail(e, "batched network kernel");
        e = launch_blur_batch(*h->basis, h->bl, h->prec, s);
        if (e != hipSuccess) return hip_fail(e, "batched blur kernel");
    }
    e = launch_warp_batch(h->bl, h->scale, s);
    if (e != hipSuccess) return hip_fail(e, "batched warp kernel");
    return P2S_OK;
}

}  // namespace

uint8_t f32_to_e4m3_rne(float x) {
    const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
    double a = std::fabs((double)x);
    if (std::isnan(a)) return 0x7F;
    if (a > 448.0) a = 448.0;
    if (a < 0.015625) {                                   // below 2^-6: subnormal steps of 2^-9
        const int m = (int)std::nearbyint(a * 512.0);     // ties to even (default rounding mode)
        return (uint8_t)(sign | (m == 8 ? 0x08 : m));
    }
    int e2;
    std::frexp(a, &e2);                                   // a = f 2^e2, f in [0.5, 1)
    int E = e2 - 1;                                       // a in [2^E, 2^(E+1))
    int m = (int)std::nearbyint((std::ldexp(a, -E) - 1.0) * 8.0);
    if (m == 8) {
        m = 0;
        ++E;
    }
    return (uint8_t)(sign | ((E + 7) << 3) | m);
}

int e4m3_scale_exponent(float amax) {
    if (!(amax > 0.0f)) return 0;
    int E;
    const double f = std::frexp((double)amax, &E);        // amax = f 2^E, 448 = 0.875 2^9
    const int e = f <= 0.875 ? 9 - E : 8 - E;
    return std::min(127, std::max(-127, e));
}

uint16_t f32_to_bf16_rne(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace p2s

namespace p2s {
namespace {

// Intermediates of the allocation-free entry point: a file-scope device array
// (one copy per GPU, allocated when the code object loads and held until the
// process ends).  In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress, once per device, with that device
// current.
constexpr size_t kScratchBytes = P2S_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

int scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(P2S_EUNSUPPORTED, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress of the device scratch");
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return P2S_OK;
}

}  // namespace
}  // namespace p2s

namespace p2s {
namespace {

// One frame through the four stages on stream s.  ws == nullptr: the
// intermediates go to the device scratch array (sized for the path that runs,
// EINVAL when it is too small); otherwise to the caller's workspace, which
// must hold p2s_workspace_bytes.
int simulate_impl(const float* image, int C, int H, int W, double D_over_r0, int n_zernike, p2s_basis_t basis,
                  p2s_mlp_t mlp, uint64_t seed, p2s_precision precision, const p2s_params* params, float* out,
                  void* ws, size_t ws_bytes, bool use_scratch, hipStream_t s, const Anchor* anc = nullptr) {
    Params pr;
    int rc = read_params(params, &pr);
    if (rc) return rc;
    if (!basis || !mlp) return fail(P2S_EINVAL, "basis or mlp is NULL");
    rc = check_frame(C, H, W);
    if (rc) return rc;
    rc = check_prec(precision);
    if (rc) return rc;
    if (n_zernike < 3 || n_zernike > P2S_MAX_ZERNIKE)
        return fail(P2S_EINVAL, "n_zernike must be in [3, %d], got %d", P2S_MAX_ZERNIKE, n_zernike);
    if (mlp->m.dims[0] != n_zernike - 2)
        return fail(P2S_EINVAL, "n_zernike - 2 = %d does not match the network input width %d", n_zernike - 2,
                    mlp->m.dims[0]);
    if (mlp->m.dims[mlp->m.L] != basis->b.K)
        return fail(P2S_EINVAL, "network output width %d does not match the basis size K = %d",
                    mlp->m.dims[mlp->m.L], basis->b.K);
    if (precision != P2S_FP32 && !basis->b.bf16_ok)
        return fail(P2S_EUNSUPPORTED, "BF16 and FP8 blur need a PSF side P = 8a + 1 (9, 17, 25, 33); got %d", basis->b.P);
    if (!image || !out || (!use_scratch && !ws)) return fail(P2S_EINVAL, "image, out or workspace is NULL");
    if (!(std::isfinite(D_over_r0) && D_over_r0 >= 0.0)) return fail(P2S_EINVAL, "D/r0 must be finite and >= 0");
    const int Nfy = grid_of(H, pr.corr_len), Nfx = grid_of(W, pr.corr_len);
    if (!anc && (Nfy > kMaxFftLen || Nfx > kMaxFftLen))
        return fail(P2S_EUNSUPPORTED, "noise grid %d x %d exceeds the single-workgroup FFT limit %d", Nfy, Nfx, kMaxFftLen);
    const bool fused = blur_mlp_supported(basis->b, mlp->m, precision);
    const size_t fws = anc ? anchor_ws_bytes(*anc) : fields_ws(H, W, n_zernike, pr);
    const SimLayout L = sim_layout_fws(C, H, W, n_zernike, basis->b.K, fws, !use_scratch || !fused);
    if (use_scratch) {
        if (L.total > kScratchBytes)
            return fail(P2S_EINVAL, "frame needs %zu bytes of intermediates, more than the %zu-byte device scratch",
                        L.total, kScratchBytes);
        rc = scratch_address(&ws);
        if (rc) return rc;
        ws_bytes = kScratchBytes;
    } else if (ws_bytes < L.total) {
        return fail(P2S_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    }
    const size_t n = (size_t)C * H * W * 4;
    if (overlap(image, n, out, n)) return fail(P2S_EINVAL, "image and out overlap");
    if (overlap(ws, L.total, out, n) || overlap(ws, L.total, image, n))
        return fail(P2S_EINVAL, "workspace overlaps image or out");
    char* base = (char*)ws;
    float* F = (float*)(base + L.fields);
    float* r2 = (float*)(base + L.region2);
    float* bl = (float*)(base + L.blurred);
    rc = anc ? anchor_fields_impl(*anc, H, W, D_over_r0, seed, F, r2, L.blurred - L.region2, s)
             : make_fields_impl(H, W, D_over_r0, n_zernike, seed, pr, F, r2, L.blurred - L.region2, s);
    if (rc) return rc;
    if (fused) {     // w never leaves the chip
        hipError_t e = launch_blur_mlp(basis->b, mlp->m, precision, image, C, H, W, F, bl, s);
        if (e != hipSuccess) return hip_fail(e, "fused network and blur kernel");
    } else {
        rc = mlp_impl(mlp->m, F, n_zernike, H, W, precision, r2, s);
        if (rc) return rc;
        rc = blur_impl(image, C, H, W, basis->b, r2, precision, bl, s);
        if (rc) return rc;
    }
    rc = warp_impl(bl, C, H, W, F, pr, out, s);
    if (rc) return rc;
    return ok();
}

}  // namespace
}  // namespace p2s

namespace p2s {
namespace {

// One colour frame with a basis and a network per channel: shared fields,
// channel c through its own network and blur (fused where that form applies),
// then every channel warped by the shared tilt.
int spectral_impl(const float* image, int C, int H, int W, double D_over_r0, int n_zernike, const p2s_basis_t* bases,
                  const p2s_mlp_t* mlps, uint64_t seed, p2s_precision precision, const p2s_params* params,
                  float* out, void* ws, size_t ws_bytes, hipStream_t s) {
    Params pr;
    int rc = read_params(params, &pr);
    if (rc) return rc;
    rc = check_frame(C, H, W);
    if (rc) return rc;
    rc = check_prec(precision);
    if (rc) return rc;
    if (!bases || !mlps) return fail(P2S_EINVAL, "bases or mlps is NULL");
    if (n_zernike < 3 || n_zernike > P2S_MAX_ZERNIKE)
        return fail(P2S_EINVAL, "n_zernike must be in [3, %d], got %d", P2S_MAX_ZERNIKE, n_zernike);
    int Kmax = 0;
    bool fused[P2S_MAX_CHANNELS];
    for (int c = 0; c < C; ++c) {
        if (!bases[c] || !mlps[c]) return fail(P2S_EINVAL, "basis or mlp of channel %d is NULL", c);
        const Mlp& m = mlps[c]->m;
        const Basis& b = bases[c]->b;
        if (m.dims[0] != n_zernike - 2)
            return fail(P2S_EINVAL, "channel %d: n_zernike - 2 = %d does not match the network input width %d", c,
                        n_zernike - 2, m.dims[0]);
        if (m.dims[m.L] != b.K)
            return fail(P2S_EINVAL, "channel %d: network output width %d does not match the basis size K = %d", c,
                        m.dims[m.L], b.K);
        if (precision != P2S_FP32 && !b.bf16_ok)
            return fail(P2S_EUNSUPPORTED, "channel %d: BF16 and FP8 blur need a PSF side P = 8a + 1; got %d", c, b.P);
        Kmax = std::max(Kmax, b.K);
        fused[c] = blur_mlp_supported(b, m, precision);
    }
    if (!image || !out || !ws) return fail(P2S_EINVAL, "image, out or workspace is NULL");
    if (!(std::isfinite(D_over_r0) && D_over_r0 >= 0.0)) return fail(P2S_EINVAL, "D/r0 must be finite and >= 0");
    const int Nfy = grid_of(H, pr.corr_len), Nfx = grid_of(W, pr.corr_len);
    if (Nfy > kMaxFftLen || Nfx > kMaxFftLen)
        return fail(P2S_EUNSUPPORTED, "noise grid %d x %d exceeds the single-workgroup FFT limit %d", Nfy, Nfx, kMaxFftLen);
    const SimLayout L = sim_layout(C, H, W, n_zernike, Kmax, pr, true);
    if (ws_bytes < L.total) return fail(P2S_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    const size_t HW = (size_t)H * W, n = (size_t)C * HW * 4;
    if (overlap(image, n, out, n)) return fail(P2S_EINVAL, "image and out overlap");
    if (overlap(ws, L.total, out, n) || overlap(ws, L.total, image, n))
        return fail(P2S_EINVAL, "workspace overlaps image or out");
    char* base = (char*)ws;
    float* F = (float*)(base + L.fields);
    float* r2 = (float*)(base + L.region2);
    float* bl = (float*)(base + L.blurred);
    rc = make_fields_impl(H, W, D_over_r0, n_zernike, seed, pr, F, r2, L.blurred - L.region2, s);
    if (rc) return rc;
    for (int c = 0; c < C; ++c) {
        const float* img_c = image + c * HW;
        float* bl_c = bl + c * HW;
        if (fused[c]) {
            hipError_t e = launch_blur_mlp(bases[c]->b, mlps[c]->m, precision, img_c, 1, H, W, F, bl_c, s);
            if (e != hipSuccess) return hip_fail(e, "fused network and blur kernel");
        } else {
            rc = mlp_impl(mlps[c]->m, F, n_zernike, H, W, precision, r2, s);
            if (rc) return rc;
            rc = blur_impl(img_c, 1, H, W, bases[c]->b, r2, precision, bl_c, s);
            if (rc) return rc;
        }
    }
    rc = warp_impl(bl, C, H, W, F, pr, out, s);
    if (rc) return rc;
    return ok();
}

}  // namespace
}  // namespace p2s

struct p2s_batch_s {
    p2s::BatchHost* h;
};

using namespace p2s;

extern "C" {

int p2s_version(void) { return P2S_ABI_VERSION; }

const char* p2s_last_error(void) { return g_err.c_str(); }

int p2s_noll_variance(int j, double* out) {
    if (j < 2) return fail(P2S_EINVAL, "Noll index must be >= 2, got %d", j);
    if (!out) return fail(P2S_EINVAL, "out is NULL");
    *out = noll_var(j);
    return ok();
}

int p2s_field_grid(int n, float corr_len_px, int* nf) {
    if (n < 1 || n > P2S_MAX_SIDE) return fail(P2S_EINVAL, "n must be in [1, %d], got %d", P2S_MAX_SIDE, n);
    if (!(std::isfinite(corr_len_px) && corr_len_px > 0.0f && corr_len_px <= 1024.0f))
        return fail(P2S_EINVAL, "corr_len_px must be in (0, 1024]");
    if (!nf) return fail(P2S_EINVAL, "nf is NULL");
    *nf = grid_of(n, corr_len_px);
    return ok();
}

size_t p2s_fields_workspace_bytes(int H, int W, int n_zernike, const p2s_params* params) {
    Params pr;
    if (read_params(params, &pr) || H < 1 || W < 1 || H > P2S_MAX_SIDE || W > P2S_MAX_SIDE || n_zernike < 1 ||
        n_zernike > P2S_MAX_ZERNIKE)
        return 0;
    return fields_ws(H, W, n_zernike, pr);
}

size_t p2s_workspace_bytes(int C, int H, int W, int n_zernike, int K, const p2s_params* params) {
    Params pr;
    if (read_params(params, &pr) || check_frame(C, H, W) || n_zernike < 1 || n_zernike > P2S_MAX_ZERNIKE || K < 1 ||
        K > P2S_MAX_K)
        return 0;
    return sim_layout(C, H, W, n_zernike, K, pr).total;
}

int p2s_basis_create(const double* host_basis, int K, int P, p2s_basis_t* out) {
    try {
        if (!host_basis || !out) return fail(P2S_EINVAL, "host_basis or out is NULL");
        if (K < 1 || K > P2S_MAX_K) return fail(P2S_EINVAL, "K must be in [1, %d], got %d", P2S_MAX_K, K);
        if (P < 1 || P > P2S_MAX_P || P % 2 == 0) return fail(P2S_EINVAL, "P must be odd in [1, %d], got %d", P2S_MAX_P, P);
        for (size_t i = 0; i < (size_t)K * P * P; ++i)
            if (!std::isfinite(host_basis[i])) return fail(P2S_EINVAL, "basis value %zu is not finite", i);
        auto* h = new (std::nothrow) p2s_basis_s();
        if (!h) return fail(P2S_ENOMEM, "host allocation failed");
        int rc = pack_basis(host_basis, K, P, &h->b);
        if (rc) {
            delete h;
            return rc;
        }
        *out = h;
        return ok();
    } catch (...) {
        return fail(P2S_ENOMEM, "host allocation failed");
    }
}

int p2s_basis_destroy(p2s_basis_t basis) {
    if (!basis) return ok();
    (void)hipFree(basis->b.f32);
    if (basis->b.bf16) (void)hipFree(basis->b.bf16);
    if (basis->b.fp8) (void)hipFree(basis->b.fp8);
    if (basis->b.fp8_scale) (void)hipFree(basis->b.fp8_scale);
    delete basis;
    return ok();
}

int p2s_basis_info(p2s_basis_t basis, int* K, int* P) {
    if (!basis) return fail(P2S_EINVAL, "basis is NULL");
    if (K) *K = basis->b.K;
    if (P) *P = basis->b.P;
    return ok();
}

int p2s_mlp_create(int n_layers, const int* dims, const float* const* host_W, const float* const* host_b,
                   p2s_mlp_t* out) {
    try {
        if (!dims || !host_W || !out) return fail(P2S_EINVAL, "dims, host_W or out is NULL");
        if (n_layers < 1 || n_layers > P2S_MAX_LAYERS)
            return fail(P2S_EINVAL, "n_layers must be in [1, %d], got %d", P2S_MAX_LAYERS, n_layers);
        for (int i = 0; i <= n_layers; ++i)
            if (dims[i] < 1 || dims[i] > P2S_MAX_WIDTH)
                return fail(P2S_EINVAL, "layer width %d must be in [1, %d], got %d", i, P2S_MAX_WIDTH, dims[i]);
        if (dims[0] > P2S_MAX_ZERNIKE - 2)
            return fail(P2S_EINVAL, "input width must be <= %d, got %d", P2S_MAX_ZERNIKE - 2, dims[0]);
        if (dims[n_layers] > P2S_MAX_K) return fail(P2S_EINVAL, "output width must be <= %d", P2S_MAX_K);
        for (int l = 0; l < n_layers; ++l) {
            if (!host_W[l]) return fail(P2S_EINVAL, "host_W[%d] is NULL", l);
            for (size_t i = 0; i < (size_t)dims[l] * dims[l + 1]; ++i)
                if (!std::isfinite(host_W[l][i])) return fail(P2S_EINVAL, "weight %zu of layer %d is not finite", i, l);
            if (host_b && host_b[l])
                for (int i = 0; i < dims[l + 1]; ++i)
                    if (!std::isfinite(host_b[l][i])) return fail(P2S_EINVAL, "bias %d of layer %d is not finite", i, l);
        }
        auto* h = new (std::nothrow) p2s_mlp_s();
        if (!h) return fail(P2S_ENOMEM, "host allocation failed");
        int rc = pack_mlp(n_layers, dims, host_W, host_b, &h->m);
        if (rc) {
            delete h;
            return rc;
        }
        *out = h;
        return ok();
    } catch (...) {
        return fail(P2S_ENOMEM, "host allocation failed");
    }
}

int p2s_mlp_destroy(p2s_mlp_t mlp) {
    if (!mlp) return ok();
    (void)hipFree(mlp->m.w32);
    (void)hipFree(mlp->m.w16);
    (void)hipFree(mlp->m.bias);
    delete mlp;
    return ok();
}

int p2s_mlp_info(p2s_mlp_t mlp, int* n_in, int* n_out) {
    if (!mlp) return fail(P2S_EINVAL, "mlp is NULL");
    if (n_in) *n_in = mlp->m.dims[0];
    if (n_out) *n_out = mlp->m.dims[mlp->m.L];
    return ok();
}

int p2s_make_fields(int H, int W, double D_over_r0, int n_zernike, uint64_t seed, const p2s_params* params,
                    float* fields, void* ws, size_t ws_bytes, void* stream) {
    Params pr;
    int rc = read_params(params, &pr);
    if (rc) return rc;
    rc = make_fields_impl(H, W, D_over_r0, n_zernike, seed, pr, fields, ws, ws_bytes, (hipStream_t)stream);
    return rc ? rc : ok();
}

int p2s_mlp(p2s_mlp_t mlp, const float* fields, int n_zernike, int H, int W, p2s_precision precision, float* w,
            void* stream) {
    if (!mlp) return fail(P2S_EINVAL, "mlp is NULL");
    int rc = mlp_impl(mlp->m, fields, n_zernike, H, W, precision, w, (hipStream_t)stream);
    return rc ? rc : ok();
}

int p2s_blur(const float* image, int C, int H, int W, p2s_basis_t basis, const float* w, p2s_precision precision,
             float* out, void* stream) {
    if (!basis) return fail(P2S_EINVAL, "basis is NULL");
    int rc = blur_impl(image, C, H, W, basis->b, w, precision, out, (hipStream_t)stream);
    return rc ? rc : ok();
}

int p2s_mlp_blur(p2s_mlp_t mlp, const float* fields, int n_zernike, const float* image, int C, int H, int W,
                 p2s_basis_t basis, p2s_precision precision, float* out, void* stream) {
    if (!mlp || !basis) return fail(P2S_EINVAL, "mlp or basis is NULL");
    int rc = check_frame(C, H, W);
    if (rc) return rc;
    rc = check_prec(precision);
    if (rc) return rc;
    const Mlp& m = mlp->m;
    const Basis& b = basis->b;
    if (n_zernike - 2 != m.dims[0])
        return fail(P2S_EINVAL, "n_zernike - 2 = %d does not match the network input width %d", n_zernike - 2,
                    m.dims[0]);
    if (m.dims[m.L] != b.K)
        return fail(P2S_EINVAL, "network output width %d does not match the basis size K = %d", m.dims[m.L], b.K);
    if (!fields || !image || !out) return fail(P2S_EINVAL, "fields, image or out is NULL");
    const size_t HW = (size_t)H * W, n = (size_t)C * HW * 4;
    if (overlap(image, n, out, n)) return fail(P2S_EINVAL, "image and out overlap");
    if (overlap(fields, (size_t)n_zernike * HW * 4, out, n)) return fail(P2S_EINVAL, "fields and out overlap");
    if (precision == P2S_FP32) return fail(P2S_EUNSUPPORTED, "the fused network and blur runs in BF16 or FP8 only");
    if (!b.bf16_ok)
        return fail(P2S_EUNSUPPORTED, "BF16 and FP8 blur need a PSF side P = 8a + 1 (9, 17, 25, 33); got %d", b.P);
    if (!blur_mlp_supported(b, m, precision))
        return fail(P2S_EUNSUPPORTED, "fused form needs every network layer within the basis' %d blocks of 16 and "
                    "its packed BF16 weights (%zu bytes) in the LDS left beside the blur tile", b.nmb, m.bytes16);
    hipError_t e = launch_blur_mlp(b, m, precision, image, C, H, W, fields, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fused network and blur kernel");
    return ok();
}

int p2s_warp(const float* in, int C, int H, int W, const float* tilt, const p2s_params* params, float* out,
             void* stream) {
    Params pr;
    int rc = read_params(params, &pr);
    if (rc) return rc;
    rc = warp_impl(in, C, H, W, tilt, pr, out, (hipStream_t)stream);
    return rc ? rc : ok();
}

int p2s_simulate(const float* image, int C, int H, int W, double D_over_r0, int n_zernike, p2s_basis_t basis,
                 p2s_mlp_t mlp, uint64_t seed, p2s_precision precision, const p2s_params* params, float* out,
                 void* ws, size_t ws_bytes, void* stream) {
    return simulate_impl(image, C, H, W, D_over_r0, n_zernike, basis, mlp, seed, precision, params, out, ws,
                         ws_bytes, false, (hipStream_t)stream);
}

int p2s_simulate_noalloc(const float* image, int C, int H, int W, double D_over_r0, int n_zernike,
                         p2s_basis_t basis, p2s_mlp_t mlp, uint64_t seed, p2s_precision precision,
                         const p2s_params* params, float* out, void* stream) {
    return simulate_impl(image, C, H, W, D_over_r0, n_zernike, basis, mlp, seed, precision, params, out, nullptr,
                         0, true, (hipStream_t)stream);
}

int p2s_anchor_create(int G, int n_zernike, const double* host_spatial, const double* host_modes,
                      p2s_anchor_t* out) {
    try {
        if (!host_spatial || !host_modes || !out) return fail(P2S_EINVAL, "host_spatial, host_modes or out is NULL");
        if (G < 2 || G > P2S_MAX_ANCHOR_GRID)
            return fail(P2S_EINVAL, "G must be in [2, %d], got %d", P2S_MAX_ANCHOR_GRID, G);
        if (n_zernike < 1 || n_zernike > P2S_MAX_ZERNIKE)
            return fail(P2S_EINVAL, "n_zernike must be in [1, %d], got %d", P2S_MAX_ZERNIKE, n_zernike);
        const size_t G2 = (size_t)G * G;
        for (size_t r = 0; r < G2; ++r)
            for (size_t c = 0; c <= r; ++c)
                if (!std::isfinite(host_spatial[r * G2 + c]))
                    return fail(P2S_EINVAL, "spatial factor entry (%zu, %zu) is not finite", r, c);
        for (int r = 0; r < n_zernike; ++r)
            for (int c = 0; c <= r; ++c)
                if (!std::isfinite(host_modes[(size_t)r * n_zernike + c]))
                    return fail(P2S_EINVAL, "mode factor entry (%d, %d) is not finite", r, c);
        auto* h = new (std::nothrow) p2s_anchor_s();
        if (!h) return fail(P2S_ENOMEM, "host allocation failed");
        int rc = pack_anchor(G, n_zernike, host_spatial, host_modes, &h->a);
        if (rc) {
            delete h;
            return rc;
        }
        *out = h;
        return ok();
    } catch (...) {
        return fail(P2S_ENOMEM, "host allocation failed");
    }
}

int p2s_anchor_destroy(p2s_anchor_t anchors) {
    if (!anchors) return ok();
    (void)hipFree(anchors->a.Ls);
    (void)hipFree(anchors->a.Lz);
    delete anchors;
    return ok();
}

int p2s_anchor_info(p2s_anchor_t anchors, int* G, int* n_zernike) {
    if (!anchors) return fail(P2S_EINVAL, "anchors is NULL");
    if (G) *G = anchors->a.G;
    if (n_zernike) *n_zernike = anchors->a.n;
    return ok();
}

size_t p2s_anchor_fields_workspace_bytes(p2s_anchor_t anchors) {
    return anchors ? anchor_ws_bytes(anchors->a) : 0;
}

int p2s_make_fields_anchor(p2s_anchor_t anchors, int H, int W, double D_over_r0, uint64_t seed, float* fields,
                           void* ws, size_t ws_bytes, void* stream) {
    if (!anchors) return fail(P2S_EINVAL, "anchors is NULL");
    int rc = anchor_fields_impl(anchors->a, H, W, D_over_r0, seed, fields, ws, ws_bytes, (hipStream_t)stream);
    return rc ? rc : ok();
}

size_t p2s_workspace_bytes_anchor(p2s_anchor_t anchors, int C, int H, int W, int K) {
    if (!anchors || check_frame(C, H, W) || K < 1 || K > P2S_MAX_K) return 0;
    return sim_layout_fws(C, H, W, anchors->a.n, K, anchor_ws_bytes(anchors->a), true).total;
}

int p2s_simulate_anchor(const float* image, int C, int H, int W, double D_over_r0, p2s_anchor_t anchors,
                        p2s_basis_t basis, p2s_mlp_t mlp, uint64_t seed, p2s_precision precision,
                        const p2s_params* params, float* out, void* ws, size_t ws_bytes, void* stream) {
    if (!anchors) return fail(P2S_EINVAL, "anchors is NULL");
    return simulate_impl(image, C, H, W, D_over_r0, anchors->a.n, basis, mlp, seed, precision, params, out, ws,
                         ws_bytes, false, (hipStream_t)stream, &anchors->a);
}

int p2s_simulate_spectral(const float* image, int C, int H, int W, double D_over_r0, int n_zernike,
                          const p2s_basis_t* bases, const p2s_mlp_t* mlps, uint64_t seed, p2s_precision precision,
                          const p2s_params* params, float* out, void* ws, size_t ws_bytes, void* stream) {
    return spectral_impl(image, C, H, W, D_over_r0, n_zernike, bases, mlps, seed, precision, params, out, ws,
                         ws_bytes, (hipStream_t)stream);
}

size_t p2s_batch_workspace_bytes(const p2s_frame* frames, int n, int n_zernike, int K, const p2s_params* params) {
    Params pr;
    if (read_params(params, &pr) || n < 0 || (n > 0 && !frames) || n_zernike < 1 || n_zernike > P2S_MAX_ZERNIKE ||
        K < 1 || K > P2S_MAX_K)
        return 0;
    BatchLayout L;
    const std::string saved = g_err;
    if (batch_layout(frames, n, n_zernike, K, pr, &L)) {
        g_err = saved;
        return 0;
    }
    return L.total;
}

int p2s_batch_create(const p2s_frame* frames, int n, int n_zernike, p2s_basis_t basis, p2s_mlp_t mlp,
                     p2s_precision precision, const p2s_params* params, const p2s_batch_options* options, void* ws,
                     size_t ws_bytes, p2s_batch_t* out) {
    try {
        if (!out) return fail(P2S_EINVAL, "out is NULL");
        if (!basis || !mlp) return fail(P2S_EINVAL, "basis or mlp is NULL");
        Params pr;
        int rc = read_params(params, &pr);
        if (rc) return rc;
        auto* hb = new (std::nothrow) p2s_batch_s();
        if (!hb) return fail(P2S_ENOMEM, "host allocation failed");
        rc = batch_create(frames, n, n_zernike, basis->b, mlp->m, precision, pr, options, ws, ws_bytes, &hb->h);
        if (rc) {
            delete hb;
            return rc;
        }
        *out = hb;
        return ok();
    } catch (...) {
        return fail(P2S_ENOMEM, "host allocation failed");
    }
}

int p2s_batch_upload(p2s_batch_t batch, void* stream) {
    if (!batch) return fail(P2S_EINVAL, "batch is NULL");
    int rc = batch_upload(batch->h, (hipStream_t)stream);
    return rc ? rc : ok();
}

int p2s_batch_launch(p2s_batch_t batch, void* stream) {
    if (!batch) return fail(P2S_EINVAL, "batch is NULL");
    int rc = batch_launch(batch->h, (hipStream_t)stream);
    return rc ? rc : ok();
}

int p2s_batch_info(p2s_batch_t batch, int* items, int* grid) {
    if (!batch) return fail(P2S_EINVAL, "batch is NULL");
    for (int st = 0; st < ST_N; ++st) {
        if (items) items[st] = batch->h->bl.items[st];
        if (grid) grid[st] = batch->h->bl.grid[st];
    }
    return ok();
}

int p2s_batch_destroy(p2s_batch_t batch) {
    if (!batch) return ok();
    batch_free(batch->h);
    delete batch;
    return ok();
}

int p2s_simulate_batch(const p2s_frame* frames, int n, int n_zernike, p2s_basis_t basis, p2s_mlp_t mlp,
                       p2s_precision precision, const p2s_params* params, void* ws, size_t ws_bytes, void* stream) {
    p2s_batch_t b = nullptr;
    int rc = p2s_batch_create(frames, n, n_zernike, basis, mlp, precision, params, nullptr, ws, ws_bytes, &b);
    if (rc) return rc;
    rc = batch_upload(b->h, (hipStream_t)stream);
    if (!rc) rc = batch_launch(b->h, (hipStream_t)stream);
    const std::string err = g_err;
    p2s_batch_destroy(b);   // waits until the plan upload has been consumed
    if (rc) {
        g_err = err;
        return rc;
    }
    return ok();
}

int p2s_debug_noise(int Nfy, int Nfx, int pair, uint64_t seed, uint32_t* raw, float* normals, void* stream) {
    if (Nfy < 1 || Nfx < 1 || Nfy > 65536 || Nfx > 65536 || (size_t)Nfy * Nfx > ((size_t)1 << 30))
        return fail(P2S_EINVAL, "bad grid %d x %d", Nfy, Nfx);
    if (pair < 0) return fail(P2S_EINVAL, "pair must be >= 0");
    if (!raw) return fail(P2S_EINVAL, "raw is NULL");
    hipError_t e = launch_debug_noise(Nfy, Nfx, pair, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), raw,
                                      normals, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "noise kernel");
    return ok();
}

}  // extern "C"
