/*
 * p2s.h -- C ABI of the MI355X (gfx950) hot path of the phase-to-space (P2S)
 * turbulence simulator (Mao, Chimitt & Chan, ICCV 2021).
 *
 * One frame goes through four stages, each a call below and all four chained
 * by p2s_simulate:
 *   fields  -- per-pixel Zernike coefficient planes alpha_j(x), spatially
 *              correlated (Sec. 2.2 Eq. 1 and Sec. 3.4), made either by
 *              filtering seeded white noise with a Gaussian PSD
 *              (p2s_make_fields) or, as in the paper, drawn on a grid of
 *              anchor points and interpolated (p2s_make_fields_anchor);
 *   mlp     -- the P2S network mapping alpha_4.. to the basis weights
 *              beta_m(x) at every pixel (Sec. 3.3);
 *   blur    -- the spatially varying blur written as M invariant
 *              convolutions with the basis PSFs and a per-pixel weighted sum
 *              (Sec. 3.1, Eq. 4-5), fused so that the convolution outputs
 *              never leave the chip;
 *   warp    -- the tilt displacement by alpha_2, alpha_3 after the blur
 *              (Sec. 2.2 and 3.3).
 *
 * Conventions shared by every call
 *   - Pointers marked "device" are device memory of the current HIP device;
 *     "host" pointers are host memory.  The caller owns every data buffer and
 *     the workspace; the library owns only the handles it creates and never
 *     frees caller memory.
 *   - Images are planar float32, [C][H][W], row-major, no padding.
 *   - Field planes are float32 [n_zernike][H][W]: plane p holds Noll mode
 *     j = p + 2 (plane 0 = x-tilt alpha_2, plane 1 = y-tilt alpha_3, planes
 *     2.. = alpha_4..), in radians of pupil phase.
 *   - Basis weights w are float32 [H*W][K] (pixel-major, K contiguous).
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every compute call
 *     only enqueues work on it and returns; results are ready once the stream
 *     is synchronised.
 *   - Return value: P2S_OK (0) or a negative p2s_status.  Arguments are
 *     validated on the host before anything is enqueued; on a validation
 *     error nothing is written.  p2s_last_error() gives a message for the
 *     last failure on the calling thread.  No C++ exception crosses the ABI.
 */
#ifndef P2S_H
#define P2S_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define P2S_ABI_VERSION 1

typedef enum {
    P2S_OK = 0,
    P2S_EINVAL = -1,        /* bad argument, size or relationship          */
    P2S_ENOMEM = -2,        /* device or host allocation failed            */
    P2S_EDEVICE = -3,       /* a HIP call or kernel launch failed           */
    P2S_EUNSUPPORTED = -4   /* valid request this build does not implement */
} p2s_status;

typedef enum {
    P2S_FP32 = 0,     /* FP32 MFMA for network and blur                     */
    P2S_BF16 = 1,     /* BF16 MFMA, FP32 accumulation; network activations
                         enter as a bf16 hi + lo pair, weights w stay FP32   */
    P2S_FP8E4M3 = 2   /* blur on FP8 E4M3 MFMA (image rounded to E4M3 after
                         clamping to +-448; basis function k scaled by a power
                         of two 2^e_k, max |phi_k| 2^e_k <= 448, before
                         rounding, the scale undone inside the MFMA), FP32
                         accumulation; the network on BF16 MFMA with its
                         activations as bf16 alone (no lo part: the FP8
                         blur's error is far larger than what it removes)    */
} p2s_precision;

/* Opaque, immutable, device-resident handles; safe to share across streams. */
typedef struct p2s_basis_s* p2s_basis_t;
typedef struct p2s_mlp_s* p2s_mlp_t;
typedef struct p2s_anchor_s* p2s_anchor_t;

/* Optional parameters; pass NULL for the defaults shown. */
typedef struct {
    float corr_len_px;   /* 16: Gaussian standard deviation, in pixels, of the
                            covariance of every field plane                  */
    float q_sampling;    /* 2: image samples per lambda/D; a tilt alpha moves
                            the image by 2*q*alpha/pi pixels                   */
} p2s_params;

/* Limits of this build. */
#define P2S_MAX_K 128          /* basis functions                            */
#define P2S_MAX_P 33           /* PSF side (odd)                             */
#define P2S_MAX_ZERNIKE 64     /* field planes (Noll 2 .. 65)                */
#define P2S_MAX_WIDTH 128      /* widest network layer                       */
#define P2S_MAX_LAYERS 4
#define P2S_MAX_SIDE 16384     /* H, W                                       */
#define P2S_MAX_CHANNELS 4
#define P2S_MAX_ANCHOR_GRID 128 /* anchor grid side G                       */

int p2s_version(void);
const char* p2s_last_error(void);

/* ---------------------------------------------------------------- host -- */

/* Variance of Noll mode j >= 2 of Kolmogorov turbulence per (D/r0)^(5/3):
 * the diagonal of R_Z (Sec. 2.2).  Computed as
 * K (n+1) Gamma(n-5/6) / (Gamma(17/6)^2 Gamma(n+23/6)) for radial order n,
 * K fixed so that the variances of all modes j >= 2 sum to 1.0299, Noll's
 * piston-removed phase variance.  Writes *out; EINVAL for j < 2. */
int p2s_noll_variance(int j, double* out);

/* Side of the periodic noise grid used for an image side n: the smallest
 * 2^a 3^b 5^c >= n + ceil(4 * corr_len_px).  Writes *nf. */
int p2s_field_grid(int n, float corr_len_px, int* nf);

/* Device bytes p2s_make_fields needs as workspace for an H x W frame. */
size_t p2s_fields_workspace_bytes(int H, int W, int n_zernike, const p2s_params* params);

/* Device bytes p2s_simulate needs as workspace: fields, weights, blurred
 * image and the field generator's intermediate (256-byte aligned pieces). */
size_t p2s_workspace_bytes(int C, int H, int W, int n_zernike, int K, const p2s_params* params);

/* ------------------------------------------------------------- handles -- */

/* Upload a PSF basis phi_m (Sec. 3.1 Eq. 4, learned by PCA in Sec. 3.2).
 * host_basis: host, float64 [K][P][P]; tap [i][j] sits at offset
 * (i - R, j - R), R = (P-1)/2, and acts as a convolution kernel.
 * K in [1, P2S_MAX_K], P odd in [1, P2S_MAX_P].  The library keeps FP32,
 * BF16 and (for P = 8a + 1) FP8 E4M3 copies laid out for its MFMA kernels.
 * *out receives the handle. */
int p2s_basis_create(const double* host_basis, int K, int P, p2s_basis_t* out);
int p2s_basis_destroy(p2s_basis_t basis);
int p2s_basis_info(p2s_basis_t basis, int* K, int* P);

/* Upload the P2S network (Sec. 3.3): n_layers fully connected layers
 * y = W x + b with ReLU after all but the last.  dims[n_layers+1] are the
 * layer widths (dims[0] = number of high-order modes, dims[n_layers] = K);
 * each width in [1, P2S_MAX_WIDTH], n_layers in [1, P2S_MAX_LAYERS].
 * host_W[l]: host float32 [dims[l+1]][dims[l]]; host_b[l]: host float32
 * [dims[l+1]] (a NULL host_b or host_b[l] means zero bias).  The BF16 path
 * rounds the weights to bfloat16 (exact if they are bf16-representable). */
int p2s_mlp_create(int n_layers, const int* dims, const float* const* host_W,
                   const float* const* host_b, p2s_mlp_t* out);
int p2s_mlp_destroy(p2s_mlp_t mlp);
int p2s_mlp_info(p2s_mlp_t mlp, int* n_in, int* n_out);

/* ------------------------------------------------------------- compute -- */

/* Stage 1: correlated Zernike fields.  Plane p carries Noll mode j = p + 2;
 * planes 2q and 2q+1 are the real and imaginary parts of one complex field
 *   G_q(y,x) = (Nf_y Nf_x)^(-1/2) sum_k sqrt(S(k)) n_q(k) e^{+2 pi i k.(y,x)/Nf}
 * on the periodic Nf_y x Nf_x grid (p2s_field_grid), cropped to the top-left
 * H x W and scaled by sqrt(V_j (D/r0)^(5/3)).  S(f) = exp(-2 pi^2 l^2 |f|^2)
 * normalised to mean 1; n_q(k) is complex white noise drawn per frequency bin
 * from Philox4x32-10 with key (seed mod 2^32, seed >> 32) and counter
 * (kx, ky, q, 0), Box-Muller on outputs 0 and 1.  Bins where a 1-D factor of
 * sqrt(S) is below 1e-9 of its peak are skipped (error < 1.5e-9 rms).
 * fields: device float32 [n_zernike][H][W].  ws: device, at least
 * p2s_fields_workspace_bytes.  n_zernike in [1, P2S_MAX_ZERNIKE]. */
int p2s_make_fields(int H, int W, double D_over_r0, int n_zernike, uint64_t seed,
                    const p2s_params* params, float* fields, void* ws, size_t ws_bytes,
                    void* stream);

/* Stage 2: the P2S network at every pixel (Sec. 3.3).  Reads planes
 * 2 .. n_zernike-1 of `fields` (device [n_zernike][H][W]); requires
 * n_zernike - 2 == the network's input width.  Writes w: device float32
 * [H*W][K], K = the network's output width.  precision: P2S_FP32, P2S_BF16
 * (BF16 MFMA, activations as bf16 hi + lo) or P2S_FP8E4M3 (BF16 MFMA,
 * activations as bf16 alone). */
int p2s_mlp(p2s_mlp_t mlp, const float* fields, int n_zernike, int H, int W,
            p2s_precision precision, float* w, void* stream);

/* Stage 3: fused basis blur (Sec. 3.1, Eq. 5):
 *   out_c(x) = sum_k w_k(x) sum_u phi_k(u) image_c(clamp(x - u)),
 * replicate border, the same weights for every channel (Sec. 3.5).
 * image, out: device float32 [C][H][W] (must not overlap); w: device float32
 * [H*W][K] with K = the basis size.  precision: P2S_FP32 (any odd P),
 * P2S_BF16 or P2S_FP8E4M3 (P = 8a + 1, e.g. 17 or 33). */
int p2s_blur(const float* image, int C, int H, int W, p2s_basis_t basis, const float* w,
             p2s_precision precision, float* out, void* stream);

/* Stages 2 and 3 in one kernel: the P2S network evaluated inside the blur's
 * epilogue, so the weights w never exist in memory.  Computes exactly what
 * p2s_mlp followed by p2s_blur computes with the same precision.  fields:
 * device [n_zernike][H][W]; image, out: device float32 [C][H][W] (out must
 * not overlap image or fields).  precision: P2S_BF16 or P2S_FP8E4M3 (network
 * in BF16); P = 8a + 1.  EUNSUPPORTED when this network does not fit the
 * fused form: a layer wider than the basis' blocks of 16 (ceil(K/16)), or
 * packed BF16 weights too large for the LDS left beside the blur tile
 * (about 78 KB for P = 33 at K <= 112); p2s_simulate then uses the two
 * stages separately. */
int p2s_mlp_blur(p2s_mlp_t mlp, const float* fields, int n_zernike, const float* image, int C, int H, int W,
                 p2s_basis_t basis, p2s_precision precision, float* out, void* stream);

/* Stage 4: tilt warp (Sec. 2.2, 3.3): out_c(y, x) = bilinear sample of in_c
 * at (y + s*tilt[1](y,x), x + s*tilt[0](y,x)), s = 2 q / pi, sample position
 * clamped to the image.  in, out: device float32 [C][H][W] (must not
 * overlap); tilt: device float32 [2][H][W] (planes 0 and 1 of the fields). */
int p2s_warp(const float* in, int C, int H, int W, const float* tilt,
             const p2s_params* params, float* out, void* stream);

/* One frame end to end: fields -> mlp -> blur -> warp (the network and blur
 * fused as in p2s_mlp_blur where that form applies), intermediates in ws
 * (device, at least p2s_workspace_bytes).  image, out: device float32
 * [C][H][W].  n_zernike - 2 must equal the network's input width and the
 * network's output width must equal the basis size K. */
int p2s_simulate(const float* image, int C, int H, int W, double D_over_r0, int n_zernike,
                 p2s_basis_t basis, p2s_mlp_t mlp, uint64_t seed, p2s_precision precision,
                 const p2s_params* params, float* out, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * frame as p2s_simulate, bit for bit, with the intermediates in a device
 * array of P2S_NOALLOC_SCRATCH_BYTES that the library holds per GPU until the
 * process ends, instead of a caller workspace.  No allocation happens in the
 * call.  The frame needs, each rounded up to 256 bytes: the fields
 * (4 n_zernike H W bytes), the field generator's intermediate (part of
 * p2s_fields_workspace_bytes) or, when the network and blur run as two
 * kernels (P2S_FP32, or a network the fused kernel cannot hold), the larger
 * of it and the weights w (4 H W K bytes), and the blurred image (4 C H W
 * bytes); EINVAL when that exceeds the scratch (a 512 x 512 frame of up to 3
 * channels fits in every precision).  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race
 * and give undefined results; order them on one stream.  Arguments as in
 * p2s_simulate. */
#define P2S_NOALLOC_SCRATCH_BYTES ((size_t)160 << 20)
int p2s_simulate_noalloc(const float* image, int C, int H, int W, double D_over_r0, int n_zernike,
                         p2s_basis_t basis, p2s_mlp_t mlp, uint64_t seed, p2s_precision precision,
                         const p2s_params* params, float* out, void* stream);

/* Wavelength-dependent colour (Sec. 3.5): channel c of a C-channel frame is
 * blurred with the PSFs of its own wavelength, through bases[c] and mlps[c]
 * (host arrays of C handles, read during the call), instead of one basis
 * and network for every channel.  The fields (stage 1) are shared: they are
 * the coefficients at a reference wavelength, and each channel's network
 * maps those to its own basis' weights (the wavelength's phase scale and
 * sampling live in its training and basis).  The tilt displacement is the
 * same at every wavelength, so every channel is warped by planes 0 and 1.
 * Otherwise as p2s_simulate: channel c computes exactly what p2s_simulate
 * computes for a one-channel frame of plane c with bases[c] and mlps[c].
 * ws: at least p2s_workspace_bytes(C, H, W, n_zernike, K, params) with K the
 * largest basis size among the channels. */
int p2s_simulate_spectral(const float* image, int C, int H, int W, double D_over_r0, int n_zernike,
                          const p2s_basis_t* bases, const p2s_mlp_t* mlps, uint64_t seed, p2s_precision precision,
                          const p2s_params* params, float* out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------- anchor grid --
 * The paper's own field model (Sec. 3.4, "Interpolation across the grid",
 * with the mode covariance R_Z of Sec. 2.2): the Zernike coefficients of a
 * G x G grid of anchor points are drawn jointly,
 *   A = L_s E L_Z^T (D/r0)^(5/6),
 * with L_s (L_s^T) the anchor correlation matrix R_s, L_Z (L_Z^T) = R_Z per
 * (D/r0)^(5/3) and E [G^2][n_zernike] standard normals, so that
 * Cov(A[p][i], A[q][k]) = R_s[p][q] R_Z[i][k] (D/r0)^(5/3); then every plane
 * is interpolated bilinearly from the anchors to the pixels (interpolation of
 * the coefficients, i.e. of the phase, not of PSFs).  E[p][i] comes from
 * Philox4x32-10 with key (seed mod 2^32, seed >> 32) and counter
 * (p, i >> 1, 0, 1), Box-Muller on outputs 0 and 1 as for p2s_make_fields
 * (cosine for even i, sine for odd i).  Anchor (a, b), index p = a G + b,
 * sits at pixel (a (H-1)/(G-1), b (W-1)/(G-1)): the grid spans the image from
 * corner to corner whatever its size, so the correlation is set in anchor
 * spacings.  Both covariances are the caller's: the library takes their
 * factors as data (any model, e.g. angle-of-arrival statistics, fits). */

/* Upload the two factors.  host_spatial: host float64 [G*G][G*G],
 * row-major, the lower-triangular L_s (entries above the diagonal are
 * ignored); host_modes: host float64 [n_zernike][n_zernike], the
 * lower-triangular L_Z for planes i = Noll mode i + 2 (above the diagonal
 * ignored).  G in [2, P2S_MAX_ANCHOR_GRID], n_zernike in
 * [1, P2S_MAX_ZERNIKE].  Both are read during the call only; the handle
 * keeps FP32 copies, 4 Gp (Gp + 32) bytes of device memory for Gp = G^2
 * rounded up to 32 (about 64 MiB for G = 64).  EINVAL on a non-finite entry. */
int p2s_anchor_create(int G, int n_zernike, const double* host_spatial, const double* host_modes,
                      p2s_anchor_t* out);
int p2s_anchor_destroy(p2s_anchor_t anchors);
int p2s_anchor_info(p2s_anchor_t anchors, int* G, int* n_zernike);

/* Device bytes p2s_make_fields_anchor needs as workspace (the normals times
 * L_Z^T, and the partial sums of the anchor product); 0 for NULL. */
size_t p2s_anchor_fields_workspace_bytes(p2s_anchor_t anchors);

/* Stage 1 with the anchor model: fields = device float32
 * [n_zernike][H][W] (n_zernike of the handle; plane i = Noll mode i + 2),
 * bilinear in every anchor cell.  ws: device, at least
 * p2s_anchor_fields_workspace_bytes, must not overlap fields.  D/r0 finite
 * and >= 0. */
int p2s_make_fields_anchor(p2s_anchor_t anchors, int H, int W, double D_over_r0, uint64_t seed, float* fields,
                           void* ws, size_t ws_bytes, void* stream);

/* Workspace of p2s_simulate_anchor for a C x H x W frame and a basis of K
 * functions; 0 on a bad argument. */
size_t p2s_workspace_bytes_anchor(p2s_anchor_t anchors, int C, int H, int W, int K);

/* One frame end to end with the anchor model as stage 1: otherwise exactly
 * p2s_simulate (network and blur fused where that form applies, then the
 * warp by planes 0 and 1).  The handle's n_zernike - 2 must equal the
 * network's input width; params: only q_sampling is used.  ws: at least
 * p2s_workspace_bytes_anchor. */
int p2s_simulate_anchor(const float* image, int C, int H, int W, double D_over_r0, p2s_anchor_t anchors,
                        p2s_basis_t basis, p2s_mlp_t mlp, uint64_t seed, p2s_precision precision,
                        const p2s_params* params, float* out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------- batches --
 * Many frames, of any sizes and channel counts, through the same four stages
 * as p2s_simulate, with one launch per stage for the whole batch: every
 * workgroup strides over a flat list of (frame, work item) pairs read from a
 * device-side plan.  Frame i of a batch gives exactly the result
 * p2s_simulate gives for it alone (same seed, D/r0, handles, precision and
 * parameters): the stages do the same arithmetic, only the schedule differs.
 *
 * Use: p2s_batch_workspace_bytes -> p2s_batch_create (host only, validates
 * everything and builds the plan) -> p2s_batch_upload (enqueues the copy of
 * the plan into the workspace) -> p2s_batch_launch (enqueues the kernels;
 * the only step that may be captured into a HIP graph, and replayed as often
 * as the plan is unchanged) -> p2s_batch_destroy.  p2s_simulate_batch does
 * all of it in one call. */

/* One frame of a batch.  image, out: device float32 [C][H][W]. */
typedef struct {
    const float* image;
    float* out;
    int C, H, W;
    double D_over_r0;
    uint64_t seed;
} p2s_frame;

/* Schedule options of a batch; NULL = the defaults shown. */
typedef struct {
    int blur_tile_rows;  /* 16: output rows per blur work item (16 or 8; 8 is
                            used anyway when the basis has K > 112)          */
    int persistent;      /* 1: launch as many workgroups as the device holds
                            at once, each striding over the items; 0: one
                            workgroup per item                               */
} p2s_batch_options;

typedef struct p2s_batch_s* p2s_batch_t;

/* Device bytes of workspace a batch needs: the plan, then per frame the same
 * pieces as p2s_workspace_bytes.  0 on a bad argument (n = 0 gives 0). */
size_t p2s_batch_workspace_bytes(const p2s_frame* frames, int n, int n_zernike, int K,
                                 const p2s_params* params);

/* Validate a batch of n >= 0 frames (host: `frames`, read during the call
 * only) and build its plan in host memory.  Every frame satisfies what
 * p2s_simulate requires; output buffers must not overlap each other or ws;
 * images must not overlap ws.  basis and mlp must outlive the batch handle.
 * ws: device, at least p2s_batch_workspace_bytes; it holds the plan and all
 * intermediates, and is bound to the handle.  *out receives the handle. */
int p2s_batch_create(const p2s_frame* frames, int n, int n_zernike, p2s_basis_t basis, p2s_mlp_t mlp,
                     p2s_precision precision, const p2s_params* params,
                     const p2s_batch_options* options, void* ws, size_t ws_bytes, p2s_batch_t* out);

/* Enqueue the copy of the plan into the workspace on `stream`.  Needed once
 * before the first launch (and again after anything else wrote ws).
 * EUNSUPPORTED while the stream is being captured. */
int p2s_batch_upload(p2s_batch_t batch, void* stream);

/* Enqueue the batched kernels (fields, network, blur, warp) on `stream`; no
 * allocation, copy or host synchronisation, so it may be captured. */
int p2s_batch_launch(p2s_batch_t batch, void* stream);

/* Work items and launched workgroups of the five batched kernels (column and
 * row field transforms, network, blur, warp); either pointer may be NULL,
 * otherwise it receives 5 ints. */
int p2s_batch_info(p2s_batch_t batch, int* items, int* grid);

/* Free the handle; blocks until a pending plan upload has been consumed. */
int p2s_batch_destroy(p2s_batch_t batch);

/* create + upload + launch + destroy with default options.  Returns once the
 * plan upload has been consumed on `stream` (that is, after the work queued
 * on the stream before this call), with the kernels enqueued. */
int p2s_simulate_batch(const p2s_frame* frames, int n, int n_zernike, p2s_basis_t basis, p2s_mlp_t mlp,
                       p2s_precision precision, const p2s_params* params, void* ws, size_t ws_bytes,
                       void* stream);

/* Test hook: the noise generator behind p2s_make_fields for plane pair
 * `pair` on an Nfy x Nfx grid of frequency bins.  raw: device uint32
 * [Nfy][Nfx][4], the four Philox outputs of counter (kx, ky, pair, 0);
 * normals: device float32 [Nfy][Nfx][2] (real, imaginary), may be NULL. */
int p2s_debug_noise(int Nfy, int Nfx, int pair, uint64_t seed, uint32_t* raw, float* normals,
                    void* stream);

#ifdef __cplusplus
}
#endif
#endif /* P2S_H */
