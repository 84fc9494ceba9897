// Host-side calls of the C ABI for a sanitizer build (AddressSanitizer and
// UndefinedBehaviorSanitizer on the library's host code; no GPU needed):
// argument validation of every entry point, the host arithmetic, and the
// operand packing of the basis, network and anchor handles, which runs on
// the host before the upload (without a device the upload then fails, and
// the handle calls return an error).  Exit status 0 when every call
// returned what the contract says.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "p2s.h"

static int failures = 0;
#define EXPECT(cond)                                                                   \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            std::fprintf(stderr, "FAILED: %s (line %d): %s\n", #cond, __LINE__,        \
                         p2s_last_error());                                            \
            ++failures;                                                                \
        }                                                                              \
    } while (0)

int main() {
    void* fake = reinterpret_cast<void*>(0x1000);
    float* ff = reinterpret_cast<float*>(0x1000);
    // host arithmetic
    for (int j = 2; j <= 36; ++j) {
        double v = 0.0;
        EXPECT(p2s_noll_variance(j, &v) == P2S_OK && v > 0.0);
    }
    EXPECT(p2s_noll_variance(1, nullptr) != P2S_OK);
    EXPECT(p2s_workspace_bytes(3, 512, 512, 35, 100, nullptr) > 0);
    EXPECT(p2s_fields_workspace_bytes(512, 512, 35, nullptr) > 0);
    // validation of the stage calls
    EXPECT(p2s_blur(ff, 1, 8, 8, nullptr, ff, P2S_BF16, ff, nullptr) == P2S_EINVAL);
    EXPECT(p2s_warp(ff, 0, 8, 8, ff, nullptr, reinterpret_cast<float*>(0x2000), nullptr) == P2S_EINVAL);
    EXPECT(p2s_warp(ff, 1, 8, 8, reinterpret_cast<float*>(0x9000), nullptr, reinterpret_cast<float*>(0x1010),
                    nullptr) == P2S_EINVAL);
    EXPECT(p2s_make_fields(8, 8, -1.0, 35, 1, nullptr, ff, fake, 1 << 30, nullptr) == P2S_EINVAL);
    EXPECT(p2s_make_fields(8, 8, 1.0, 65, 1, nullptr, ff, fake, 1 << 30, nullptr) == P2S_EINVAL);
    EXPECT(p2s_make_fields(8, 8, 1.0, 35, 1, nullptr, ff, fake, 16, nullptr) == P2S_EINVAL);
    EXPECT(p2s_make_fields(16000, 8, 1.0, 35, 1, nullptr, ff, fake, (size_t)1 << 40, nullptr) == P2S_EUNSUPPORTED);
    EXPECT(p2s_simulate(ff, 1, 8, 8, 1.0, 35, nullptr, nullptr, 1, P2S_FP32, nullptr, ff, fake, 1 << 30, nullptr) ==
           P2S_EINVAL);
    EXPECT(p2s_debug_noise(4, 4, 0, 1, nullptr, nullptr, nullptr) == P2S_EINVAL);
    // handles: invalid shapes and values are refused before any packing
    p2s_basis_t b = nullptr;
    std::vector<double> bad(4 * 6 * 6, 0.0);
    EXPECT(p2s_basis_create(bad.data(), 4, 6, &b) == P2S_EINVAL);
    std::vector<double> nan(2 * 5 * 5, std::nan(""));
    EXPECT(p2s_basis_create(nan.data(), 2, 5, &b) == P2S_EINVAL);
    // valid handles: packed on the host (every precision's layout), then the
    // upload fails without a device
    for (int P : {9, 17, 33}) {
        const int K = P == 33 ? 100 : 16;
        std::vector<double> basis((size_t)K * P * P);
        for (size_t i = 0; i < basis.size(); ++i) basis[i] = std::sin(0.37 * (double)i) / (double)(P * P);
        b = nullptr;
        const int rc = p2s_basis_create(basis.data(), K, P, &b);
        EXPECT(rc == P2S_OK || rc == P2S_EDEVICE || rc == P2S_ENOMEM);
        if (rc == P2S_OK) p2s_basis_destroy(b);
    }
    {
        const int dims[4] = {33, 100, 100, 100};
        std::vector<std::vector<float>> W(3), B(3);
        const float* Wp[3];
        const float* Bp[3];
        for (int l = 0; l < 3; ++l) {
            W[l].resize((size_t)dims[l] * dims[l + 1]);
            B[l].resize(dims[l + 1]);
            for (size_t i = 0; i < W[l].size(); ++i) W[l][i] = 0.01f * std::cos(0.11f * (float)i);
            for (size_t i = 0; i < B[l].size(); ++i) B[l][i] = 0.001f * (float)i;
            Wp[l] = W[l].data();
            Bp[l] = B[l].data();
        }
        p2s_mlp_t m = nullptr;
        const int rc = p2s_mlp_create(3, dims, Wp, Bp, &m);
        EXPECT(rc == P2S_OK || rc == P2S_EDEVICE || rc == P2S_ENOMEM);
        if (rc == P2S_OK) p2s_mlp_destroy(m);
        const int wide[3] = {33, 200, 16};
        EXPECT(p2s_mlp_create(2, wide, Wp, Bp, &m) == P2S_EINVAL);
    }
    // batches
    p2s_frame fr{};
    fr.image = ff;
    fr.out = reinterpret_cast<float*>(0x2000);
    fr.C = 1;
    fr.H = 8;
    fr.W = 8;
    fr.D_over_r0 = 1.0;
    p2s_batch_t bt = nullptr;
    EXPECT(p2s_batch_create(&fr, 1, 35, nullptr, nullptr, P2S_BF16, nullptr, nullptr, reinterpret_cast<void*>(0x9000),
                            (size_t)1 << 30, &bt) == P2S_EINVAL);
    EXPECT(p2s_batch_destroy(nullptr) == P2S_OK);
    EXPECT(p2s_batch_workspace_bytes(&fr, 1, 35, 100, nullptr) > 0);
    if (failures) std::fprintf(stderr, "%d failures\n", failures);
    else std::printf("abi driver: all host-side checks passed\n");
    return failures ? 1 : 0;
}
