// Internal layout of the summary-statistics emulator (libcpm's emu_* calls).
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace cpm {
namespace emu {

constexpr int kIn = 6;        // inputs per point
constexpr int kHidden = 256;  // width of the three hidden layers
constexpr int kOut = 8;       // outputs per point
constexpr int kInPad = 32;    // K of the first layer, padded to one MFMA k-step
constexpr int kOutPad = 64;   // N of the last layer, padded to one 64-wide GEMM tile
constexpr int kRows = 64;     // batch rows are padded to a multiple of this
constexpr int kLayers = 4;
constexpr int kSplitK = 1024; // K per workgroup in the weight-gradient GEMMs

// Packed fp32 parameter vector: W1 (256 x 6), b1, W2 (256 x 256), b2,
// W3 (256 x 256), b3, W4 (8 x 256), b4; W[l] is (out x in), row-major.
constexpr int64_t kW1 = 0, kB1 = kW1 + kHidden * kIn;
constexpr int64_t kW2 = kB1 + kHidden, kB2 = kW2 + kHidden * kHidden;
constexpr int64_t kW3 = kB2 + kHidden, kB3 = kW3 + kHidden * kHidden;
constexpr int64_t kW4 = kB3 + kHidden, kB4 = kW4 + kOut * kHidden;
constexpr int64_t kParams = kB4 + kOut;  // 135,432

enum Epilogue { kEpiPlain = 0, kEpiBias = 1, kEpiBiasGelu = 2, kEpiGeluGrad = 3 };

// C[M x N] = A[M x K] . B[N x K]^T over k in [z * k_chunk, (z + 1) * k_chunk)
// for workgroup z; bf16 operands, K-contiguous rows; M, N multiples of 64,
// K and k_chunk multiples of 32.  Only C entries with m < m_store and
// n < n_store are stored.
struct GemmArgs {
    const uint16_t *A;
    const uint16_t *B;
    int32_t lda, ldb;
    int32_t M, N, K, k_chunk;
    int32_t m_store, n_store;
    float *C;             // fp32 result (plain / bias / pre-activation); partial z at C + z * c_split
    int64_t c_split;
    int32_t ldc;
    const float *bias;    // per column n
    uint16_t *out;        // bf16 activation or gradient, row-major
    int32_t ldo;
    uint16_t *out_t;      // its transpose (nullable for activations)
    int32_t ldot;
    const float *Z;       // pre-activation read by the GELU-gradient epilogue
    int32_t ldz;
};

// One segment of the packed parameter vector for the Adam kernel, with its
// bf16 copies (rows x cols, row-major with pitch ld16) and transposed copy
// (cols x rows, pitch ldt16).  Biases have no copies.
struct AdamSeg {
    int64_t begin;
    int32_t rows, cols;
    uint16_t *w16;
    int32_t ld16;
    uint16_t *w16_t;
    int32_t ldt16;
};

struct AdamArgs {
    float *param, *m, *v;
    const float *grad;
    int64_t n;
    // 1 - beta is passed separately: 1 - 0.999f in fp32 is 1.3e-5 off 0.001
    float lr, beta1, beta2, one_minus_beta1, one_minus_beta2, eps, c1, c2;  // c1, c2: bias corrections 1 - beta^t
    AdamSeg seg[2 * kLayers];
};

hipError_t launch_gemm(int epi, const GemmArgs &g, hipStream_t st);
hipError_t launch_split_reduce(const float *part, int splits, int64_t split_stride, int M, int N, int m_store,
                               int n_store, float *out, int ldo, hipStream_t st);
hipError_t launch_rowsum(const uint16_t *g_t, int rows, int n_pad, float *out, hipStream_t st);
hipError_t launch_input(const float *x, int n, int n_pad, const float *norm, uint16_t *out, uint16_t *out_t,
                        int ldot, hipStream_t st);
hipError_t launch_output(const float *y, int n, const float *norm, float *out, hipStream_t st);
hipError_t launch_loss(const float *y, const float *t, int n, int n_pad, const float *norm, uint16_t *g,
                       uint16_t *g_t, float *loss_rows, hipStream_t st);
hipError_t launch_loss_sum(const float *loss_rows, int n, float *out, hipStream_t st);
hipError_t launch_adam(const AdamArgs &a, hipStream_t st);
hipError_t launch_cast(const AdamSeg &s, const float *param, hipStream_t st);
hipError_t launch_fit_norm(const float *x, const float *t, int n, int log_mask, float *norm, hipStream_t st);
hipError_t launch_fill_u16(uint16_t *p, uint16_t v, int64_t n, hipStream_t st);
hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t st);

}  // namespace emu
}  // namespace cpm
