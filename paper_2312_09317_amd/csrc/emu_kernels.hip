// Kernels of the summary-statistics emulator: a 6 -> 256 -> 256 -> 256 -> 8
// MLP with the exact (erf) GELU after each hidden layer, bf16 operands on the
// gfx950 matrix cores with fp32 accumulation, fp32 master weights and Adam.
//
// One GEMM kernel serves every layer and pass: C[M x N] = A[M x K] . B[N x K]^T
// with both operands K-contiguous bf16.  A workgroup computes a 64 x 64 block
// of C with four waves, each a 32 x 32 quarter made of 2 x 2 tiles of
// v_mfma_f32_16x16x32_bf16.  For that instruction lane l supplies row l % 16
// of the A tile and column l % 16 of the B tile, eight consecutive k each
// (k block l / 16, the same for A and B, so the pairing of k between the two
// operands is fixed whatever order the unit adds them in), and receives rows
// 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16 of the 16 x 16 result.
#include "emu_internal.hpp"

namespace cpm {
namespace emu {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// GELU(z) = z Phi(z) with the standard normal distribution function Phi.
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

// d/dz z Phi(z) = Phi(z) + z phi(z).
__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    bf16x8 r;
    __builtin_memcpy(&r, &v, 16);
    return r;
}

template <int EPI>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int n0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const int k_begin = blockIdx.z * g.k_chunk;
    const int k_end = min(g.K, k_begin + g.k_chunk);
    f32x4 acc00 = {0.f, 0.f, 0.f, 0.f}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
    const uint16_t *a0 = g.A + (size_t)(m0 + r) * g.lda + kq;
    const uint16_t *a1 = a0 + (size_t)16 * g.lda;
    const uint16_t *b0 = g.B + (size_t)(n0 + r) * g.ldb + kq;
    const uint16_t *b1 = b0 + (size_t)16 * g.ldb;
    for (int k = k_begin; k < k_end; k += 32) {
        const bf16x8 x0 = load8(a0 + k), x1 = load8(a1 + k);
        const bf16x8 y0 = load8(b0 + k), y1 = load8(b1 + k);
        acc00 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, y0, acc00, 0, 0, 0);
        acc01 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, y1, acc01, 0, 0, 0);
        acc10 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, y0, acc10, 0, 0, 0);
        acc11 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, y1, acc11, 0, 0, 0);
    }
    float *C = g.C ? g.C + (size_t)blockIdx.z * g.c_split : nullptr;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x4 acc = t == 0 ? acc00 : t == 1 ? acc01 : t == 2 ? acc10 : acc11;
        const int n = n0 + 16 * (t & 1) + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = m0 + 16 * (t >> 1) + (lane >> 4) * 4 + e;
            if (m >= g.m_store || n >= g.n_store) continue;
            const float v = acc[e];
            if (EPI == kEpiPlain) {
                C[(size_t)m * g.ldc + n] = v;
            } else if (EPI == kEpiBias) {
                C[(size_t)m * g.ldc + n] = v + g.bias[n];
            } else if (EPI == kEpiBiasGelu) {
                const float z = v + g.bias[n];
                if (C) C[(size_t)m * g.ldc + n] = z;  // kept for the backward pass
                const uint16_t y = to_bf16(gelu(z));
                g.out[(size_t)m * g.ldo + n] = y;
                if (g.out_t) g.out_t[(size_t)n * g.ldot + m] = y;
            } else {  // v = dL/da; dL/dz = dL/da * GELU'(z)
                const uint16_t d = to_bf16(v * gelu_grad(g.Z[(size_t)m * g.ldz + n]));
                g.out[(size_t)m * g.ldo + n] = d;
                g.out_t[(size_t)n * g.ldot + m] = d;
            }
        }
    }
}

// out[m, n] = sum over z of part[z][m, n] (m < m_store, n < n_store), in z order.
__global__ void split_reduce_kernel(const float *part, int splits, int64_t stride, int N, int m_store, int n_store,
                                    float *out, int ldo)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)m_store * n_store) return;
    const int m = (int)(i / n_store), n = (int)(i - (int64_t)m * n_store);
    const float *p = part + (size_t)m * N + n;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += p[(size_t)z * stride];
    out[(size_t)m * ldo + n] = s;
}

// out[r] = sum over i < n_pad of g_t[r, i]: bias gradients from the transposed dL/dz.
__global__ void __launch_bounds__(256) rowsum_kernel(const uint16_t *g_t, int n_pad, float *out)
{
    __shared__ float red[256];
    const uint16_t *row = g_t + (size_t)blockIdx.x * n_pad;
    float s = 0.f;
    for (int i = threadIdx.x; i < n_pad; i += 256) s += from_bf16(row[i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Raw inputs -> z-scored bf16 rows, zero-padded to kInPad columns and n_pad
// rows, and (optionally) the transposed copy, kOutPad rows of pitch ldot (the
// N of the first layer's weight-gradient product).
__global__ void input_kernel(const float *x, int n, int n_pad, const float *norm, uint16_t *out, uint16_t *out_t,
                             int ldot)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    for (int c = 0; c < kOutPad; ++c) {
        float v = 0.f;
        if (i < n && c < kIn) v = (x[(size_t)i * kIn + c] - norm[c]) / norm[kIn + c];
        const uint16_t b = to_bf16(v);
        if (c < kInPad) out[(size_t)i * kInPad + c] = b;
        if (out_t) out_t[(size_t)c * ldot + i] = b;
    }
}

// Target transform of output c: log(t + off) when its offset is positive.
__device__ __forceinline__ float to_target_space(float t, float off) { return off > 0.f ? logf(t + off) : t; }
__device__ __forceinline__ float from_target_space(float u, float off) { return off > 0.f ? expf(u) - off : u; }

// Normalised outputs (pitch kOut) -> raw outputs.
__global__ void output_kernel(const float *y, int n, const float *norm, float *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *mean = norm + 2 * kIn, *sd = mean + kOut, *off = sd + kOut;
    for (int c = 0; c < kOut; ++c)
        out[(size_t)i * kOut + c] = from_target_space(y[(size_t)i * kOut + c] * sd[c] + mean[c], off[c]);
}

// Mean squared error over the n x 8 normalised outputs: dL/dy = 2 (y - t) / (8 n)
// as bf16 rows (pitch kOutPad, zero beyond column 8 and row n) and their
// transpose (pitch n_pad), and the per-row squared error.
__global__ void loss_kernel(const float *y, const float *t_raw, int n, int n_pad, const float *norm, uint16_t *g,
                            uint16_t *g_t, float *loss_rows)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    const float *mean = norm + 2 * kIn, *sd = mean + kOut, *off = sd + kOut;
    const float scale = 2.0f / (float)((int64_t)n * kOut);
    float l = 0.f;
    for (int c = 0; c < kOutPad; ++c) {
        float d = 0.f;
        if (i < n && c < kOut) {
            const float t = (to_target_space(t_raw[(size_t)i * kOut + c], off[c]) - mean[c]) / sd[c];
            const float e = y[(size_t)i * kOut + c] - t;
            l += e * e;
            d = scale * e;
        }
        const uint16_t b = to_bf16(d);
        g[(size_t)i * kOutPad + c] = b;
        g_t[(size_t)c * n_pad + i] = b;
    }
    if (i < n) loss_rows[i] = l;
}

__global__ void __launch_bounds__(256) loss_sum_kernel(const float *loss_rows, int n, float *out)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += loss_rows[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] / (float)((int64_t)n * kOut);
}

__device__ __forceinline__ void write_copies(const AdamSeg &s, int64_t j, float p)
{
    if (!s.w16) return;
    const int o = (int)(j / s.cols), c = (int)(j - (int64_t)o * s.cols);
    const uint16_t b = to_bf16(p);
    s.w16[(size_t)o * s.ld16 + c] = b;
    if (s.w16_t) s.w16_t[(size_t)c * s.ldt16 + o] = b;
}

// Adam with bias correction on the fp32 master parameters, then the bf16 copies.
__global__ void adam_kernel(AdamArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const float g = a.grad[i];
    const float m = a.beta1 * a.m[i] + a.one_minus_beta1 * g;
    const float v = a.beta2 * a.v[i] + a.one_minus_beta2 * g * g;
    a.m[i] = m;
    a.v[i] = v;
    const float p = a.param[i] - a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
    a.param[i] = p;
    int s = 0;
    while (s + 1 < 2 * kLayers && i >= a.seg[s + 1].begin) ++s;
    write_copies(a.seg[s], i - a.seg[s].begin, p);
}

__global__ void cast_kernel(AdamSeg s, const float *param)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (int64_t)s.rows * s.cols) return;
    write_copies(s, j, param[s.begin + j]);
}

__device__ void block_sums(double &s1, double &s2, double *r1, double *r2)
{
    r1[threadIdx.x] = s1;
    r2[threadIdx.x] = s2;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            r1[threadIdx.x] += r1[threadIdx.x + k];
            r2[threadIdx.x] += r2[threadIdx.x + k];
        }
        __syncthreads();
    }
    s1 = r1[0];
    s2 = r2[0];
    __syncthreads();
}

// Column means and population standard deviations (FP64 sums) of the inputs
// (6 columns) and the targets (8 columns), the targets of the columns set in
// log_mask first mapped to log(t + off) with off = G / 100, G the geometric
// mean of the column's positive values (off = 1 if it has none):
// norm = [mean_x, sd_x, mean_t, sd_t, off_t].  The offset follows the bulk
// of a column that spans decades, where its arithmetic mean follows the
// largest values.
// A column with zero spread gets sd = 1.
__global__ void __launch_bounds__(256) fit_norm_kernel(const float *x, const float *t, int n, int log_mask,
                                                       float *norm)
{
    __shared__ double r1[256], r2[256];
    const int col = blockIdx.x;  // 0..13
    const bool is_x = col < kIn;
    const float *src = is_x ? x : t;
    const int c = is_x ? col : col - kIn;
    const int w = is_x ? kIn : kOut;
    const bool logt = !is_x && ((log_mask >> c) & 1);
    float off = 0.f;
    if (logt) {
        double s1 = 0.0, s2 = 0.0;  // sum of log t and count over t > 0
        for (int i = threadIdx.x; i < n; i += 256) {
            const float v = src[(size_t)i * w + c];
            if (v > 0.f) {
                s1 += log((double)v);
                s2 += 1.0;
            }
        }
        block_sums(s1, s2, r1, r2);
        off = s2 > 0.0 ? (float)(exp(s1 / s2) / 100.0) : 1.f;
    }
    double s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const float raw = src[(size_t)i * w + c];
        const double v = (double)(logt ? to_target_space(raw, off) : raw);
        s1 += v;
        s2 += v * v;
    }
    block_sums(s1, s2, r1, r2);
    if (threadIdx.x == 0) {
        const double mean = s1 / n;
        const double var = fmax(s2 / n - mean * mean, 0.0);
        const double sd = var > 0.0 ? sqrt(var) : 1.0;
        const int base = is_x ? 0 : 2 * kIn;
        norm[base + c] = (float)mean;
        norm[base + w + c] = (float)sd;
        if (!is_x) norm[2 * kIn + 2 * kOut + c] = off;
    }
}

__global__ void fill_u16_kernel(uint16_t *p, uint16_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_f32_kernel(float *p, float v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_gemm(int epi, const GemmArgs &g, hipStream_t st)
{
    const dim3 grid(g.M / 64, g.N / 64, (g.K + g.k_chunk - 1) / g.k_chunk);
    switch (epi) {
    case kEpiPlain: gemm_kernel<kEpiPlain><<<grid, 256, 0, st>>>(g); break;
    case kEpiBias: gemm_kernel<kEpiBias><<<grid, 256, 0, st>>>(g); break;
    case kEpiBiasGelu: gemm_kernel<kEpiBiasGelu><<<grid, 256, 0, st>>>(g); break;
    default: gemm_kernel<kEpiGeluGrad><<<grid, 256, 0, st>>>(g); break;
    }
    return hipGetLastError();
}

hipError_t launch_split_reduce(const float *part, int splits, int64_t split_stride, int M, int N, int m_store,
                               int n_store, float *out, int ldo, hipStream_t st)
{
    (void)M;
    split_reduce_kernel<<<blocks((int64_t)m_store * n_store, 256), 256, 0, st>>>(part, splits, split_stride, N,
                                                                                 m_store, n_store, out, ldo);
    return hipGetLastError();
}

hipError_t launch_rowsum(const uint16_t *g_t, int rows, int n_pad, float *out, hipStream_t st)
{
    rowsum_kernel<<<rows, 256, 0, st>>>(g_t, n_pad, out);
    return hipGetLastError();
}

hipError_t launch_input(const float *x, int n, int n_pad, const float *norm, uint16_t *out, uint16_t *out_t,
                        int ldot, hipStream_t st)
{
    input_kernel<<<blocks(n_pad, 256), 256, 0, st>>>(x, n, n_pad, norm, out, out_t, ldot);
    return hipGetLastError();
}

hipError_t launch_output(const float *y, int n, const float *norm, float *out, hipStream_t st)
{
    output_kernel<<<blocks(n, 256), 256, 0, st>>>(y, n, norm, out);
    return hipGetLastError();
}

hipError_t launch_loss(const float *y, const float *t, int n, int n_pad, const float *norm, uint16_t *g,
                       uint16_t *g_t, float *loss_rows, hipStream_t st)
{
    loss_kernel<<<blocks(n_pad, 256), 256, 0, st>>>(y, t, n, n_pad, norm, g, g_t, loss_rows);
    return hipGetLastError();
}

hipError_t launch_loss_sum(const float *loss_rows, int n, float *out, hipStream_t st)
{
    loss_sum_kernel<<<1, 256, 0, st>>>(loss_rows, n, out);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t st)
{
    adam_kernel<<<blocks(a.n, 256), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_cast(const AdamSeg &s, const float *param, hipStream_t st)
{
    cast_kernel<<<blocks((int64_t)s.rows * s.cols, 256), 256, 0, st>>>(s, param);
    return hipGetLastError();
}

hipError_t launch_fit_norm(const float *x, const float *t, int n, int log_mask, float *norm, hipStream_t st)
{
    fit_norm_kernel<<<kIn + kOut, 256, 0, st>>>(x, t, n, log_mask, norm);
    return hipGetLastError();
}

hipError_t launch_fill_u16(uint16_t *p, uint16_t v, int64_t n, hipStream_t st)
{
    if (n > 0) fill_u16_kernel<<<blocks(n, 256), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t st)
{
    if (n > 0) fill_f32_kernel<<<blocks(n, 256), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}

}  // namespace emu
}  // namespace cpm
