// HIP kernels around the sweep: counting volumes / surfaces from the lattice,
// centroid sums, activity decay, fills and counter copies.
#include "cpm_device.hpp"

namespace cpm {
namespace {

template <int D>
struct Geo {
    int L0, L1, L2;
    __device__ __forceinline__ int idx(int x, int y, int z) const { return x + L0 * (y + L1 * z); }
};

template <int D>
__global__ void __launch_bounds__(kBlock) count_kernel(SweepArgs a, int32_t *v_out, int32_t *s_out, int stride)
{
    const int64_t n_sites = (int64_t)a.L[0] * a.L[1] * a.L[2];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_sites) return;
    const int32_t c = a.lat[i];
    if (c <= 0) return;
    const Geo<D> g{a.L[0], a.L[1], a.L[2]};
    const int x = (int)(i % g.L0), y = (int)((i / g.L0) % g.L1), z = (int)(i / ((int64_t)g.L0 * g.L1));
    constexpr int NNB = D == 2 ? 8 : 26;
    int unlike = 0;
#pragma unroll
    for (int n = 0; n < NNB; ++n) {
        int dx, dy, dz;
        dx = nb_dx<D>(n); dy = nb_dy<D>(n); dz = nb_dz<D>(n);
        unlike += a.lat[g.idx(wrap_once(x + dx, g.L0), wrap_once(y + dy, g.L1), D == 3 ? wrap_once(z + dz, g.L2) : 0)] != c;
    }
    atomicAdd(&v_out[(size_t)c * stride], 1);
    atomicAdd(&s_out[(size_t)c * stride], unlike);
}

__global__ void fill_i32_kernel(int32_t *p, int32_t value, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = value;
}

__global__ void act_decay_kernel(uint8_t *act, size_t n)
{
    const size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 16;
    if (i + 16 <= n) {
        uint4 v = *reinterpret_cast<const uint4 *>(act + i);
        uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // per-byte saturating decrement
            uint32_t x = w[e];
            uint32_t nz = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu | x) & 0x80808080u;  // 0x80 where byte != 0
            w[e] = x - (nz >> 7);
        }
        *reinterpret_cast<uint4 *>(act + i) = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
        for (size_t j = i; j < n; ++j)
            if (act[j] > 0) act[j] = (uint8_t)(act[j] - 1);
    }
}

template <int D>
__global__ void __launch_bounds__(kBlock) centroid_ref_kernel(SweepArgs a, int32_t *ref)
{
    const int64_t n_sites = (int64_t)a.L[0] * a.L[1] * a.L[2];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_sites) return;
    const int32_t c = a.lat[i];
    if (c >= 1) atomicMin(&ref[c], (int32_t)i);
}

template <int D>
__global__ void __launch_bounds__(kBlock) centroid_sum_kernel(SweepArgs a, const int32_t *ref, int64_t *out)
{
    const int64_t n_sites = (int64_t)a.L[0] * a.L[1] * a.L[2];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_sites) return;
    const int32_t c = a.lat[i];
    if (c < 1) return;
    const int L[3] = {a.L[0], a.L[1], a.L[2]};
    const int p[3] = {(int)(i % L[0]), (int)((i / L[0]) % L[1]), (int)(i / ((int64_t)L[0] * L[1]))};
    const int r0 = ref[c];
    const int r[3] = {r0 % L[0], (r0 / L[0]) % L[1], r0 / (L[0] * L[1])};
#pragma unroll
    for (int d = 0; d < D; ++d) {
        int diff = p[d] - r[d];
        if (diff > L[d] / 2) diff -= L[d];
        if (diff < -(L[d] - 1) / 2) diff += L[d];
        atomicAdd(reinterpret_cast<unsigned long long *>(&out[(size_t)c * D + d]),
                  (unsigned long long)(int64_t)(r[d] + diff));
    }
}

__global__ void copy_counters_kernel(const int32_t *pairs, int32_t n_labels, int32_t *v_out, int32_t *s_out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_labels) return;
    v_out[i] = i == 0 ? 0 : pairs[2 * i];
    s_out[i] = i == 0 ? 0 : pairs[2 * i + 1];
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_fill_i32(int32_t *p, int32_t value, size_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    fill_i32_kernel<<<blocks_for(n), kBlock, 0, stream>>>(p, value, n);
    return hipGetLastError();
}

hipError_t launch_count(const SweepArgs &a, int ndim, int32_t *v_out, int32_t *s_out, int stride,
                        hipStream_t stream)
{
    const size_t n = (size_t)a.L[0] * a.L[1] * a.L[2];
    if (ndim == 2)
        count_kernel<2><<<blocks_for(n), kBlock, 0, stream>>>(a, v_out, s_out, stride);
    else
        count_kernel<3><<<blocks_for(n), kBlock, 0, stream>>>(a, v_out, s_out, stride);
    return hipGetLastError();
}

hipError_t launch_act_decay(uint8_t *act, size_t n, hipStream_t stream)
{
    const size_t threads = (n + 15) / 16;
    act_decay_kernel<<<blocks_for(threads), kBlock, 0, stream>>>(act, n);
    return hipGetLastError();
}

hipError_t launch_centroids(const SweepArgs &a, int ndim, int32_t n_cells, int32_t *ref, int64_t *out,
                            hipStream_t stream)
{
    const size_t n = (size_t)a.L[0] * a.L[1] * a.L[2];
    hipError_t e = launch_fill_i32(ref, INT32_MAX, (size_t)n_cells + 1, stream);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(reinterpret_cast<int32_t *>(out), 0, ((size_t)n_cells + 1) * ndim * 2, stream);
    if (e != hipSuccess) return e;
    if (ndim == 2) {
        centroid_ref_kernel<2><<<blocks_for(n), kBlock, 0, stream>>>(a, ref);
        centroid_sum_kernel<2><<<blocks_for(n), kBlock, 0, stream>>>(a, ref, out);
    } else {
        centroid_ref_kernel<3><<<blocks_for(n), kBlock, 0, stream>>>(a, ref);
        centroid_sum_kernel<3><<<blocks_for(n), kBlock, 0, stream>>>(a, ref, out);
    }
    return hipGetLastError();
}

hipError_t launch_copy_counters(const int32_t *pairs, int32_t n_labels, int32_t *v_out, int32_t *s_out,
                                hipStream_t stream)
{
    copy_counters_kernel<<<blocks_for((size_t)n_labels), kBlock, 0, stream>>>(pairs, n_labels, v_out, s_out);
    return hipGetLastError();
}

}  // namespace cpm
