// HIP kernels of the CPM sweep for gfx950.
//
// One launch of `activation_kernel` runs one activation of the checkerboard
// scheme (paper, Results, "Designing a parallel execution scheme", Fig. 2A):
// one thread per thread area makes k copy attempts inside the area's
// sub-area of the active colour.  Per-cell counters are double buffered:
// activation g reads buffer g&1 and adds both its own deltas and those of
// activation g-1 into buffer (g+1)&1, so buffer g&1 always holds the exact
// state at the start of activation g while the other holds that of g-1.
#include "cpm_internal.hpp"

namespace cpm {
namespace {

constexpr int kBlock = 256;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ int wrap(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

template <int D>
struct Geo {
    int L0, L1, L2;
    __device__ __forceinline__ int idx(int x, int y, int z) const { return x + L0 * (y + L1 * z); }
};

// Moore offset n (lexicographic, z slowest, x fastest, zero left out).
template <int D>
__device__ __forceinline__ void moore_offset(int n, int &dx, int &dy, int &dz)
{
    if (D == 2) {
        const int m = n < 4 ? n : n + 1;  // skip the centre of the 3x3 block
        dx = m % 3 - 1;
        dy = m / 3 - 1;
        dz = 0;
    } else {
        const int m = n < 13 ? n : n + 1;  // skip the centre of the 3x3x3 block
        dx = m % 3 - 1;
        dy = (m / 3) % 3 - 1;
        dz = m / 9 - 1;
    }
}

__device__ __forceinline__ int type_of(const SweepArgs &a, int32_t label)
{
    return label < 0 ? a.obstacle_type : a.cell_type[label];
}

// exp(l * 2^-24) * 2^16, floor-composed from the split tables.
__device__ __forceinline__ int64_t gm_from_log(const DeviceModel *m, uint64_t ell)
{
    const uint64_t p1 = (m->EH[ell >> 16] * m->EM[(ell >> 8) & 255]) >> 31;
    const uint64_t p2 = (p1 * m->EL[ell & 255]) >> 30;
    return (int64_t)(p2 >> 8);
}

// Geometric mean of the activity over site (x,y,z) and its Moore neighbours
// of the same cell (eq. 8), 2^16 fixed point; 0 for medium, obstacles,
// non-motile cells and when any activity in the set is 0.
template <int D>
__device__ int64_t gm_act(const SweepArgs &a, const Geo<D> &g, int x, int y, int z)
{
    const int c0 = g.idx(x, y, z);
    const int32_t cell = a.lat[c0];
    if (cell <= 0) return 0;
    const DeviceModel *m = a.model;
    if (m->max_act[a.cell_type[cell]] <= 0) return 0;
    const uint32_t a0 = a.act[c0];
    if (a0 == 0) return 0;
    uint64_t sum = (uint64_t)m->LG[a0];
    uint32_t cnt = 1;
    constexpr int NNB = D == 2 ? 8 : 26;
#pragma unroll
    for (int n = 0; n < NNB; ++n) {
        int dx, dy, dz;
        moore_offset<D>(n, dx, dy, dz);
        const int u = g.idx(wrap(x + dx, g.L0), wrap(y + dy, g.L1), D == 3 ? wrap(z + dz, g.L2) : 0);
        if (a.lat[u] != cell) continue;
        const uint32_t au = a.act[u];
        if (au == 0) return 0;
        sum += (uint64_t)m->LG[au];
        ++cnt;
    }
    return gm_from_log(m, sum / cnt);
}

__device__ __forceinline__ bool metropolis(const DeviceModel *m, int64_t q, uint32_t u)
{
    if (q <= 0) return true;
    const uint64_t h = (uint64_t)q >> 16;
    if (h >= (uint64_t)m->n_ti) return false;
    uint64_t thr;
    if ((q & 0xFFFF) == 0) {
        thr = m->TI[h];
    } else {
        // TM * TL < 2^64 whenever (m, l) != (0, 0); floor(TI * P / 2^64) exactly.
        const uint64_t p = m->TM[(q >> 8) & 255] * m->TL[q & 255];
        thr = __umul64hi(m->TI[h], p);
    }
    return (uint64_t)u < thr;
}

__device__ __forceinline__ void add_deltas(int32_t *wr, int4 d)
{
    if (d.x == d.y) return;  // no accepted copy recorded
    if (d.x >= 1) {
        atomicAdd(&wr[2 * d.x], -1);
        atomicAdd(&wr[2 * d.x + 1], d.z);
    }
    if (d.y >= 1) {
        atomicAdd(&wr[2 * d.y], 1);
        atomicAdd(&wr[2 * d.y + 1], d.w);
    }
}

template <int D, bool ACT>
__global__ void __launch_bounds__(kBlock) activation_kernel(SweepArgs a, uint32_t mcs, uint32_t alpha,
                                                            int parity)
{
    const uint32_t area = blockIdx.x * kBlock + threadIdx.x;
    if (area >= a.n_areas) return;
    const int32_t *rd = a.counters[parity];
    int32_t *wr = a.counters[parity ^ 1];
    const DeviceModel *m = a.model;
    const Geo<D> g{a.L[0], a.L[1], a.L[2]};
    const int k = a.k;
    int4 *prev = a.prev + (size_t)area * k;

    // deltas of the previous activation go into the write buffer too
    for (int j = 0; j < k; ++j) add_deltas(wr, prev[j]);

    const int ax = area % a.na[0];
    const int ay = (area / a.na[0]) % a.na[1];
    const int az = D == 3 ? area / (a.na[0] * a.na[1]) : 0;
    const uint32_t phi = alpha & ((1u << D) - 1);
    const int s = a.s;
    const int bx = 2 * s * ax + s * (int)(phi & 1);
    const int by = 2 * s * ay + s * (int)((phi >> 1) & 1);
    const int bz = D == 3 ? 2 * s * az + s * (int)((phi >> 2) & 1) : 0;
    const uint32_t sd = D == 2 ? (uint32_t)(s * s) : (uint32_t)(s * s * s);
    constexpr int NNB = D == 2 ? 8 : 26;

    for (int j = 0; j < k; ++j) {
        const uint4 u = philox(make_uint4(area, mcs, (alpha << 8) | (uint32_t)j, a.lattice_id), a.key0, a.key1);
        const uint32_t o = (uint32_t)(((uint64_t)u.x * sd) >> 32);
        const int tx = bx + (int)(o % (uint32_t)s);
        const int ty = by + (int)((o / (uint32_t)s) % (uint32_t)s);
        const int tz = D == 3 ? bz + (int)(o / (uint32_t)(s * s)) : 0;
        const int nsel = (int)(((uint64_t)u.y * NNB) >> 32);
        int ndx, ndy, ndz;
        moore_offset<D>(nsel, ndx, ndy, ndz);
        const int sx = wrap(tx + ndx, g.L0), sy = wrap(ty + ndy, g.L1);
        const int sz = D == 3 ? wrap(tz + ndz, g.L2) : 0;
        const int t = g.idx(tx, ty, tz);
        const int32_t lt = a.lat[t];
        const int32_t ls = a.lat[g.idx(sx, sy, sz)];
        int4 rec = make_int4(0, 0, 0, 0);
        if (lt != ls && lt >= 0 && ls >= 0) {
            const int tt = type_of(a, lt), ts = type_of(a, ls);
            int64_t adh = 0;
            int k_old = 0, k_new = 0;
#pragma unroll
            for (int n = 0; n < NNB; ++n) {
                int dx, dy, dz;
                moore_offset<D>(n, dx, dy, dz);
                const int uidx = g.idx(wrap(tx + dx, g.L0), wrap(ty + dy, g.L1),
                                       D == 3 ? wrap(tz + dz, g.L2) : 0);
                const int32_t lu = a.lat[uidx];
                const int tu = type_of(a, lu);
                if (lu != ls) adh += m->J[ts * kMaxTypes + tu];
                if (lu != lt) adh -= m->J[tt * kMaxTypes + tu];
                k_old += lu == lt;
                k_new += lu == ls;
            }
            const int64_t dso = 2 * k_old - NNB;
            const int64_t dsn = NNB - 2 * k_new;
            int64_t q = adh;
            if (lt >= 1) {
                int64_t v = rd[2 * lt], sf = rd[2 * lt + 1];
                for (int jj = 0; jj < j; ++jj) {  // this thread's own earlier deltas
                    const int4 e = prev[jj];
                    if (e.x == lt) { v -= 1; sf += e.z; }
                    if (e.y == lt) { v += 1; sf += e.w; }
                }
                q += m->lam_v[tt] * (1 - 2 * (v - m->v_target[tt]));
                q += m->lam_s[tt] * (2 * dso * (sf - m->s_target[tt]) + dso * dso);
            }
            if (ls >= 1) {
                int64_t v = rd[2 * ls], sf = rd[2 * ls + 1];
                for (int jj = 0; jj < j; ++jj) {
                    const int4 e = prev[jj];
                    if (e.x == ls) { v -= 1; sf += e.z; }
                    if (e.y == ls) { v += 1; sf += e.w; }
                }
                q += m->lam_v[ts] * (2 * (v - m->v_target[ts]) + 1);
                q += m->lam_s[ts] * (2 * dsn * (sf - m->s_target[ts]) + dsn * dsn);
            }
            if (ACT) {
                const int64_t gt = gm_act<D>(a, g, tx, ty, tz);
                const int64_t gs = gm_act<D>(a, g, sx, sy, sz);
                const int64_t rt = lt >= 1 ? m->r_act[tt] : 0;
                const int64_t rs = ls >= 1 ? m->r_act[ts] : 0;
                q += (rt * gt - rs * gs) >> 16;
            }
            if (metropolis(m, q, u.z)) {
                a.lat[t] = ls;
                if (ACT) a.act[t] = (ls >= 1 && m->max_act[ts] > 0) ? (uint8_t)m->max_act[ts] : (uint8_t)0;
                rec = make_int4(lt, ls, (int)dso, (int)dsn);
                add_deltas(wr, rec);
            }
        }
        prev[j] = rec;
    }
}

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
        moore_offset<D>(n, dx, dy, dz);
        unlike += a.lat[g.idx(wrap(x + dx, g.L0), wrap(y + dy, g.L1), D == 3 ? wrap(z + dz, g.L2) : 0)] != c;
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

hipError_t launch_activation(const SweepArgs &a, int ndim, bool act, uint32_t mcs, uint32_t alpha,
                             int parity, hipStream_t stream)
{
    const unsigned nb = blocks_for(a.n_areas);
    if (ndim == 2) {
        if (act)
            activation_kernel<2, true><<<nb, kBlock, 0, stream>>>(a, mcs, alpha, parity);
        else
            activation_kernel<2, false><<<nb, kBlock, 0, stream>>>(a, mcs, alpha, parity);
    } else {
        if (act)
            activation_kernel<3, true><<<nb, kBlock, 0, stream>>>(a, mcs, alpha, parity);
        else
            activation_kernel<3, false><<<nb, kBlock, 0, stream>>>(a, mcs, alpha, parity);
    }
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
