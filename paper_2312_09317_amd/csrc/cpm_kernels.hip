// HIP kernels around the sweep: counting volumes / surfaces from the lattice,
// centroid sums, activity decay, fills and counter copies.
#include <algorithm>
#include <type_traits>

#include "cpm_device.hpp"

namespace cpm {
namespace {

// Per-workgroup label map in LDS: sums per cell label are combined in LDS
// and flushed with one global atomic per label and workgroup.  A label that
// finds no free slot within kProbe probes goes straight to global memory.
constexpr int kMapSize = 1024;
constexpr int kProbe = 32;
constexpr int kSitesPerThread = 16;
constexpr int kSitesPerBlock = kBlock * kSitesPerThread;

// Brick of the run-based reductions: kTX threads of kSitesPerThread sites
// along x, kY rows, kZ planes (kTX * kY * kZ = kBlock).
template <int D>
struct ReduceBrick {
    static constexpr int kTX = D == 3 ? 1 : 4;
    static constexpr int kY = D == 3 ? 16 : 64;
    static constexpr int kZ = D == 3 ? 16 : 1;
    static constexpr int kX = kTX * kSitesPerThread;
    static_assert(kTX * kY * kZ == kBlock, "one thread per brick row segment");
};

template <int D>
__host__ __device__ inline int64_t reduce_bricks(const int *L)
{
    using B = ReduceBrick<D>;
    return (int64_t)((L[0] + B::kX - 1) / B::kX) * ((L[1] + B::kY - 1) / B::kY) * ((L[2] + B::kZ - 1) / B::kZ);
}

enum ReduceMode { kCount = 0, kRef = 1, kCentroid = 2 };

struct LabelMap {
    int32_t key[kMapSize];
    int32_t a[kMapSize];                // volume, or minimum site index
    int32_t b[kMapSize];                // surface
    unsigned long long c[kMapSize][3];  // centroid sums
};

__device__ __forceinline__ int map_slot(LabelMap &m, int label)
{
    uint32_t h = ((uint32_t)label * 2654435761u) & (kMapSize - 1);
    for (int p = 0; p < kProbe; ++p) {
        const int k = atomicCAS(&m.key[h], -1, label);
        if (k == -1 || k == label) return (int)h;
        h = (h + 1) & (kMapSize - 1);
    }
    return -1;
}

// The kSitesPerThread consecutive labels from site i0 (n of them valid),
// vector loads where the row of them is whole and 16-byte aligned.
// A label from an int32 lattice word: the label itself, or a packed word.
template <int WORDS>
__device__ __forceinline__ int word_label(int32_t v)
{
    if (WORDS == kWordsPacked) return label_of((uint32_t)v);
    if (WORDS == kWordsPackedAct) return label_of((char32_t)(uint32_t)v);
    return v;
}

template <int WORDS>
__device__ __forceinline__ void load_run_labels(const SweepArgs &a, int64_t i0, int n, int (&lab)[kSitesPerThread])
{
    static_assert(kSitesPerThread == 16, "vector loads below assume 16 sites per thread");
    if (WORDS == kWords16) {
        const uint16_t *src = reinterpret_cast<const uint16_t *>(a.cells) + i0;
        if (n == kSitesPerThread && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
            const uint4 v[2] = {reinterpret_cast<const uint4 *>(src)[0], reinterpret_cast<const uint4 *>(src)[1]};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t w = (&v[k >> 2].x)[k & 3];
                lab[2 * k] = label_of((uint16_t)(w & 0xFFFFu));
                lab[2 * k + 1] = label_of((uint16_t)(w >> 16));
            }
        } else {
#pragma unroll
            for (int k = 0; k < kSitesPerThread; ++k) lab[k] = k < n ? label_of(src[k]) : 0;
        }
    } else {
        const int32_t *src = a.lat + i0;
        if (n == kSitesPerThread && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int4 v = reinterpret_cast<const int4 *>(src)[k];
                lab[4 * k] = word_label<WORDS>(v.x);
                lab[4 * k + 1] = word_label<WORDS>(v.y);
                lab[4 * k + 2] = word_label<WORDS>(v.z);
                lab[4 * k + 3] = word_label<WORDS>(v.w);
            }
        } else {
#pragma unroll
            for (int k = 0; k < kSitesPerThread; ++k) lab[k] = k < n ? word_label<WORDS>(src[k]) : 0;
        }
    }
}

// One workgroup's share of a reduction over lattice a, read from its int32
// labels, its 16-bit working copy or its packed words (WORDS).  kCount
// (int32 labels only): kSitesPerBlock sites
// from `block`, thread t taking sites t, t + kBlock, ... (its neighbours'
// reads coalesce).  kRef, kCentroid: brick `block` (ReduceBrick), thread t
// taking kSitesPerThread consecutive sites of one row and touching the label
// map once per run of one label: at the run's first site (the smallest index
// of the run) for kRef, with the run's summed coordinates for kCentroid.
// Bricks rather than row strips keep the workgroups that see one cell, and
// so the global atomics per cell, few.
template <int D, int MODE, int WORDS = kWords32>
__device__ __forceinline__ void reduce_block(const SweepArgs &a, int64_t block, int32_t *v_out, int32_t *s_out,
                                             int stride, int32_t *ref, int64_t *cent)
{
    __shared__ LabelMap m;
    const int tid = threadIdx.x;
    for (int i = tid; i < kMapSize; i += kBlock) {
        m.key[i] = -1;
        m.a[i] = MODE == kRef ? INT32_MAX : 0;
        m.b[i] = 0;
        m.c[i][0] = m.c[i][1] = m.c[i][2] = 0;
    }
    __syncthreads();
    const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2];
    const int64_t n_sites = (int64_t)L0 * L1 * L2;
    const int64_t base = block * kSitesPerBlock;
    constexpr int NNB = D == 2 ? 8 : 26;
    if (MODE == kCount) {
        for (int j = 0; j < kSitesPerThread; ++j) {
            const int64_t i = base + tid + (int64_t)j * kBlock;
            if (i >= n_sites) break;
            const int32_t c = a.lat[i];
            if (c <= 0) continue;
            const int x = (int)(i % L0), y = (int)((i / L0) % L1), z = (int)(i / ((int64_t)L0 * L1));
            const int slot = map_slot(m, c);
            int unlike = 0;
#pragma unroll
            for (int n = 0; n < NNB; ++n) {
                const int u = wrap_once(x + nb_dx<D>(n), L0) +
                              L0 * (wrap_once(y + nb_dy<D>(n), L1) + L1 * (D == 3 ? wrap_once(z + nb_dz<D>(n), L2) : 0));
                unlike += a.lat[u] != c;
            }
            if (slot >= 0) {
                atomicAdd(&m.a[slot], 1);
                atomicAdd(&m.b[slot], unlike);
            } else {
                atomicAdd(&v_out[(size_t)c * stride], 1);
                atomicAdd(&s_out[(size_t)c * stride], unlike);
            }
        }
    } else {
        using B = ReduceBrick<D>;
        const int nbx = (L0 + B::kX - 1) / B::kX, nby = (L1 + B::kY - 1) / B::kY;
        const int bx = (int)(block % nbx), by = (int)((block / nbx) % nby), bz = (int)(block / ((int64_t)nbx * nby));
        const int tx = tid % B::kTX, ty = (tid / B::kTX) % B::kY, tz = tid / (B::kTX * B::kY);
        int x = bx * B::kX + tx * kSitesPerThread;
        const int y = by * B::kY + ty, z = bz * B::kZ + tz;
        if (x < L0 && y < L1 && z < L2) {
            const int n = min(kSitesPerThread, L0 - x);
            const int first = (z * L1 + y) * L0 + x;  // lattices hold fewer than 2^31 sites
            int lab[kSitesPerThread];
            load_run_labels<WORDS>(a, first, n, lab);
            int cur = INT32_MIN;  // label of the open run
            int r[3] = {0, 0, 0};
            int64_t acc[3] = {0, 0, 0};
            auto flush = [&]() {
                const int slot = map_slot(m, cur);
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    if (slot >= 0) atomicAdd(&m.c[slot][d], (unsigned long long)acc[d]);
                    else atomicAdd(reinterpret_cast<unsigned long long *>(&cent[(size_t)cur * D + d]),
                                   (unsigned long long)acc[d]);
                }
            };
            const int L[3] = {L0, L1, L2};
#pragma unroll
            for (int j = 0; j < kSitesPerThread; ++j) {
                if (j < n) {
                    const int c = lab[j];
                    if (c != cur) {
                        if (MODE == kCentroid && cur > 0) flush();
                        cur = c;
                        if (c > 0 && MODE == kRef) {
                            const int slot = map_slot(m, c);
                            if (slot >= 0) atomicMin(&m.a[slot], first + j);
                            else atomicMin(&ref[c], first + j);
                        } else if (c > 0) {
                            const int r0 = ref[c];
                            r[0] = r0 % L0;
                            r[1] = (r0 / L0) % L1;
                            r[2] = r0 / (L0 * L1);
                            acc[0] = acc[1] = acc[2] = 0;
                        }
                    }
                    if (MODE == kCentroid && c > 0) {
                        const int p[3] = {x, y, z};
#pragma unroll
                        for (int d = 0; d < D; ++d) {
                            int diff = p[d] - r[d];
                            if (diff > L[d] / 2) diff -= L[d];
                            if (diff < -(L[d] - 1) / 2) diff += L[d];
                            acc[d] += r[d] + diff;
                        }
                    }
                    ++x;
                }
            }
            if (MODE == kCentroid && cur > 0) flush();
        }
    }
    __syncthreads();
    for (int h = tid; h < kMapSize; h += kBlock) {
        const int c = m.key[h];
        if (c < 0) continue;
        if (MODE == kCount) {
            atomicAdd(&v_out[(size_t)c * stride], m.a[h]);
            atomicAdd(&s_out[(size_t)c * stride], m.b[h]);
        } else if (MODE == kRef) {
            atomicMin(&ref[c], m.a[h]);
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d)
                atomicAdd(reinterpret_cast<unsigned long long *>(&cent[(size_t)c * D + d]), m.c[h][d]);
        }
    }
}

template <int D, int MODE, int WORDS = kWords32>
__global__ void __launch_bounds__(kBlock) reduce_kernel(SweepArgs a, int32_t *v_out, int32_t *s_out, int stride,
                                                        int32_t *ref, int64_t *cent)
{
    static_assert(WORDS == kWords32 || MODE != kCount, "counts read the int32 labels");
    reduce_block<D, MODE, WORDS>(a, blockIdx.x, v_out, s_out, stride, ref, cent);
}

// Every lattice of a batch in one launch: blockIdx.y is the lattice, outputs
// are packed per label (label_off) as in the batch's per-cell arrays.
template <int D, int MODE>
__global__ void __launch_bounds__(kBlock) batch_reduce_kernel(const SweepArgs *args, const int64_t *label_off,
                                                              int32_t *v_out, int32_t *s_out, int32_t *ref,
                                                              int64_t *cent)
{
    const SweepArgs &a = args[blockIdx.y];
    const int64_t n_sites = (int64_t)a.L[0] * a.L[1] * a.L[2];
    if (MODE == kCount ? (int64_t)blockIdx.x * kSitesPerBlock >= n_sites : blockIdx.x >= reduce_bricks<D>(a.L))
        return;  // uniform over the block
    const int64_t o = label_off[blockIdx.y];
    reduce_block<D, MODE>(a, blockIdx.x, v_out ? v_out + o : nullptr, s_out ? s_out + o : nullptr, 1,
                          ref ? ref + o : nullptr, cent ? cent + o * D : nullptr);
}

// Ordered Moore pairs (x, y) of different labels, neither an obstacle, counted
// by (type of x, type of y); the medium is type 0.  Per-wave LDS histograms,
// one 64-bit global atomic per bin and workgroup.
template <int D>
__global__ void __launch_bounds__(kBlock) contact_kernel(SweepArgs a, unsigned long long *out, int n_types)
{
    constexpr int kBins = kMaxTypes * kMaxTypes;
    __shared__ uint32_t hist[kBlock / 64][kBins];
    const int tid = threadIdx.x, wave = tid >> 6;
    for (int i = tid; i < (kBlock / 64) * kBins; i += kBlock) (&hist[0][0])[i] = 0;
    __syncthreads();
    const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2];
    const int64_t n_sites = (int64_t)L0 * L1 * L2;
    const int64_t base = (int64_t)blockIdx.x * kSitesPerBlock;
    constexpr int NNB = D == 2 ? 8 : 26;
    for (int j = 0; j < kSitesPerThread; ++j) {
        const int64_t i = base + tid + (int64_t)j * kBlock;
        if (i >= n_sites) break;
        const int32_t c = a.lat[i];
        if (c < 0) continue;
        const int tc = c == 0 ? 0 : a.cell_type[c];
        const int x = (int)(i % L0), y = (int)((i / L0) % L1), z = (int)(i / ((int64_t)L0 * L1));
#pragma unroll
        for (int n = 0; n < NNB; ++n) {
            const int u = wrap_once(x + nb_dx<D>(n), L0) +
                          L0 * (wrap_once(y + nb_dy<D>(n), L1) + L1 * (D == 3 ? wrap_once(z + nb_dz<D>(n), L2) : 0));
            const int32_t lu = a.lat[u];
            if (lu == c || lu < 0) continue;
            const int tu = lu == 0 ? 0 : a.cell_type[lu];
            atomicAdd(&hist[wave][tc * kMaxTypes + tu], 1u);
        }
    }
    __syncthreads();
    for (int b = tid; b < kBins; b += kBlock) {
        const int ta = b / kMaxTypes, tb = b % kMaxTypes;
        if (ta >= n_types || tb >= n_types) continue;
        unsigned long long v = 0;
        for (int w = 0; w < kBlock / 64; ++w) v += hist[w][b];
        if (v) atomicAdd(&out[ta * n_types + tb], v);
    }
}

// floor(sqrt(n)) for 0 <= n < 2^62; the FP64 root is only a first guess
__device__ __forceinline__ int64_t isqrt_floor(int64_t n)
{
    if (n <= 0) return 0;
    int64_t r = (int64_t)sqrt((double)n);
    while (r > 0 && r * r > n) --r;
    while ((r + 1) * (r + 1) <= n) ++r;
    return r;
}

__device__ __forceinline__ int64_t div_floor(int64_t a, int64_t b)  // b > 0
{
    const int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

// One thread per label (label 0 untouched).  t == 0: initialise; t >= 1:
// update number t, writing history slot t mod slots and reading slot
// (t + 1) mod slots (the centroid of update t - dt, or the initial one).
__global__ void persist_kernel(PersistArgs p, int64_t t)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < 1 || c >= p.n_labels) return;
    const int64_t v = p.pairs[2 * c];
    int64_t X[3] = {0, 0, 0};
    for (int d = 0; d < p.ndim; ++d)
        if (v > 0) X[d] = div_floor(p.csum[(int64_t)c * p.ndim + d] * 65536, v);
    int64_t *h = p.hist + (int64_t)c * p.slots * 3;
    // the sweeps unwrap an accepted copy's site to the image nearest this
    // point (the centroid rounded to a site), in the frame of the sums
    if (v > 0) {
        int r[3] = {0, 0, 0};
        for (int d = 0; d < p.ndim; ++d) r[d] = (int)div_floor(X[d] + 32768, 65536);
        p.cpos[c] = make_int4(r[0], r[1], r[2], 0);
    }
    if (t == 0) {
        for (int k = 0; k < p.slots; ++k)
            for (int d = 0; d < 3; ++d) h[3 * k + d] = X[d];
        p.pdir[c] = make_int4(0, 0, 0, 0);
        return;
    }
    if (v == 0) {
        p.pdir[c] = make_int4(0, 0, 0, 0);
        return;
    }
    const int64_t *old = h + 3 * ((t + 1) % p.slots);
    int64_t D[3];
    for (int d = 0; d < 3; ++d) {
        const int64_t W = (int64_t)p.L[d] * 65536;
        int64_t w = (X[d] - old[d]) % W;
        if (w < 0) w += W;
        if (w >= W / 2) w -= W;
        D[d] = d < p.ndim ? w : 0;
    }
    int64_t *slot = h + 3 * (t % p.slots);
    for (int d = 0; d < 3; ++d) slot[d] = X[d];
    const int64_t nd = isqrt_floor(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    const int4 prev = p.pdir[c];
    const int64_t pp[3] = {prev.x, prev.y, prev.z};
    const int64_t mu = p.model->mu_p[p.cell_type[c]];
    int64_t q[3];
    for (int d = 0; d < 3; ++d) {
        const int64_t u = nd > 0 ? (D[d] * 16384) / nd : 0;
        q[d] = (16384 - mu) * u + mu * pp[d];
    }
    const int64_t np = isqrt_floor(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    p.pdir[c] = np > 0 ? make_int4((int)((q[0] * 16384) / np), (int)((q[1] * 16384) / np),
                                   (int)((q[2] * 16384) / np), 0)
                       : make_int4(0, 0, 0, 0);
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

__global__ void copy_counters_kernel(const int32_t *pairs, int32_t n_labels, int32_t *v_out, int32_t *s_out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_labels) return;
    v_out[i] = i == 0 ? 0 : pairs[2 * i];
    s_out[i] = i == 0 ? 0 : pairs[2 * i + 1];
}

// Sites whose label lies outside [-1, n_cells], or is an obstacle (-1) in a
// model without an obstacle type: counted into *bad (one atomic per wave).
__global__ void __launch_bounds__(kBlock) bad_label_kernel(const int32_t *lat, size_t n, int32_t n_cells,
                                                           int allow_obstacle, int32_t *bad)
{
    const int lo = allow_obstacle ? -1 : 0;
    int cnt = 0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        const int v = lat[i];
        cnt += v < lo || v > n_cells;
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(bad, cnt);
}

// Labels 1..n_labels-1 whose tracked (V, S) pair differs from the recount
// (v, s): counted into *bad.
__global__ void compare_counters_kernel(const int32_t *pairs, const int32_t *v, const int32_t *s, int32_t n_labels,
                                        int32_t *bad)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < 1 || i >= n_labels) return;
    if (pairs[2 * i] != v[i] || pairs[2 * i + 1] != s[i]) atomicAdd(bad, 1);
}

__global__ void set_u32_kernel(uint32_t *p, uint32_t v) { *p = v; }
__global__ void add_u32_kernel(uint32_t *p, uint32_t v) { *p += v; }

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
    const unsigned grid = (unsigned)((n + kSitesPerBlock - 1) / kSitesPerBlock);
    if (ndim == 2)
        reduce_kernel<2, kCount><<<grid, kBlock, 0, stream>>>(a, v_out, s_out, stride, nullptr, nullptr);
    else
        reduce_kernel<3, kCount><<<grid, kBlock, 0, stream>>>(a, v_out, s_out, stride, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_contacts(const SweepArgs &a, int ndim, int n_types, int64_t *out, hipStream_t stream)
{
    hipError_t e = launch_fill_i32(reinterpret_cast<int32_t *>(out), 0, (size_t)n_types * n_types * 2, stream);
    if (e != hipSuccess) return e;
    const size_t n = (size_t)a.L[0] * a.L[1] * a.L[2];
    const unsigned grid = (unsigned)((n + kSitesPerBlock - 1) / kSitesPerBlock);
    auto *o = reinterpret_cast<unsigned long long *>(out);
    if (ndim == 2) contact_kernel<2><<<grid, kBlock, 0, stream>>>(a, o, n_types);
    else contact_kernel<3><<<grid, kBlock, 0, stream>>>(a, o, n_types);
    return hipGetLastError();
}

hipError_t launch_persist(const PersistArgs &p, int64_t t, hipStream_t stream)
{
    persist_kernel<<<blocks_for((size_t)p.n_labels), kBlock, 0, stream>>>(p, t);
    return hipGetLastError();
}

hipError_t launch_act_decay(uint8_t *act, size_t n, hipStream_t stream)
{
    const size_t threads = (n + 15) / 16;
    act_decay_kernel<<<blocks_for(threads), kBlock, 0, stream>>>(act, n);
    return hipGetLastError();
}

hipError_t launch_centroids(const SweepArgs &a, int ndim, int32_t n_cells, int32_t *ref, int64_t *out,
                            hipStream_t stream, int words)
{
    const unsigned grid = (unsigned)(ndim == 2 ? reduce_bricks<2>(a.L) : reduce_bricks<3>(a.L));
    hipError_t e = launch_fill_i32(ref, INT32_MAX, (size_t)n_cells + 1, stream);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(reinterpret_cast<int32_t *>(out), 0, ((size_t)n_cells + 1) * ndim * 2, stream);
    if (e != hipSuccess) return e;
    auto run = [&](auto d_tag, auto w_tag) {
        constexpr int D = decltype(d_tag)::value, W = decltype(w_tag)::value;
        reduce_kernel<D, kRef, W><<<grid, kBlock, 0, stream>>>(a, nullptr, nullptr, 0, ref, nullptr);
        reduce_kernel<D, kCentroid, W><<<grid, kBlock, 0, stream>>>(a, nullptr, nullptr, 0, ref, out);
    };
    using D2 = std::integral_constant<int, 2>;
    using D3 = std::integral_constant<int, 3>;
    using W32 = std::integral_constant<int, kWords32>;
    using W16 = std::integral_constant<int, kWords16>;
    using WP = std::integral_constant<int, kWordsPacked>;
    using WPA = std::integral_constant<int, kWordsPackedAct>;
    if (ndim == 2) {
        if (words == kWords16) run(D2{}, W16{});
        else if (words == kWordsPacked) run(D2{}, WP{});
        else if (words == kWordsPackedAct) run(D2{}, WPA{});
        else run(D2{}, W32{});
    } else {
        if (words == kWords16) run(D3{}, W16{});
        else if (words == kWordsPacked) run(D3{}, WP{});
        else if (words == kWordsPackedAct) run(D3{}, WPA{});
        else run(D3{}, W32{});
    }
    return hipGetLastError();
}

namespace {
__global__ void copy_dirs_kernel(const int4 *pdir, int32_t n_labels, int32_t *out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_labels) return;
    const int4 v = i == 0 ? make_int4(0, 0, 0, 0) : pdir[i];
    out[3 * i] = v.x;
    out[3 * i + 1] = v.y;
    out[3 * i + 2] = v.z;
}
}  // namespace

namespace {
__global__ void occupancy_kernel(const int32_t *lat, int n_lattices, size_t n_sites, int32_t *counts)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_sites) return;
    int32_t c = 0;
    for (int l = 0; l < n_lattices; ++l) c += lat[(size_t)l * n_sites + i] > 0;
    counts[i] = c;
}
}  // namespace

hipError_t launch_occupancy(const int32_t *lattices, int n_lattices, size_t n_sites, int32_t *counts,
                            hipStream_t st)
{
    occupancy_kernel<<<blocks_for(n_sites), kBlock, 0, st>>>(lattices, n_lattices, n_sites, counts);
    return hipGetLastError();
}

int64_t reduce_brick_count(const int *L, int ndim) { return ndim == 2 ? reduce_bricks<2>(L) : reduce_bricks<3>(L); }

hipError_t launch_copy_dirs(const int4 *pdir, int32_t n_labels, int32_t *out, hipStream_t stream)
{
    copy_dirs_kernel<<<blocks_for((size_t)n_labels), kBlock, 0, stream>>>(pdir, n_labels, out);
    return hipGetLastError();
}

hipError_t launch_batch_cell_stats(const SweepArgs *d_args, const int64_t *d_label_off, int n_lattices, int ndim,
                                   size_t max_sites, int64_t max_bricks, size_t total_labels, int32_t *v_out,
                                   int32_t *s_out, int32_t *ref, int64_t *cent, hipStream_t stream)
{
    const dim3 grid((unsigned)((max_sites + kSitesPerBlock - 1) / kSitesPerBlock), (unsigned)n_lattices);
    const dim3 grid_b((unsigned)max_bricks, (unsigned)n_lattices);
    hipError_t e;
    if ((e = launch_fill_i32(v_out, 0, total_labels, stream)) != hipSuccess) return e;
    if ((e = launch_fill_i32(s_out, 0, total_labels, stream)) != hipSuccess) return e;
    if (ndim == 2) batch_reduce_kernel<2, kCount><<<grid, kBlock, 0, stream>>>(d_args, d_label_off, v_out, s_out, nullptr, nullptr);
    else batch_reduce_kernel<3, kCount><<<grid, kBlock, 0, stream>>>(d_args, d_label_off, v_out, s_out, nullptr, nullptr);
    if ((e = hipGetLastError()) != hipSuccess || !cent) return e;
    if ((e = launch_fill_i32(ref, INT32_MAX, total_labels, stream)) != hipSuccess) return e;
    if ((e = launch_fill_i32(reinterpret_cast<int32_t *>(cent), 0, total_labels * ndim * 2, stream)) != hipSuccess)
        return e;
    if (ndim == 2) {
        batch_reduce_kernel<2, kRef><<<grid_b, kBlock, 0, stream>>>(d_args, d_label_off, nullptr, nullptr, ref, nullptr);
        batch_reduce_kernel<2, kCentroid><<<grid_b, kBlock, 0, stream>>>(d_args, d_label_off, nullptr, nullptr, ref, cent);
    } else {
        batch_reduce_kernel<3, kRef><<<grid_b, kBlock, 0, stream>>>(d_args, d_label_off, nullptr, nullptr, ref, nullptr);
        batch_reduce_kernel<3, kCentroid><<<grid_b, kBlock, 0, stream>>>(d_args, d_label_off, nullptr, nullptr, ref, cent);
    }
    return hipGetLastError();
}

hipError_t launch_copy_counters(const int32_t *pairs, int32_t n_labels, int32_t *v_out, int32_t *s_out,
                                hipStream_t stream)
{
    copy_counters_kernel<<<blocks_for((size_t)n_labels), kBlock, 0, stream>>>(pairs, n_labels, v_out, s_out);
    return hipGetLastError();
}

hipError_t launch_bad_labels(const int32_t *lat, size_t n, int32_t n_cells, bool allow_obstacle, int32_t *bad,
                             hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const unsigned grid = std::min<unsigned>(blocks_for(n), 4096u);
    bad_label_kernel<<<grid, kBlock, 0, stream>>>(lat, n, n_cells, allow_obstacle ? 1 : 0, bad);
    return hipGetLastError();
}

hipError_t launch_compare_counters(const int32_t *pairs, const int32_t *v, const int32_t *s, int32_t n_labels,
                                   int32_t *bad, hipStream_t stream)
{
    compare_counters_kernel<<<blocks_for((size_t)n_labels), kBlock, 0, stream>>>(pairs, v, s, n_labels, bad);
    return hipGetLastError();
}

hipError_t launch_set_u32(uint32_t *p, uint32_t value, hipStream_t stream)
{
    set_u32_kernel<<<1, 1, 0, stream>>>(p, value);
    return hipGetLastError();
}

hipError_t launch_add_u32(uint32_t *p, uint32_t value, hipStream_t stream)
{
    add_u32_kernel<<<1, 1, 0, stream>>>(p, value);
    return hipGetLastError();
}

}  // namespace cpm
