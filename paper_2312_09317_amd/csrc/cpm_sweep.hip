// Host side of the activation kernels: the stored-word conversions a sweep
// runs before and after its activations (16-bit working copy, packed label /
// type / activity words), the Act decay on words, and the dispatch of one
// activation to the kernel instantiated for the model's stored words and
// dimension (cpm_sweep_kernels.hpp, cpm_sweep_inst.hip).
#include <algorithm>
#include <type_traits>

#include "cpm_device.hpp"

namespace cpm {
namespace {

__host__ __device__ constexpr int align16(int v) { return (v + 15) & ~15; }

// The caller's int32 lattice rewritten in place as packed words and back.
__global__ void pack_kernel(int32_t *lat, const int32_t *cell_type, int obstacle_type, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int v = lat[i];
    const int t = v < 0 ? obstacle_type : cell_type[v];
    lat[i] = (int32_t)packed_word(v, t);
}

__global__ void unpack_kernel(int32_t *lat, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    lat[i] = label_of((uint32_t)lat[i]);
}

__global__ void pack_act_kernel(int32_t *lat, const uint8_t *act, const int32_t *cell_type, int obstacle_type,
                                size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int v = lat[i];
    const int t = v < 0 ? obstacle_type : cell_type[v];
    lat[i] = (int32_t)(uint32_t)act_word(v, t, act[i]);
}

__global__ void unpack_act_kernel(int32_t *lat, uint8_t *act, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const char32_t w = (char32_t)(uint32_t)lat[i];
    lat[i] = label_of(w);
    act[i] = (uint8_t)((uint32_t)w >> 24);
}

// Act decay (one per MCS, to 0) in the activity bits of the words.
__global__ void act_decay_words_kernel(int32_t *lat, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t w = (uint32_t)lat[i];
    if (w >> 24) lat[i] = (int32_t)(w - (1u << 24));
}

__device__ __forceinline__ ushort4 encode4(int4 v)
{
    ushort4 w;
    w.x = stored_label<uint16_t>(v.x);
    w.y = stored_label<uint16_t>(v.y);
    w.z = stored_label<uint16_t>(v.z);
    w.w = stored_label<uint16_t>(v.w);
    return w;
}

__device__ __forceinline__ int4 decode4(ushort4 w)
{
    return make_int4(label_of(w.x), label_of(w.y), label_of(w.z), label_of(w.w));
}

__global__ void to_mirror_kernel(const int32_t *__restrict__ lat, uint16_t *__restrict__ mir, size_t n)
{
    const size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 4;
    if (i + 4 <= n) {
        *reinterpret_cast<ushort4 *>(mir + i) = encode4(*reinterpret_cast<const int4 *>(lat + i));
    } else {
        for (size_t j = i; j < n; ++j) mir[j] = stored_label<uint16_t>(lat[j]);
    }
}

__global__ void from_mirror_kernel(const uint16_t *__restrict__ mir, int32_t *__restrict__ lat, size_t n)
{
    const size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 4;
    if (i + 4 <= n) {
        *reinterpret_cast<int4 *>(lat + i) = decode4(*reinterpret_cast<const ushort4 *>(mir + i));
    } else {
        for (size_t j = i; j < n; ++j) lat[j] = label_of(mir[j]);
    }
}

// All lattices of a batch to / from their 16-bit working copies in one
// launch: blockIdx.y is the lattice, x blocks stride over its sites in
// groups of 4 (lattice sizes are multiples of (2s)^d, bases 16-byte aligned).
template <bool TO>
__global__ void batch_mirror_kernel(const SweepArgs *__restrict__ args)
{
    const SweepArgs &a = args[blockIdx.y];
    const size_t n = (size_t)a.L[0] * a.L[1] * a.L[2];
    uint16_t *mir = static_cast<uint16_t *>(a.cells);
    for (size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 4; i < n; i += (size_t)gridDim.x * kBlock * 4) {
        if (i + 4 <= n) {
            if (TO) *reinterpret_cast<ushort4 *>(mir + i) = encode4(*reinterpret_cast<const int4 *>(a.lat + i));
            else *reinterpret_cast<int4 *>(a.lat + i) = decode4(*reinterpret_cast<const ushort4 *>(mir + i));
        } else {
            for (size_t j = i; j < n; ++j) {
                if (TO) mir[j] = stored_label<uint16_t>(a.lat[j]);
                else a.lat[j] = label_of(mir[j]);
            }
        }
    }
}

// 16-bit label-activity words (label + 1 in bits 0..10, activity in 11..15)
// of a whole batch, four sites per thread (lattices hold multiples of 16
// sites, so only the batch's end can be ragged).
__global__ void to_act16_kernel(const int32_t *__restrict__ lat, const uint8_t *__restrict__ act,
                                uint16_t *__restrict__ w, size_t n, int32_t *overflow)
{
    const size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 4;
    bool over = false;
    for (size_t j = i; j < i + 4 && j < n; ++j) {
        over |= act[j] > 31;
        w[j] = (uint16_t)((uint32_t)(lat[j] + 1) | ((uint32_t)act[j] << 11));
    }
    if (over) atomicOr(overflow, 1);
}

__global__ void count_above_kernel(const uint8_t *act, size_t n, int limit, int32_t *count)
{
    int cnt = 0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        cnt += act[i] > limit;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(count, cnt);
}

__global__ void from_act16_kernel(const uint16_t *__restrict__ w, int32_t *__restrict__ lat,
                                  uint8_t *__restrict__ act, size_t n)
{
    const size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 4;
    for (size_t j = i; j < i + 4 && j < n; ++j) {
        const uint32_t v = w[j];
        lat[j] = (int)(v & 0x7FFu) - 1;
        act[j] = (uint8_t)(v >> 11);
    }
}

// Act decay in 16-bit words: activity bits minus one where nonzero, eight
// words per thread.
__global__ void act16_decay_kernel(uint16_t *w, size_t n)
{
    const size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 8;
    if (i + 8 <= n && (reinterpret_cast<uintptr_t>(w + i) & 15) == 0) {
        uint4 v = *reinterpret_cast<const uint4 *>(w + i);
        uint32_t q[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // each half: activity in bits 11..15; subtract 1 << 11 where nonzero
            const uint32_t lo = (q[e] & 0xF800u) ? (1u << 11) : 0u;
            const uint32_t hi = (q[e] & 0xF8000000u) ? (1u << 27) : 0u;
            q[e] -= lo + hi;
        }
        *reinterpret_cast<uint4 *>(w + i) = make_uint4(q[0], q[1], q[2], q[3]);
    } else {
        for (size_t j = i; j < i + 8 && j < n; ++j)
            if (w[j] >> 11) w[j] = (uint16_t)(w[j] - (1u << 11));
    }
}

// All lattices of a batch to / from label-type-activity words in place
// (blockIdx.y is the lattice).
template <bool TO>
__global__ void batch_act_words_kernel(const SweepArgs *__restrict__ args)
{
    const SweepArgs &a = args[blockIdx.y];
    const size_t n = (size_t)a.L[0] * a.L[1] * a.L[2];
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        if (TO) {
            const int v = a.lat[i];
            a.lat[i] = (int32_t)(uint32_t)act_word(v, v < 0 ? a.obstacle_type : a.cell_type[v], a.act[i]);
        } else {
            const char32_t w = (char32_t)(uint32_t)a.lat[i];
            a.lat[i] = label_of(w);
            a.act[i] = (uint8_t)((uint32_t)w >> 24);
        }
    }
}

}  // namespace

size_t sweep_lds_bytes(int ndim, bool act, bool mirror, int box_sites)
{
    (void)ndim;
    const int cell = mirror ? 2 : 4;
    return (size_t)align16(box_sites * cell) + (act ? (size_t)align16(box_sites) : 0);
}

hipError_t launch_activation(const SweepArgs &a, int ndim, bool act, int words, uint32_t mcs, uint32_t alpha,
                             int parity, hipStream_t stream)
{
    const size_t lds = (size_t)a.tg.lds_bytes;
    const bool d2 = ndim == 2;
    switch (words) {
    case kWords16:
        return d2 ? sweep_words<uint16_t, 2>(a, act, mcs, alpha, parity, lds, stream)
                  : sweep_words<uint16_t, 3>(a, act, mcs, alpha, parity, lds, stream);
    case kWordsPacked:
        return d2 ? sweep_words<uint32_t, 2>(a, act, mcs, alpha, parity, lds, stream)
                  : sweep_words<uint32_t, 3>(a, act, mcs, alpha, parity, lds, stream);
    case kWordsPackedAct:  // Act models only
        return d2 ? sweep_words<char32_t, 2>(a, act, mcs, alpha, parity, lds, stream)
                  : sweep_words<char32_t, 3>(a, act, mcs, alpha, parity, lds, stream);
    default:
        return d2 ? sweep_words<int32_t, 2>(a, act, mcs, alpha, parity, lds, stream)
                  : sweep_words<int32_t, 3>(a, act, mcs, alpha, parity, lds, stream);
    }
}

hipError_t launch_pack(int32_t *lat, const int32_t *cell_type, int obstacle_type, size_t n, hipStream_t stream)
{
    pack_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, stream>>>(lat, cell_type, obstacle_type, n);
    return hipGetLastError();
}

hipError_t launch_pack_act(int32_t *lat, const uint8_t *act, const int32_t *cell_type, int obstacle_type, size_t n,
                           hipStream_t stream)
{
    pack_act_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, stream>>>(lat, act, cell_type, obstacle_type, n);
    return hipGetLastError();
}

hipError_t launch_unpack_act(int32_t *lat, uint8_t *act, size_t n, hipStream_t stream)
{
    unpack_act_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, stream>>>(lat, act, n);
    return hipGetLastError();
}

hipError_t launch_act_decay_words(int32_t *lat, size_t n, hipStream_t stream)
{
    act_decay_words_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, stream>>>(lat, n);
    return hipGetLastError();
}

hipError_t launch_unpack(int32_t *lat, size_t n, hipStream_t stream)
{
    unpack_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, stream>>>(lat, n);
    return hipGetLastError();
}

hipError_t launch_batch_activation(const BatchLaunch &b, uint32_t alpha, int parity, hipStream_t stream)
{
    const bool d2 = b.ndim == 2;
    if (b.act16)
        return d2 ? batch_words<char16_t, 2>(b, alpha, parity, stream) : batch_words<char16_t, 3>(b, alpha, parity, stream);
    if (b.act_words)
        return d2 ? batch_words<char32_t, 2>(b, alpha, parity, stream) : batch_words<char32_t, 3>(b, alpha, parity, stream);
    if (b.mirror)
        return d2 ? batch_words<uint16_t, 2>(b, alpha, parity, stream) : batch_words<uint16_t, 3>(b, alpha, parity, stream);
    return d2 ? batch_words<int32_t, 2>(b, alpha, parity, stream) : batch_words<int32_t, 3>(b, alpha, parity, stream);
}

hipError_t launch_batch_persistent(const BatchLaunch &b, const PersistentLaunch &p, hipStream_t stream)
{
    const bool d2 = b.ndim == 2;
    if (b.act16)
        return d2 ? batch_persistent_words<char16_t, 2>(b, p, stream) : batch_persistent_words<char16_t, 3>(b, p, stream);
    if (b.act_words)
        return d2 ? batch_persistent_words<char32_t, 2>(b, p, stream) : batch_persistent_words<char32_t, 3>(b, p, stream);
    if (b.mirror)
        return d2 ? batch_persistent_words<uint16_t, 2>(b, p, stream) : batch_persistent_words<uint16_t, 3>(b, p, stream);
    return d2 ? batch_persistent_words<int32_t, 2>(b, p, stream) : batch_persistent_words<int32_t, 3>(b, p, stream);
}

hipError_t launch_batch_act_words(const SweepArgs *d_args, int n_lattices, size_t max_sites, bool to_words,
                                  hipStream_t stream)
{
    const size_t groups = (max_sites + kBlock - 1) / kBlock;
    const dim3 grid((unsigned)std::min<size_t>(groups, 256), (unsigned)n_lattices);
    if (to_words) batch_act_words_kernel<true><<<grid, kBlock, 0, stream>>>(d_args);
    else batch_act_words_kernel<false><<<grid, kBlock, 0, stream>>>(d_args);
    return hipGetLastError();
}

hipError_t launch_to_act16(const int32_t *lat, const uint8_t *act, uint16_t *words, size_t n, int32_t *overflow,
                           hipStream_t stream)
{
    const size_t threads = (n + 3) / 4;
    to_act16_kernel<<<(unsigned)((threads + kBlock - 1) / kBlock), kBlock, 0, stream>>>(lat, act, words, n, overflow);
    return hipGetLastError();
}

hipError_t launch_count_above(const uint8_t *act, size_t n, int limit, int32_t *count, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<size_t>((n + kBlock - 1) / kBlock, 4096);
    count_above_kernel<<<grid, kBlock, 0, stream>>>(act, n, limit, count);
    return hipGetLastError();
}

hipError_t launch_from_act16(const uint16_t *words, int32_t *lat, uint8_t *act, size_t n, hipStream_t stream)
{
    const size_t threads = (n + 3) / 4;
    from_act16_kernel<<<(unsigned)((threads + kBlock - 1) / kBlock), kBlock, 0, stream>>>(words, lat, act, n);
    return hipGetLastError();
}

hipError_t launch_act16_decay(uint16_t *words, size_t n, hipStream_t stream)
{
    const size_t threads = (n + 7) / 8;
    act16_decay_kernel<<<(unsigned)((threads + kBlock - 1) / kBlock), kBlock, 0, stream>>>(words, n);
    return hipGetLastError();
}

hipError_t launch_to_mirror(const int32_t *lat, uint16_t *mirror, size_t n, hipStream_t stream)
{
    const size_t threads = (n + 3) / 4;
    to_mirror_kernel<<<(unsigned)((threads + kBlock - 1) / kBlock), kBlock, 0, stream>>>(lat, mirror, n);
    return hipGetLastError();
}

hipError_t launch_from_mirror(const uint16_t *mirror, int32_t *lat, size_t n, hipStream_t stream)
{
    const size_t threads = (n + 3) / 4;
    from_mirror_kernel<<<(unsigned)((threads + kBlock - 1) / kBlock), kBlock, 0, stream>>>(mirror, lat, n);
    return hipGetLastError();
}

hipError_t launch_batch_mirror(const SweepArgs *d_args, int n_lattices, size_t max_sites, bool to_mirror,
                               hipStream_t stream)
{
    const size_t groups = (max_sites + 4 * kBlock - 1) / (4 * kBlock);
    const dim3 grid((unsigned)std::min<size_t>(groups, 64), (unsigned)n_lattices);
    if (to_mirror) batch_mirror_kernel<true><<<grid, kBlock, 0, stream>>>(d_args);
    else batch_mirror_kernel<false><<<grid, kBlock, 0, stream>>>(d_args);
    return hipGetLastError();
}

}  // namespace cpm