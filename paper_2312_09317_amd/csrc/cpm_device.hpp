// Device-side building blocks of the CPM sweep: Philox, the Moore
// neighbourhood, the Metropolis threshold and the Act geometric mean.
#pragma once

#include "cpm_internal.hpp"

namespace cpm {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products, key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each product as one 32x32->64 multiply (both halves at once)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ int wrap_once(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

// Labels as stored.  int32: the label itself.  The 16-bit working copy holds
// label + 1 (obstacle -1 -> 0, medium 0 -> 1, cells 1..65534 -> 2..65535),
// so lattices of up to 65,534 cells sweep on half the bytes.
__device__ __forceinline__ int label_of(int32_t v) { return v; }
__device__ __forceinline__ int label_of(uint16_t v) { return (int)v - 1; }
template <typename Cell>
__device__ __forceinline__ Cell stored_label(int label) { return (Cell)label; }
template <>
__device__ __forceinline__ uint16_t stored_label<uint16_t>(int label) { return (uint16_t)(label + 1); }

// Packed words (uint32, the caller's int32 lattice rewritten in place for
// the length of a sweep): label + 1 in bits 0..23, the cell type in bits
// 24..31 (obstacle: the obstacle type; medium: 0), so a neighbour's type
// arrives with its label.
__device__ __forceinline__ int label_of(uint32_t v) { return (int)(v & 0xFFFFFFu) - 1; }
__device__ __forceinline__ uint32_t packed_word(int label, int type)
{
    return (uint32_t)(label + 1) | ((uint32_t)type << 24);
}

// Packed words with activity (char32_t; Act models of up to 2^20 - 2
// cells): label + 1 in bits 0..19, the cell type in bits 20..23, the site's
// activity in bits 24..31, so the Act term reads a neighbourhood's activity
// with its labels.
__device__ __forceinline__ int label_of(char32_t v) { return (int)((uint32_t)v & 0xFFFFFu) - 1; }
__device__ __forceinline__ char32_t act_word(int label, int type, uint32_t act)
{
    return (char32_t)((uint32_t)(label + 1) | ((uint32_t)type << 20) | (act << 24));
}

// 16-bit label-activity words (char16_t; Act batches whose lattices hold at
// most 2,046 cells of one type, Max_act <= 31): label + 1 in bits 0..10, the
// site's activity in bits 11..15.
__device__ __forceinline__ int label_of(char16_t v) { return (int)((uint32_t)v & 0x7FFu) - 1; }

// Where a stored word keeps the site's activity (kIn): bits kShift and up,
// the rest (kKeep) being label and type.
template <typename Cell>
struct WordAct {
    static constexpr bool kIn = false;
    static constexpr int kShift = 0;
    static constexpr uint32_t kKeep = 0xFFFFFFFFu;
};
template <>
struct WordAct<char32_t> {
    static constexpr bool kIn = true;
    static constexpr int kShift = 24;
    static constexpr uint32_t kKeep = 0xFFFFFFu;
};
template <>
struct WordAct<char16_t> {
    static constexpr bool kIn = true;
    static constexpr int kShift = 11;
    static constexpr uint32_t kKeep = 0x7FFu;
};

// Activity of LDS / lattice index i: from the word, or from the activity array.
template <typename Cell>
__device__ __forceinline__ uint32_t act_at(const Cell *lab, const uint8_t *lact, int i) { return lact[i]; }
template <>
__device__ __forceinline__ uint32_t act_at<char32_t>(const char32_t *lab, const uint8_t *, int i)
{
    return (uint32_t)lab[i] >> 24;
}
template <>
__device__ __forceinline__ uint32_t act_at<char16_t>(const char16_t *lab, const uint8_t *, int i)
{
    return (uint32_t)lab[i] >> 11;
}

// Cell type of a site from its stored word (`label` = label_of(word)).
template <typename A>
__device__ __forceinline__ int type_of_word(const A &a, uint32_t word, int) { return (int)(word >> 24); }
template <typename A>
__device__ __forceinline__ int type_of_word(const A &a, char32_t word, int)
{
    return (int)(((uint32_t)word >> 20) & 15u);
}
// Type of a label from the cell-type array (obstacle: the obstacle type).
// Both values are read and one of them kept: a choice between the two
// addresses, one inside the argument block, makes the compiler copy the
// whole block to scratch memory.  Entry 0 (medium) stands in for obstacles.
template <typename A>
__device__ __forceinline__ int type_of_label(const A &a, int label)
{
    const int to = a.obstacle_type;
    const int tc = a.cell_type[label < 0 ? 0 : label];
    return label < 0 ? to : tc;
}
template <typename A>
__device__ __forceinline__ int type_of_word(const A &a, int32_t, int label) { return type_of_label(a, label); }
template <typename A>
__device__ __forceinline__ int type_of_word(const A &a, uint16_t, int label) { return type_of_label(a, label); }
template <typename A>
__device__ __forceinline__ int type_of_word(const A &a, char16_t, int label) { return type_of_label(a, label); }

// Division by a divisor fixed for a whole workgroup: q = floor(n / d) as one
// multiply-high, exact whenever n * d < 2^32 (m = floor((2^32 - 1) / d) + 1
// overshoots 2^32 / d by less than 1, so the error n / 2^32 stays below the
// gap 1 / d between floor(n / d) + 1 and the largest fraction).
struct FastDiv {
    uint32_t d, m;
    __device__ __forceinline__ explicit FastDiv(uint32_t div) : d(div), m(div > 1 ? 0xFFFFFFFFu / div + 1u : 0u) {}
    // with the multiplier computed beforehand (the host's tile geometry)
    __device__ __forceinline__ FastDiv(uint32_t div, uint32_t mul) : d(div), m(mul) {}
    __device__ __forceinline__ uint32_t div(uint32_t n) const { return d > 1 ? __umulhi(n, m) : n; }
};

// Moore offset n (lexicographic, z slowest, x fastest, the centre left out).
template <int D>
__device__ __forceinline__ constexpr int nb_dx(int n) { return (D == 2 ? (n < 4 ? n : n + 1) : (n < 13 ? n : n + 1)) % 3 - 1; }
template <int D>
__device__ __forceinline__ constexpr int nb_dy(int n) { return (D == 2 ? (n < 4 ? n : n + 1) / 3 : ((n < 13 ? n : n + 1) / 3) % 3) - 1; }
template <int D>
__device__ __forceinline__ constexpr int nb_dz(int n) { return D == 2 ? 0 : (n < 13 ? n : n + 1) / 9 - 1; }

// Threshold tables as 32-bit words; entry 0 of each stands for 2^32 and is
// never read.
struct ThrTables {
    const uint32_t *tm, *tl, *ti;
    int n_ti;
};

// Accept iff q <= 0 or u < floor(TI[h] TM[m] TL[l] / 2^64), q = h*2^16 + m*2^8 + l.
// The three table entries are read in one round (indices clamped into the
// tables) and the decision is taken without branches: the entries a case
// does not use are ignored.
__device__ __forceinline__ bool metropolis32(const ThrTables &tb, int64_t q, uint32_t u)
{
    const uint64_t h = (uint64_t)q >> 16;
    const bool in = q > 0 && h < (uint64_t)tb.n_ti;
    const int mm = (int)((q >> 8) & 255), ll = (int)(q & 255);
    const uint64_t two32 = (uint64_t)1 << 32;
    const uint32_t ti_w = tb.ti[in ? h : 0], tm_w = tb.tm[mm], tl_w = tb.tl[ll];
    // an empty asm that takes the three entries keeps the compiler from
    // moving the loads of tm and tl into the branch that uses them
    asm volatile("" ::"v"(ti_w), "v"(tm_w), "v"(tl_w));
    const uint64_t ti_e = ti_w, tm_e = tm_w, tl_e = tl_w;
    const uint64_t ti = h == 0 ? two32 : ti_e;
    const uint64_t tm = mm ? tm_e : two32, tl = ll ? tl_e : two32;
    // tm * tl < 2^64 whenever (mm, ll) != (0, 0), the only case it is used
    const uint64_t thr = (q & 0xFFFF) == 0 ? ti : __umul64hi(ti, tm * tl);
    return (q <= 0) | (in & ((uint64_t)u < thr));
}

// exp(l * 2^-24) in 2^16 fixed point, floor-composed from the split tables.
__device__ __forceinline__ int64_t exp_log24(const DeviceModel *m, uint64_t ell)
{
    const uint64_t p1 = (m->EH[ell >> 16] * m->EM[(ell >> 8) & 255]) >> 31;
    const uint64_t p2 = (p1 * m->EL[ell & 255]) >> 30;
    return (int64_t)(p2 >> 8);
}

}  // namespace cpm
