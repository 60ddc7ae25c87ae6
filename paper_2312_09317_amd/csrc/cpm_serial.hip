// The serial CPM on the GPU (Methods, first paragraph): per MCS, N copy
// attempts at uniformly drawn targets, each seeing the lattice and the
// per-cell counters exactly as the attempt before it left them.  It is the
// reference the parallel scheme is compared with (Fig. 5, Fig. 6E), run for
// every lattice of a batch at once: one wave per lattice, attempts one after
// another.
//
// Within an attempt the wave's lanes load in parallel: lanes 0..31 the
// target's neighbourhood (lane l < |NB|: Moore neighbour l; lane 31: the
// target), lanes 32..63 the source's (lane 32 + l: its neighbour l; lane 63:
// the source).  Sums over neighbours are reductions within a half-wave.  Every
// load of data the kernel writes (labels, activity, counters) has a
// lane-dependent address, so it is a vector load that sees the wave's earlier
// stores; lane 0 commits.
#include <type_traits>

#include "cpm_device.hpp"

namespace cpm {
namespace {

// Sum over the 32 lanes of this lane's half-wave.
__device__ __forceinline__ int64_t half_sum(int64_t v)
{
#pragma unroll
    for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int half_or(int v)
{
#pragma unroll
    for (int o = 16; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// The Metropolis decision of metropolis32, reading only the table entries
// it needs, after the branches on q: attempts here run one at a time and
// most decisions need no table, so an unconditional round of loads per
// attempt would add up.
__device__ __forceinline__ bool metropolis32_lazy(const ThrTables &tb, int64_t q, uint32_t u)
{
    if (q <= 0) return true;
    const uint64_t h = (uint64_t)q >> 16;
    if (h >= (uint64_t)tb.n_ti) return false;
    const uint64_t two32 = (uint64_t)1 << 32;
    const uint64_t ti = h == 0 ? two32 : (uint64_t)tb.ti[h];
    if ((q & 0xFFFF) == 0) return (uint64_t)u < ti;
    const int mm = (int)((q >> 8) & 255), ll = (int)(q & 255);
    const uint64_t tm = mm ? (uint64_t)tb.tm[mm] : two32, tl = ll ? (uint64_t)tb.tl[ll] : two32;
    return (uint64_t)u < __umul64hi(ti, tm * tl);  // tm * tl < 2^64 since (mm, ll) != (0, 0)
}

template <int D>
__device__ __forceinline__ int site_at(const int *L, int x, int y, int z)
{
    return wrap_once(x, L[0]) + L[0] * (wrap_once(y, L[1]) + L[1] * (D == 3 ? wrap_once(z, L[2]) : 0));
}

// One MCS of the serial CPM on lattice blockIdx.x.  Counters are the exact
// (V, S) pairs of buffer `parity`.
template <typename Cell, int D, bool ACT>
__global__ void __launch_bounds__(64) serial_mcs_kernel(const SweepArgs *args, uint32_t mcs, int parity)
{
    constexpr int NNB = D == 2 ? 8 : 26;
    const SweepArgs &a = args[blockIdx.x];
    const DeviceModel *m = a.model;
    const int lane = threadIdx.x;
    const int half = lane >> 5, hl = lane & 31;
    const int L[3] = {a.L[0], a.L[1], a.L[2]};
    const uint32_t N = (uint32_t)L[0] * (uint32_t)L[1] * (uint32_t)L[2];
    // int32 labels: the caller's lattice itself (a batch may keep other words
    // for its parallel sweeps in a.cells)
    Cell *cells = std::is_same<Cell, int32_t>::value ? reinterpret_cast<Cell *>(a.lat) : reinterpret_cast<Cell *>(a.cells);
    int32_t *cnt = a.counters[parity];
    const ThrTables tb{m->TM32, m->TL32, m->TI32, m->n_ti};
    uint32_t n_nontrivial = 0, n_accepted = 0;

    for (uint32_t i = 0; i < N; ++i) {
        const uint4 u = philox4x32_10(make_uint4(i, mcs, 0xFFFFFF00u, a.lattice_id), a.key0, a.key1);
        const int t = (int)(((uint64_t)u.x * N) >> 32);
        const int tx = t % L[0], ty = (t / L[0]) % L[1], tz = t / (L[0] * L[1]);
        const int nsel = (int)(((uint64_t)u.y * (uint32_t)NNB) >> 32);
        const int dx = nb_dx<D>(nsel), dy = nb_dy<D>(nsel), dz = nb_dz<D>(nsel);
        const int sx = tx + dx, sy = ty + dy, sz = tz + dz;
        // this lane's site: a neighbour of the target (half 0) or of the source
        const int cx = half ? sx : tx, cy = half ? sy : ty, cz = half ? sz : tz;
        const int own = hl == 31;
        const int n_of = hl < NNB ? hl : 0;
        const int site = own ? site_at<D>(L, cx, cy, cz)
                             : site_at<D>(L, cx + nb_dx<D>(n_of), cy + nb_dy<D>(n_of), cz + nb_dz<D>(n_of));
        const bool used = own || hl < NNB;
        const int lab = used ? label_of(cells[site]) : INT32_MIN;
        const int lt = __shfl(lab, 31, 64), ls = __shfl(lab, 63, 64);
        if (lt == ls || lt < 0 || ls < 0) continue;
        ++n_nontrivial;
        const int src = __shfl(site, 63, 64);
        const int tt = lt == 0 ? 0 : a.cell_type[lt], ts = ls == 0 ? 0 : a.cell_type[ls];
        // adhesion and the neighbour counts of the target (half 0)
        int64_t adh = 0, k_old = 0, k_new = 0;
        if (half == 0 && hl < NNB) {
            const int tu = lab == 0 ? 0 : (lab < 0 ? a.obstacle_type : a.cell_type[lab]);
            if (lab != ls) adh += m->J[ts * kMaxTypes + tu];
            if (lab != lt) adh -= m->J[tt * kMaxTypes + tu];
            k_old = lab == lt;
            k_new = lab == ls;
        }
        adh = __shfl(half_sum(adh), 0, 64);
        k_old = __shfl(half_sum(k_old), 0, 64);
        k_new = __shfl(half_sum(k_new), 0, 64);
        // counters of both cells (lanes 0 and 1) and the field at the source (lane 2)
        int2 pair = make_int2(0, 0);
        if (lane == 0 && lt >= 1) pair = reinterpret_cast<const int2 *>(cnt)[lt];
        if (lane == 1 && ls >= 1) pair = reinterpret_cast<const int2 *>(cnt)[ls];
        int64_t chem_dot = 0;
        const int o = (dx < 0 ? 2 : (dx > 0 ? 0 : 1)) + 3 * (dy < 0 ? 2 : (dy > 0 ? 0 : 1)) +
                      9 * (dz < 0 ? 2 : (dz > 0 ? 0 : 1));  // offset target - source = -(dx, dy, dz)
        if (lane == 2 && a.chem) {
            const int16_t *c = a.chem + (size_t)D * src;
            chem_dot = (int64_t)m->unit[o][0] * c[0] + (int64_t)m->unit[o][1] * c[1] +
                       (D == 3 ? (int64_t)m->unit[o][2] * c[2] : 0);
        }
        const int vt = __shfl(pair.x, 0, 64), st_ = __shfl(pair.y, 0, 64);
        const int vs = __shfl(pair.x, 1, 64), ss = __shfl(pair.y, 1, 64);
        chem_dot = __shfl(chem_dot, 2, 64);
        const int64_t dso = 2 * k_old - NNB, dsn = NNB - 2 * k_new;
        int64_t q = adh;
        if (lt >= 1) {
            q += m->lam_v[tt] * (1 - 2 * ((int64_t)vt - m->v_target[tt]));
            q += m->lam_s[tt] * (2 * dso * ((int64_t)st_ - m->s_target[tt]) + dso * dso);
        }
        if (ls >= 1) {
            q += m->lam_v[ts] * (2 * ((int64_t)vs - m->v_target[ts]) + 1);
            q += m->lam_s[ts] * (2 * dsn * ((int64_t)ss - m->s_target[ts]) + dsn * dsn);
        }
        if (ACT) {
            // geometric means over each half's own site and its neighbours of the same cell
            const int me = half ? ls : lt;
            const bool motile = me > 0 && m->max_act[me == lt ? tt : ts] > 0;
            const bool mine = used && lab == me;
            const uint32_t av = mine ? a.act[site] : 1u;
            const int64_t sum = half_sum(mine ? m->LG[av] : 0);
            const int64_t cntn = half_sum(mine ? 1 : 0);
            const int zero = half_or(mine && av == 0);
            const int64_t gm = (!motile || zero) ? 0 : exp_log24(m, (uint64_t)sum / (uint64_t)cntn);
            const int64_t gt = __shfl(gm, 0, 64), gs = __shfl(gm, 32, 64);
            const int64_t rt = lt >= 1 ? m->r_act[tt] : 0, rs = ls >= 1 ? m->r_act[ts] : 0;
            q += (rt * gt - rs * gs) >> 16;
        }
        if (a.chem && ls >= 1) q -= (m->lam_c[ts] * chem_dot) >> 28;
        if (!metropolis32_lazy(tb, q, u.z)) continue;
        ++n_accepted;
        if (lane == 0) {
            cells[t] = stored_label<Cell>(ls);
            if (ACT) a.act[t] = (ls >= 1 && m->max_act[ts] > 0) ? (uint8_t)m->max_act[ts] : (uint8_t)0;
            if (lt >= 1) {
                cnt[2 * lt] -= 1;
                cnt[2 * lt + 1] += (int)dso;
            }
            if (ls >= 1) {
                cnt[2 * ls] += 1;
                cnt[2 * ls + 1] += (int)dsn;
            }
        }
        // the next attempt's loads (other lanes) see this commit
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
    if (ACT) {
        // Act decay at the end of the MCS
        for (uint32_t s = lane; s < N; s += 64) {
            const uint8_t v = a.act[s];
            a.act[s] = v > 0 ? (uint8_t)(v - 1) : (uint8_t)0;
        }
    }
    if (lane == 0) {
        a.stats[0] += n_nontrivial;
        a.stats[1] += n_accepted;
    }
}

}  // namespace

hipError_t launch_serial_mcs(const SweepArgs *d_args, int n_lattices, int ndim, bool act, bool mirror, uint32_t mcs,
                             int parity, hipStream_t st)
{
    const dim3 grid((unsigned)n_lattices), block(64);
    if (mirror) {
        if (ndim == 2) {
            if (act) serial_mcs_kernel<uint16_t, 2, true><<<grid, block, 0, st>>>(d_args, mcs, parity);
            else serial_mcs_kernel<uint16_t, 2, false><<<grid, block, 0, st>>>(d_args, mcs, parity);
        } else {
            if (act) serial_mcs_kernel<uint16_t, 3, true><<<grid, block, 0, st>>>(d_args, mcs, parity);
            else serial_mcs_kernel<uint16_t, 3, false><<<grid, block, 0, st>>>(d_args, mcs, parity);
        }
    } else {
        if (ndim == 2) {
            if (act) serial_mcs_kernel<int32_t, 2, true><<<grid, block, 0, st>>>(d_args, mcs, parity);
            else serial_mcs_kernel<int32_t, 2, false><<<grid, block, 0, st>>>(d_args, mcs, parity);
        } else {
            if (act) serial_mcs_kernel<int32_t, 3, true><<<grid, block, 0, st>>>(d_args, mcs, parity);
            else serial_mcs_kernel<int32_t, 3, false><<<grid, block, 0, st>>>(d_args, mcs, parity);
        }
    }
    return hipGetLastError();
}

}  // namespace cpm
