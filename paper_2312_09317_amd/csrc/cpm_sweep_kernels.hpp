#pragma once
// The activation kernel of the CPM sweep for gfx950 (templates; instantiated
// per stored-word type and dimension in cpm_sweep_inst.hip).
//
// One launch runs one activation of the checkerboard scheme (paper, Results,
// "Designing a parallel execution scheme", Fig. 2A; one barrier per copy
// attempt, Fig. 3A): every thread area makes k copy attempts inside its
// sub-area of the active colour.
//
// Work split: one workgroup per tile of up to 256 thread areas (one thread
// per area).  The tile's active sub-areas plus their read halo are staged
// into LDS with coalesced loads (paper, Methods, "GPU implementation
// details": shared-memory caching of the active regions, write-through on
// accepted copies).  Two LDS layouts:
//   full rows - the tile spans whole lattice rows along x; each LDS row holds
//               one whole lattice row, copied with aligned 16-byte loads, and
//               neighbours wrap around x inside LDS;
//   box       - any tile shape; the staged box is the tile's sub-areas plus
//               the halo, copied element by element.
// Tiles go to XCDs in contiguous slabs (workgroups are dispatched to the 8
// XCDs round-robin), so every activation of a sweep finds the XCD's slab in
// the same L2.
//
// For k = 1 the copy attempts of a workgroup run in two phases: all threads
// draw their attempt and drop the trivial ones (equal labels or an
// obstacle); the rest are compacted into an LDS queue and worked off by the
// first threads, so the energy evaluation runs on as few waves as needed.
//
// Per-cell counters are double buffered: activation g reads buffer g&1 (the
// exact state at its start) and adds its own deltas plus those of activation
// g-1 (kept per tile in `dlist`) into buffer (g+1)&1, which so becomes the
// exact state at the start of g+1.
#include <algorithm>
#include <type_traits>

#include "cpm_device.hpp"

namespace cpm {
namespace {

__device__ __forceinline__ void add_deltas(int32_t *wr, int4 d)
{
    if (d.x >= 1) {
        atomicAdd(&wr[2 * d.x], -1);
        atomicAdd(&wr[2 * d.x + 1], d.z);
    }
    if (d.y >= 1) {
        atomicAdd(&wr[2 * d.y], 1);
        atomicAdd(&wr[2 * d.y + 1], d.w);
    }
}

__host__ __device__ constexpr int align16(int v) { return (v + 15) & ~15; }

constexpr int kQueue = 128;  // queued attempts per workgroup; the rest are evaluated where drawn

// Where the sites an attempt reads live.  kBox: an LDS box, coordinates
// box-local; kFullRow: LDS rows spanning the lattice along x, x global and
// wrapping, y, z box-local; kDirect: the lattice itself in global memory,
// every coordinate global and wrapping.
enum Layout { kBox = 0, kFullRow = 1, kDirect = 2 };

// A pointer of the sweep arguments as a plain (generic) pointer; loads
// through a global-memory one converted here stay global loads.
template <typename T>
__device__ __forceinline__ T *plain(T *p)
{
    return p;
}
template <typename T>
__device__ __forceinline__ T *plain(__attribute__((address_space(1))) T *p)
{
    return (T *)p;
}

template <int LAYOUT>
struct LdsMap {
    int pitch;  // sites per row
    int rows;   // rows per z plane
    int L0, L1, L2;
    __device__ __forceinline__ int x(int v) const { return LAYOUT == kBox ? v : wrap_once(v, L0); }
    __device__ __forceinline__ int row(int vy, int vz) const
    {
        return LAYOUT == kDirect ? L0 * (wrap_once(vy, L1) + L1 * wrap_once(vz, L2)) : pitch * (vy + rows * vz);
    }
    __device__ __forceinline__ int at(int vx, int vy, int vz) const { return x(vx) + row(vy, vz); }
};

// The mean of ln(activity) (2^-24 units) over a site and its Moore
// neighbours of the same cell (the exponent of eq. 8), from words (and
// activities) already loaded; `dead` when any of those activities is 0.
// Every table entry is read and the ones of other labels masked, so the
// loop has no branch.  The sum fits 32 bits: ln(255) 2^24 < 2^27, at most
// 27 terms.
template <typename Cell, int NNB>
__device__ __forceinline__ uint32_t mean_log_act(const int64_t *lg, uint32_t a0, const Cell *w, const uint32_t *av,
                                                 int cell, bool &dead)
{
    uint32_t sum = (uint32_t)lg[a0];
    uint32_t cnt = 1;
    bool zero = a0 == 0;
#pragma unroll
    for (int n = 0; n < NNB; ++n) {
        const bool same = label_of(w[n]) == cell;
        const uint32_t au = WordAct<Cell>::kIn ? (uint32_t)w[n] >> WordAct<Cell>::kShift : av[n];
        const uint32_t v = (uint32_t)lg[au];
        zero |= same && au == 0;
        sum += same ? v : 0u;
        cnt += same ? 1u : 0u;
    }
    dead = zero;
    return sum / cnt;
}

// Geometric mean of the activity over the site at (x,y,z) (label `cell`) and
// its Moore neighbours of the same cell (eq. 8), 2^16 fixed point.
template <typename Cell, int D, int LAYOUT>
__device__ __forceinline__ int64_t gm_lds(const DeviceModel *m, const int64_t *lg, const Cell *lab,
                                          const uint8_t *lact, const LdsMap<LAYOUT> &map, int x, int y, int z,
                                          int cell, bool motile)
{
    if (cell <= 0 || !motile) return 0;
    const int c = map.at(x, y, z);
    constexpr int NNB = D == 2 ? 8 : 26;
    const uint32_t a0 = act_at(lab, lact, c);
    if (LAYOUT == kDirect) {
        // in place (global memory): the neighbourhood's words (and
        // activities) in one round, then the masked sums
        Cell w[NNB];
        uint32_t av[NNB];
#pragma unroll
        for (int n = 0; n < NNB; ++n) {
            const int u = map.at(x + nb_dx<D>(n), y + nb_dy<D>(n), z + nb_dz<D>(n));
            w[n] = lab[u];
            av[n] = WordAct<Cell>::kIn ? 0u : (uint32_t)lact[u];
        }
        bool dead;
        const uint32_t ell = mean_log_act<Cell, NNB>(lg, a0, w, av, cell, dead);
        return dead ? 0 : exp_log24(m, ell);
    }
    // staged (LDS): reads are cheap, only like labels are looked up
    uint64_t sum = (uint64_t)lg[a0];
    uint32_t cnt = 1;
    bool zero = a0 == 0;
#pragma unroll
    for (int n = 0; n < NNB; ++n) {
        const int u = map.at(x + nb_dx<D>(n), y + nb_dy<D>(n), z + nb_dz<D>(n));
        const int lu = label_of(lab[u]);
        const uint32_t au = act_at(lab, lact, u);
        if (lu == cell) {
            zero |= au == 0;
            sum += (uint64_t)lg[au];
            ++cnt;
        }
    }
    return zero ? 0 : exp_log24(m, sum / cnt);
}

// J rows of the medium type and of the single cell type (when all cells share one type).
struct JRows {
    int64_t cc, cm, co, mc, mm, mo;
};

// Per-workgroup LDS copies of the model tables an attempt reads: J
// (multi-type models), the Act log table and the per-type parameters.
struct SharedTables {
    const int32_t *J;  // J in 2^-16 fixed point: |J| < 2^15, so each entry fits 32 bits
    const int64_t *lg;
    const TypeParams *tp;
};

// One copy attempt past the early rejection: energy change of copying label
// ls into the target (x,y,z) (eq. 1, eq. 3, eq. 7) and the Metropolis test
// (eq. 2).  cnt_t / cnt_s are the (V, S) counters of the two cells as the
// attempt sees them.  Returns acceptance; dso / dsn are the surface deltas.
// nbl(n) gives the label of the target's n-th Moore neighbour.
template <typename Cell, int D, bool ACT, bool SINGLE, int LAYOUT, bool EXT, typename NB, typename A>
__device__ __forceinline__ bool evaluate_nb(const A &a, const ThrTables &tb, const JRows &jr,
                                            const SharedTables &st, const NB &nbl, Cell *lab, uint8_t *lact,
                                            const LdsMap<LAYOUT> &map, int tx_, int ty_, int tz_, int sx_, int sy_,
                                            int sz_, int src_gi, int lt, int ls, int tt, int ts, int2 cnt_t, int2 cnt_s,
                                            uint32_t u2, int64_t &dso_out, int64_t &dsn_out)
{
    constexpr int NNB = D == 2 ? 8 : 26;
    constexpr bool kIn = WordAct<Cell>::kIn;
    const DeviceModel *m = plain(a.model);
    const TypeParams *tp = st.tp;
    // In place (global memory), the target's neighbourhood comes first, in
    // a block without branches, so that it is read in one round (several
    // cell types, or the Act term, whose target mean reuses it); staged
    // layouts read LDS as they go.  The source's neighbourhood (Act) is read
    // only for a motile source, in its own round: reading it with the
    // target's measured slower (registers).
    constexpr bool GROUP = LAYOUT == kDirect && (!SINGLE || ACT);
    constexpr bool GACT = GROUP && ACT;
    Cell nw[NNB];
    uint32_t nav[GACT && !kIn ? NNB : 1];
    uint32_t ca_t = 0;
    if (GROUP) {
#pragma unroll
        for (int n = 0; n < NNB; ++n) nw[n] = nbl(n);
        if (GACT) {
            ca_t = act_at(lab, lact, map.at(tx_, ty_, tz_));
            if (!kIn) {
#pragma unroll
                for (int n = 0; n < NNB; ++n)
                    nav[n] = lact[map.at(tx_ + nb_dx<D>(n), ty_ + nb_dy<D>(n), tz_ + nb_dz<D>(n))];
            }
        }
    }
    int k_old = 0, k_new = 0;
    int n_cell = 0, n_med = 0, n_obs = 0;
    int64_t adh = 0;
#pragma unroll
    for (int n = 0; n < NNB; ++n) {
        const Cell word = GROUP ? nw[n] : nbl(n);
        const int lu = label_of(word);
        k_old += lu == lt;
        k_new += lu == ls;
        if (SINGLE) {
            n_cell += lu > 0;
            n_med += lu == 0;
            n_obs += lu < 0;
        } else if (GROUP) {
            // every J entry read, the ones of like labels masked
            const int tu = type_of_word(a, word, lu);
            const int64_t js = st.J[ts * kMaxTypes + tu], jt = st.J[tt * kMaxTypes + tu];
            adh += (lu != ls ? js : 0) - (lu != lt ? jt : 0);
        } else {
            const int tu = type_of_word(a, word, lu);
            if (lu != ls) adh += st.J[ts * kMaxTypes + tu];
            if (lu != lt) adh -= st.J[tt * kMaxTypes + tu];
        }
    }
    if (SINGLE) {
        // neighbours unlike the label, weighted by J(label type, their type)
        const int64_t cs = n_cell - (ls > 0 ? k_new : 0), ms = n_med - (ls == 0 ? k_new : 0);
        const int64_t ct = n_cell - (lt > 0 ? k_old : 0), mt = n_med - (lt == 0 ? k_old : 0);
        adh = (ls > 0 ? jr.cc * cs + jr.cm * ms + jr.co * n_obs : jr.mc * cs + jr.mm * ms + jr.mo * n_obs) -
              (lt > 0 ? jr.cc * ct + jr.cm * mt + jr.co * n_obs : jr.mc * ct + jr.mm * mt + jr.mo * n_obs);
    }
    const int64_t dso = 2 * k_old - NNB;
    const int64_t dsn = NNB - 2 * k_new;
    int64_t q = adh;
    if (lt >= 1) {
        q += tp->lam_v[tt] * (1 - 2 * ((int64_t)cnt_t.x - tp->v_target[tt]));
        q += tp->lam_s[tt] * (2 * dso * ((int64_t)cnt_t.y - tp->s_target[tt]) + dso * dso);
    }
    if (ls >= 1) {
        q += tp->lam_v[ts] * (2 * ((int64_t)cnt_s.x - tp->v_target[ts]) + 1);
        q += tp->lam_s[ts] * (2 * dsn * ((int64_t)cnt_s.y - tp->s_target[ts]) + dsn * dsn);
    }
    if (ACT) {
        const bool mot_t = lt > 0 && tp->max_act[tt] > 0, mot_s = ls > 0 && tp->max_act[ts] > 0;
        int64_t gt;
        if (GACT) {
            bool dead_t;
            const uint32_t ell_t = mean_log_act<Cell, NNB>(st.lg, ca_t, nw, nav, lt, dead_t);
            const int64_t et = exp_log24(m, ell_t);
            gt = mot_t && !dead_t ? et : 0;
        } else {
            gt = gm_lds<Cell, D, LAYOUT>(m, st.lg, lab, lact, map, tx_, ty_, tz_, lt, mot_t);
        }
        const int64_t gs = gm_lds<Cell, D, LAYOUT>(m, st.lg, lab, lact, map, sx_, sy_, sz_, ls, mot_s);
        const int64_t rt = lt >= 1 ? tp->r_act[tt] : 0;
        const int64_t rs = ls >= 1 ? tp->r_act[ts] : 0;
        q += (rt * gt - rs * gs) >> 16;
    }
    if (EXT && a.pdir && ls >= 1) {
        // persistence: the copying cell ls extends from the source into the
        // target; copies along its direction are favoured
        const int o = (tx_ - sx_ + 1) + 3 * (ty_ - sy_ + 1) + 9 * (tz_ - sz_ + 1);
        const int4 pd = plain(a.pdir)[ls];
        const int64_t dot = (int64_t)m->unit[o][0] * pd.x + (int64_t)m->unit[o][1] * pd.y +
                            (int64_t)m->unit[o][2] * pd.z;
        q -= (m->lam_p[ts] * dot) >> 28;
    }
    if (EXT && a.chem && ls >= 1) {
        // chemotaxis: the field at the source, dotted with the copy's direction
        const int o = (tx_ - sx_ + 1) + 3 * (ty_ - sy_ + 1) + 9 * (tz_ - sz_ + 1);
        int64_t dot;
        if (D == 2) {
            const short2 c = reinterpret_cast<const short2 *>(plain(a.chem))[src_gi];
            dot = (int64_t)m->unit[o][0] * c.x + (int64_t)m->unit[o][1] * c.y;
        } else {
            const int16_t *c = plain(a.chem) + 3 * (size_t)src_gi;
            dot = (int64_t)m->unit[o][0] * c[0] + (int64_t)m->unit[o][1] * c[1] + (int64_t)m->unit[o][2] * c[2];
        }
        q -= (m->lam_c[ts] * dot) >> 28;
    }
    dso_out = dso;
    dsn_out = dsn;
    return metropolis32(tb, q, u2);
}

// evaluate_nb with the neighbour labels read through `map`.
template <typename Cell, int D, bool ACT, bool SINGLE, int LAYOUT, bool EXT, typename A>
__device__ __forceinline__ bool evaluate(const A &a, const ThrTables &tb, const JRows &jr,
                                         const SharedTables &st, Cell *lab, uint8_t *lact,
                                         const LdsMap<LAYOUT> &map, int tx_, int ty_, int tz_, int sx_, int sy_,
                                         int sz_, int src_gi, int lt, int ls, int tt, int ts, int2 cnt_t, int2 cnt_s,
                                         uint32_t u2, int64_t &dso_out, int64_t &dsn_out)
{
    const int xm = map.x(tx_ - 1), x0 = map.x(tx_), xp = map.x(tx_ + 1);
    auto nbl = [&](int n) {
        const int dx = nb_dx<D>(n);
        const int xx = dx < 0 ? xm : (dx > 0 ? xp : x0);
        return lab[xx + map.row(ty_ + nb_dy<D>(n), tz_ + nb_dz<D>(n))];
    };
    return evaluate_nb<Cell, D, ACT, SINGLE, LAYOUT, EXT>(a, tb, jr, st, nbl, lab, lact, map, tx_, ty_, tz_, sx_, sy_,
                                                     sz_, src_gi, lt, ls, tt, ts, cnt_t, cnt_s, u2, dso_out, dsn_out);
}

// Counters of label c as an attempt of this thread sees them: the read
// buffer plus the deltas of the thread's own earlier accepted copies in this
// activation (n_own records: the first kOwnInRegs in registers, the rest in
// its spill array).
__device__ __forceinline__ int2 seen_counters(const int32_t *rd, int c, const int4 *own, int n_own,
                                              const int4 *spill = nullptr)
{
    if (c < 1) return make_int2(0, 0);
    int2 v = reinterpret_cast<const int2 *>(rd)[c];
#pragma unroll
    for (int jj = 0; jj < kOwnInRegs; ++jj) {
        if (jj < n_own && own[jj].x == c) { v.x -= 1; v.y += own[jj].z; }
        if (jj < n_own && own[jj].y == c) { v.x += 1; v.y += own[jj].w; }
    }
    for (int jj = kOwnInRegs; jj < n_own; ++jj) {
        const int4 r = spill[jj - kOwnInRegs];
        if (r.x == c) { v.x -= 1; v.y += r.z; }
        if (r.y == c) { v.x += 1; v.y += r.w; }
    }
    return v;
}

// Composite variable tracking (Methods): an accepted copy moves its target
// site (global index gi) from cell lt's centroid sums to cell ls's.  The
// site enters each sum as its periodic image nearest that cell's reference
// point (the centroid rounded to a site at the last direction update), so
// the sums stay those of one unwrapped copy of the cell while it is smaller
// than half the lattice.  Integer atomics: the result does not depend on
// the order of the copies.
// The site at (gx, gy, gz); ref_s / ref_t are the reference points of ls
// and lt (read beforehand).
template <int D, typename A>
__device__ __forceinline__ void move_centroids_at(const A &a, int gx, int gy, int gz, int lt, int ls, int4 ref_t,
                                                  int4 ref_s)
{
    const int L[3] = {a.L[0], a.L[1], a.L[2]};
    const int g[3] = {gx, gy, gz};
    unsigned long long *cs = reinterpret_cast<unsigned long long *>(plain(a.csum));
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int c = side == 0 ? ls : lt;
        if (c < 1) continue;
        const int4 r4 = side == 0 ? ref_s : ref_t;
        const int r[3] = {r4.x, r4.y, r4.z};
#pragma unroll
        for (int d = 0; d < D; ++d) {
            int u = (g[d] - r[d]) % L[d];
            if (u < 0) u += L[d];
            if (u >= L[d] - L[d] / 2) u -= L[d];  // into [-L/2, L/2)
            const int64_t x = (int64_t)r[d] + u;
            atomicAdd(cs + (size_t)c * D + d, (unsigned long long)(side == 0 ? x : -x));
        }
    }
}

// The same from the site's global index, reading the reference points here.
template <int D, typename A>
__device__ __forceinline__ void move_centroids(const A &a, int gi, int lt, int ls)
{
    const int L0 = a.L[0], L1 = a.L[1];
    const int4 *cp = plain(a.cpos);
    const int4 zero = make_int4(0, 0, 0, 0);
    move_centroids_at<D>(a, gi % L0, (gi / L0) % L1, D == 3 ? gi / (L0 * L1) : 0, lt, ls, lt > 0 ? cp[lt] : zero,
                         ls > 0 ? cp[ls] : zero);
}

// One workgroup's share of one activation: tile `tile` of the lattice `a`.
template <typename Cell, int D, bool ACT, bool SINGLE, bool K1, int LAYOUT, bool EXT, typename A>
__device__ __forceinline__ void sweep_tile(const A &a, int tile, uint32_t mcs, uint32_t alpha, int parity)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int list_n, queue_n;
    __shared__ uint32_t n_nontrivial, n_accepted, waves_done;
    // compacted attempts.  Staged layouts: packed target / source
    // coordinates and draw, and the counters (V, S) of both cells fetched
    // while drawing.  In place, 16 bytes per attempt (the LDS a workgroup
    // holds bounds how many fit on a CU): target x | y << 16, z | the
    // source's Moore offset << 16, the draw, and the target's stored word
    // (16-bit words: both words; wider ones: the source's in queue_ws).
    constexpr bool EAGER_Q = LAYOUT == kDirect && K1;
    // in place, 3D multi-type sweeps evaluate where they draw (below)
    constexpr bool COMPACT = EAGER_Q && !(D == 3 && !SINGLE);
    constexpr bool kWideCell = sizeof(Cell) > 2;
    constexpr int kQ = COMPACT ? kBlock : (K1 && !EAGER_Q ? kQueue : 1);
    __shared__ int4 queue[kQ];
    __shared__ int4 queue_cnt[COMPACT ? 1 : kQ];
    __shared__ uint32_t queue_ws[COMPACT && kWideCell ? kBlock : 1];
    __shared__ int32_t j_lds[SINGLE ? 1 : kMaxTypes * kMaxTypes];
    // the Act log table: 16-bit label-activity words index its first 32 entries
    constexpr int kLgLds = std::is_same<Cell, char16_t>::value ? kMaxAct16Activity + 1 : 256;
    __shared__ int64_t lg_lds[ACT ? kLgLds : 1];
    __shared__ __align__(16) TypeParams tp_lds;
    constexpr int R = ACT ? 2 : 1;           // read radius: the Act term reads neighbours of the source
    constexpr int NNB = D == 2 ? 8 : 26;

    const TileGeometry &tg = a.tg;
    const int tid = threadIdx.x;
    const int L0 = a.L[0], L1 = a.L[1], L2 = a.L[2];
    const int s = a.s;
    const uint32_t phi = alpha & ((1u << D) - 1);
    const int cx = (int)(phi & 1), cy = (int)((phi >> 1) & 1), cz = (int)((phi >> 2) & 1);
    // tile coordinates: tile = tx + nt0 (ty + nt1 tz), divisions by the
    // geometry's multipliers (uniform over the workgroup)
    const FastDiv by_nt0((uint32_t)tg.nt[0], tg.div_nt[0]), by_nt1((uint32_t)tg.nt[1], tg.div_nt[1]);
    const int tq = (int)by_nt0.div((uint32_t)tile), tx = tile - tq * tg.nt[0];
    const int tz = (int)by_nt1.div((uint32_t)tq), ty = tq - tz * tg.nt[1];
    const int A0 = tx * tg.T[0], A1 = ty * tg.T[1], A2 = tz * tg.T[2];
    const int n0 = min(tg.T[0], a.na[0] - A0), n1 = min(tg.T[1], a.na[1] - A1);
    const int n2 = D == 3 ? min(tg.T[2], a.na[2] - A2) : 1;
    constexpr bool FULLROW = LAYOUT == kFullRow, DIRECT = LAYOUT == kDirect;
    // staged box: sub-areas of the active colour plus the read halo (none
    // for the direct layout, which reads the lattice in place)
    const int b0 = FULLROW ? L0 : 2 * s * (n0 - 1) + s + 2 * R;
    const int b1 = 2 * s * (n1 - 1) + s + 2 * R;
    const int b2 = D == 3 ? 2 * s * (n2 - 1) + s + 2 * R : 1;
    const int o0 = FULLROW || DIRECT ? 0 : 2 * s * A0 + s * cx - R;
    const int o1 = DIRECT ? 0 : 2 * s * A1 + s * cy - R;
    const int o2 = D == 3 && !DIRECT ? 2 * s * A2 + s * cz - R : 0;
    const LdsMap<LAYOUT> map{DIRECT ? L0 : b0, DIRECT ? L1 : b1, L0, L1, L2};
    Cell *cells = static_cast<Cell *>(plain(a.cells));
    Cell *lab = DIRECT ? cells : reinterpret_cast<Cell *>(smem);
    uint8_t *lact = DIRECT ? plain(a.act) : smem + align16(tg.box_sites * (int)sizeof(Cell));
    const int32_t *rd = plain(a.counters[parity]);
    int32_t *wr = plain(a.counters[parity ^ 1]);
    // delta lists: this activation's records go to the list of its parity;
    // the previous activation's (other parity) are re-added into wr
    int4 *dl = plain(a.dlist[parity]) + (size_t)tile * a.dlist_cap;
    const int4 *dl_prev = plain(a.dlist[parity ^ 1]) + (size_t)tile * a.dlist_cap;

    if (tid == 0) {
        list_n = 0;
        queue_n = 0;
        n_nontrivial = 0;
        n_accepted = 0;
        waves_done = 0;
    }
    // model tables read per neighbour, copied to LDS (visible after the
    // staging barrier): at most one entry of each per thread, all loads
    // issued before the first LDS store
    static_assert(kMaxTypes * kMaxTypes <= kBlock && 256 <= kBlock, "one table entry per thread");
    {
        constexpr int kTpWords = (int)(sizeof(TypeParams) / sizeof(int4));
        static_assert(kTpWords <= kBlock, "one 16-byte word of the type block per thread");
        const DeviceModel *mdl = plain(a.model);
        const bool j_mine = !SINGLE && tid < a.n_types * kMaxTypes;
        const bool lg_mine = ACT && tid < min(a.lg_entries, kLgLds);
        const bool tp_mine = tid < kTpWords;
        const int32_t jv = j_mine ? (int32_t)mdl->J[tid] : 0;
        const int64_t lgv = lg_mine ? mdl->LG[tid] : 0;
        const int4 tpv = tp_mine ? reinterpret_cast<const int4 *>(mdl->lam_v)[tid] : make_int4(0, 0, 0, 0);
        if (j_mine) j_lds[tid] = jv;
        if (lg_mine) lg_lds[tid] = lgv;
        if (tp_mine) reinterpret_cast<int4 *>(&tp_lds)[tid] = tpv;
    }
    const SharedTables sht{j_lds, lg_lds, &tp_lds};
    // deltas of the previous activation go into the write buffer as well
    // k = 1 in place: every attempt is evaluated by the thread that draws it
    // (no queue): measured faster than queueing the nontrivial attempts across
    // the workgroup (9.3 vs 9.8 us per 3D activation, 2.34 vs 2.92 ms per MCS
    // of 512 batched 2D lattices with the Act term)
    constexpr bool EAGER = EAGER_Q;
    if (!EAGER) {
        const int prev_n = a.dcount[parity ^ 1][tile];
        for (int i = tid; i < prev_n; i += kBlock) add_deltas(wr, dl_prev[i]);
    }
    // threshold tables, read from the model (they stay in L2: every tile reads them)
    const DeviceModel *model = plain(a.model);
    const ThrTables tb{model->TM32, model->TL32, model->TI32, model->n_ti};

    const int areas = n0 * n1 * n2;
    const uint32_t sd = D == 2 ? (uint32_t)(s * s) : (uint32_t)(s * s * s);
    // draw of one attempt: target and source in LDS coordinates
    const FastDiv by_n0((uint32_t)n0, tx == tg.nt[0] - 1 ? tg.div_last[0] : tg.div_T[0]);
    const FastDiv by_n1((uint32_t)n1, ty == tg.nt[1] - 1 ? tg.div_last[1] : tg.div_T[1]);
    const FastDiv by_s((uint32_t)s, tg.div_s);
    auto draw = [&](int area_local, int j, int &ttx, int &tty, int &ttz, int &ssx, int &ssy, int &ssz, uint32_t &u2,
                    uint32_t &area_id) {
        const int q0 = (int)by_n0.div((uint32_t)area_local), ax = area_local - q0 * n0;
        const int az = (int)by_n1.div((uint32_t)q0), ay = q0 - az * n1;
        area_id = (uint32_t)(A0 + ax) + (uint32_t)a.na[0] * ((uint32_t)(A1 + ay) + (uint32_t)a.na[1] * (uint32_t)(A2 + az));
        const uint4 u = philox4x32_10(make_uint4(area_id, mcs, (alpha << 8) | (uint32_t)j, a.lattice_id), a.key0, a.key1);
        const uint32_t o = (uint32_t)(((uint64_t)u.x * sd) >> 32);
        const int q1 = (int)by_s.div(o), ox = (int)o - q1 * s;
        const int oz = D == 3 ? (int)by_s.div((uint32_t)q1) : 0, oy = q1 - oz * s;
        ttx = DIRECT ? 2 * s * (A0 + ax) + s * cx + ox : (FULLROW ? 2 * s * ax + s * cx + ox : 2 * s * ax + R + ox);
        tty = DIRECT ? 2 * s * (A1 + ay) + s * cy + oy : 2 * s * ay + R + oy;
        ttz = D == 3 ? (DIRECT ? 2 * s * (A2 + az) + s * cz + oz : 2 * s * az + R + oz) : 0;
        const int nsel = (int)(((uint64_t)u.y * (uint32_t)NNB) >> 32);
        const int msel = nsel < NNB / 2 ? nsel : nsel + 1;
        ssx = ttx + msel % 3 - 1;
        ssy = tty + (msel / 3) % 3 - 1;
        ssz = D == 3 ? ttz + msel / 9 - 1 : 0;
        u2 = u.z;
    };
    auto global_index = [&](int vx, int vy, int vz) {
        if (DIRECT) return map.at(vx, vy, vz);
        const int gx = FULLROW ? wrap_once(vx, L0) : wrap_once(o0 + vx, L0);
        const int gy = wrap_once(o1 + vy, L1);
        const int gz = D == 3 ? wrap_once(o2 + vz, L2) : 0;
        return (int)(((size_t)gz * L1 + gy) * L0 + gx);
    };
    // the cell types of an attempt's two labels (their stored words at hand)
    auto types = [&](Cell wt, int lt_, Cell ws, int ls_, int &tt_, int &ts_) {
        tt_ = lt_ == 0 ? 0 : (SINGLE ? a.single_type : type_of_word(a, wt, lt_));
        ts_ = ls_ == 0 ? 0 : (SINGLE ? a.single_type : type_of_word(a, ws, ls_));
    };
    // the target takes the source's stored word (its label, and its type in
    // packed words); words with activity carry the target's new activity
    constexpr bool kActWord = WordAct<Cell>::kIn;
    auto commit = [&](int t, int gi, int lt, int ls, Cell ws, int ts, int64_t dso, int64_t dsn) {
        uint8_t na = 0;
        if (ACT) na = (ls >= 1 && tp_lds.max_act[ts] > 0) ? (uint8_t)tp_lds.max_act[ts] : (uint8_t)0;
        const Cell nw = kActWord ? (Cell)(((uint32_t)ws & WordAct<Cell>::kKeep) | ((uint32_t)na << WordAct<Cell>::kShift))
                                 : ws;
        if (!DIRECT) lab[t] = nw;
        cells[gi] = nw;
        if (EXT && !DIRECT && a.csum) move_centroids<D>(a, gi, lt, ls);
        if (ACT && !kActWord) {
            if (!DIRECT) lact[t] = na;
            a.act[gi] = na;
        }
        const int4 rec = make_int4(lt, ls, (int)dso, (int)dsn);
        add_deltas(wr, rec);
        dl[atomicAdd(&list_n, 1)] = rec;
        return rec;
    };

    if (EAGER) {
        // round 1: the previous list's count, its first kEarlyRecords
        // records (one per thread; a tile's accepted copies rarely fill more,
        // and loading all of its slots would read one 16-byte slot per area
        // in every activation) and the attempt's two labels; round 2,
        // nontrivial attempts only (packed into the first lanes, below): the
        // target's neighbours and both cells' counters (and any later
        // records of the previous list); round 3: the Act means' tables, or
        // the source's neighbourhood of a motile source; last: the
        // acceptance threshold
        constexpr int kEarlyRecords = 16;
        const int prev_n = a.dcount[parity ^ 1][tile];
        const int4 early_rec = tid < kEarlyRecords ? dl_prev[tid] : make_int4(0, 0, 0, 0);
        int ttx = 0, tty = 0, ttz = 0, ssx = 0, ssy = 0, ssz = 0, lt = 0, ls = 0;
        Cell wt = 0, ws = 0;
        uint32_t u2 = 0, area_id = 0;
        const bool mine = tid < areas;
        // the single type's J rows: uniform over the workgroup, read while
        // the labels load
        JRows jr{0, 0, 0, 0, 0, 0};
        if (SINGLE) {
            const int64_t *J = model->J;
            const int tc = a.single_type, to = a.obstacle_type;
            jr = JRows{J[tc * kMaxTypes + tc], J[tc * kMaxTypes], J[tc * kMaxTypes + to], J[tc], J[0], J[to]};
        }
        if (mine) {
            draw(tid, 0, ttx, tty, ttz, ssx, ssy, ssz, u2, area_id);
            wt = lab[map.at(ttx, tty, ttz)];
            ws = lab[map.at(ssx, ssy, ssz)];
            lt = label_of(wt);
            ls = label_of(ws);
        }
        __syncthreads();  // LDS counters and tables initialised
        if (tid < prev_n) add_deltas(wr, tid < kEarlyRecords ? early_rec : dl_prev[tid]);
        // The nontrivial attempts are packed into the first lanes of the
        // workgroup: the energy change, which most attempts skip, then runs
        // on as few waves as there are 64 of them, not on every wave that
        // holds one (the sweep is bound by instruction issue more than by
        // memory).  3D multi-type sweeps, bound by memory and with many
        // nontrivial attempts, evaluate where they draw: the extra barrier
        // measured slower there.
        uint32_t accepted = 0;
        int qn = 0;
        if (COMPACT) {
            if (mine && lt != ls && lt >= 0 && ls >= 0) {
                const int slot = atomicAdd(&queue_n, 1);
                const uint32_t off = (uint32_t)((ssx - ttx + 1) + 3 * (ssy - tty + 1) + 9 * (ssz - ttz + 1));
                const uint32_t words = kWideCell ? (uint32_t)wt : ((uint32_t)wt | ((uint32_t)ws << 16));
                queue[slot] = make_int4((int)((uint32_t)ttx | ((uint32_t)tty << 16)),
                                        (int)((uint32_t)ttz | (off << 16)), (int)u2, (int)words);
                if (kWideCell) queue_ws[slot] = (uint32_t)ws;
            }
            __syncthreads();
            qn = queue_n;
            if (tid < qn) {
                const int4 e = queue[tid];
                const uint32_t ex = (uint32_t)e.x, ey = (uint32_t)e.y, off = ey >> 16;
                ttx = (int)(ex & 0xFFFFu), tty = (int)(ex >> 16), ttz = (int)(ey & 0xFFFFu);
                ssx = ttx + (int)(off % 3u) - 1, ssy = tty + (int)((off / 3u) % 3u) - 1;
                ssz = D == 3 ? ttz + (int)(off / 9u) - 1 : 0;
                u2 = (uint32_t)e.z;
                wt = kWideCell ? (Cell)(uint32_t)e.w : (Cell)((uint32_t)e.w & 0xFFFFu);
                ws = kWideCell ? (Cell)queue_ws[tid] : (Cell)((uint32_t)e.w >> 16);
                lt = label_of(wt), ls = label_of(ws);
            }
        } else if (mine && lt != ls && lt >= 0 && ls >= 0) {
            atomicAdd(&n_nontrivial, 1u);
        }
        if (COMPACT ? tid < qn : (mine && lt != ls && lt >= 0 && ls >= 0)) {
            int64_t dso, dsn;
            int tt, ts;
            types(wt, lt, ws, ls, tt, ts);
            // incremental centroids: both cells' reference points, read with
            // the counters
            int4 ref_t = make_int4(0, 0, 0, 0), ref_s = ref_t;
            if (EXT && a.csum) {
                const int4 *cp = plain(a.cpos);
                if (lt > 0) ref_t = cp[lt];
                if (ls > 0) ref_s = cp[ls];
            }
            if (evaluate<Cell, D, ACT, SINGLE, LAYOUT, EXT>(a, tb, jr, sht, lab, lact, map, ttx, tty, ttz, ssx, ssy, ssz,
                                                       map.at(ssx, ssy, ssz), lt, ls, tt, ts,
                                                       seen_counters(rd, lt, nullptr, 0),
                                                       seen_counters(rd, ls, nullptr, 0), u2, dso, dsn)) {
                accepted = 1;
                const int gi = map.at(ttx, tty, ttz);
                commit(gi, gi, lt, ls, ws, ts, dso, dsn);
                if (EXT && a.csum) move_centroids_at<D>(a, ttx, tty, ttz, lt, ls, ref_t, ref_s);
            }
        }
        if (accepted) atomicAdd(&n_accepted, 1u);
        // The wave that finishes last writes the tile's list length and
        // statistics, so that no wave waits at a barrier for the others:
        // waves without nontrivial attempts leave at once and free their
        // slots for the next workgroups.  Each wave's LDS updates complete
        // before it counts itself done.
        if ((tid & 63) == 0) {
            __threadfence_block();
            if (atomicAdd(&waves_done, 1u) == kBlock / 64 - 1) {
                __threadfence_block();
                a.dcount[parity][tile] = list_n;
                a.stats[2 * tile] += COMPACT ? (uint32_t)qn : n_nontrivial;
                a.stats[2 * tile + 1] += n_accepted;
            }
        }
        return;
    }

    // k = 1: the attempt of this thread's area, its two labels (from LDS) and,
    // when nontrivial, their counters as the activation began.  Drawing while
    // the staging loads are in flight, or reading the labels from global
    // memory then, measured slower on gfx950 (the wait for the labels also
    // waits for every staging load issued before them).
    int d_ttx = 0, d_tty = 0, d_ttz = 0, d_ssx = 0, d_ssy = 0, d_ssz = 0, d_lt = 0, d_ls = 0;
    Cell d_wt = 0, d_ws = 0;
    uint32_t d_u2 = 0;
    bool d_nontrivial = false;
    int2 d_ct = make_int2(0, 0), d_cs = make_int2(0, 0);
    auto draw_k1 = [&]() {
        if (!K1 || tid >= areas) return;
        uint32_t area_id;
        draw(tid, 0, d_ttx, d_tty, d_ttz, d_ssx, d_ssy, d_ssz, d_u2, area_id);
        d_wt = lab[map.at(d_ttx, d_tty, d_ttz)];
        d_ws = lab[map.at(d_ssx, d_ssy, d_ssz)];
        d_lt = label_of(d_wt);
        d_ls = label_of(d_ws);
        d_nontrivial = d_lt != d_ls && d_lt >= 0 && d_ls >= 0;
        if (d_nontrivial) {
            d_ct = seen_counters(rd, d_lt, nullptr, 0);
            d_cs = seen_counters(rd, d_ls, nullptr, 0);
        }
    };

    // stage the box (labels, and activity for the Act term)
    const int rows = b1 * b2;
    if (DIRECT) {
        // nothing to stage: attempts read the lattice in place (no other
        // attempt of this activation writes a site that one reads)
    } else if (FULLROW) {
        // whole rows in the widest chunks (16, 8 or 4 bytes) that tile a row,
        // eight loads in flight per thread
        const FastDiv by_b1((uint32_t)b1);
        auto copy_rows = [&](auto chunk, const void *src_v, void *dst_v, int row_bytes) {
            using Chunk = decltype(chunk);
            const Chunk *src = reinterpret_cast<const Chunk *>(src_v);
            Chunk *dst = reinterpret_cast<Chunk *>(dst_v);
            const int per_row = row_bytes / (int)sizeof(Chunk);
            const FastDiv by_row((uint32_t)per_row);
            auto row_chunk = [&](int c) {
                const int r = (int)by_row.div((uint32_t)c), off = c - r * per_row;
                const int rz = (int)by_b1.div((uint32_t)r), ry = r - rz * b1;
                const int gy = wrap_once(o1 + ry, L1);
                const int gz = D == 3 ? wrap_once(o2 + rz, L2) : 0;
                return ((size_t)gz * L1 + gy) * per_row + off;
            };
            const int total = rows * per_row;
            int c0 = tid;
            for (; c0 + 7 * kBlock < total; c0 += 8 * kBlock) {
                // eight independent loads before the first LDS store
                const Chunk v0 = src[row_chunk(c0)];
                const Chunk v1 = src[row_chunk(c0 + kBlock)];
                const Chunk v2 = src[row_chunk(c0 + 2 * kBlock)];
                const Chunk v3 = src[row_chunk(c0 + 3 * kBlock)];
                const Chunk v4 = src[row_chunk(c0 + 4 * kBlock)];
                const Chunk v5 = src[row_chunk(c0 + 5 * kBlock)];
                const Chunk v6 = src[row_chunk(c0 + 6 * kBlock)];
                const Chunk v7 = src[row_chunk(c0 + 7 * kBlock)];
                dst[c0] = v0;
                dst[c0 + kBlock] = v1;
                dst[c0 + 2 * kBlock] = v2;
                dst[c0 + 3 * kBlock] = v3;
                dst[c0 + 4 * kBlock] = v4;
                dst[c0 + 5 * kBlock] = v5;
                dst[c0 + 6 * kBlock] = v6;
                dst[c0 + 7 * kBlock] = v7;
            }
            for (; c0 < total; c0 += kBlock) dst[c0] = src[row_chunk(c0)];
        };
        auto copy_any = [&](int chunk, const void *src, void *dst, int row_bytes) {
            if (chunk == 16) copy_rows(uint4{}, src, dst, row_bytes);
            else if (chunk == 8) copy_rows(uint2{}, src, dst, row_bytes);
            else copy_rows(uint32_t{}, src, dst, row_bytes);
        };
        copy_any(tg.row_chunk, cells, lab, L0 * (int)sizeof(Cell));
        if (ACT && !WordAct<Cell>::kIn) copy_any(tg.act_chunk, plain(a.act), lact, L0);
    } else {
        // the box x fastest, site c of the box at LDS index c: consecutive
        // threads read consecutive sites of a row, eight loads (and eight
        // activity loads) in flight per thread before the LDS stores
        const int total = b0 * rows;
        const FastDiv by_b0((uint32_t)b0), by_b1((uint32_t)b1);
        auto src = [&](int c) {
            const int r = (int)by_b0.div((uint32_t)c), x = c - r * b0;
            const int rz = (int)by_b1.div((uint32_t)r), ry = r - rz * b1;
            const int gx = wrap_once(o0 + x, L0);
            const int gy = wrap_once(o1 + ry, L1);
            const int gz = D == 3 ? wrap_once(o2 + rz, L2) : 0;
            return (int)(((size_t)gz * L1 + gy) * L0 + gx);
        };
        // kBatch sites per thread per round: all their loads are issued
        // before the first LDS store (the arrays are indexed by unrolled
        // constants only, so they stay in registers)
        constexpr int kBatch = 8;
        int c0 = tid;
        for (; c0 + (kBatch - 1) * kBlock < total; c0 += kBatch * kBlock) {
            int idx[kBatch];
            Cell v[kBatch];
            uint8_t w[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) idx[q] = src(c0 + q * kBlock);
#pragma unroll
            for (int q = 0; q < kBatch; ++q) v[q] = cells[idx[q]];
            if (ACT && !WordAct<Cell>::kIn) {
#pragma unroll
                for (int q = 0; q < kBatch; ++q) w[q] = a.act[idx[q]];
            }
#pragma unroll
            for (int q = 0; q < kBatch; ++q) lab[c0 + q * kBlock] = v[q];
            if (ACT && !WordAct<Cell>::kIn) {
#pragma unroll
                for (int q = 0; q < kBatch; ++q) lact[c0 + q * kBlock] = w[q];
            }
        }
        for (; c0 < total; c0 += kBlock) {
            const int i = src(c0);
            lab[c0] = cells[i];
            if (ACT && !WordAct<Cell>::kIn) lact[c0] = a.act[i];
        }
    }
    __syncthreads();

    uint32_t my_accepted = 0;
    JRows jr{0, 0, 0, 0, 0, 0};
    if (SINGLE) {
        const int64_t *J = model->J;
        const int tc = a.single_type, to = a.obstacle_type;
        jr = JRows{J[tc * kMaxTypes + tc], J[tc * kMaxTypes], J[tc * kMaxTypes + to],
                   J[tc], J[0], J[to]};
    }
    if (K1) {
        draw_k1();
        // phase 1: queue the nontrivial attempts with their counters
        if (d_nontrivial) {
            const int slot = atomicAdd(&queue_n, 1);
            if (slot < kQueue) {
                queue[slot] = make_int4(d_ttx | (d_tty << 16), d_ttz | (d_ssz << 16), (d_ssx & 0xFFFF) | (d_ssy << 16),
                                        (int)d_u2);
                queue_cnt[slot] = make_int4(d_ct.x, d_ct.y, d_cs.x, d_cs.y);
            } else {
                // queue full: evaluate here (no other attempt reads this sub-area)
                int64_t dso, dsn;
                int tt, ts;
                types(d_wt, d_lt, d_ws, d_ls, tt, ts);
                if (evaluate<Cell, D, ACT, SINGLE, LAYOUT, EXT>(a, tb, jr, sht, lab, lact, map, d_ttx, d_tty, d_ttz, d_ssx,
                                                            d_ssy, d_ssz, EXT && a.chem ? global_index(d_ssx, d_ssy, d_ssz) : 0,
                                                            d_lt, d_ls, tt, ts, d_ct, d_cs, d_u2, dso, dsn)) {
                    ++my_accepted;
                    commit(map.at(d_ttx, d_tty, d_ttz), global_index(d_ttx, d_tty, d_ttz), d_lt, d_ls, d_ws, ts, dso,
                           dsn);
                }
            }
        }
        __syncthreads();
        // phase 2: energy change and Metropolis test of the queued attempts
        const int qn = queue_n;
        // entry i goes to lane i / 4 of wave i % 4: the work spreads over all waves
        for (int i = ((tid & 63) << 2) | (tid >> 6); i < min(qn, kQueue); i += kBlock) {
            const int4 e = queue[i], c = queue_cnt[i];
            const int ttx = e.x & 0xFFFF, tty = e.x >> 16, ttz = e.y & 0xFFFF;
            const int ssz = e.y >> 16, ssx = (int)(int16_t)(e.z & 0xFFFF), ssy = e.z >> 16;
            const int t = map.at(ttx, tty, ttz);
            const Cell wt = lab[t], ws = lab[map.at(ssx, ssy, ssz)];
            const int lt = label_of(wt), ls = label_of(ws);
            int64_t dso, dsn;
            int tt, ts;
            types(wt, lt, ws, ls, tt, ts);
            if (evaluate<Cell, D, ACT, SINGLE, LAYOUT, EXT>(a, tb, jr, sht, lab, lact, map, ttx, tty, ttz, ssx, ssy, ssz,
                                                        EXT && a.chem ? global_index(ssx, ssy, ssz) : 0, lt, ls, tt, ts,
                                                        make_int2(c.x, c.y), make_int2(c.z, c.w), (uint32_t)e.w,
                                                        dso, dsn)) {
                ++my_accepted;
                commit(t, global_index(ttx, tty, ttz), lt, ls, ws, ts, dso, dsn);
            }
        }
        if (tid == 0) n_nontrivial = (uint32_t)qn;
    } else {
        uint32_t my_nontrivial = 0;
        if (tid < areas) {
            // own accepted copies of this activation: registers, then the spill array
            int4 own[kOwnInRegs];
            int n_own = 0;
            const size_t slot = (size_t)tile * (size_t)(tg.T[0] * tg.T[1] * tg.T[2]) + (size_t)tid;
            int4 *spill = a.own_spill ? plain(a.own_spill) + slot * (size_t)(a.k - kOwnInRegs) : nullptr;
            for (int j = 0; j < a.k; ++j) {
                int ttx, tty, ttz, ssx, ssy, ssz;
                uint32_t u2, area_id;
                draw(tid, j, ttx, tty, ttz, ssx, ssy, ssz, u2, area_id);
                const int t = map.at(ttx, tty, ttz);
                const Cell wt = lab[t], ws = lab[map.at(ssx, ssy, ssz)];
                const int lt = label_of(wt), ls = label_of(ws);
                if (lt != ls && lt >= 0 && ls >= 0) {
                    ++my_nontrivial;
                    int64_t dso, dsn;
                    int tt, ts;
                    types(wt, lt, ws, ls, tt, ts);
                    if (evaluate<Cell, D, ACT, SINGLE, LAYOUT, EXT>(a, tb, jr, sht, lab, lact, map, ttx, tty, ttz, ssx, ssy,
                                                                ssz, EXT && a.chem ? global_index(ssx, ssy, ssz) : 0, lt, ls,
                                                                tt, ts, seen_counters(rd, lt, own, n_own, spill),
                                                                seen_counters(rd, ls, own, n_own, spill), u2, dso, dsn)) {
                        ++my_accepted;
                        const int4 rec = commit(t, global_index(ttx, tty, ttz), lt, ls, ws, ts, dso, dsn);
#pragma unroll
                        for (int jj = 0; jj < kOwnInRegs; ++jj)
                            if (jj == n_own) own[jj] = rec;
                        if (n_own >= kOwnInRegs) spill[n_own - kOwnInRegs] = rec;
                        ++n_own;
                    }
                }
            }
        }
        if (my_nontrivial) atomicAdd(&n_nontrivial, my_nontrivial);
    }
    if (my_accepted) atomicAdd(&n_accepted, my_accepted);
    __syncthreads();
    if (tid == 0) {
        a.dcount[parity][tile] = list_n;
        a.stats[2 * tile] += n_nontrivial;
        a.stats[2 * tile + 1] += n_accepted;
    }
}

// The tile of workgroup b of a single lattice: workgroups go to the XCDs
// round-robin, so b takes the (b div 8)-th tile of the slab of XCD b mod 8:
// in index order, or brick by brick (TileGeometry).
__device__ __forceinline__ int xcd_tile(const TileGeometry &tg, unsigned b)
{
    const int x = (int)(b % kXcds), j = (int)(b / kXcds);
    if (tg.brick_y == 0) return x * tg.tiles_per_xcd + j;
    const int per = tg.brick_y * tg.brick_z;
    const int br = j / per, r = j - br * per;
    const int nby = tg.nt[1] / tg.brick_y;
    const int by = br % nby, bz = br / nby;
    const int ty = by * tg.brick_y + r % tg.brick_y;
    const int tz = x * tg.layers_per_xcd + bz * tg.brick_z + r / tg.brick_y;
    return ty + tg.nt[1] * tz;
}

// One lattice: workgroup b takes tile xcd_tile(b), so each XCD sweeps one
// contiguous slab of tiles in every activation.
template <typename Cell, int D, bool ACT, bool SINGLE, bool K1, int LAYOUT, bool EXT>
__global__ void __launch_bounds__(kBlock) tile_sweep_kernel(SweepArgs a, uint32_t mcs, uint32_t alpha, int parity)
{
    const int tile = xcd_tile(a.tg, blockIdx.x);
    if (tile >= a.tg.n_tiles) return;  // uniform over the block
    sweep_tile<Cell, D, ACT, SINGLE, K1, LAYOUT, EXT>(a, tile, mcs, alpha, parity);
}

// Packed words serve large multi-type lattices and Act models, whose sweeps
// wait on memory: more waves per SIMD hide more of that latency, up to the
// point where the register budget the cap leaves (512 / waves per lane)
// forces spills to scratch memory.  Each cap below is the largest that
// leaves its instantiations spill-free: a 3D multi-type sweep in place holds
// the 26 neighbour words and their J entries at once (loaded in one round;
// with the Act term, the words' activities too); k > 1 attempts per
// activation keep the attempt loop's state; 3D Act terms, the persistence /
// chemotaxis terms in 3D and those of 2D Act models need more than 64
// registers.
#ifndef CPM_PACKED_WAVES
#define CPM_PACKED_WAVES 8
#endif
#ifndef CPM_PACKED_WAVES_3D
#define CPM_PACKED_WAVES_3D 5
#endif
template <typename Word, int D, bool ACT, bool SINGLE, bool K1, int LAYOUT, bool EXT>
struct PackedWaves {
    static constexpr bool kWordAct = std::is_same<Word, char32_t>::value;
    static constexpr int value =
        !K1 ? (ACT && (D == 3 || (SINGLE && EXT)) ? 3 : 4)
        : D == 3 && LAYOUT == kDirect && !SINGLE ? (kWordAct ? CPM_PACKED_WAVES_3D : ACT ? 4 : 6)
        : D == 3 && ACT ? (SINGLE ? 5 : 6)
        : D == 3 && EXT ? 6
        : D == 2 && ACT && (EXT || (LAYOUT == kDirect && !kWordAct)) ? 6
        : CPM_PACKED_WAVES;
};
template <typename Word, int D, bool ACT, bool SINGLE, bool K1, int LAYOUT, bool EXT>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(PackedWaves<Word, D, ACT, SINGLE, K1, LAYOUT, EXT>::value)))
tile_sweep_kernel_packed(SweepArgs a, uint32_t mcs, uint32_t alpha, int parity)
{
    const int tile = xcd_tile(a.tg, blockIdx.x);
    if (tile >= a.tg.n_tiles) return;  // uniform over the block
    sweep_tile<Word, D, ACT, SINGLE, K1, LAYOUT, EXT>(a, tile, mcs, alpha, parity);
}

// Many lattices advanced together: work[b] = (lattice, tile) of workgroup b
// (lattice -1: padding); all lattices share the MCS counter at *mcs.
// The batch kernels read each lattice's arguments from device memory: seen
// through global-memory pointer types, the pointers they hold are read
// through with global loads (a pointer loaded from memory is otherwise a
// flat one, whose loads also hold up the scalar loads' waits).
struct GlobalPtrs {
    template <typename T>
    using ptr = __attribute__((address_space(1))) T *;
};
using SweepArgsG = SweepArgsT<GlobalPtrs>;
static_assert(sizeof(SweepArgsG) == sizeof(SweepArgs) && offsetof(SweepArgsG, tg) == offsetof(SweepArgs, tg),
              "the same bytes seen with other pointer types");

template <typename Cell, int D, bool ACT, bool SINGLE, bool K1, int LAYOUT, bool EXT>
__global__ void __launch_bounds__(kBlock) batch_sweep_kernel(const SweepArgsG *args, const int2 *work,
                                                             const uint32_t *mcs, uint32_t alpha, int parity)
{
    const int2 w = work[blockIdx.x];
    if (w.x < 0) return;  // uniform over the block
    sweep_tile<Cell, D, ACT, SINGLE, K1, LAYOUT, EXT>(args[w.x], w.y, *mcs, alpha, parity);
}

// Device-wide barrier of a persistent launch.  Thread 0 of each workgroup
// arrives after an agent-scope release fence (the workgroup's writes, made
// visible to it by the workgroup barrier, become visible device-wide); the
// last arrival resets the count and bumps the generation, the others poll
// it with relaxed agent-scope loads, and one acquire fence follows the wait
// (an acquire per poll would invalidate the caches at every poll).  A wait
// is bounded: after spin_limit polls the workgroup raises the abort flag,
// and every workgroup leaves at its next barrier once the flag is raised,
// so the launch always ends.  Returns false when leaving.
__device__ __forceinline__ bool grid_sync(const PersistentLaunch &p, uint32_t &gen)
{
    __shared__ uint32_t s_go;
    __syncthreads();
    if (threadIdx.x == 0) {
        GridBarrier *bar = p.bar;
        uint32_t go = 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t g = gen;
        if (__hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1) {
            // the last arrival acquires every other workgroup's release (the
            // count's increments form one release sequence) before its own
            // release of the generation passes them on
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t polls = 0;
            while (__hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                    polls++ >= p.spin_limit) {
                    __hip_atomic_store(&bar->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    go = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        gen = g + 1;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) go = 0;
        s_go = go;
    }
    __syncthreads();
    return s_go != 0u;
}

// The Act decay of a whole batch (one MCS), grid-stride: the activity as
// stored (uint8 array, or the bits of the words), lowered by one where
// positive.
__device__ __forceinline__ void decay_all(const PersistentLaunch &p)
{
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < p.n_sites; i += stride) {
        if (p.decay_mode == 1) {
            uint8_t *a = static_cast<uint8_t *>(p.decay_ptr);
            const uint8_t v = a[i];
            if (v) a[i] = (uint8_t)(v - 1);
        } else if (p.decay_mode == 2) {
            uint32_t *w = static_cast<uint32_t *>(p.decay_ptr);
            const uint32_t v = w[i];
            if (v >> 24) w[i] = v - (1u << 24);
        } else if (p.decay_mode == 3) {
            uint16_t *w = static_cast<uint16_t *>(p.decay_ptr);
            const uint32_t v = w[i];
            if (v >> 11) w[i] = (uint16_t)(v - (1u << 11));
        }
    }
}

// n_mcs MCS of a batch swept in place (k = 1) in one launch: the workgroups
// (all resident) loop over the work table (entry w on workgroup w mod grid,
// which keeps the table's XCD assignment when the grid is a multiple of the
// XCD count), and meet at a grid barrier after each activation and after
// each MCS's Act decay.
template <typename Cell, int D, bool ACT, bool SINGLE, bool EXT>
__global__ void __launch_bounds__(kBlock) batch_persistent_kernel(const SweepArgsG *args, const int2 *work,
                                                                  PersistentLaunch p)
{
    uint32_t gen = 0;
    for (int m = 0; m < p.n_mcs; ++m) {
        const uint32_t mcs = p.mcs0 + (uint32_t)m;
        for (uint32_t alpha = 0; alpha < p.n_act; ++alpha) {
            for (int w = (int)blockIdx.x; w < p.n_work; w += (int)gridDim.x) {
                const int2 wk = work[w];
                if (wk.x < 0) continue;  // uniform over the block
                sweep_tile<Cell, D, ACT, SINGLE, true, kDirect, EXT>(args[wk.x], wk.y, mcs, alpha, (int)(alpha & 1));
                __syncthreads();
            }
            if (!grid_sync(p, gen)) return;
        }
        if (ACT) {
            decay_all(p);
            if (!grid_sync(p, gen)) return;
        }
    }
}

template <typename Cell, int D, bool ACT, bool SINGLE, bool EXT>
hipError_t launch_persistent_k(const BatchLaunch &b, const PersistentLaunch &p, hipStream_t st)
{
    const void *kern = reinterpret_cast<const void *>(&batch_persistent_kernel<Cell, D, ACT, SINGLE, EXT>);
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_persistent_kernel<Cell, D, ACT, SINGLE, EXT>,
                                                               kBlock, b.lds);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int grid = std::min(per_cu * cus, b.grid);
    grid = grid / kXcds * kXcds;
    if (grid < kXcds) return hipErrorInvalidConfiguration;
    const SweepArgsG *args = reinterpret_cast<const SweepArgsG *>(b.args);
    const int2 *work = b.work;
    PersistentLaunch pl = p;
    void *kargs[] = {(void *)&args, (void *)&work, (void *)&pl};
    return hipLaunchCooperativeKernel(kern, dim3((unsigned)grid), dim3(kBlock), kargs, (unsigned)b.lds, st);
}

template <typename Cell, int D, bool ACT, bool SINGLE, bool EXT>
hipError_t launch_k(const SweepArgs &a, bool k1, int layout, uint32_t mcs, uint32_t alpha, int parity, size_t lds,
                    hipStream_t st)
{
    if (k1 && layout == kDirect)
        tile_sweep_kernel<Cell, D, ACT, SINGLE, true, kDirect, EXT><<<a.tg.grid, kBlock, lds, st>>>(a, mcs, alpha, parity);
    else if (k1 && layout == kFullRow)
        tile_sweep_kernel<Cell, D, ACT, SINGLE, true, kFullRow, EXT><<<a.tg.grid, kBlock, lds, st>>>(a, mcs, alpha, parity);
    else if (k1)
        tile_sweep_kernel<Cell, D, ACT, SINGLE, true, kBox, EXT><<<a.tg.grid, kBlock, lds, st>>>(a, mcs, alpha, parity);
    else
        tile_sweep_kernel<Cell, D, ACT, SINGLE, false, kBox, EXT><<<a.tg.grid, kBlock, lds, st>>>(a, mcs, alpha, parity);
    return hipGetLastError();
}

template <typename Cell, int D, bool ACT>
hipError_t launch_s(const SweepArgs &a, uint32_t mcs, uint32_t alpha, int parity, size_t lds, hipStream_t st)
{
    const bool k1 = a.k == 1;
    const int layout = a.tg.layout;
    // the persistence and chemotaxis terms are compiled in only where used
    const bool ext = a.pdir || a.chem;
    if (a.single_type >= 0)
        return ext ? launch_k<Cell, D, ACT, true, true>(a, k1, layout, mcs, alpha, parity, lds, st)
                   : launch_k<Cell, D, ACT, true, false>(a, k1, layout, mcs, alpha, parity, lds, st);
    return ext ? launch_k<Cell, D, ACT, false, true>(a, k1, layout, mcs, alpha, parity, lds, st)
               : launch_k<Cell, D, ACT, false, false>(a, k1, layout, mcs, alpha, parity, lds, st);
}

// Packed words (multi-type models only): no single-type kernels needed.
template <typename Word, int D, bool ACT, bool SINGLE, bool EXT>
hipError_t launch_packed_k(const SweepArgs &a, uint32_t mcs, uint32_t alpha, int parity, size_t lds, hipStream_t st)
{
    const bool k1 = a.k == 1;
    const int layout = a.tg.layout;
    if (k1 && layout == kDirect)
        tile_sweep_kernel_packed<Word, D, ACT, SINGLE, true, kDirect, EXT><<<a.tg.grid, kBlock, lds, st>>>(a, mcs, alpha, parity);
    else if (k1 && layout == kFullRow)
        tile_sweep_kernel_packed<Word, D, ACT, SINGLE, true, kFullRow, EXT><<<a.tg.grid, kBlock, lds, st>>>(a, mcs, alpha, parity);
    else if (k1)
        tile_sweep_kernel_packed<Word, D, ACT, SINGLE, true, kBox, EXT><<<a.tg.grid, kBlock, lds, st>>>(a, mcs, alpha, parity);
    else
        tile_sweep_kernel_packed<Word, D, ACT, SINGLE, false, kBox, EXT><<<a.tg.grid, kBlock, lds, st>>>(a, mcs, alpha, parity);
    return hipGetLastError();
}

// Label-type words serve multi-type models only; label-type-activity words
// serve every Act model that fits them.
template <typename Word, int D, bool ACT>
hipError_t launch_packed_s(const SweepArgs &a, uint32_t mcs, uint32_t alpha, int parity, size_t lds, hipStream_t st)
{
    const bool ext = a.pdir || a.chem;
    if constexpr (std::is_same<Word, char32_t>::value) {
        if (a.single_type >= 0)
            return ext ? launch_packed_k<Word, D, ACT, true, true>(a, mcs, alpha, parity, lds, st)
                       : launch_packed_k<Word, D, ACT, true, false>(a, mcs, alpha, parity, lds, st);
    }
    return ext ? launch_packed_k<Word, D, ACT, false, true>(a, mcs, alpha, parity, lds, st)
               : launch_packed_k<Word, D, ACT, false, false>(a, mcs, alpha, parity, lds, st);
}


template <typename Cell, int D, bool ACT, bool SINGLE, bool EXT>
hipError_t launch_batch_k(const BatchLaunch &b, uint32_t alpha, int parity, hipStream_t st)
{
    if (b.k1 && b.layout == kDirect)
        batch_sweep_kernel<Cell, D, ACT, SINGLE, true, kDirect, EXT><<<b.grid, kBlock, b.lds, st>>>(reinterpret_cast<const SweepArgsG *>(b.args), b.work, b.mcs, alpha, parity);
    else if (b.k1 && b.layout == kFullRow)
        batch_sweep_kernel<Cell, D, ACT, SINGLE, true, kFullRow, EXT><<<b.grid, kBlock, b.lds, st>>>(reinterpret_cast<const SweepArgsG *>(b.args), b.work, b.mcs, alpha, parity);
    else if (b.k1)
        batch_sweep_kernel<Cell, D, ACT, SINGLE, true, kBox, EXT><<<b.grid, kBlock, b.lds, st>>>(reinterpret_cast<const SweepArgsG *>(b.args), b.work, b.mcs, alpha, parity);
    else
        batch_sweep_kernel<Cell, D, ACT, SINGLE, false, kBox, EXT><<<b.grid, kBlock, b.lds, st>>>(reinterpret_cast<const SweepArgsG *>(b.args), b.work, b.mcs, alpha, parity);
    return hipGetLastError();
}

template <typename Cell, int D, bool ACT>
hipError_t launch_batch_s(const BatchLaunch &b, uint32_t alpha, int parity, hipStream_t st)
{
    if (b.single)
        return b.ext ? launch_batch_k<Cell, D, ACT, true, true>(b, alpha, parity, st)
                     : launch_batch_k<Cell, D, ACT, true, false>(b, alpha, parity, st);
    return b.ext ? launch_batch_k<Cell, D, ACT, false, true>(b, alpha, parity, st)
                 : launch_batch_k<Cell, D, ACT, false, false>(b, alpha, parity, st);
}

}  // namespace

// One activation of a single lattice whose sweep reads stored words of type
// Cell, in D dimensions: the kernel specialised for the model's terms,
// cell types, k and layout.
template <typename Cell, int D>
hipError_t sweep_words(const SweepArgs &a, bool act, uint32_t mcs, uint32_t alpha, int parity, size_t lds,
                       hipStream_t st)
{
    if constexpr (std::is_same<Cell, int32_t>::value || std::is_same<Cell, uint16_t>::value)
        return act ? launch_s<Cell, D, true>(a, mcs, alpha, parity, lds, st)
                   : launch_s<Cell, D, false>(a, mcs, alpha, parity, lds, st);
    else if constexpr (std::is_same<Cell, uint32_t>::value)
        return act ? launch_packed_s<Cell, D, true>(a, mcs, alpha, parity, lds, st)
                   : launch_packed_s<Cell, D, false>(a, mcs, alpha, parity, lds, st);
    else  // words that carry the activity serve Act models only
        return launch_packed_s<Cell, D, true>(a, mcs, alpha, parity, lds, st);
}

// A persistent launch of a batch (in place, k = 1).
template <typename Cell, int D>
hipError_t batch_persistent_words(const BatchLaunch &b, const PersistentLaunch &p, hipStream_t st)
{
    constexpr bool kWordAct = WordAct<Cell>::kIn;
    if constexpr (std::is_same<Cell, char16_t>::value)  // one cell type, no chemotaxis
        return launch_persistent_k<Cell, D, true, true, false>(b, p, st);
    else if constexpr (kWordAct)
        return b.single ? (b.ext ? launch_persistent_k<Cell, D, true, true, true>(b, p, st)
                                 : launch_persistent_k<Cell, D, true, true, false>(b, p, st))
                        : (b.ext ? launch_persistent_k<Cell, D, true, false, true>(b, p, st)
                                 : launch_persistent_k<Cell, D, true, false, false>(b, p, st));
    else if (b.act)
        return b.single ? (b.ext ? launch_persistent_k<Cell, D, true, true, true>(b, p, st)
                                 : launch_persistent_k<Cell, D, true, true, false>(b, p, st))
                        : (b.ext ? launch_persistent_k<Cell, D, true, false, true>(b, p, st)
                                 : launch_persistent_k<Cell, D, true, false, false>(b, p, st));
    else
        return b.single ? (b.ext ? launch_persistent_k<Cell, D, false, true, true>(b, p, st)
                                 : launch_persistent_k<Cell, D, false, true, false>(b, p, st))
                        : (b.ext ? launch_persistent_k<Cell, D, false, false, true>(b, p, st)
                                 : launch_persistent_k<Cell, D, false, false, false>(b, p, st));
}

// One activation of every lattice of a batch.
template <typename Cell, int D>
hipError_t batch_words(const BatchLaunch &b, uint32_t alpha, int parity, hipStream_t st)
{
    if constexpr (std::is_same<Cell, int32_t>::value || std::is_same<Cell, uint16_t>::value)
        return b.act ? launch_batch_s<Cell, D, true>(b, alpha, parity, st)
                     : launch_batch_s<Cell, D, false>(b, alpha, parity, st);
    else if constexpr (std::is_same<Cell, char16_t>::value)  // one cell type, no chemotaxis
        return launch_batch_k<Cell, D, true, true, false>(b, alpha, parity, st);
    else
        return launch_batch_s<Cell, D, true>(b, alpha, parity, st);
}

}  // namespace cpm
