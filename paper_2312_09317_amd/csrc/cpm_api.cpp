// Host side of libcpm: parameter validation, fixed-point quantisation,
// FP64-built acceptance / activity tables, workspace carving and the C ABI
// declared in include/cpm.h.
#include <algorithm>
#include <cmath>
#include <vector>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>

#include "../../include/cpm.h"
#include "cpm_internal.hpp"

using cpm::DeviceModel;
using cpm::SweepArgs;

struct cpm_handle {
    int32_t ndim = 0;
    int32_t L[3] = {1, 1, 1};
    int32_t s = 0, k = 0;
    int32_t n_cells = 0;
    int32_t n_types = 0;
    bool act = false;
    bool mirror = false;             // sweeps run on a 16-bit copy of the lattice
    uint16_t *mirror_cells = nullptr;
    int words = cpm::kWords32;       // what sweeps read: int32 labels, the 16-bit copy or packed words
    SweepArgs args{};
    int32_t *ref = nullptr;          // centroid reference sites, n_cells + 1
    int32_t *check = nullptr;        // invariant checks: flag word, then recounted V and S
    bool obstacles = false;          // the model has an obstacle type (label -1 allowed)
    // persistence (NULL pdir = off): directions, centroid history, centroid
    // sums (kept by the sweeps) and the cells' reference points
    int4 *pdir = nullptr;
    int64_t *hist = nullptr;
    int64_t *csum = nullptr;
    int4 *cpos = nullptr;
    bool incremental = false;        // centroid sums kept by the sweeps (else recounted per update)
    int32_t persist_slots = 0;
    int64_t persist_t = 0;           // direction updates done
    uint64_t mcs = 0;                // next MCS index
    uint64_t activation = 0;         // activations run so far (buffer parity)
    uint64_t attempts_run = 0;       // copy attempts run since init
    std::unique_ptr<DeviceModel> host_model;  // source of the async upload
    int static_device = -1;          // device whose static workspace the handle holds (cpm_init_static), else -1
};

struct cpm_batch {
    int32_t n = 0;
    int32_t ndim = 0, s = 0, k = 0;
    bool act = false, mirror = false, single = false;
    bool act_words = false;          // Act batches sweep on label-type-activity words
    bool act16 = false;              // ... or, with small lattices of one cell type, on 16-bit label-activity words
    uint16_t *words16 = nullptr;     // those words, packed like the int32 lattices
    int layout = 0;
    std::vector<SweepArgs> args;                     // host copies, one per lattice
    std::vector<int32_t> n_cells;
    std::vector<size_t> site_off, label_off;         // packed offsets of lattices / cell-type arrays
    std::vector<int32_t *> ref;
    std::vector<int32_t *> check;                    // per lattice: flag word, then recounted V and S
    std::vector<uint8_t> obstacles;                  // per lattice: label -1 allowed
    std::vector<uint16_t *> mirror_cells;
    std::vector<std::unique_ptr<DeviceModel>> models;
    std::vector<int2> work;
    SweepArgs *d_args = nullptr;
    int2 *d_work = nullptr;
    uint32_t *d_mcs = nullptr;
    int32_t *lattices = nullptr;
    uint8_t *act_field = nullptr;
    size_t total_sites = 0;
    cpm::BatchLaunch launch{};
    cpm::StatsTables stats_tables{};
    int32_t *scratch_v = nullptr, *scratch_s = nullptr;
    int64_t *scratch_c = nullptr;
    int32_t *scratch_ref = nullptr;  // centroid reference sites, packed per label
    std::vector<int64_t> host_label_off;
    std::vector<int32_t> host_dims;
    uint64_t mcs = 0;
    uint64_t activation = 0;
    uint64_t mcs_run = 0;
    size_t max_sites = 0;
    int64_t max_bricks = 0;          // largest centroid-reduction grid of the lattices
    bool use_graph = true;
    int mode = 0;                    // 0: one graph replay per MCS, 1: kernels one by one, 2: persistent launch
    cpm::GridBarrier *bar = nullptr; // barrier of the persistent launch
    uint32_t spin_limit = 1u << 20;  // polls of a barrier wait before the launch gives up
    hipGraphExec_t mcs_graph = nullptr;  // one MCS: every activation, act decay, MCS counter
    ~cpm_batch()
    {
        if (mcs_graph) (void)hipGraphExecDestroy(mcs_graph);
    }
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int device_fail(hipError_t e, const char *where)
{
    return fail(CPM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace

int cpm::report_error(int code, const char *msg) { return fail(code, msg); }

namespace {

// Round half away from zero onto the 2^-16 grid.
int64_t to_fixed(double x) { return (int64_t)std::llround(x * 65536.0); }

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t model, counters0, counters1, dlist, dcount, stats, own, ref, check, mirror, pdir, hist, csum, cpos, total;
    cpm::TileGeometry tg;
    bool mirror_on;
    int32_t dlist_cap;
};

// Labels fit the 16-bit working copy (label + 1): cells 1..65534, medium 0,
// obstacle -1.
bool use_mirror(int32_t n_cells) { return n_cells <= 65534; }
// Act models of up to 2^20 - 2 cells sweep on label-type-activity words
// instead (one load per neighbour for label and activity).
bool use_act_words(const cpm_params *p, int32_t n_cells);
// The 16-bit copy for a single lattice of this model.
bool use_mirror(const cpm_params *p, int32_t n_cells) { return use_mirror(n_cells) && !use_act_words(p, n_cells); }
// Packed words hold label + 1 in 24 bits.
constexpr int32_t kMaxPackedCells = (1 << 24) - 2;
// ... and in 20 bits when the activity shares the word.
constexpr int32_t kMaxPackedActCells = (1 << 20) - 2;

bool use_act_words(const cpm_params *p, int32_t n_cells) { return p->act_enabled && n_cells <= kMaxPackedActCells; }

// Widest load (16, 8 or 4 bytes) that divides both a row and the base address.
int32_t chunk_for(const void *base, size_t row_bytes)
{
    const uintptr_t v = reinterpret_cast<uintptr_t>(base) | (uintptr_t)row_bytes;
    return (v % 16 == 0) ? 16 : (v % 8 == 0 ? 8 : 4);
}

// Thread areas per workgroup tile.  Preferred: whole rows of areas along x
// (full-row LDS layout: every staged row is one aligned lattice row, no row
// staged twice), growing along y then z up to kBlock areas while the staged
// rows fit 64 KiB of LDS.  Otherwise a box tile, shrunk until it fits.
// k = 1 sweeps read the lattice in place (no LDS staging) unless the
// parameters ask for another layout.
constexpr bool kDirectForK1 = true;
constexpr size_t kLdsLimit = 160 * 1024;  // LDS per workgroup on gfx950

// Tile geometry for layout L (0 = halo boxes, 1 = full rows, 2 = in place;
// -1 = choose), honouring the requested tile (p->tile, 0 = choose).  Returns
// false when the layout cannot run this model.
// act_in_word: the stored words carry the activity, so no activity array is
// staged next to them.
bool tile_geometry(const cpm_params *p, bool mirror, int force_layout, cpm::TileGeometry &g, bool act_in_word = false)
{
    g = cpm::TileGeometry{};
    const int s = p->sub, R = p->act_enabled ? 2 : 1;
    const bool act = p->act_enabled != 0 && !act_in_word;  // an activity array staged in LDS
    const int cell = mirror ? 2 : 4;
    int na[3] = {1, 1, 1};
    for (int d = 0; d < p->ndim; ++d) na[d] = p->dims[d] / (2 * s);
    auto extent = [&](int T) { return 2 * s * (T - 1) + s + 2 * R; };
    const size_t budget = 65536;
    int T[3] = {1, 1, 1};
    const int L0 = p->dims[0];
    const int *want = p->tile;
    auto finish = [&](int layout) {
        g.layout = layout;
        g.n_tiles = 1;
        for (int d = 0; d < 3; ++d) {
            g.T[d] = T[d];
            g.nt[d] = (na[d] + T[d] - 1) / T[d];
            g.n_tiles *= g.nt[d];
        }
        g.tiles_per_xcd = (g.n_tiles + cpm::kXcds - 1) / cpm::kXcds;
        g.grid = g.tiles_per_xcd * cpm::kXcds;
        // floor(n / d) = umulhi(n, m) with m = floor((2^32 - 1) / d) + 1,
        // exact for n d < 2^32 (the kernel's FastDiv)
        auto magic = [](int d) { return d > 1 ? 0xFFFFFFFFu / (uint32_t)d + 1u : 0u; };
        for (int d = 0; d < 2; ++d) {
            g.div_nt[d] = magic(g.nt[d]);
            g.div_T[d] = magic(T[d]);
            g.div_last[d] = magic(na[d] - (g.nt[d] - 1) * T[d]);
        }
        g.div_s = magic(s);
        // the tile index divisions are exact while n_tiles * nt < 2^32
        if ((uint64_t)g.n_tiles * (uint64_t)std::max(g.nt[0], g.nt[1]) >= ((uint64_t)1 << 32)) return false;
        if (p->tile_order == 2) {
            // bricks need 3D tiles spanning whole rows and whole layers per XCD
            if (p->ndim != 3 || g.nt[0] != 1 || g.nt[2] % cpm::kXcds != 0) return false;
            g.layers_per_xcd = g.nt[2] / cpm::kXcds;
            g.brick_y = 1;
            for (int by = 1; by <= std::min(16, g.nt[1]); ++by)
                if (g.nt[1] % by == 0) g.brick_y = by;
            g.brick_z = 1;
            for (int bz = 1; bz <= std::min(16, g.layers_per_xcd); ++bz)
                if (g.layers_per_xcd % bz == 0 && g.brick_y * bz <= 256) g.brick_z = bz;
        }
        return true;
    };
    const bool k1 = p->attempts == 1;
    // in place needs every side below 2^16 (queued attempts hold their
    // coordinates in 16 bits); larger lattices take a staged layout
    bool direct_ok = k1;
    for (int d = 0; d < p->ndim; ++d) direct_ok = direct_ok && p->dims[d] <= 65535;
    if (force_layout < 0) force_layout = direct_ok && kDirectForK1 ? 2 : -1;
    if (force_layout == 2) {
        if (!direct_ok) return false;
        // in place: tiles of up to kBlock areas, whole rows of areas first;
        // in 3D the rest split evenly between y and z (a squarer cross
        // section shares more of its neighbours' rows)
        T[0] = want[0] ? want[0] : std::min(na[0], cpm::kBlock);
        const int rest = cpm::kBlock / T[0];
        int t1 = rest;
        if (p->ndim == 3)
            while (t1 > 1 && t1 * t1 > rest) --t1;
        T[1] = want[1] ? want[1] : std::min(na[1], t1);
        T[2] = p->ndim == 3 ? (want[2] ? want[2] : std::min(na[2], cpm::kBlock / (T[0] * T[1]))) : 1;
        g.box_sites = 0;
        g.lds_bytes = 0;
        return finish(2);
    }
    // rows are staged in 16-, 8- or 4-byte chunks: 16-bit rows are even-length
    // (L0 is a multiple of 2s), activity rows a multiple of 4 bytes (s >= 2)
    const bool can_rows = k1 && na[0] <= cpm::kBlock && (L0 * cell) % 4 == 0 && (!act || L0 % 4 == 0) &&
                          (want[0] == 0 || want[0] == na[0]);
    if (force_layout == 1 || force_layout < 0) {
        auto lds_for = [&](int t1, int t2) {
            const int rows = extent(t1) * (p->ndim == 3 ? extent(t2) : 1);
            return cpm::sweep_lds_bytes(p->ndim, act, mirror, rows * L0);
        };
        T[0] = na[0];
        bool ok = can_rows;
        if (ok && (want[1] || want[2])) {
            T[1] = want[1] ? want[1] : 1;
            T[2] = p->ndim == 3 && want[2] ? want[2] : 1;
            ok = lds_for(T[1], T[2]) <= kLdsLimit && T[0] * T[1] * T[2] <= cpm::kBlock;
        } else if (ok) {
            ok = lds_for(1, 1) <= budget;
            if (ok) {
                while (T[1] < na[1] && T[0] * (T[1] + 1) <= cpm::kBlock && lds_for(T[1] + 1, 1) <= budget) ++T[1];
                if (p->ndim == 3)
                    while (T[2] < na[2] && T[0] * T[1] * (T[2] + 1) <= cpm::kBlock &&
                           lds_for(T[1], T[2] + 1) <= budget)
                        ++T[2];
            }
        }
        if (ok) {
            const int rows = extent(T[1]) * (p->ndim == 3 ? extent(T[2]) : 1);
            g.box_sites = rows * L0;
            g.lds_bytes = (int32_t)lds_for(T[1], T[2]);
            return finish(1);
        }
        if (force_layout == 1) return false;
        T[0] = T[1] = T[2] = 1;
    }
    // Box tiles: the requested tile, or of all tiles of at most kBlock areas
    // whose box fits the budget, the one that moves the fewest bytes per
    // activation over the whole lattice, counting every staged row in
    // 128-byte cache lines (halo overlap, ragged edge tiles and short rows all
    // cost); ties go to larger tiles.
    if (want[0] || want[1] || want[2]) {
        T[0] = want[0] ? want[0] : 1;
        T[1] = want[1] ? want[1] : 1;
        T[2] = p->ndim == 3 && want[2] ? want[2] : 1;
        const int box = extent(T[0]) * extent(T[1]) * (p->ndim == 3 ? extent(T[2]) : 1);
        const size_t bytes = cpm::sweep_lds_bytes(p->ndim, act, mirror, box);
        if (bytes > kLdsLimit) return false;
        g.box_sites = box;
        g.lds_bytes = (int32_t)bytes;
        return finish(0);
    }
    const int t2max = p->ndim == 3 ? std::min(na[2], cpm::kBlock) : 1;
    double best = -1.0;
    int best_areas = 0;
    for (int t0 = 1; t0 <= std::min(na[0], cpm::kBlock); ++t0)
        for (int t1 = 1; t1 <= std::min(na[1], cpm::kBlock / t0); ++t1)
            for (int t2 = 1; t2 <= std::min(t2max, cpm::kBlock / (t0 * t1)); ++t2) {
                const int e0 = extent(t0), e1 = extent(t1), e2 = p->ndim == 3 ? extent(t2) : 1;
                const int box = e0 * e1 * e2;
                const size_t bytes = cpm::sweep_lds_bytes(p->ndim, act, mirror, box);
                if (bytes > budget && !(t0 == 1 && t1 == 1 && t2 == 1)) continue;
                const double tiles =
                    (double)((na[0] + t0 - 1) / t0) * ((na[1] + t1 - 1) / t1) * ((na[2] + t2 - 1) / t2);
                const double seg = 128.0;
                double row = std::ceil(e0 * (double)cell / seg) * seg;
                if (act) row += std::ceil(e0 / seg) * seg;
                const double cost = tiles * row * e1 * e2;
                const int areas = t0 * t1 * t2;
                if (best < 0 || cost < best * 0.999 || (cost <= best * 1.001 && areas > best_areas)) {
                    best = cost;
                    best_areas = areas;
                    T[0] = t0, T[1] = t1, T[2] = t2;
                    g.box_sites = box;
                    g.lds_bytes = (int32_t)bytes;
                }
            }
    return finish(0);
}

// The layout the parameters ask for (0 in cpm_params = the library's choice).
int requested_layout(const cpm_params *p) { return p->layout >= 1 && p->layout <= 3 ? p->layout - 1 : -1; }

constexpr size_t kCheckPad = 64;

Layout layout_of(const cpm_params *p, int32_t n_cells, int mirror = -1, int force_layout = -1)
{
    Layout l{};
    l.mirror_on = mirror < 0 ? use_mirror(p, n_cells) : mirror != 0;
    tile_geometry(p, l.mirror_on, force_layout >= 0 ? force_layout : requested_layout(p), l.tg,
                  !l.mirror_on && use_act_words(p, n_cells));
    l.dlist_cap = l.tg.T[0] * l.tg.T[1] * l.tg.T[2] * p->attempts;
    int64_t n_sites = (int64_t)p->dims[0] * p->dims[1] * p->dims[2];
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    l.model = take(sizeof(DeviceModel));
    l.counters0 = take(sizeof(int32_t) * 2 * ((size_t)n_cells + 1));
    l.counters1 = take(sizeof(int32_t) * 2 * ((size_t)n_cells + 1));
    l.dlist = take(2 * sizeof(int4) * (size_t)l.tg.n_tiles * (size_t)l.dlist_cap);
    l.dcount = take(2 * sizeof(int32_t) * (size_t)l.tg.n_tiles);
    l.stats = take(sizeof(uint64_t) * 2 * (size_t)l.tg.n_tiles);
    // own accepted copies past the first kOwnInRegs of a thread in one activation
    const size_t spill = p->attempts > cpm::kOwnInRegs ? (size_t)(p->attempts - cpm::kOwnInRegs) : 0;
    l.own = take(sizeof(int4) * (size_t)l.tg.n_tiles * (size_t)(l.tg.T[0] * l.tg.T[1] * l.tg.T[2]) * spill);
    l.ref = take(sizeof(int32_t) * ((size_t)n_cells + 1));
    // invariant checks: a flag word (padded to 64 words), then a recount of V and S
    l.check = take(sizeof(int32_t) * (kCheckPad + 2 * ((size_t)n_cells + 1)));
    l.mirror = take(l.mirror_on ? sizeof(uint16_t) * (size_t)n_sites : 0);
    const bool pers = p->lambda_persistence != nullptr;
    const size_t labels = (size_t)n_cells + 1;
    l.pdir = take(pers ? sizeof(int4) * labels : 0);
    l.hist = take(pers ? sizeof(int64_t) * 3 * labels * (size_t)(p->persistence_dt + 1) : 0);
    l.csum = take(pers ? sizeof(int64_t) * (size_t)p->ndim * labels : 0);
    l.cpos = take(pers ? sizeof(int4) * labels : 0);
    l.total = off;
    return l;
}

int n_neighbours(int ndim) { return ndim == 2 ? 8 : 26; }

// Largest h with floor(2^32 exp(-h/T)) >= 1, plus one.
int table_length(double T)
{
    int h = 0;
    while (h <= cpm::kMaxTI && std::floor(std::exp(-(double)h / T) * 4294967296.0) >= 1.0) ++h;
    return h;
}

int validate(const cpm_params *p, int32_t n_cells)
{
    if (!p) return fail(CPM_EINVAL, "params is NULL");
    if (p->ndim != 2 && p->ndim != 3) return fail(CPM_EINVAL, "ndim must be 2 or 3");
    if (p->ndim == 2 && p->dims[2] != 1) return fail(CPM_EINVAL, "dims[2] must be 1 in 2D");
    if (p->sub < 1) return fail(CPM_EINVAL, "sub (s) must be >= 1");
    int64_t n_sites = 1;
    for (int d = 0; d < 3; ++d) {
        if (p->dims[d] < 1) return fail(CPM_EINVAL, "dims must be positive");
        n_sites *= p->dims[d];
    }
    for (int d = 0; d < p->ndim; ++d)
        if (p->dims[d] % (2 * p->sub) != 0) return fail(CPM_EINVAL, "every dim must be divisible by 2*sub");
    if (n_sites > ((int64_t)1 << 31) - 1) return fail(CPM_EINVAL, "lattice has more than 2^31-1 sites");
    int64_t sd = 1;
    for (int d = 0; d < p->ndim; ++d) sd *= p->sub;
    if (p->attempts < 1 || sd % p->attempts != 0)
        return fail(CPM_EINVAL, "attempts (k) must be >= 1 and divide sub^ndim");
    if (((int64_t)1 << p->ndim) * sd / p->attempts > ((int64_t)1 << 24))
        return fail(CPM_EINVAL, "too many activations per MCS");
    if (p->attempts > 255) return fail(CPM_EINVAL, "attempts (k) must be <= 255");
    if (n_cells < 0 || n_cells > INT32_MAX - 1) return fail(CPM_EINVAL, "n_cells out of range");
    if (p->n_types < 1 || p->n_types > CPM_MAX_TYPES) return fail(CPM_EINVAL, "n_types must be in 1..16");
    if (p->obstacle_type < -1 || p->obstacle_type >= p->n_types) return fail(CPM_EINVAL, "bad obstacle_type");
    if (!(p->temperature > 0.0) || !std::isfinite(p->temperature))
        return fail(CPM_EINVAL, "temperature must be positive and finite");
    if (!p->J || !p->lambda_volume || !p->volume_target) return fail(CPM_EINVAL, "J / lambda_volume / volume_target NULL");
    if (p->lambda_surface && !p->surface_target) return fail(CPM_EINVAL, "surface_target NULL");
    if (p->act_enabled) {
        if (!p->lambda_act || !p->max_act) return fail(CPM_EINVAL, "lambda_act / max_act NULL with act enabled");
        if (p->sub < 2) return fail(CPM_EINVAL, "the Act term reads two sites out: sub must be >= 2");
    }
    if (p->layout < 0 || p->layout > 3) return fail(CPM_EINVAL, "layout must be 0..3");
    if (p->tile_order < 0 || p->tile_order > 2) return fail(CPM_EINVAL, "tile_order must be 0..2");
    {
        int areas = 1;
        for (int d = 0; d < 3; ++d) {
            const int na = d < p->ndim ? p->dims[d] / (2 * p->sub) : 1;
            if (p->tile[d] < 0 || p->tile[d] > na) return fail(CPM_EINVAL, "tile exceeds the thread areas per axis");
            areas *= p->tile[d] ? p->tile[d] : 1;
        }
        if (areas > cpm::kBlock) return fail(CPM_EINVAL, "a tile holds at most 256 thread areas");
        if (p->ndim == 2 && p->tile[2] > 1) return fail(CPM_EINVAL, "tile[2] must be 0 or 1 in 2D");
        if (p->layout >= 2 && p->attempts != 1) return fail(CPM_ENOTSUP, "layouts 2 and 3 need attempts == 1");
        cpm::TileGeometry g;
        if (!tile_geometry(p, use_mirror(p, n_cells), requested_layout(p), g, use_act_words(p, n_cells)))
            return fail(CPM_ENOTSUP, "the requested layout / tile / tile order does not fit this model");
    }
    const int n = p->n_types;
    const int nnb = n_neighbours(p->ndim);
    const double lim = 2147483647.0 / 65536.0;  // |parameter| < 2^15
    double jmax = 0, lvmax = 0, lsmax = 0, ramax = 0, vtmax = 0, stmax = 0;
    for (int a = 0; a < n; ++a) {
        for (int b = 0; b < n; ++b) {
            const double j = p->J[a * n + b];
            if (!std::isfinite(j) || std::fabs(j) >= lim) return fail(CPM_ERANGE, "J out of range");
            if (to_fixed(j) != to_fixed(p->J[b * n + a])) return fail(CPM_EINVAL, "J must be symmetric");
            jmax = std::fmax(jmax, std::fabs(j));
        }
        const double lv = p->lambda_volume[a];
        const double ls = p->lambda_surface ? p->lambda_surface[a] : 0.0;
        if (!std::isfinite(lv) || std::fabs(lv) >= lim || !std::isfinite(ls) || std::fabs(ls) >= lim)
            return fail(CPM_ERANGE, "lambda out of range");
        lvmax = std::fmax(lvmax, std::fabs(lv));
        lsmax = std::fmax(lsmax, std::fabs(ls));
        vtmax = std::fmax(vtmax, std::fabs((double)p->volume_target[a]));
        if (p->lambda_surface) stmax = std::fmax(stmax, std::fabs((double)p->surface_target[a]));
        if (p->act_enabled) {
            if (p->max_act[a] < 0 || p->max_act[a] > 255) return fail(CPM_EINVAL, "max_act must be in 0..255");
            if (a == 0 && p->max_act[a] != 0) return fail(CPM_EINVAL, "the medium type cannot be motile");
            const double la = p->lambda_act[a];
            if (!std::isfinite(la) || std::fabs(la) >= lim) return fail(CPM_ERANGE, "lambda_act out of range");
            if (p->max_act[a] > 0) ramax = std::fmax(ramax, std::fabs(la / p->max_act[a]));
        }
    }
    // worst case |dH| in 2^-16 units must stay well inside int64
    const double N = (double)n_sites;
    // |V - Vt| <= N + |Vt|, |S - St| <= nnb N + |St|, |dS| <= nnb
    const double bound = 65536.0 * (2.0 * nnb * 2.0 * jmax + 2.0 * lvmax * (2.0 * (N + vtmax) + 1.0) +
                                    2.0 * lsmax * (2.0 * nnb * (nnb * N + stmax) + nnb * nnb) +
                                    2.0 * ramax * 256.0);
    if (bound >= 4.0e18) return fail(CPM_ERANGE, "fixed-point energy change could overflow int64");
    if (p->lambda_persistence) {
        if (!p->persistence_mu) return fail(CPM_EINVAL, "persistence_mu NULL with persistence enabled");
        if (p->persistence_dt < 1 || p->persistence_dt > 4096) return fail(CPM_EINVAL, "persistence_dt must be in 1..4096");
        if (p->persistence_centroids != 0 && p->persistence_centroids != 1)
            return fail(CPM_EINVAL, "persistence_centroids must be 0 (recount) or 1 (incremental)");
        for (int d = 0; d < p->ndim; ++d)
            if (p->dims[d] < 4 || p->dims[d] > 32768)
                return fail(CPM_EINVAL, "persistence needs every dim in 4..32768");
        double lpmax = 0;
        for (int a = 0; a < n; ++a) {
            const double lp = p->lambda_persistence[a], mu = p->persistence_mu[a];
            if (!std::isfinite(lp) || std::fabs(lp) >= lim) return fail(CPM_ERANGE, "lambda_persistence out of range");
            if (!(mu >= 0.0 && mu <= 1.0)) return fail(CPM_EINVAL, "persistence_mu must be in 0..1");
            lpmax = std::fmax(lpmax, std::fabs(lp));
        }
        // |U . P| <= 3 * 2^28: the term adds at most 3 * 2^16 * lambda
        if (bound + 65536.0 * 3.0 * lpmax >= 4.0e18) return fail(CPM_ERANGE, "fixed-point energy change could overflow int64");
    }
    if (p->lambda_chemotaxis) {
        if (!p->d_chemotaxis_field) return fail(CPM_EINVAL, "d_chemotaxis_field NULL with chemotaxis enabled");
        if (reinterpret_cast<uintptr_t>(p->d_chemotaxis_field) % 4 != 0)
            return fail(CPM_EINVAL, "d_chemotaxis_field must be 4-byte aligned");
        for (int d = 0; d < p->ndim; ++d)
            if (p->dims[d] < 4) return fail(CPM_EINVAL, "chemotaxis needs every dim >= 4");
        double lcmax = 0;
        for (int a = 0; a < n; ++a) {
            const double lc = p->lambda_chemotaxis[a];
            if (!std::isfinite(lc) || std::fabs(lc) >= lim) return fail(CPM_ERANGE, "lambda_chemotaxis out of range");
            lcmax = std::fmax(lcmax, std::fabs(lc));
        }
        // |U . C| < 3 * 2^14 * 2^15: the term adds at most 6 * 2^16 * lambda
        if (bound + 65536.0 * 6.0 * lcmax >= 4.0e18) return fail(CPM_ERANGE, "fixed-point energy change could overflow int64");
    }
    if (table_length(p->temperature) > cpm::kMaxTI) return fail(CPM_ENOTSUP, "temperature too high for the threshold table");
    return CPM_OK;
}

void build_model(const cpm_params *p, DeviceModel *m)
{
    std::memset(m, 0, sizeof(*m));
    const int n = p->n_types;
    for (int a = 0; a < n; ++a) {
        for (int b = 0; b < n; ++b) m->J[a * cpm::kMaxTypes + b] = to_fixed(p->J[a * n + b]);
        m->lam_v[a] = to_fixed(p->lambda_volume[a]);
        m->v_target[a] = p->volume_target[a];
        m->lam_s[a] = p->lambda_surface ? to_fixed(p->lambda_surface[a]) : 0;
        m->s_target[a] = p->lambda_surface ? p->surface_target[a] : 0;
        if (p->act_enabled && p->max_act[a] > 0) {
            m->max_act[a] = p->max_act[a];
            m->r_act[a] = to_fixed(p->lambda_act[a] / (double)p->max_act[a]);
        }
        if (p->lambda_chemotaxis) m->lam_c[a] = to_fixed(p->lambda_chemotaxis[a]);
        if (p->lambda_persistence) {
            m->lam_p[a] = to_fixed(p->lambda_persistence[a]);
            m->mu_p[a] = (int64_t)std::llround(p->persistence_mu[a] * 16384.0);
        }
    }
    // unit vectors of the Moore offsets, 2^-14 (eq. 5)
    for (int i = 0; i < 27; ++i) {
        const int o[3] = {i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1};
        const double len = std::sqrt((double)(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]));
        for (int d = 0; d < 3; ++d) m->unit[i][d] = len > 0 ? (int32_t)std::llround(o[d] / len * 16384.0) : 0;
    }
    // Acceptance: TI[h] = floor(2^32 e^{-h/T}) while nonzero, TM, TL finer steps.
    const double T = p->temperature;
    const double two32 = 4294967296.0;
    m->n_ti = table_length(T);
    for (int h = 0; h < m->n_ti; ++h) m->TI[h] = (uint64_t)std::floor(std::exp(-(double)h / T) * two32);
    for (int i = 0; i < 256; ++i) {
        m->TM[i] = (uint64_t)std::floor(std::exp(-(double)i / (256.0 * T)) * two32);
        m->TL[i] = (uint64_t)std::floor(std::exp(-(double)i / (65536.0 * T)) * two32);
    }
    for (int h = 1; h < m->n_ti; ++h) m->TI32[h] = (uint32_t)m->TI[h];
    for (int i = 1; i < 256; ++i) {
        m->TM32[i] = (uint32_t)m->TM[i];
        m->TL32[i] = (uint32_t)m->TL[i];
    }
    // Activity geometric mean tables.
    for (int a = 1; a < 256; ++a) m->LG[a] = (int64_t)std::llround(std::log((double)a) * 16777216.0);
    for (int i = 0; i < 2048; ++i) m->EH[i] = (uint64_t)std::floor(std::exp((double)i / 256.0) * 16777216.0);
    for (int i = 0; i < 256; ++i) {
        m->EM[i] = (uint64_t)std::floor(std::exp((double)i / 65536.0) * 2147483648.0);
        m->EL[i] = (uint64_t)std::floor(std::exp((double)i / 16777216.0) * 1073741824.0);
    }
}

// Cell types read back from the device: entry 0 is the medium's type 0, every
// cell's type is valid; *single gets the type all cells share, or -1.
int check_types(const cpm_params *p, const int32_t *types, int32_t n_cells, int32_t *single)
{
    if (types[0] != 0) return fail(CPM_EINVAL, "cell_type[0] must be 0 (the medium's type)");
    int32_t one = n_cells >= 1 ? types[1] : 0;
    for (int32_t c = 1; c <= n_cells; ++c) {
        if (types[c] < 0 || types[c] >= p->n_types) return fail(CPM_EINVAL, "cell type out of range");
        if (types[c] != one) one = -1;
    }
    *single = one;
    return CPM_OK;
}

// The kernel arguments of one lattice whose workspace sections start at ws.
void fill_args(SweepArgs &a, const cpm_params *p, const Layout &lay, char *ws, int32_t *d_lattice,
               const int32_t *d_cell_type, uint8_t *d_act, int32_t single)
{
    a = SweepArgs{};
    a.lat = d_lattice;
    a.cells = lay.mirror_on ? static_cast<void *>(ws + lay.mirror) : static_cast<void *>(d_lattice);
    a.cell_type = d_cell_type;
    a.act = p->act_enabled ? d_act : nullptr;
    a.chem = p->lambda_chemotaxis ? p->d_chemotaxis_field : nullptr;
    a.model = reinterpret_cast<const DeviceModel *>(ws + lay.model);
    a.counters[0] = reinterpret_cast<int32_t *>(ws + lay.counters0);
    a.counters[1] = reinterpret_cast<int32_t *>(ws + lay.counters1);
    a.dlist[0] = reinterpret_cast<int4 *>(ws + lay.dlist);
    a.dlist[1] = a.dlist[0] + (size_t)lay.tg.n_tiles * (size_t)lay.dlist_cap;
    a.dcount[0] = reinterpret_cast<int32_t *>(ws + lay.dcount);
    a.dcount[1] = a.dcount[0] + lay.tg.n_tiles;
    a.stats = reinterpret_cast<uint64_t *>(ws + lay.stats);
    a.own_spill = p->attempts > cpm::kOwnInRegs ? reinterpret_cast<int4 *>(ws + lay.own) : nullptr;
    uint32_t n_areas = 1;
    for (int d = 0; d < 3; ++d) {
        a.L[d] = p->dims[d];
        a.na[d] = d < p->ndim ? p->dims[d] / (2 * p->sub) : 1;
        n_areas *= (uint32_t)a.na[d];
    }
    a.n_areas = n_areas;
    a.s = p->sub;
    a.k = p->attempts;
    a.dlist_cap = lay.dlist_cap;
    a.obstacle_type = p->obstacle_type < 0 ? 0 : p->obstacle_type;
    a.single_type = single;
    a.n_types = p->n_types;
    a.lg_entries = 256;
    a.key0 = (uint32_t)p->seed;
    a.key1 = (uint32_t)(p->seed >> 32);
    a.lattice_id = p->lattice_id;
    a.tg = lay.tg;
    a.tg.row_chunk = chunk_for(a.cells, (size_t)p->dims[0] * (lay.mirror_on ? 2 : 4));
    a.tg.act_chunk = p->act_enabled ? chunk_for(d_act, (size_t)p->dims[0]) : 4;
}

// Uploads the model, clears the bookkeeping and counts V, S from the lattice.
hipError_t start_lattice(const SweepArgs &a, const Layout &lay, char *ws, const DeviceModel *host_model, int ndim,
                         int32_t n_cells, hipStream_t st)
{
    hipError_t e = hipMemcpyAsync(ws + lay.model, host_model, sizeof(DeviceModel), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    const size_t pairs = 2 * ((size_t)n_cells + 1);
    if ((e = cpm::launch_fill_i32(a.counters[0], 0, pairs, st)) != hipSuccess) return e;
    if ((e = cpm::launch_fill_i32(a.dcount[0], 0, 2 * (size_t)lay.tg.n_tiles, st)) != hipSuccess) return e;
    if ((e = cpm::launch_fill_i32(reinterpret_cast<int32_t *>(a.stats), 0, 4 * (size_t)lay.tg.n_tiles, st)) != hipSuccess)
        return e;
    if ((e = cpm::launch_count(a, ndim, a.counters[0], a.counters[0] + 1, 2, st)) != hipSuccess) return e;
    return hipMemcpyAsync(a.counters[1], a.counters[0], sizeof(int32_t) * pairs, hipMemcpyDeviceToDevice, st);
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// The workspace of cpm_init_static: a device array of the library's own, one
// copy per GPU, held by at most one handle per GPU at a time.  Host code
// never passes `scratch` itself to the device (in host code the name stands
// for a host-side shadow, not a device address): it takes each device's
// address once, with hipGetSymbolAddress, and passes that.
constexpr size_t kStaticScratchBytes = CPM_STATIC_WORKSPACE_BYTES;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_busy[kMaxDevices] = {};

// The current device's static workspace, claimed for one handle.
int claim_static_scratch(void **ptr, int *device)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(CPM_ENOTSUP, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_busy[dev])
        return fail(CPM_EINVAL, "the static workspace of this device is held by another handle (cpm_destroy it first)");
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return device_fail(e, "static workspace address");
        if (!p) return fail(CPM_EDEVICE, "static workspace address is NULL");
        g_scratch_ptr[dev] = p;
    }
    g_scratch_busy[dev] = true;
    *ptr = g_scratch_ptr[dev];
    *device = dev;
    return CPM_OK;
}

void release_static_scratch(int dev)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (dev >= 0 && dev < kMaxDevices) g_scratch_busy[dev] = false;
}

int init_impl(const cpm_params *params, int32_t *d_lattice, const int32_t *d_cell_type, int32_t n_cells,
              uint8_t *d_act, void *d_workspace, size_t workspace_bytes, void *stream, cpm_handle **out);

// Number of sites of an int32 lattice labelled outside [-1, n_cells] (or -1
// without an obstacle type), counted on the device into *flag and read back
// (waits for the stream).
hipError_t count_bad_labels(const int32_t *lat, size_t n_sites, int32_t n_cells, bool obstacles, int32_t *flag,
                            hipStream_t st, int32_t *bad)
{
    hipError_t e = cpm::launch_fill_i32(flag, 0, 1, st);
    if (e == hipSuccess) e = cpm::launch_bad_labels(lat, n_sites, n_cells, obstacles, flag, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

// Persistence directions after update t, one thread per cell, from the
// centroid sums: recounted from the lattice (sites unwrapped around each
// cell's lowest-index site) at every update, or, with incremental
// centroids, only at t = 0 (initialisation), the sweeps keeping them after
// that (each accepted copy moves its site between the two cells' sums).
hipError_t persist_step(cpm_handle *h, int64_t t, int words, hipStream_t st)
{
    if (t == 0 || !h->incremental) {
        const hipError_t e = cpm::launch_centroids(h->args, h->ndim, h->n_cells, h->ref, h->csum, st, words);
        if (e != hipSuccess) return e;
    }
    cpm::PersistArgs p{};
    p.pdir = h->pdir;
    p.hist = h->hist;
    p.cpos = h->cpos;
    p.csum = h->csum;
    p.pairs = h->args.counters[h->activation & 1];
    p.cell_type = h->args.cell_type;
    p.model = h->args.model;
    p.n_labels = h->n_cells + 1;
    p.ndim = h->ndim;
    p.slots = h->persist_slots;
    for (int d = 0; d < 3; ++d) p.L[d] = h->L[d];
    return cpm::launch_persist(p, t, st);
}

}  // namespace

extern "C" {

int cpm_validate(const cpm_params *params, int32_t n_cells) { return validate(params, n_cells); }

int cpm_workspace_bytes(const cpm_params *params, int32_t n_cells, size_t *bytes)
{
    const int rc = validate(params, n_cells);
    if (rc != CPM_OK) return rc;
    if (!bytes) return fail(CPM_EINVAL, "bytes is NULL");
    *bytes = layout_of(params, n_cells).total;
    return CPM_OK;
}

int cpm_tile_shape(const cpm_params *params, int32_t n_cells, int32_t *out)
{
    const int rc = validate(params, n_cells);
    if (rc != CPM_OK) return rc;
    if (!out) return fail(CPM_EINVAL, "out is NULL");
    const Layout l = layout_of(params, n_cells);
    for (int d = 0; d < 3; ++d) out[d] = l.tg.T[d];
    out[3] = l.tg.layout;
    out[4] = l.tg.lds_bytes;
    out[5] = l.tg.n_tiles;
    out[6] = l.mirror_on ? 1 : 0;
    return CPM_OK;
}

int cpm_init(const cpm_params *params, int32_t *d_lattice, const int32_t *d_cell_type, int32_t n_cells,
             uint8_t *d_act, void *d_workspace, size_t workspace_bytes, void *stream, cpm_handle **out)
{
    return init_impl(params, d_lattice, d_cell_type, n_cells, d_act, d_workspace, workspace_bytes, stream, out);
}

int cpm_init_static(const cpm_params *params, int32_t *d_lattice, const int32_t *d_cell_type, int32_t n_cells,
                    uint8_t *d_act, void *stream, cpm_handle **out)
{
    if (!out) return fail(CPM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(params, n_cells);
    if (rc != CPM_OK) return rc;
    const size_t need = layout_of(params, n_cells).total;
    if (need > kStaticScratchBytes)
        return fail(CPM_ENOMEM, "this model needs " + std::to_string(need) + " bytes of workspace; the static one holds " +
                                    std::to_string(kStaticScratchBytes) + " (use cpm_init with a caller workspace)");
    void *ws = nullptr;
    int dev = -1;
    if ((rc = claim_static_scratch(&ws, &dev)) != CPM_OK) return rc;
    rc = init_impl(params, d_lattice, d_cell_type, n_cells, d_act, ws, kStaticScratchBytes, stream, out);
    if (rc != CPM_OK) {
        release_static_scratch(dev);
        return rc;
    }
    (*out)->static_device = dev;
    return CPM_OK;
}

}  // extern "C"

namespace {

int init_impl(const cpm_params *params, int32_t *d_lattice, const int32_t *d_cell_type, int32_t n_cells,
              uint8_t *d_act, void *d_workspace, size_t workspace_bytes, void *stream, cpm_handle **out)
{
    if (!out) return fail(CPM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(params, n_cells);
    if (rc != CPM_OK) return rc;
    if (!d_lattice || !d_cell_type || !d_workspace) return fail(CPM_EINVAL, "NULL device buffer");
    if (params->act_enabled && !d_act) return fail(CPM_EINVAL, "act enabled but d_act is NULL");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) return fail(CPM_EINVAL, "workspace not 256-byte aligned");
    const Layout lay = layout_of(params, n_cells);
    if (workspace_bytes < lay.total) return fail(CPM_ENOMEM, "workspace smaller than cpm_workspace_bytes()");

    std::unique_ptr<cpm_handle> h(new (std::nothrow) cpm_handle());
    if (!h) return fail(CPM_EINVAL, "host allocation failed");
    h->host_model.reset(new (std::nothrow) DeviceModel);
    if (!h->host_model) return fail(CPM_EINVAL, "host allocation failed");
    build_model(params, h->host_model.get());

    std::vector<int32_t> types((size_t)n_cells + 1);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(types.data(), d_cell_type, sizeof(int32_t) * types.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_fail(e, "read cell types");
    int32_t single = -1;
    if ((rc = check_types(params, types.data(), n_cells, &single)) != CPM_OK) return rc;

    char *ws = static_cast<char *>(d_workspace);
    const size_t n_sites = (size_t)params->dims[0] * params->dims[1] * params->dims[2];
    int32_t n_bad = 0;
    if ((e = count_bad_labels(d_lattice, n_sites, n_cells, params->obstacle_type >= 0,
                              reinterpret_cast<int32_t *>(ws + lay.check), st, &n_bad)) != hipSuccess)
        return device_fail(e, "check labels");
    if (n_bad) return fail(CPM_EINVAL, "lattice labels must lie in [-1, n_cells], -1 only with an obstacle type");
    h->ndim = params->ndim;
    for (int d = 0; d < 3; ++d) h->L[d] = params->dims[d];
    h->s = params->sub;
    h->k = params->attempts;
    h->n_cells = n_cells;
    h->n_types = params->n_types;
    h->act = params->act_enabled != 0;
    h->mirror = lay.mirror_on;
    h->mirror_cells = lay.mirror_on ? reinterpret_cast<uint16_t *>(ws + lay.mirror) : nullptr;
    h->ref = reinterpret_cast<int32_t *>(ws + lay.ref);
    h->check = reinterpret_cast<int32_t *>(ws + lay.check);
    h->obstacles = params->obstacle_type >= 0;
    fill_args(h->args, params, lay, ws, d_lattice, d_cell_type, d_act, single);
    if (params->lambda_persistence) {
        h->pdir = reinterpret_cast<int4 *>(ws + lay.pdir);
        h->hist = reinterpret_cast<int64_t *>(ws + lay.hist);
        h->csum = reinterpret_cast<int64_t *>(ws + lay.csum);
        h->cpos = reinterpret_cast<int4 *>(ws + lay.cpos);
        h->persist_slots = params->persistence_dt + 1;
        h->incremental = params->persistence_centroids == 1;
        h->args.pdir = h->pdir;
        if (h->incremental) {
            h->args.csum = h->csum;
            h->args.cpos = h->cpos;
        }
    }
    if ((e = start_lattice(h->args, lay, ws, h->host_model.get(), params->ndim, n_cells, st)) != hipSuccess)
        return device_fail(e, "init");
    if (h->pdir && (e = persist_step(h.get(), 0, cpm::kWords32, st)) != hipSuccess)
        return device_fail(e, "persistence init");
    // multi-type lattices too large for the 16-bit copy sweep on packed
    // words (label and type in one word) written over the int32 lattice
    // (with the Act term and up to 2^20 - 2 cells the word holds the activity too)
    h->words = h->mirror ? cpm::kWords16
               : use_act_words(params, n_cells) ? cpm::kWordsPackedAct
               : single >= 0 ? cpm::kWords32
               : n_cells <= kMaxPackedCells ? cpm::kWordsPacked : cpm::kWords32;
    *out = h.release();
    return CPM_OK;
}

}  // namespace

namespace {

// n_mcs MCS of a single lattice.
int sweep_impl(cpm_handle *h, int32_t n_mcs, hipStream_t st)
{
    int64_t sd = 1;
    for (int d = 0; d < h->ndim; ++d) sd *= h->s;
    const uint32_t n_act = (uint32_t)(((int64_t)1 << h->ndim) * sd / h->k);
    const size_t n_sites = (size_t)h->L[0] * h->L[1] * h->L[2];
    hipError_t e;
    if (h->words == cpm::kWordsPacked &&
        (e = cpm::launch_pack(h->args.lat, h->args.cell_type, h->args.obstacle_type, n_sites, st)) != hipSuccess)
        return device_fail(e, "pack label and type words");
    if (h->words == cpm::kWordsPackedAct &&
        (e = cpm::launch_pack_act(h->args.lat, h->args.act, h->args.cell_type, h->args.obstacle_type, n_sites, st)) !=
            hipSuccess)
        return device_fail(e, "pack label, type and activity words");
    if (h->mirror && (e = cpm::launch_to_mirror(h->args.lat, h->mirror_cells, n_sites, st)) != hipSuccess)
        return device_fail(e, "to 16-bit working copy");
    for (int32_t i = 0; i < n_mcs; ++i) {
        const uint32_t mcs = (uint32_t)h->mcs;
        for (uint32_t alpha = 0; alpha < n_act; ++alpha) {
            e = cpm::launch_activation(h->args, h->ndim, h->act, h->words, mcs, alpha, (int)(h->activation & 1), st);
            if (e != hipSuccess) return device_fail(e, "activation");
            ++h->activation;
        }
        if (h->act)
            e = h->words == cpm::kWordsPackedAct ? cpm::launch_act_decay_words(h->args.lat, n_sites, st)
                                                 : cpm::launch_act_decay(h->args.act, n_sites, st);
        if (h->act && e != hipSuccess) return device_fail(e, "act decay");
        if (h->pdir && (e = persist_step(h, ++h->persist_t, h->words, st)) != hipSuccess)
            return device_fail(e, "persistence update");
        ++h->mcs;
        h->attempts_run += (uint64_t)n_sites;
    }
    if (h->mirror && (e = cpm::launch_from_mirror(h->mirror_cells, h->args.lat, n_sites, st)) != hipSuccess)
        return device_fail(e, "from 16-bit working copy");
    if (h->words == cpm::kWordsPacked && (e = cpm::launch_unpack(h->args.lat, n_sites, st)) != hipSuccess)
        return device_fail(e, "unpack labels");
    if (h->words == cpm::kWordsPackedAct &&
        (e = cpm::launch_unpack_act(h->args.lat, h->args.act, n_sites, st)) != hipSuccess)
        return device_fail(e, "unpack labels and activity");
    return CPM_OK;
}

}  // namespace

extern "C" {

int cpm_sweep(cpm_handle *h, int32_t n_mcs, void *stream)
{
    if (!h) return fail(CPM_EINVAL, "handle is NULL");
    if (n_mcs < 0) return fail(CPM_EINVAL, "n_mcs must be >= 0");
    if (n_mcs == 0) return CPM_OK;
    return sweep_impl(h, n_mcs, as_stream(stream));
}

int cpm_attempt_stats(cpm_handle *h, uint64_t *out, void *stream)
{
    if (!h || !out) return fail(CPM_EINVAL, "NULL argument");
    hipStream_t st = as_stream(stream);
    const int n = h->args.tg.n_tiles;
    std::vector<uint64_t> per(2 * (size_t)n);
    hipError_t e = hipMemcpyAsync(per.data(), h->args.stats, sizeof(uint64_t) * per.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_fail(e, "read stats");
    out[0] = h->attempts_run;
    out[1] = 0;
    out[2] = 0;
    for (int i = 0; i < n; ++i) {
        out[1] += per[2 * (size_t)i];
        out[2] += per[2 * (size_t)i + 1];
    }
    return CPM_OK;
}

int cpm_cell_stats(cpm_handle *h, int32_t *d_volume, int32_t *d_surface, int64_t *d_centroid_sum, void *stream)
{
    if (!h || !d_volume || !d_surface) return fail(CPM_EINVAL, "NULL argument");
    hipStream_t st = as_stream(stream);
    const size_t n = (size_t)h->n_cells + 1;
    hipError_t e;
    if ((e = cpm::launch_fill_i32(d_volume, 0, n, st)) != hipSuccess) return device_fail(e, "clear volume");
    if ((e = cpm::launch_fill_i32(d_surface, 0, n, st)) != hipSuccess) return device_fail(e, "clear surface");
    if ((e = cpm::launch_count(h->args, h->ndim, d_volume, d_surface, 1, st)) != hipSuccess)
        return device_fail(e, "count");
    if (d_centroid_sum) {
        if ((e = cpm::launch_centroids(h->args, h->ndim, h->n_cells, h->ref, d_centroid_sum, st)) != hipSuccess)
            return device_fail(e, "centroids");
    }
    return CPM_OK;
}

int cpm_contacts(cpm_handle *h, int64_t *d_out, void *stream)
{
    if (!h || !d_out) return fail(CPM_EINVAL, "NULL argument");
    const hipError_t e = cpm::launch_contacts(h->args, h->ndim, h->n_types, d_out, as_stream(stream));
    return e == hipSuccess ? CPM_OK : device_fail(e, "contacts");
}

int cpm_persistence(cpm_handle *h, int32_t *d_dir, void *stream)
{
    if (!h || !d_dir) return fail(CPM_EINVAL, "NULL argument");
    if (!h->pdir) return fail(CPM_EINVAL, "persistence is off for this lattice");
    const hipError_t e = cpm::launch_copy_dirs(h->pdir, h->n_cells + 1, d_dir, as_stream(stream));
    return e == hipSuccess ? CPM_OK : device_fail(e, "copy directions");
}

int cpm_counters(cpm_handle *h, int32_t *d_volume, int32_t *d_surface, void *stream)
{
    if (!h || !d_volume || !d_surface) return fail(CPM_EINVAL, "NULL argument");
    const hipError_t e = cpm::launch_copy_counters(h->args.counters[h->activation & 1], h->n_cells + 1, d_volume,
                                                   d_surface, as_stream(stream));
    if (e != hipSuccess) return device_fail(e, "copy counters");
    return CPM_OK;
}

int cpm_check_invariants(cpm_handle *h, void *stream, int32_t *h_ok)
{
    if (!h || !h_ok) return fail(CPM_EINVAL, "NULL argument");
    *h_ok = 0;
    hipStream_t st = as_stream(stream);
    const size_t n_sites = (size_t)h->L[0] * h->L[1] * h->L[2];
    const size_t labels = (size_t)h->n_cells + 1;
    int32_t *flag = h->check, *rv = h->check + kCheckPad, *rs = rv + labels;
    int32_t bad = 0;
    // labels first: the recount indexes its outputs by label
    hipError_t e = count_bad_labels(h->args.lat, n_sites, h->n_cells, h->obstacles, flag, st, &bad);
    if (e != hipSuccess) return device_fail(e, "check labels");
    if (bad) return CPM_OK;
    if ((e = cpm::launch_fill_i32(rv, 0, 2 * labels, st)) == hipSuccess &&
        (e = cpm::launch_count(h->args, h->ndim, rv, rs, 1, st)) == hipSuccess &&
        (e = cpm::launch_fill_i32(flag, 0, 1, st)) == hipSuccess &&
        (e = cpm::launch_compare_counters(h->args.counters[h->activation & 1], rv, rs, (int32_t)labels, flag, st)) ==
            hipSuccess &&
        (e = hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st)) == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_fail(e, "check counters");
    *h_ok = bad == 0 ? 1 : 0;
    return CPM_OK;
}

int cpm_set_mcs(cpm_handle *h, uint64_t mcs)
{
    if (!h) return fail(CPM_EINVAL, "handle is NULL");
    h->mcs = mcs;
    return CPM_OK;
}

int cpm_get_mcs(const cpm_handle *h, uint64_t *mcs)
{
    if (!h || !mcs) return fail(CPM_EINVAL, "NULL argument");
    *mcs = h->mcs;
    return CPM_OK;
}

int cpm_destroy(cpm_handle *h)
{
    if (h && h->static_device >= 0) release_static_scratch(h->static_device);
    delete h;
    return CPM_OK;
}

const char *cpm_strerror(int code)
{
    switch (code) {
    case CPM_OK: return "ok";
    case CPM_EINVAL: return "invalid argument";
    case CPM_ERANGE: return "fixed-point range exceeded";
    case CPM_ENOMEM: return "workspace too small";
    case CPM_EDEVICE: return "HIP runtime error";
    case CPM_ENOTSUP: return "not supported by the library";
    default: return "unknown error";
    }
}

const char *cpm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ------------------------------------------------------------------ batches

namespace {

struct BatchLayout {
    std::vector<Layout> lat;
    std::vector<size_t> base;  // workspace offset of each lattice's sections
    size_t args, work, mcs, barrier, label_off, dims, scratch_v, scratch_s, scratch_c, scratch_ref, total;
    size_t total_labels;
    int grid;
    bool mirror, feasible;
    bool act_words;
    bool act16_ok;             // every lattice fits 16-bit label-activity words
    size_t words16;            // their region: one uint16 per site of the batch
    int layout;
};


int validate_batch(const cpm_params *p, int32_t n, const int32_t *n_cells)
{
    if (!p || !n_cells || n < 1) return fail(CPM_EINVAL, "empty batch");
    for (int32_t i = 0; i < n; ++i) {
        const int rc = validate(&p[i], n_cells[i]);
        if (rc != CPM_OK) return rc;
        if (p[i].lambda_persistence) return fail(CPM_ENOTSUP, "persistence is not available in batches");
        if (p[i].ndim != p[0].ndim || p[i].sub != p[0].sub || p[i].attempts != p[0].attempts ||
            (p[i].act_enabled != 0) != (p[0].act_enabled != 0) || p[i].layout != p[0].layout)
            return fail(CPM_EINVAL, "lattices of a batch must share ndim, sub, attempts, act_enabled and layout");
    }
    return CPM_OK;
}

BatchLayout batch_layout_of(const cpm_params *p, int32_t n, const int32_t *n_cells)
{
    BatchLayout b{};
    // Act batches of up to 2^20 - 2 cells per lattice sweep on label, type
    // and activity words written over their int32 lattices; others on the
    // 16-bit copy when every lattice fits it
    b.act_words = true;
    for (int32_t i = 0; i < n; ++i) b.act_words = b.act_words && use_act_words(&p[i], n_cells[i]);
    b.mirror = !b.act_words;
    // Act batches of small lattices (at most 2,046 cells, Max_act <= 31, no
    // chemotaxis) sweep on 16-bit label-activity words when their cells are
    // of one type (known at init), halving the bytes per site
    b.act16_ok = b.act_words;
    for (int32_t i = 0; i < n && b.act16_ok; ++i) {
        b.act16_ok = n_cells[i] <= cpm::kMaxAct16Cells && p[i].lambda_chemotaxis == nullptr;
        for (int t = 0; t < p[i].n_types && b.act16_ok; ++t) b.act16_ok = p[i].max_act[t] <= cpm::kMaxAct16Activity;
    }
    for (int32_t i = 0; i < n; ++i) b.mirror = b.mirror && use_mirror(n_cells[i]);
    // one kernel variant for the whole batch: the layout every lattice
    // chooses, else halo boxes (valid for all)
    b.feasible = true;
    for (int32_t i = 0; i < n; ++i) b.lat.push_back(layout_of(&p[i], n_cells[i], b.mirror ? 1 : 0));
    b.layout = b.lat[0].tg.layout;
    for (int32_t i = 1; i < n; ++i)
        if (b.lat[i].tg.layout != b.layout) b.layout = 0;
    if (b.layout == 0)
        for (int32_t i = 0; i < n; ++i) b.lat[i] = layout_of(&p[i], n_cells[i], b.mirror ? 1 : 0, 0);
    for (int32_t i = 0; i < n; ++i) {
        cpm::TileGeometry g;
        b.feasible = b.feasible && tile_geometry(&p[i], b.mirror, b.layout, g, b.act_words);
    }
    // workgroups: every (lattice, tile) pair, padded to a multiple of the XCD count
    b.grid = 0;
    for (const Layout &l : b.lat) b.grid += l.tg.n_tiles;
    b.grid = (b.grid + cpm::kXcds - 1) / cpm::kXcds * cpm::kXcds;
    size_t off = 0;
    b.args = off;
    off = align_up(off + sizeof(SweepArgs) * (size_t)n);
    b.work = off;
    off = align_up(off + sizeof(int2) * (size_t)b.grid);
    b.mcs = off;
    off = align_up(off + sizeof(uint32_t));
    b.barrier = off;
    off = align_up(off + sizeof(cpm::GridBarrier));
    b.total_labels = 0;
    for (int32_t i = 0; i < n; ++i) b.total_labels += (size_t)n_cells[i] + 1;
    b.label_off = off;
    off = align_up(off + sizeof(int64_t) * ((size_t)n + 1));
    b.dims = off;
    off = align_up(off + sizeof(int32_t) * 3 * (size_t)n);
    b.scratch_v = off;
    off = align_up(off + sizeof(int32_t) * b.total_labels);
    b.scratch_s = off;
    off = align_up(off + sizeof(int32_t) * b.total_labels);
    b.scratch_c = off;
    off = align_up(off + sizeof(int64_t) * 3 * b.total_labels);
    b.scratch_ref = off;
    off = align_up(off + sizeof(int32_t) * b.total_labels);
    size_t total_sites = 0;
    for (int32_t i = 0; i < n; ++i) total_sites += (size_t)p[i].dims[0] * p[i].dims[1] * p[i].dims[2];
    b.words16 = off;
    off = align_up(off + (b.act16_ok ? sizeof(uint16_t) * total_sites : 0));
    for (const Layout &l : b.lat) {
        b.base.push_back(off);
        off = align_up(off + l.total);
    }
    b.total = off;
    return b;
}

}  // namespace

extern "C" {

int cpm_batch_workspace_bytes(const cpm_params *params, int32_t n, const int32_t *n_cells, size_t *bytes)
{
    const int rc = validate_batch(params, n, n_cells);
    if (rc != CPM_OK) return rc;
    if (!bytes) return fail(CPM_EINVAL, "bytes is NULL");
    const BatchLayout bl = batch_layout_of(params, n, n_cells);
    if (!bl.feasible) return fail(CPM_ENOTSUP, "the requested layout / tile does not fit every lattice of the batch");
    *bytes = bl.total;
    return CPM_OK;
}

int cpm_batch_init(const cpm_params *params, int32_t n, const int32_t *n_cells, int32_t *d_lattices,
                   const int32_t *d_cell_types, uint8_t *d_act, void *d_workspace, size_t workspace_bytes,
                   void *stream, cpm_batch **out)
{
    if (!out) return fail(CPM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_batch(params, n, n_cells);
    if (rc != CPM_OK) return rc;
    if (!d_lattices || !d_cell_types || !d_workspace) return fail(CPM_EINVAL, "NULL device buffer");
    if (params[0].act_enabled && !d_act) return fail(CPM_EINVAL, "act enabled but d_act is NULL");
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) return fail(CPM_EINVAL, "workspace not 256-byte aligned");
    const BatchLayout bl = batch_layout_of(params, n, n_cells);
    if (!bl.feasible) return fail(CPM_ENOTSUP, "the requested layout / tile does not fit every lattice of the batch");
    if (workspace_bytes < bl.total) return fail(CPM_ENOMEM, "workspace smaller than cpm_batch_workspace_bytes()");

    std::unique_ptr<cpm_batch> b(new (std::nothrow) cpm_batch());
    if (!b) return fail(CPM_EINVAL, "host allocation failed");
    b->n = n;
    b->ndim = params[0].ndim;
    b->s = params[0].sub;
    b->k = params[0].attempts;
    b->act = params[0].act_enabled != 0;
    b->mirror = bl.mirror;
    b->act_words = bl.act_words;
    b->layout = bl.layout;
    b->lattices = d_lattices;
    b->act_field = d_act;
    size_t sites = 0, labels = 0;
    for (int32_t i = 0; i < n; ++i) {
        b->site_off.push_back(sites);
        b->label_off.push_back(labels);
        sites += (size_t)params[i].dims[0] * params[i].dims[1] * params[i].dims[2];
        labels += (size_t)n_cells[i] + 1;
        b->n_cells.push_back(n_cells[i]);
    }
    b->total_sites = sites;
    for (int32_t i = 0; i < n; ++i) {
        b->max_sites = std::max(b->max_sites, (size_t)params[i].dims[0] * params[i].dims[1] * params[i].dims[2]);
        b->max_bricks = std::max(b->max_bricks, cpm::reduce_brick_count(params[i].dims, params[i].ndim));
    }

    std::vector<int32_t> types(labels);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(types.data(), d_cell_types, sizeof(int32_t) * labels, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_fail(e, "read cell types");

    char *ws = static_cast<char *>(d_workspace);
    // every label in range before the first recount indexes counters by it
    {
        int32_t *flag = reinterpret_cast<int32_t *>(ws + bl.base[0] + bl.lat[0].check);
        int32_t n_bad = 0;
        e = cpm::launch_fill_i32(flag, 0, 1, st);
        for (int32_t i = 0; i < n && e == hipSuccess; ++i)
            e = cpm::launch_bad_labels(d_lattices + b->site_off[i],
                                       (size_t)params[i].dims[0] * params[i].dims[1] * params[i].dims[2], n_cells[i],
                                       params[i].obstacle_type >= 0, flag, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&n_bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return device_fail(e, "check labels");
        if (n_bad)
            return fail(CPM_EINVAL, "lattice labels must lie in [-1, n_cells], -1 only with an obstacle type");
    }
    b->single = true;
    size_t lds = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t single = -1;
        if ((rc = check_types(&params[i], types.data() + b->label_off[i], n_cells[i], &single)) != CPM_OK) return rc;
        b->single = b->single && single >= 0;
        char *lws = ws + bl.base[i];
        const Layout &lay = bl.lat[i];
        SweepArgs a;
        fill_args(a, &params[i], lay, lws, d_lattices + b->site_off[i], d_cell_types + b->label_off[i],
                  b->act ? d_act + b->site_off[i] : nullptr, single);
        b->args.push_back(a);
        b->ref.push_back(reinterpret_cast<int32_t *>(lws + lay.ref));
        b->check.push_back(reinterpret_cast<int32_t *>(lws + lay.check));
        b->obstacles.push_back(params[i].obstacle_type >= 0 ? 1 : 0);
        b->mirror_cells.push_back(lay.mirror_on ? reinterpret_cast<uint16_t *>(lws + lay.mirror) : nullptr);
        b->models.emplace_back(new (std::nothrow) DeviceModel);
        if (!b->models.back()) return fail(CPM_EINVAL, "host allocation failed");
        build_model(&params[i], b->models.back().get());
        for (int32_t t = 0; t < lay.tg.n_tiles; ++t) b->work.push_back(make_int2(i, t));
        lds = std::max(lds, (size_t)lay.tg.lds_bytes);
        if ((e = start_lattice(a, lay, lws, b->models.back().get(), b->ndim, n_cells[i], st)) != hipSuccess)
            return device_fail(e, "init");
    }
    b->d_args = reinterpret_cast<SweepArgs *>(ws + bl.args);
    b->d_work = reinterpret_cast<int2 *>(ws + bl.work);
    b->d_mcs = reinterpret_cast<uint32_t *>(ws + bl.mcs);
    b->bar = reinterpret_cast<cpm::GridBarrier *>(ws + bl.barrier);
    if ((e = cpm::launch_fill_i32(reinterpret_cast<int32_t *>(b->bar), 0, 4, st)) != hipSuccess)
        return device_fail(e, "clear barrier");
    // one cell type throughout, small lattices and every activity within 5
    // bits: 16-bit label-activity words
    b->act16 = bl.act16_ok && b->single;
    if (b->act16) {
        int32_t *flag = reinterpret_cast<int32_t *>(ws + bl.base[0] + bl.lat[0].check);
        int32_t over = 0;
        if ((e = cpm::launch_fill_i32(flag, 0, 1, st)) == hipSuccess &&
            (e = cpm::launch_count_above(d_act, sites, cpm::kMaxAct16Activity, flag, st)) == hipSuccess &&
            (e = hipMemcpyAsync(&over, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st)) == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess) return device_fail(e, "check activities");
        b->act16 = over == 0;
    }
    if (b->act16) {
        b->words16 = reinterpret_cast<uint16_t *>(ws + bl.words16);
        b->act_words = false;
        for (int32_t i = 0; i < n; ++i) {
            SweepArgs &a = b->args[i];
            a.cells = b->words16 + b->site_off[i];
            a.tg.row_chunk = chunk_for(a.cells, (size_t)a.L[0] * sizeof(uint16_t));
            a.lg_entries = cpm::kMaxAct16Activity + 1;  // the words hold activities 0..31
        }
    }
    // Workgroups go to the XCDs round-robin: workgroup g takes entry
    // (g mod 8) * (grid / 8) + g div 8 of the (lattice, tile) list, so each
    // XCD sweeps one contiguous run of it and neighbouring tiles of a
    // lattice, whose halos overlap, share that XCD's L2.  Padding entries
    // are (-1, -1).
    {
        const size_t grid = (size_t)bl.grid, per = grid / cpm::kXcds;
        std::vector<int2> order(grid, make_int2(-1, -1));
        for (size_t g = 0; g < grid; ++g) {
            const size_t src = (g % cpm::kXcds) * per + g / cpm::kXcds;
            if (src < b->work.size()) order[g] = b->work[src];
        }
        b->work.swap(order);
    }
    e = hipMemcpyAsync(b->d_args, b->args.data(), sizeof(SweepArgs) * (size_t)n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_work, b->work.data(), sizeof(int2) * b->work.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return device_fail(e, "upload batch tables");
    for (int32_t i = 0; i <= n; ++i) b->host_label_off.push_back(i < n ? (int64_t)b->label_off[i] : (int64_t)labels);
    for (int32_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) b->host_dims.push_back(params[i].dims[d]);
    int64_t *d_label_off = reinterpret_cast<int64_t *>(ws + bl.label_off);
    int32_t *d_dims = reinterpret_cast<int32_t *>(ws + bl.dims);
    e = hipMemcpyAsync(d_label_off, b->host_label_off.data(), sizeof(int64_t) * b->host_label_off.size(),
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_dims, b->host_dims.data(), sizeof(int32_t) * b->host_dims.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return device_fail(e, "upload stats tables");
    b->stats_tables = cpm::StatsTables{d_label_off, d_dims, n, b->ndim, (int64_t)labels};
    b->scratch_v = reinterpret_cast<int32_t *>(ws + bl.scratch_v);
    b->scratch_s = reinterpret_cast<int32_t *>(ws + bl.scratch_s);
    b->scratch_c = reinterpret_cast<int64_t *>(ws + bl.scratch_c);
    b->scratch_ref = reinterpret_cast<int32_t *>(ws + bl.scratch_ref);
    cpm::BatchLaunch &L = b->launch;
    L.args = b->d_args;
    L.work = b->d_work;
    L.mcs = b->d_mcs;
    L.grid = bl.grid;
    L.lds = lds;
    L.ndim = b->ndim;
    L.act = b->act;
    L.mirror = b->mirror;
    L.single = b->single;
    L.k1 = b->k == 1;
    L.act_words = b->act_words;
    L.act16 = b->act16;
    L.ext = false;
    for (const SweepArgs &a : b->args) L.ext = L.ext || a.chem != nullptr;
    L.layout = b->layout;
    *out = b.release();
    return CPM_OK;
}

namespace {

// The kernels of one MCS of a batch, in order.  Every MCS has an even number
// of activations and sweeps always run whole MCS, so activation alpha of an
// MCS always reads counter buffer alpha & 1 and the sequence is the same for
// every MCS (the MCS index comes from the device counter).
hipError_t enqueue_mcs(const cpm_batch *b, uint32_t n_act, hipStream_t st)
{
    hipError_t e;
    for (uint32_t alpha = 0; alpha < n_act; ++alpha)
        if ((e = cpm::launch_batch_activation(b->launch, alpha, (int)(alpha & 1), st)) != hipSuccess) return e;
    if (b->act) {
        e = b->act16       ? cpm::launch_act16_decay(b->words16, b->total_sites, st)
            : b->act_words ? cpm::launch_act_decay_words(b->lattices, b->total_sites, st)
                           : cpm::launch_act_decay(b->act_field, b->total_sites, st);
        if (e != hipSuccess) return e;
    }
    return cpm::launch_add_u32(b->d_mcs, 1u, st);
}

// CPM_EDEVICE when a persistent launch of the batch gave up waiting at a
// grid barrier (its state is then invalid); waits for the stream.
int check_barrier(cpm_batch *b, hipStream_t st)
{
    cpm::GridBarrier g{};
    hipError_t e = hipMemcpyAsync(&g, b->bar, sizeof(g), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return device_fail(e, "read barrier");
    if (g.abort)
        return fail(CPM_EDEVICE, "a persistent launch of this batch gave up at a grid barrier (spin limit reached); "
                                 "the batch state is invalid");
    if (g.act_overflow)
        return fail(CPM_EDEVICE, "an activity above 31 was written into a batch that sweeps on 16-bit words; "
                                 "the batch state is invalid");
    return CPM_OK;
}

// Capture one MCS into an executable graph, on a private stream of default
// priority (the caller's stream is never put into capture mode).  The graph
// holds kernel nodes only.
hipError_t capture_mcs(cpm_batch *b, uint32_t n_act)
{
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t launched = enqueue_mcs(b, n_act, cs);
        e = hipStreamEndCapture(cs, &g);
        if (launched != hipSuccess) e = launched;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->mcs_graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) b->mcs_graph = nullptr;
    return e;
}

}  // namespace

int cpm_batch_sweep(cpm_batch *b, int32_t n_mcs, void *stream)
{
    if (!b) return fail(CPM_EINVAL, "batch is NULL");
    if (n_mcs < 0) return fail(CPM_EINVAL, "n_mcs must be >= 0");
    if (n_mcs == 0) return CPM_OK;
    hipStream_t st = as_stream(stream);
    int64_t sd = 1;
    for (int d = 0; d < b->ndim; ++d) sd *= b->s;
    const uint32_t n_act = (uint32_t)(((int64_t)1 << b->ndim) * sd / b->k);
    hipError_t e;
    if (b->mode == 0 && !b->mcs_graph && (e = capture_mcs(b, n_act)) != hipSuccess)
        return device_fail(e, "capture MCS graph");
    if (b->mirror && (e = cpm::launch_batch_mirror(b->d_args, b->n, b->max_sites, true, st)) != hipSuccess)
        return device_fail(e, "to 16-bit working copy");
    if (b->act_words && (e = cpm::launch_batch_act_words(b->d_args, b->n, b->max_sites, true, st)) != hipSuccess)
        return device_fail(e, "to label-type-activity words");
    if (b->act16 &&
        (e = cpm::launch_to_act16(b->lattices, b->act_field, b->words16, b->total_sites,
                                  reinterpret_cast<int32_t *>(&b->bar->act_overflow), st)) != hipSuccess)
        return device_fail(e, "to 16-bit label-activity words");
    if ((e = cpm::launch_set_u32(b->d_mcs, (uint32_t)b->mcs, st)) != hipSuccess) return device_fail(e, "set mcs");
    if (b->mode == 2) {
        // every MCS in one launch; the barrier's count and generation start
        // at 0 (its abort flag is sticky)
        cpm::PersistentLaunch p{};
        p.bar = b->bar;
        p.mcs0 = (uint32_t)b->mcs;
        p.n_mcs = n_mcs;
        p.n_act = n_act;
        p.n_work = b->launch.grid;
        p.spin_limit = b->spin_limit;
        p.decay_mode = !b->act ? 0 : b->act16 ? 3 : b->act_words ? 2 : 1;
        p.decay_ptr = !b->act ? nullptr : b->act16 ? static_cast<void *>(b->words16)
                    : b->act_words ? static_cast<void *>(b->lattices) : static_cast<void *>(b->act_field);
        p.n_sites = b->total_sites;
        if ((e = cpm::launch_fill_i32(reinterpret_cast<int32_t *>(b->bar), 0, 2, st)) != hipSuccess ||
            (e = cpm::launch_batch_persistent(b->launch, p, st)) != hipSuccess)
            return device_fail(e, "persistent launch");
        b->activation += (uint64_t)n_act * (uint64_t)n_mcs;
        b->mcs += (uint64_t)n_mcs;
        b->mcs_run += (uint64_t)n_mcs;
    }
    for (int32_t m = 0; m < n_mcs && b->mode != 2; ++m) {
        e = b->mode == 0 ? hipGraphLaunch(b->mcs_graph, st) : enqueue_mcs(b, n_act, st);
        if (e != hipSuccess) return device_fail(e, "MCS");
        b->activation += n_act;
        ++b->mcs;
        ++b->mcs_run;
    }
    if (b->mirror && (e = cpm::launch_batch_mirror(b->d_args, b->n, b->max_sites, false, st)) != hipSuccess)
        return device_fail(e, "from 16-bit working copy");
    if (b->act_words && (e = cpm::launch_batch_act_words(b->d_args, b->n, b->max_sites, false, st)) != hipSuccess)
        return device_fail(e, "from label-type-activity words");
    if (b->act16 && (e = cpm::launch_from_act16(b->words16, b->lattices, b->act_field, b->total_sites, st)) != hipSuccess)
        return device_fail(e, "from 16-bit label-activity words");
    return CPM_OK;
}

int cpm_batch_sweep_serial(cpm_batch *b, int32_t n_mcs, void *stream)
{
    if (!b) return fail(CPM_EINVAL, "batch is NULL");
    if (n_mcs < 0) return fail(CPM_EINVAL, "n_mcs must be >= 0");
    if (n_mcs == 0) return CPM_OK;
    hipStream_t st = as_stream(stream);
    const int parity = (int)(b->activation & 1);
    hipError_t e;
    if (b->mirror && (e = cpm::launch_batch_mirror(b->d_args, b->n, b->max_sites, true, st)) != hipSuccess)
        return device_fail(e, "to 16-bit working copy");
    for (int32_t m = 0; m < n_mcs; ++m) {
        e = cpm::launch_serial_mcs(b->d_args, b->n, b->ndim, b->act, b->mirror, (uint32_t)b->mcs, parity, st);
        if (e != hipSuccess) return device_fail(e, "serial MCS");
        ++b->mcs;
        ++b->mcs_run;
    }
    // the other counter buffer and the pending delta lists as the next
    // parallel activation expects them: exact counters, no deltas to re-add
    for (int32_t i = 0; i < b->n; ++i) {
        const SweepArgs &a = b->args[i];
        e = hipMemcpyAsync(a.counters[parity ^ 1], a.counters[parity], sizeof(int32_t) * 2 * ((size_t)b->n_cells[i] + 1),
                           hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = cpm::launch_fill_i32(a.dcount[parity ^ 1], 0, (size_t)a.tg.n_tiles, st);
        if (e != hipSuccess) return device_fail(e, "counters after serial MCS");
    }
    if (b->mirror && (e = cpm::launch_batch_mirror(b->d_args, b->n, b->max_sites, false, st)) != hipSuccess)
        return device_fail(e, "from 16-bit working copy");
    return CPM_OK;
}

int cpm_batch_occupancy(cpm_batch *b, int32_t *d_counts, void *stream)
{
    if (!b || !d_counts) return fail(CPM_EINVAL, "NULL argument");
    const size_t n_sites = (size_t)b->args[0].L[0] * b->args[0].L[1] * b->args[0].L[2];
    for (int32_t i = 1; i < b->n; ++i)
        if ((size_t)b->args[i].L[0] * b->args[i].L[1] * b->args[i].L[2] != n_sites ||
            b->args[i].L[0] != b->args[0].L[0] || b->args[i].L[1] != b->args[0].L[1])
            return fail(CPM_EINVAL, "occupancy needs lattices of one shape");
    const hipError_t e = cpm::launch_occupancy(b->lattices, b->n, n_sites, d_counts, as_stream(stream));
    return e == hipSuccess ? CPM_OK : device_fail(e, "occupancy");
}

int cpm_batch_launch_mode(cpm_batch *b, int32_t mode)
{
    if (!b) return fail(CPM_EINVAL, "batch is NULL");
    if (mode < 0 || mode > 2) return fail(CPM_EINVAL, "mode must be 0, 1 or 2");
    if (mode == 2 && !(b->k == 1 && b->layout == 2))
        return fail(CPM_ENOTSUP, "the persistent launch runs batches swept in place (k = 1)");
    b->mode = mode;
    b->use_graph = mode == 0;
    return CPM_OK;
}

int cpm_batch_set_barrier_spin_limit(cpm_batch *b, uint32_t polls)
{
    if (!b) return fail(CPM_EINVAL, "batch is NULL");
    b->spin_limit = polls;
    return CPM_OK;
}

int cpm_batch_use_graph(cpm_batch *b, int32_t enabled)
{
    if (!b) return fail(CPM_EINVAL, "batch is NULL");
    b->use_graph = enabled != 0;
    b->mode = enabled ? 0 : 1;
    return CPM_OK;
}

int cpm_batch_counters(cpm_batch *b, int32_t *d_volume, int32_t *d_surface, void *stream)
{
    if (!b || !d_volume || !d_surface) return fail(CPM_EINVAL, "NULL argument");
    for (int32_t i = 0; i < b->n; ++i) {
        const hipError_t e = cpm::launch_copy_counters(b->args[i].counters[b->activation & 1], b->n_cells[i] + 1,
                                                       d_volume + b->label_off[i], d_surface + b->label_off[i],
                                                       as_stream(stream));
        if (e != hipSuccess) return device_fail(e, "copy counters");
    }
    return CPM_OK;
}

int cpm_batch_cell_stats(cpm_batch *b, int32_t *d_volume, int32_t *d_surface, int64_t *d_centroid_sum, void *stream)
{
    if (!b || !d_volume || !d_surface) return fail(CPM_EINVAL, "NULL argument");
    const hipError_t e = cpm::launch_batch_cell_stats(b->d_args, b->stats_tables.label_off, b->n, b->ndim,
                                                      b->max_sites, b->max_bricks, (size_t)b->stats_tables.total_labels, d_volume,
                                                      d_surface, b->scratch_ref, d_centroid_sum, as_stream(stream));
    return e == hipSuccess ? CPM_OK : device_fail(e, "cell stats");
}

int cpm_batch_attempt_stats(cpm_batch *b, uint64_t *out, void *stream)
{
    if (!b || !out) return fail(CPM_EINVAL, "NULL argument");
    hipStream_t st = as_stream(stream);
    int rc = check_barrier(b, st);
    if (rc != CPM_OK) return rc;
    for (int32_t i = 0; i < b->n; ++i) {
        const SweepArgs &a = b->args[i];
        std::vector<uint64_t> per(2 * (size_t)a.tg.n_tiles);
        hipError_t e = hipMemcpyAsync(per.data(), a.stats, sizeof(uint64_t) * per.size(), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return device_fail(e, "read stats");
        out[3 * i] = b->mcs_run * (uint64_t)a.L[0] * a.L[1] * a.L[2];
        out[3 * i + 1] = 0;
        out[3 * i + 2] = 0;
        for (int t = 0; t < a.tg.n_tiles; ++t) {
            out[3 * i + 1] += per[2 * (size_t)t];
            out[3 * i + 2] += per[2 * (size_t)t + 1];
        }
    }
    return CPM_OK;
}

int cpm_batch_sample(cpm_batch *b, double *d_samples, int32_t k, int32_t n_samples, void *stream)
{
    if (!b || !d_samples) return fail(CPM_EINVAL, "NULL argument");
    if (n_samples < 1 || k < 0 || k >= n_samples) return fail(CPM_EINVAL, "sample index out of range");
    const int rc = cpm_batch_cell_stats(b, b->scratch_v, b->scratch_s, b->scratch_c, stream);
    if (rc != CPM_OK) return rc;
    const hipError_t e = cpm::launch_sample(b->stats_tables, b->scratch_v, b->scratch_s, b->scratch_c, d_samples, k,
                                            n_samples, as_stream(stream));
    if (e != hipSuccess) return device_fail(e, "sample");
    return CPM_OK;
}

int cpm_batch_summary(cpm_batch *b, const double *d_samples, int32_t n_samples, double interval, double *d_out,
                      void *stream)
{
    if (!b || !d_samples || !d_out) return fail(CPM_EINVAL, "NULL argument");
    if (n_samples < 1 || !(interval > 0.0)) return fail(CPM_EINVAL, "need samples and a positive interval");
    const hipError_t e = cpm::launch_summary(b->stats_tables, d_samples, n_samples, interval, d_out, as_stream(stream));
    if (e != hipSuccess) return device_fail(e, "summary");
    return CPM_OK;
}

int cpm_batch_autocorrelation(cpm_batch *b, const double *d_samples, int32_t n_samples, double *d_out, void *stream)
{
    if (!b || !d_samples || !d_out) return fail(CPM_EINVAL, "NULL argument");
    if (n_samples < 2) return fail(CPM_EINVAL, "need at least two samples");
    const hipError_t e = cpm::launch_autocorrelation(b->stats_tables, d_samples, n_samples, d_out, as_stream(stream));
    return e == hipSuccess ? CPM_OK : device_fail(e, "autocorrelation");
}

int cpm_batch_check_invariants(cpm_batch *b, void *stream, int32_t *h_ok)
{
    if (!b || !h_ok) return fail(CPM_EINVAL, "NULL argument");
    hipStream_t st = as_stream(stream);
    int rc = check_barrier(b, st);
    if (rc != CPM_OK) return rc;
    const int32_t n = b->n;
    std::vector<int32_t> bad((size_t)n, 0);
    auto sites = [&](int32_t i) { return (size_t)b->args[i].L[0] * b->args[i].L[1] * b->args[i].L[2]; };
    auto read_flags = [&]() {
        hipError_t e = hipSuccess;
        for (int32_t i = 0; i < n && e == hipSuccess; ++i)
            e = hipMemcpyAsync(&bad[i], b->check[i], sizeof(int32_t), hipMemcpyDeviceToHost, st);
        return e == hipSuccess ? hipStreamSynchronize(st) : e;
    };
    hipError_t e = hipSuccess;
    for (int32_t i = 0; i < n && e == hipSuccess; ++i) {
        h_ok[i] = 0;
        if ((e = cpm::launch_fill_i32(b->check[i], 0, 1, st)) == hipSuccess)
            e = cpm::launch_bad_labels(b->args[i].lat, sites(i), b->n_cells[i], b->obstacles[i] != 0, b->check[i], st);
    }
    if (e == hipSuccess) e = read_flags();
    if (e != hipSuccess) return device_fail(e, "check labels");
    std::vector<uint8_t> labels_ok((size_t)n);
    for (int32_t i = 0; i < n; ++i) labels_ok[i] = bad[i] == 0;
    const int parity = (int)(b->activation & 1);
    for (int32_t i = 0; i < n && e == hipSuccess; ++i) {
        if (!labels_ok[i]) continue;  // the recount indexes its outputs by label
        const size_t labels = (size_t)b->n_cells[i] + 1;
        int32_t *rv = b->check[i] + kCheckPad, *rs = rv + labels;
        if ((e = cpm::launch_fill_i32(rv, 0, 2 * labels, st)) == hipSuccess &&
            (e = cpm::launch_count(b->args[i], b->ndim, rv, rs, 1, st)) == hipSuccess)
            e = cpm::launch_compare_counters(b->args[i].counters[parity], rv, rs, (int32_t)labels, b->check[i], st);
    }
    if (e == hipSuccess) e = read_flags();
    if (e != hipSuccess) return device_fail(e, "check counters");
    for (int32_t i = 0; i < n; ++i) h_ok[i] = labels_ok[i] && bad[i] == 0 ? 1 : 0;
    return CPM_OK;
}

int cpm_batch_set_mcs(cpm_batch *b, uint64_t mcs)
{
    if (!b) return fail(CPM_EINVAL, "batch is NULL");
    b->mcs = mcs;
    return CPM_OK;
}

int cpm_batch_get_mcs(const cpm_batch *b, uint64_t *mcs)
{
    if (!b || !mcs) return fail(CPM_EINVAL, "NULL argument");
    *mcs = b->mcs;
    return CPM_OK;
}

int cpm_batch_destroy(cpm_batch *b)
{
    delete b;
    return CPM_OK;
}

}  // extern "C"
