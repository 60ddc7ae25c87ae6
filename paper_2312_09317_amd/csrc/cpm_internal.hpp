// Internal layout shared by the host side of libcpm and its HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace cpm {

constexpr int kMaxTypes = 16;
constexpr int kMaxTI = 4096;  // TI entries: enough for T up to ~184
// A thread keeps the records of its own accepted copies of one activation
// (the deltas its later attempts see) in registers, up to kOwnInRegs of
// them; with more attempts per activation (k > kOwnInRegs) the rest go to a
// per-thread-area spill array in the workspace.
constexpr int kOwnInRegs = 8;
constexpr int kBlock = 256;   // threads per sweep workgroup (one per thread area)
constexpr int kXcds = 8;      // MI355X: workgroups go round-robin to 8 XCDs, each with its own L2
// 16-bit label-activity words: label + 1 in 11 bits, activity in 5
constexpr int kMaxAct16Cells = 2046;
constexpr int kMaxAct16Activity = 31;

// Records msg as the calling thread's last error (cpm_last_error) and returns code.
int report_error(int code, const char *msg);

// Quantised model + acceptance / activity tables, copied once into the
// workspace at init.  Energies in units of 2^-16.
struct DeviceModel {
    int64_t J[kMaxTypes * kMaxTypes];
    int64_t lam_v[kMaxTypes];
    int64_t lam_s[kMaxTypes];
    int64_t r_act[kMaxTypes];   // lambda_act / max_act, quantised
    int32_t v_target[kMaxTypes];
    int32_t s_target[kMaxTypes];
    int32_t max_act[kMaxTypes];
    int32_t n_ti;
    int32_t pad_;
    uint64_t TI[kMaxTI];
    uint64_t TM[256];
    uint64_t TL[256];
    // the same tables as 32-bit words (entry 0, which is 2^32, left 0)
    uint32_t TI32[kMaxTI];
    uint32_t TM32[256];
    uint32_t TL32[256];
    // Act geometric mean in the log domain: LG[a] = round(ln a * 2^24);
    // exp(l * 2^-24) = EH[l >> 16] * EM[(l >> 8) & 255] * EL[l & 255] with
    // EH in 2^24, EM in 2^31 and EL in 2^30 units.
    int64_t LG[256];
    uint64_t EH[2048];
    uint64_t EM[256];
    uint64_t EL[256];
    // persistence: strength (2^-16), previous-direction weight (2^-14), and
    // the unit vectors of the Moore offsets, index (dx+1) + 3(dy+1) + 9(dz+1) (2^-14)
    int64_t lam_p[kMaxTypes];
    int64_t mu_p[kMaxTypes];
    // chemotaxis strength (2^-16)
    int64_t lam_c[kMaxTypes];
    int32_t unit[27][3];
};

// The per-type energy parameters of DeviceModel (lam_v through max_act, in
// its order): sweeps copy this block into LDS, where an attempt reads it
// without a round trip to global memory.
struct TypeParams {
    int64_t lam_v[kMaxTypes];
    int64_t lam_s[kMaxTypes];
    int64_t r_act[kMaxTypes];
    int32_t v_target[kMaxTypes];
    int32_t s_target[kMaxTypes];
    int32_t max_act[kMaxTypes];
};
static_assert(offsetof(DeviceModel, lam_v) % 16 == 0, "the block is copied in 16-byte words");
static_assert(sizeof(TypeParams) % 16 == 0, "the block is copied in 16-byte words");
static_assert(offsetof(DeviceModel, max_act) + sizeof(DeviceModel::max_act) - offsetof(DeviceModel, lam_v) ==
                      sizeof(TypeParams) &&
                  offsetof(DeviceModel, lam_s) - offsetof(DeviceModel, lam_v) == offsetof(TypeParams, lam_s) &&
                  offsetof(DeviceModel, r_act) - offsetof(DeviceModel, lam_v) == offsetof(TypeParams, r_act) &&
                  offsetof(DeviceModel, v_target) - offsetof(DeviceModel, lam_v) == offsetof(TypeParams, v_target) &&
                  offsetof(DeviceModel, s_target) - offsetof(DeviceModel, lam_v) == offsetof(TypeParams, s_target) &&
                  offsetof(DeviceModel, max_act) - offsetof(DeviceModel, lam_v) == offsetof(TypeParams, max_act),
              "TypeParams mirrors the per-type block of DeviceModel");

// How thread areas are grouped into workgroup tiles.  Tiles are numbered x
// fastest; the tiles of XCD x are the contiguous range
// [x * tiles_per_xcd, (x + 1) * tiles_per_xcd), so each XCD sweeps one slab
// of the lattice in every activation and its L2 keeps that slab.
struct TileGeometry {
    int32_t T[3];          // thread areas per tile per axis
    int32_t nt[3];         // tiles per axis
    int32_t n_tiles;
    int32_t tiles_per_xcd;
    int32_t grid;          // workgroups launched: kXcds * tiles_per_xcd
    int32_t box_sites;     // LDS sites of the largest staged box
    int32_t lds_bytes;
    int32_t layout;        // 0: halo boxes in LDS; 1: whole rows along x in LDS; 2: no staging (in place)
    int32_t row_chunk;     // bytes per load when staging label rows (16, 8 or 4)
    int32_t act_chunk;     // bytes per load when staging activity rows
    // 3D bricks (0 = tile index order): an XCD's slab is layers_per_xcd
    // layers of nt[1] x 1 tiles (tiles span whole rows, nt[0] == 1), taken in
    // bricks of brick_y x brick_z tiles, y fastest inside a brick and bricks
    // y fastest
    int32_t brick_y, brick_z, layers_per_xcd;
    // multipliers of the divisions a workgroup makes (FastDiv): by nt[0] and
    // nt[1], by T[0] and T[1], by the thread areas of the last tile along x
    // and y (na - (nt - 1) T), and by the sub-area edge s; 0 for a divisor of 1
    uint32_t div_nt[2], div_T[2], div_last[2], div_s;
};

// Pointer types of the sweep arguments: plain ones (the host, and kernels
// that take the struct by value); kernels that read the struct from device
// memory (batches) use SweepArgsT with global-memory pointers (defined next
// to them), so that the compiler reads through them with global, not flat,
// loads.
struct PlainPtrs {
    template <typename T>
    using ptr = T *;
};

// Everything a sweep kernel needs, passed by value.
template <typename PP>
struct SweepArgsT {
    template <typename T>
    using P = typename PP::template ptr<T>;
    P<void> cells;            // lattice the sweep works on: the caller's int32 one or the 16-bit mirror (label + 1)
    P<int32_t> lat;           // the caller's int32 lattice
    P<const int32_t> cell_type;
    P<uint8_t> act;
    P<const int4> pdir;       // persistence direction per label (x, y, z, unused), 2^-14; NULL when off
    P<const int16_t> chem;    // chemotaxis field, ndim components per site, 2^-14; NULL when off
    P<const DeviceModel> model;
    P<int32_t> counters[2];   // ping-pong (V, S) pairs per label
    P<int4> dlist[2];         // per tile: accepted copies of an activation, by activation parity
    P<int32_t> dcount[2];     // per tile: number of records in dlist[parity]
    P<uint64_t> stats;        // per tile: attempts past the early rejection, accepted copies
    P<int4> own_spill;        // k > kOwnInRegs: per tile and area, k - kOwnInRegs own records; else NULL
    // persistence: per label, the centroid sums (ndim int64) an accepted
    // copy updates, and the reference point (x, y, z, unused) its site is
    // unwrapped against; NULL when off
    P<int64_t> csum;
    P<const int4> cpos;
    int32_t L[3];
    int32_t na[3];         // thread areas per axis
    uint32_t n_areas;
    int32_t s;
    int32_t k;
    int32_t dlist_cap;     // records per tile
    int32_t obstacle_type;
    int32_t single_type;   // the one type of every cell, or -1 when cells differ in type
    int32_t n_types;       // types of the model (rows of J a sweep reads)
    int32_t lg_entries;    // entries of the Act log table a sweep can read: the largest activity + 1
    uint32_t key0, key1;
    uint32_t lattice_id;
    TileGeometry tg;
};
using SweepArgs = SweepArgsT<PlainPtrs>;

// A batched activation: all lattices of a batch in one launch.
struct BatchLaunch {
    const SweepArgs *args;  // device array, one per lattice
    const int2 *work;       // device array, (lattice, tile) per workgroup
    const uint32_t *mcs;    // device MCS counter shared by the batch
    int grid;
    size_t lds;
    int ndim;
    bool act, mirror, single, k1;
    bool ext;               // some lattice uses the chemotaxis term
    bool act_words;         // lattices hold label-type-activity words during the sweep
    bool act16;             // lattices sweep on 16-bit label-activity words (one cell type, no chemotaxis)
    int layout;
};

// State of the device-wide barrier of a persistent batch launch (device
// memory): arrivals, generation, and a sticky flag raised by a workgroup
// that gave up waiting.
struct GridBarrier {
    uint32_t count;
    uint32_t gen;
    uint32_t abort;
    uint32_t act_overflow;  // sticky: an activity too large for 16-bit words was met
};

// One persistent launch: n_mcs MCS of a batch (every activation, then the
// Act decay) in one kernel, workgroups looping over the work table and
// meeting at a grid barrier between phases.
struct PersistentLaunch {
    GridBarrier *bar;
    uint32_t mcs0;           // MCS index of the first MCS
    int32_t n_mcs;
    uint32_t n_act;          // activations per MCS
    int32_t n_work;          // entries of the work table
    uint32_t spin_limit;     // polls of a barrier wait before giving up
    int32_t decay_mode;      // Act decay after each MCS: 0 none, 1 uint8 array, 2 int32 words (bits 24..31),
                             // 3 16-bit words (bits 11..15)
    void *decay_ptr;
    size_t n_sites;          // sites of the whole batch
};

// Per-lattice tables for the summary statistics of a batch (device arrays).
struct StatsTables {
    const int64_t *label_off;  // n + 1 label offsets (labels of lattice i: [off[i], off[i+1]))
    const int32_t *dims;       // 3 per lattice
    int n;
    int ndim;
    int64_t total_labels;
};

// Launchers.  All asynchronous on `stream`.
hipError_t launch_fill_i32(int32_t *p, int32_t value, size_t n, hipStream_t stream);
// Persistence directions: init (P = 0, every history slot = the current
// centroid) or one update (update index t >= 1), from centroid sums (ndim per
// label) and volumes (the V of (V, S) counter pairs).
struct PersistArgs {
    int4 *pdir;
    int64_t *hist;         // per label: slots x 3 centroids, 2^-16
    int4 *cpos;            // per label: the centroid rounded to a site, the sweeps' reference point
    const int64_t *csum;
    const int32_t *pairs;
    const int32_t *cell_type;
    const DeviceModel *model;
    int32_t n_labels, ndim, slots;
    int32_t L[3];
};
hipError_t launch_persist(const PersistArgs &p, int64_t t, hipStream_t stream);
// n_types x n_types int64 contact counts of a lattice (cleared first).
hipError_t launch_contacts(const SweepArgs &a, int ndim, int n_types, int64_t *out, hipStream_t stream);
// Volume, surface and (cent != NULL) centroid sums of every lattice of a
// batch, packed per label; ref is scratch of total_labels entries.
// max_bricks: the largest reduce_brick_count of the batch's lattices.
hipError_t launch_batch_cell_stats(const SweepArgs *d_args, const int64_t *d_label_off, int n_lattices, int ndim,
                                   size_t max_sites, int64_t max_bricks, size_t total_labels, int32_t *v_out,
                                   int32_t *s_out, int32_t *ref, int64_t *cent, hipStream_t stream);
// One MCS of the serial CPM on every lattice of a batch (one wave each);
// counters: the exact buffer `parity`.
hipError_t launch_serial_mcs(const SweepArgs *d_args, int n_lattices, int ndim, bool act, bool mirror, uint32_t mcs,
                             int parity, hipStream_t st);
// Per site, how many lattices of a batch hold a cell there (all lattices of
// one size, n_sites each, packed back to back).
hipError_t launch_occupancy(const int32_t *lattices, int n_lattices, size_t n_sites, int32_t *counts,
                            hipStream_t st);
// Workgroups of the centroid reductions over a lattice of dims L.
int64_t reduce_brick_count(const int *L, int ndim);
hipError_t launch_count(const SweepArgs &a, int ndim, int32_t *v_out, int32_t *s_out, int stride,
                        hipStream_t stream);
// Stored words the sweep works on: the caller's int32 labels, the 16-bit
// working copy, or the int32 lattice rewritten in place as packed words.
enum Words { kWords32 = 0, kWords16 = 1, kWordsPacked = 2, kWordsPackedAct = 3 };
hipError_t launch_activation(const SweepArgs &a, int ndim, bool act, int words, uint32_t mcs, uint32_t alpha,
                             int parity, hipStream_t stream);
// The activation kernels for stored words Cell in D dimensions (defined in
// cpm_sweep_kernels.hpp, instantiated in cpm_sweep_inst.hip).
template <typename Cell, int D>
hipError_t sweep_words(const SweepArgs &a, bool act, uint32_t mcs, uint32_t alpha, int parity, size_t lds,
                       hipStream_t st);
template <typename Cell, int D>
hipError_t batch_words(const BatchLaunch &b, uint32_t alpha, int parity, hipStream_t st);
// A persistent launch of a batch swept in place (k = 1): as many workgroups
// as fit the device at once (a multiple of the XCD count), launched
// cooperatively so that all are resident.
template <typename Cell, int D>
hipError_t batch_persistent_words(const BatchLaunch &b, const PersistentLaunch &p, hipStream_t st);
hipError_t launch_batch_persistent(const BatchLaunch &b, const PersistentLaunch &p, hipStream_t stream);
hipError_t launch_pack(int32_t *lat, const int32_t *cell_type, int obstacle_type, size_t n, hipStream_t stream);
hipError_t launch_unpack(int32_t *lat, size_t n, hipStream_t stream);
// The same with the activity in bits 24..31 (label + 1 in 0..19, type in 20..23).
hipError_t launch_pack_act(int32_t *lat, const uint8_t *act, const int32_t *cell_type, int obstacle_type, size_t n,
                           hipStream_t stream);
hipError_t launch_unpack_act(int32_t *lat, uint8_t *act, size_t n, hipStream_t stream);
hipError_t launch_act_decay_words(int32_t *lat, size_t n, hipStream_t stream);
// Every lattice of a batch to (to_words) or from label-type-activity words.
hipError_t launch_batch_act_words(const SweepArgs *d_args, int n_lattices, size_t max_sites, bool to_words,
                                  hipStream_t stream);
hipError_t launch_to_mirror(const int32_t *lat, uint16_t *mirror, size_t n, hipStream_t stream);
hipError_t launch_from_mirror(const uint16_t *mirror, int32_t *lat, size_t n, hipStream_t stream);
// Every lattice of a batch (args[i].lat <-> args[i].cells) in one launch.
hipError_t launch_batch_mirror(const SweepArgs *d_args, int n_lattices, size_t max_sites, bool to_mirror,
                               hipStream_t stream);
hipError_t launch_act_decay(uint8_t *act, size_t n, hipStream_t stream);
// 16-bit label-activity words of a whole batch (n sites, packed like the
// int32 lattices): from / to the int32 labels and uint8 activities, and the
// per-MCS Act decay in the words.
// launch_to_act16 raises *overflow (sticky) when an activity exceeds the
// 5 bits of the words.
hipError_t launch_to_act16(const int32_t *lat, const uint8_t *act, uint16_t *words, size_t n, int32_t *overflow,
                           hipStream_t stream);
// Adds to *count the number of activities above `limit`.
hipError_t launch_count_above(const uint8_t *act, size_t n, int limit, int32_t *count, hipStream_t stream);
hipError_t launch_from_act16(const uint16_t *words, int32_t *lat, uint8_t *act, size_t n, hipStream_t stream);
hipError_t launch_act16_decay(uint16_t *words, size_t n, hipStream_t stream);
hipError_t launch_centroids(const SweepArgs &a, int ndim, int32_t n_cells, int32_t *ref,
                            int64_t *out, hipStream_t stream, int words = kWords32);
// Persistence directions (x, y, z of each int4) into out, 3 x n_labels int32.
hipError_t launch_copy_dirs(const int4 *pdir, int32_t n_labels, int32_t *out, hipStream_t stream);
hipError_t launch_copy_counters(const int32_t *pairs, int32_t n_labels, int32_t *v_out,
                                int32_t *s_out, hipStream_t stream);
hipError_t launch_batch_activation(const BatchLaunch &b, uint32_t alpha, int parity, hipStream_t stream);
hipError_t launch_set_u32(uint32_t *p, uint32_t value, hipStream_t stream);
// Adds to *bad the number of sites of an int32 lattice labelled outside
// [-1, n_cells] (or -1 when !allow_obstacle).
hipError_t launch_bad_labels(const int32_t *lat, size_t n, int32_t n_cells, bool allow_obstacle, int32_t *bad,
                             hipStream_t stream);
// Adds to *bad the number of labels 1..n_labels-1 whose (V, S) pair in
// `pairs` differs from v[label], s[label].
hipError_t launch_compare_counters(const int32_t *pairs, const int32_t *v, const int32_t *s, int32_t n_labels,
                                   int32_t *bad, hipStream_t stream);
hipError_t launch_add_u32(uint32_t *p, uint32_t value, hipStream_t stream);
hipError_t launch_sample(const StatsTables &t, const int32_t *vol, const int32_t *surf, const int64_t *csum,
                         double *samples, int k, int n_samples, hipStream_t stream);
hipError_t launch_summary(const StatsTables &t, const double *samples, int n_samples, double interval, double *out,
                          hipStream_t stream);
hipError_t launch_autocorrelation(const StatsTables &t, const double *samples, int n_samples, double *out,
                                  hipStream_t stream);
size_t sweep_lds_bytes(int ndim, bool act, bool mirror, int box_sites);

}  // namespace cpm
