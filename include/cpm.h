/*
 * cpm.h - C ABI of the MI355X cellular Potts model sweep library (libcpm.so).
 *
 * The library advances a cellular Potts model (CPM) lattice by Monte Carlo
 * steps (MCS) under the checkerboard parallel update scheme of Sultan, Devi,
 * Mueller & Textor (2023), "A parallelized cellular Potts model that enables
 * simulations at tissue scale", on an AMD Instinct MI355X (gfx950).
 *
 * Model (paper, Methods):
 *   H = sum_{i,j Moore neighbours} J(tau(sigma_i), tau(sigma_j)) (1 - delta(sigma_i, sigma_j))
 *     + sum_sigma lambda_V(tau) (V(sigma) - V_t(tau))^2                           (eq. 1)
 *     + sum_sigma lambda_S(tau) (S(sigma) - S_t(tau))^2                           (eq. 3)
 *   with S(sigma) the number of (site of sigma, Moore neighbour not of sigma)
 *   pairs; optional Act term dH_act (eq. 7) with the geometric mean of eq. 8.
 *   A copy attempt at site t from a Moore neighbour is accepted with
 *   probability 1 if dH <= 0, else exp(-dH/T) (eq. 2).
 *
 * Parallel scheme (paper, Results, "Designing a parallel execution scheme"
 * and "Aligning the lattice update statistics"; Fig. 2A-B, Fig. 3):
 *   the lattice is cut into thread areas of edge 2s; each area holds 2^d
 *   sub-areas of edge s, one per colour.  One MCS is (2s)^d / k activations;
 *   activation a activates colour a mod 2^d and every area makes k copy
 *   attempts inside its sub-area of that colour.  All attempts of one
 *   activation read the per-cell volume / surface counters as they stood at
 *   the start of the activation (plus the attempting thread's own earlier
 *   deltas); all accepted copies' deltas are summed into the counters before
 *   the next activation, so tracked volumes always equal lattice counts.
 *
 * Determinism: every copy attempt draws its random numbers from Philox4x32-10
 * (Salmon et al., SC'11) with key (seed lo, seed hi) and counter
 * (area index, MCS, activation << 8 | attempt, lattice_id).  Results depend
 * only on the initial state, the quantised parameters, s, k, seed, lattice_id
 * and the MCS counter - never on launch geometry or timing - and equal, bit
 * for bit, those of a serial run of the same scheme.
 *
 * Fixed point: energies are int64 in units of 2^-16; every energy parameter
 * (J, lambda_*) is rounded half away from zero to that grid at init.
 * Acceptance compares a uniform 32-bit draw u with
 * THR(q) = floor(TI[h] * TM[m] * TL[l] / 2^64), q = dH * 2^16 = h*2^16 + m*2^8 + l,
 * TI[h] = floor(2^32 exp(-h/T)), TM[m] = floor(2^32 exp(-m/(256 T))),
 * TL[l] = floor(2^32 exp(-l/(65536 T))), built in FP64 on the host;
 * accept iff q <= 0 or u < THR(q).
 *
 * Memory: every device buffer (lattice, cell types, activity, workspace,
 * outputs) is allocated and owned by the caller (e.g. as torch tensors) and
 * borrowed by the handle until cpm_destroy.  The library allocates no device
 * memory.  The handle owns host state only.
 *
 * Streams: calls taking `stream` (a hipStream_t) enqueue work on it and
 * return without waiting; the caller synchronises.  Calls on one handle must
 * be issued on one stream (or be ordered by the caller).
 *
 * Errors: every call returns CPM_OK (0) or a CPM_E* code; cpm_last_error()
 * returns a thread-local message for the last failure.  No call aborts or
 * throws across the ABI.  A failed call leaves the handle usable unless it
 * returned CPM_EDEVICE.
 */
#ifndef CPM_H
#define CPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPM_OK 0
#define CPM_EINVAL 1  /* invalid argument: dims, s, k, labels, null pointers */
#define CPM_ERANGE 2  /* a fixed-point energy could overflow int64 */
#define CPM_ENOMEM 3  /* workspace smaller than cpm_workspace_bytes() */
#define CPM_EDEVICE 4 /* HIP runtime error */
#define CPM_ENOTSUP 5 /* valid model the library does not run */

#define CPM_MAX_TYPES 16

/*
 * Model and scheme description.  All pointers are host memory, read during
 * cpm_validate / cpm_workspace_bytes / cpm_init only.
 *
 * Lattice values: -1 = static obstacle (never copied, never overwritten),
 * 0 = medium, 1..n_cells = cells.  Type 0 is the medium's type.
 */
typedef struct cpm_params {
    int32_t ndim;          /* 2 or 3 */
    int32_t dims[3];       /* Lx, Ly, Lz; Lz = 1 when ndim == 2; each divisible by 2*sub */
    int32_t sub;           /* s, sub-area edge (>= 1; >= 2 when act_enabled) */
    int32_t attempts;      /* k, copy attempts per thread area per activation; divides s^ndim */
    int32_t n_types;       /* 1..CPM_MAX_TYPES, including the medium type 0 */
    int32_t obstacle_type; /* type used for J against obstacle sites; -1 if the lattice has none */
    double temperature;    /* T > 0 (eq. 2) */
    uint64_t seed;         /* Philox key */
    uint32_t lattice_id;   /* fourth Philox counter word: tells replicate lattices apart */
    int32_t act_enabled;   /* 1: Act term (eq. 7-8) and activity bookkeeping */
    const double *J;              /* n_types * n_types, row-major, symmetric */
    const double *lambda_volume;  /* n_types */
    const int32_t *volume_target; /* n_types */
    const double *lambda_surface; /* n_types (may be NULL: no surface term) */
    const int32_t *surface_target;/* n_types (may be NULL when lambda_surface is NULL) */
    const double *lambda_act;     /* n_types (read when act_enabled) */
    const int32_t *max_act;       /* n_types, 0..255; a type is motile iff max_act > 0 */
    /* How the sweep is laid out on the GPU (results never depend on it; an
     * autotuner picks it by timing): 0 = the library's choice, 1 = halo boxes
     * staged in LDS, 2 = whole lattice rows staged in LDS (k = 1), 3 = the
     * lattice read in place (k = 1).  A layout that cannot run this model
     * gives CPM_ENOTSUP. */
    int32_t layout;
    int32_t tile[3];              /* thread areas per workgroup tile (product <= 256); 0 = the library's choice.
                                     With layout 2 tile[0] must be 0 or the whole row of areas. */
    /* Persistence (Methods, eq. 5-6; NULL lambda_persistence = off; not for
     * batches).  Every cell has a direction P, updated after each MCS from the
     * displacement D of its centroid over the last persistence_dt MCS, in
     * integers: centroids X = floor(centroid sum * 2^16 / V) (sums as in
     * cpm_cell_stats); D = X - X(dt MCS ago) per axis at its minimum image;
     * u = trunc(D * 2^14 / |D|); p = (2^14 - mu) u + mu P with
     * mu = round(persistence_mu * 2^14); P = trunc(p * 2^14 / |p|); |.| the
     * floor of the Euclidean norm, 0 / 0 = 0, dead cells P = 0.  A copy
     * from source s into target t by cell c of type tc adds
     * -floor(lambda * (U(t - s) . P_c) / 2^28) (2^-16 units) to the energy
     * change, U the offset's unit vector rounded to 2^-14: copies along a
     * cell's direction are favoured (the paper's sign convention is read
     * this way; its formula alone would penalise them). */
    const double *lambda_persistence; /* n_types (2^-16 quantised like J) */
    const double *persistence_mu;     /* n_types, 0..1 */
    int32_t persistence_dt;           /* >= 1 */
    /* Chemotaxis (Methods, eq. 4; NULL lambda_chemotaxis = off).  A fixed
     * vector field C: d_chemotaxis_field is device memory, int16, ndim
     * components (x, y[, z]) per site in lattice order, in units of 2^-14
     * (|C| <= 1 in the paper), 4-byte aligned, owned by the caller and read
     * until the handle is destroyed.  A copy from source s into target t by
     * cell c of type tc adds -floor(lambda * (U(t - s) . C(s)) / 2^28) (2^-16
     * units) to the energy change, U as for persistence: copies along the
     * field at their source are favoured (the sign read as for persistence).
     * Medium copies get no term. */
    const double *lambda_chemotaxis;  /* n_types (2^-16 quantised like J) */
    const int16_t *d_chemotaxis_field;
    /* Order in which each XCD works through its slab of tiles (results never
     * depend on it): 0 = the library's choice, 1 = tile index order, 2 = 3D
     * bricks of up to 16 x 16 tiles across y and z, so that the workgroups
     * resident on an XCD at once share their halo planes in its L2 (3D
     * lattices whose tiles span whole rows along x and divide evenly among
     * the XCDs; CPM_ENOTSUP otherwise). */
    int32_t tile_order;
    /* How the persistence update gets each cell's centroid (Methods, eq. 6;
     * composite variable tracking): 0 = recounted from the lattice at every
     * update, each site taken as its periodic image nearest the cell's
     * lowest-index site (the default; exact for cells of any shape); 1 =
     * kept by the sweeps, each accepted copy moving its site between the two
     * cells' integer sums as the image nearest each cell's reference point
     * (its centroid rounded to a site at the last update).  The two agree,
     * bit for bit in every direction, while every cell spans less than half
     * the lattice along each axis; mode 1 saves the recount's two passes over
     * the lattice per MCS.  Ignored without persistence. */
    int32_t persistence_centroids;
} cpm_params;

typedef struct cpm_handle cpm_handle;

/* Checks a model description without touching any device.  n_cells is the
 * largest cell label.  Returns CPM_OK, CPM_EINVAL, CPM_ERANGE or
 * CPM_ENOTSUP. */
int cpm_validate(const cpm_params *params, int32_t n_cells);

/* Device workspace size (bytes) cpm_init needs for this model; host only. */
int cpm_workspace_bytes(const cpm_params *params, int32_t n_cells, size_t *bytes);

/* How cpm_init will tile this model (host only, for reports and tests):
 * out[0..2] thread areas per workgroup tile along x, y, z; out[3] the layout:
 * 0 = each tile stages its active sub-areas with their halo in LDS, 1 = tiles
 * span whole lattice rows staged in LDS, 2 = attempts read the lattice in
 * place (k = 1); out[4] staged LDS bytes per workgroup; out[5] tiles per
 * activation; out[6] 1 if sweeps run on a 16-bit copy of the labels (up to
 * 65,534 cells).  Results
 * never depend on the tiling or layout. */
int cpm_tile_shape(const cpm_params *params, int32_t n_cells, int32_t *out);

/*
 * Binds a lattice to a new handle and counts every cell's volume and surface
 * from the lattice (the counters the sweep then keeps exact).
 *   d_lattice   int32[Lz][Ly][Lx] device, read/write; labels in [-1, n_cells]
 *   d_cell_type int32[n_cells + 1] device, read only; entry 0 must be 0
 *   d_act       uint8[Lz][Ly][Lx] device activity field when act_enabled,
 *               else NULL; read/write
 *   d_workspace device buffer of at least cpm_workspace_bytes(), 256-byte
 *               aligned, contents arbitrary; owned by the library until
 *               cpm_destroy
 * Every label is checked on the device before anything else runs (the call
 * waits for the stream): a label outside [-1, n_cells], or -1 in a model
 * with obstacle_type = -1, gives CPM_EINVAL and no handle.  The MCS counter
 * starts at 0.
 */
int cpm_init(const cpm_params *params, int32_t *d_lattice, const int32_t *d_cell_type,
             int32_t n_cells, uint8_t *d_act, void *d_workspace, size_t workspace_bytes,
             void *stream, cpm_handle **out);

/*
 * cpm_init without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The handle's device state lives in a
 * static array of the library, CPM_STATIC_WORKSPACE_BYTES per GPU, held
 * from this call to cpm_destroy; the call allocates no device memory (the
 * handle's host state comes from the host heap, as with cpm_init).
 * Arguments, behaviour and results are those of cpm_init.  Errors, besides
 * cpm_init's: CPM_ENOMEM when the model needs a larger workspace than the
 * array (cpm_workspace_bytes), CPM_EINVAL while another handle holds the
 * array of the current device (one such handle per GPU at a time: calls on
 * two handles would race on the same memory).  The array keeps the last
 * handle's contents; init clears everything a sweep reads before writing.
 */
#define CPM_STATIC_WORKSPACE_BYTES (16u << 20)
int cpm_init_static(const cpm_params *params, int32_t *d_lattice, const int32_t *d_cell_type, int32_t n_cells,
                    uint8_t *d_act, void *stream, cpm_handle **out);

/* Advances the lattice by n_mcs Monte Carlo steps (n_mcs >= 0) and the MCS
 * counter with it.  Asynchronous on `stream`.  While the call's work runs,
 * d_lattice and d_act may hold an internal encoding (lattices of more than
 * 65,534 cells of several types are rewritten in place as label-and-type
 * words, with the activity in the same word when the Act term is on and
 * there are at most 2^20 - 2 cells, and restored at the end of the call's
 * work); read or write them only on `stream` or after that work, as for
 * any buffer the sweep updates. */
int cpm_sweep(cpm_handle *h, int32_t n_mcs, void *stream);

/*
 * Recounts, from the lattice alone, every label's volume V and surface S
 * (d_volume, d_surface: int32[n_cells + 1] device; entry 0 is the medium's)
 * and, if d_centroid_sum is not NULL, int64[(n_cells + 1) * ndim] sums of
 * each cell's site coordinates, each site taken as the periodic image nearest
 * to the cell's lowest-index site (entry 0 is zero).  Asynchronous.
 */
int cpm_cell_stats(cpm_handle *h, int32_t *d_volume, int32_t *d_surface, int64_t *d_centroid_sum,
                   void *stream);

/* Contact statistics of the lattice by cell type, the read-out of the cell
 * sorting experiments (Results, cell sorting; Fig. 4: homotypic and
 * heterotypic cell borders): d_out[a * n_types + b] (int64, device, n_types^2
 * entries, overwritten) = the number of ordered pairs (x, y), y a Moore
 * neighbour of x, with different labels, neither an obstacle, x of type a and
 * y of type b (the medium is type 0).  The matrix is symmetric; row a summed
 * over b is the surface (cpm_cell_stats) of the cells of type a, less their
 * contacts with obstacles.  Asynchronous. */
int cpm_contacts(cpm_handle *h, int64_t *d_out, void *stream);

/* Persistence directions P of every label (int32, device, (n_cells + 1) x 3:
 * x, y, z in 2^-14 units; label 0 and dead cells 0), as the parameters'
 * persistence fields define them.  CPM_EINVAL when persistence is off.
 * Asynchronous. */
int cpm_persistence(cpm_handle *h, int32_t *d_dir, void *stream);

/* Copies the volume / surface counters the sweep tracks (int32[n_cells + 1]
 * each, device; entry 0 unused and written as 0).  Asynchronous. */
int cpm_counters(cpm_handle *h, int32_t *d_volume, int32_t *d_surface, void *stream);

/*
 * Failure detection.  The scheme guarantees that a cell's tracked size
 * equals the number of lattice sites it occupies, whatever order the atomic
 * updates of concurrent copies land in (paper, Results, "Designing a
 * parallel execution scheme", Fig. 2B: atomic updates of per-cell
 * variables).  This call recounts every label's volume and surface from the
 * lattice on the device (as cpm_cell_stats does) and compares them with the
 * counters the sweep tracks: *h_ok (host) = 1 when every site's label lies
 * in [-1, n_cells] (-1 only with an obstacle type) and every cell's tracked
 * (V, S) equals the recount, else 0.  Labels are checked first; out-of-range
 * labels give 0 without a recount.  Uses the check section of the handle's
 * workspace; changes neither the lattice nor the counters.  Waits for the
 * stream.  Returns CPM_OK whatever the verdict (CPM_EINVAL for NULL
 * arguments, CPM_EDEVICE for a HIP error).
 */
int cpm_check_invariants(cpm_handle *h, void *stream, int32_t *h_ok);

/* Copy-attempt statistics since cpm_init, read synchronously on `stream`
 * (waits for the stream): out[0] attempts, out[1] attempts past the early
 * rejection (distinct, non-obstacle labels), out[2] accepted copies. */
int cpm_attempt_stats(cpm_handle *h, uint64_t *out, void *stream);

/* MCS counter (the second Philox counter word of the next MCS).  Setting it
 * lets a run resume bit-exactly from a saved lattice / activity state. */
int cpm_set_mcs(cpm_handle *h, uint64_t mcs);
int cpm_get_mcs(const cpm_handle *h, uint64_t *mcs);

/* Releases host state; the caller's device buffers are untouched. */
int cpm_destroy(cpm_handle *h);

const char *cpm_strerror(int code);
const char *cpm_last_error(void);

/*
 * Batches: n independent lattices (replicates or parameter sweeps, paper,
 * Results, "Serial Cellular Potts Models are limited to sub-millimetre scale",
 * Fig. 1B) advanced together, every activation of all of them in one launch.
 * Lattice i follows params[i] (its own dims, energies, temperature, seed,
 * lattice_id); all share ndim, sub, attempts and act_enabled.  Each lattice
 * evolves exactly as it would alone under cpm_sweep.
 *
 * Device buffers are packed back to back in params order:
 *   d_lattices   int32, lattice i occupies dims[0]*dims[1]*dims[2] sites
 *   d_cell_types int32, lattice i occupies n_cells[i] + 1 entries
 *   d_act        uint8 activity, packed like d_lattices (NULL unless act)
 * Per-cell outputs (counters, cell stats) are packed like d_cell_types
 * (centroid sums: ndim entries per label).  The batch shares one MCS counter.
 * Ownership, streams and errors as for single lattices.
 */
typedef struct cpm_batch cpm_batch;

int cpm_batch_workspace_bytes(const cpm_params *params, int32_t n, const int32_t *n_cells, size_t *bytes);
int cpm_batch_init(const cpm_params *params, int32_t n, const int32_t *n_cells, int32_t *d_lattices,
                   const int32_t *d_cell_types, uint8_t *d_act, void *d_workspace, size_t workspace_bytes,
                   void *stream, cpm_batch **out);
/* Runs n_mcs MCS of every lattice.  By default each MCS is one launch of an
 * executable HIP graph captured at the first call (the activations, the Act
 * decay and the MCS counter update, kernel nodes only); the graph is
 * captured on a private stream and launched on `stream`. */
int cpm_batch_sweep(cpm_batch *b, int32_t n_mcs, void *stream);
/* enabled = 0: cpm_batch_sweep launches the same kernels one by one instead
 * of the graph (same results).  Pure host. */
int cpm_batch_use_graph(cpm_batch *b, int32_t enabled);
/* How cpm_batch_sweep launches its work (same results in every mode; pure
 * host): 0 = one replay of the captured MCS graph per MCS (the default),
 * 1 = the graph's kernels one by one, 2 = one persistent launch per call:
 * as many workgroups as the GPU holds at once (launched cooperatively, so
 * all are resident) loop over the (lattice, tile) work table and meet at a
 * device-wide barrier after every activation and after every MCS's Act
 * decay (paper, Results, "Designing a parallel execution scheme": the
 * whole grid synchronises between activations).  Mode 2 needs batches swept
 * in place (k = 1; CPM_ENOTSUP otherwise).  A barrier wait is bounded (see
 * cpm_batch_set_barrier_spin_limit): a launch whose wait runs out ends
 * early and leaves the batch invalid, which cpm_batch_attempt_stats and
 * cpm_batch_check_invariants report as CPM_EDEVICE. */
int cpm_batch_launch_mode(cpm_batch *b, int32_t mode);
/* Polls of one barrier wait before a persistent launch gives up (default
 * 2^20, about a second; a barrier normally completes in microseconds).
 * Pure host. */
int cpm_batch_set_barrier_spin_limit(cpm_batch *b, uint32_t polls);
/* Runs n_mcs MCS of the serial CPM on every lattice (Methods, first
 * paragraph; the reference of Fig. 5 and Fig. 6E): per MCS, N = sites copy
 * attempts, attempt i at target floor(u0 * N / 2^32) with the Philox counter
 * (i, MCS, 0xFFFFFF00, lattice_id), a Moore neighbour as source from u1 and
 * the acceptance draw u2; every attempt sees the lattice, the activity and
 * the per-cell counters as the attempt before it left them; Act decays at
 * the end of each MCS.  Energies as for cpm_batch_sweep (adhesion, volume,
 * surface, Act, chemotaxis).  One wave per lattice: this is the slow
 * reference, not a fast path.  Shares the MCS counter and the attempt
 * statistics with cpm_batch_sweep, and may be mixed with it. */
int cpm_batch_sweep_serial(cpm_batch *b, int32_t n_mcs, void *stream);
/* Per site, the number of lattices of the batch that hold a cell (label
 * >= 1) there: d_counts int32, one entry per site of one lattice (device,
 * overwritten).  Every lattice must have the same dims.  The per-pixel
 * occupancy of an ensemble (Fig. 5A, Fig. 6E). */
int cpm_batch_occupancy(cpm_batch *b, int32_t *d_counts, void *stream);
int cpm_batch_counters(cpm_batch *b, int32_t *d_volume, int32_t *d_surface, void *stream);
int cpm_batch_cell_stats(cpm_batch *b, int32_t *d_volume, int32_t *d_surface, int64_t *d_centroid_sum,
                         void *stream);
/* out: 3 entries per lattice, as cpm_attempt_stats; waits for the stream. */
int cpm_batch_attempt_stats(cpm_batch *b, uint64_t *out, void *stream);
/* cpm_check_invariants for every lattice of a batch: h_ok (host, n
 * entries), 1 where lattice i passes.  cpm_batch_init checks every label
 * of every lattice as cpm_init does (CPM_EINVAL). */
int cpm_batch_check_invariants(cpm_batch *b, void *stream, int32_t *h_ok);
/*
 * Cell-level summary statistics of a batch.  cpm_batch_sample records, for
 * every lattice i and label c, the record (V, S, x, y, z) of sample k:
 * volume and surface recounted from the lattice and the centroid
 * (centroid sum / V, reduced into [0, L) per axis; 0 for dead cells).
 * d_samples is a device array of doubles packed per lattice: lattice i starts
 * at label_offset(i) * n_samples * 5 and holds [n_samples][n_cells_i + 1][5].
 * cpm_batch_summary reduces n_samples samples taken `interval` MCS apart to
 * 8 doubles per lattice (d_out[8 i + j]): mean and population variance of
 * volume, of surface (cells alive at a sample), of speed (minimum-image
 * centroid displacement between consecutive samples / interval) and of
 * persistence time (per cell, the first lag at which the mean dot product of
 * unit displacements drops below 1/e, linearly interpolated, in MCS; the
 * longest defined lag if it never does).  The paper's motility read-outs are
 * speed and directional autocorrelation (Results, Fig. 5B); these formulas
 * are this library's reading.
 */
int cpm_batch_sample(cpm_batch *b, double *d_samples, int32_t k, int32_t n_samples, void *stream);
int cpm_batch_summary(cpm_batch *b, const double *d_samples, int32_t n_samples, double interval, double *d_out,
                      void *stream);
/* Directional autocorrelation (Fig. 5B) from n_samples >= 2 samples of
 * cpm_batch_sample: for lattice i and lag tau = 0..n_samples-2 (in sample
 * intervals), d_out[2 ((n_samples - 1) i + tau)] = the sum over cells c and
 * steps k of u_k(c) . u_{k+tau}(c), u the unit minimum-image displacement
 * of the centroid between samples k and k+1 (defined when the cell is alive
 * at both and moved), over the pairs where both are defined, and
 * d_out[... + 1] = the number of such pairs (doubles, device).  Their ratio
 * is A(tau); runs pool by adding sums and counts. */
int cpm_batch_autocorrelation(cpm_batch *b, const double *d_samples, int32_t n_samples, double *d_out,
                              void *stream);
int cpm_batch_set_mcs(cpm_batch *b, uint64_t mcs);
int cpm_batch_get_mcs(const cpm_batch *b, uint64_t *mcs);
int cpm_batch_destroy(cpm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* CPM_H */
