// Internal layout shared by the host side of libcpm and its HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace cpm {

constexpr int kMaxTypes = 16;
constexpr int kMaxTI = 4096;  // TI entries: enough for T up to ~184
constexpr int kMaxAttempts = 8;

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
    // Act geometric mean in the log domain: LG[a] = round(ln a * 2^24);
    // exp(l * 2^-24) = EH[l >> 16] * EM[(l >> 8) & 255] * EL[l & 255] with
    // EH in 2^24, EM in 2^31 and EL in 2^30 units.
    int64_t LG[256];
    uint64_t EH[2048];
    uint64_t EM[256];
    uint64_t EL[256];
};

// Everything a sweep kernel needs, passed by value.
struct SweepArgs {
    int32_t *lat;
    const int32_t *cell_type;
    uint8_t *act;
    const DeviceModel *model;
    int32_t *counters[2];  // ping-pong (V, S) pairs per label
    int4 *prev;            // per area and attempt: deltas of the previous activation
    int32_t L[3];
    int32_t na[3];         // thread areas per axis
    uint32_t n_areas;
    int32_t s;
    int32_t k;
    int32_t obstacle_type;
    uint32_t key0, key1;
    uint32_t lattice_id;
};

// Launchers (cpm_kernels.hip).  All asynchronous on `stream`.
hipError_t launch_fill_i32(int32_t *p, int32_t value, size_t n, hipStream_t stream);
hipError_t launch_count(const SweepArgs &a, int ndim, int32_t *v_out, int32_t *s_out, int stride,
                        hipStream_t stream);
hipError_t launch_activation(const SweepArgs &a, int ndim, bool act, uint32_t mcs, uint32_t alpha,
                             int parity, hipStream_t stream);
hipError_t launch_act_decay(uint8_t *act, size_t n, hipStream_t stream);
hipError_t launch_centroids(const SweepArgs &a, int ndim, int32_t n_cells, int32_t *ref,
                            int64_t *out, hipStream_t stream);
hipError_t launch_copy_counters(const int32_t *pairs, int32_t n_labels, int32_t *v_out,
                                int32_t *s_out, hipStream_t stream);

}  // namespace cpm
