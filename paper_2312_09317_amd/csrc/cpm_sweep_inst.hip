// Instantiations of the activation kernels, one group per compilation of
// this file (CPM_SWEEP_PART = 0..6) so that the groups build in parallel.
#include "cpm_sweep_kernels.hpp"

#ifndef CPM_SWEEP_PART
#error "compile with -DCPM_SWEEP_PART=<0..6>"
#endif

namespace cpm {

#define CPM_SWEEP(CELL, D)                                                                                        \
    template hipError_t sweep_words<CELL, D>(const SweepArgs &, bool, uint32_t, uint32_t, int, size_t, hipStream_t);
#define CPM_BATCH(CELL, D)                                                                                        \
    template hipError_t batch_words<CELL, D>(const BatchLaunch &, uint32_t, int, hipStream_t);                  \
    template hipError_t batch_persistent_words<CELL, D>(const BatchLaunch &, const PersistentLaunch &, hipStream_t);

#if CPM_SWEEP_PART == 0
CPM_SWEEP(int32_t, 2)
CPM_BATCH(int32_t, 2)
#elif CPM_SWEEP_PART == 1
CPM_SWEEP(int32_t, 3)
CPM_BATCH(int32_t, 3)
#elif CPM_SWEEP_PART == 2
CPM_SWEEP(uint16_t, 2)
CPM_BATCH(uint16_t, 2)
#elif CPM_SWEEP_PART == 3
CPM_SWEEP(uint16_t, 3)
CPM_BATCH(uint16_t, 3)
#elif CPM_SWEEP_PART == 4
CPM_SWEEP(uint32_t, 2)
CPM_SWEEP(uint32_t, 3)
#elif CPM_SWEEP_PART == 5
CPM_SWEEP(char32_t, 2)
CPM_SWEEP(char32_t, 3)
#elif CPM_SWEEP_PART == 6
CPM_BATCH(char32_t, 2)
CPM_BATCH(char32_t, 3)
CPM_BATCH(char16_t, 2)
CPM_BATCH(char16_t, 3)
#endif

}  // namespace cpm
