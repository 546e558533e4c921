// One search variant per translation unit, so that the variants compile in
// parallel: BANG_VARIANT = host-resident adjacency (bit 0) | visited filter
// << 1 (bits 1-2: none, Bloom, seen bitmap) | timed (bit 3, per-phase
// cycles), instantiated for every compiled (dtype, m, d/m) and table form.
#include "search_kernel.h"

#ifndef BANG_VARIANT
#error "compile with -DBANG_VARIANT=<host | filter << 1 | timed << 3>"
#endif

namespace bang {

namespace {

constexpr bool kHostV = (BANG_VARIANT & 1) != 0;
constexpr int kFiltV = (BANG_VARIANT >> 1) & 3;  // the filter
constexpr bool kPhasesV = (BANG_VARIANT & 8) != 0;
static_assert(kFiltV <= kFiltSeen, "unknown filter");

template <int DT, int M, int DS>
struct Launch {
  static hipError_t run(const SearchArgs& a, int table, uint32_t grid,
                        size_t lds, hipStream_t s) {
    switch (table) {
      case kTabF32:
        hipLaunchKernelGGL((search_kernel<DT, M, DS, kTabF32, kHostV, kFiltV, kPhasesV>),
                           dim3(grid), dim3(kWave), lds, s, a);
        break;
      case kTabF16:
        hipLaunchKernelGGL((search_kernel<DT, M, DS, kTabF16, kHostV, kFiltV, kPhasesV>),
                           dim3(grid), dim3(kWave), lds, s, a);
        break;
      case kTabU8:
        hipLaunchKernelGGL((search_kernel<DT, M, DS, kTabU8, kHostV, kFiltV, kPhasesV>),
                           dim3(grid), dim3(kWave), lds, s, a);
        break;
      case kTabExact:
        hipLaunchKernelGGL(
            (search_kernel<DT, M, DS, kTabExact, kHostV, kFiltV, kPhasesV>), dim3(grid),
            dim3(kWave), lds, s, a);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
};

template <int DT, int M, int DS>
struct Occupancy {
  static hipError_t run(int table, size_t lds, int* per_cu) {
    switch (table) {
      case kTabF32:
        return occupancy_of(search_kernel<DT, M, DS, kTabF32, kHostV, kFiltV, kPhasesV>,
                            lds, per_cu);
      case kTabF16:
        return occupancy_of(search_kernel<DT, M, DS, kTabF16, kHostV, kFiltV, kPhasesV>,
                            lds, per_cu);
      case kTabU8:
        return occupancy_of(search_kernel<DT, M, DS, kTabU8, kHostV, kFiltV, kPhasesV>,
                            lds, per_cu);
      case kTabExact:
        return occupancy_of(
            search_kernel<DT, M, DS, kTabExact, kHostV, kFiltV, kPhasesV>, lds, per_cu);
    }
    return hipErrorInvalidValue;
  }
};

}  // namespace

#define BANG_CAT2(a, b) a##b
#define BANG_CAT(a, b) BANG_CAT2(a, b)

hipError_t BANG_CAT(search_launch_v, BANG_VARIANT)(const SearchArgs& a,
                                                   int dt, uint32_t m,
                                                   uint32_t ds, int table,
                                                   uint32_t grid, size_t lds,
                                                   hipStream_t s) {
  return dispatch<Launch>(dt, m, ds, a, table, grid, lds, s);
}

hipError_t BANG_CAT(search_occupancy_v, BANG_VARIANT)(int dt, uint32_t m,
                                                      uint32_t ds, int table,
                                                      size_t lds,
                                                      int* per_cu) {
  return dispatch<Occupancy>(dt, m, ds, table, lds, per_cu);
}

}  // namespace bang
