// 2D right-hand sides (plain Navier--Stokes and the Boussinesq system of
// Sec. 3.2): not built yet.
#include "ns_internal.hpp"

namespace nsk {

size_t rhs2d_scratch_bytes(const Geom&, int) { return 0; }

hipError_t rhs2d_compact(const Geom&, int, const double2*, double2*, const RhsParams&,
                         const RhsBufs&, const void*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace nsk
