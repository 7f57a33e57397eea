// The 3D right-hand side on the zero-padded grids of the 3/2 rule (Sec.
// 2.1.1): n = 3 * 2^k points per direction carry the products of an N = 2n/3
// grid's modes |k_j| <= N/2 - 1.  With K = (n - 1)/3 = N/2 - 1 these are the
// same kernels as on the power-of-two grids (their FFTs take a radix-24
// first pass).
#include "rhs3d_kernels.hpp"

namespace nsk {

template <typename T, typename UT>
hipError_t dispatch3d_padded(const Geom& g, const UT* U, double2* K, const RhsParams& p,
                             const RhsBufs& b, const void* tw, hipStream_t st) {
  switch (g.n) {
    case 24: return run3d<24, T, UT>(g, U, K, p, b, tw, st);
    case 48: return run3d<48, T, UT>(g, U, K, p, b, tw, st);
    case 96: return run3d<96, T, UT>(g, U, K, p, b, tw, st);
    case 192: return run3d<192, T, UT>(g, U, K, p, b, tw, st);
    case 384: return run3d<384, T, UT>(g, U, K, p, b, tw, st);
    case 768: return run3d<768, T, UT>(g, U, K, p, b, tw, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t dispatch3d_padded<double, double2>(const Geom&, const double2*, double2*, const RhsParams&,
                                                       const RhsBufs&, const void*, hipStream_t);
template hipError_t dispatch3d_padded<float, float2>(const Geom&, const float2*, double2*, const RhsParams&,
                                                     const RhsBufs&, const void*, hipStream_t);
template hipError_t dispatch3d_padded<float, double2>(const Geom&, const double2*, double2*, const RhsParams&,
                                                      const RhsBufs&, const void*, hipStream_t);

}  // namespace nsk
