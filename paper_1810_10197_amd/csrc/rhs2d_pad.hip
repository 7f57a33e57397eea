// The 2D right-hand side on the zero-padded grids of the 3/2 rule (Sec.
// 2.1.1): n = 3 * 2^k points per direction carry the products of an N = 2n/3
// grid's modes |k_j| <= N/2 - 1 = (n - 1)/3, with the kernels of the
// power-of-two grids.
#include "rhs2d_kernels.hpp"

namespace nsk {

template <typename T, bool SCALAR>
hipError_t dispatch2d_padded(const Geom& g, const double2* U, const float2* U32, double2* K, const RhsParams& p,
                             const RhsBufs& b, const void* tw, hipStream_t st) {
  switch (g.n) {
    case 24: return run2d<24, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 48: return run2d<48, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 96: return run2d<96, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 192: return run2d<192, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 384: return run2d<384, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 768: return run2d<768, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 1536: return run2d<1536, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t dispatch2d_padded<double, true>(const Geom&, const double2*, const float2*, double2*, const RhsParams&,
                                                    const RhsBufs&, const void*, hipStream_t);
template hipError_t dispatch2d_padded<double, false>(const Geom&, const double2*, const float2*, double2*, const RhsParams&,
                                                     const RhsBufs&, const void*, hipStream_t);
template hipError_t dispatch2d_padded<float, true>(const Geom&, const double2*, const float2*, double2*, const RhsParams&,
                                                   const RhsBufs&, const void*, hipStream_t);
template hipError_t dispatch2d_padded<float, false>(const Geom&, const double2*, const float2*, double2*, const RhsParams&,
                                                    const RhsBufs&, const void*, hipStream_t);

}  // namespace nsk
