// Host side of the 2D right-hand side: dispatch over grid sizes.  The
// kernels are in rhs2d_kernels.hpp; the zero-padded grids of the 3/2 rule
// (n = 3 * 2^k) are instantiated in rhs2d_pad.hip.
#include "rhs2d_kernels.hpp"

namespace nsk {

template <typename T, bool SCALAR>
hipError_t dispatch2d_padded(const Geom& g, const double2* U, const float2* U32, double2* K, const RhsParams& p,
                             const RhsBufs& b, const void* tw, hipStream_t st);

template <typename T, bool SCALAR>
static hipError_t dispatch2d(const Geom& g, const double2* U, const float2* U32, double2* K, const RhsParams& p,
                             const RhsBufs& b, const void* tw, hipStream_t st) {
  switch (g.n) {
    case 8: return run2d<8, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 16: return run2d<16, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 32: return run2d<32, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 64: return run2d<64, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 128: return run2d<128, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 256: return run2d<256, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 512: return run2d<512, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    case 1024: return run2d<1024, T, SCALAR>(g, U, U32, K, p, b, tw, st);
    default: return dispatch2d_padded<T, SCALAR>(g, U, U32, K, p, b, tw, st);
  }
}

hipError_t rhs2d_compact(const Geom& g, int fp64, const double2* U, const float2* U32, double2* K,
                         const RhsParams& p, const RhsBufs& b, const void* tw, hipStream_t st) {
  const bool sc = g.ncomp == 3;
  if (fp64) {
    if (U32) return hipErrorInvalidValue;
    return sc ? dispatch2d<double, true>(g, U, nullptr, K, p, b, tw, st)
              : dispatch2d<double, false>(g, U, nullptr, K, p, b, tw, st);
  }
  return sc ? dispatch2d<float, true>(g, U, U32, K, p, b, tw, st) : dispatch2d<float, false>(g, U, U32, K, p, b, tw, st);
}

size_t rhs2d_scratch_bytes(const Geom& g, int fp64) {
  const size_t cb = fp64 ? 16 : 8;
  return 2 * (size_t)g.batch * 4 * g.n * g.Kx * cb;      // B1 and B2
}

}  // namespace nsk
