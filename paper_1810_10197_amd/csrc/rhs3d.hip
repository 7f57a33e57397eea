// Host side of the 3D right-hand side: the slab schedule and the dispatch
// over grid sizes.  The kernels are in rhs3d_kernels.hpp; the zero-padded
// grids of the 3/2 rule (n = 3 * 2^k) are instantiated in rhs3d_pad.hip, a
// translation unit of their own so that both compile in parallel.
#include "rhs3d_kernels.hpp"

namespace nsk {

template <typename T, typename UT>
hipError_t dispatch3d_padded(const Geom& g, const UT* U, double2* K, const RhsParams& p,
                             const RhsBufs& b, const void* tw, hipStream_t st);

bool slab_two_streams(int v) { return (v >= 5 && v < 9) || v >= 11; }

int slab_planes(const Geom& g, int v) {
  const int sh = v < 0 ? 0 : (v < 5 ? v : (v < 9 ? v - 4 : (v < 11 ? v - 4 : v - 6)));
  const int zs = g.n >> sh;
  return zs < 1 ? 1 : zs;
}

int default_slab_variant(const Geom& g, int fp64) {
  const size_t per_plane = (size_t)g.batch * 9 * g.n * g.Kx * (fp64 ? 16 : 8);
  int v = 0;
  while (v < 4 && (size_t)slab_planes(g, v) * per_plane > ((size_t)96 << 20)) ++v;
  return v;
}

template <typename T, typename UT>
static hipError_t dispatch3d(const Geom& g, const UT* U, double2* K, const RhsParams& p,
                             const RhsBufs& b, const void* tw, hipStream_t st) {
  switch (g.n) {
    case 8: return run3d<8, T, UT>(g, U, K, p, b, tw, st);
    case 16: return run3d<16, T, UT>(g, U, K, p, b, tw, st);
    case 32: return run3d<32, T, UT>(g, U, K, p, b, tw, st);
    case 64: return run3d<64, T, UT>(g, U, K, p, b, tw, st);
    case 128: return run3d<128, T, UT>(g, U, K, p, b, tw, st);
    case 256: return run3d<256, T, UT>(g, U, K, p, b, tw, st);
    case 512: return run3d<512, T, UT>(g, U, K, p, b, tw, st);
    case 1024: return run3d<1024, T, UT>(g, U, K, p, b, tw, st);
    default: return dispatch3d_padded<T, UT>(g, U, K, p, b, tw, st);
  }
}

hipError_t rhs3d_compact(const Geom& g, int fp64, const double2* U, const float2* U32, double2* K,
                         const RhsParams& p, const RhsBufs& b, const void* tw, hipStream_t st) {
  if (fp64) return dispatch3d<double, double2>(g, U, K, p, b, tw, st);
  if (U32) return dispatch3d<float, float2>(g, U32, K, p, b, tw, st);
  return dispatch3d<float, double2>(g, U, K, p, b, tw, st);
}

size_t rhs3d_scratch_bytes(const Geom& g, int fp64) { return scratch3d(g, fp64).total; }

}  // namespace nsk
