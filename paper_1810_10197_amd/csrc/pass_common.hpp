// Launch shapes and small helpers shared by the 3D and 2D pass kernels.
#pragma once
#include "fft_core.hpp"
#include "ns_internal.hpp"

namespace nsk {

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int floor_pow2(int x) { int p = 1; while (p * 2 <= x) p *= 2; return p; }

// Column passes: C adjacent columns per block (CW: requested width, 0 = the
// default of >= 16 columns and >= 256 threads), N/E threads per column.
template <class PL, typename T, int CW = 0> struct ColCfg {
  using V = cplx<T>;
  static constexpr int N = PL::N;
  static constexpr int E = PL::E;
  static constexpr int TT = N / E;
  static constexpr int LDS_BUDGET = 80 * 1024;
  static constexpr int C = floor_pow2(cmin(CW > 0 ? CW : cmax(256 / TT, 16),
                                           cmin(1024 / TT, LDS_BUDGET / ((N + 1) * (int)sizeof(V)))));
  static constexpr int NT = C * TT;
  static constexpr int LD = N + 1;      // padded LDS stride per column
};

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8, each with its own L2).  With a grid padded to a multiple of 8 this
// remap hands each XCD a contiguous range of logical block ids, so blocks
// with neighbouring logical ids share an L2.
__device__ __forceinline__ long long xcd_logical(long long b, long long nb_padded) {
  return (b & 7) * (nb_padded >> 3) + (b >> 3);
}

// Row pass: N/E threads per row (inside one wavefront), RPB rows per block,
// each row's transform buffer padded against LDS bank conflicts.
template <class PL, typename T> struct RowCfg {
  static constexpr int N = PL::N;
  static constexpr int E = PL::E;
  static constexpr int TT = N / E;
  static constexpr int RPB = 256 / TT;              // rows per block
  static constexpr int LD = LdsLen<N, true>::value;
  static constexpr int NT = RPB * TT;
};

template <typename V> __device__ __forceinline__ V shfl_c(V v, int src, int width) {
  return mk<V>(__shfl(v.x, src, width), __shfl(v.y, src, width));
}

}  // namespace nsk
