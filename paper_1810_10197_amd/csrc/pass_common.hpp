// Launch shapes and small helpers shared by the 3D and 2D pass kernels.
#pragma once
#include <type_traits>

#include "fft_core.hpp"
#include "ns_internal.hpp"

namespace nsk {

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int floor_pow2(int x) { int p = 1; while (p * 2 <= x) p *= 2; return p; }

// A stage input read as FP64 (the FP64 state, or its FP32 rounding widened).
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2((double)v.x, (double)v.y); }

// Column passes: C adjacent columns per block (CW: requested width, 0 = the
// default of >= 16 columns and >= 256 threads), N/E threads per column.  A
// request of 64 columns may use up to 160 KB of LDS (one block per CU): the
// longer contiguous runs per row can outweigh the lower block count.
// LDS stride of one column's transform buffer in a column pass.  A wavefront
// holds C columns (lane % C) of 64 / C transform threads each (lane / C), and
// the transforms' exchanges step through a buffer in units of one element per
// thread.  With 16 or more columns the columns alone fill the 16 lanes that
// share an LDS cycle, and a stride of N + 1 spreads them over the banks.  With
// fewer columns, a group of 16 lanes spans 16 / C consecutive threads of each
// column: a stride congruent to 16 / C modulo 32 elements puts the columns
// 16 / C elements apart, so that the threads' unit offsets fill the gaps
// instead of landing on the next column's banks.
__host__ __device__ constexpr int col_ld(int n, int c) {
  return c >= 16 ? n + 1 : n + ((16 / c - n) % 32 + 32) % 32;
}

template <class PL, typename T, int CW = 0> struct ColCfg {
  using V = cplx<T>;
  static constexpr int N = PL::N;
  static constexpr int E = PL::E;
  static constexpr int TT = N / E;
  static constexpr int LDS_BUDGET = (CW >= 64 ? 160 : 80) * 1024;
  static constexpr int C = floor_pow2(cmin(CW > 0 ? CW : cmax(256 / TT, 16),
                                           cmin(1024 / TT, LDS_BUDGET / ((N + 1) * (int)sizeof(V)))));
  static constexpr int NT = C * TT;
  static constexpr int LD = col_ld(N, C);
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

// The retained band |k| <= K of a length-N axis in FFT order is k <= K or
// k >= N - K; the rest (the gap) is zero on input and dropped on output.  A
// register of a transform holds element c + t in thread t < TT (c fixed per
// register), so whether it meets the band is known at compile time except
// where the range straddles a band edge.  Bits: 1 low part, 2 gap, 4 high part.
enum { BAND_LO = 1, BAND_GAP = 2, BAND_HI = 4 };
__host__ __device__ constexpr int band_bits(int c, int tt, int n, int k) {
  const int a = c, b = c + tt - 1;
  const int lo = a <= k ? BAND_LO : 0;
  const int hi = b >= n - k ? BAND_HI : 0;
  const int g0 = a > k ? a : k + 1, g1 = b < n - k - 1 ? b : n - k - 1;
  return lo | hi | (g0 <= g1 ? BAND_GAP : 0);
}

// Element c + t of a transform register (in_pos: c = i TT; out_pos: c =
// TT s + r N/RL).
template <class PL> __host__ __device__ constexpr int in_base(int i) { return i * PL::TT; }
template <class PL> __host__ __device__ constexpr int out_base(int i) {
  return PL::TT * (i / PL::RL) + (i % PL::RL) * (PL::N / PL::RL);
}

// Store with the nontemporal hint (the line is not kept in the caches for
// reuse).  Used for outputs that no pass reads back soon: f of the z-forward
// pass (read by the step's final combination and reduction, after the other
// stages) and the y-inverse's slab rows (each read once, by the x-pass).
// Measured at 256^3: 3.4% off the right-hand side; the same hint on the
// outputs that the next pass reads at once (the z-inverse's, the x-pass's,
// the y-forward's and f's FP32 copy) made it slower.  At 512^3 it cost 4%
// (there the 256 MB memory-side cache holds only a small part of any pass's
// data), so st_out applies it to transforms of at most 256 points.
__device__ __forceinline__ void st_nt(float2* p, float2 v) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  f2v x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<f2v*>(p));
}
__device__ __forceinline__ void st_nt(double2* p, double2 v) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  d2v x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<d2v*>(p));
}

template <int N, typename V> __device__ __forceinline__ void st_out(V* p, V v) {
  if constexpr (N <= 256) st_nt(p, v);
  else *p = v;
}

// Load with the nontemporal hint, for the y-inverse's input (the z-inverse's
// output, read exactly once): y/x/y phase 1-3% faster at 256^3, 5% at 512^3.
// On the x-pass's, the y-forward's and the z-forward's inputs it made the
// phase slower or left it as it was.
__device__ __forceinline__ float2 ld_nt(const float2* p) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v x = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
  return make_float2(x.x, x.y);
}
__device__ __forceinline__ double2 ld_nt(const double2* p) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  const d2v x = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  return make_double2(x.x, x.y);
}

// Pointer plus a 32-bit byte offset: with a block-uniform base this maps to
// loads and stores that take the base in scalar registers and only the
// offset per lane.
template <typename P> __device__ __forceinline__ P* byte_at(P* base, unsigned off) {
  using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<C*>(base) + off);
}

template <typename V> __device__ __forceinline__ V shfl_c(V v, int src, int width) {
  return mk<V>(__shfl(v.x, src, width), __shfl(v.y, src, width));
}

}  // namespace nsk
