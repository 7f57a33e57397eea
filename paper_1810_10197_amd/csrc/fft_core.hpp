// Device building blocks for the batched real/complex FFT passes of the
// pseudo-spectral right-hand side (Sec. 2.1: the nonlinear term is formed in
// physical space and transformed back).
//
// A length-N complex DFT is done as a mixed-radix Stockham sequence of
// passes; each of the N/E threads that own one transform holds E values in
// registers, runs radix-R butterflies on them (R in {2,4,8,16}), multiplies by
// the inter-pass twiddles and exchanges through LDS between passes.  Pass p
// with radix R and span NS (product of the earlier radices) reads element
// j + r*N/R of butterfly j and writes element (j/NS)*NS*R + j%NS + r*NS; the
// output comes out in natural order.
//
// Twiddles come from a table of exp(-2 pi i m / TWN), m < TWN, computed on
// the host in double precision (std::cos/std::sin) and rounded once.  The
// radix-8/16 butterfly constants are cos/sin of multiples of pi/8, written
// from their half-angle closed forms: cos(pi/4) = sqrt(2)/2,
// cos(pi/8) = sqrt(2+sqrt(2))/2, sin(pi/8) = sqrt(2-sqrt(2))/2.
#pragma once
#include <hip/hip_runtime.h>

namespace nsk {

constexpr int TWN = 1024;   // twiddle table length; every N divides it

template <typename T> struct cx;
template <> struct cx<float> { using type = float2; };
template <> struct cx<double> { using type = double2; };
template <typename T> using cplx = typename cx<T>::type;

template <typename V> __device__ __forceinline__ V mk(decltype(V::x) a, decltype(V::x) b) {
  V r; r.x = a; r.y = b; return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return mk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return mk<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return mk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return mk<V>(a.x, -a.y); }
// multiply by s*i, s = +1 or -1
template <int S, typename V> __device__ __forceinline__ V mul_si(V a) {
  return S > 0 ? mk<V>(-a.y, a.x) : mk<V>(a.y, -a.x);
}

// cos and sin of 2*pi*k/16, k = 0..7 (closed forms above)
#define NSK_C1 0.92387953251128675613
#define NSK_C2 0.70710678118654752440
#define NSK_C3 0.38268343236508977173
__device__ __forceinline__ double cos16(int k) {
  switch (k & 15) {
    case 0: return 1.0; case 1: return NSK_C1; case 2: return NSK_C2; case 3: return NSK_C3;
    case 4: return 0.0; case 5: return -NSK_C3; case 6: return -NSK_C2; case 7: return -NSK_C1;
    case 8: return -1.0; case 9: return -NSK_C1; case 10: return -NSK_C2; case 11: return -NSK_C3;
    case 12: return 0.0; case 13: return NSK_C3; case 14: return NSK_C2; default: return NSK_C1;
  }
}
__device__ __forceinline__ double sin16(int k) { return cos16(k - 4); }

// v <- DFT_R(v) with kernel exp(DIR * 2 pi i n k / R); DIR = -1 forward.
template <int R, int DIR, typename V> struct Dft;

template <int DIR, typename V> struct Dft<2, DIR, V> {
  static __device__ __forceinline__ void run(V* v) {
    V a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  }
};

template <int DIR, typename V> struct Dft<4, DIR, V> {
  static __device__ __forceinline__ void run(V* v) {
    V a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    V a2 = cadd(v[1], v[3]), a3 = mul_si<DIR>(csub(v[1], v[3]));
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a1, a3);
    v[3] = csub(a1, a3);
  }
};

// radix 2M from two radix-M halves (even / odd samples), twiddle w_{2M}^k
template <int R, int DIR, typename V> struct DftSplit {
  static __device__ __forceinline__ void run(V* v) {
    using T = decltype(V::x);
    constexpr int M = R / 2;
    V e[M], o[M];
#pragma unroll
    for (int i = 0; i < M; ++i) { e[i] = v[2 * i]; o[i] = v[2 * i + 1]; }
    Dft<M, DIR, V>::run(e);
    Dft<M, DIR, V>::run(o);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int k16 = k * (16 / R);
      const V w = mk<V>((T)cos16(k16), (T)(DIR * sin16(k16)));
      V t = (k == 0) ? o[k] : cmul(o[k], w);
      v[k] = cadd(e[k], t);
      v[k + M] = csub(e[k], t);
    }
  }
};
template <int DIR, typename V> struct Dft<8, DIR, V> : DftSplit<8, DIR, V> {};
template <int DIR, typename V> struct Dft<16, DIR, V> : DftSplit<16, DIR, V> {};

// Radix plans: E values per thread, N/E threads per transform.
template <int N> struct Plan;
template <> struct Plan<8>    { static constexpr int E = 8,  P = 1, R0 = 8,  R1 = 1, R2 = 1; };
template <> struct Plan<16>   { static constexpr int E = 16, P = 1, R0 = 16, R1 = 1, R2 = 1; };
template <> struct Plan<32>   { static constexpr int E = 8,  P = 2, R0 = 8,  R1 = 4, R2 = 1; };
template <> struct Plan<64>   { static constexpr int E = 8,  P = 2, R0 = 8,  R1 = 8, R2 = 1; };
template <> struct Plan<128>  { static constexpr int E = 16, P = 2, R0 = 16, R1 = 8, R2 = 1; };
template <> struct Plan<256>  { static constexpr int E = 16, P = 2, R0 = 16, R1 = 16, R2 = 1; };
template <> struct Plan<512>  { static constexpr int E = 8,  P = 3, R0 = 8,  R1 = 8, R2 = 8; };
template <> struct Plan<1024> { static constexpr int E = 16, P = 3, R0 = 16, R1 = 16, R2 = 4; };

// Butterflies of one pass on the thread's registers: radix R, span NS.
template <int N, int E, int R, int NS, int DIR, typename V>
__device__ __forceinline__ void pass_compute(V (&v)[E], int t, const V* __restrict__ tw) {
  constexpr int TT = N / E;
  constexpr int S = E / R;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if constexpr (NS > 1) {
      const int j = t + TT * s;
      const int jm = j & (NS - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        V w = tw[(jm * r * (N / (NS * R))) * (TWN / N)];
        if constexpr (DIR > 0) w.y = -w.y;
        v[s * R + r] = cmul(v[s * R + r], w);
      }
    }
    Dft<R, DIR, V>::run(&v[s * R]);
  }
}

// Write a pass's outputs to a transform buffer (unit element stride).
template <int N, int E, int R, int NS, typename V>
__device__ __forceinline__ void pass_write(const V (&v)[E], int t, V* buf) {
  constexpr int TT = N / E;
  constexpr int S = E / R;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = t + TT * s;
    const int base = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
    for (int r = 0; r < R; ++r) buf[base + r * NS] = v[s * R + r];
  }
}

// Read the inputs of a pass with radix R from a transform buffer.
template <int N, int E, int R, typename V>
__device__ __forceinline__ void pass_read(V (&v)[E], int t, const V* buf) {
  constexpr int TT = N / E;
  constexpr int S = E / R;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = t + TT * s;
#pragma unroll
    for (int r = 0; r < R; ++r) v[s * R + r] = buf[j + r * (N / R)];
  }
}

// Element index held in v[i] after the last pass (natural order output).
template <int N> __device__ __forceinline__ int out_pos(int t, int i) {
  using P = Plan<N>;
  constexpr int RL = P::P == 1 ? P::R0 : (P::P == 2 ? P::R1 : P::R2);
  constexpr int TT = N / P::E;
  const int s = i / RL, r = i % RL;
  return t + TT * s + r * (N / RL);
}
// Element index expected in v[i] before the first pass (R0 == E for all plans).
template <int N> __device__ __forceinline__ int in_pos(int t, int i) {
  constexpr int TT = N / Plan<N>::E;
  return t + i * TT;
}

// Whole transform on registers: v holds the inputs at in_pos on entry and the
// outputs at out_pos on exit.  buf is this transform's LDS scratch (N values);
// every thread of the block must call this (it synchronises the block).
template <int N, int DIR, typename V>
__device__ __forceinline__ void fft_regs(V (&v)[Plan<N>::E], int t, V* buf, const V* __restrict__ tw) {
  using P = Plan<N>;
  constexpr int E = P::E;
  pass_compute<N, E, P::R0, 1, DIR>(v, t, tw);
  if constexpr (P::P >= 2) {
    pass_write<N, E, P::R0, 1>(v, t, buf);
    __syncthreads();
    pass_read<N, E, P::R1>(v, t, buf);
    pass_compute<N, E, P::R1, P::R0, DIR>(v, t, tw);
  }
  if constexpr (P::P >= 3) {
    __syncthreads();
    pass_write<N, E, P::R1, P::R0>(v, t, buf);
    __syncthreads();
    pass_read<N, E, P::R2>(v, t, buf);
    pass_compute<N, E, P::R2, P::R0 * P::R1, DIR>(v, t, tw);
  }
}

// Transform held entirely in an LDS buffer (natural order in and out).
// active == false threads only take part in the barriers.
template <int N, int DIR, typename V>
__device__ __forceinline__ void fft_lds(V* buf, int t, bool active, const V* __restrict__ tw) {
  using P = Plan<N>;
  constexpr int E = P::E;
  V v[E];
  if (active) pass_read<N, E, P::R0>(v, t, buf);
  if (active) pass_compute<N, E, P::R0, 1, DIR>(v, t, tw);
  __syncthreads();
  if (active) pass_write<N, E, P::R0, 1>(v, t, buf);
  __syncthreads();
  if constexpr (P::P >= 2) {
    if (active) {
      pass_read<N, E, P::R1>(v, t, buf);
      pass_compute<N, E, P::R1, P::R0, DIR>(v, t, tw);
    }
    __syncthreads();
    if (active) pass_write<N, E, P::R1, P::R0>(v, t, buf);
    __syncthreads();
  }
  if constexpr (P::P >= 3) {
    if (active) {
      pass_read<N, E, P::R2>(v, t, buf);
      pass_compute<N, E, P::R2, P::R0 * P::R1, DIR>(v, t, tw);
    }
    __syncthreads();
    if (active) pass_write<N, E, P::R2, P::R0 * P::R1>(v, t, buf);
    __syncthreads();
  }
}

}  // namespace nsk
