// Device building blocks for the batched real/complex FFT passes of the
// pseudo-spectral right-hand side (Sec. 2.1: the nonlinear term is formed in
// physical space and transformed back).
//
// A length-N complex DFT is done as a mixed-radix Stockham sequence of up to
// four passes; each of the N/E threads that own one transform holds E values
// in registers, runs radix-R butterflies on them (the first pass R = E in
// {8, 12, 16, 24}, later passes R in {2, 4, 8, 16}), multiplies by the
// inter-pass twiddles and exchanges through LDS between passes.  Pass p with
// radix R and span NS (product of the earlier radices) reads element
// j + r*N/R of butterfly j and writes element (j/NS)*NS*R + j%NS + r*NS; the
// output comes out in natural order.
//
// Lengths are 2^k, or 3 * 2^k with a radix-24 (3 x 8) or radix-12 (3 x 4)
// first pass.  Twiddles come from a table of exp(-2 pi i m / TWN), m < TWN,
// computed on the host in double precision (std::cos/std::sin) and rounded
// once; a pass with radix R loads log2(R) entries per butterfly and
// multiplies them together for the rest (see Tw below).  The radix-8/16
// butterfly constants are cos/sin of multiples of pi/8, written from their
// half-angle closed forms: cos(pi/4) = sqrt(2)/2, cos(pi/8) =
// sqrt(2+sqrt(2))/2, sin(pi/8) = sqrt(2-sqrt(2))/2; those of the radix-3/12/24
// butterflies are multiples of 15 degrees (below).
#pragma once
#include <hip/hip_runtime.h>

namespace nsk {

constexpr int TWN = 3072;   // twiddle table length; every N (2^k and 3 * 2^k) divides it

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
      const int k16 = k * (16 / R);     // twiddle angle in units of 2 pi / 16
      V t;
      if (k16 == 0) {
        t = o[k];
      } else if (k16 == 4) {            // exp(DIR i pi/2) = DIR i
        t = mul_si<DIR>(o[k]);
      } else if (k16 == 2 || k16 == 6) {
        // w = c (1 + DIR i) or c (-1 + DIR i), c = cos(pi/4): two products
        const T c = (T)NSK_C2, x = o[k].x, y = o[k].y;
        if (k16 == 2)
          t = DIR > 0 ? mk<V>(c * (x - y), c * (x + y)) : mk<V>(c * (x + y), c * (y - x));
        else
          t = DIR > 0 ? mk<V>(-(c * (x + y)), c * (x - y)) : mk<V>(c * (y - x), -(c * (x + y)));
      } else {
        const V w = mk<V>((T)cos16(k16), (T)(DIR * sin16(k16)));
        t = cmul(o[k], w);
      }
      v[k] = cadd(e[k], t);
      v[k + M] = csub(e[k], t);
    }
  }
};
template <int DIR, typename V> struct Dft<8, DIR, V> : DftSplit<8, DIR, V> {};
template <int DIR, typename V> struct Dft<16, DIR, V> : DftSplit<16, DIR, V> {};

// sqrt(3)/2 = sin(pi/3); cos and sin of multiples of 2 pi / 24 (15 degrees)
// from the closed forms cos(pi/12) = (sqrt 6 + sqrt 2)/4, sin(pi/12) =
// (sqrt 6 - sqrt 2)/4, cos(pi/6) = sqrt(3)/2, cos(pi/4) = sqrt(2)/2.
#define NSK_S3 0.86602540378443864676
#define NSK_C15 0.96592582628906828675
#define NSK_S15 0.25881904510252076235
__device__ __forceinline__ double cos24(int k) {
  switch (((k % 24) + 24) % 24) {
    case 0: return 1.0; case 1: return NSK_C15; case 2: return NSK_S3; case 3: return NSK_C2;
    case 4: return 0.5; case 5: return NSK_S15; case 6: return 0.0; case 7: return -NSK_S15;
    case 8: return -0.5; case 9: return -NSK_C2; case 10: return -NSK_S3; case 11: return -NSK_C15;
    case 12: return -1.0; case 13: return -NSK_C15; case 14: return -NSK_S3; case 15: return -NSK_C2;
    case 16: return -0.5; case 17: return -NSK_S15; case 18: return 0.0; case 19: return NSK_S15;
    case 20: return 0.5; case 21: return NSK_C2; case 22: return NSK_S3; default: return NSK_C15;
  }
}
__device__ __forceinline__ double sin24(int k) { return cos24(k - 6); }

// 3-point DFT: X1,2 = a - (b + c)/2 +- DIR i (sqrt(3)/2) (b - c).
template <int DIR, typename V> struct Dft<3, DIR, V> {
  static __device__ __forceinline__ void run(V* v) {
    using T = decltype(V::x);
    const T h = (T)0.5, r3 = (T)NSK_S3;
    const V a = v[0], t1 = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const V t2 = mk<V>(a.x - h * t1.x, a.y - h * t1.y);
    const V t3 = mul_si<DIR>(mk<V>(r3 * d.x, r3 * d.y));
    v[0] = cadd(a, t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  }
};

// 3M-point DFT (M = 4 or 8) as 3 x M: with n = n1 + 3 n2 and k = M k1 + k2,
// M-point transforms over n2 for each n1, the twiddles w_3M^(n1 k2), then
// three-point transforms over n1 for each k2.
template <int M, int DIR, typename V> struct Dft3xM {
  static __device__ __forceinline__ void run(V* v) {
    using T = decltype(V::x);
    constexpr int U = 8 / M;                    // w_3M = w_24^U
    V y[3][M];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
#pragma unroll
      for (int n2 = 0; n2 < M; ++n2) y[n1][n2] = v[n1 + 3 * n2];
      Dft<M, DIR, V>::run(y[n1]);
    }
#pragma unroll
    for (int n1 = 1; n1 < 3; ++n1) {
#pragma unroll
      for (int k2 = 1; k2 < M; ++k2) {
        const int m = n1 * k2 * U;
        const V w = mk<V>((T)cos24(m), (T)(DIR * sin24(m)));
        y[n1][k2] = cmul(y[n1][k2], w);
      }
    }
#pragma unroll
    for (int k2 = 0; k2 < M; ++k2) {
      V z[3] = {y[0][k2], y[1][k2], y[2][k2]};
      Dft<3, DIR, V>::run(z);
#pragma unroll
      for (int k1 = 0; k1 < 3; ++k1) v[M * k1 + k2] = z[k1];
    }
  }
};
template <int DIR, typename V> struct Dft<12, DIR, V> : Dft3xM<4, DIR, V> {};
template <int DIR, typename V> struct Dft<24, DIR, V> : Dft3xM<8, DIR, V> {};

// Radix plans: a transform of length N in P passes of radices R0, R1, R2, R3
// (R0 = E, the values each thread holds; N/E threads per transform).
template <int N_, int E_, int P_, int R0_, int R1_, int R2_, int R3_ = 1> struct PlanT {
  static constexpr int N = N_, E = E_, P = P_, R0 = R0_, R1 = R1_, R2 = R2_, R3 = R3_;
  static constexpr int TT = N / E;
  static constexpr int RL = P == 1 ? R0 : (P == 2 ? R1 : (P == 3 ? R2 : R3));   // last radix
  static_assert(R0 * R1 * R2 * R3 == N && R0 == E, "radix plan");
  static_assert((R1 & (R1 - 1)) == 0 && (R2 & (R2 - 1)) == 0 && (R3 & (R3 - 1)) == 0,
                "later passes have power-of-two radices");
  static_assert(E % R1 == 0 && E % R2 == 0 && E % R3 == 0, "whole butterflies per thread");
};
// Wide plans: few passes, up to 16 values per thread.
template <int N> struct Plan;
template <> struct Plan<8>    : PlanT<8, 8, 1, 8, 1, 1> {};
template <> struct Plan<16>   : PlanT<16, 16, 1, 16, 1, 1> {};
template <> struct Plan<32>   : PlanT<32, 8, 2, 8, 4, 1> {};
template <> struct Plan<64>   : PlanT<64, 8, 2, 8, 8, 1> {};
template <> struct Plan<128>  : PlanT<128, 16, 2, 16, 8, 1> {};
template <> struct Plan<256>  : PlanT<256, 16, 2, 16, 16, 1> {};
template <> struct Plan<512>  : PlanT<512, 8, 3, 8, 8, 8> {};
template <> struct Plan<1024> : PlanT<1024, 16, 3, 16, 16, 4> {};
// 3 * 2^k (the 3/2-padded grids of n = 2^(k+1)): a radix-24 first pass.
template <> struct Plan<24>   : PlanT<24, 24, 1, 24, 1, 1> {};
template <> struct Plan<48>   : PlanT<48, 24, 2, 24, 2, 1> {};
template <> struct Plan<96>   : PlanT<96, 24, 2, 24, 4, 1> {};
template <> struct Plan<192>  : PlanT<192, 24, 2, 24, 8, 1> {};
template <> struct Plan<384>  : PlanT<384, 24, 3, 24, 8, 2> {};
template <> struct Plan<768>  : PlanT<768, 24, 3, 24, 8, 4> {};
template <> struct Plan<1536> : PlanT<1536, 24, 3, 24, 8, 8> {};
// Narrow plans: at most 8 values per thread (fewer registers, one more pass).
template <int N> struct PlanS;
template <> struct PlanS<8>    : PlanT<8, 8, 1, 8, 1, 1> {};
template <> struct PlanS<16>   : PlanT<16, 8, 2, 8, 2, 1> {};
template <> struct PlanS<32>   : PlanT<32, 8, 2, 8, 4, 1> {};
template <> struct PlanS<64>   : PlanT<64, 8, 2, 8, 8, 1> {};
template <> struct PlanS<128>  : PlanT<128, 8, 3, 8, 8, 2> {};
template <> struct PlanS<256>  : PlanT<256, 8, 3, 8, 8, 4> {};
template <> struct PlanS<512>  : PlanT<512, 8, 3, 8, 8, 8> {};
template <> struct PlanS<1024> : PlanT<1024, 8, 4, 8, 8, 8, 2> {};
// 3 * 2^k: a radix-12 (3 x 4) first pass, 12 values per thread.
template <> struct PlanS<24>   : PlanT<24, 12, 2, 12, 2, 1> {};
template <> struct PlanS<48>   : PlanT<48, 12, 2, 12, 4, 1> {};
template <> struct PlanS<96>   : PlanT<96, 12, 3, 12, 4, 2> {};
template <> struct PlanS<192>  : PlanT<192, 12, 3, 12, 4, 4> {};
template <> struct PlanS<384>  : PlanT<384, 12, 4, 12, 4, 4, 2> {};
template <> struct PlanS<768>  : PlanT<768, 12, 4, 12, 4, 4, 4> {};
template <> struct PlanS<1536> : Plan<1536> {};      // 12 x 128 would need five passes

// log2 and highest set bit for 1 <= x < 32, written without recursion so that
// they fold to constants inside unrolled loops.
__host__ __device__ constexpr int ilog2(int x) {
  return x >= 16 ? 4 : (x >= 8 ? 3 : (x >= 4 ? 2 : (x >= 2 ? 1 : 0)));
}
__host__ __device__ constexpr int highbit(int x) {
  return x >= 16 ? 16 : (x >= 8 ? 8 : (x >= 4 ? 4 : (x >= 2 ? 2 : x)));
}

// Twiddles of the passes after the first.  Pass p (radix R, span NS) scales
// input r of butterfly j by b^r, b = w_N^(jm N / (NS R)), jm = j mod NS.  A
// thread loads only the bases b^(2^q), q < log2 R, of each of its butterflies
// (one table entry each, loaded once at the start of the transform, before
// any exchange, so that their latency overlaps the first pass) and forms the
// other powers as products of at most log2(R) - 1 of them.
template <class P, typename V> struct Tw {
  static constexpr int S1 = P::P >= 2 ? P::E / P::R1 : 1, L1 = P::P >= 2 ? ilog2(P::R1) : 1;
  static constexpr int S2 = P::P >= 3 ? P::E / P::R2 : 1, L2 = P::P >= 3 ? ilog2(P::R2) : 1;
  static constexpr int S3 = P::P >= 4 ? P::E / P::R3 : 1, L3 = P::P >= 4 ? ilog2(P::R3) : 1;
  V b1[S1][L1];
  V b2[S2][L2];
  V b3[S3][L3];
};

template <class P, typename V>
__device__ __forceinline__ void tw_load(Tw<P, V>& w, int t, const V* __restrict__ tab) {
  constexpr int N = P::N, TT = P::TT;
  if constexpr (P::P >= 2) {
    constexpr int R = P::R1, NS = P::R0;
#pragma unroll
    for (int s = 0; s < Tw<P, V>::S1; ++s) {
      const int e = ((t + TT * s) % NS) * (N / (NS * R));
#pragma unroll
      for (int q = 0; q < Tw<P, V>::L1; ++q) w.b1[s][q] = tab[(e << q) * (TWN / N)];
    }
  }
  if constexpr (P::P >= 3) {
    constexpr int R = P::R2, NS = P::R0 * P::R1;
#pragma unroll
    for (int s = 0; s < Tw<P, V>::S2; ++s) {
      const int e = ((t + TT * s) % NS) * (N / (NS * R));
#pragma unroll
      for (int q = 0; q < Tw<P, V>::L2; ++q) w.b2[s][q] = tab[(e << q) * (TWN / N)];
    }
  }
  if constexpr (P::P >= 4) {
    constexpr int R = P::R3, NS = P::R0 * P::R1 * P::R2;
#pragma unroll
    for (int s = 0; s < Tw<P, V>::S3; ++s) {
      const int e = ((t + TT * s) % NS) * (N / (NS * R));
#pragma unroll
      for (int q = 0; q < Tw<P, V>::L3; ++q) w.b3[s][q] = tab[(e << q) * (TWN / N)];
    }
  }
}

// v[r] *= b^r (DIR > 0: conj(b)^r), r = 1..R-1, from the bases b^(2^q).
template <int R, int DIR, typename V, int L>
__device__ __forceinline__ void twiddle_mul(V* v, const V (&b)[L]) {
  V w[R];
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const int hb = highbit(r);
    w[r] = r == hb ? b[ilog2(r)] : cmul(w[hb], w[r - hb]);
    const V x = v[r], c = w[r];
    v[r] = DIR > 0 ? mk<V>(x.x * c.x + x.y * c.y, x.y * c.x - x.x * c.y) : cmul(x, c);
  }
}

// Butterflies of one pass on the thread's registers: radix R, twiddle bases b
// (one set per butterfly; none for the first pass).
template <int E, int R, int DIR, typename V>
__device__ __forceinline__ void pass_first(V (&v)[E]) {
#pragma unroll
  for (int s = 0; s < E / R; ++s) Dft<R, DIR, V>::run(&v[s * R]);
}
template <int E, int R, int DIR, typename V, int S, int L>
__device__ __forceinline__ void pass_tw(V (&v)[E], const V (&b)[S][L]) {
  static_assert(S == E / R, "one twiddle set per butterfly");
#pragma unroll
  for (int s = 0; s < S; ++s) {
    twiddle_mul<R, DIR>(&v[s * R], b[s]);
    Dft<R, DIR, V>::run(&v[s * R]);
  }
}

// LDS slot of element pos: with PAD one spare slot follows every 16
// elements, so that threads writing pos = 16 t + r (a radix-16 pass with
// unit span) hit distinct banks.  A padded buffer holds N + N/16 values.
template <bool PAD> __device__ __forceinline__ int lslot(int pos) { return PAD ? pos + (pos >> 4) : pos; }
template <int N, bool PAD> struct LdsLen { static constexpr int value = PAD ? N + N / 16 : N; };

// Write a pass's outputs to a transform buffer (unit element stride).
template <int N, int E, int R, int NS, typename V, bool PAD = false>
__device__ __forceinline__ void pass_write(const V (&v)[E], int t, V* buf) {
  constexpr int TT = N / E;
  constexpr int S = E / R;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = t + TT * s;
    const int base = (j / NS) * NS * R + j % NS;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[lslot<PAD>(base + r * NS)] = v[s * R + r];
  }
}

// Read the inputs of a pass with radix R from a transform buffer.
template <int N, int E, int R, typename V, bool PAD = false>
__device__ __forceinline__ void pass_read(V (&v)[E], int t, const V* buf) {
  constexpr int TT = N / E;
  constexpr int S = E / R;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = t + TT * s;
#pragma unroll
    for (int r = 0; r < R; ++r) v[s * R + r] = buf[lslot<PAD>(j + r * (N / R))];
  }
}

// Element index held in v[i] after the last pass (natural order output).
template <class PL> __device__ __forceinline__ int out_pos(int t, int i) {
  const int s = i / PL::RL, r = i % PL::RL;
  return t + PL::TT * s + r * (PL::N / PL::RL);
}
// Element index expected in v[i] before the first pass (R0 == E for all plans).
template <class PL> __device__ __forceinline__ int in_pos(int t, int i) { return t + i * PL::TT; }

// Synchronisation of the threads sharing a transform buffer: the whole block,
// or (WAVE) only the wavefront, when every transform's threads lie inside one
// wavefront -- LDS operations of one wavefront complete in order, so a
// wavefront-scope fence plus a scheduling barrier orders the exchange.
template <bool WAVE> __device__ __forceinline__ void group_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Whole transform on registers: v holds the inputs at in_pos on entry and the
// outputs at out_pos on exit.  buf is this transform's LDS scratch
// (LdsLen<N, PAD> values); every thread of the block (WAVE: of the wavefront)
// must call this, since it synchronises them.  w holds the thread's twiddle
// bases (tw_load); the overload without it loads them first.
template <class P, int DIR, typename V, bool PAD = false, bool WAVE = false>
__device__ __forceinline__ void fft_regs(V (&v)[P::E], int t, V* buf, const Tw<P, V>& w) {
  constexpr int N = P::N;
  constexpr int E = P::E;
  pass_first<E, P::R0, DIR>(v);
  if constexpr (P::P >= 2) {
    pass_write<N, E, P::R0, 1, V, PAD>(v, t, buf);
    group_sync<WAVE>();
    pass_read<N, E, P::R1, V, PAD>(v, t, buf);
    pass_tw<E, P::R1, DIR>(v, w.b1);
  }
  if constexpr (P::P >= 3) {
    group_sync<WAVE>();
    pass_write<N, E, P::R1, P::R0, V, PAD>(v, t, buf);
    group_sync<WAVE>();
    pass_read<N, E, P::R2, V, PAD>(v, t, buf);
    pass_tw<E, P::R2, DIR>(v, w.b2);
  }
  if constexpr (P::P >= 4) {
    group_sync<WAVE>();
    pass_write<N, E, P::R2, P::R0 * P::R1, V, PAD>(v, t, buf);
    group_sync<WAVE>();
    pass_read<N, E, P::R3, V, PAD>(v, t, buf);
    pass_tw<E, P::R3, DIR>(v, w.b3);
  }
}
template <class P, int DIR, typename V, bool PAD = false, bool WAVE = false>
__device__ __forceinline__ void fft_regs(V (&v)[P::E], int t, V* buf, const V* __restrict__ tw) {
  Tw<P, V> w;
  tw_load<P>(w, t, tw);
  fft_regs<P, DIR, V, PAD, WAVE>(v, t, buf, w);
}

// Register index that holds output element (N - pos) mod N, where pos is the
// element held in register i of thread t after fft_regs (natural order,
// out_pos).  Thread t >= 1 finds it in thread TT - t ("partner", same
// register map); thread 0 in itself.  Returns the register index for the
// partner case (self == false) or the thread-0 case (self == true).
template <class P> __device__ __forceinline__ constexpr int mirror_reg(int i, bool self) {
  constexpr int RL = P::RL;
  constexpr int S = P::E / RL;
  const int s = i / RL, r = i % RL;
  if (!self) return (S - 1 - s) * RL + (RL - 1 - r);
  if (s >= 1) return (S - s) * RL + (RL - 1 - r);
  return r == 0 ? 0 : RL - r;
}

// Register index i' (in in_pos order) of the element held in out_pos register i.
template <class P> __device__ __forceinline__ constexpr int out_to_in(int i) {
  constexpr int RL = P::RL;
  constexpr int S = P::E / RL;
  return (i / RL) + (i % RL) * S;
}

}  // namespace nsk
