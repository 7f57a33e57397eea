// Fused pass kernels of the 3D pseudo-spectral right-hand side, Eq. (2):
//
//   f(u_hat) = N_hat - k (k . N_hat)/|k|^2 - nu |k|^2 u_hat,
//   N_hat    = mask * DFT(u x omega) / n^3,  omega_hat = i k x u_hat,
//
// evaluated pseudo-spectrally (Sec. 2.1) on an n^3 grid that keeps the modes
// |k_j| <= K = (n - 1)/3: the 2/3 rule on n, or -- with n the zero-padded
// 3N/2 of an N grid, K = N/2 - 1 -- the 3/2 rule of Sec. 2.1.1.  Five passes
// over pencils, each reading and writing only what the retained set needs:
//
//   P1 z-inverse  compact FP64 u_hat -> curl, cast to T, length-n inverse DFT
//                 along z of 2K+1 non-zero inputs, for 6 fields (u, omega)
//   P2 y-inverse  per (field, z) plane: 2K+1 non-zero ky -> n values of y
//   P3 x-pass     per (z, y) row: three paired C2R transforms (two real
//                 fields per complex DFT), u x omega at every point, forward
//                 DFTs of (n_x + i n_y) (split into the two half spectra) and
//                 of (n_z + 0i), keep kx <= K
//   P4 y-forward  n values of y -> the 2K+1 retained ky
//   P5 z-forward  n values of z -> the 2K+1 retained kz, then the projection,
//                 the viscous term and the cast to FP64, fused
//
// P2, P3 and P4 only couple values of one z plane, so they run over slabs of
// Zs planes (z0 .. z0+Zs-1) through two slab buffers that are reused for
// every slab: small enough, they stay in the memory-side cache between the
// three passes instead of going to HBM and back.  Intermediate layouts (T
// complex), chosen so that every column pass tiles a contiguous run of
// columns:
//   A1  [m][6][ky'][z][kx]   written by P1, read by P2 (columns (z, kx)); rows of
//                            a1_pitch(n) values (K + 1, padded from n = 512 on)
//   A2s [m][6][y][zl][kx]    slab: written by P2 (whole y rows of the slab),
//                            read by P3 (rows (y, zl), y-major)
//   A3s [m][3][y][zl][kx]    slab: written by P3, read by P4 (columns (zl, kx))
//   A4  [m][3][z][ky'][kx]   written by P4, read by P5 (columns (ky', kx)); the
//                            z-row pitch is padded to a multiple of 32 values so
//                            that P5's column tiles are whole cache lines
#pragma once
#include <type_traits>

#include "pass_common.hpp"

namespace nsk {

static_assert(TWN == TWN_TABLE, "twiddle table length");

// The band limit K = (n - 1)/3 of the 2/3 rule is a compile-time constant of
// every kernel (n is), so registers that only ever hold gap elements are
// neither loaded nor stored, and those that always hold band elements need no
// per-lane test.  Addresses are a block-uniform base plus a 32-bit per-lane
// byte offset; what a register adds on top is uniform again.

// Row pitch of A1 (values per (ky', z) row): K + 1, padded to a multiple of
// 16 on the power-of-two grids from 512 on.  There A1 (1.4 GB at 512^3) is far
// larger than the memory-side cache, and P1's column tiles write 128-byte
// chunks into rows of 1,368 bytes: every chunk straddles two lines and the
// writes ran at 2.6 TB/s; in rows of 176 values, with the pad columns written
// as zeros, the same writes run at 5.4 TB/s.  Below 512 the rows stay K + 1
// (at 256^3 A1 fits the cache and padding gained nothing there), and the
// padded 3 * 2^k grids have K + 1 = 2^k already.
__host__ __device__ constexpr int a1_pitch(int n) {
  return (n >= 512 && (n & (n - 1)) == 0) ? ((n - 1) / 3 + 1 + 15) / 16 * 16 : (n - 1) / 3 + 1;
}

// ---------------------------------------------------------------- P1
// Column loads of P1 from the compact FP64 state: component pa (and pb for
// the curl) at every kz' the thread's registers hold, zero in the gap, with
// kz per register.  No branches on lanes (band tests fold or become
// selects), so that all of a thread's loads are in flight together.
template <class PL, bool PAIR, typename UT>
__device__ __forceinline__ void zinv_loads(const UT* pa, const UT* pb, unsigned lane, int colc, int t,
                                           double2 (&a)[PL::E], double2 (&b)[PL::E], int (&kzs)[PL::E]) {
  constexpr int N = PL::N, K = (N - 1) / 3, KF = 2 * K + 1, KX = K + 1, NCOL = KF * KX, TT = PL::TT;
  const double2 zero2 = make_double2(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < PL::E; ++i) {
    const int c = in_base<PL>(i);
    const int bd = band_bits(c, TT, N, K);
    if (bd == BAND_GAP) {
      a[i] = zero2; b[i] = zero2; kzs[i] = 0;
      continue;
    }
    long long rowb = 0;
    unsigned off = lane;
    bool use = true;
    if (bd == BAND_LO) {
      rowb = c;
      kzs[i] = c + t;
    } else if (bd == BAND_HI) {
      rowb = c - N + KF;
      kzs[i] = c + t - N;
    } else {
      const int e = c + t;
      use = (e <= K) || (e >= N - K);
      const int kz = e <= K ? e : e - N;
      kzs[i] = kz;
      off = (unsigned)(colc + (use ? (kz >= 0 ? kz : kz + KF) : 0) * NCOL) * (unsigned)sizeof(UT);
    }
    const double2 x = to_d2(*byte_at(pa + rowb * NCOL, off));
    a[i] = use ? x : zero2;
    if (PAIR) {
      const double2 y = to_d2(*byte_at(pb + rowb * NCOL, off));
      b[i] = use ? y : zero2;
    } else {
      b[i] = zero2;
    }
  }
}

// Logical block id = (member, column tile, field) with the field fastest: the
// six blocks of one tile run on one XCD back to back and read u_hat once from
// HBM, the rest from L2.
template <class PL, typename T, int CW, typename UT>
__global__ __launch_bounds__((ColCfg<PL, T, CW>::NT)) void k_zinv(const UT* __restrict__ U,
                                                             cplx<T>* __restrict__ A1, long long nblocks,
                                                             const cplx<T>* __restrict__ tw,
                                                             const int* __restrict__ active) {
  constexpr int N = PL::N, K = (N - 1) / 3, KF = 2 * K + 1, KX = K + 1, NCOL = KF * KX;
  constexpr int KXA = a1_pitch(N), NCOLA = KF * KXA;   // A1's columns (ky', kx), padded rows
  constexpr long long MR = (long long)NCOL * KF;
  using V = cplx<T>;
  using CF = ColCfg<PL, T, CW>;
  constexpr int E = CF::E, C = CF::C, TT = CF::TT;
  __shared__ V lds[C * CF::LD];
  const long long L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= nblocks) return;                     // uniform per block
  constexpr int ntiles = (NCOLA + C - 1) / C;
  const int f = (int)(L % 6);
  const long long q = L / 6;
  const int tile = (int)(q % ntiles);
  const int m = (int)(q / ntiles);
  if (active && !active[m]) return;             // member not evaluated (uniform per block)
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int col = tile * C + lc;                // column of A1: ky' * KXA + kx
  const bool valid = col < NCOLA;
  const int colc = valid ? col : 0;
  const int kyp = colc / KXA;
  const int kx = colc - kyp * KXA;
  const bool real = KXA == KX || kx < KX;       // pad columns transform zeros and write them
  const int colu = real ? kyp * KX + kx : 0;    // the column in the compact state
  const int ky = kyp <= K ? kyp : kyp - KF;
  Tw<PL, V> w;
  tw_load<PL>(w, t, tw);
  // components read by field f: u_f, or the pair (a, b) of omega_f = i (ka b - kb a)
  const int ca = f < 3 ? f : (f == 3 ? 2 : (f == 4 ? 0 : 1));
  const int cb = f == 3 ? 1 : (f == 4 ? 2 : 0);
  const UT* Um = U + (long long)m * 3 * MR;
  const unsigned lane = (unsigned)(colu + t * NCOL) * (unsigned)sizeof(UT);
  double2 a[E], b[E];
  int kzs[E];
  if (f < 3) zinv_loads<PL, false, UT>(Um + ca * MR, Um, lane, colu, t, a, b, kzs);
  else zinv_loads<PL, true, UT>(Um + ca * MR, Um + cb * MR, lane, colu, t, a, b, kzs);
  V v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    double vx, vy;
    if (f < 3) {
      vx = a[i].x; vy = a[i].y;
    } else {
      const double kz = kzs[i];
      const double ka = f == 3 ? ky : (f == 4 ? kz : kx);
      const double kb = f == 3 ? kz : (f == 4 ? kx : ky);
      const double wr = ka * a[i].x - kb * b[i].x, wi = ka * a[i].y - kb * b[i].y;
      vx = -wi; vy = wr;
    }
    v[i] = real ? mk<V>((T)vx, (T)vy) : mk<V>((T)0, (T)0);
  }
  fft_regs<PL, +1>(v, t, lds + lc * CF::LD, w);
  if (valid) {
    V* out = A1 + (long long)(m * 6 + f) * KF * N * KXA;
    const unsigned lo = (unsigned)((kyp * N + t) * KXA + kx) * (unsigned)sizeof(V);
#pragma unroll
    for (int i = 0; i < E; ++i) *byte_at(out + out_base<PL>(i) * KXA, lo) = v[i];
  }
}

// ---------------------------------------------------------------- P2
// Columns (zl, kx) of one (member, field) in the slab z0 .. z0+zs-1: 2K+1
// non-zero ky' -> N values of y.  Logical block id = (member, field, column
// tile), remapped so that each XCD takes a contiguous range: neighbouring
// tiles, whose output rows share cache lines at the tile edges, then write
// through the same L2 (about 1% faster than the plain 2D grid at 256^3).
// One block's work (logical block id L, LDS of C * (N + 1) values).
template <class PL, typename T, int CW>
__device__ __forceinline__ void yinv_block(const cplx<T>* __restrict__ A1, cplx<T>* __restrict__ A2s, int z0,
                                           int zs, long long L, cplx<T>* lds, const cplx<T>* __restrict__ tw,
                                           const int* __restrict__ active) {
  constexpr int N = PL::N, K = (N - 1) / 3, KF = 2 * K + 1, KX = K + 1, NKX = N * KX;
  constexpr int KXA = a1_pitch(N), NKXA = N * KXA;  // A1's padded rows
  using V = cplx<T>;
  using CF = ColCfg<PL, T, CW>;
  constexpr int E = CF::E, C = CF::C, TT = CF::TT;
  const int ntx = (zs * KXA + C - 1) / C;
  const long long bf = L / ntx;                   // member * 6 + field
  const int bx = (int)(L - bf * ntx);
  if (active && !active[bf / 6]) return;
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int cz = bx * C + lc;                     // slab column of A1: zl * KXA + kx
  const bool inb = cz < zs * KXA;
  const int czc = inb ? cz : 0;
  const int zl = czc / KXA, kx = czc - zl * KXA;
  const bool valid = inb && (KXA == KX || kx < KX);   // pad columns are read (zeros), not written
  Tw<PL, V> w;
  tw_load<PL>(w, t, tw);
  const V* in = A1 + bf * KF * NKXA + z0 * KXA;
  const unsigned lane = (unsigned)(czc + t * NKXA) * (unsigned)sizeof(V);
  V v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int c = in_base<PL>(i);
    const int bd = band_bits(c, TT, N, K);
    const V zero = mk<V>((T)0, (T)0);
    if (bd == BAND_GAP) {
      v[i] = zero;
    } else if (bd == BAND_LO) {
      v[i] = ld_nt(byte_at(in + (long long)c * NKXA, lane));
    } else if (bd == BAND_HI) {
      v[i] = ld_nt(byte_at(in + (long long)(c - N + KF) * NKXA, lane));
    } else {
      const int e = c + t;
      const bool ret = (e <= K) || (e >= N - K);
      const int kyp = e <= K ? e : (ret ? e - N + KF : 0);
      const V x = ld_nt(byte_at(in, (unsigned)(czc + kyp * NKXA) * (unsigned)sizeof(V)));
      v[i] = ret ? x : zero;
    }
  }
  fft_regs<PL, +1>(v, t, lds + lc * CF::LD, w);
  if (valid) {
    const int nkxs = zs * KX;                     // one y row of the slab: every (zl, kx)
    V* out = A2s + bf * zs * NKX;
    const unsigned lo = (unsigned)(zl * KX + kx + t * nkxs) * (unsigned)sizeof(V);
#pragma unroll
    for (int i = 0; i < E; ++i) st_out<N>(byte_at(out + (long long)out_base<PL>(i) * nkxs, lo), v[i]);
  }
}

template <class PL, typename T, int CW>
__global__ __launch_bounds__((ColCfg<PL, T, CW>::NT)) void k_yinv(const cplx<T>* __restrict__ A1,
                                                             cplx<T>* __restrict__ A2s, int z0, int zs,
                                                             long long nblocks,
                                                             const cplx<T>* __restrict__ tw,
                                                             const int* __restrict__ active) {
  using CF = ColCfg<PL, T, CW>;
  __shared__ cplx<T> lds[CF::C * CF::LD];
  const long long L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= nblocks) return;                       // uniform per block
  yinv_block<PL, T, CW>(A1, A2s, z0, zs, L, lds, tw, active);
}

// ---------------------------------------------------------------- P3
// One group of N/E threads per (member, z, y) row, everything in registers:
//  1. the three paired half spectra (u_x + i u_y), (u_z + i w_x), (w_y + i w_z)
//     are loaded straight into the first pass's registers, completing each
//     Hermitian half to the full spectrum Z = A + iB on the fly;
//  2. three inverse transforms; their outputs sit at the same positions in
//     every thread, so u x omega is formed in registers;
//  3. forward transforms of (n_x + i n_y) and of (n_z + 0i) start from those
//     registers (the last inverse pass's output positions are the first
//     forward pass's input positions);
//  4. n_x, n_y are split from Z(k) and conj(Z(N-k)), the mirror value coming
//     from the partner thread through a cross-lane shuffle; keep kx <= K.
// One block's rows rb * RPB .. rb * RPB + RPB - 1 of member m (LDS of RPB
// padded rows).
template <class PL, typename T, int RPB>
__device__ __forceinline__ void xpass_block(const cplx<T>* __restrict__ A2s, cplx<T>* __restrict__ A3s, int zs,
                                            long long rb, long long m, cplx<T>* lds,
                                            const cplx<T>* __restrict__ tw, const int* __restrict__ active) {
  constexpr int N = PL::N, K = (N - 1) / 3, KX = K + 1;
  using V = cplx<T>;
  using RC = RowCfg<PL, T>;
  constexpr int E = RC::E, TT = RC::TT;
  const int grp = threadIdx.x / TT, t = threadIdx.x % TT;
  const long long RPM = (long long)zs * N;        // rows (y, zl) per member in the slab, y-major
  if (active && !active[m]) return;
  const long long row = rb * RPB + grp;
  const bool valid = row < RPM;
  const long long rr = valid ? row : 0;
  const T zero = (T)0;
  V* buf = lds + grp * RC::LD;
  Tw<PL, V> w;
  tw_load<PL>(w, t, tw);

  V z0[E], z1[E], z2[E];
  {
    // Z = A + iB at k <= K and conj(A) + i conj(B) at N - k.  Registers in
    // the low band read A[c + t], those in the high band A[N - c - t]; both
    // are a per-lane base plus a compile-time offset.
    const V* base = A2s + (m * 6 * RPM + rr) * KX;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const V* pa = base + (long long)(2 * p) * RPM * KX;
      const V* pb = pa + RPM * KX;
      const V* pa_lo = pa + t;
      const V* pb_lo = pb + t;
      const V* pa_hi = pa + (N - t);
      const V* pb_hi = pb + (N - t);
      V* z = p == 0 ? z0 : (p == 1 ? z1 : z2);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int c = in_base<PL>(i);
        const int bd = band_bits(c, TT, N, K);
        V r;
        if (bd == BAND_GAP) {
          r = mk<V>(zero, zero);
        } else if (bd == BAND_LO) {
          const V a = pa_lo[c], b = pb_lo[c];
          if (c == 0) {                           // k = 0 of a real field is real
            const T ay = t == 0 ? zero : a.y, by = t == 0 ? zero : b.y;
            r = mk<V>(a.x - by, ay + b.x);
          } else {
            r = mk<V>(a.x - b.y, a.y + b.x);
          }
        } else if (bd == BAND_HI) {
          const V a = pa_hi[-c], b = pb_hi[-c];
          r = mk<V>(a.x + b.y, b.x - a.y);
        } else {
          const int pos = c + t;
          const bool lo = pos <= K, hi = pos >= N - K;
          const int k0 = lo ? pos : N - pos;
          const int kk = k0 <= K ? k0 : K;
          const V a = pa[kk], b = pb[kk];
          const T sg = lo ? (T)1 : (T)-1;
          const T ay = kk == 0 ? zero : a.y, by = kk == 0 ? zero : b.y;
          const V x = mk<V>(a.x - sg * by, sg * ay + b.x);
          r = (lo || hi) ? x : mk<V>(zero, zero);
        }
        z[i] = valid ? r : mk<V>(zero, zero);
      }
    }
  }
  static_assert(64 % TT == 0, "a row's threads must lie in one wavefront");
  fft_regs<PL, +1, V, true, true>(z0, t, buf, w);
  group_sync<true>();
  fft_regs<PL, +1, V, true, true>(z1, t, buf, w);
  group_sync<true>();
  fft_regs<PL, +1, V, true, true>(z2, t, buf, w);

  V nxy[E], nz[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const T ux = z0[i].x, uy = z0[i].y, uz = z1[i].x, wx = z1[i].y, wy = z2[i].x, wz = z2[i].y;
    nxy[out_to_in<PL>(i)] = mk<V>(uy * wz - uz * wy, uz * wx - ux * wz);
    nz[out_to_in<PL>(i)] = mk<V>(ux * wy - uy * wx, zero);
  }
  group_sync<true>();
  fft_regs<PL, -1, V, true, true>(nxy, t, buf, w);
  group_sync<true>();
  fft_regs<PL, -1, V, true, true>(nz, t, buf, w);

  const int partner = (TT - t) & (TT - 1);
  V* out = A3s + (m * 3 * RPM + rr) * KX + t;
  const long long CST = RPM * KX;
  const T half = (T)0.5;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int c = out_base<PL>(i);
    const int bd = band_bits(c, TT, N, K);
    if (!(bd & BAND_LO)) continue;               // kx > K for every thread: dropped
    const V own = nxy[mirror_reg<PL>(i, true)];
    V pv = own;
    if constexpr (TT > 1) {
      const V sh = shfl_c(nxy[mirror_reg<PL>(i, false)], partner, TT);
      if (t != 0) pv = sh;
    }
    if (valid && (bd == BAND_LO || c + t <= K)) {
      const V zk = nxy[i];
      out[c] = mk<V>(half * (zk.x + pv.x), half * (zk.y - pv.y));
      out[CST + c] = mk<V>(half * (zk.y + pv.y), half * (pv.x - zk.x));
      out[2 * CST + c] = nz[i];
    }
  }
}

template <class PL, typename T>
__global__ __launch_bounds__((RowCfg<PL, T>::NT)) void k_xpass(const cplx<T>* __restrict__ A2s,
                                                              cplx<T>* __restrict__ A3s, int zs,
                                                              const cplx<T>* __restrict__ tw,
                                                              const int* __restrict__ active) {
  using RC = RowCfg<PL, T>;
  __shared__ cplx<T> lds[RC::RPB * RC::LD];
  xpass_block<PL, T, RC::RPB>(A2s, A3s, zs, blockIdx.x, blockIdx.y, lds, tw, active);
}

// ---------------------------------------------------------------- P4
// Columns (zl, kx) of one (member, component) in the slab: N values of y ->
// 2K+1 retained ky, written to plane z0 + zl of A4 (blocks XCD-grouped as in
// P2).
template <class PL, typename T, int CW>
__device__ __forceinline__ void yfwd_block(const cplx<T>* __restrict__ A3s, cplx<T>* __restrict__ A4, int z0,
                                           int zs, long long L, cplx<T>* lds, const cplx<T>* __restrict__ tw,
                                           const int* __restrict__ active) {
  constexpr int N = PL::N, K = (N - 1) / 3, KF = 2 * K + 1, KX = K + 1;
  using V = cplx<T>;
  using CF = ColCfg<PL, T, CW>;
  constexpr int E = CF::E, C = CF::C, TT = CF::TT;
  const int nkxs = zs * KX;                       // row length of the slab buffer
  const int ntx = (nkxs + C - 1) / C;
  const long long bc = L / ntx;                   // member * 3 + component
  const int bx = (int)(L - bc * ntx);
  if (active && !active[bc / 3]) return;
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int cz = bx * C + lc;
  const bool valid = cz < nkxs;
  const int czc = valid ? cz : 0;
  Tw<PL, V> w;
  tw_load<PL>(w, t, tw);
  const V* in = A3s + bc * N * nkxs;
  const unsigned lane = (unsigned)(czc + t * nkxs) * (unsigned)sizeof(V);
  V v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = *byte_at(in + (long long)in_base<PL>(i) * nkxs, lane);
  fft_regs<PL, -1>(v, t, lds + lc * CF::LD, w);
  if (valid) {
    constexpr int NCOLP = (KF * KX + 31) / 32 * 32;  // line-aligned z-row pitch of A4
    const int zl = cz / KX, kx = cz - zl * KX;
    V* out = A4 + (bc * N + z0) * NCOLP;
    const unsigned lo = (unsigned)(zl * NCOLP + t * KX + kx) * (unsigned)sizeof(V);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int c = out_base<PL>(i);
      const int bd = band_bits(c, TT, N, K);
      if (bd == BAND_GAP) continue;
      if (bd == BAND_LO) {
        *byte_at(out + c * KX, lo) = v[i];
      } else if (bd == BAND_HI) {
        *byte_at(out + (c - N + KF) * KX, lo) = v[i];
      } else {
        const int e = c + t;
        if (e <= K) *byte_at(out + c * KX, lo) = v[i];
        else if (e >= N - K) *byte_at(out + (c - N + KF) * KX, lo) = v[i];
      }
    }
  }
}

template <class PL, typename T, int CW>
__global__ __launch_bounds__((ColCfg<PL, T, CW>::NT)) void k_yfwd(const cplx<T>* __restrict__ A3s,
                                                             cplx<T>* __restrict__ A4, int z0, int zs,
                                                             long long nblocks,
                                                             const cplx<T>* __restrict__ tw,
                                                             const int* __restrict__ active) {
  using CF = ColCfg<PL, T, CW>;
  __shared__ cplx<T> lds[CF::C * CF::LD];
  const long long L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= nblocks) return;                       // uniform per block
  yfwd_block<PL, T, CW>(A3s, A4, z0, zs, L, lds, tw, active);
}

// ---------------------------------------------------------------- P5
template <class PL, typename T, int CW, typename UT>
__global__ __launch_bounds__((ColCfg<PL, T, CW>::NT)) void k_zfwd(const cplx<T>* __restrict__ A4,
                                                           const UT* __restrict__ U,
                                                           double2* __restrict__ Kout,
                                                           float2* __restrict__ K32,
                                                           const double* __restrict__ nu,
                                                           const cplx<T>* __restrict__ tw,
                                                           const int* __restrict__ active,
                                                           long long nblocks) {
  constexpr int N = PL::N, K = (N - 1) / 3, KF = 2 * K + 1, KX = K + 1, NCOL = KF * KX;
  constexpr int NCOLP = (NCOL + 31) / 32 * 32;      // line-aligned z-row pitch of A4
  constexpr long long MR = (long long)NCOL * KF;
  using V = cplx<T>;
  using CF = ColCfg<PL, T, CW>;
  constexpr int E = CF::E, C = CF::C, TT = CF::TT;
  __shared__ V lds[C * CF::LD];
  // logical block = (member, column tile), XCD-grouped on the power-of-two
  // grids: neighbouring tiles share the cache lines at their edges in the
  // compact u_hat and f rows (256^3: u_hat reads 1.18x -> 1.01x of the model;
  // 512^3: 821 -> 639 us).  On the zero-padded 3 * 2^k grids the grouping made
  // the pass slower (384: 231 -> 300 us), and tiles keep the launch order.
  constexpr bool GROUP = (N & (N - 1)) == 0;
  const long long L = GROUP ? xcd_logical(blockIdx.x, gridDim.x) : (long long)blockIdx.x;
  if (L >= nblocks) return;                     // uniform per block
  constexpr int ntiles = (NCOL + C - 1) / C;
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int col = (int)(L % ntiles) * C + lc;
  const int m = (int)(L / ntiles);
  if (active && !active[m]) return;
  const bool valid = col < NCOL;
  const int colc = valid ? col : 0;
  Tw<PL, V> w;
  tw_load<PL>(w, t, tw);
  const unsigned lane = (unsigned)(colc + t * NCOLP) * (unsigned)sizeof(V);
  V o[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c > 0) __syncthreads();                // LDS reuse across fields
    const V* in = A4 + (long long)(m * 3 + c) * N * NCOLP;
#pragma unroll
    for (int i = 0; i < E; ++i) o[c][i] = *byte_at(in + (long long)in_base<PL>(i) * NCOLP, lane);
    fft_regs<PL, -1>(o[c], t, lds + lc * CF::LD, w);
  }
  if (!valid) return;
  const int kyp = col / KX;
  const int kx = col - kyp * KX;
  const int ky = kyp <= K ? kyp : kyp - KF;
  const double scale = 1.0 / ((double)N * (double)N * (double)N);
  const double num = nu[m];
  const UT* Um = U + (long long)m * 3 * MR;
  double2* Km = Kout + (long long)m * 3 * MR;
  float2* K32m = K32 ? K32 + (long long)m * 3 * MR : nullptr;     // uniform per launch
  const unsigned lo = (unsigned)(col + t * NCOL) * 16u;
  constexpr unsigned USZ = (unsigned)sizeof(UT);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int c = out_base<PL>(i);
    const int bd = band_bits(c, TT, N, K);
    if (bd == BAND_GAP) continue;
    const int e = c + t;
    if (bd != BAND_LO && bd != BAND_HI && !((e <= K) || (e >= N - K))) continue;
    const int kz = e <= K ? e : e - N;
    // row kz' of this register: c + t (low band) or c + t - N + 2K+1 (high)
    const long long rowb = bd == BAND_LO ? c : (bd == BAND_HI ? c - N + KF : 0);
    const unsigned off = (bd == BAND_LO || bd == BAND_HI)
                             ? lo
                             : (unsigned)(col + (kz >= 0 ? kz : kz + KF) * NCOL) * 16u;
    const unsigned offu = off / 16u * USZ;       // the same element in the input's precision
    const UT* up = Um + rowb * NCOL;
    double2* kp = Km + rowb * NCOL;
    const double n0x = (double)o[0][i].x * scale, n0y = (double)o[0][i].y * scale;
    const double n1x = (double)o[1][i].x * scale, n1y = (double)o[1][i].y * scale;
    const double n2x = (double)o[2][i].x * scale, n2y = (double)o[2][i].y * scale;
    const double k2 = (double)(kx * kx + ky * ky + kz * kz);
    double2 f0, f1, f2;
    if (k2 == 0.0) {
      f0 = make_double2(0.0, 0.0); f1 = f0; f2 = f0;
    } else {
      const double2 u0 = to_d2(*byte_at(up, offu)), u1 = to_d2(*byte_at(up + MR, offu)),
                    u2 = to_d2(*byte_at(up + 2 * MR, offu));
      const double px = (kx * n0x + ky * n1x + kz * n2x) / k2;
      const double py = (kx * n0y + ky * n1y + kz * n2y) / k2;
      const double vk = num * k2;
      f0 = make_double2(n0x - kx * px - vk * u0.x, n0y - kx * py - vk * u0.y);
      f1 = make_double2(n1x - ky * px - vk * u1.x, n1y - ky * py - vk * u1.y);
      f2 = make_double2(n2x - kz * px - vk * u2.x, n2y - kz * py - vk * u2.y);
    }
    st_out<N>(byte_at(kp, off), f0);
    st_out<N>(byte_at(kp + MR, off), f1);
    st_out<N>(byte_at(kp + 2 * MR, off), f2);
    if (K32m) {
      float2* kq = K32m + rowb * NCOL;
      *byte_at(kq, off / 2u) = make_float2((float)f0.x, (float)f0.y);
      *byte_at(kq + MR, off / 2u) = make_float2((float)f1.x, (float)f1.y);
      *byte_at(kq + 2 * MR, off / 2u) = make_float2((float)f2.x, (float)f2.y);
    }
  }
}

// ---------------------------------------------------------------- host side
// Launch variants of each pass, chosen at run time (the autotuner times them
// on the live workspace): column passes 0 wide plan / 16 columns, 1 wide /
// 32, 2 narrow plan / 16, 3 narrow / 32, 4 wide / 64 (as many as the LDS
// and the 1024-thread limit allow); x-pass 0 wide, 1 narrow.  Sizes below 64
// always use variant 0.
template <int N, int V> struct ColVar {
  using PL = typename std::conditional<(V >= 2 && V <= 3 && N >= 64), PlanS<N>, Plan<N>>::type;
  static constexpr int CW = N < 64 ? 16 : (V == 4 ? 64 : ((V & 1) ? 32 : 16));
};

#define NSK_MARK(id, ph, stream) \
  if (bufs.hook && bufs.fine != 2) bufs.hook(bufs.hook_ctx, id, ph, stream)
#define NSK_MARK_RHS(ph) \
  if (bufs.hook && bufs.fine == 2) bufs.hook(bufs.hook_ctx, PROF_RHS, ph, st)

template <int N, typename T, int V, typename UT>
static void launch_zinv(const Geom& g, const UT* U, cplx<T>* A1, const cplx<T>* tw, const int* act,
                        hipStream_t st) {
  using CV = ColVar<N, V>;
  using CF = ColCfg<typename CV::PL, T, CV::CW>;
  const int ncol = g.Kf * a1_pitch(N);
  const long long nb = (long long)g.batch * 6 * ((ncol + CF::C - 1) / CF::C);
  const long long nbp = (nb + 7) / 8 * 8;
  hipLaunchKernelGGL((k_zinv<typename CV::PL, T, CV::CW, UT>), dim3((unsigned)nbp), dim3(CF::NT), 0, st, U, A1,
                     nb, tw, act);
}
template <int N, typename T, int V>
static void launch_yinv(const Geom& g, const cplx<T>* A1, cplx<T>* A2s, int z0, int zs, const cplx<T>* tw,
                        const int* act, hipStream_t st) {
  using CV = ColVar<N, V>;
  using CF = ColCfg<typename CV::PL, T, CV::CW>;
  const int ncol = zs * a1_pitch(N);
  const int ntx = (ncol + CF::C - 1) / CF::C;
  const long long nb = (long long)ntx * g.batch * 6;
  const dim3 grid((unsigned)((nb + 7) / 8 * 8));
  hipLaunchKernelGGL((k_yinv<typename CV::PL, T, CV::CW>), grid, dim3(CF::NT), 0, st, A1, A2s, z0, zs, nb, tw,
                     act);
}
template <int N, typename T, int V>
static void launch_xpass(const Geom& g, const cplx<T>* A2s, cplx<T>* A3s, int zs, const cplx<T>* tw,
                         const int* act, hipStream_t st) {
  // the narrow plan only where a row's threads still fit in one wavefront
  using PL = typename std::conditional<(V == 1 && N >= 64 && PlanS<N>::TT <= 64), PlanS<N>, Plan<N>>::type;
  using RC = RowCfg<PL, T>;
  const long long rows = (long long)zs * N;       // per member
  hipLaunchKernelGGL((k_xpass<PL, T>), dim3((unsigned)((rows + RC::RPB - 1) / RC::RPB), g.batch), dim3(RC::NT),
                     0, st, A2s, A3s, zs, tw, act);
}
template <int N, typename T, int V>
static void launch_yfwd(const Geom& g, const cplx<T>* A3s, cplx<T>* A4, int z0, int zs, const cplx<T>* tw,
                        const int* act, hipStream_t st) {
  using CV = ColVar<N, V>;
  using CF = ColCfg<typename CV::PL, T, CV::CW>;
  const int ncol = zs * g.Kx;
  const int ntx = (ncol + CF::C - 1) / CF::C;
  const long long nb = (long long)ntx * g.batch * 3;
  const dim3 grid((unsigned)((nb + 7) / 8 * 8));
  hipLaunchKernelGGL((k_yfwd<typename CV::PL, T, CV::CW>), grid, dim3(CF::NT), 0, st, A3s, A4, z0, zs, nb, tw,
                     act);
}
template <int N, typename T, int V, typename UT>
static void launch_zfwd(const Geom& g, const cplx<T>* A4, const UT* U, double2* K, float2* K32,
                        const double* nu, const cplx<T>* tw, const int* act, hipStream_t st) {
  // P5 holds three transformed fields: a 64-column block would exceed the
  // registers of 1024 threads, so its variant 4 is variant 1
  using CV = ColVar<N, V == 4 ? 1 : V>;
  using CF = ColCfg<typename CV::PL, T, CV::CW>;
  const int ncol = g.Kf * g.Kx;
  const long long nb = (long long)((ncol + CF::C - 1) / CF::C) * g.batch;
  const long long nbp = (nb + 7) / 8 * 8;
  hipLaunchKernelGGL((k_zfwd<typename CV::PL, T, CV::CW, UT>), dim3((unsigned)nbp), dim3(CF::NT), 0, st, A4, U,
                     K, K32, nu, tw, act, nb);
}

// Scratch regions of one evaluation (T complex), each 256-byte aligned: A1,
// A4, slab buffer 0 (up to n planes) and slab buffer 1 (up to n/2 planes,
// used by the two-stream schedule).
struct Scratch3d {
  size_t a1, a4, a2s[2], a3s[2], total;
};
inline size_t al256(size_t x) { return (x + 255) / 256 * 256; }
inline Scratch3d scratch3d(const Geom& g, int fp64) {
  const size_t cb = fp64 ? 16 : 8;
  const size_t n = (size_t)g.n, B = (size_t)g.batch, plane = (size_t)g.Kf * g.Kx;
  const size_t p2 = B * 6 * n * g.Kx * cb, p3 = B * 3 * n * g.Kx * cb;   // per z plane
  Scratch3d s;
  s.a1 = 0;
  s.a4 = al256(B * 6 * n * (size_t)g.Kf * a1_pitch(g.n) * cb);   // A1 with its padded rows
  const size_t planep = (plane + 31) / 32 * 32;       // A4's padded z-row pitch
  s.a2s[0] = s.a4 + al256(B * 3 * n * planep * cb);
  s.a3s[0] = s.a2s[0] + al256(p2 * n);
  s.a2s[1] = s.a3s[0] + al256(p3 * n);
  s.a3s[1] = s.a2s[1] + al256(p2 * (n / 2));
  s.total = s.a3s[1] + al256(p3 * (n / 2));
  return s;
}

template <int N, typename T, typename UT>
static hipError_t run3d(const Geom& g, const UT* U, double2* K, const RhsParams& p,
                        const RhsBufs& bufs, const void* twv, hipStream_t st) {
  using V = cplx<T>;
  const V* tw = (const V*)twv;
  const Scratch3d sc = scratch3d(g, sizeof(T) == 8);
  char* base = (char*)bufs.a1;
  V* A1 = (V*)(base + sc.a1);
  V* A4 = (V*)(base + sc.a4);
  const int* tv = bufs.variant;
  const int* act = p.active;                       // members to evaluate (null: all)
  const bool two = slab_two_streams(tv[5]) && bufs.side && N >= 2;
  const int zs = slab_planes(g, tv[5]);
  NSK_MARK_RHS(0);
  NSK_MARK(PROF_P1, 0, st);
  switch (tv[0]) {
    case 1: launch_zinv<N, T, 1, UT>(g, U, A1, tw, act, st); break;
    case 2: launch_zinv<N, T, 2, UT>(g, U, A1, tw, act, st); break;
    case 3: launch_zinv<N, T, 3, UT>(g, U, A1, tw, act, st); break;
      case 4: launch_zinv<N, T, 4, UT>(g, U, A1, tw, act, st); break;
    default: launch_zinv<N, T, 0, UT>(g, U, A1, tw, act, st);
  }
  NSK_MARK(PROF_P1, 1, st);
  // the slab phase is timed as a whole: its launches may overlap on two
  // streams, and events between them would perturb it (with bufs.fine every
  // launch is also bracketed, on its own stream)
  NSK_MARK(PROF_SLAB, 0, st);
  if (two) {
    hipError_t e = hipEventRecord(bufs.fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(bufs.side, bufs.fork, 0);
    if (e != hipSuccess) return e;
  }
  int slab = 0;
  for (int z0 = 0; z0 < N; z0 += zs, ++slab) {
    const int nz = N - z0 < zs ? N - z0 : zs;
    const int b = two ? (slab & 1) : 0;
    hipStream_t ss = b ? bufs.side : st;
    V* A2s = (V*)(base + sc.a2s[b]);
    V* A3s = (V*)(base + sc.a3s[b]);
    if (bufs.fine == 1) NSK_MARK(PROF_P2, 0, ss);
    switch (tv[1]) {
      case 1: launch_yinv<N, T, 1>(g, A1, A2s, z0, nz, tw, act, ss); break;
      case 2: launch_yinv<N, T, 2>(g, A1, A2s, z0, nz, tw, act, ss); break;
      case 3: launch_yinv<N, T, 3>(g, A1, A2s, z0, nz, tw, act, ss); break;
      case 4: launch_yinv<N, T, 4>(g, A1, A2s, z0, nz, tw, act, ss); break;
      default: launch_yinv<N, T, 0>(g, A1, A2s, z0, nz, tw, act, ss);
    }
    if (bufs.fine == 1) {
      NSK_MARK(PROF_P2, 1, ss);
      NSK_MARK(PROF_P3, 0, ss);
    }
    if (tv[2] == 1) launch_xpass<N, T, 1>(g, A2s, A3s, nz, tw, act, ss);
    else launch_xpass<N, T, 0>(g, A2s, A3s, nz, tw, act, ss);
    if (bufs.fine == 1) {
      NSK_MARK(PROF_P3, 1, ss);
      NSK_MARK(PROF_P4, 0, ss);
    }
    switch (tv[3]) {
      case 1: launch_yfwd<N, T, 1>(g, A3s, A4, z0, nz, tw, act, ss); break;
      case 2: launch_yfwd<N, T, 2>(g, A3s, A4, z0, nz, tw, act, ss); break;
      case 3: launch_yfwd<N, T, 3>(g, A3s, A4, z0, nz, tw, act, ss); break;
      case 4: launch_yfwd<N, T, 4>(g, A3s, A4, z0, nz, tw, act, ss); break;
      default: launch_yfwd<N, T, 0>(g, A3s, A4, z0, nz, tw, act, ss);
    }
    if (bufs.fine == 1) NSK_MARK(PROF_P4, 1, ss);
  }
  if (two) {
    hipError_t e = hipEventRecord(bufs.join, bufs.side);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, bufs.join, 0);
    if (e != hipSuccess) return e;
  }
  NSK_MARK(PROF_SLAB, 1, st);
  NSK_MARK(PROF_P5, 0, st);
  float2* k32 = sizeof(T) == 4 ? p.k32 : nullptr;   // FP32 copies only of an FP32 right-hand side
  switch (tv[4]) {
    case 1: launch_zfwd<N, T, 1, UT>(g, A4, U, K, k32, p.nu, tw, act, st); break;
    case 2: launch_zfwd<N, T, 2, UT>(g, A4, U, K, k32, p.nu, tw, act, st); break;
    case 3: launch_zfwd<N, T, 3, UT>(g, A4, U, K, k32, p.nu, tw, act, st); break;
    case 4: launch_zfwd<N, T, 4, UT>(g, A4, U, K, k32, p.nu, tw, act, st); break;
    default: launch_zfwd<N, T, 0, UT>(g, A4, U, K, k32, p.nu, tw, act, st);
  }
  NSK_MARK(PROF_P5, 1, st);
  NSK_MARK_RHS(1);
  return hipGetLastError();
}
#undef NSK_MARK
#undef NSK_MARK_RHS

}  // namespace nsk
