// Fused pass kernels of the 3D pseudo-spectral right-hand side, Eq. (2):
//
//   f(u_hat) = N_hat - k (k . N_hat)/|k|^2 - nu |k|^2 u_hat,
//   N_hat    = mask * DFT(u x omega) / n^3,  omega_hat = i k x u_hat,
//
// evaluated pseudo-spectrally (Sec. 2.1) with 2/3-rule dealiasing.  Five
// passes over pencils, each reading and writing only what the retained set
// (|k_j| <= K) needs:
//
//   P1 z-inverse  compact FP64 u_hat -> curl, cast to T, length-n inverse DFT
//                 along z of 2K+1 non-zero inputs, for 6 fields (u, omega)
//   P2 y-inverse  per (field, z) plane: 2K+1 non-zero ky -> n values of y
//   P3 x-pass     per (z, y) row: three paired C2R transforms (two real
//                 fields per complex DFT), u x omega at every point, R2C of
//                 (n_x + i n_y) and of n_z paired across two rows, keep kx <= K
//   P4 y-forward  n values of y -> the 2K+1 retained ky
//   P5 z-forward  n values of z -> the 2K+1 retained kz, then the projection,
//                 the viscous term and the cast to FP64, fused
//
// Intermediate layouts (T complex), chosen so that every column pass tiles a
// contiguous run of columns:
//   A1 [m][6][ky'][z][kx]   written by P1, read by P2 (columns (z, kx))
//   A2 [m][6][z][y][kx]     written by P2, read by P3 (rows (z, y))
//   A3 [m][3][y][z][kx]     written by P3 (reuses A1), read by P4 (columns (z, kx))
//   A4 [m][3][z][ky'][kx]   written by P4 (reuses A2), read by P5 (columns (ky', kx))
#include <type_traits>

#include "pass_common.hpp"

namespace nsk {

static_assert(TWN == TWN_TABLE, "twiddle table length");

// ---------------------------------------------------------------- P1
// Logical block id = (member, column tile, field) with the field fastest: the
// six blocks of one tile run on one XCD back to back and read u_hat once from
// HBM, the rest from L2.
template <class PL, typename T, int CW>
__global__ __launch_bounds__((ColCfg<PL, T, CW>::NT)) void k_zinv(const double2* __restrict__ U,
                                                             cplx<T>* __restrict__ A1, Geom g,
                                                             long long nblocks,
                                                             const cplx<T>* __restrict__ tw) {
  constexpr int N = PL::N;
  using V = cplx<T>;
  using CF = ColCfg<PL, T, CW>;
  constexpr int E = CF::E, C = CF::C;
  __shared__ V lds[C * CF::LD];
  const long long L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= nblocks) return;                     // uniform per block
  const int ncol = g.Kf * g.Kx;
  const int ntiles = (ncol + C - 1) / C;
  const int f = (int)(L % 6);
  const long long q = L / 6;
  const int tile = (int)(q % ntiles);
  const int m = (int)(q / ntiles);
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int col = tile * C + lc;
  const bool valid = col < ncol;
  int kx = 0, ky = 0, kyp = 0;
  if (valid) {
    kyp = col / g.Kx;
    kx = col - kyp * g.Kx;
    ky = kyp <= g.K ? kyp : kyp - g.Kf;
  }
  const long long cs = g.mr;
  const double2* Um = U + (long long)m * 3 * cs + (valid ? col : 0);
  // Loads without branches (clamped addresses, zeroed by selects) so that all
  // of a thread's loads are in flight together.
  double2 a[E], b[E];
  bool use[E];
  int kzs[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int e = in_pos<PL>(t, i);
    const bool ret = (e <= g.K) || (e >= N - g.K);
    use[i] = valid && ret;
    const int kz = e <= g.K ? e : e - N;
    kzs[i] = kz;
    const int kzp = ret ? (kz >= 0 ? kz : kz + g.Kf) : 0;
    const double2* pp = Um + (long long)kzp * ncol;
    if (f < 3) {
      a[i] = pp[f * cs];
    } else {
      // omega_hat = i k x u_hat: (ky, kz, kx) pair with (u_z, u_y), (u_x, u_z), (u_y, u_x)
      a[i] = pp[(f == 3 ? 2 : (f == 4 ? 0 : 1)) * cs];
      b[i] = pp[(f == 3 ? 1 : (f == 4 ? 2 : 0)) * cs];
    }
  }
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
    v[i] = use[i] ? mk<V>((T)vx, (T)vy) : mk<V>((T)0, (T)0);
  }
  fft_regs<PL, +1>(v, t, lds + lc * CF::LD, tw);
  if (valid) {
    const long long nkx = (long long)N * g.Kx;
    V* out = A1 + ((long long)(m * 6 + f) * g.Kf + kyp) * nkx + kx;
#pragma unroll
    for (int i = 0; i < E; ++i) out[(long long)out_pos<PL>(t, i) * g.Kx] = v[i];
  }
}

// ---------------------------------------------------------------- P2
// Columns (z, kx) of one (member, field): 2K+1 non-zero ky' -> N values of y.
template <class PL, typename T, int CW>
__global__ __launch_bounds__((ColCfg<PL, T, CW>::NT)) void k_yinv(const cplx<T>* __restrict__ A1,
                                                             cplx<T>* __restrict__ A2, Geom g,
                                                             const cplx<T>* __restrict__ tw) {
  constexpr int N = PL::N;
  using V = cplx<T>;
  using CF = ColCfg<PL, T, CW>;
  constexpr int E = CF::E, C = CF::C;
  __shared__ V lds[C * CF::LD];
  const long long bf = blockIdx.y;                // member * 6 + field
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int nkx = N * g.Kx;
  const int cz = blockIdx.x * C + lc;
  const bool valid = cz < nkx;
  const V* in = A1 + bf * g.Kf * nkx + (valid ? cz : 0);
  V v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int e = in_pos<PL>(t, i);
    const bool ret = (e <= g.K) || (e >= N - g.K);
    const int kyp = e <= g.K ? e : (ret ? e - N + g.Kf : 0);
    const V x = in[(long long)kyp * nkx];
    v[i] = (valid && ret) ? x : mk<V>((T)0, (T)0);
  }
  fft_regs<PL, +1>(v, t, lds + lc * CF::LD, tw);
  if (valid) {
    const int z = cz / g.Kx, kx = cz - z * g.Kx;
    V* out = A2 + (bf * N + z) * (long long)nkx + kx;
#pragma unroll
    for (int i = 0; i < E; ++i) out[(long long)out_pos<PL>(t, i) * g.Kx] = v[i];
  }
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
template <class PL, typename T>
__global__ __launch_bounds__((RowCfg<PL, T>::NT)) void k_xpass(const cplx<T>* __restrict__ A2,
                                                              cplx<T>* __restrict__ A3, Geom g,
                                                              long long nrows,
                                                              const cplx<T>* __restrict__ tw) {
  constexpr int N = PL::N;
  using V = cplx<T>;
  using RC = RowCfg<PL, T>;
  constexpr int E = RC::E, TT = RC::TT;
  __shared__ V lds[RC::RPB * RC::LD];
  const int grp = threadIdx.x / TT, t = threadIdx.x - grp * TT;
  const long long row = (long long)blockIdx.x * RC::RPB + grp;
  const bool valid = row < nrows;
  const long long rpm = (long long)N * N;
  const long long m = valid ? row / rpm : 0, rr = valid ? row - m * rpm : 0;
  const int K = g.K, Kx = g.Kx;
  const T zero = (T)0;
  V* buf = lds + grp * RC::LD;

  V z0[E], z1[E], z2[E];
  {
    // Loads without branches: every lane reads a clamped in-row address and
    // zeroes what lies outside the retained band with selects, so a whole
    // pair's loads are in flight together.  Z = A + iB at k <= K and
    // conj(A) + i conj(B) at N - k (s = +1 / -1 below).
    const V* base = A2 + (m * 6 * rpm + rr) * Kx;
    int kk[E];
    T sg[E];
    bool use[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int pos = in_pos<PL>(t, i);
      const bool lo = pos <= K, hi = pos >= N - K;
      use[i] = valid && (lo || hi);
      const int k0 = lo ? pos : N - pos;
      kk[i] = k0 <= K ? k0 : K;
      sg[i] = lo ? (T)1 : (T)-1;
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      V a[E], b[E];
      const V* pa = base + (long long)(2 * p) * rpm * Kx;
      const V* pb = pa + rpm * Kx;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        a[i] = pa[kk[i]];
        b[i] = pb[kk[i]];
      }
      V* z = p == 0 ? z0 : (p == 1 ? z1 : z2);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const T ay = kk[i] == 0 ? zero : a[i].y, by = kk[i] == 0 ? zero : b[i].y;
        const V r = mk<V>(a[i].x - sg[i] * by, sg[i] * ay + b[i].x);
        z[i] = use[i] ? r : mk<V>(zero, zero);
      }
    }
  }
  static_assert(64 % TT == 0, "a row's threads must lie in one wavefront");
  fft_regs<PL, +1, V, true, true>(z0, t, buf, tw);
  group_sync<true>();
  fft_regs<PL, +1, V, true, true>(z1, t, buf, tw);
  group_sync<true>();
  fft_regs<PL, +1, V, true, true>(z2, t, buf, tw);

  V nxy[E], nz[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const T ux = z0[i].x, uy = z0[i].y, uz = z1[i].x, wx = z1[i].y, wy = z2[i].x, wz = z2[i].y;
    nxy[out_to_in<PL>(i)] = mk<V>(uy * wz - uz * wy, uz * wx - ux * wz);
    nz[out_to_in<PL>(i)] = mk<V>(ux * wy - uy * wx, zero);
  }
  group_sync<true>();
  fft_regs<PL, -1, V, true, true>(nxy, t, buf, tw);
  group_sync<true>();
  fft_regs<PL, -1, V, true, true>(nz, t, buf, tw);

  const int partner = (TT - t) & (TT - 1);
  V* out = A3 + ((m * 3) * N + (rr % N)) * (long long)N * Kx + (rr / N) * (long long)Kx;
  const long long cstride = rpm * Kx;
  const T half = (T)0.5;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const V own = nxy[mirror_reg<PL>(i, true)];
    V pv = own;
    if constexpr (TT > 1) {
      const V sh = shfl_c(nxy[mirror_reg<PL>(i, false)], partner, TT);
      if (t != 0) pv = sh;
    }
    const int pos = out_pos<PL>(t, i);
    if (valid && pos <= K) {
      const V zk = nxy[i];
      out[pos] = mk<V>(half * (zk.x + pv.x), half * (zk.y - pv.y));
      out[cstride + pos] = mk<V>(half * (zk.y + pv.y), half * (pv.x - zk.x));
      out[2 * cstride + pos] = nz[i];
    }
  }
}

// ---------------------------------------------------------------- P4
// Columns (z, kx) of one (member, component): N values of y -> 2K+1 retained ky.
template <class PL, typename T, int CW>
__global__ __launch_bounds__((ColCfg<PL, T, CW>::NT)) void k_yfwd(const cplx<T>* __restrict__ A3,
                                                             cplx<T>* __restrict__ A4, Geom g,
                                                             const cplx<T>* __restrict__ tw) {
  constexpr int N = PL::N;
  using V = cplx<T>;
  using CF = ColCfg<PL, T, CW>;
  constexpr int E = CF::E, C = CF::C;
  __shared__ V lds[C * CF::LD];
  const long long bc = blockIdx.y;                // member * 3 + component
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int nkx = N * g.Kx;
  const int cz = blockIdx.x * C + lc;
  const bool valid = cz < nkx;
  const V* in = A3 + bc * N * (long long)nkx + (valid ? cz : 0);
  V v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = in[(long long)in_pos<PL>(t, i) * nkx];
  fft_regs<PL, -1>(v, t, lds + lc * CF::LD, tw);
  if (valid) {
    const int z = cz / g.Kx, kx = cz - z * g.Kx;
    V* out = A4 + (bc * N + z) * (long long)g.Kf * g.Kx + kx;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = out_pos<PL>(t, i);
      if (e <= g.K) out[(long long)e * g.Kx] = v[i];
      else if (e >= N - g.K) out[(long long)(e - N + g.Kf) * g.Kx] = v[i];
    }
  }
}

// ---------------------------------------------------------------- P5
template <class PL, typename T, int CW>
__global__ __launch_bounds__((ColCfg<PL, T, CW>::NT)) void k_zfwd(const cplx<T>* __restrict__ A4,
                                                           const double2* __restrict__ U,
                                                           double2* __restrict__ Kout, Geom g,
                                                           const double* __restrict__ nu,
                                                           const cplx<T>* __restrict__ tw) {
  constexpr int N = PL::N;
  using V = cplx<T>;
  using CF = ColCfg<PL, T, CW>;
  constexpr int E = CF::E, C = CF::C;
  __shared__ V lds[C * CF::LD];
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int ncol = g.Kf * g.Kx;
  const int col = blockIdx.x * C + lc;
  const int m = blockIdx.y;
  const bool valid = col < ncol;
  V o[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c > 0) __syncthreads();                // LDS reuse across fields
    const V* in = A4 + ((long long)(m * 3 + c) * N) * ncol + (valid ? col : 0);
#pragma unroll
    for (int i = 0; i < E; ++i) o[c][i] = in[(long long)in_pos<PL>(t, i) * ncol];
    fft_regs<PL, -1>(o[c], t, lds + lc * CF::LD, tw);
  }
  if (!valid) return;
  const int kyp = col / g.Kx;
  const int kx = col - kyp * g.Kx;
  const int ky = kyp <= g.K ? kyp : kyp - g.Kf;
  const double scale = 1.0 / ((double)N * (double)N * (double)N);
  const double num = nu[m];
  const long long cs = g.mr;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int e = out_pos<PL>(t, i);
    if (!((e <= g.K) || (e >= N - g.K))) continue;
    const int kz = e <= g.K ? e : e - N;
    const long long idx = (long long)m * 3 * cs + (long long)(kz >= 0 ? kz : kz + g.Kf) * ncol + col;
    const double n0x = (double)o[0][i].x * scale, n0y = (double)o[0][i].y * scale;
    const double n1x = (double)o[1][i].x * scale, n1y = (double)o[1][i].y * scale;
    const double n2x = (double)o[2][i].x * scale, n2y = (double)o[2][i].y * scale;
    const double k2 = (double)(kx * kx + ky * ky + kz * kz);
    double2 f0, f1, f2;
    if (k2 == 0.0) {
      f0 = make_double2(0.0, 0.0); f1 = f0; f2 = f0;
    } else {
      const double2 u0 = U[idx], u1 = U[idx + cs], u2 = U[idx + 2 * cs];
      const double px = (kx * n0x + ky * n1x + kz * n2x) / k2;
      const double py = (kx * n0y + ky * n1y + kz * n2y) / k2;
      const double vk = num * k2;
      f0 = make_double2(n0x - kx * px - vk * u0.x, n0y - kx * py - vk * u0.y);
      f1 = make_double2(n1x - ky * px - vk * u1.x, n1y - ky * py - vk * u1.y);
      f2 = make_double2(n2x - kz * px - vk * u2.x, n2y - kz * py - vk * u2.y);
    }
    Kout[idx] = f0;
    Kout[idx + cs] = f1;
    Kout[idx + 2 * cs] = f2;
  }
}

// ---------------------------------------------------------------- host side
// Launch variants of each pass, chosen at run time (the autotuner times them
// on the live workspace): column passes 0 wide plan / 16 columns, 1 wide /
// 32, 2 narrow plan / 16, 3 narrow / 32; x-pass 0 wide, 1 narrow.  Sizes
// below 64 always use variant 0.
template <int N, int V> struct ColVar {
  using PL = typename std::conditional<(V >= 2 && N >= 64), PlanS<N>, Plan<N>>::type;
  static constexpr int CW = (V & 1) && N >= 64 ? 32 : 16;
};

#define NSK_MARK(id, ph) \
  if (bufs.hook) bufs.hook(bufs.hook_ctx, id, ph)

template <int N, typename T, int V>
static void launch_zinv(const Geom& g, const double2* U, cplx<T>* A1, const cplx<T>* tw, hipStream_t st) {
  using CV = ColVar<N, V>;
  using CF = ColCfg<typename CV::PL, T, CV::CW>;
  const int ncol = g.Kf * g.Kx;
  const long long nb = (long long)g.batch * 6 * ((ncol + CF::C - 1) / CF::C);
  const long long nbp = (nb + 7) / 8 * 8;
  hipLaunchKernelGGL((k_zinv<typename CV::PL, T, CV::CW>), dim3((unsigned)nbp), dim3(CF::NT), 0, st, U, A1, g,
                     nb, tw);
}
template <int N, typename T, int V>
static void launch_yinv(const Geom& g, const cplx<T>* A1, cplx<T>* A2, const cplx<T>* tw, hipStream_t st) {
  using CV = ColVar<N, V>;
  using CF = ColCfg<typename CV::PL, T, CV::CW>;
  const int nkx = N * g.Kx;
  hipLaunchKernelGGL((k_yinv<typename CV::PL, T, CV::CW>), dim3((nkx + CF::C - 1) / CF::C, g.batch * 6),
                     dim3(CF::NT), 0, st, A1, A2, g, tw);
}
template <int N, typename T, int V>
static void launch_xpass(const Geom& g, const cplx<T>* A2, cplx<T>* A3, const cplx<T>* tw, hipStream_t st) {
  using PL = typename std::conditional<(V == 1 && N >= 64), PlanS<N>, Plan<N>>::type;
  using RC = RowCfg<PL, T>;
  const long long rows = (long long)g.batch * N * N;
  hipLaunchKernelGGL((k_xpass<PL, T>), dim3((unsigned)((rows + RC::RPB - 1) / RC::RPB)), dim3(RC::NT), 0, st,
                     A2, A3, g, rows, tw);
}
template <int N, typename T, int V>
static void launch_yfwd(const Geom& g, const cplx<T>* A3, cplx<T>* A4, const cplx<T>* tw, hipStream_t st) {
  using CV = ColVar<N, V>;
  using CF = ColCfg<typename CV::PL, T, CV::CW>;
  const int nkx = N * g.Kx;
  hipLaunchKernelGGL((k_yfwd<typename CV::PL, T, CV::CW>), dim3((nkx + CF::C - 1) / CF::C, g.batch * 3),
                     dim3(CF::NT), 0, st, A3, A4, g, tw);
}
template <int N, typename T, int V>
static void launch_zfwd(const Geom& g, const cplx<T>* A4, const double2* U, double2* K, const double* nu,
                        const cplx<T>* tw, hipStream_t st) {
  using CV = ColVar<N, V>;
  using CF = ColCfg<typename CV::PL, T, CV::CW>;
  const int ncol = g.Kf * g.Kx;
  hipLaunchKernelGGL((k_zfwd<typename CV::PL, T, CV::CW>), dim3((ncol + CF::C - 1) / CF::C, g.batch),
                     dim3(CF::NT), 0, st, A4, U, K, g, nu, tw);
}

template <int N, typename T>
static hipError_t run3d(const Geom& g, const double2* U, double2* K, const RhsParams& p,
                        const RhsBufs& bufs, const void* twv, hipStream_t st) {
  using V = cplx<T>;
  const V* tw = (const V*)twv;
  V* A1 = (V*)bufs.a1;
  V* A2 = (V*)bufs.a2;
  const int* tv = bufs.variant;
  NSK_MARK(PROF_P1, 0);
  switch (tv[0]) {
    case 1: launch_zinv<N, T, 1>(g, U, A1, tw, st); break;
    case 2: launch_zinv<N, T, 2>(g, U, A1, tw, st); break;
    case 3: launch_zinv<N, T, 3>(g, U, A1, tw, st); break;
    default: launch_zinv<N, T, 0>(g, U, A1, tw, st);
  }
  NSK_MARK(PROF_P1, 1);
  NSK_MARK(PROF_P2, 0);
  switch (tv[1]) {
    case 1: launch_yinv<N, T, 1>(g, A1, A2, tw, st); break;
    case 2: launch_yinv<N, T, 2>(g, A1, A2, tw, st); break;
    case 3: launch_yinv<N, T, 3>(g, A1, A2, tw, st); break;
    default: launch_yinv<N, T, 0>(g, A1, A2, tw, st);
  }
  NSK_MARK(PROF_P2, 1);
  NSK_MARK(PROF_P3, 0);
  if (tv[2] == 1) launch_xpass<N, T, 1>(g, A2, A1, tw, st);
  else launch_xpass<N, T, 0>(g, A2, A1, tw, st);
  NSK_MARK(PROF_P3, 1);
  NSK_MARK(PROF_P4, 0);
  switch (tv[3]) {
    case 1: launch_yfwd<N, T, 1>(g, A1, A2, tw, st); break;
    case 2: launch_yfwd<N, T, 2>(g, A1, A2, tw, st); break;
    case 3: launch_yfwd<N, T, 3>(g, A1, A2, tw, st); break;
    default: launch_yfwd<N, T, 0>(g, A1, A2, tw, st);
  }
  NSK_MARK(PROF_P4, 1);
  NSK_MARK(PROF_P5, 0);
  switch (tv[4]) {
    case 1: launch_zfwd<N, T, 1>(g, A2, U, K, p.nu, tw, st); break;
    case 2: launch_zfwd<N, T, 2>(g, A2, U, K, p.nu, tw, st); break;
    case 3: launch_zfwd<N, T, 3>(g, A2, U, K, p.nu, tw, st); break;
    default: launch_zfwd<N, T, 0>(g, A2, U, K, p.nu, tw, st);
  }
  NSK_MARK(PROF_P5, 1);
  return hipGetLastError();
}
#undef NSK_MARK

template <typename T>
static hipError_t dispatch3d(const Geom& g, const double2* U, double2* K, const RhsParams& p,
                             const RhsBufs& b, const void* tw, hipStream_t st) {
  switch (g.n) {
    case 8: return run3d<8, T>(g, U, K, p, b, tw, st);
    case 16: return run3d<16, T>(g, U, K, p, b, tw, st);
    case 32: return run3d<32, T>(g, U, K, p, b, tw, st);
    case 64: return run3d<64, T>(g, U, K, p, b, tw, st);
    case 128: return run3d<128, T>(g, U, K, p, b, tw, st);
    case 256: return run3d<256, T>(g, U, K, p, b, tw, st);
    case 512: return run3d<512, T>(g, U, K, p, b, tw, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t rhs3d_compact(const Geom& g, int fp64, const double2* U, double2* K, const RhsParams& p,
                         const RhsBufs& b, const void* tw, hipStream_t st) {
  return fp64 ? dispatch3d<double>(g, U, K, p, b, tw, st) : dispatch3d<float>(g, U, K, p, b, tw, st);
}

size_t rhs3d_scratch_bytes(const Geom& g, int fp64) {
  const size_t cb = fp64 ? 16 : 8;
  const size_t n = (size_t)g.n, B = (size_t)g.batch;
  const size_t a1 = B * 6 * n * (size_t)g.Kf * g.Kx * cb;     // also holds A3
  const size_t a2 = B * 6 * n * n * (size_t)g.Kx * cb;        // also holds A4
  return a1 + a2;
}

}  // namespace nsk
