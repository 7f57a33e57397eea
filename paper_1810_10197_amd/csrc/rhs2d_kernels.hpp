// Fused pass kernels of the 2D right-hand sides: plain Navier--Stokes
// (components u, v) and the Boussinesq system of Sec. 3.2, Eqs. (4a-b)
// (components u, v, rho), in two dimensions with gravity along -y:
//
//   f_u   = P(N_hat - Ri rho_hat e_y) - nu |k|^2 u_hat,   P = I - k k^T/|k|^2,
//   f_rho = -i k . (rho u)^ - kappa |k|^2 rho_hat,
//   N_hat = DFT(u x omega)/n^2 = DFT(v omega, -u omega)/n^2, omega = dv/dx - du/dy,
//
// both products 2/3-dealiased; f = 0 at k = 0.  Three passes:
//
//   Q1 y-inverse  compact FP64 state -> u, v, omega = i(kx v - ky u), rho cast
//                 to T, 2K+1 non-zero ky -> n values of y        B1 [m][4][y][kx]
//   Q2 x-pass     per (member, y) row: C2R transforms of (u + iv), omega and
//                 rho, the products at every point, R2C of
//                 (v omega - i u omega) and (rho u + i rho v), keep kx <= K
//                                      B2 [m][4][y][kx], or (COLB2) [m][4][kx][y]
//   Q3 y-forward  n values of y -> 2K+1 retained ky, then projection,
//                 buoyancy, diffusion and the cast to FP64, fused.
//
// K = (n - 1)/3: the 2/3 rule on n, or, with n the zero-padded 3N/2 of an N
// grid (K = N/2 - 1), the 3/2 rule of Sec. 2.1.1.
#pragma once
#include "pass_common.hpp"

namespace nsk {

// ---------------------------------------------------------------- Q1
// CW: column tile width (0 = the default); narrower tiles give more blocks
// but shorter runs per row.
// UT: the stage input's type (double2: the FP64 state; float2: the FP32
// stage input of an FP32 right-hand side inside a step).
template <class PL, typename T, int CW, typename UT>
__global__ __launch_bounds__((ColCfg<PL, T, CW>::NT)) void k2_yinv(const UT* __restrict__ U,
                                                              cplx<T>* __restrict__ B1, Geom g,
                                                              int nfield, long long nblocks,
                                                              const cplx<T>* __restrict__ tw) {
  constexpr int N = PL::N;
  using V = cplx<T>;
  using CF = ColCfg<PL, T, CW>;
  constexpr int E = CF::E, C = CF::C;
  __shared__ V lds[C * CF::LD];
  const long long L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= nblocks) return;                    // uniform per block
  const int ntiles = (g.Kx + C - 1) / C;
  const int f = (int)(L % nfield);
  const long long q = L / nfield;
  const int tile = (int)(q % ntiles);
  const int m = (int)(q / ntiles);
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int kx = tile * C + lc;
  const bool valid = kx < g.Kx;
  const long long cs = g.mr;
  const UT* Um = U + (long long)m * g.ncomp * cs + (valid ? kx : 0);
  // field f: 0 u, 1 v, 2 omega = i (kx v - ky u), 3 rho
  const int ca = f == 2 ? 1 : (f == 3 ? 2 : f);
  double2 a[E], b[E];
  bool use[E];
  int kys[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int e = in_pos<PL>(t, i);
    const bool ret = (e <= g.K) || (e >= N - g.K);
    use[i] = valid && ret;
    const int ky = e <= g.K ? e : e - N;
    kys[i] = ky;
    const int kyp = ret ? (ky >= 0 ? ky : ky + g.Kf) : 0;
    const UT* pp = Um + (long long)kyp * g.Kx;
    a[i] = to_d2(pp[ca * cs]);
    if (f == 2) b[i] = to_d2(pp[0]);
  }
  V v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    double vx = a[i].x, vy = a[i].y;
    if (f == 2) {
      const double ky = kys[i];
      const double wr = kx * a[i].x - ky * b[i].x, wi = kx * a[i].y - ky * b[i].y;
      vx = -wi;
      vy = wr;
    }
    v[i] = use[i] ? mk<V>((T)vx, (T)vy) : mk<V>((T)0, (T)0);
  }
  fft_regs<PL, +1>(v, t, lds + lc * CF::LD, tw);
  if (valid) {
    V* out = B1 + ((long long)(m * 4 + f) * N) * g.Kx + kx;
#pragma unroll
    for (int i = 0; i < E; ++i) out[(long long)out_pos<PL>(t, i) * g.Kx] = v[i];
  }
}

// ---------------------------------------------------------------- Q2
// Split a forward transform of (a + ib) held at out_pos registers into the
// half spectra of a and b at position pos, the mirror value from the partner.
template <class PL, typename V, typename T>
__device__ __forceinline__ void split_pair(const V (&z)[PL::E], int i, int t, int partner, V& ah, V& bh) {
  constexpr int TT = PL::TT;
  V pv = z[mirror_reg<PL>(i, true)];
  if constexpr (TT > 1) {
    const V sh = shfl_c(z[mirror_reg<PL>(i, false)], partner, TT);
    if (t != 0) pv = sh;
  }
  const T half = (T)0.5;
  const V zk = z[i];
  ah = mk<V>(half * (zk.x + pv.x), half * (zk.y - pv.y));
  bh = mk<V>(half * (zk.y + pv.y), half * (pv.x - zk.x));
}

// COLB2: write B2 column-major, [m][4][kx][y], so that Q3's columns are
// contiguous (each block's rows then fill RPB consecutive entries per kx).
template <class PL, typename T, bool SCALAR, bool COLB2>
__global__ __launch_bounds__((RowCfg<PL, T>::NT)) void k2_xpass(const cplx<T>* __restrict__ B1,
                                                               cplx<T>* __restrict__ B2, Geom g,
                                                               long long nrows,
                                                               const cplx<T>* __restrict__ tw) {
  constexpr int N = PL::N;
  using V = cplx<T>;
  using RC = RowCfg<PL, T>;
  constexpr int E = RC::E, TT = RC::TT;
  static_assert(64 % TT == 0, "a row's threads must lie in one wavefront");
  __shared__ V lds[RC::RPB * RC::LD];
  const int grp = threadIdx.x / TT, t = threadIdx.x - grp * TT;
  const long long row = (long long)blockIdx.x * RC::RPB + grp;
  const bool valid = row < nrows;
  const long long m = valid ? row / N : 0, y = valid ? row - m * N : 0;
  const int K = g.K, Kx = g.Kx;
  const T zero = (T)0;
  V* buf = lds + grp * RC::LD;
  const long long fs = (long long)N * Kx;          // field stride
  const V* base = B1 + (m * 4 * N + y) * Kx;

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
  // Z = A + iB at k <= K, conj(A) + i conj(B) at N - k.  Transforms:
  // (u + iv), (omega + 0i) and, with the scalar, (rho + 0i): rho is not
  // packed with omega, whose magnitude (~|k||u|) would swamp its rounding.
  constexpr int NZ = SCALAR ? 3 : 2;
  V z[NZ][E];
#pragma unroll
  for (int p = 0; p < NZ; ++p) {
    V a[E], b[E];
    const V* pa = base + (p == 0 ? 0 : p + 1) * fs;      // fields u | omega | rho
#pragma unroll
    for (int i = 0; i < E; ++i) {
      a[i] = pa[kk[i]];
      b[i] = p == 0 ? pa[fs + kk[i]] : mk<V>(zero, zero);
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const T ay = kk[i] == 0 ? zero : a[i].y, by = kk[i] == 0 ? zero : b[i].y;
      const V r = mk<V>(a[i].x - sg[i] * by, sg[i] * ay + b[i].x);
      z[p][i] = use[i] ? r : mk<V>(zero, zero);
    }
  }
  fft_regs<PL, +1, V, true, true>(z[0], t, buf, tw);
  group_sync<true>();
  fft_regs<PL, +1, V, true, true>(z[1], t, buf, tw);
  if constexpr (SCALAR) {
    group_sync<true>();
    fft_regs<PL, +1, V, true, true>(z[NZ - 1], t, buf, tw);
  }

  // products at every point: n = (v w, -u w), q = (rho u, rho v)
  V nn[E], qq[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const T u = z[0][i].x, v = z[0][i].y, w = z[1][i].x, r = SCALAR ? z[NZ - 1][i].x : zero;
    nn[out_to_in<PL>(i)] = mk<V>(v * w, -(u * w));
    qq[out_to_in<PL>(i)] = mk<V>(r * u, r * v);
  }
  group_sync<true>();
  fft_regs<PL, -1, V, true, true>(nn, t, buf, tw);
  if constexpr (SCALAR) {
    group_sync<true>();
    fft_regs<PL, -1, V, true, true>(qq, t, buf, tw);
  }
  const int partner = (TT - t) & (TT - 1);
  // element (field f, kx) of this row: row-major f * fs + kx, column-major
  // f * fs + kx * N (fs = N * Kx either way)
  V* out = COLB2 ? B2 + m * 4 * fs + y : B2 + (m * 4 * N + y) * Kx;
  const long long ks = COLB2 ? N : 1;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    V nx, ny, qx, qy;
    split_pair<PL, V, T>(nn, i, t, partner, nx, ny);
    if constexpr (SCALAR) split_pair<PL, V, T>(qq, i, t, partner, qx, qy);
    const int pos = out_pos<PL>(t, i);
    if (valid && pos <= K) {
      out[pos * ks] = nx;
      out[fs + pos * ks] = ny;
      if constexpr (SCALAR) {
        out[2 * fs + pos * ks] = qx;
        out[3 * fs + pos * ks] = qy;
      }
    }
  }
}

// Q2 with one row per block and one wavefront per transform: the inverse
// transforms of (u + iv), omega and (Boussinesq) rho run side by side in NZ
// wavefronts, the fields meet in LDS for the products, and the forward
// transforms of (v omega - i u omega) and (rho u + i rho v) run side by side
// in the first two.  A large single grid has too few rows to fill the GPU
// with one wavefront per row; this gives NZ times the wavefronts.  Same
// arithmetic per point as k2_xpass.
template <class PL, typename T, bool SCALAR, bool COLB2>
__global__ __launch_bounds__((SCALAR ? 3 : 2) * (PL::N / PL::E)) void k2_xpass_split(
    const cplx<T>* __restrict__ B1, cplx<T>* __restrict__ B2, Geom g, long long nrows,
    const cplx<T>* __restrict__ tw) {
  constexpr int N = PL::N, E = PL::E, TT = N / E;
  constexpr int NZ = SCALAR ? 3 : 2;
  constexpr int LD = LdsLen<N, true>::value;
  static_assert(TT == 64, "one wavefront per transform");
  using V = cplx<T>;
  __shared__ V lds[NZ * LD];
  const int grp = threadIdx.x / TT, t = threadIdx.x - grp * TT;   // grp: wavefront = transform
  const long long row = blockIdx.x;                                // uniform per block
  if (row >= nrows) return;
  const long long m = row / N, y = row - m * N;
  const int K = g.K, Kx = g.Kx;
  const T zero = (T)0;
  const long long fs = (long long)N * Kx;
  const V* base = B1 + (m * 4 * N + y) * Kx;
  V* buf = lds + grp * LD;
  // wavefront grp loads and inverts field pair 0 (u + iv), 1 (omega), 2 (rho)
  V z[E];
  {
    const V* pa = base + (grp == 0 ? 0 : grp + 1) * fs;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int pos = in_pos<PL>(t, i);
      const bool lo = pos <= K, hi = pos >= N - K;
      const int k0 = lo ? pos : N - pos;
      const int kk = k0 <= K ? k0 : K;
      const T sg = lo ? (T)1 : (T)-1;
      const V a = pa[kk];
      const V b = grp == 0 ? pa[fs + kk] : mk<V>(zero, zero);
      const T ay = kk == 0 ? zero : a.y, by = kk == 0 ? zero : b.y;
      const V r = mk<V>(a.x - sg * by, sg * ay + b.x);
      z[i] = (lo || hi) ? r : mk<V>(zero, zero);
    }
  }
  fft_regs<PL, +1, V, true, true>(z, t, buf, tw);
  // physical values by point: omega and rho (real parts) in buffer 1 as two
  // arrays of N reals, (u, v) in buffer NZ - 1 (SCALAR) or 0
  __syncthreads();
  T* wr = reinterpret_cast<T*>(lds + LD);          // omega [N], rho [N]
  V* uv = lds + (SCALAR ? 2 : 0) * LD;
  static_assert(2 * N <= 2 * LD, "two real arrays fit one buffer");
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int pos = out_pos<PL>(t, i);
    if (grp == 0) uv[pos] = z[i];
    else if (grp == 1) wr[pos] = z[i].x;
    else wr[N + pos] = z[i].x;
  }
  __syncthreads();
  V pr[E];                                          // group 0: n, group 1: q (in_pos order)
  if (grp < 2) {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int pos = out_pos<PL>(t, i);
      const V w2 = uv[pos];
      const T u = w2.x, v = w2.y;
      if (grp == 0) {
        const T w = wr[pos];
        pr[out_to_in<PL>(i)] = mk<V>(v * w, -(u * w));
      } else {
        const T r = SCALAR ? wr[N + pos] : zero;
        pr[out_to_in<PL>(i)] = mk<V>(r * u, r * v);
      }
    }
  }
  __syncthreads();                                  // the exchange buffers are free again
  if (grp >= (SCALAR ? 2 : 1)) return;              // uniform per wavefront; no block barrier follows
  fft_regs<PL, -1, V, true, true>(pr, t, lds + grp * LD, tw);
  const int partner = (TT - t) & (TT - 1);
  V* out = COLB2 ? B2 + m * 4 * fs + y : B2 + (m * 4 * N + y) * Kx;
  const long long ks = COLB2 ? N : 1;
  V* o0 = out + (grp == 0 ? 0 : 2) * fs;            // (n_x, n_y) or (q_x, q_y)
#pragma unroll
  for (int i = 0; i < E; ++i) {
    V a, b;
    split_pair<PL, V, T>(pr, i, t, partner, a, b);
    const int pos = out_pos<PL>(t, i);
    if (pos <= K) {
      o0[pos * ks] = a;
      o0[fs + pos * ks] = b;
    }
  }
}

// ---------------------------------------------------------------- Q3
// One block per tile of C columns kx; the NF transformed fields of a column
// are transformed side by side by NF thread groups (so that a 1024-point
// column still gives enough blocks), their outputs meet in LDS, and the
// epilogue's modes are shared out over all groups.  CMAX caps the tile
// width (fewer columns per block, more blocks).
template <class PL, typename T, int NF, int CMAX = 8> struct Q3Cfg {
  static constexpr int N = PL::N;
  static constexpr int TT = N / PL::E;
  static constexpr int LDS_BUDGET = 160 * 1024;
  static constexpr int C = cmax(
      1, cmin(cmin(1024 / (TT * NF), CMAX), floor_pow2(LDS_BUDGET / (NF * (N + 32) * (int)sizeof(cplx<T>)))));
  static constexpr int LD = col_ld(N, C);
  static constexpr int NT = C * TT * NF;
};

// With SPLIT (Boussinesq only) a block takes two of the four fields: group 0
// the velocity pair (n_x, n_y) and its projection, group 1 the density flux
// (q_x, q_y) and its divergence; the logical block row is 2 member + group.  Half the
// fields per block leaves room for twice the columns per tile.
template <bool SCALAR, bool SPLIT> struct Q3Fields {
  static constexpr int NF = SCALAR ? 4 : 2;
  static constexpr int NFB = (SCALAR && SPLIT) ? 2 : NF;   // fields per block
};

// f is written in FP64 to Kout and, where K32 is not null, rounded to FP32
// to K32 (the copy a later FP32 stage combination reads).  UT as in Q1.
__device__ __forceinline__ void put_f(double2* K, float2* K32, long long i, double2 v) {
  K[i] = v;
  if (K32) K32[i] = make_float2((float)v.x, (float)v.y);
}

template <class PL, typename T, bool SCALAR, int CMAX, bool COLB2, bool SPLIT, typename UT>
__global__ __launch_bounds__((Q3Cfg<PL, T, Q3Fields<SCALAR, SPLIT>::NFB, CMAX>::NT)) void k2_yfwd(
    const cplx<T>* __restrict__ B2, const UT* __restrict__ U, double2* __restrict__ Kout,
    float2* __restrict__ K32, Geom g, const double* __restrict__ nu, double ri, double kappa,
    const cplx<T>* __restrict__ tw, long long nblocks) {
  constexpr int N = PL::N;
  constexpr int NFB = Q3Fields<SCALAR, SPLIT>::NFB;
  constexpr bool SP = SCALAR && SPLIT;
  using V = cplx<T>;
  using QC = Q3Cfg<PL, T, NFB, CMAX>;
  constexpr int E = PL::E, C = QC::C, TT = QC::TT, LD = QC::LD;
  __shared__ V lds[NFB * C * LD];
  // logical block: tile + ntiles * (member, group); XCD-grouped so that the
  // neighbouring tiles, which share cache lines of B2 and of the state, run on
  // one XCD (one L2)
  const long long L = xcd_logical(blockIdx.x, gridDim.x);
  if (L >= nblocks) return;                      // uniform per block
  const int ntiles = (g.Kx + C - 1) / C;
  const int bxt = (int)(L % ntiles), byt = (int)(L / ntiles);
  const int f = threadIdx.x / (C * TT);
  const int rem = threadIdx.x - f * (C * TT);
  // transform phase: lanes along the column when it is contiguous (COLB2),
  // else across the tile's columns
  const int lc = COLB2 ? rem / TT : rem % C, t = COLB2 ? rem % TT : rem / C;
  const int grp = SP ? (byt & 1) : 0;
  const int m = SP ? (byt >> 1) : byt;
  const int fg = grp * 2 + f;                    // field of B2 this thread group transforms
  {
    const int kxt = bxt * C + lc;
    const bool vt = kxt < g.Kx;
    V* buf = lds + (f * C + lc) * LD;
    V o[E];
    const V* in = COLB2 ? B2 + ((long long)(m * 4 + fg) * g.Kx + (vt ? kxt : 0)) * N
                        : B2 + ((long long)(m * 4 + fg) * N) * g.Kx + (vt ? kxt : 0);
    const long long ys = COLB2 ? 1 : g.Kx;
#pragma unroll
    for (int i = 0; i < E; ++i) o[i] = in[(long long)in_pos<PL>(t, i) * ys];
    fft_regs<PL, -1>(o, t, buf, tw);
    __syncthreads();                             // every group done with its exchanges
#pragma unroll
    for (int i = 0; i < E; ++i) buf[out_pos<PL>(t, i)] = o[i];
    __syncthreads();
  }
  // epilogue: lanes across the tile's columns (adjacent kx of the state)
  const int elc = rem % C, et = rem / C;
  const int kx = bxt * C + elc;
  if (kx >= g.Kx) return;
  const double scale = 1.0 / ((double)N * (double)N);
  const double num = nu[m];
  const long long cs = g.mr;
  const V* col0 = lds + elc * LD;                // field c of this column: col0 + c * C * LD
  const bool vel = !SP || grp == 0;              // this block writes f_u, f_v
  const bool sca = SCALAR && (!SP || grp == 1);  // this block writes f_rho
#pragma unroll
  for (int i = f; i < E; i += NFB) {
    const int e = out_pos<PL>(et, i);
    if (!((e <= g.K) || (e >= N - g.K))) continue;
    const int ky = e <= g.K ? e : e - N;
    const long long idx = (long long)m * g.ncomp * cs + (long long)(ky >= 0 ? ky : ky + g.Kf) * g.Kx + kx;
    const double k2 = (double)(kx * kx + ky * ky);
    if (k2 == 0.0) {
      if (vel) {
        put_f(Kout, K32, idx, make_double2(0.0, 0.0));
        put_f(Kout, K32, idx + cs, make_double2(0.0, 0.0));
      }
      if (sca) put_f(Kout, K32, idx + 2 * cs, make_double2(0.0, 0.0));
      continue;
    }
    double2 rh = make_double2(0.0, 0.0);
    if constexpr (SCALAR) rh = to_d2(U[idx + 2 * cs]);
    if (vel) {
      const V v0 = col0[e], v1 = col0[C * LD + e];
      double nx = (double)v0.x * scale, nxi = (double)v0.y * scale;
      double ny = (double)v1.x * scale, nyi = (double)v1.y * scale;
      const double2 u0 = to_d2(U[idx]), u1 = to_d2(U[idx + cs]);
      if constexpr (SCALAR) {
        ny -= ri * rh.x;               // buoyancy -Ri rho e_y, before the projection
        nyi -= ri * rh.y;
      }
      const double px = (kx * nx + ky * ny) / k2, py = (kx * nxi + ky * nyi) / k2;
      const double vk = num * k2;
      put_f(Kout, K32, idx, make_double2(nx - kx * px - vk * u0.x, nxi - kx * py - vk * u0.y));
      put_f(Kout, K32, idx + cs, make_double2(ny - ky * px - vk * u1.x, nyi - ky * py - vk * u1.y));
    }
    if (sca) {
      // -i k . q_hat - kappa |k|^2 rho_hat (q_x, q_y are this block's fields 0, 1 when split)
      constexpr int q0 = SP ? 0 : 2;
      const V v2 = col0[q0 * C * LD + e], v3 = col0[(q0 + 1) * C * LD + e];
      const double sx = kx * ((double)v2.x * scale) + ky * ((double)v3.x * scale);
      const double sy = kx * ((double)v2.y * scale) + ky * ((double)v3.y * scale);
      const double kk2 = kappa * k2;
      put_f(Kout, K32, idx + 2 * cs, make_double2(sy - kk2 * rh.x, -sx - kk2 * rh.y));
    }
  }
}

// ---------------------------------------------------------------- host side
// Launch variants (the autotuner's choice; grids below 256 points use 0):
// Q1 (tuning slot 0) 0 default tile, 1 four columns, 2 two columns, 3 narrow
// plan default tile, 4 narrow plan two columns; Q3 (slot 4) 0 up to eight
// columns, 1 two, 2 one (Boussinesq: the fields split over two blocks, up to
// eight columns), 3 narrow plan up to eight, 4 narrow plan one (Boussinesq:
// split, up to eight), 5 two and 6 four (Boussinesq: split, so that a
// single grid gives two to four times the blocks of variant 1); slot 2: the layout of B2 (bit 0: 0 row-major, 1
// column-major) and, from 2 on, the row-split x-pass (one wavefront per
// transform; where a row's transform is one wavefront).  The x-pass keeps
// the wide plan (a row stays inside one wavefront).
template <int N, int V> struct Q1Var {
  using PL = typename std::conditional<(V >= 3 && N >= 256), PlanS<N>, Plan<N>>::type;
  static constexpr int CW = N < 256 ? 0 : (V == 1 ? 4 : (V == 2 || V == 4 ? 2 : 0));
};
template <int N, int V, bool SCALAR> struct Q3Var {
  using PL = typename std::conditional<((V == 3 || V == 4) && N >= 256), PlanS<N>, Plan<N>>::type;
  static constexpr bool SPLIT = SCALAR && N >= 256 && (V == 2 || V == 4 || V == 5 || V == 6);
  static constexpr int CMAX = N < 256 ? 8
                              : (V == 1 || V == 5) ? 2
                              : V == 6 ? 4
                              : ((V == 2 || V == 4) && !SPLIT ? 1 : 8);
};

template <int N, typename T, int VAR, typename UT>
static void launch_q1(const Geom& g, const UT* U, cplx<T>* B1, int nfield, const cplx<T>* tw,
                      hipStream_t st) {
  using QV = Q1Var<N, VAR>;
  using CF = ColCfg<typename QV::PL, T, QV::CW>;
  const long long nb1 = (long long)g.batch * nfield * ((g.Kx + CF::C - 1) / CF::C);
  const long long nb1p = (nb1 + 7) / 8 * 8;
  hipLaunchKernelGGL((k2_yinv<typename QV::PL, T, QV::CW, UT>), dim3((unsigned)nb1p), dim3(CF::NT), 0, st, U, B1,
                     g, nfield, nb1, tw);
}
template <int N, typename T, typename UT>
static void launch_q1v(int v1, const Geom& g, const UT* U, cplx<T>* B1, int nfield, const cplx<T>* tw,
                       hipStream_t st) {
  switch (v1) {
    case 1: launch_q1<N, T, N >= 256 ? 1 : 0>(g, U, B1, nfield, tw, st); break;
    case 2: launch_q1<N, T, N >= 256 ? 2 : 0>(g, U, B1, nfield, tw, st); break;
    case 3: launch_q1<N, T, N >= 256 ? 3 : 0>(g, U, B1, nfield, tw, st); break;
    case 4: launch_q1<N, T, N >= 256 ? 4 : 0>(g, U, B1, nfield, tw, st); break;
    default: launch_q1<N, T, 0>(g, U, B1, nfield, tw, st);
  }
}
template <int N, typename T, bool SCALAR, int VAR, bool COLB2, typename UT>
static void launch_q3(const Geom& g, const cplx<T>* B2, const UT* U, double2* K, const RhsParams& p,
                      const cplx<T>* tw, hipStream_t st) {
  using QV = Q3Var<N, VAR, SCALAR>;
  using QC = Q3Cfg<typename QV::PL, T, Q3Fields<SCALAR, QV::SPLIT>::NFB, QV::CMAX>;
  const long long nb = (long long)((g.Kx + QC::C - 1) / QC::C) * g.batch * (QV::SPLIT ? 2 : 1);
  const long long nbp = (nb + 7) / 8 * 8;
  hipLaunchKernelGGL((k2_yfwd<typename QV::PL, T, SCALAR, QV::CMAX, COLB2, QV::SPLIT, UT>), dim3((unsigned)nbp),
                     dim3(QC::NT), 0, st, B2, U, K, p.k32, g, p.nu, p.ri, p.kappa, tw, nb);
}
template <int N, typename T, bool SCALAR, bool COLB2, typename UT>
static void launch_q3v(int v3, const Geom& g, const cplx<T>* B2, const UT* U, double2* K,
                       const RhsParams& p, const cplx<T>* tw, hipStream_t st) {
  switch (v3) {
    case 1: launch_q3<N, T, SCALAR, N >= 256 ? 1 : 0, COLB2>(g, B2, U, K, p, tw, st); break;
    case 2: launch_q3<N, T, SCALAR, N >= 256 ? 2 : 0, COLB2>(g, B2, U, K, p, tw, st); break;
    case 3: launch_q3<N, T, SCALAR, N >= 256 ? 3 : 0, COLB2>(g, B2, U, K, p, tw, st); break;
    case 4: launch_q3<N, T, SCALAR, N >= 256 ? 4 : 0, COLB2>(g, B2, U, K, p, tw, st); break;
    case 5: launch_q3<N, T, SCALAR, N >= 256 ? 5 : 0, COLB2>(g, B2, U, K, p, tw, st); break;
    case 6: launch_q3<N, T, SCALAR, N >= 256 ? 6 : 0, COLB2>(g, B2, U, K, p, tw, st); break;
    default: launch_q3<N, T, SCALAR, 0, COLB2>(g, B2, U, K, p, tw, st);
  }
}

// U: the FP64 stage input; U32 (FP32 right-hand side only, else null): its
// FP32 rounding, read instead of U where given (the stage input of an FP32
// step, which the transforms round to FP32 anyway).
template <int N, typename T, bool SCALAR>
static hipError_t run2d(const Geom& g, const double2* U, const float2* U32, double2* K, const RhsParams& p,
                        const RhsBufs& bufs, const void* twv, hipStream_t st) {
  using V = cplx<T>;
  using PL = Plan<N>;
  using RC = RowCfg<PL, T>;
  const V* tw = (const V*)twv;
  V* B1 = (V*)bufs.a1;
  V* B2 = (V*)bufs.a2;
  const int nfield = SCALAR ? 4 : 3;
  // variants only matter (and are only built) from 256 points on
  const int v1 = N >= 256 ? bufs.variant[0] : 0, v3 = N >= 256 ? bufs.variant[4] : 0;
  const bool colb2 = N >= 256 && (bufs.variant[2] & 1);
  // the row-split x-pass (one wavefront per transform) where a row is one wavefront
  constexpr bool can_split = N >= 256 && PL::N / PL::E == 64;
  const bool split = can_split && bufs.variant[2] >= 2;
#define NSK_MARK(id, ph) \
  if (bufs.hook && bufs.fine != 2) bufs.hook(bufs.hook_ctx, id, ph, st)
  if (bufs.hook && bufs.fine == 2) bufs.hook(bufs.hook_ctx, PROF_RHS, 0, st);
  constexpr bool f32 = std::is_same<T, float>::value;
  if (!f32 && U32) return hipErrorInvalidValue;
  if (!U32 && !U) return hipErrorInvalidValue;
  NSK_MARK(PROF_P1, 0);
  if constexpr (f32) {
    if (U32) launch_q1v<N, T>(v1, g, U32, B1, nfield, tw, st);
    else launch_q1v<N, T>(v1, g, U, B1, nfield, tw, st);
  } else {
    launch_q1v<N, T>(v1, g, U, B1, nfield, tw, st);
  }
  NSK_MARK(PROF_P1, 1);
  const long long rows = (long long)g.batch * N;
  NSK_MARK(PROF_P3, 0);
  if constexpr (can_split) {
    if (split) {
      constexpr int NT = (SCALAR ? 3 : 2) * 64;
      if (colb2)
        hipLaunchKernelGGL((k2_xpass_split<PL, T, SCALAR, true>), dim3((unsigned)rows), dim3(NT), 0, st, B1, B2, g,
                           rows, tw);
      else
        hipLaunchKernelGGL((k2_xpass_split<PL, T, SCALAR, false>), dim3((unsigned)rows), dim3(NT), 0, st, B1, B2,
                           g, rows, tw);
    }
  }
  if (!split) {
    if (colb2)
      hipLaunchKernelGGL((k2_xpass<PL, T, SCALAR, N >= 256>), dim3((unsigned)((rows + RC::RPB - 1) / RC::RPB)),
                         dim3(RC::NT), 0, st, B1, B2, g, rows, tw);
    else
      hipLaunchKernelGGL((k2_xpass<PL, T, SCALAR, false>), dim3((unsigned)((rows + RC::RPB - 1) / RC::RPB)),
                         dim3(RC::NT), 0, st, B1, B2, g, rows, tw);
  }
  NSK_MARK(PROF_P3, 1);
  NSK_MARK(PROF_P5, 0);
  if constexpr (f32) {
    if (U32) {
      if (colb2) launch_q3v<N, T, SCALAR, N >= 256>(v3, g, B2, U32, K, p, tw, st);
      else launch_q3v<N, T, SCALAR, false>(v3, g, B2, U32, K, p, tw, st);
    }
  }
  if (!U32) {
    if (colb2) launch_q3v<N, T, SCALAR, N >= 256>(v3, g, B2, U, K, p, tw, st);
    else launch_q3v<N, T, SCALAR, false>(v3, g, B2, U, K, p, tw, st);
  }
  NSK_MARK(PROF_P5, 1);
  if (bufs.hook && bufs.fine == 2) bufs.hook(bufs.hook_ctx, PROF_RHS, 1, st);
#undef NSK_MARK
  return hipGetLastError();
}

}  // namespace nsk
