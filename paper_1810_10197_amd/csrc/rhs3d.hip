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
// Intermediate layouts (T complex):  A1 [m][6][z][ky'][kx],  A2 [m][6][z][y][kx],
// A3 [m][3][z][y][kx] (reuses A1),   A4 [m][3][z][ky'][kx] (reuses A2).
#include "fft_core.hpp"
#include "ns_internal.hpp"

namespace nsk {

static_assert(TWN == TWN_TABLE, "twiddle table length");

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int floor_pow2(int x) { int p = 1; while (p * 2 <= x) p *= 2; return p; }

// Column passes: C adjacent columns per block, N/E threads per column.
template <int N, typename T> struct ColCfg {
  using V = cplx<T>;
  static constexpr int E = Plan<N>::E;
  static constexpr int TT = N / E;
  static constexpr int LDS_BUDGET = 80 * 1024;
  static constexpr int C = floor_pow2(cmin(cmax(256 / TT, 16), LDS_BUDGET / ((N + 1) * (int)sizeof(V))));
  static constexpr int NT = C * TT;
  static constexpr int LD = N + 1;      // padded LDS stride per column
};

// Row pass: ROWS rows per block, three transforms per row.
template <int N, typename T> struct RowCfg {
  static constexpr int E = Plan<N>::E;
  static constexpr int TT = N / E;
  static constexpr int ROWS = cmin(32, cmax(2, 64 / TT));
  static constexpr int NBUF = 3 * ROWS;
  static constexpr int NT = NBUF * TT;
  static constexpr int LD = N + 1;
};

__device__ __forceinline__ long long batch_index() {
  return (long long)blockIdx.y + (long long)blockIdx.z * gridDim.y;
}

// ---------------------------------------------------------------- P1
template <int N, typename T>
__global__ __launch_bounds__((ColCfg<N, T>::NT)) void k_zinv(const double2* __restrict__ U,
                                                           cplx<T>* __restrict__ A1, Geom g,
                                                           const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  using CF = ColCfg<N, T>;
  constexpr int E = CF::E, C = CF::C;
  __shared__ V lds[C * CF::LD];
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int ncol = g.Kf * g.Kx;
  const int col = blockIdx.x * C + lc;
  const int f = blockIdx.y, m = blockIdx.z;
  const bool valid = col < ncol;
  int kx = 0, ky = 0;
  if (valid) {
    const int kyp = col / g.Kx;
    kx = col - kyp * g.Kx;
    ky = kyp <= g.K ? kyp : kyp - g.Kf;
  }
  const long long cs = g.mr;
  const double2* Um = U + (long long)m * 3 * cs + col;
  V v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int e = in_pos<N>(t, i);
    const bool ret = (e <= g.K) || (e >= N - g.K);
    const int kz = e <= g.K ? e : e - N;
    double vx = 0.0, vy = 0.0;
    if (valid && ret) {
      const double2* p = Um + (long long)(kz >= 0 ? kz : kz + g.Kf) * ncol;
      if (f < 3) {
        const double2 a = p[f * cs];
        vx = a.x; vy = a.y;
      } else {
        // omega_hat = i k x u_hat, one component per field
        double2 a, b;
        double ka, kb;
        if (f == 3) { a = p[2 * cs]; ka = ky; b = p[cs]; kb = kz; }
        else if (f == 4) { a = p[0]; ka = kz; b = p[2 * cs]; kb = kx; }
        else { a = p[cs]; ka = kx; b = p[0]; kb = ky; }
        const double wr = ka * a.x - kb * b.x, wi = ka * a.y - kb * b.y;
        vx = -wi; vy = wr;
      }
    }
    v[i] = mk<V>((T)vx, (T)vy);
  }
  fft_regs<N, +1>(v, t, lds + lc * CF::LD, tw);
  if (valid) {
    V* out = A1 + ((long long)(m * 6 + f) * N) * ncol + col;
#pragma unroll
    for (int i = 0; i < E; ++i) out[(long long)out_pos<N>(t, i) * ncol] = v[i];
  }
}

// ---------------------------------------------------------------- P2
template <int N, typename T>
__global__ __launch_bounds__((ColCfg<N, T>::NT)) void k_yinv(const cplx<T>* __restrict__ A1,
                                                           cplx<T>* __restrict__ A2, Geom g,
                                                           long long nbatch,
                                                           const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  using CF = ColCfg<N, T>;
  constexpr int E = CF::E, C = CF::C;
  __shared__ V lds[C * CF::LD];
  const long long b = batch_index();
  if (b >= nbatch) return;                      // uniform per block
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int col = blockIdx.x * C + lc;
  const bool valid = col < g.Kx;
  const V* in = A1 + b * g.Kf * g.Kx + col;
  V v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int e = in_pos<N>(t, i);
    const bool ret = (e <= g.K) || (e >= N - g.K);
    const int kyp = e <= g.K ? e : e - N + g.Kf;
    v[i] = (valid && ret) ? in[(long long)kyp * g.Kx] : mk<V>((T)0, (T)0);
  }
  fft_regs<N, +1>(v, t, lds + lc * CF::LD, tw);
  if (valid) {
    V* out = A2 + b * N * g.Kx + col;
#pragma unroll
    for (int i = 0; i < E; ++i) out[(long long)out_pos<N>(t, i) * g.Kx] = v[i];
  }
}

// ---------------------------------------------------------------- P3
template <int N, typename T>
__global__ __launch_bounds__((RowCfg<N, T>::NT)) void k_xpass(const cplx<T>* __restrict__ A2,
                                                            cplx<T>* __restrict__ A3, Geom g,
                                                            const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  using RC = RowCfg<N, T>;
  constexpr int ROWS = RC::ROWS, NBUF = RC::NBUF, NT = RC::NT, LD = RC::LD, TT = RC::TT;
  __shared__ V lds[NBUF * LD];
  const long long rpm = (long long)N * N;             // rows per member
  const long long row0 = (long long)blockIdx.x * ROWS;
  const int K = g.K, Kx = g.Kx;
  const T zero = (T)0;

  // 1. paired half spectra -> full spectra Z = A + iB (A, B Hermitian)
  for (int idx = threadIdx.x; idx < NBUF * Kx; idx += NT) {
    const int buf = idx / Kx, kk = idx - buf * Kx;
    const int r = buf / 3, p = buf - 3 * r;
    const long long grow = row0 + r;
    const long long m = grow / rpm, rr = grow - m * rpm;
    V A = A2[((m * 6 + 2 * p) * rpm + rr) * Kx + kk];
    V B = A2[((m * 6 + 2 * p + 1) * rpm + rr) * Kx + kk];
    if (kk == 0) { A.y = zero; B.y = zero; }
    V* L = lds + buf * LD;
    L[kk] = mk<V>(A.x - B.y, A.y + B.x);
    if (kk > 0) L[N - kk] = mk<V>(A.x + B.y, B.x - A.y);
  }
  const int nmid = N - 2 * K - 1;
  for (int idx = threadIdx.x; idx < NBUF * nmid; idx += NT) {
    const int buf = idx / nmid, q = idx - buf * nmid;
    lds[buf * LD + K + 1 + q] = mk<V>(zero, zero);
  }
  __syncthreads();

  // 2. inverse transforms: (u_x + i u_y), (u_z + i w_x), (w_y + i w_z)
  const int grp = threadIdx.x / TT, tt = threadIdx.x - grp * TT;
  fft_lds<N, +1>(lds + grp * LD, tt, true, tw);

  // 3. n = u x omega at every point; n_z of the two rows of a pair shares one buffer
  for (int idx = threadIdx.x; idx < (ROWS / 2) * N; idx += NT) {
    const int pr = idx / N, x = idx - pr * N;
    T nz[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = 2 * pr + h;
      V* L0 = lds + (3 * r) * LD;
      const V a = L0[x], b = L0[LD + x], c = L0[2 * LD + x];
      const T ux = a.x, uy = a.y, uz = b.x, wx = b.y, wy = c.x, wz = c.y;
      L0[x] = mk<V>(uy * wz - uz * wy, uz * wx - ux * wz);
      nz[h] = ux * wy - uy * wx;
    }
    lds[(3 * (2 * pr) + 1) * LD + x] = mk<V>(nz[0], nz[1]);
  }
  __syncthreads();

  // 4. forward transforms of (n_x + i n_y) per row and (n_z(r0) + i n_z(r1)) per pair
  {
    const int r = grp / 3, p = grp - 3 * r;
    const bool active = (p == 0) || (p == 1 && (r & 1) == 0);
    fft_lds<N, -1>(lds + grp * LD, tt, active, tw);
  }

  // 5. split the paired spectra, keep kx <= K
  for (int idx = threadIdx.x; idx < ROWS * Kx; idx += NT) {
    const int r = idx / Kx, kk = idx - r * Kx;
    const long long grow = row0 + r;
    const long long m = grow / rpm, rr = grow - m * rpm;
    const V* Z = lds + (3 * r) * LD;
    const V zk = Z[kk], zm = Z[(N - kk) & (N - 1)];
    const V* P = lds + (3 * (r & ~1) + 1) * LD;
    const V pk = P[kk], pm = P[(N - kk) & (N - 1)];
    const T half = (T)0.5;
    // (X + conj(Y))/2 and (X - conj(Y))/(2i)
    const V nx = mk<V>(half * (zk.x + zm.x), half * (zk.y - zm.y));
    const V ny = mk<V>(half * (zk.y + zm.y), half * (zm.x - zk.x));
    const V nzv = (r & 1) == 0 ? mk<V>(half * (pk.x + pm.x), half * (pk.y - pm.y))
                               : mk<V>(half * (pk.y + pm.y), half * (pm.x - pk.x));
    V* out = A3 + ((m * 3) * rpm + rr) * Kx + kk;
    out[0] = nx;
    out[rpm * Kx] = ny;
    out[2 * rpm * Kx] = nzv;
  }
}

// ---------------------------------------------------------------- P4
template <int N, typename T>
__global__ __launch_bounds__((ColCfg<N, T>::NT)) void k_yfwd(const cplx<T>* __restrict__ A3,
                                                           cplx<T>* __restrict__ A4, Geom g,
                                                           long long nbatch,
                                                           const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  using CF = ColCfg<N, T>;
  constexpr int E = CF::E, C = CF::C;
  __shared__ V lds[C * CF::LD];
  const long long b = batch_index();
  if (b >= nbatch) return;
  const int lc = threadIdx.x % C, t = threadIdx.x / C;
  const int col = blockIdx.x * C + lc;
  const bool valid = col < g.Kx;
  const V* in = A3 + b * N * g.Kx + col;
  V v[E];
#pragma unroll
  for (int i = 0; i < E; ++i)
    v[i] = valid ? in[(long long)in_pos<N>(t, i) * g.Kx] : mk<V>((T)0, (T)0);
  fft_regs<N, -1>(v, t, lds + lc * CF::LD, tw);
  if (valid) {
    V* out = A4 + b * g.Kf * g.Kx + col;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = out_pos<N>(t, i);
      if (e <= g.K) out[(long long)e * g.Kx] = v[i];
      else if (e >= N - g.K) out[(long long)(e - N + g.Kf) * g.Kx] = v[i];
    }
  }
}

// ---------------------------------------------------------------- P5
template <int N, typename T>
__global__ __launch_bounds__((ColCfg<N, T>::NT)) void k_zfwd(const cplx<T>* __restrict__ A4,
                                                           const double2* __restrict__ U,
                                                           double2* __restrict__ Kout, Geom g,
                                                           const double* __restrict__ nu,
                                                           const cplx<T>* __restrict__ tw) {
  using V = cplx<T>;
  using CF = ColCfg<N, T>;
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
    const V* in = A4 + ((long long)(m * 3 + c) * N) * ncol + col;
#pragma unroll
    for (int i = 0; i < E; ++i)
      o[c][i] = valid ? in[(long long)in_pos<N>(t, i) * ncol] : mk<V>((T)0, (T)0);
    fft_regs<N, -1>(o[c], t, lds + lc * CF::LD, tw);
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
    const int e = out_pos<N>(t, i);
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
static void batch_grid(long long nb, unsigned& y, unsigned& z) {
  y = (unsigned)(nb < 32768 ? nb : 32768);
  z = (unsigned)((nb + y - 1) / y);
}

template <int N, typename T>
static hipError_t run3d(const Geom& g, const double2* U, double2* K, const RhsParams& p,
                        const RhsBufs& bufs, const void* twv, hipStream_t st) {
  using V = cplx<T>;
  using CF = ColCfg<N, T>;
  using RC = RowCfg<N, T>;
  const V* tw = (const V*)twv;
  V* A1 = (V*)bufs.a1;
  V* A2 = (V*)bufs.a2;
  const int ncol = g.Kf * g.Kx;
  unsigned y, z;
#define NSK_MARK(id, ph) \
  if (bufs.hook) bufs.hook(bufs.hook_ctx, id, ph)
  NSK_MARK(PROF_P1, 0);
  hipLaunchKernelGGL((k_zinv<N, T>), dim3((ncol + CF::C - 1) / CF::C, 6, g.batch), dim3(CF::NT), 0, st,
                     U, A1, g, tw);
  NSK_MARK(PROF_P1, 1);
  const long long nb2 = (long long)g.batch * 6 * N;
  batch_grid(nb2, y, z);
  NSK_MARK(PROF_P2, 0);
  hipLaunchKernelGGL((k_yinv<N, T>), dim3((g.Kx + CF::C - 1) / CF::C, y, z), dim3(CF::NT), 0, st,
                     A1, A2, g, nb2, tw);
  NSK_MARK(PROF_P2, 1);
  const long long rows = (long long)g.batch * N * N;
  NSK_MARK(PROF_P3, 0);
  hipLaunchKernelGGL((k_xpass<N, T>), dim3((unsigned)(rows / RC::ROWS)), dim3(RC::NT), 0, st,
                     A2, A1, g, tw);
  NSK_MARK(PROF_P3, 1);
  const long long nb4 = (long long)g.batch * 3 * N;
  batch_grid(nb4, y, z);
  NSK_MARK(PROF_P4, 0);
  hipLaunchKernelGGL((k_yfwd<N, T>), dim3((g.Kx + CF::C - 1) / CF::C, y, z), dim3(CF::NT), 0, st,
                     A1, A2, g, nb4, tw);
  NSK_MARK(PROF_P4, 1);
  NSK_MARK(PROF_P5, 0);
  hipLaunchKernelGGL((k_zfwd<N, T>), dim3((ncol + CF::C - 1) / CF::C, g.batch), dim3(CF::NT), 0, st,
                     A2, U, K, g, p.nu, tw);
  NSK_MARK(PROF_P5, 1);
#undef NSK_MARK
  return hipGetLastError();
}

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
