// FP64 state kernels around the right-hand side: Runge--Kutta stage
// combinations (Sec. 2.2), the embedded error norm of Sec. 2.2.1 fused with
// the kinetic-energy / dissipation / shell diagnostics of Sec. 3.1, and the
// conversions between the full half-spectrum layout of the C ABI and the
// compact retained-mode layout used internally.  All reductions are
// deterministic: a fixed number of blocks per member, fixed per-thread
// strides, fixed shuffle trees and a fixed-order final sum.
#include "ns_internal.hpp"

namespace nsk {

// Decode a compact element index (within one member) into component and
// signed wavenumbers.
struct Modes {
  int c, kx, ky, kz;
};
__device__ __forceinline__ Modes decode(const Geom& g, long long i) {
  Modes r;
  r.c = (int)(i / g.mr);
  long long q = i - (long long)r.c * g.mr;
  r.kx = (int)(q % g.Kx);
  q /= g.Kx;
  const int kyp = (int)(q % g.Kf);
  r.ky = kyp <= g.K ? kyp : kyp - g.Kf;
  if (g.dim == 3) {
    const int kzp = (int)(q / g.Kf);
    r.kz = kzp <= g.K ? kzp : kzp - g.Kf;
  } else {
    r.kz = 0;
  }
  return r;
}

// Offset of a retained mode in the full half-spectrum layout of one component.
__device__ __forceinline__ long long full_offset(const Geom& g, const Modes& md) {
  const long long nh = g.nf / 2 + 1;
  const int iy = md.ky < 0 ? md.ky + g.nf : md.ky;
  if (g.dim == 3) {
    const int iz = md.kz < 0 ? md.kz + g.nf : md.kz;
    return ((long long)iz * g.nf + iy) * nh + md.kx;
  }
  return (long long)iy * nh + md.kx;
}

// Streaming loads (the nontemporal hint) for operands that a kernel reads
// once: the state and stage-derivative arrays are far larger than the caches
// and are next read a whole right-hand side later, so keeping them out of the
// caches leaves those to the lines being written.  The values are those of a
// plain load.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
  return make_float2(v.x, v.y);
}
// Store with the same hint, for outputs that are next read only after a
// whole right-hand side: the FP64 u_{n+1} and the partial embedded difference
// of an FP32 step's last combination (the next pass reads the FP32 stage
// input, which keeps plain stores so that it can stay in the caches).
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
  const d2v x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<d2v*>(p));
}

// Grid of the element-wise kernels: one element per thread, blockIdx.y =
// member (no per-element division to find the member).
static dim3 member_grid(long long per_member, int batch) {
  long long gx = (per_member + 255) / 256;
  if (gx > 65535) gx = 65535;
  if (gx < 1) gx = 1;
  return dim3((unsigned)gx, (unsigned)batch);
}

// out = base + h_m sum_j coef_j src_j with NT terms known at compile time, so
// that every term's load is in flight at once; written in FP64 (out64)
// and/or rounded to FP32 (out32, the stage input of an FP32 right-hand side);
// with D2 also out2 = sum_j coef2_j src_j from the same loads.
template <int NT, bool W64, bool W32, bool D2>
__global__ __launch_bounds__(256) void k_combine(const double2* __restrict__ base, Combo c,
                                                 const double* __restrict__ h, double2* __restrict__ out64,
                                                 float2* __restrict__ out32, double2* __restrict__ out2,
                                                 long long epm) {
  const long long off = (long long)blockIdx.y * epm;
  const double hm = h[blockIdx.y];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < epm; i += stride) {
    double2 v[NT > 0 ? NT : 1];
#pragma unroll
    for (int j = 0; j < NT; ++j) v[j] = ld_stream(c.src[j] + off + i);
    double2 r = base ? ld_stream(base + off + i) : make_double2(0.0, 0.0);
    double sx = 0.0, sy = 0.0, dx = 0.0, dy = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      sx += c.coef[j] * v[j].x;
      sy += c.coef[j] * v[j].y;
      if (D2) {
        dx += c.coef2[j] * v[j].x;
        dy += c.coef2[j] * v[j].y;
      }
    }
    r.x += hm * sx;
    r.y += hm * sy;
    if (W64) {
      if (W32) st_stream(out64 + off + i, r);   // FP32 step: the FP32 copy is the next input
      else out64[off + i] = r;
    }
    if (W32) out32[off + i] = make_float2((float)r.x, (float)r.y);
    if (D2) st_stream(out2 + off + i, make_double2(dx, dy));
  }
}

// out32 = base + h_m sum_j coef_j src32_j (FP64 accumulation of FP32 sources),
// rounded to FP32.  The base is the FP64 state or its FP32 rounding (BT).
__device__ __forceinline__ double2 to_d2s(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2s(float2 v) { return make_double2((double)v.x, (double)v.y); }
template <int NT, typename BT>
__global__ __launch_bounds__(256) void k_combine_s32(const BT* __restrict__ base, Combo c,
                                                     const double* __restrict__ h, float2* __restrict__ out32,
                                                     long long epm) {
  const long long off = (long long)blockIdx.y * epm;
  const double hm = h[blockIdx.y];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < epm; i += stride) {
    float2 v[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) v[j] = ld_stream(c.src32[j] + off + i);
    const double2 r = to_d2s(ld_stream(base + off + i));
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      sx += c.coef[j] * (double)v[j].x;
      sy += c.coef[j] * (double)v[j].y;
    }
    out32[off + i] = make_float2((float)(r.x + hm * sx), (float)(r.y + hm * sy));
  }
}

static unsigned grid_for(long long total, int bs) {
  long long b = (total + bs - 1) / bs;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

template <bool W64, bool W32, bool D2>
static hipError_t combine_to(const Geom& g, const double2* base, const Combo& c, const double* h,
                             double2* out64, float2* out32, double2* out2, hipStream_t st) {
  const dim3 grid = member_grid(g.epm, g.batch);
  switch (c.nterms) {
#define NSK_COMBINE(k)                                                                                 \
    case k:                                                                                            \
      hipLaunchKernelGGL((k_combine<k, W64, W32, D2>), grid, dim3(256), 0, st, base, c, h, out64, out32, \
                         out2, g.epm);                                                                 \
      break;
    NSK_COMBINE(0) NSK_COMBINE(1) NSK_COMBINE(2) NSK_COMBINE(3) NSK_COMBINE(4)
    NSK_COMBINE(5) NSK_COMBINE(6) NSK_COMBINE(7) NSK_COMBINE(8) NSK_COMBINE(9)
#undef NSK_COMBINE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename BT>
static hipError_t combine_s32_from(const Geom& g, const BT* base, const Combo& c, const double* h, float2* out32,
                                   hipStream_t st) {
  if (!base || !out32) return hipErrorInvalidValue;
  for (int j = 0; j < c.nterms; ++j)
    if (!c.src32[j]) return hipErrorInvalidValue;
  const dim3 grid = member_grid(g.epm, g.batch);
  switch (c.nterms) {
#define NSK_COMBINE(k)                                                                                  \
    case k:                                                                                             \
      hipLaunchKernelGGL((k_combine_s32<k, BT>), grid, dim3(256), 0, st, base, c, h, out32, g.epm); \
      break;
    NSK_COMBINE(1) NSK_COMBINE(2) NSK_COMBINE(3) NSK_COMBINE(4) NSK_COMBINE(5)
    NSK_COMBINE(6) NSK_COMBINE(7) NSK_COMBINE(8) NSK_COMBINE(9)
#undef NSK_COMBINE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t combine_s32(const Geom& g, const double2* base, const Combo& c, const double* h, float2* out32,
                       hipStream_t st) {
  return combine_s32_from(g, base, c, h, out32, st);
}
hipError_t combine_s32(const Geom& g, const float2* base, const Combo& c, const double* h, float2* out32,
                       hipStream_t st) {
  return combine_s32_from(g, base, c, h, out32, st);
}

hipError_t combine(const Geom& g, const double2* base, const Combo& c, const double* h,
                   double2* out, hipStream_t st) {
  return combine_to<true, false, false>(g, base, c, h, out, nullptr, nullptr, st);
}

hipError_t combine2(const Geom& g, const double2* base, const Combo& c, const double* h, double2* out64,
                    float2* out32, double2* out2, hipStream_t st) {
  if (out2) {
    if (out64 && out32) return combine_to<true, true, true>(g, base, c, h, out64, out32, out2, st);
    if (out64) return combine_to<true, false, true>(g, base, c, h, out64, nullptr, out2, st);
    return hipErrorInvalidValue;               // the delta part comes with the last stage only
  }
  if (out64 && out32) return combine_to<true, true, false>(g, base, c, h, out64, out32, nullptr, st);
  if (out32) return combine_to<false, true, false>(g, base, c, h, nullptr, out32, nullptr, st);
  return combine_to<true, false, false>(g, base, c, h, out64, nullptr, nullptr, st);
}

__global__ void k_pack(const double2* __restrict__ full, double2* __restrict__ compact, Geom g,
                       long long total) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const long long m = i / g.epm, q = i - m * g.epm;
    const Modes md = decode(g, q);
    compact[i] = full[(m * g.ncomp + md.c) * g.full + full_offset(g, md)];
  }
}

hipError_t pack_state(const Geom& g, const double2* full, double2* compact, hipStream_t st) {
  const long long total = g.epm * g.batch;
  hipLaunchKernelGGL(k_pack, dim3(grid_for(total, 256)), dim3(256), 0, st, full, compact, g, total);
  return hipGetLastError();
}

__global__ void k_unpack(const double2* __restrict__ compact, double2* __restrict__ full, Geom g,
                         long long total) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long nh = g.nf / 2 + 1;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const long long mc = i / g.full, q = i - mc * g.full;       // member*ncomp + c
    const int kx = (int)(q % nh);
    const long long r = q / nh;
    const int iy = (int)(r % g.nf);
    const int iz = (int)(r / g.nf);                            // 0 in 2D
    const int ky = iy < g.nf / 2 ? iy : iy - g.nf;
    const int kz = iz < g.nf / 2 ? iz : iz - g.nf;
    const bool keep = kx <= g.K && ky <= g.K && -ky <= g.K && (g.dim == 2 || (kz <= g.K && -kz <= g.K));
    double2 v = make_double2(0.0, 0.0);
    if (keep) {
      const long long m = mc / g.ncomp, c = mc - m * g.ncomp;
      const int kyp = ky >= 0 ? ky : ky + g.Kf;
      long long off = (long long)kyp * g.Kx + kx;
      if (g.dim == 3) off += (long long)(kz >= 0 ? kz : kz + g.Kf) * g.Kf * g.Kx;
      v = compact[m * g.epm + c * g.mr + off];
    }
    full[i] = v;
  }
}

hipError_t unpack_state(const Geom& g, const double2* compact, double2* full, hipStream_t st) {
  const long long total = g.full * g.ncomp * g.batch;
  hipLaunchKernelGGL(k_unpack, dim3(grid_for(total, 256)), dim3(256), 0, st, compact, full, g, total);
  return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
constexpr int RBS = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Blocks per member: eight elements per thread (a thread takes every
// component of its modes, so about three modes per thread), at most 1024
// blocks.  Measured with events around the reduction and its final sum: at
// 1024^2 in 2D 343 blocks take 21.5 us and at 128^3 456 blocks 23.5 us, where
// 1024 blocks (one mode per thread, each block paying the 22-sum epilogue for
// little load work) took 24.7 and 27.2 us.  The count depends on the member
// size only, so a member's sums are the same alone or in an ensemble.
static int reduce_blocks(const Geom& g) {
  long long nb = (g.epm + (long long)RBS * 8 - 1) / ((long long)RBS * 8);
  if (nb < 1) nb = 1;
  if (nb > 1024) nb = 1024;
  return (int)nb;
}

size_t reduce_scratch_bytes(const Geom& g) {
  return (size_t)reduce_blocks(g) * g.batch * NRED * sizeof(double);
}

// Partial sums of one member (blockIdx.y) over a fixed set of modes.  N and
// DIM are compile-time so that decoding a mode index into (kz', ky', kx)
// divides by constants; NT >= 0 is the number of error terms (loads all in
// flight), NT < 0 takes it from the arguments.  A thread takes every
// component of its modes, so the mode's wavenumber, weight and shell are
// worked out once for all of them.
template <int N, int DIM, int NT>
__global__ __launch_bounds__(RBS) void k_reduce(ReduceArgs a, double* __restrict__ partials, int nblk,
                                                int nvel, int epm) {
  constexpr int K = (N - 1) / 3, KF = 2 * K + 1, KX = K + 1;
  constexpr int MRC = DIM == 3 ? KX * KF * KF : KX * KF;
  const int m = blockIdx.y;
  const int ncomp = epm / MRC;
  double acc[NRED];
#pragma unroll
  for (int q = 0; q < NRED; ++q) acc[q] = 0.0;
  const long long base = (long long)m * epm;
  const double hm = a.h ? a.h[m] : 0.0;
  const int nt = NT >= 0 ? NT : a.delta.nterms;
  for (int q = blockIdx.x * RBS + threadIdx.x; q < MRC; q += nblk * RBS) {
    const int kx = q % KX;
    int r = q / KX;
    const int kyp = r % KF;
    const int ky = kyp <= K ? kyp : kyp - KF;
    int kz = 0;
    if (DIM == 3) {
      const int kzp = r / KF;
      kz = kzp <= K ? kzp : kzp - KF;
    }
    const double w = kx == 0 ? 1.0 : 2.0;
    // every load of the mode first (all in flight together), then the sums
    constexpr int NC = 3;                          // at most three components
    constexpr int NTL = NT > 0 ? NT : 1;
    double2 un[NC], uo[NC], f[NC], v[NC][NTL];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const long long gi = base + (long long)(c < ncomp ? c : 0) * MRC + q;
      un[c] = ld_stream(a.un + gi);
      if (nt > 0) uo[c] = ld_stream(a.uo + gi);
      if (NT > 0) {
#pragma unroll
        for (int j = 0; j < NTL; ++j) v[c][j] = ld_stream(a.delta.src[j] + gi);
      }
      if (a.fk && c < nvel) f[c] = ld_stream(a.fk + gi);
    }
    double e = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (c >= ncomp) break;
      if (nt > 0) {
        double dx = 0.0, dy = 0.0;
        if (NT > 0) {
#pragma unroll
          for (int j = 0; j < NTL; ++j) {
            dx += a.delta.coef[j] * v[c][j].x;
            dy += a.delta.coef[j] * v[c][j].y;
          }
        } else {
          const long long gi = base + (long long)c * MRC + q;
          for (int j = 0; j < nt; ++j) {
            const double2 vv = ld_stream(a.delta.src[j] + gi);
            dx += a.delta.coef[j] * vv.x;
            dy += a.delta.coef[j] * vv.y;
          }
        }
        dx *= hm;
        dy *= hm;
        const double mo = sqrt(uo[c].x * uo[c].x + uo[c].y * uo[c].y);
        const double mn = sqrt(un[c].x * un[c].x + un[c].y * un[c].y);
        const double sc = a.atol + a.rtol * (mo > mn ? mo : mn);
        acc[c] += (dx * dx + dy * dy) / (sc * sc);
      }
      if (c < nvel) {
        e += 0.5 * w * (un[c].x * un[c].x + un[c].y * un[c].y);
        if (a.fk) acc[4] -= w * (un[c].x * f[c].x + un[c].y * f[c].y);
      }
    }
    acc[3] += e;
    const int k2i = kx * kx + ky * ky + kz * kz;
    const double kmag = sqrt((double)k2i);
    int bin = (int)floor((16.0 * kmag) / (double)(K > 0 ? K : 1));
    bin = bin > NBINS - 1 ? NBINS - 1 : bin;
#pragma unroll
    for (int b = 0; b < NBINS; ++b) acc[5 + b] += (b == bin) ? e : 0.0;
    acc[21] += (k2i > 0 && (double)k2i <= a.kf2) ? e : 0.0;
  }
  __shared__ double red[RBS / 64][NRED];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NRED; ++q) {
    const double s = wave_sum(acc[q]);
    if (lane == 0) red[wv][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < NRED) {
    double s = 0.0;
    for (int w = 0; w < RBS / 64; ++w) s += red[w][threadIdx.x];
    partials[((long long)m * nblk + blockIdx.x) * NRED + threadIdx.x] = s;
  }
}

// One block per (sum q, member): thread i adds partial blocks i, i + RBS, ...
// of sum q in order, then a fixed shuffle tree and a fixed-order sum over the
// waves.  Every sum is formed in the same order whatever the batch; spreading
// the NRED sums over blocks keeps each block's strided loads few (one member's
// partials are up to 1024 x NRED doubles, which one block read in 11-12 us).
__global__ __launch_bounds__(RBS) void k_reduce_final(const double* __restrict__ partials, int nblk,
                                                      double* __restrict__ out) {
  const int q = blockIdx.x, m = blockIdx.y;
  __shared__ double red[RBS / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double* p = partials + (long long)m * nblk * NRED + q;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += RBS) s += p[(long long)b * NRED];
  const double t = wave_sum(s);
  if (lane == 0) red[wv] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < RBS / 64; ++w) r += red[w];
    out[(long long)m * NRED + q] = r;
  }
}

template <int N, int DIM>
static void launch_reduce(const Geom& g, const ReduceArgs& a, double* partials, int nblk, int nvel,
                          hipStream_t st) {
  const dim3 grid(nblk, g.batch);
  const int epm = (int)g.epm;
  switch (a.delta.nterms) {
    case 0: hipLaunchKernelGGL((k_reduce<N, DIM, 0>), grid, dim3(RBS), 0, st, a, partials, nblk, nvel, epm); break;
    case 2: hipLaunchKernelGGL((k_reduce<N, DIM, 2>), grid, dim3(RBS), 0, st, a, partials, nblk, nvel, epm); break;
    case 6: hipLaunchKernelGGL((k_reduce<N, DIM, 6>), grid, dim3(RBS), 0, st, a, partials, nblk, nvel, epm); break;
    case 7: hipLaunchKernelGGL((k_reduce<N, DIM, 7>), grid, dim3(RBS), 0, st, a, partials, nblk, nvel, epm); break;
    default: hipLaunchKernelGGL((k_reduce<N, DIM, -1>), grid, dim3(RBS), 0, st, a, partials, nblk, nvel, epm);
  }
}

hipError_t reduce_state(const Geom& g, const ReduceArgs& a, double* partials, double* out,
                        hipStream_t st) {
  const int nblk = reduce_blocks(g);
  const int nvel = g.dim == 3 ? 3 : 2;
  if (g.epm > 0x7fffffffLL) return hipErrorInvalidValue;
  if (g.dim == 3) {
    switch (g.n) {
      case 8: launch_reduce<8, 3>(g, a, partials, nblk, nvel, st); break;
      case 16: launch_reduce<16, 3>(g, a, partials, nblk, nvel, st); break;
      case 32: launch_reduce<32, 3>(g, a, partials, nblk, nvel, st); break;
      case 64: launch_reduce<64, 3>(g, a, partials, nblk, nvel, st); break;
      case 128: launch_reduce<128, 3>(g, a, partials, nblk, nvel, st); break;
      case 256: launch_reduce<256, 3>(g, a, partials, nblk, nvel, st); break;
      case 512: launch_reduce<512, 3>(g, a, partials, nblk, nvel, st); break;
      case 1024: launch_reduce<1024, 3>(g, a, partials, nblk, nvel, st); break;
      case 24: launch_reduce<24, 3>(g, a, partials, nblk, nvel, st); break;
      case 48: launch_reduce<48, 3>(g, a, partials, nblk, nvel, st); break;
      case 96: launch_reduce<96, 3>(g, a, partials, nblk, nvel, st); break;
      case 192: launch_reduce<192, 3>(g, a, partials, nblk, nvel, st); break;
      case 384: launch_reduce<384, 3>(g, a, partials, nblk, nvel, st); break;
      case 768: launch_reduce<768, 3>(g, a, partials, nblk, nvel, st); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (g.n) {
      case 8: launch_reduce<8, 2>(g, a, partials, nblk, nvel, st); break;
      case 16: launch_reduce<16, 2>(g, a, partials, nblk, nvel, st); break;
      case 32: launch_reduce<32, 2>(g, a, partials, nblk, nvel, st); break;
      case 64: launch_reduce<64, 2>(g, a, partials, nblk, nvel, st); break;
      case 128: launch_reduce<128, 2>(g, a, partials, nblk, nvel, st); break;
      case 256: launch_reduce<256, 2>(g, a, partials, nblk, nvel, st); break;
      case 512: launch_reduce<512, 2>(g, a, partials, nblk, nvel, st); break;
      case 1024: launch_reduce<1024, 2>(g, a, partials, nblk, nvel, st); break;
      case 24: launch_reduce<24, 2>(g, a, partials, nblk, nvel, st); break;
      case 48: launch_reduce<48, 2>(g, a, partials, nblk, nvel, st); break;
      case 96: launch_reduce<96, 2>(g, a, partials, nblk, nvel, st); break;
      case 192: launch_reduce<192, 2>(g, a, partials, nblk, nvel, st); break;
      case 384: launch_reduce<384, 2>(g, a, partials, nblk, nvel, st); break;
      case 768: launch_reduce<768, 2>(g, a, partials, nblk, nvel, st); break;
      case 1536: launch_reduce<1536, 2>(g, a, partials, nblk, nvel, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  hipLaunchKernelGGL(k_reduce_final, dim3(NRED, g.batch), dim3(RBS), 0, st, partials, nblk, out);
  return hipGetLastError();
}

template <typename E>
__global__ void k_masked_copy(const E* __restrict__ src, E* __restrict__ dst,
                              const int* __restrict__ mask, long long epm, long long total) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
    if (mask[i / epm]) dst[i] = src[i];
}

// The band 0 < |k|^2 <= kf2 lies in the cube |k_j| <= kc = floor(sqrt(kf2)):
// one thread per (member, component, cube mode).
__global__ void k_scale_band(double2* __restrict__ u, const double* __restrict__ alpha, Geom g,
                             double kf2, int kc) {
  const int side = 2 * kc + 1;
  const long long per = (long long)side * side * (kc + 1);
  const long long total = per * g.ncomp * g.batch;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long long mc = i / per, q = i - mc * per;
  const int kx = (int)(q % (kc + 1));
  const long long r = q / (kc + 1);
  const int ky = (int)(r % side) - kc, kz = (int)(r / side) - kc;
  const int k2 = kx * kx + ky * ky + kz * kz;
  if (k2 == 0 || (double)k2 > kf2) return;
  const long long m = mc / g.ncomp, c = mc - m * g.ncomp;
  const long long off = ((long long)(kz >= 0 ? kz : kz + g.Kf) * g.Kf + (ky >= 0 ? ky : ky + g.Kf)) * g.Kx + kx;
  double2* p = u + m * g.epm + c * g.mr + off;
  const double a = alpha[m];
  *p = make_double2(p->x * a, p->y * a);
}

// Energy of the band 0 < |k|^2 <= kf2 per shell: one thread per member walks
// the band's cube |k_j| <= kc in a fixed order (a few hundred modes), so the
// sums are deterministic.  Shells as in k_reduce.
template <int N>
__global__ void k_band_bins(const double2* __restrict__ u, Geom g, double kf2, int kc, double* __restrict__ out) {
  constexpr int K = (N - 1) / 3, KF = 2 * K + 1, KX = K + 1;
  constexpr long long MRC = (long long)KX * KF * KF;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= g.batch) return;
  double acc[NBINS];
  for (int b = 0; b < NBINS; ++b) acc[b] = 0.0;
  const long long base = (long long)m * g.epm;
  const int kcc = kc < K ? kc : K;
  for (int kz = -kcc; kz <= kcc; ++kz)
    for (int ky = -kcc; ky <= kcc; ++ky)
      for (int kx = 0; kx <= kcc; ++kx) {
        const int k2 = kx * kx + ky * ky + kz * kz;
        if (k2 == 0 || (double)k2 > kf2) continue;
        const long long q = ((long long)(kz >= 0 ? kz : kz + KF) * KF + (ky >= 0 ? ky : ky + KF)) * KX + kx;
        const double w = kx == 0 ? 1.0 : 2.0;
        double e = 0.0;
        for (int c = 0; c < 3; ++c) {
          const double2 v = u[base + c * MRC + q];
          e += 0.5 * w * (v.x * v.x + v.y * v.y);
        }
        int bin = (int)floor((16.0 * sqrt((double)k2)) / (double)(K > 0 ? K : 1));
        bin = bin > NBINS - 1 ? NBINS - 1 : bin;
        acc[bin] += e;
      }
  for (int b = 0; b < NBINS; ++b) out[m * NBINS + b] = acc[b];
}

hipError_t band_bins(const Geom& g, const double2* u, double kf2, double* out, hipStream_t st) {
  const int kc = (int)floor(sqrt(kf2));
  const dim3 grid((g.batch + 63) / 64), blk(64);
  switch (g.n) {
    case 8: hipLaunchKernelGGL(k_band_bins<8>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 16: hipLaunchKernelGGL(k_band_bins<16>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 24: hipLaunchKernelGGL(k_band_bins<24>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 32: hipLaunchKernelGGL(k_band_bins<32>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 48: hipLaunchKernelGGL(k_band_bins<48>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 64: hipLaunchKernelGGL(k_band_bins<64>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 96: hipLaunchKernelGGL(k_band_bins<96>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 128: hipLaunchKernelGGL(k_band_bins<128>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 192: hipLaunchKernelGGL(k_band_bins<192>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 256: hipLaunchKernelGGL(k_band_bins<256>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 384: hipLaunchKernelGGL(k_band_bins<384>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 512: hipLaunchKernelGGL(k_band_bins<512>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 768: hipLaunchKernelGGL(k_band_bins<768>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    case 1024: hipLaunchKernelGGL(k_band_bins<1024>, grid, blk, 0, st, u, g, kf2, kc, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t scale_band(const Geom& g, double2* u, const double* alpha, double kf2, hipStream_t st) {
  int kc = (int)floor(sqrt(kf2));
  if (kc > g.K) kc = g.K;
  if (kc < 1) return hipSuccess;
  const long long total = (long long)(2 * kc + 1) * (2 * kc + 1) * (kc + 1) * g.ncomp * g.batch;
  hipLaunchKernelGGL(k_scale_band, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, u, alpha, g,
                     kf2, kc);
  return hipGetLastError();
}

__global__ void k_fill(double* __restrict__ p, double v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t fill(double* p, double v, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t masked_copy(const Geom& g, const double2* src, double2* dst, const int* mask_dev,
                       hipStream_t st) {
  const long long total = g.epm * g.batch;
  hipLaunchKernelGGL(k_masked_copy<double2>, dim3(grid_for(total, 256)), dim3(256), 0, st, src, dst,
                     mask_dev, g.epm, total);
  return hipGetLastError();
}

hipError_t masked_copy32(const Geom& g, const float2* src, float2* dst, const int* mask_dev, hipStream_t st) {
  const long long total = g.epm * g.batch;
  hipLaunchKernelGGL(k_masked_copy<float2>, dim3(grid_for(total, 256)), dim3(256), 0, st, src, dst,
                     mask_dev, g.epm, total);
  return hipGetLastError();
}

}  // namespace nsk
