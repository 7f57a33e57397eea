// Internal interfaces between the kernel translation units and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace nsk {

constexpr int TWN_TABLE = 3072;   // twiddle table length (exp(-2 pi i m / 3072))

// Grid geometry of one member.  Retained modes (2/3 rule): |k_j| <= K on every
// axis.  Compact spectral layout per component: [kz'][ky'][kx] (3D) or
// [ky'][kx] (2D) with kz', ky' in 0..2K (k = k' for k' <= K, k' - (2K+1)
// otherwise) and kx in 0..K.
struct Geom {
  int dim, n, K, Kf, Kx;   // n: grid of the physical-space products (the FFT length)
  int nf;                  // grid of the caller's half-spectrum layout (n, or 2n/3 when padded)
  int ncomp;          // state components: 3 (3D), 2 or 3 (2D)
  long long mr;       // retained modes per component
  long long epm;      // compact elements per member = ncomp * mr
  long long full;     // half-spectrum entries per component (nf^(d-1) (nf/2+1))
  int batch;
};

// Physical parameters seen by the RHS epilogue.
struct RhsParams {
  const double* nu;   // [batch]
  double ri, kappa;   // Boussinesq
  float2* k32 = nullptr;   // FP32 right-hand side: also write f rounded to FP32 (may be null)
  const int* active = nullptr;   // 3D: [batch] device flags, evaluate only members with a nonzero
                                 // flag (their f and copies are left as they are); null: all
};

// Optional timing hook called around every kernel launch: phase 0 before,
// 1 after, on the stream of the launch; id is one of the PROF_* values
// (PROF_SLAB brackets the whole y/x/y slab phase on the solver's stream).
typedef void (*HookFn)(void* ctx, int id, int phase, hipStream_t st);
enum { PROF_P1 = 0, PROF_P2, PROF_P3, PROF_P4, PROF_P5, PROF_COMBINE, PROF_REDUCE, PROF_OTHER, PROF_SLAB, PROF_RHS, NPROF };

// Scratch for one RHS evaluation (rhs precision T).
struct RhsBufs {
  void* a1;           // after the first inverse pass
  void* a2;           // after the second inverse pass
  HookFn hook;        // may be null
  void* hook_ctx;
  int variant[6];     // launch variant of each 3D pass, then the slab schedule (the autotuner's choice)
  hipStream_t side;   // second stream of the two-stream slab schedule (default priority)
  hipEvent_t fork, join;   // order `side` after / before the solver's stream
  int fine = 0;       // timing brackets: 0 passes, 1 also every y/x/y launch (on its
                      // own stream), 2 whole evaluations only (PROF_RHS)
};
constexpr int NVARIANT_COL = 5, NVARIANT_ROW = 2, NVARIANT_SLAB = 13;
constexpr int NVARIANT_Q3_2D = 7;    // 2D y-forward slot: Q3 variants 0-6
constexpr int NVARIANT_ROW2D = 4;   // 2D x-pass slot: B2 layout x (row per wavefront | row split)
// 3D slab schedule of the y/x/y passes, variant v: v < 5 one stream with
// slabs of n >> v planes; 5 <= v < 9 slabs of n >> (v - 4) planes alternating
// between two streams and two slab buffers, so that the passes of one slab
// overlap those of the next; 9, 10 one stream and 11, 12 two streams with the
// finer slabs n >> 5 and n >> 6 (for the large grids, whose planes are big).
// The default is the largest one-stream slab whose buffers fit in 96 MiB.
int slab_planes(const Geom& g, int v);
bool slab_two_streams(int v);
int default_slab_variant(const Geom& g, int fp64);

// k = f(U) on compact FP64 buffers for every member (3D: rhs3d.hip,
// 2D: rhs2d.hip).  tw: table of TWN twiddles in the rhs precision.  In 3D
// with an FP32 right-hand side the input may instead be U32, the same state
// rounded to FP32 (U is then ignored and may be null).
size_t rhs3d_scratch_bytes(const Geom& g, int fp64);
hipError_t rhs3d_compact(const Geom& g, int fp64, const double2* U, const float2* U32, double2* k,
                         const RhsParams& p, const RhsBufs& b, const void* tw, hipStream_t st);
size_t rhs2d_scratch_bytes(const Geom& g, int fp64);
hipError_t rhs2d_compact(const Geom& g, int fp64, const double2* U, const float2* U32, double2* k,
                         const RhsParams& p, const RhsBufs& b, const void* tw, hipStream_t st);

// ---- FP64 state kernels (step.hip) ----
constexpr int MAXTERMS = 9;
struct Combo {
  const double2* src[MAXTERMS];
  const float2* src32[MAXTERMS];   // FP32 copies of the sources (combine_s32)
  double coef[MAXTERMS];
  int nterms;
  double coef2[MAXTERMS];   // second combination of the same sources (combine2's out2)
};
// out = base + h_m * sum_j coef_j src_j (per member m; base may be null = 0);
// combine2 writes it to out64 and/or, rounded, to out32 (either may be null),
// and, if out2 is not null, sum_j coef2_j src_j to out2 from the same loads.
hipError_t combine(const Geom& g, const double2* base, const Combo& c, const double* h,
                   double2* out, hipStream_t st);
hipError_t combine2(const Geom& g, const double2* base, const Combo& c, const double* h, double2* out64,
                    float2* out32, double2* out2, hipStream_t st);

// Full <-> compact state conversions.
hipError_t pack_state(const Geom& g, const double2* full, double2* compact, hipStream_t st);
hipError_t unpack_state(const Geom& g, const double2* compact, double2* full, hipStream_t st);

// Fused reduction: embedded error sums (if delta != null), energy,
// dissipation (if fk != null) and shell spectrum of `un` per member.
// out[m*NRED + ...]: [0..2] sum |delta_j/sc_j|^2, [3] E, [4] eps, [5..20] shells,
// [21] energy of the forcing band 0 < |k|^2 <= kf2.
constexpr int NRED = 22;
constexpr int NBINS = 16;
struct ReduceArgs {
  const double2* uo;      // u_n (for sc), may be null when no error
  const double2* un;      // state whose diagnostics are taken (u_{n+1})
  const double2* fk;      // f(un) for the dissipation, may be null
  Combo delta;            // delta = h_m * sum coef_j src_j (nterms = 0: no error)
  const double* h;        // [batch]
  double atol, rtol;
  double kf2;             // forcing band |k|^2 <= kf2 (<= 0: none)
};
size_t reduce_scratch_bytes(const Geom& g);
hipError_t reduce_state(const Geom& g, const ReduceArgs& a, double* partials, double* out,
                        hipStream_t st);

// p[0..n) = v
hipError_t fill(double* p, double v, int n, hipStream_t st);

// u_hat <- alpha_m u_hat on the modes 0 < |k|^2 <= kf2 of every member
// (alpha per member, device array; 3D only).
hipError_t scale_band(const Geom& g, double2* u, const double* alpha, double kf2, hipStream_t st);

// Copy member slices src -> dst for members with mask[m] != 0 (host mask copied
// as a device array).
// out32 = FP32 rounding of base + h_m sum_j coef_j src32_j, accumulated in FP64
// from the FP32 copies of the sources (an FP32 stage input: its own rounding
// exceeds that of the copies by the factor |U| / (h sum |a_j k_j|)).
hipError_t combine_s32(const Geom& g, const double2* base, const Combo& c, const double* h, float2* out32,
                       hipStream_t st);
// The same from the FP32 rounding of the base (the committed state's FP32 copy).
hipError_t combine_s32(const Geom& g, const float2* base, const Combo& c, const double* h, float2* out32,
                       hipStream_t st);
hipError_t masked_copy32(const Geom& g, const float2* src, float2* dst, const int* mask_dev, hipStream_t st);
hipError_t masked_copy(const Geom& g, const double2* src, double2* dst, const int* mask_dev,
                       hipStream_t st);

// ---- step-size proposer network (mlp.hip) ----
constexpr int MLP_NPARAM = 5569;     // W1 64x20, b1, W2 64x64, b2, W3 1x64, b3
constexpr int MLP_NWEIGHTS = 5609;   // + feature mean [20] and scale [20]
// Features (and, with infer, the proposal) of every member from its
// reduction and error history.  With bandbins (non-null) the features are
// those of the state after the Sec. 3.3.1 forcing: bandbins[m][b] is the
// energy of the forcing band's modes in shell b, and the band is rescaled by
// alpha^2 = max(e0 - (E - E_band), 0) / E_band as the forcing does.
hipError_t mlp_propose(const double* red, const double* errhist, double M, int ncomp, const float* w,
                       int infer, float* xout, float* yout, int batch, const double* bandbins, double e0,
                       hipStream_t st);
// bandbins[m][b]: energy 1/2 w |u_hat|^2 of the modes 0 < |k|^2 <= kf2 of
// member m that fall in shell b (3D).
hipError_t band_bins(const Geom& g, const double2* u, double kf2, double* bandbins, hipStream_t st);
hipError_t mlp_forward(const float* w, const float* x, float* y, int n, hipStream_t st);
size_t mlp_act_floats(int nmax);
hipError_t mlp_grad(const float* w, const float* x, const float* t, const int* rows, int n, float* act,
                    float* grad, float* loss, hipStream_t st);
hipError_t mlp_adam(float* w, const float* grad, float* mom, float* vel, float lr, long long t,
                    hipStream_t st);
hipError_t mlp_rows(int* rows, int n, unsigned long long seed, long long iter, int nrows, hipStream_t st);
hipError_t mlp_stats(float* w, const float* x, int nrows, hipStream_t st);

// ---- device-side controller (control.hip) ----
struct CtlState {         // one entry per member, device memory
  double* t;              // time reached
  double* h;              // unclipped step proposed by the controller
  double* hc;             // step of the next attempt (clipped; 0 when done)
  double* hacc;           // step of the attempt just decided
  double* err;            // its error estimate
  double* errhist;        // [3] previous accepted errors, oldest first
  int* prev_rej;
  int* consec;
  int* done;
  int* last;              // the next attempt is clipped to t_end
  int* clipped;           // the attempt just decided was clipped
  int* accept;            // the attempt just decided is accepted
  int* fail;
  long long* nacc;
  long long* nrej;
  long long* nrhs;
};
hipError_t control_step(const CtlState& c, const double* red, double M, int ncomp, double t_end, int batch,
                        const float* mlp_y, int use_mlp, int stage_rhs, int extra_rhs, hipStream_t st);
hipError_t control_start(const CtlState& c, double t_end, int batch, hipStream_t st);
hipError_t collect_rows(const CtlState& c, const float* xnew, float* pend_x, double* pend_h, int* pend_ok,
                        float* ring_x, float* ring_y, long long* ring_count, int cap, int batch,
                        hipStream_t st);
hipError_t force_alpha(const double* red, const int* accept, double e0, double* alpha, int batch,
                       hipStream_t st);

}  // namespace nsk
