// Device-side step-size control (Sec. 2.2.1) for every ensemble member, so
// that a whole adaptive attempt -- stages, error norm, decision, commit --
// runs without the host and can be replayed as one HIP graph.
//
// Per member, after the fused reduction of an attempt with step hc:
//   err = max_j sqrt(sum_k |delta_j / sc_j|^2 / M)   (non-finite: reject)
//   fac = 0.8 err^(-1/5) clamped to [0.01, dmax], dmax = 1 if the attempt
//         is accepted right after a rejection, 2 otherwise; err = 0 gives dmax
//   accept iff err <= 1; the next step is hc * fac, or with the learned
//   proposer (after an accepted step) hc * clamp(exp(y), 0.7 fac, fac): the
//   proposer can only shorten a step, and 0.7 dmax > 1 keeps a wrong proposer
//   from holding the step down
//   the next attempt is clipped to land on t_end; 50 consecutive
//   rejections, or a step too small to advance t, stop the member.
#include "ns_internal.hpp"

namespace nsk {

__device__ __forceinline__ double step_factor_dev(double err, bool cap_at_one) {
  if (!isfinite(err)) return 0.01;
  const double fmax = cap_at_one ? 1.0 : 2.0;
  if (err == 0.0) return fmax;
  double fac = 0.8 * pow(err, -0.2);
  fac = fac < 0.01 ? 0.01 : fac;
  return fac > fmax ? fmax : fac;
}

__global__ void k_control(CtlState c, const double* __restrict__ red, double M, int ncomp, double t_end,
                          int batch, const float* __restrict__ mlp_y, int use_mlp, int stage_rhs,
                          int extra_rhs) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= batch) return;
  c.accept[m] = 0;
  if (c.done[m]) {
    c.hc[m] = 0.0;
    return;
  }
  const double* r = red + (long long)m * NRED;
  double err = 0.0;
  bool finite = true;
  for (int j = 0; j < ncomp; ++j) {
    const double v = sqrt(r[j] / M);
    if (!isfinite(v)) finite = false;
    err = v > err ? v : err;
  }
  if (!finite) err = NAN;
  const bool ok = finite && err <= 1.0;
  const bool prev_rej = c.prev_rej[m] != 0;
  const double hc = c.hc[m];
  double hnew = hc * step_factor_dev(err, ok && prev_rej);
  c.nrhs[m] += stage_rhs;                      // new stages of the attempt (FSAL first stage reused)
  c.err[m] = err;
  c.hacc[m] = hc;
  c.clipped[m] = c.last[m];
  if (ok) {
    c.t[m] = c.last[m] ? t_end : c.t[m] + hc;
    c.nacc[m] += 1;
    c.nrhs[m] += extra_rhs;                    // first stage recomputed after forcing
    if (use_mlp) {
      const float y = mlp_y[m];
      if (isfinite(y)) {
        // the proposer may only shorten the controller's step, by at most 30%
        const double fac = step_factor_dev(err, prev_rej);
        const double lo = 0.7 * fac, hi = fac;
        double g = exp((double)y);
        g = g < lo ? lo : (g > hi ? hi : g);
        hnew = hc * g;
      }
    }
    c.errhist[3 * m + 0] = c.errhist[3 * m + 1];
    c.errhist[3 * m + 1] = c.errhist[3 * m + 2];
    c.errhist[3 * m + 2] = err;
    c.prev_rej[m] = 0;
    c.consec[m] = 0;
    c.accept[m] = 1;
    if (c.t[m] >= t_end) c.done[m] = 1;
  } else {
    c.prev_rej[m] = 1;
    c.nrej[m] += 1;
    if (++c.consec[m] >= 50) {
      c.done[m] = 1;
      c.fail[m] = 1;
    }
  }
  c.h[m] = hnew;
  // a step that no longer advances t (t + h == t) can never reach t_end
  if (!c.done[m] && !(c.t[m] + hnew > c.t[m])) {
    c.done[m] = 1;
    c.fail[m] = 1;
  }
  if (!c.done[m]) {
    const int last = hnew >= t_end - c.t[m];
    c.last[m] = last;
    c.hc[m] = last ? t_end - c.t[m] : hnew;
  } else {
    c.hc[m] = 0.0;
  }
}

// Prepare the first attempt of every member (the controller's state is reset
// by the caller): clip h to t_end.
__global__ void k_control_start(CtlState c, double t_end, int batch) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= batch) return;
  c.done[m] = c.t[m] >= t_end ? 1 : 0;
  const double h = c.h[m];
  const int last = h >= t_end - c.t[m];
  c.last[m] = last;
  c.hc[m] = c.done[m] ? 0.0 : (last ? t_end - c.t[m] : h);
}

// Training rows from accepted steps: the features recorded after the previous
// accepted step and the label log(h_accepted / h_previous).  Steps clipped to
// t_end are not labels.  One thread walks the members in order, so the row
// order is deterministic.
__global__ void k_collect(CtlState c, const float* __restrict__ xnew, float* __restrict__ pend_x,
                          double* __restrict__ pend_h, int* __restrict__ pend_ok, float* __restrict__ ring_x,
                          float* __restrict__ ring_y, long long* __restrict__ ring_count, int cap, int batch) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  long long cnt = *ring_count;
  for (int m = 0; m < batch; ++m) {
    if (!c.accept[m]) continue;
    const double h = c.hacc[m];
    if (pend_ok[m] && !c.clipped[m] && h > 0.0 && pend_h[m] > 0.0) {
      const long long slot = cnt % cap;
      for (int f = 0; f < 20; ++f) ring_x[slot * 20 + f] = pend_x[m * 20 + f];
      ring_y[slot] = (float)log(h / pend_h[m]);
      ++cnt;
    }
    for (int f = 0; f < 20; ++f) pend_x[m * 20 + f] = xnew[m * 20 + f];
    pend_h[m] = h;
    pend_ok[m] = c.clipped[m] ? 0 : 1;
  }
  *ring_count = cnt;
}

// Forcing factor per accepted member: alpha = sqrt(max(E0 - (E - Eb), 0) / Eb)
// from the reduction of the committed state; 1 for the others.
__global__ void k_force_alpha(const double* __restrict__ red, const int* __restrict__ accept, double e0,
                              double* __restrict__ alpha, int batch) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= batch) return;
  const double* r = red + (long long)m * NRED;
  const double e = r[3], eb = r[21];
  double a = 1.0;
  if ((!accept || accept[m]) && eb > 0.0) {
    const double rest = e0 - (e - eb);
    a = sqrt((rest > 0.0 ? rest : 0.0) / eb);
  }
  alpha[m] = a;
}

hipError_t control_step(const CtlState& c, const double* red, double M, int ncomp, double t_end, int batch,
                        const float* mlp_y, int use_mlp, int stage_rhs, int extra_rhs, hipStream_t st) {
  hipLaunchKernelGGL(k_control, dim3((batch + 63) / 64), dim3(64), 0, st, c, red, M, ncomp, t_end, batch, mlp_y,
                     use_mlp, stage_rhs, extra_rhs);
  return hipGetLastError();
}

hipError_t control_start(const CtlState& c, double t_end, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_control_start, dim3((batch + 63) / 64), dim3(64), 0, st, c, t_end, batch);
  return hipGetLastError();
}

hipError_t collect_rows(const CtlState& c, const float* xnew, float* pend_x, double* pend_h, int* pend_ok,
                        float* ring_x, float* ring_y, long long* ring_count, int cap, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_collect, dim3(1), dim3(1), 0, st, c, xnew, pend_x, pend_h, pend_ok, ring_x, ring_y,
                     ring_count, cap, batch);
  return hipGetLastError();
}

hipError_t force_alpha(const double* red, const int* accept, double e0, double* alpha, int batch, hipStream_t st) {
  hipLaunchKernelGGL(k_force_alpha, dim3((batch + 63) / 64), dim3(64), 0, st, red, accept, e0, alpha, batch);
  return hipGetLastError();
}

}  // namespace nsk
