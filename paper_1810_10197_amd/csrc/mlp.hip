// Learned step-size proposer: a 20-64-64-1 tanh network, FP32, hand-written
// forward, backward and Adam kernels.  The paper's discussion (Sec. 4) expects
// better step-size controllers than the elementary one of Sec. 2.2.1 to help;
// the network proposes log(h_next / h) from the state's shell spectrum and
// the recent error estimates, and the embedded error estimate still accepts or
// rejects every step.
//
// Features (20): log10(E_b / E + 1e-30) for the 16 shell energies E_b of the
// diagnostics reduction, then log10(max(err, 1e-30)) of the last four accepted
// error estimates (oldest first, padded with 1.0).  They are normalised with
// per-feature mean and scale stored after the parameters.
//
// Parameter vector (floats): W1 [64][20], b1 [64], W2 [64][64], b2 [64],
// W3 [64], b3 [1]  (5569), then mean [20], scale [20]  (5609 in total).
#include "ns_internal.hpp"

namespace nsk {

constexpr int MI = 20, MH = 64;
constexpr int OW1 = 0, OB1 = OW1 + MH * MI, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH,
              OB3 = OW3 + MH, ONP = OB3 + 1, OMEAN = ONP, OSCALE = OMEAN + MI;
static_assert(ONP == MLP_NPARAM && OSCALE + MI == MLP_NWEIGHTS, "parameter layout");

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Forward pass of one sample by one 64-thread block; returns y on thread 0
// and leaves the activations in a1s / a2s (LDS) and zs (normalised input).
__device__ __forceinline__ float mlp_forward_block(const float* __restrict__ w, const float* x, float* zs,
                                                   float* a1s, float* a2s) {
  const int j = threadIdx.x;
  if (j < MI) zs[j] = (x[j] - w[OMEAN + j]) / w[OSCALE + j];
  __syncthreads();
  float s = w[OB1 + j];
  for (int i = 0; i < MI; ++i) s += w[OW1 + j * MI + i] * zs[i];
  a1s[j] = tanhf(s);
  __syncthreads();
  s = w[OB2 + j];
  for (int i = 0; i < MH; ++i) s += w[OW2 + j * MH + i] * a1s[i];
  const float a2 = tanhf(s);
  a2s[j] = a2;
  const float y = wave_sum_f(w[OW3 + j] * a2);
  __syncthreads();
  return y + w[OB3];
}

// Per member: features of the candidate state from the reduction output
// (shells, energy, error sums) and the previous accepted errors; optionally the
// network's proposal.  One 64-thread block per member.
__global__ __launch_bounds__(64) void k_mlp_propose(const double* __restrict__ red,
                                                    const double* __restrict__ errhist, double M,
                                                    int ncomp, const float* __restrict__ w, int infer,
                                                    float* __restrict__ xout, float* __restrict__ yout,
                                                    const double* __restrict__ bandbins, double e0) {
  const int m = blockIdx.x, j = threadIdx.x;
  __shared__ float xs[MI], zs[MI], a1s[MH], a2s[MH];
  const double* r = red + (long long)m * NRED;
  if (j < 16) {
    double e = r[3], sb = r[5 + j];
    if (bandbins) {
      // the state after the forcing: the band's modes scaled by alpha
      const double eb = r[21];
      if (eb > 0.0) {
        const double rest = e0 - (e - eb);
        const double a2 = (rest > 0.0 ? rest : 0.0) / eb;
        sb += (a2 - 1.0) * bandbins[m * 16 + j];
        e += (a2 - 1.0) * eb;
      }
    }
    e = e > 1e-300 ? e : 1e-300;
    xs[j] = (float)log10(sb / e + 1e-30);
  } else if (j < 19) {
    const double v = errhist[m * 3 + (j - 16)];
    xs[j] = (float)log10(v > 1e-30 ? v : 1e-30);
  } else if (j == 19) {
    double err = 0.0;
    for (int c = 0; c < ncomp; ++c) {
      const double v = sqrt(r[c] / M);
      err = v > err ? v : err;
    }
    xs[j] = (float)log10(err > 1e-30 ? err : 1e-30);
  }
  __syncthreads();
  if (j < MI) xout[m * MI + j] = xs[j];
  if (!infer) return;
  const float y = mlp_forward_block(w, xs, zs, a1s, a2s);
  if (j == 0) yout[m] = y;
}

// Inference on explicit raw feature rows x [n][20] -> y [n].
__global__ __launch_bounds__(64) void k_mlp_forward(const float* __restrict__ w, const float* __restrict__ x,
                                                    float* __restrict__ y) {
  __shared__ float zs[MI], a1s[MH], a2s[MH];
  const float v = mlp_forward_block(w, x + (long long)blockIdx.x * MI, zs, a1s, a2s);
  if (threadIdx.x == 0) y[blockIdx.x] = v;
}

// Training, step 1: forward and backward of one sample per block.  Writes
// the per-sample factors the gradient needs: z [20], a1 [64], a2 [64],
// dz1 [64], dz2 [64] and dy (= dL/dy = 2 (y - t) / n) into act[s][AS].
constexpr int AS = MI + 4 * MH + 2;
__global__ __launch_bounds__(64) void k_mlp_sample_grad(const float* __restrict__ w, const float* __restrict__ xs_all,
                                                        const float* __restrict__ ts, const int* __restrict__ rows,
                                                        int n, float* __restrict__ act) {
  const int s = blockIdx.x, j = threadIdx.x;
  const int row = rows ? rows[s] : s;
  __shared__ float zs[MI], a1s[MH], a2s[MH], dz2s[MH];
  const float y = mlp_forward_block(w, xs_all + (long long)row * MI, zs, a1s, a2s);
  const float res = __shfl(y, 0, 64) - ts[row];
  const float dy = 2.0f * res / (float)n;
  const float a2 = a2s[j], a1 = a1s[j];
  const float dz2 = dy * w[OW3 + j] * (1.0f - a2 * a2);
  dz2s[j] = dz2;
  __syncthreads();
  float da1 = 0.0f;
  for (int k = 0; k < MH; ++k) da1 += dz2s[k] * w[OW2 + k * MH + j];
  const float dz1 = da1 * (1.0f - a1 * a1);
  float* o = act + (long long)s * AS;
  if (j < MI) o[j] = zs[j];
  o[MI + j] = a1;
  o[MI + MH + j] = a2;
  o[MI + 2 * MH + j] = dz1;
  o[MI + 3 * MH + j] = dz2;
  if (j == 0) {
    o[MI + 4 * MH] = dy;
    o[MI + 4 * MH + 1] = res * res;
  }
}

// Training, step 2: each thread owns one parameter and sums its gradient over
// the samples in order (deterministic); thread ONP sums the loss.
__global__ void k_mlp_reduce_grad(const float* __restrict__ act, int n, float* __restrict__ grad,
                                  float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > ONP) return;
  float g = 0.0f;
  for (int s = 0; s < n; ++s) {
    const float* o = act + (long long)s * AS;
    const float* z = o;
    const float* a1 = o + MI;
    const float* a2 = o + MI + MH;
    const float* dz1 = o + MI + 2 * MH;
    const float* dz2 = o + MI + 3 * MH;
    const float dy = o[MI + 4 * MH];
    float v;
    if (p < OB1) v = dz1[p / MI] * z[p % MI];
    else if (p < OW2) v = dz1[p - OB1];
    else if (p < OB2) v = dz2[(p - OW2) / MH] * a1[(p - OW2) % MH];
    else if (p < OW3) v = dz2[p - OB2];
    else if (p < OB3) v = dy * a2[p - OW3];
    else if (p == OB3) v = dy;
    else v = o[MI + 4 * MH + 1];                 // p == ONP: squared residual
    g += v;
  }
  if (p < ONP) grad[p] = g;
  else loss[0] = g / (float)n;
}

// Training, step 3: Adam (beta1 = 0.9, beta2 = 0.999, eps = 1e-8), step t >= 1.
__global__ void k_mlp_adam(float* __restrict__ w, const float* __restrict__ grad, float* __restrict__ mom,
                           float* __restrict__ vel, float lr, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ONP) return;
  const float g = grad[p];
  const float m = 0.9f * mom[p] + 0.1f * g;
  const float v = 0.999f * vel[p] + 0.001f * g * g;
  mom[p] = m;
  vel[p] = v;
  const float mh = m / bc1, vh = v / bc2;
  w[p] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

// Minibatch rows from a counter-based generator: splitmix64 (Steele, Lea &
// Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) of
// seed + iteration * batch + sample, reduced modulo the row count.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void k_mlp_rows(int* __restrict__ rows, int n, unsigned long long seed, long long iter, int nrows) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  rows[s] = (int)(splitmix64(seed + (unsigned long long)(iter * n + s)) % (unsigned long long)nrows);
}

// Feature statistics over the collected rows (mean, population std clamped
// below at 1e-6), one thread per feature, rows summed in order.
__global__ void k_mlp_stats(float* __restrict__ w, const float* __restrict__ x, int nrows) {
  const int f = threadIdx.x;
  if (f >= MI) return;
  double s = 0.0, s2 = 0.0;
  for (int r = 0; r < nrows; ++r) {
    const double v = x[(long long)r * MI + f];
    s += v;
    s2 += v * v;
  }
  const double mean = s / nrows;
  double var = s2 / nrows - mean * mean;
  var = var > 0.0 ? var : 0.0;
  const double sd = sqrt(var);
  w[OMEAN + f] = (float)mean;
  w[OSCALE + f] = (float)(sd > 1e-6 ? sd : 1e-6);
}

// ---------------------------------------------------------------- host side
hipError_t mlp_propose(const double* red, const double* errhist, double M, int ncomp, const float* w,
                       int infer, float* xout, float* yout, int batch, const double* bandbins, double e0,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_propose, dim3(batch), dim3(64), 0, st, red, errhist, M, ncomp, w, infer, xout, yout,
                     bandbins, e0);
  return hipGetLastError();
}

hipError_t mlp_forward(const float* w, const float* x, float* y, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3(n), dim3(64), 0, st, w, x, y);
  return hipGetLastError();
}

size_t mlp_act_floats(int nmax) { return (size_t)nmax * AS; }

hipError_t mlp_grad(const float* w, const float* x, const float* t, const int* rows, int n, float* act,
                    float* grad, float* loss, hipStream_t st) {
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mlp_sample_grad, dim3(n), dim3(64), 0, st, w, x, t, rows, n, act);
  hipLaunchKernelGGL(k_mlp_reduce_grad, dim3((ONP + 1 + 255) / 256), dim3(256), 0, st, act, n, grad, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(float* w, const float* grad, float* mom, float* vel, float lr, long long t, hipStream_t st) {
  const float bc1 = (float)(1.0 - pow(0.9, (double)t));
  const float bc2 = (float)(1.0 - pow(0.999, (double)t));
  hipLaunchKernelGGL(k_mlp_adam, dim3((ONP + 255) / 256), dim3(256), 0, st, w, grad, mom, vel, lr, bc1, bc2);
  return hipGetLastError();
}

hipError_t mlp_rows(int* rows, int n, unsigned long long seed, long long iter, int nrows, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_rows, dim3((n + 255) / 256), dim3(256), 0, st, rows, n, seed, iter, nrows);
  return hipGetLastError();
}

hipError_t mlp_stats(float* w, const float* x, int nrows, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_stats, dim3(1), dim3(64), 0, st, w, x, nrows);
  return hipGetLastError();
}

}  // namespace nsk
