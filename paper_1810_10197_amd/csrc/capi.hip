// C ABI of the solver (declared in include/ns.h): argument checking,
// workspace carving, the Runge--Kutta drivers of Sec. 2.2 and the host-side
// step-size controller of Sec. 2.2.1.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "ns_internal.hpp"
#include "../../include/ns.h"

using nsk::Combo;
using nsk::Geom;

namespace {

// Butcher tableaux as exact rationals p/q (each converted once, correctly
// rounded).  RK4: the classical method.  BS5: Appendix A.3, Eq. (8); its last
// row of A equals b (FSAL) and bh is the embedded error estimator b_hat.
struct Q { double p, q; };
constexpr double rq(Q v) { return v.p / v.q; }

const Q BS5_A[8][7] = {
    {{0, 1}},
    {{1, 6}},
    {{2, 27}, {4, 27}},
    {{183, 1372}, {-162, 343}, {1053, 1372}},
    {{68, 297}, {-4, 11}, {42, 143}, {1960, 3861}},
    {{597, 22528}, {81, 352}, {63099, 585728}, {58653, 366080}, {4617, 20480}},
    {{174197, 959244}, {-30942, 79937}, {8152137, 19744439}, {666106, 1039181}, {-29421, 29068},
     {482048, 414219}},
    {{587, 8064}, {0, 1}, {4440339, 15491840}, {24353, 124800}, {387, 44800}, {2152, 5985},
     {7267, 94080}},
};
const Q BS5_B[8] = {{587, 8064}, {0, 1}, {4440339, 15491840}, {24353, 124800},
                    {387, 44800}, {2152, 5985}, {7267, 94080}, {0, 1}};
const Q BS5_BH[8] = {{2479, 34992}, {0, 1}, {123, 416}, {612941, 3411720},
                     {43, 1440}, {2272, 6561}, {79937, 1113912}, {3293, 556956}};

constexpr int MAX_CONSEC_REJECT = 50;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool valid_config(const ns_config* c) {
  if (!c) return false;
  if (c->dim != 2 && c->dim != 3) return false;
  const int maxn = c->dim == 3 ? 512 : 1024;
  if (c->n < 8 || c->n > maxn || (c->n & (c->n - 1))) return false;
  if (c->batch < 1 || c->batch > 65535) return false;
  if (c->rhs_precision != NS_FP32 && c->rhs_precision != NS_FP64) return false;
  if (c->scalar != 0 && !(c->dim == 2 && c->scalar == 1)) return false;
  return true;
}

Geom make_geom(const ns_config* c) {
  Geom g;
  g.dim = c->dim;
  g.n = c->n;
  g.K = (c->n - 1) / 3;
  g.Kf = 2 * g.K + 1;
  g.Kx = g.K + 1;
  g.ncomp = c->dim == 3 ? 3 : (c->scalar ? 3 : 2);
  g.mr = (long long)g.Kx * g.Kf * (c->dim == 3 ? g.Kf : 1);
  g.epm = g.mr * g.ncomp;
  g.full = (long long)(c->n / 2 + 1) * c->n * (c->dim == 3 ? c->n : 1);
  g.batch = c->batch;
  return g;
}

struct Layout {
  size_t tw32, tw64, nu, h, red_out, mask, red_part, fields[10], a1, a2, total;
};

Layout make_layout(const ns_config* c) {
  const Geom g = make_geom(c);
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  L.tw32 = take(nsk::TWN_TABLE * 8);
  L.tw64 = take(nsk::TWN_TABLE * 16);
  L.nu = take((size_t)g.batch * 8);
  L.h = take((size_t)g.batch * 8);
  L.red_out = take((size_t)g.batch * nsk::NRED * 8);
  L.mask = take((size_t)g.batch * 4);
  L.red_part = take(nsk::reduce_scratch_bytes(g));
  for (int i = 0; i < 10; ++i) L.fields[i] = take((size_t)g.epm * g.batch * 16);
  const int fp64 = c->rhs_precision == NS_FP64;
  const size_t scratch = c->dim == 3 ? nsk::rhs3d_scratch_bytes(g, fp64) : nsk::rhs2d_scratch_bytes(g, fp64);
  const size_t cb = fp64 ? 16 : 8;
  const size_t a1 = c->dim == 3 ? (size_t)g.batch * 6 * g.n * g.Kf * g.Kx * cb : scratch / 2;
  L.a1 = take(a1);
  L.a2 = take(scratch - a1);
  L.total = off;
  return L;
}

}  // namespace

struct ns_solver {
  ns_config cfg;
  Geom g;
  hipStream_t st;
  int fp64;
  char* ws;
  Layout L;
  double* nu_d;
  double* h_d;
  double* red_out;
  double* red_part;
  int* mask_d;
  void* tw;          // twiddles in the rhs precision
  double2* u;        // committed state u_n (compact)
  double2* U;        // stage / candidate state
  double2* k[8];     // stage derivatives; k[0] = f(u_n) when k1_valid
  nsk::RhsBufs rb;
  bool have_state;
  bool k1_valid;
  std::vector<double> t;          // per-member time
  std::vector<double> hbuf;       // per-member step staging for uploads
  std::vector<int> maskbuf;
  std::vector<double> red_host;   // per-member reductions
  // kernel timing (ns_profile_start/stop)
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_id;
  size_t prof_used = 0;
};

static constexpr size_t PROF_POOL = 16384;

static void prof_hook(void* ctx, int id, int phase) {
  ns_solver* s = (ns_solver*)ctx;
  if (!s->prof_on || s->prof_used >= s->prof_ev.size()) return;
  if (phase == 0 && s->prof_used + 2 > s->prof_ev.size()) return;   // no room for the pair
  if (hipEventRecord(s->prof_ev[s->prof_used], s->st) != hipSuccess) return;
  s->prof_id[s->prof_used] = id * 2 + phase;
  ++s->prof_used;
}

#define NS_HIP(call)                         \
  do {                                       \
    if ((call) != hipSuccess) return NS_ERR_HIP; \
  } while (0)

static int rhs(ns_solver* s, const double2* U, double2* K) {
  nsk::RhsParams p;
  p.nu = s->nu_d;
  p.ri = s->cfg.ri;
  p.kappa = s->cfg.kappa;
  hipError_t e = s->g.dim == 3 ? nsk::rhs3d_compact(s->g, s->fp64, U, K, p, s->rb, s->tw, s->st)
                               : nsk::rhs2d_compact(s->g, s->fp64, U, K, p, s->rb, s->tw, s->st);
  return e == hipSuccess ? NS_OK : NS_ERR_HIP;
}

static int ensure_k1(ns_solver* s) {
  if (s->k1_valid) return NS_OK;
  int rc = rhs(s, s->u, s->k[0]);
  if (rc == NS_OK) s->k1_valid = true;
  return rc;
}

static int upload_h(ns_solver* s) {
  NS_HIP(hipMemcpyAsync(s->h_d, s->hbuf.data(), sizeof(double) * s->g.batch, hipMemcpyHostToDevice, s->st));
  return NS_OK;
}

static int fetch_reductions(ns_solver* s) {
  NS_HIP(hipMemcpyAsync(s->red_host.data(), s->red_out, sizeof(double) * nsk::NRED * s->g.batch,
                        hipMemcpyDeviceToHost, s->st));
  NS_HIP(hipStreamSynchronize(s->st));
  return NS_OK;
}

// One BS5 attempt with the per-member steps already in h_d.  Leaves the
// candidate u_{n+1} in U and f(u_{n+1}) in k[7]; errs receives err per member.
static int bs5_attempt(ns_solver* s, double atol, double rtol, std::vector<double>& errs) {
  int rc = ensure_k1(s);
  if (rc) return rc;
  for (int i = 1; i < 8; ++i) {
    Combo c;
    c.nterms = 0;
    for (int j = 0; j < i; ++j) {
      const double a = rq(BS5_A[i][j]);
      if (a == 0.0) continue;
      c.src[c.nterms] = s->k[j];
      c.coef[c.nterms] = a;
      ++c.nterms;
    }
    prof_hook(s, nsk::PROF_COMBINE, 0);
    NS_HIP(nsk::combine(s->g, s->u, c, s->h_d, s->U, s->st));
    prof_hook(s, nsk::PROF_COMBINE, 1);
    rc = rhs(s, s->U, s->k[i]);
    if (rc) return rc;
  }
  nsk::ReduceArgs ra;
  ra.uo = s->u;
  ra.un = s->U;
  ra.fk = s->k[7];
  ra.delta.nterms = 0;
  for (int j = 0; j < 8; ++j) {
    const double e = rq(BS5_B[j]) - rq(BS5_BH[j]);
    if (e == 0.0) continue;
    ra.delta.src[ra.delta.nterms] = s->k[j];
    ra.delta.coef[ra.delta.nterms] = e;
    ++ra.delta.nterms;
  }
  ra.h = s->h_d;
  ra.atol = atol;
  ra.rtol = rtol;
  prof_hook(s, nsk::PROF_REDUCE, 0);
  NS_HIP(nsk::reduce_state(s->g, ra, s->red_part, s->red_out, s->st));
  prof_hook(s, nsk::PROF_REDUCE, 1);
  rc = fetch_reductions(s);
  if (rc) return rc;
  const double M = (double)s->g.full;
  errs.assign(s->g.batch, 0.0);
  for (int m = 0; m < s->g.batch; ++m) {
    double e = 0.0;
    bool finite = true;
    for (int j = 0; j < s->g.ncomp; ++j) {
      const double v = std::sqrt(s->red_host[(size_t)m * nsk::NRED + j] / M);
      if (!std::isfinite(v)) finite = false;
      e = v > e ? v : e;
    }
    errs[m] = finite ? e : NAN;
  }
  return NS_OK;
}

// Commit the candidate for members with accept[m] != 0: u <- U, k1 <- k8.
static int commit(ns_solver* s, const std::vector<int>& accept) {
  int nacc = 0;
  for (int a : accept) nacc += a ? 1 : 0;
  if (nacc == 0) return NS_OK;
  if (nacc == s->g.batch) {
    std::swap(s->u, s->U);
    std::swap(s->k[0], s->k[7]);
    return NS_OK;
  }
  s->maskbuf = accept;
  NS_HIP(hipMemcpyAsync(s->mask_d, s->maskbuf.data(), sizeof(int) * s->g.batch, hipMemcpyHostToDevice, s->st));
  NS_HIP(nsk::masked_copy(s->g, s->U, s->u, s->mask_d, s->st));
  NS_HIP(nsk::masked_copy(s->g, s->k[7], s->k[0], s->mask_d, s->st));
  return NS_OK;
}

// Sec. 2.2.1 step-size factor; cap_at_one after a rejection.
static double step_factor(double err, bool cap_at_one) {
  if (!std::isfinite(err)) return 0.01;
  const double fmax = cap_at_one ? 1.0 : 2.0;
  if (err == 0.0) return fmax;
  double fac = 0.8 * std::pow(err, -0.2);
  if (fac < 0.01) fac = 0.01;
  if (fac > fmax) fac = fmax;
  return fac;
}

extern "C" {

size_t ns_workspace_bytes(const ns_config* cfg) {
  if (!valid_config(cfg)) return 0;
  return make_layout(cfg).total;
}

int ns_init(const ns_config* cfg, const double* nu_host, void* workspace, size_t workspace_bytes,
            void* stream, ns_solver** out) {
  if (!out) return NS_ERR_ARG;
  *out = nullptr;
  if (!valid_config(cfg) || !nu_host || !workspace) return NS_ERR_ARG;
  if (((uintptr_t)workspace) & 255) return NS_ERR_ARG;
  const Layout L = make_layout(cfg);
  if (workspace_bytes < L.total) return NS_ERR_NOMEM;
  ns_solver* s = new (std::nothrow) ns_solver();
  if (!s) return NS_ERR_NOMEM;
  s->cfg = *cfg;
  s->g = make_geom(cfg);
  s->st = (hipStream_t)stream;
  s->fp64 = cfg->rhs_precision == NS_FP64;
  s->ws = (char*)workspace;
  s->L = L;
  s->nu_d = (double*)(s->ws + L.nu);
  s->h_d = (double*)(s->ws + L.h);
  s->red_out = (double*)(s->ws + L.red_out);
  s->red_part = (double*)(s->ws + L.red_part);
  s->mask_d = (int*)(s->ws + L.mask);
  s->tw = s->ws + (s->fp64 ? L.tw64 : L.tw32);
  s->u = (double2*)(s->ws + L.fields[0]);
  s->U = (double2*)(s->ws + L.fields[1]);
  for (int i = 0; i < 8; ++i) s->k[i] = (double2*)(s->ws + L.fields[2 + i]);
  s->rb.a1 = s->ws + L.a1;
  s->rb.a2 = s->ws + L.a2;
  s->rb.hook = prof_hook;
  s->rb.hook_ctx = s;
  s->have_state = false;
  s->k1_valid = false;
  s->t.assign(cfg->batch, 0.0);
  s->hbuf.assign(cfg->batch, 0.0);
  s->maskbuf.assign(cfg->batch, 0);
  s->red_host.assign((size_t)cfg->batch * nsk::NRED, 0.0);
  // twiddles exp(-2 pi i m / TWN) from the host's double-precision libm
  std::vector<float> t32(2 * nsk::TWN_TABLE);
  std::vector<double> t64(2 * nsk::TWN_TABLE);
  const double two_pi = 2.0 * std::acos(-1.0);
  for (int m = 0; m < nsk::TWN_TABLE; ++m) {
    const double a = -two_pi * (double)m / (double)nsk::TWN_TABLE;
    t64[2 * m] = std::cos(a);
    t64[2 * m + 1] = std::sin(a);
    t32[2 * m] = (float)t64[2 * m];
    t32[2 * m + 1] = (float)t64[2 * m + 1];
  }
  bool ok = hipMemcpyAsync(s->ws + L.tw32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice, s->st) == hipSuccess &&
            hipMemcpyAsync(s->ws + L.tw64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice, s->st) == hipSuccess &&
            hipMemcpyAsync(s->nu_d, nu_host, sizeof(double) * cfg->batch, hipMemcpyHostToDevice, s->st) == hipSuccess &&
            hipStreamSynchronize(s->st) == hipSuccess;
  if (!ok) {
    delete s;
    return NS_ERR_HIP;
  }
  *out = s;
  return NS_OK;
}

int ns_set_nu(ns_solver* s, const double* nu_host) {
  if (!s || !nu_host) return NS_ERR_ARG;
  NS_HIP(hipMemcpyAsync(s->nu_d, nu_host, sizeof(double) * s->g.batch, hipMemcpyHostToDevice, s->st));
  NS_HIP(hipStreamSynchronize(s->st));
  s->k1_valid = false;
  return NS_OK;
}

int ns_set_state(ns_solver* s, const void* uhat) {
  if (!s || !uhat) return NS_ERR_ARG;
  NS_HIP(nsk::pack_state(s->g, (const double2*)uhat, s->u, s->st));
  s->have_state = true;
  s->k1_valid = false;
  return NS_OK;
}

int ns_get_state(ns_solver* s, void* uhat) {
  if (!s || !uhat) return NS_ERR_ARG;
  if (!s->have_state) return NS_ERR_STATE;
  NS_HIP(nsk::unpack_state(s->g, s->u, (double2*)uhat, s->st));
  return NS_OK;
}

int ns_rhs(ns_solver* s, const void* uhat, void* f) {
  if (!s || !uhat || !f || uhat == f) return NS_ERR_ARG;
  NS_HIP(nsk::pack_state(s->g, (const double2*)uhat, s->U, s->st));
  int rc = rhs(s, s->U, s->k[7]);
  if (rc) return rc;
  NS_HIP(nsk::unpack_state(s->g, s->k[7], (double2*)f, s->st));
  return NS_OK;
}

int ns_refresh_rhs(ns_solver* s) {
  if (!s) return NS_ERR_ARG;
  if (!s->have_state) return NS_ERR_STATE;
  s->k1_valid = false;
  return ensure_k1(s);
}

int ns_step_rk4(ns_solver* s, double h) {
  if (!s || !std::isfinite(h) || h < 0.0) return NS_ERR_ARG;
  if (!s->have_state) return NS_ERR_STATE;
  int rc = ensure_k1(s);
  if (rc) return rc;
  NS_HIP(nsk::fill(s->h_d, h, s->g.batch, s->st));
  // classical RK4: c = (0, 1/2, 1/2, 1), b = (1/6, 1/3, 1/3, 1/6)
  const double stage_a[3] = {0.5, 0.5, 1.0};
  for (int i = 1; i < 4; ++i) {
    Combo c;
    c.nterms = 1;
    c.src[0] = s->k[i - 1];
    c.coef[0] = stage_a[i - 1];
    NS_HIP(nsk::combine(s->g, s->u, c, s->h_d, s->U, s->st));
    rc = rhs(s, s->U, s->k[i]);
    if (rc) return rc;
  }
  Combo c;
  c.nterms = 4;
  const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  for (int j = 0; j < 4; ++j) {
    c.src[j] = s->k[j];
    c.coef[j] = b[j];
  }
  NS_HIP(nsk::combine(s->g, s->u, c, s->h_d, s->U, s->st));
  std::swap(s->u, s->U);
  s->k1_valid = false;
  for (double& tm : s->t) tm += h;
  return NS_OK;
}

int ns_step_bs5(ns_solver* s, double h, double atol, double rtol, int flags, double* err_host) {
  if (!s || !std::isfinite(h) || h < 0.0 || !(atol >= 0.0) || !(rtol >= 0.0) || atol + rtol <= 0.0)
    return NS_ERR_ARG;
  if (!s->have_state) return NS_ERR_STATE;
  NS_HIP(nsk::fill(s->h_d, h, s->g.batch, s->st));
  std::vector<double> errs;
  int rc = bs5_attempt(s, atol, rtol, errs);
  if (rc) return rc;
  std::vector<int> acc(s->g.batch);
  bool any_rej = false;
  for (int m = 0; m < s->g.batch; ++m) {
    acc[m] = (flags & NS_FORCE_COMMIT) || (std::isfinite(errs[m]) && errs[m] <= 1.0);
    if (acc[m]) s->t[m] += h;
    else any_rej = true;
    if (err_host) err_host[m] = errs[m];
  }
  rc = commit(s, acc);
  if (rc) return rc;
  return any_rej ? NS_STEP_REJECTED : NS_OK;
}

int ns_integrate(ns_solver* s, double t_end, double h0, double atol, double rtol, int controller,
                 ns_stats* stats_host) {
  if (!s || !std::isfinite(t_end) || !(h0 > 0.0) || !(atol >= 0.0) || !(rtol >= 0.0) || atol + rtol <= 0.0)
    return NS_ERR_ARG;
  if (controller != NS_CTRL_PI) return NS_ERR_UNSUPPORTED;
  if (!s->have_state) return NS_ERR_STATE;
  const int B = s->g.batch;
  std::vector<double> h(B, h0), hc(B, 0.0), errs;
  std::vector<int> prev_rej(B, 0), consec(B, 0), acc(B, 0), last(B, 0), done(B, 0);
  std::vector<ns_stats> st(B);
  for (int m = 0; m < B; ++m) {
    st[m] = ns_stats{s->t[m], h0, 0.0, 0, 0, 0};
    done[m] = s->t[m] >= t_end;
  }
  int status = NS_OK;
  for (;;) {
    bool any = false;
    for (int m = 0; m < B; ++m) {
      if (done[m]) { hc[m] = 0.0; continue; }
      any = true;
      last[m] = h[m] >= t_end - s->t[m];
      hc[m] = last[m] ? t_end - s->t[m] : h[m];
    }
    if (!any) break;
    const bool first = !s->k1_valid;
    s->hbuf = hc;
    int rc = upload_h(s);
    if (rc) return rc;
    rc = bs5_attempt(s, atol, rtol, errs);
    if (rc) return rc;
    for (int m = 0; m < B; ++m) {
      acc[m] = 0;
      if (done[m]) continue;
      st[m].n_rhs += first ? 8 : 7;
      const double err = errs[m];
      const bool ok = std::isfinite(err) && err <= 1.0;
      const double fac = step_factor(err, ok && prev_rej[m]);
      st[m].last_err = err;
      if (ok) {
        acc[m] = 1;
        s->t[m] = last[m] ? t_end : s->t[m] + hc[m];
        prev_rej[m] = 0;
        consec[m] = 0;
        st[m].n_accept++;
        h[m] = hc[m] * fac;
        if (s->t[m] >= t_end) done[m] = 1;
      } else {
        prev_rej[m] = 1;
        st[m].n_reject++;
        h[m] = hc[m] * fac;
        if (++consec[m] >= MAX_CONSEC_REJECT) {
          done[m] = 1;
          status = NS_ERR_STEPFAIL;
        }
      }
    }
    rc = commit(s, acc);
    if (rc) return rc;
  }
  if (stats_host) {
    for (int m = 0; m < B; ++m) {
      st[m].t = s->t[m];
      st[m].h_next = h[m];
      stats_host[m] = st[m];
    }
  }
  return status;
}

int ns_get_time(ns_solver* s, double* t_host) {
  if (!s || !t_host) return NS_ERR_ARG;
  for (int m = 0; m < s->g.batch; ++m) t_host[m] = s->t[m];
  return NS_OK;
}

int ns_set_time(ns_solver* s, const double* t_host) {
  if (!s || !t_host) return NS_ERR_ARG;
  for (int m = 0; m < s->g.batch; ++m) s->t[m] = t_host[m];
  return NS_OK;
}

int ns_diagnostics(ns_solver* s, double* energy_host, double* dissipation_host, double* shells_host) {
  if (!s) return NS_ERR_ARG;
  if (!s->have_state) return NS_ERR_STATE;
  int rc = ensure_k1(s);
  if (rc) return rc;
  nsk::ReduceArgs ra;
  ra.uo = nullptr;
  ra.un = s->u;
  ra.fk = s->k[0];
  ra.delta.nterms = 0;
  ra.h = nullptr;
  ra.atol = ra.rtol = 0.0;
  NS_HIP(nsk::reduce_state(s->g, ra, s->red_part, s->red_out, s->st));
  rc = fetch_reductions(s);
  if (rc) return rc;
  for (int m = 0; m < s->g.batch; ++m) {
    const double* r = s->red_host.data() + (size_t)m * nsk::NRED;
    if (energy_host) energy_host[m] = r[3];
    if (dissipation_host) dissipation_host[m] = r[4];
    if (shells_host)
      for (int b = 0; b < nsk::NBINS; ++b) shells_host[(size_t)m * nsk::NBINS + b] = r[5 + b];
  }
  return NS_OK;
}

int ns_profile_start(ns_solver* s) {
  if (!s) return NS_ERR_ARG;
  if (s->prof_ev.empty()) {
    s->prof_ev.resize(PROF_POOL);
    s->prof_id.resize(PROF_POOL);
    for (auto& e : s->prof_ev)
      if (hipEventCreate(&e) != hipSuccess) return NS_ERR_HIP;
  }
  s->prof_used = 0;
  s->prof_on = true;
  return NS_OK;
}

int ns_profile_stop(ns_solver* s, ns_kernel_times* out) {
  if (!s || !out) return NS_ERR_ARG;
  s->prof_on = false;
  NS_HIP(hipStreamSynchronize(s->st));
  for (int i = 0; i < NS_NPROF; ++i) {
    out->ms[i] = 0.0;
    out->count[i] = 0;
  }
  int open_idx[NS_NPROF];
  for (int i = 0; i < NS_NPROF; ++i) open_idx[i] = -1;
  for (size_t k = 0; k < s->prof_used; ++k) {
    const int id = s->prof_id[k] / 2, ph = s->prof_id[k] % 2;
    if (ph == 0) {
      open_idx[id] = (int)k;
    } else if (open_idx[id] >= 0) {
      float ms = 0.0f;
      NS_HIP(hipEventElapsedTime(&ms, s->prof_ev[open_idx[id]], s->prof_ev[k]));
      out->ms[id] += ms;
      out->count[id] += 1;
      open_idx[id] = -1;
    }
  }
  s->prof_used = 0;
  return NS_OK;
}

const char* ns_strerror(int status) {
  switch (status) {
    case NS_OK: return "ok";
    case NS_STEP_REJECTED: return "step rejected (error estimate above tolerance)";
    case NS_ERR_ARG: return "invalid argument or configuration";
    case NS_ERR_HIP: return "HIP runtime error";
    case NS_ERR_NOMEM: return "workspace too small";
    case NS_ERR_NONFINITE: return "non-finite value in a reduction";
    case NS_ERR_STEPFAIL: return "too many consecutive rejected steps";
    case NS_ERR_UNSUPPORTED: return "size or mode not supported";
    case NS_ERR_STATE: return "call out of order (state not set)";
    default: return "unknown status";
  }
}

void ns_free(ns_solver* s) {
  if (!s) return;
  for (auto& e : s->prof_ev) (void)hipEventDestroy(e);
  delete s;
}

}  // extern "C"
