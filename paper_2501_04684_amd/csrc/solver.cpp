// Restarted GMRES over a bound plan (C ABI, declared in include/ubf.h):
// solves (sigma I + Z^F) x = b, Z^F the far-zone product of the plan, for
// nrhs independent right-hand sides whose products share each launch.
//
// The whole Krylov state lives in the caller's device workspace; the host
// only enqueues steps and reads a small status block (one pinned copy per
// step), so steps can be queued back to back without waiting.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "capi_internal.hpp"
#include "gmres.hpp"

using ubf::fail;
using ubf::hip_fail;
using ubf::ok;

struct ubf_gmres {
  ubf_plan* plan = nullptr;
  int R = 0, m = 0;
  int64_t n = 0;
  double sr = 0, si = 0, tol = 0;
  int32_t max_steps = 0;
  // device
  float2* V = nullptr;  // (m+1) blocks of [R][n]
  float2* W = nullptr;  // [R][n]
  double2* partial = nullptr;
  ubf::GmresState st{};
  ubf::GmresStatusRow* d_status = nullptr;
  // host
  ubf::GmresStatusRow* h_status = nullptr;  // pinned
  hipEvent_t ev = nullptr;
  const float2* b = nullptr;
  float2* x = nullptr;
  int j = 0;
  int32_t steps = 0, restarts = 0;
  bool started = false, finished = false, recorded = false;
  ~ubf_gmres() {
    if (ev) (void)hipEventDestroy(ev);
    if (h_status) (void)hipHostFree(h_status);
  }
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct GmresLayout {
  size_t V, W, partial, H, h1, h2, nrm, cs, sn, g, y, scale, bnorm, res, active, k, iters,
      status, total;
};

GmresLayout gmres_layout(int64_t n, int R, int m) {
  GmresLayout L{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t here = at;
    at = align256(at + bytes);
    return here;
  };
  const size_t vec = (size_t)R * n * sizeof(float2);
  L.V = take((size_t)(m + 1) * vec);
  L.W = take(vec);
  L.partial = take((size_t)ubf::kDotBlocks * R * (ubf::kMaxRestart + 1) * sizeof(double2));
  L.H = take((size_t)R * m * (m + 1) * sizeof(double2));
  L.h1 = take((size_t)R * (m + 1) * sizeof(double2));
  L.h2 = take((size_t)R * (m + 1) * sizeof(double2));
  L.nrm = take((size_t)R * sizeof(double2));
  L.cs = take((size_t)R * m * sizeof(double));
  L.sn = take((size_t)R * m * sizeof(double2));
  L.g = take((size_t)R * (m + 1) * sizeof(double2));
  L.y = take((size_t)R * m * sizeof(double2));
  L.scale = take((size_t)R * sizeof(double));
  L.bnorm = take((size_t)R * sizeof(double));
  L.res = take((size_t)R * sizeof(double));
  L.active = take((size_t)R * sizeof(int32_t));
  L.k = take((size_t)R * sizeof(int32_t));
  L.iters = take((size_t)R * sizeof(int32_t));
  L.status = take((size_t)R * sizeof(ubf::GmresStatusRow));
  L.total = at;
  return L;
}

float2* col(const ubf_gmres* s, int c) { return s->V + (int64_t)c * s->R * s->n; }

#define UBF_TRY(expr, what)                  \
  do {                                       \
    const int e_ = (expr);                   \
    if (e_) return hip_fail(e_, what);       \
  } while (0)

// Norm of `v` ([R][n]) into st.nrm (sum |v|^2 in the real part).
int norm_into(ubf_gmres* s, const float2* v, hipStream_t q) {
  UBF_TRY(ubf::launch_gmres_dots(v, 0, 1, v, s->n, s->R, s->partial, s->st.nrm, 1, q),
          "norm");
  return UBF_OK;
}

// New cycle from the residual already in V_0 (unnormalised).
int start_cycle(ubf_gmres* s, int first, hipStream_t q) {
  int e = norm_into(s, col(s, 0), q);
  if (e) return e;
  UBF_TRY(ubf::launch_gmres_cycle_start(s->st, s->R, first, s->tol, q), "cycle start");
  UBF_TRY(ubf::launch_gmres_scale(col(s, 0), col(s, 0), s->st.scale, s->n, s->R, q),
          "scale");
  s->j = 0;
  return UBF_OK;
}

// x += V y over the columns of the current cycle.
int close_cycle(ubf_gmres* s, hipStream_t q) {
  UBF_TRY(ubf::launch_gmres_backsolve(s->st, s->R, q), "backsolve");
  UBF_TRY(ubf::launch_gmres_combine(s->V, (int64_t)s->R * s->n, s->st, s->x, s->n, s->R, q),
          "combine");
  return UBF_OK;
}

int publish(ubf_gmres* s, hipStream_t q) {
  UBF_TRY(ubf::launch_gmres_status(s->st, s->R, s->d_status, q), "status");
  hipError_t e = hipMemcpyAsync(s->h_status, s->d_status,
                                (size_t)s->R * sizeof(ubf::GmresStatusRow),
                                hipMemcpyDeviceToHost, q);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (status)");
  e = hipEventRecord(s->ev, q);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord (status)");
  s->recorded = true;
  return UBF_OK;
}

int check_solver(ubf_gmres* s) {
  if (!s) return fail(UBF_EINVAL, "solver is NULL");
  const ubf::Plan& p = s->plan->p;
  if (!p.ws) return fail(UBF_ESTATE, "the solver's plan is no longer bound");
  if (p.nb_total() != s->n)
    return fail(UBF_ESTATE, "the plan's basis changed since the solver was created");
  // a plan bound again with a smaller max_nrhs has no room for R vectors
  if (s->R > p.max_nrhs)
    return fail(UBF_ESTATE, "the plan was bound again with max_nrhs below the solver's nrhs");
  return UBF_OK;
}

}  // namespace

extern "C" {

size_t ubf_gmres_workspace_bytes(const ubf_plan* plan, int32_t nrhs, int32_t restart) {
  if (!plan || nrhs < 1 || nrhs > ubf::kMaxGmresRhs || restart < 1 ||
      restart > ubf::kMaxRestart)
    return 0;
  return gmres_layout(plan->p.nb_total(), nrhs, restart).total;
}

int ubf_gmres_create(ubf_plan* plan, int32_t nrhs, int32_t restart, double sigma_re,
                     double sigma_im, double tol, int32_t max_steps, void* d_workspace,
                     size_t bytes, ubf_gmres** out) {
  if (!plan || !d_workspace || !out) return fail(UBF_EINVAL, "plan, workspace or out is NULL");
  if (nrhs < 1 || nrhs > ubf::kMaxGmresRhs)
    return fail(UBF_EINVAL, "nrhs must be in 1..64");
  if (restart < 1 || restart > ubf::kMaxRestart)
    return fail(UBF_EINVAL, "restart must be in 1..128");
  if (!(tol > 0.0) || !(tol < 1.0)) return fail(UBF_EINVAL, "tol must be in (0, 1)");
  if (max_steps < 1) return fail(UBF_EINVAL, "max_steps must be >= 1");
  if (((uintptr_t)d_workspace & 255) != 0)
    return fail(UBF_EINVAL, "workspace must be 256-byte aligned");
  if (!plan->p.ws) return fail(UBF_ESTATE, "plan is not bound to a workspace");
  if (nrhs > plan->p.max_nrhs)
    return fail(UBF_EINVAL, "nrhs exceeds the plan binding's max_nrhs");
  const int64_t n = plan->p.nb_total();
  const GmresLayout L = gmres_layout(n, nrhs, restart);
  if (bytes < L.total)
    return fail(UBF_ENOMEM, "solver workspace too small: need " + std::to_string(L.total) +
                                " bytes, got " + std::to_string(bytes));
  ubf_gmres* s = new (std::nothrow) ubf_gmres();
  if (!s) return fail(UBF_ENOMEM, "host allocation failed");
  s->plan = plan;
  s->R = nrhs;
  s->m = restart;
  s->n = n;
  s->sr = sigma_re;
  s->si = sigma_im;
  s->tol = tol;
  s->max_steps = max_steps;
  char* ws = (char*)d_workspace;
  s->V = (float2*)(ws + L.V);
  s->W = (float2*)(ws + L.W);
  s->partial = (double2*)(ws + L.partial);
  ubf::GmresState& st = s->st;
  st.m = restart;
  st.H = (double2*)(ws + L.H);
  st.h1 = (double2*)(ws + L.h1);
  st.h2 = (double2*)(ws + L.h2);
  st.nrm = (double2*)(ws + L.nrm);
  st.cs = (double*)(ws + L.cs);
  st.sn = (double2*)(ws + L.sn);
  st.g = (double2*)(ws + L.g);
  st.y = (double2*)(ws + L.y);
  st.scale = (double*)(ws + L.scale);
  st.bnorm = (double*)(ws + L.bnorm);
  st.res = (double*)(ws + L.res);
  st.active = (int32_t*)(ws + L.active);
  st.k = (int32_t*)(ws + L.k);
  st.iters = (int32_t*)(ws + L.iters);
  s->d_status = (ubf::GmresStatusRow*)(ws + L.status);
  hipError_t e = hipHostMalloc((void**)&s->h_status, (size_t)nrhs * sizeof(ubf::GmresStatusRow),
                               hipHostMallocDefault);
  if (e != hipSuccess) {
    s->h_status = nullptr;
    delete s;
    return hip_fail(e, "hipHostMalloc (status)");
  }
  std::memset(s->h_status, 0, (size_t)nrhs * sizeof(ubf::GmresStatusRow));
  e = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    s->ev = nullptr;
    delete s;
    return hip_fail(e, "hipEventCreate (status)");
  }
  *out = s;
  return ok();
}

int ubf_gmres_start(ubf_gmres* s, const void* d_b, void* d_x, void* hip_stream) {
  int e = check_solver(s);
  if (e) return e;
  if (!d_b || !d_x) return fail(UBF_EINVAL, "b or x is NULL");
  const size_t vec = (size_t)s->R * s->n * sizeof(float2);
  const char* pb = (const char*)d_b;
  const char* px = (const char*)d_x;
  if (pb < px + vec && px < pb + vec) return fail(UBF_EINVAL, "b and x overlap");
  hipStream_t q = (hipStream_t)hip_stream;
  s->b = (const float2*)d_b;
  s->x = (float2*)d_x;
  s->steps = 0;
  s->restarts = 0;
  s->finished = false;
  // x_0 = 0, so r_0 = b
  UBF_TRY(ubf::launch_gmres_zero(s->x, (int64_t)s->R * s->n, q), "zero x");
  hipError_t he = hipMemcpyAsync(col(s, 0), s->b, vec, hipMemcpyDeviceToDevice, q);
  if (he != hipSuccess) return hip_fail(he, "hipMemcpyAsync (start)");
  e = start_cycle(s, 1, q);
  if (e) return e;
  e = publish(s, q);
  if (e) return e;
  s->started = true;
  return ok();
}

int ubf_gmres_step(ubf_gmres* s, void* hip_stream) {
  int e = check_solver(s);
  if (e) return e;
  if (!s->started || s->finished) return fail(UBF_ESTATE, "solver not started or finished");
  hipStream_t q = (hipStream_t)hip_stream;
  const int R = s->R, j = s->j, ld = s->m + 1;
  const int64_t n = s->n, vs = (int64_t)R * n;
  // w = (sigma I + Z^F) v_j
  e = ubf::enqueue_mvm(s->plan->p, col(s, j), s->W, R, q, s->plan->next_events());
  if (e) return e;
  UBF_TRY(ubf::launch_gmres_add_shift(s->W, col(s, j), s->sr, s->si, vs, q), "shift");
  // two classical Gram-Schmidt passes against v_0..v_j
  UBF_TRY(ubf::launch_gmres_dots(s->V, vs, j + 1, s->W, n, R, s->partial, s->st.h1, ld, q),
          "dots");
  UBF_TRY(ubf::launch_gmres_update(s->V, vs, j + 1, s->st.h1, ld, s->W, n, R, q), "update");
  UBF_TRY(ubf::launch_gmres_dots(s->V, vs, j + 1, s->W, n, R, s->partial, s->st.h2, ld, q),
          "dots");
  UBF_TRY(ubf::launch_gmres_update(s->V, vs, j + 1, s->st.h2, ld, s->W, n, R, q), "update");
  e = norm_into(s, s->W, q);
  if (e) return e;
  UBF_TRY(ubf::launch_gmres_tail(s->st, R, j, s->tol, q), "arnoldi");
  UBF_TRY(ubf::launch_gmres_scale(col(s, j + 1), s->W, s->st.scale, n, R, q), "scale");
  s->j = j + 1;
  s->steps += 1;
  if (s->j == s->m) {  // restart: x += V y, r = b - A x
    e = close_cycle(s, q);
    if (e) return e;
    e = ubf::enqueue_mvm(s->plan->p, s->x, s->W, R, q, s->plan->next_events());
    if (e) return e;
    UBF_TRY(ubf::launch_gmres_residual(col(s, 0), s->b, s->x, s->W, s->sr, s->si, vs, q),
            "residual");
    e = start_cycle(s, 0, q);
    if (e) return e;
    s->restarts += 1;
  }
  e = publish(s, q);
  if (e) return e;
  return ok();
}

int ubf_gmres_poll(ubf_gmres* s, int32_t wait, ubf_gmres_status* out, double* rel_res) {
  if (!s || !out) return fail(UBF_EINVAL, "solver or out is NULL");
  std::memset(out, 0, sizeof(*out));
  out->steps = s->steps;
  out->restarts = s->restarts;
  if (!s->recorded) return fail(UBF_ESTATE, "solver not started");
  hipError_t e = wait ? hipEventSynchronize(s->ev) : hipEventQuery(s->ev);
  if (e == hipErrorNotReady) {
    out->ready = 0;
    return ok();
  }
  if (e != hipSuccess) return hip_fail(e, "status event");
  out->ready = 1;
  int active = 0;
  double worst = 0.0;
  for (int r = 0; r < s->R; ++r) {
    active += s->h_status[r].active ? 1 : 0;
    if (s->h_status[r].res > worst) worst = s->h_status[r].res;
    if (rel_res) rel_res[r] = s->h_status[r].res;
  }
  out->converged = active == 0 && worst <= s->tol ? 1 : 0;
  out->done = (active == 0 || s->steps >= s->max_steps) ? 1 : 0;
  out->max_rel_res = worst;
  return ok();
}

int ubf_gmres_finish(ubf_gmres* s, void* hip_stream) {
  int e = check_solver(s);
  if (e) return e;
  if (!s->started || s->finished) return fail(UBF_ESTATE, "solver not started or finished");
  e = close_cycle(s, (hipStream_t)hip_stream);
  if (e) return e;
  s->finished = true;
  return ok();
}

int ubf_gmres_norm_estimate(ubf_gmres* s, int32_t iters, uint64_t seed, void* hip_stream,
                            double* out) {
  int e = check_solver(s);
  if (e) return e;
  if (!out) return fail(UBF_EINVAL, "out is NULL");
  if (iters < 1 || iters > 100) return fail(UBF_EINVAL, "iters must be in 1..100");
  // Z^H Z v is formed as conj(Z conj(Z v)), which needs Z complex symmetric:
  // T = S^T (or the identity basis) with the operator table. An explicit T
  // or the networks of Sec. 3 (not linear) give another operator.
  if (s->plan->p.d_T)
    return fail(UBF_EINVAL, "norm estimate needs T = S^T; the plan has an explicit T");
  if (s->plan->p.hidden > 0)
    return fail(UBF_EINVAL, "norm estimate needs the operator table; the plan uses networks");
  hipStream_t q = (hipStream_t)hip_stream;
  const int64_t n = s->n;
  float2* v = col(s, 0);  // first right-hand-side row of two Krylov blocks
  float2* u = col(s, 1);
  s->started = false;     // the Krylov blocks are overwritten
  UBF_TRY(ubf::launch_gmres_rand(v, n, seed, q), "rand");
  UBF_TRY(ubf::launch_gmres_dots(v, 0, 1, v, n, 1, s->partial, s->st.nrm, 1, q), "norm");
  UBF_TRY(ubf::launch_gmres_inv_norm(s->st.nrm, s->st.scale, q), "inv norm");
  UBF_TRY(ubf::launch_gmres_scale(v, v, s->st.scale, n, 1, q), "scale");
  for (int it = 0; it < iters; ++it) {
    // u = conj(Z conj(Z v)) = Z^H Z v  (Z complex symmetric)
    e = ubf::enqueue_mvm(s->plan->p, v, s->W, 1, q, nullptr);
    if (e) return e;
    UBF_TRY(ubf::launch_gmres_conj(u, s->W, n, q), "conj");
    e = ubf::enqueue_mvm(s->plan->p, u, s->W, 1, q, nullptr);
    if (e) return e;
    UBF_TRY(ubf::launch_gmres_conj(u, s->W, n, q), "conj");
    // Rayleigh quotient v^H u (||v|| = 1), then v = u / ||u||
    UBF_TRY(ubf::launch_gmres_dots(v, 0, 1, u, n, 1, s->partial, s->st.h1, 1, q), "dots");
    UBF_TRY(ubf::launch_gmres_dots(u, 0, 1, u, n, 1, s->partial, s->st.nrm, 1, q), "norm");
    UBF_TRY(ubf::launch_gmres_inv_norm(s->st.nrm, s->st.scale, q), "inv norm");
    UBF_TRY(ubf::launch_gmres_scale(v, u, s->st.scale, n, 1, q), "scale");
  }
  double2 rq;
  hipError_t he = hipMemcpyAsync(&rq, s->st.h1, sizeof(rq), hipMemcpyDeviceToHost, q);
  if (he == hipSuccess) he = hipStreamSynchronize(q);
  if (he != hipSuccess) return hip_fail(he, "norm estimate readback");
  *out = std::sqrt(std::sqrt(rq.x * rq.x + rq.y * rq.y));
  return ok();
}

int ubf_gmres_set_shift(ubf_gmres* s, double sigma_re, double sigma_im) {
  if (!s) return fail(UBF_EINVAL, "solver is NULL");
  s->sr = sigma_re;
  s->si = sigma_im;
  return ok();
}

void ubf_gmres_destroy(ubf_gmres* s) { delete s; }

}  // extern "C"
