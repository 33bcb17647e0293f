// C ABI of the far-zone product (declared in include/ubf.h).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "capi_internal.hpp"
#include "kernels.hpp"
#include "networks.hpp"

namespace ubf {

namespace {
thread_local std::string g_last_error;
}  // namespace

int fail(int status, const std::string& why) {
  g_last_error = why;
  return status;
}

int ok() {
  g_last_error.clear();
  return UBF_OK;
}

int hip_fail(int err, const char* what) {
  return fail(UBF_EDEVICE, std::string(what) + ": " +
                               hipGetErrorString((hipError_t)err));
}

const std::string& last_error_text() { return g_last_error; }

// Stage 2 by the plan's networks when it has them, else by the operator
// table (the staged kernel for box sizes too wide for the register kernels).
int launch_stage2(const Plan& p, const float* P, float* part, int nrhs, hipStream_t s,
                  const StageEvents* ev) {
  if (p.hidden > 0) return launch_translate_cvfcnn(p, P, part, nrhs, s, ev);
  if (staged_translate_supported(p)) return launch_translate_staged(p, P, part, nrhs, s, ev);
  return launch_translate(p, P, part, nrhs, s, ev);
}

int enqueue_mvm(const Plan& p, const void* d_x, void* d_y, int32_t nrhs, hipStream_t s,
                hipEvent_t* ev) {
  const StageEvents st[3] = {{ev ? ev[0] : nullptr, ev ? ev[1] : nullptr},
                             {ev ? ev[2] : nullptr, ev ? ev[3] : nullptr},
                             {ev ? ev[4] : nullptr, ev ? ev[5] : nullptr}};
  int e = launch_aggregate(p, d_x, p.d_P, nrhs, s, ev ? &st[0] : nullptr);
  if (e) return hip_fail(e, "aggregate launch");
  e = launch_stage2(p, p.d_P, p.d_part, nrhs, s, ev ? &st[1] : nullptr);
  if (e) return hip_fail(e, "translate launch");
  e = launch_disaggregate(p, true, p.d_part, nullptr, d_y, nrhs, s, false,
                          ev ? &st[2] : nullptr);
  if (e) return hip_fail(e, "disaggregate launch");
  return ok();
}

}  // namespace ubf

namespace {

using ubf::enqueue_mvm;
using ubf::fail;
using ubf::hip_fail;
using ubf::ok;

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

namespace ubf {

// Common checks of the compute entry points.
int check_call(ubf_plan* plan, const void* in, void* out, int32_t nrhs,
               size_t in_bytes, size_t out_bytes) {
  if (!plan) return fail(UBF_EINVAL, "plan is NULL");
  if (!in || !out) return fail(UBF_EINVAL, "input or output pointer is NULL");
  if (!plan->p.ws) return fail(UBF_ESTATE, "plan is not bound to a workspace");
  if (nrhs < 1 || nrhs > plan->p.max_nrhs)
    return fail(UBF_EINVAL, "nrhs must be in 1..max_nrhs of the binding (" +
                                std::to_string(plan->p.max_nrhs) + ")");
  if (overlaps(in, in_bytes, out, out_bytes))
    return fail(UBF_EINVAL, "input and output overlap");
  return UBF_OK;
}

size_t basis_vec_bytes(const ubf::Plan& p, int32_t nrhs) {
  return (size_t)nrhs * p.nb_total() * 8;
}

}  // namespace ubf

namespace {

using ubf::basis_vec_bytes;
using ubf::check_call;

size_t box_vec_bytes(const ubf::Plan& p, int32_t nrhs) {
  return (size_t)nrhs * p.n_box * p.nu * 8;
}

// Shared body of ubf_plan_create and ubf_plan_create_batch.
int create(const ubf_problem* problem, const int64_t* scat_ptr, int64_t n_scat,
           ubf_plan** out) {
  if (!problem || !out) return fail(UBF_EINVAL, "problem or out is NULL");
  ubf_plan* plan = new (std::nothrow) ubf_plan();
  if (!plan) return fail(UBF_ENOMEM, "host allocation failed");
  std::string why;
  try {
    why = ubf::build_plan(problem->box_ijk, problem->n_boxes, problem->a,
                          problem->k, problem->eta, problem->n_d,
                          problem->far_mode, problem->precision, problem->operators,
                          scat_ptr, n_scat, plan->p);
  } catch (const std::bad_alloc&) {
    delete plan;
    return fail(UBF_ENOMEM, "host allocation failed while building the plan");
  } catch (...) {
    delete plan;
    return fail(UBF_EINVAL, "plan construction failed");
  }
  if (!why.empty()) {
    delete plan;
    return fail(UBF_EINVAL, why);
  }
  *out = plan;
  return ok();
}


// ---------------------------------------------------------------- tuner

// Persistent grid of the plan's current stage-2 kernel.
int current_groups(const ubf::Plan& p) {
  return (p.split() && (p.split_kernel == ubf::kSplitRounds ||
                        p.split_kernel == ubf::kSplitRoundsDouble))
             ? p.n_round_groups()
             : p.n_groups();
}

// Select a stage-2 kernel and grid, and upload the work partition it reads.
int apply_schedule(ubf::Plan& p, int kernel, int64_t groups, hipStream_t s) {
  p.split_kernel = p.split() ? kernel : ubf::kSplitChunks;
  hipError_t e;
  if (p.split_kernel == ubf::kSplitRounds || p.split_kernel == ubf::kSplitRoundsDouble) {
    ubf::build_rounds(p, groups);
    e = hipMemcpyAsync(p.d_rounds, p.rounds.data(), p.rounds.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p.d_wg_round_ptr, p.wg_round_ptr.data(),
                         p.wg_round_ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
  } else {
    ubf::partition_groups(p, groups);
    e = hipMemcpyAsync(p.d_wg_ptr, p.wg_ptr.data(), p.wg_ptr.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return (int)e;
}

struct Candidate {
  int kernel;
  int64_t groups;
};

// Stage-2 schedules the tuner times: persistent chunk grids of 256..4096
// workgroups; for the 16-bit forms also the walk over right-hand sides
// (several vectors), and with a table the rounds at two workgroups per
// compute unit (512..2048) and the double-buffered rounds at one (256).
// Grids that the work caps to the same size are timed once.
std::vector<Candidate> tune_candidates(const ubf::Plan& p, int nrhs) {
  std::vector<Candidate> c;
  const int64_t grids[] = {256, 512, 1024, 2048, 4096};
  auto capped = [](int64_t g, int64_t units) {
    g = std::min<int64_t>(g, std::max<int64_t>(units, 1));
    return std::min<int64_t>((g + 7) / 8 * 8, ubf::kMaxTranslateGroups);
  };
  auto add = [&](int kernel, int64_t g, int64_t units) {
    const int64_t eff = capped(g, units);
    for (const Candidate& x : c)
      if (x.kernel == kernel && x.groups == eff) return;
    c.push_back({kernel, eff});
  };
  for (int64_t g : grids) add(ubf::kSplitChunks, g, p.n_chunks());
  if (p.split()) {
    if (nrhs > 1)
      for (int64_t g : grids) add(ubf::kSplitChunksWalk, g, p.n_chunks());
    if (!p.gen_ops) {  // the round kernels copy operators from the table
      for (int64_t g : {512, 1024, 2048}) add(ubf::kSplitRounds, g, p.n_items());
      add(ubf::kSplitRoundsDouble, 256, p.n_items());
    }
  }
  return c;
}

// The plan statistics a schedule is chosen for: the stage-2 form, box size,
// vectors per call and the sizes of the far set and its partition.
std::string tune_key(const ubf::Plan& p, int nrhs) {
  return "v2 precision=" + std::to_string(p.precision) +
         " operators=" + std::to_string(p.gen_ops ? 1 : 0) + " nu=" + std::to_string(p.nu) +
         " nrhs=" + std::to_string(nrhs) + " boxes=" + std::to_string(p.n_box) +
         " scatterers=" + std::to_string(p.n_scat()) + " pairs=" + std::to_string(p.n_pairs()) +
         " offsets=" + std::to_string(p.n_off()) + " chunks=" + std::to_string(p.n_chunks()) +
         " items=" + std::to_string(p.n_items());
}

// Cache file (UBF_TUNE_CACHE): one line per key, "<key>\t<kernel> <groups>
// <ms> <timings>". The last line of a key wins.
bool cache_lookup(const char* path, const std::string& key, int* kernel, int* groups) {
  std::FILE* f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char line[4096];
  while (std::fgets(line, sizeof line, f)) {
    const char* tab = std::strchr(line, '\t');
    if (!tab || (size_t)(tab - line) != key.size() || key.compare(0, key.size(), line, key.size()))
      continue;
    int k = -1, g = 0;
    if (std::sscanf(tab + 1, "%d %d", &k, &g) == 2 && k >= 0 && k <= ubf::kSplitRoundsDouble &&
        g >= 1 && g <= ubf::kMaxTranslateGroups) {
      *kernel = k;
      *groups = g;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, int kernel, int groups, float ms,
                 const std::string& report) {
  std::FILE* f = std::fopen(path, "a");
  if (!f) return;  // a cache that cannot be written only costs the next tuning
  std::fprintf(f, "%s\t%d %d %.6f%s\n", key.c_str(), kernel, groups, (double)ms, report.c_str());
  std::fclose(f);
}

}  // namespace

extern "C" {

int ubf_plan_create(const ubf_problem* problem, ubf_plan** out) {
  return create(problem, nullptr, 0, out);
}

int ubf_plan_create_batch(const ubf_problem* problem, int32_t n_scatterers,
                          const int64_t* scatterer_ptr, ubf_plan** out) {
  if (!scatterer_ptr) return fail(UBF_EINVAL, "scatterer_ptr is NULL");
  if (n_scatterers < 1) return fail(UBF_EINVAL, "n_scatterers must be >= 1");
  return create(problem, scatterer_ptr, n_scatterers, out);
}

size_t ubf_workspace_bytes(const ubf_plan* plan, int32_t max_nrhs) {
  if (!plan || max_nrhs < 1) return 0;
  return ubf::workspace_layout(plan->p, max_nrhs).total;
}

int ubf_plan_bind(ubf_plan* plan, void* d_workspace, size_t bytes,
                  int32_t max_nrhs, void* hip_stream) {
  if (!plan || !d_workspace) return fail(UBF_EINVAL, "plan or workspace is NULL");
  if (max_nrhs < 1) return fail(UBF_EINVAL, "max_nrhs must be >= 1");
  if (((uintptr_t)d_workspace & 255) != 0)
    return fail(UBF_EINVAL, "workspace must be 256-byte aligned");
  ubf::Plan& p = plan->p;
  const ubf::Layout L = ubf::workspace_layout(p, max_nrhs);
  if (bytes < L.total)
    return fail(UBF_ENOMEM, "workspace too small: need " + std::to_string(L.total) +
                                " bytes, got " + std::to_string(bytes));
  plan->drop_graph();
  char* ws = (char*)d_workspace;
  hipStream_t s = (hipStream_t)hip_stream;
  struct Copy {
    size_t at;
    const void* src;
    size_t n;
  };
  std::vector<int64_t> nb(p.n_box + 1);
  if (p.has_basis) {
    nb = p.nb_ptr;
  } else {
    for (int64_t i = 0; i <= p.n_box; ++i) nb[i] = i * p.nu;
  }
  const Copy copies[] = {
      {L.table, p.split() ? (const void*)p.table_bf16.data() : (const void*)p.table.data(),
       p.table_bytes()},
      {L.chunks, p.chunks.data(), p.chunks.size() * sizeof(int32_t)},
      {L.items, p.items.data(), p.items.size() * sizeof(int32_t)},
      {L.wg_ptr, p.wg_ptr.data(), p.wg_ptr.size() * sizeof(int32_t)},
      {L.rounds, p.rounds.data(), p.rounds.size() * sizeof(int32_t)},
      {L.wg_round_ptr, p.wg_round_ptr.data(), p.wg_round_ptr.size() * sizeof(int32_t)},
      {L.pair_src, p.pair_src.data(), p.pair_src.size() * sizeof(int32_t)},
      {L.pair_dst, p.pair_dst.data(), p.pair_dst.size() * sizeof(int32_t)},
      {L.test_ptr, p.test_ptr.data(), p.test_ptr.size() * sizeof(int32_t)},
      {L.nb_ptr, nb.data(), nb.size() * sizeof(int64_t)},
      {L.off_scale, p.off_scale.data(), p.off_scale.size() * sizeof(float)},
      {L.offsets, p.offsets.data(), p.offsets.size() * sizeof(int32_t)},
  };
  for (const Copy& c : copies) {
    if (c.n == 0) continue;
    hipError_t e = hipMemcpyAsync(ws + c.at, c.src, c.n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (bind)");
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize (bind)");
  p.ws = ws;
  p.ws_bytes = bytes;
  p.max_nrhs = max_nrhs;
  p.d_table = (float*)(ws + L.table);
  p.d_chunks = (int32_t*)(ws + L.chunks);
  p.d_items = (int32_t*)(ws + L.items);
  p.d_wg_ptr = (int32_t*)(ws + L.wg_ptr);
  p.d_rounds = (int32_t*)(ws + L.rounds);
  p.d_wg_round_ptr = (int32_t*)(ws + L.wg_round_ptr);
  p.d_pair_src = (int32_t*)(ws + L.pair_src);
  p.d_test_ptr = (int32_t*)(ws + L.test_ptr);
  p.d_pair_dst = (int32_t*)(ws + L.pair_dst);
  p.d_nb_ptr = (int64_t*)(ws + L.nb_ptr);
  p.d_P = (float*)(ws + L.P);
  p.d_part = (float*)(ws + L.part);
  p.d_off_scale = (float*)(ws + L.off_scale);
  p.d_box_scale = (float*)(ws + L.box_scale);
  p.d_offsets = (int32_t*)(ws + L.offsets);
  return ok();
}

int ubf_plan_set_basis(ubf_plan* plan, const int64_t* nb_ptr, const void* d_S,
                       const void* d_T) {
  if (!plan) return fail(UBF_EINVAL, "plan is NULL");
  ubf::Plan& p = plan->p;
  plan->drop_graph();
  if (!nb_ptr && !d_S && !d_T) {
    if (!p.ws) return fail(UBF_ESTATE, "plan is not bound to a workspace");
    std::vector<int64_t> nb(p.n_box + 1);
    for (int64_t i = 0; i <= p.n_box; ++i) nb[i] = i * p.nu;
    hipError_t e = hipMemcpy(p.d_nb_ptr, nb.data(), nb.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy (set_basis)");
    p.has_basis = false;
    p.nb_ptr.clear();
    p.d_S = p.d_T = nullptr;
    return ok();
  }
  if (!nb_ptr || !d_S) return fail(UBF_EINVAL, "nb_ptr and d_S are both required");
  if (nb_ptr[0] != 0) return fail(UBF_EINVAL, "nb_ptr[0] must be 0");
  for (int64_t i = 0; i < p.n_box; ++i)
    if (nb_ptr[i + 1] < nb_ptr[i]) return fail(UBF_EINVAL, "nb_ptr must be non-decreasing");
  if (nb_ptr[p.n_box] > (int64_t(1) << 40)) return fail(UBF_EINVAL, "too many basis functions");
  if (!p.ws) return fail(UBF_ESTATE, "plan is not bound to a workspace");
  hipError_t e = hipMemcpy(p.d_nb_ptr, nb_ptr, (p.n_box + 1) * sizeof(int64_t),
                           hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy (set_basis)");
  p.nb_ptr.assign(nb_ptr, nb_ptr + p.n_box + 1);
  p.has_basis = true;
  p.d_S = d_S;
  p.d_T = d_T;
  return ok();
}

int ubf_far_mvm(ubf_plan* plan, const void* d_x, void* d_y, int32_t nrhs,
                void* hip_stream) {
  int st = check_call(plan, d_x, d_y, nrhs,
                      plan ? basis_vec_bytes(plan->p, nrhs) : 0,
                      plan ? basis_vec_bytes(plan->p, nrhs) : 0);
  if (st != UBF_OK) return st;
  return enqueue_mvm(plan->p, d_x, d_y, nrhs, (hipStream_t)hip_stream,
                     plan->next_events());
}

int ubf_plan_capture(ubf_plan* plan, const void* d_x, void* d_y, int32_t nrhs) {
  int st = check_call(plan, d_x, d_y, nrhs,
                      plan ? basis_vec_bytes(plan->p, nrhs) : 0,
                      plan ? basis_vec_bytes(plan->p, nrhs) : 0);
  if (st != UBF_OK) return st;
  plan->drop_graph();
  hipError_t e;
  if (!plan->cap_stream) {
    e = hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      plan->cap_stream = nullptr;
      return hip_fail(e, "hipStreamCreateWithFlags (capture)");
    }
  }
  e = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  const int launched = enqueue_mvm(plan->p, d_x, d_y, nrhs, plan->cap_stream, nullptr);
  const std::string why = ubf::last_error_text();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(plan->cap_stream, &g);
  if (launched != UBF_OK) {
    if (g) (void)hipGraphDestroy(g);
    return fail(launched, why);
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  plan->graph = g;
  plan->exec = x;
  return ok();
}

int ubf_plan_replay(ubf_plan* plan, void* hip_stream) {
  if (!plan) return fail(UBF_EINVAL, "plan is NULL");
  if (!plan->exec) return fail(UBF_ESTATE, "no captured product (ubf_plan_capture)");
  hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ok();
}

int ubf_plan_schedule(ubf_plan* plan, int32_t kernel, int32_t groups, void* hip_stream) {
  if (!plan) return fail(UBF_EINVAL, "plan is NULL");
  ubf::Plan& p = plan->p;
  if (!p.ws) return fail(UBF_ESTATE, "plan is not bound to a workspace");
  if (kernel < 0 || kernel > ubf::kSplitRoundsDouble)
    return fail(UBF_EINVAL, "unknown stage-2 kernel");
  if (kernel != ubf::kSplitChunks && !p.split())
    return fail(UBF_EINVAL, "only the 16-bit forms have stage-2 kernels other than 0");
  if (p.gen_ops && (kernel == ubf::kSplitRounds || kernel == ubf::kSplitRoundsDouble))
    return fail(UBF_EINVAL, "the round kernels need an operator table (generated operators "
                            "run the chunk kernels)");
  if (groups < 1 || groups > ubf::kMaxTranslateGroups)
    return fail(UBF_EINVAL, "groups must be in 1.." + std::to_string(ubf::kMaxTranslateGroups));
  if (p.hidden > 0 || ubf::staged_translate_supported(p))
    return fail(UBF_EINVAL, "this plan's stage 2 (networks, or 192 coefficients per box) runs "
                            "one workgroup per item and has no schedule to choose");
  plan->drop_graph();
  const int e = apply_schedule(p, kernel, groups, (hipStream_t)hip_stream);
  if (e) return hip_fail(e, "upload (schedule)");
  return ok();
}

int ubf_plan_tune(ubf_plan* plan, int32_t nrhs, int32_t reps, void* hip_stream,
                  int32_t* groups_out) {
  if (!plan) return fail(UBF_EINVAL, "plan is NULL");
  ubf::Plan& p = plan->p;
  if (!p.ws) return fail(UBF_ESTATE, "plan is not bound to a workspace");
  if (nrhs < 1 || nrhs > p.max_nrhs)
    return fail(UBF_EINVAL, "nrhs must be in 1..max_nrhs of the binding");
  if (reps < 1 || reps > 1000) return fail(UBF_EINVAL, "reps must be in 1..1000");
  if (p.hidden > 0 || ubf::staged_translate_supported(p)) {
    // stage 2 runs one workgroup per 32 pairs here: nothing to choose
    if (groups_out) *groups_out = (int32_t)p.n_groups();
    return ok();
  }
  plan->drop_graph();
  hipStream_t s = (hipStream_t)hip_stream;
  const std::string key = tune_key(p, nrhs);
  const char* cache = std::getenv("UBF_TUNE_CACHE");
  int kernel = -1, groups = 0;
  const auto usable = [&](int k) {  // a cache line may hold any kernel number
    return k == ubf::kSplitChunks ||
           (p.split() && (k == ubf::kSplitChunksWalk ||
                          (!p.gen_ops && (k == ubf::kSplitRounds || k == ubf::kSplitRoundsDouble))));
  };
  if (cache && *cache && cache_lookup(cache, key, &kernel, &groups) && usable(kernel)) {
    const int e = apply_schedule(p, kernel, groups, s);
    if (e) return hip_fail(e, "upload (tune cache)");
    if (groups_out) *groups_out = current_groups(p);
    return ok();
  }
  const ubf::Layout L = ubf::workspace_layout(p, p.max_nrhs);
  // Column values do not change the timing; start them from zero.
  hipError_t e = hipMemsetAsync(p.d_P, 0, L.part - L.P, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync (tune)");
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if ((e = hipEventCreate(&t0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  if ((e = hipEventCreate(&t1)) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return hip_fail(e, "hipEventCreate");
  }
  const int before_kernel = p.split_kernel;
  const int before_groups = current_groups(p);
  int best_kernel = before_kernel, best_groups = before_groups;
  float best_ms = 0.f;
  int status = UBF_OK;
  std::string why, report;
  for (const Candidate& c : tune_candidates(p, nrhs)) {
    int le = apply_schedule(p, c.kernel, c.groups, s);
    if (le) { status = hip_fail(le, "upload (tune)"); break; }
    le = ubf::launch_translate(p, p.d_P, p.d_part, nrhs, s);  // warm-up
    if (!le && hipEventRecord(t0, s) != hipSuccess) le = (int)hipGetLastError();
    for (int r = 0; r < reps && !le; ++r) le = ubf::launch_translate(p, p.d_P, p.d_part, nrhs, s);
    if (!le && hipEventRecord(t1, s) != hipSuccess) le = (int)hipGetLastError();
    if (!le) le = (int)hipEventSynchronize(t1);
    float ms = 0.f;
    if (!le) le = (int)hipEventElapsedTime(&ms, t0, t1);
    if (le) { status = hip_fail(le, "translate (tune)"); break; }
    ms /= (float)reps;
    report += " " + std::to_string(c.kernel) + ":" + std::to_string(current_groups(p)) + ":" +
              std::to_string(ms * 1e3f);
    if (best_ms == 0.f || ms < best_ms) {
      best_ms = ms;
      best_kernel = c.kernel;
      best_groups = current_groups(p);
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (status != UBF_OK) {
    why = ubf::last_error_text();
    (void)apply_schedule(p, before_kernel, before_groups, s);
    return fail(status, why);
  }
  if ((e = (hipError_t)apply_schedule(p, best_kernel, best_groups, s)) != hipSuccess)
    return hip_fail(e, "upload (tune)");
  if (cache && *cache) cache_store(cache, key, best_kernel, best_groups, best_ms, report);
  if (groups_out) *groups_out = current_groups(p);
  return ok();
}

int ubf_profile_begin(ubf_plan* plan, int32_t max_calls, int32_t every) {
  if (!plan) return fail(UBF_EINVAL, "plan is NULL");
  if (max_calls < 1) return fail(UBF_EINVAL, "max_calls must be >= 1");
  if (every < 1) return fail(UBF_EINVAL, "every must be >= 1");
  for (hipEvent_t e : plan->events) (void)hipEventDestroy(e);
  plan->events.clear();
  plan->profiling = false;
  plan->events.reserve(ubf_plan::kEventsPerCall * (size_t)max_calls);
  for (size_t i = 0; i < ubf_plan::kEventsPerCall * (size_t)max_calls; ++i) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return hip_fail(err, "hipEventCreate");
    plan->events.push_back(e);
  }
  plan->prof_max = max_calls;
  plan->prof_n = 0;
  plan->prof_every = every;
  plan->prof_seen = 0;
  plan->profiling = true;
  return ok();
}

int ubf_profile_end(ubf_plan* plan, double* stage_ms, float* call_ms,
                    int32_t* n_calls) {
  if (!plan) return fail(UBF_EINVAL, "plan is NULL");
  if (!plan->profiling) return fail(UBF_ESTATE, "no profile begun");
  plan->profiling = false;
  double sum[3] = {0, 0, 0};
  for (int32_t c = 0; c < plan->prof_n; ++c) {
    hipEvent_t* ev = &plan->events[ubf_plan::kEventsPerCall * (size_t)c];
    hipError_t err = hipEventSynchronize(ev[5]);
    if (err != hipSuccess) return hip_fail(err, "hipEventSynchronize");
    for (int st = 0; st < 3; ++st) {
      float ms = 0.f;
      err = hipEventElapsedTime(&ms, ev[2 * st], ev[2 * st + 1]);
      if (err != hipSuccess) return hip_fail(err, "hipEventElapsedTime");
      sum[st] += ms;
    }
    if (call_ms) {
      err = hipEventElapsedTime(&call_ms[c], ev[0], ev[5]);
      if (err != hipSuccess) return hip_fail(err, "hipEventElapsedTime");
    }
  }
  if (stage_ms)
    for (int st = 0; st < 3; ++st) stage_ms[st] = sum[st];
  if (n_calls) *n_calls = plan->prof_n;
  for (hipEvent_t e : plan->events) (void)hipEventDestroy(e);
  plan->events.clear();
  return ok();
}

int ubf_aggregate(ubf_plan* plan, const void* d_x, void* d_P, int32_t nrhs,
                  void* hip_stream) {
  int st = check_call(plan, d_x, d_P, nrhs,
                      plan ? basis_vec_bytes(plan->p, nrhs) : 0,
                      plan ? box_vec_bytes(plan->p, nrhs) : 0);
  if (st != UBF_OK) return st;
  const ubf::Plan& p = plan->p;
  int e = ubf::launch_aggregate(p, d_x, p.d_P, nrhs, hip_stream);
  if (e) return hip_fail(e, "aggregate launch");
  e = ubf::launch_unpack(p, p.d_P, d_P, nrhs, hip_stream);
  if (e) return hip_fail(e, "unpack launch");
  return ok();
}

int ubf_translate(ubf_plan* plan, const void* d_P, void* d_E, int32_t nrhs,
                  void* hip_stream) {
  int st = check_call(plan, d_P, d_E, nrhs,
                      plan ? box_vec_bytes(plan->p, nrhs) : 0,
                      plan ? box_vec_bytes(plan->p, nrhs) : 0);
  if (st != UBF_OK) return st;
  const ubf::Plan& p = plan->p;
  // Stage 2 alone maps box vectors to box vectors whatever the basis.
  int e = ubf::launch_pack(p, d_P, p.d_P, nrhs, hip_stream);
  if (e) return hip_fail(e, "pack launch");
  e = ubf::launch_stage2(p, p.d_P, p.d_part, nrhs, (hipStream_t)hip_stream, nullptr);
  if (e) return hip_fail(e, "translate launch");
  e = ubf::launch_disaggregate(p, true, p.d_part, nullptr, d_E, nrhs, hip_stream,
                               /*identity=*/true);
  if (e) return hip_fail(e, "reduce launch");
  return ok();
}

int ubf_disaggregate(ubf_plan* plan, const void* d_E, void* d_y, int32_t nrhs,
                     void* hip_stream) {
  int st = check_call(plan, d_E, d_y, nrhs,
                      plan ? box_vec_bytes(plan->p, nrhs) : 0,
                      plan ? basis_vec_bytes(plan->p, nrhs) : 0);
  if (st != UBF_OK) return st;
  const ubf::Plan& p = plan->p;
  int e = ubf::launch_disaggregate(p, false, nullptr, d_E, d_y, nrhs, hip_stream);
  if (e) return hip_fail(e, "disaggregate launch");
  return ok();
}

size_t ubf_network_bytes(const ubf_plan* plan, int32_t hidden) {
  if (!plan || !ubf::network_shape_supported(plan->p.nu, hidden)) return 0;
  return ubf::network_image_bytes(plan->p, hidden);
}

int ubf_plan_set_networks(ubf_plan* plan, int32_t hidden, const void* d_W1, const void* d_b1,
                          const void* d_W2, const void* d_b2, void* d_net, size_t net_bytes,
                          void* hip_stream) {
  if (!plan) return fail(UBF_EINVAL, "plan is NULL");
  ubf::Plan& p = plan->p;
  if (hidden == 0) {  // back to the operator table
    plan->drop_graph();
    p.hidden = 0;
    p.d_net = nullptr;
    return ok();
  }
  if (!p.ws) return fail(UBF_ESTATE, "plan is not bound");
  if (p.precision != 0) return fail(UBF_EINVAL, "networks need the FP32 form (precision 0)");
  if (hidden < 0 || hidden > ubf::kMaxHidden)
    return fail(UBF_EINVAL, "hidden must be in 1.." + std::to_string(ubf::kMaxHidden));
  if (!ubf::network_shape_supported(p.nu, hidden))
    return fail(UBF_EINVAL, "networks need n_d 2, 3 or 4 (n_u 24, 81 or 192)");
  // a plan without far pairs has no offsets and so no weights to convert
  if ((p.n_off() > 0 && (!d_W1 || !d_b1 || !d_W2 || !d_b2)) || !d_net)
    return fail(UBF_EINVAL, "weight, bias or image pointer is NULL");
  if (((uintptr_t)d_net & 15) != 0) return fail(UBF_EINVAL, "image must be 16-byte aligned");
  const size_t need = ubf::network_image_bytes(p, hidden);
  if (net_bytes < need)
    return fail(UBF_ENOMEM, "network image too small: need " + std::to_string(need) +
                                " bytes, got " + std::to_string(net_bytes));
  plan->drop_graph();
  int e = ubf::launch_network_pack(p, hidden, d_W1, d_b1, d_W2, d_b2, (float*)d_net,
                                   hip_stream);
  if (e) return hip_fail(e, "network pack launch");
  p.hidden = hidden;
  p.d_net = (const float*)d_net;
  return ok();
}

int ubf_plan_info(const ubf_plan* plan, ubf_info* out) {
  if (!plan || !out) return fail(UBF_EINVAL, "plan or out is NULL");
  const ubf::Plan& p = plan->p;
  std::memset(out, 0, sizeof(*out));
  out->n_boxes = p.n_box;
  out->n_pairs = p.n_pairs();
  out->n_offsets = p.n_off();
  out->n_orbits = p.n_orbits;
  out->n_u = p.nu;
  out->n_d = p.n_d;
  out->n_chunks = p.n_chunks();
  out->table_bytes = (int64_t)p.table_bytes();
  out->translate_flops = 8.0 * p.nu * (double)p.nu * (double)p.n_pairs();
  out->mfma = (ubf::translate_uses_mfma(p) || ubf::staged_translate_supported(p)) ? 1 : 0;
  out->precision = p.precision;
  out->n_scatterers = p.n_scat();
  out->n_items = p.n_items();
  out->translate_kernel = p.split_kernel;
  out->translate_groups = current_groups(p);
  out->operators = p.gen_ops ? UBF_OPERATORS_GENERATED : UBF_OPERATORS_TABLE;
  return ok();
}

int ubf_plan_offsets(const ubf_plan* plan, int32_t* out) {
  if (!plan || !out) return fail(UBF_EINVAL, "plan or out is NULL");
  // an empty far set has no offsets (and vector::data() may then be null)
  if (!plan->p.offsets.empty())
    std::memcpy(out, plan->p.offsets.data(), plan->p.offsets.size() * sizeof(int32_t));
  return ok();
}

int ubf_plan_far_pairs(const ubf_plan* plan, int32_t* test, int32_t* src,
                       int32_t* offset_index) {
  if (!plan) return fail(UBF_EINVAL, "plan is NULL");
  const ubf::Plan& p = plan->p;
  const size_t n = p.pair_src.size() * sizeof(int32_t);
  if (n == 0) return ok();  // vector::data() of an empty far set may be null
  if (test) std::memcpy(test, p.pair_test.data(), n);
  if (src) std::memcpy(src, p.pair_src.data(), n);
  if (offset_index) std::memcpy(offset_index, p.pair_off.data(), n);
  return ok();
}

int ubf_plan_operator(const ubf_plan* plan, int32_t o, double* out) {
  if (!plan || !out) return fail(UBF_EINVAL, "plan or out is NULL");
  const ubf::Plan& p = plan->p;
  if (o < 0 || o >= p.n_off()) return fail(UBF_EINVAL, "offset index out of range");
  std::vector<std::complex<double>> G;
  ubf::operator_fp64(&p.offsets[3 * o], p.a, p.k, p.eta, p.n_d, G);
  std::memcpy(out, G.data(), G.size() * sizeof(std::complex<double>));
  return ok();
}

void ubf_plan_destroy(ubf_plan* plan) { delete plan; }

const char* ubf_status_string(int status) {
  switch (status) {
    case UBF_OK: return "ok";
    case UBF_EINVAL: return "invalid argument";
    case UBF_ENOMEM: return "out of memory (workspace too small or host allocation failed)";
    case UBF_EDEVICE: return "HIP runtime error";
    case UBF_ESTATE: return "plan not bound / invalid state";
    default: return "unknown status";
  }
}

const char* ubf_last_error(void) { return ubf::last_error_text().c_str(); }

}  // extern "C"
