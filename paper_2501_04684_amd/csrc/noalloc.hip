// The far-zone product for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the per-call intermediates live in one static device array
// instead of the plan's bound workspace.
//
// The array is file-scope and fixed in size; each GPU the library runs on
// holds its own copy until the process ends. Host code never passes the
// array's name to a kernel or a copy (on the host that name is only a
// stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, once per device, on the entry point's first call with
// that device current, and is kept per device.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "capi_internal.hpp"

// Room for one call's box vectors, partial rows and FP16 box scales: the
// 3,338-box shell (108,888 far pairs) needs 75.6 MB for one right-hand side.
constexpr size_t kScratchBytes = UBF_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up once).
int device_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return ubf::hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return ubf::fail(UBF_EDEVICE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return ubf::hip_fail(e, "hipGetSymbolAddress (static scratch)");
    if (!ptr) return ubf::fail(UBF_EDEVICE, "hipGetSymbolAddress returned no address");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return UBF_OK;
}

}  // namespace

extern "C" {

int ubf_far_mvm_noalloc(ubf_plan* plan, const void* d_x, void* d_y, int32_t nrhs,
                        void* hip_stream) {
  int st = ubf::check_call(plan, d_x, d_y, nrhs,
                           plan ? ubf::basis_vec_bytes(plan->p, nrhs) : 0,
                           plan ? ubf::basis_vec_bytes(plan->p, nrhs) : 0);
  if (st != UBF_OK) return st;
  ubf::Plan& p = plan->p;
  const ubf::ScratchLayout L = ubf::scratch_layout(p, nrhs);
  if (L.total > kScratchBytes)
    return ubf::fail(UBF_EINVAL, "this product needs " + std::to_string(L.total) +
                                     " bytes of static scratch; the limit is " +
                                     std::to_string(kScratchBytes) + " bytes (" +
                                     std::to_string(kScratchBytes >> 20) + " MiB)");
  void* base = nullptr;
  st = device_scratch(&base);
  if (st != UBF_OK) return st;
  char* b = static_cast<char*>(base);
  // The launches read the intermediates' addresses (and the spare partial
  // row, at max_nrhs * n_pairs) from the plan: point them into the static
  // array for this call only. A plan is used by one stream at a time and
  // kernel arguments are taken at launch, so restoring them afterwards is
  // safe. Every intermediate is written before it is read within the call
  // (box vectors including their zero padding by stage 1, every partial row
  // by stage 2), so nothing needs clearing.
  float* const keep_P = p.d_P;
  float* const keep_part = p.d_part;
  float* const keep_box_scale = p.d_box_scale;
  const int32_t keep_max_nrhs = p.max_nrhs;
  p.d_P = reinterpret_cast<float*>(b + L.P);
  p.d_part = reinterpret_cast<float*>(b + L.part);
  p.d_box_scale = reinterpret_cast<float*>(b + L.box_scale);
  p.max_nrhs = nrhs;
  st = ubf::enqueue_mvm(p, d_x, d_y, nrhs, (hipStream_t)hip_stream, plan->next_events());
  p.d_P = keep_P;
  p.d_part = keep_part;
  p.d_box_scale = keep_box_scale;
  p.max_nrhs = keep_max_nrhs;
  return st;
}

}  // extern "C"
