// bbfmm_apply_noalloc: bbfmm_apply with its work arrays in a fixed device array of the library
// instead of the plan's buffers, for callers that cannot allocate device memory.
#include <mutex>
#include <string>

#include "internal.h"

namespace bbfmm {
namespace {

// 64 MiB per device, held from the library's load until the process ends.
constexpr long long kScratchDoubles = 8LL << 20;
constexpr int kScratchDevices = 64;

// The work arrays of every bbfmm_apply_noalloc call on a device. In host code this name is a
// host-side stand-in: device code reaches the array only through the address looked up below.
__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mutex;
double* g_scratch_ptr[kScratchDevices] = {};

// The device address of `scratch` on device `dev` (the current device), looked up on the first
// call on that device and kept.
bbfmm_status scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kScratchDevices)
    return fail(BBFMM_EUNSUPPORTED, "bbfmm_apply_noalloc supports device indices below 64");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(BBFMM_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return BBFMM_OK;
}

// 256-byte alignment of each work array.
long long aligned(long long doubles) { return (doubles + 31) / 32 * 32; }

}  // namespace
}  // namespace bbfmm

using namespace bbfmm;

extern "C" {

bbfmm_status bbfmm_apply_noalloc(bbfmm_plan* p, const double* d_q, int32_t nrhs, double* d_phi, void* stream) {
  bbfmm_status st = check_apply_args(p, d_q, nrhs, d_phi);
  if (st != BBFMM_OK) return st;
  if (p->variant != BBFMM_VARIANT_BLOCKED)
    return fail(BBFMM_EUNSUPPORTED, "bbfmm_apply_noalloc runs the blocked M2L variant only");
  const bbfmm_tree* t = p->tree;
  const long long nq = aligned(t->n * (long long)nrhs);
  const long long ne = t->depth >= 2 ? aligned(p->exp_elems * (long long)nrhs) : 0;
  const long long need = 2 * nq + 2 * ne;
  if (need > kScratchDoubles)
    return fail(BBFMM_EINVAL, "bbfmm_apply_noalloc: this tree and nrhs need " + std::to_string(need * 8) +
                                  " bytes of work arrays, above its fixed " + std::to_string(kScratchDoubles * 8) +
                                  " bytes; use bbfmm_apply");
  int dev = -1;
  BBFMM_HIP_TRY(hipGetDevice(&dev));
  if (dev != t->device) return fail(BBFMM_EINVAL, "the plan's device must be the current device");
  double* base = nullptr;
  if ((st = scratch_address(dev, &base)) != BBFMM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = begin_call(p, s)) != BBFMM_OK) return st;
  // qs | phis | W | F, each 256-byte aligned; every pass overwrites what it later reads, so the
  // previous call's contents need no clearing
  Work wk;
  wk.qs = base;
  wk.phis = base + nq;
  wk.W = ne ? base + 2 * nq : nullptr;
  wk.F = ne ? base + 2 * nq + ne : nullptr;
  wk.trace = false;
  st = run_chain_work(p, d_q, nrhs, d_phi, wk, s);
  // the plan's own forward locals are not those of this call: bbfmm_eval_grad and the expansion
  // copy need a bbfmm_apply first
  p->slot_nrhs[0] = 0;
  return end_call(p, s, st);
}

}  // extern "C"
