// lb_invariants_noalloc: the domain totals of lb_invariants for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc). The partial sums go to a fixed
// per-device array of the library instead of a workspace allocated on first use;
// the kernels are those of lb_invariants, so the results are bitwise the same.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <map>
#include <mutex>
#include <string>

#include "../../include/lbkt.h"
#include "lbkt_internal.hpp"

// One record of 4 partial sums per block of lb_invariants' partition, which has
// at most LBKT_INV_MAX_PARTS blocks: 4096 x 4 doubles = 128 KiB per device, held
// until the process ends. In host code `scratch` names a host-side stand-in,
// not device memory: only the address from hipGetSymbolAddress is passed on.
static constexpr int kScratchParts = LBKT_INV_MAX_PARTS;
static __device__ __align__(256) double scratch[kScratchParts * 4];

namespace {
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;   // device ordinal -> that device's copy of `scratch`
}  // namespace

// Device address of the current device's copy of `scratch`, looked up on the
// first call on that device (with it current) and kept.
static lb_status scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lbkt_fail(LB_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return lbkt_fail(LB_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = g_scratch_ptr.emplace(dev, (double*)p).first;
  }
  *out = it->second;
  return LB_OK;
}

extern "C" lb_status lb_invariants_noalloc(const lb_grid* g, int32_t prec_code, const void* f, double* out4,
                                           void* stream) {
  lb_status s;
  if ((s = lbkt_invariants_args(g, prec_code, f, out4))) return s;
  const lb_prec prec = (lb_prec)prec_code;
  int rpb, nb;
  lbkt_inv_partition(g, &rpb, &nb);
  if (nb > kScratchParts) {
    char buf[128];
    std::snprintf(buf, sizeof(buf), "the grid needs %d partial sums; the fixed array holds %d", nb, kScratchParts);
    return lbkt_fail(LB_EINVAL, buf);
  }
  double* part = nullptr;
  if ((s = scratch_ptr(&part))) return s;
  lbkt::KTConsts K;
  lbkt_build_consts(g, &K);
  // every partial record the final sum reads is written by this call's first
  // kernel, so nothing in the array needs clearing
  return lbkt_launch_invariants(K, prec, f, rpb, nb, part, out4, (hipStream_t)stream);
}
