// The allocation-free variant of cmcg_apply (first-order problems): the solver's device memory
// is carved from one statically sized device array per GPU instead of being allocated, so the
// call makes no device, pinned-host, stream or event allocation.  The array persists until the
// process ends; every call on a GPU reuses that GPU's copy.
#include <mutex>

#include "solver.h"

namespace cmcg {
namespace {

// The fixed device buffer (its capacity is CMCG_STATIC_SCRATCH_BYTES of include/cmcg.h).  In
// host code `scratch` names a host-side stand-in: its device address is taken once per device
// with hipGetSymbolAddress and only that address is passed to kernels and copies.
constexpr size_t kScratchBytes = CMCG_STATIC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on device `dev` (current), looked up once per device.
cmcg_status scratch_on(int dev, void **ptr) {
  if (dev < 0 || dev >= kMaxDevices) return set_error("device ordinal out of range"), CMCG_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)),
             CMCG_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return CMCG_OK;
}

__global__ void zero_kernel(uint4 *p, size_t n16, unsigned char *tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t k = t0; k < n16; k += stride) p[k] = make_uint4(0u, 0u, 0u, 0u);
  if (t0 < ntail) tail[t0] = 0;
}

}  // namespace

hipError_t zero_device(void *p, size_t bytes, hipStream_t s) {
  // p is 256-byte aligned (every fixed-buffer piece is)
  const size_t n16 = bytes / 16, ntail = bytes % 16;
  const int blocks = grid_for(n16 > 0 ? n16 : 1);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, static_cast<uint4 *>(p), n16,
                     static_cast<unsigned char *>(p) + n16 * 16, ntail);
  return hipGetLastError();
}

}  // namespace cmcg

using namespace cmcg;

extern "C" cmcg_status cmcg_apply_static(const cmcg_problem *P, const cmcg_options *O, int32_t op,
                                         int32_t steps, const double *in, double *out) {
  set_error("");
  if (!P || !O || !in || !out) return set_error("null argument"), CMCG_EINVAL;
  if (op < CMCG_OP_FORWARD || op > CMCG_OP_RIESZ) return set_error("unknown op"), CMCG_EINVAL;
  if (steps < 0) return set_error("steps must be >= 0"), CMCG_EINVAL;
  if (P->formulation != 1)
    return set_error("cmcg_apply_static serves first-order problems"), CMCG_EUNSUPPORTED;
  hipStream_t stream = static_cast<hipStream_t>(O->hip_stream);
  SolverConfig cfg;
  CMCG_TRY(make_config(P, O, stream, &cfg));
  // the solver's fields per padded cell, checked before any device work (FP64 set: four
  // states, kap, two source fields; FP32 set alike; direction, iterate, residual, filter
  // sums); the carving itself rejects anything beyond the buffer as well
  const size_t nx = (size_t)P->n[0], ny = (size_t)P->n[1];
  const size_t fs = ny * ((nx + 63) / 64 * 64);
  const bool mixed = O->precision == CMCG_FP32_MIXED;
  const size_t need = fs * (120 + (mixed ? 60 + 12 : 24) + 48 + 16);
  if (need > kScratchBytes)
    return set_error("the problem needs about " + std::to_string(need >> 20) +
                     " MiB of device memory; cmcg_apply_static has " +
                     std::to_string(kScratchBytes >> 20) + " MiB"),
           CMCG_ENOMEM;
  CMCG_HIP(hipSetDevice(O->device));
  void *base = nullptr;
  CMCG_TRY(scratch_on(O->device, &base));
  Solver *S = nullptr;
  cmcg_status st = make_f1_solver_in(P, cfg, base, kScratchBytes, &S);
  if (st != CMCG_OK) return st;
  st = S->apply(op, steps, in, out);
  delete S;   // synchronises the stream; frees nothing on the device
  return st;
}
