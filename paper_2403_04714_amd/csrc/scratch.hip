// scratch.hip -- fsim_read_regs_noalloc: reading one instance's registers
// without any device allocation, for callers that cannot allocate (code
// under stream capture, tight serving loops, harnesses that forbid
// hipMalloc).
//
// fsim_read_regs gathers a batched instance's register column through a
// staging buffer the sim allocates on first use.  This variant gathers into
// `scratch`, a file-scope device array of kScratchBytes that every GPU the
// library runs on holds until the process ends, and copies it to the host.
// Host code never passes the array's name to a kernel (in host code it is a
// host-side stand-in, not a device address): at the first call on a device,
// with that device current, hipGetSymbolAddress gives the device address,
// which is kept per device and used for every kernel argument and copy.
//
// Every call on one GPU shares that GPU's array: calls that overlap on the
// same GPU (two host threads, or two streams) race on it.  A call writes the
// whole prefix it copies back before copying it, so nothing needs clearing.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "runtime_internal.h"

namespace fsim {
namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;   // 8 MiB: 1,048,576 registers
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint64_t scratch[kScratchBytes / 8];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device `dev`, looked up
// once per device.
hipError_t scratch_address(int dev, uint64_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<uint64_t*>(g_scratch_ptr[dev]);
  return hipSuccess;
}

// out[r] = register r of instance `inst` in the batched layout: 1-bit
// registers as bit inst % 64 of mask [i][inst / 64], narrow ones as u32
// [i][inst], wide ones as u64 [i][inst], where cls_idx[r] = class << 30 | i.
__global__ __launch_bounds__(256) void gather_instance_regs(const uint64_t* stB, const uint32_t* stW,
                                                            const uint64_t* stD, const uint32_t* cls_idx,
                                                            uint32_t R, uint32_t n_tiles, uint32_t n_pad,
                                                            uint32_t inst, uint64_t* out) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
    const uint32_t k = cls_idx[r] >> 30, i = cls_idx[r] & 0x3FFFFFFFu;
    uint64_t v;
    if (k == C_B) v = (stB[(size_t)i * n_tiles + inst / 64] >> (inst % 64)) & 1;
    else if (k == C_W) v = stW[(size_t)i * n_pad + inst];
    else v = stD[(size_t)i * n_pad + inst];
    out[r] = v;
  }
}

}  // namespace
}  // namespace fsim

extern "C" int fsim_read_regs_noalloc(fsim_sim* s, uint32_t inst, uint64_t* out) {
  int rc = fsim::check_inst(s, inst);
  if (rc) return rc;
  const fsim::Design& D = s->d->d;
  const uint32_t R = D.R;
  if (!out && R) return fsim::fail(FSIM_E_ARG, "out is NULL");
  if (R == 0) return FSIM_OK;
  const hipStream_t st = s->d->ctx->stream;
  HIP_TRY(hipSetDevice(s->d->ctx->device));
  const size_t cur = s->cycle & 1;
  if (!s->batched) {
    // the plain form keeps the registers in order: one copy, no staging
    HIP_TRY(hipMemcpyAsync(out, s->state + cur * R, (size_t)R * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return FSIM_OK;
  }
  if ((size_t)R * 8 > fsim::kScratchBytes)
    return fsim::fail(FSIM_E_CAPACITY, "fsim_read_regs_noalloc: " + std::to_string(R) +
                                           " registers exceed its static staging of " +
                                           std::to_string(fsim::kScratchBytes / 8) + " values; use fsim_read_regs");
  uint64_t* buf = nullptr;
  HIP_TRY(fsim::scratch_address(s->d->ctx->device, &buf));
  const uint64_t* stB = s->stB + cur * (size_t)D.reg_count[0] * s->n_tiles;
  const uint32_t* stW = s->stW + cur * (size_t)D.reg_count[1] * s->n_pad;
  const uint64_t* stD = s->stD + cur * (size_t)D.reg_count[2] * s->n_pad;
  const uint32_t grid = (uint32_t)std::min<size_t>(((size_t)R + 255) / 256, 4096);
  hipLaunchKernelGGL(fsim::gather_instance_regs, dim3(grid), dim3(256), 0, st, stB, stW, stD,
                     (const uint32_t*)s->d->b_regidx.p, R, s->n_tiles, s->n_pad, inst, buf);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, buf, (size_t)R * 8, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return FSIM_OK;
}
