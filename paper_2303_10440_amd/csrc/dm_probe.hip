// Throughput probes of the FP32 vector ALU: independent dependency chains of
// one instruction kind per lane, enough lanes to fill every SIMD.  Used to
// price the sweeps' transcendentals against their fused multiply-adds.
#include <hip/hip_runtime.h>

#include "dm_probe.h"

namespace {

constexpr int CH = 8;   // independent chains per lane and kind
constexpr int PROBE_T = 256;

// DMP_FMA takes its multiplier and addend from VGPRs (lane-dependent values),
// DMP_FMA_SGPR from the kernel arguments (wave-uniform, held in SGPRs).
template <int OP>
__global__ void __launch_bounds__(PROBE_T) k_alu_probe(float* __restrict__ out, int iters, float ms, float as) {
  const float mv = 0.999f + 1e-7f * (float)(threadIdx.x & 1), av = 1e-4f + 1e-9f * (float)(threadIdx.x & 2);
  float x[CH], y[2];
#pragma unroll
  for (int c = 0; c < CH; ++c) x[c] = 0.25f + 1e-3f * (float)((threadIdx.x + 7 * c) & 63);
  y[0] = x[0] * 0.5f;
  y[1] = x[1] * 0.5f;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (OP == DMP_FMA || OP == DMP_MIX) x[c] = fmaf(x[c], mv, av);
      if (OP == DMP_FMA_SGPR) x[c] = fmaf(x[c], ms, as);
      if (OP == DMP_SIN) x[c] = __builtin_amdgcn_sinf(x[c]);
      if (OP == DMP_COS) x[c] = __builtin_amdgcn_cosf(x[c]);
      if (OP == DMP_RCP) x[c] = __builtin_amdgcn_rcpf(x[c]);
    }
    if (OP == DMP_MIX) {
      y[0] = __builtin_amdgcn_sinf(y[0]);
      y[1] = __builtin_amdgcn_sinf(y[1]);
    }
  }
  float s = OP == DMP_MIX ? y[0] + y[1] : 0.0f;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += x[c];
  out[(size_t)blockIdx.x * PROBE_T + threadIdx.x] = s;
}

template <int OP>
hipError_t launch(float* out, int blocks, int iters) {
  k_alu_probe<OP><<<blocks, PROBE_T>>>(out, iters, 0.999f, 1e-4f);
  return hipGetLastError();
}

hipError_t launch_op(int op, float* out, int blocks, int iters) {
  switch (op) {
    case DMP_FMA: return launch<DMP_FMA>(out, blocks, iters);
    case DMP_SIN: return launch<DMP_SIN>(out, blocks, iters);
    case DMP_COS: return launch<DMP_COS>(out, blocks, iters);
    case DMP_RCP: return launch<DMP_RCP>(out, blocks, iters);
    case DMP_FMA_SGPR: return launch<DMP_FMA_SGPR>(out, blocks, iters);
    default: return launch<DMP_MIX>(out, blocks, iters);
  }
}

}  // namespace

extern "C" int dmp_alu_time(int device, int op, int blocks, int iters, int reps, double* ms_out) {
  if (op < DMP_FMA || op > DMP_FMA_SGPR || blocks < 1 || iters < 1 || reps < 1 || ms_out == nullptr) return -1;
  if (hipSetDevice(device) != hipSuccess) return -5;
  float* out = nullptr;
  if (hipMalloc(&out, sizeof(float) * (size_t)blocks * PROBE_T) != hipSuccess) return -5;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0;
  float ms = 0.0f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -5;
  if (rc == 0 && launch_op(op, out, blocks, iters) != hipSuccess) rc = -5;
  if (rc == 0 && hipEventRecord(e0, nullptr) != hipSuccess) rc = -5;
  for (int r = 0; rc == 0 && r < reps; ++r)
    if (launch_op(op, out, blocks, iters) != hipSuccess) rc = -5;
  if (rc == 0 && hipEventRecord(e1, nullptr) != hipSuccess) rc = -5;
  if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = -5;
  if (rc == 0 && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -5;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (hipFree(out) != hipSuccess) rc = -5;
  if (rc == 0) *ms_out = (double)ms / reps;
  return rc;
}
