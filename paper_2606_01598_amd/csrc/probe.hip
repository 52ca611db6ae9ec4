// LDS bandwidth probe (measurement support): conflict-free 16-byte reads or 64-bit
// integer atomic adds, each lane on consecutive addresses of a 64 KiB array.
#include <hip/hip_runtime.h>

#include "../../include/pme.h"
#include "../../include/probe.h"

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeVec = 4096;   // float4 entries (64 KiB)

__global__ void __launch_bounds__(kProbeThreads) k_lds_read(int iters, float* out) {
  __shared__ float4 buf[kProbeVec];
  const int t = threadIdx.x;
  for (int i = t; i < kProbeVec; i += kProbeThreads)
    buf[i] = make_float4(float(i), 1.0f, 2.0f, 3.0f);
  __syncthreads();
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int it = 0; it < iters; ++it) {
    const float4 v = buf[(t + (it & 15) * kProbeThreads) & (kProbeVec - 1)];
    acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    asm volatile("" ::: "memory");   // every iteration reads LDS again
  }
  __shared__ float red[kProbeThreads];
  red[t] = acc.x + acc.y + acc.z + acc.w;
  __syncthreads();
  if (t == 0) {
    float s = 0.f;
    for (int i = 0; i < kProbeThreads; ++i) s += red[i];
    out[blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(kProbeThreads) k_lds_atomic(int iters, float* out) {
  __shared__ unsigned long long buf[2 * kProbeVec];
  const int t = threadIdx.x;
  for (int i = t; i < 2 * kProbeVec; i += kProbeThreads) buf[i] = 0ull;
  __syncthreads();
  for (int it = 0; it < iters; ++it)
    atomicAdd(&buf[(t + (it & 31) * kProbeThreads) & (2 * kProbeVec - 1)], 1ull);
  __syncthreads();
  if (t == 0) {
    unsigned long long s = 0ull;
    for (int i = 0; i < 2 * kProbeVec; ++i) s += buf[i];
    out[blockIdx.x] = float(s);
  }
}

}  // namespace

extern "C" int pme_lds_probe(void* stream, int32_t kind, int32_t iters, int32_t nblocks,
                             float* out) {
  if (!out || iters < 1 || nblocks < 1 ||
      (kind != PME_PROBE_LDS_READ && kind != PME_PROBE_LDS_ATOMIC))
    return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (kind == PME_PROBE_LDS_READ)
    hipLaunchKernelGGL(k_lds_read, dim3(nblocks), dim3(kProbeThreads), 0, s, iters, out);
  else
    hipLaunchKernelGGL(k_lds_atomic, dim3(nblocks), dim3(kProbeThreads), 0, s, iters, out);
  return hipGetLastError() == hipSuccess ? PME_OK : PME_EHIP;
}
