// Measurement support: LDS bandwidth (conflict-free 16-byte reads or 64-bit integer
// atomic adds, each lane on consecutive addresses of a 64 KiB array) and the
// global-memory cost of combining the overlapping per-tile regions of a
// scatter-once spread (64-bit atomics, or contiguous region blocks and a fold).
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

struct HaloGeo {
  int N[3], T[3], R[3], nt[3];
  int lo;                            // points of a region before its tile
};

__device__ __forceinline__ int wrap_axis(int m, int n) { return m < 0 ? m + n : (m >= n ? m - n : m); }

// one workgroup per tile: its region, x-major, z fastest
template <bool ATOMIC>
__global__ void __launch_bounds__(kProbeThreads) k_halo_region(HaloGeo g, unsigned long long* regions,
                                                               unsigned long long* mesh) {
  int t = blockIdx.x;
  const int tz = t % g.nt[2];
  t /= g.nt[2];
  const int ty = t % g.nt[1], tx = t / g.nt[1];
  const int o[3] = {tx * g.T[0] - g.lo, ty * g.T[1] - g.lo, tz * g.T[2] - g.lo};
  const int vol = g.R[0] * g.R[1] * g.R[2];
  for (int e = threadIdx.x; e < vol; e += kProbeThreads) {
    if (ATOMIC) {
      const int rz = e % g.R[2], r = e / g.R[2];
      const int ry = r % g.R[1], rx = r / g.R[1];
      // o[a] + r lies in [-lo, N + R - lo): one wrap suffices since R <= N
      const size_t idx = (size_t(wrap_axis(o[0] + rx, g.N[0])) * g.N[1] + wrap_axis(o[1] + ry, g.N[1])) *
                             g.N[2] + wrap_axis(o[2] + rz, g.N[2]);
      atomicAdd(mesh + idx, 1ull);
    } else {
      regions[size_t(blockIdx.x) * vol + e] = 1ull;
    }
  }
}

// one thread per mesh point: along each axis the point lies in the region of tile
// k0 = (c + lo) / T (at offset (c + lo) mod T) and, when that offset is below
// R - T, also in the region of the tile before (offset + T); summed in a fixed order
__global__ void __launch_bounds__(kProbeThreads) k_halo_fold(HaloGeo g, const long long* regions,
                                                             float* mesh) {
  const long long M = (long long)g.N[0] * g.N[1] * g.N[2];
  const long long i = (long long)blockIdx.x * kProbeThreads + threadIdx.x;
  if (i >= M) return;
  const int z = int(i % g.N[2]);
  const long long r = i / g.N[2];
  const int c[3] = {int(r / g.N[1]), int(r % g.N[1]), z};
  int k[3][2], off[3][2], cnt[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int u = c[a] + g.lo;
    if (u >= g.N[a]) u -= g.N[a];
    const int k0 = u / g.T[a], r0 = u - k0 * g.T[a];
    k[a][0] = k0;
    off[a][0] = r0;
    k[a][1] = (k0 == 0) ? g.nt[a] - 1 : k0 - 1;
    off[a][1] = r0 + g.T[a];
    cnt[a] = (r0 < g.R[a] - g.T[a]) ? 2 : 1;
  }
  const long long vol = (long long)g.R[0] * g.R[1] * g.R[2];
  long long acc = 0;
  for (int ax = 0; ax < cnt[0]; ++ax)
    for (int ay = 0; ay < cnt[1]; ++ay)
      for (int az = 0; az < cnt[2]; ++az) {
        const long long t = ((long long)k[0][ax] * g.nt[1] + k[1][ay]) * g.nt[2] + k[2][az];
        acc += regions[t * vol + ((long long)off[0][ax] * g.R[1] + off[1][ay]) * g.R[2] + off[2][az]];
      }
  mesh[i] = float(acc);
}

}  // namespace

extern "C" int pme_halo_probe(void* stream, int32_t kind, const int32_t N[3], const int32_t T[3],
                              int32_t p, void* regions, void* mesh) {
  if (!N || !T || p < 1 || p > 8 || !mesh) return PME_EINVAL;
  if (kind != PME_PROBE_HALO_ATOMIC && kind != PME_PROBE_HALO_WRITE && kind != PME_PROBE_HALO_FOLD)
    return PME_EINVAL;
  if (kind != PME_PROBE_HALO_ATOMIC && !regions) return PME_EINVAL;
  HaloGeo g;
  g.lo = (p - 1) / 2;            // the stencil of an anchor b starts at b - (p - 1) / 2
  long long tiles = 1, points = 1;
  for (int a = 0; a < 3; ++a) {
    if (T[a] < 1 || N[a] < 1 || N[a] > 4096 || N[a] % T[a] != 0 || N[a] < T[a] + p - 1)
      return PME_EINVAL;
    g.N[a] = N[a];
    g.T[a] = T[a];
    g.R[a] = T[a] + p - 1;
    g.nt[a] = N[a] / T[a];
    tiles *= g.nt[a];
    points *= N[a];
  }
  if (tiles > (1LL << 31) - 1 || (points + kProbeThreads - 1) / kProbeThreads > (1LL << 31) - 1)
    return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* rg = static_cast<unsigned long long*>(regions);
  if (kind == PME_PROBE_HALO_ATOMIC)
    hipLaunchKernelGGL(k_halo_region<true>, dim3(unsigned(tiles)), dim3(kProbeThreads), 0, s, g, rg,
                       static_cast<unsigned long long*>(mesh));
  else if (kind == PME_PROBE_HALO_WRITE)
    hipLaunchKernelGGL(k_halo_region<false>, dim3(unsigned(tiles)), dim3(kProbeThreads), 0, s, g, rg,
                       static_cast<unsigned long long*>(mesh));
  else
    hipLaunchKernelGGL(k_halo_fold, dim3(unsigned((points + kProbeThreads - 1) / kProbeThreads)),
                       dim3(kProbeThreads), 0, s, g, static_cast<const long long*>(regions),
                       static_cast<float*>(mesh));
  return hipGetLastError() == hipSuccess ? PME_OK : PME_EHIP;
}

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
