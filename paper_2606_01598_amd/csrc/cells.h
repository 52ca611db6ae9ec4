// Cell list for the real-space pair kernels (polarizable model, dipole-head
// features): atoms binned by fractional coordinate into a grid of cells at least
// one cutoff wide, by a counting sort (count, exclusive scan, scatter).  A pair
// kernel visits, for each atom, the 3 x 3 x 3 neighbouring cells, or every cell
// along an axis with fewer than three, so that with the cutoff below half the
// smallest perpendicular width every pair within the cutoff is seen once under the
// minimum image.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/pme.h"

namespace {

struct CellGrid {
  float C[9];                       // rows are lattice vectors
  float Ci[9];                      // inverse: s = r Ci
  int nc[3];
  int ncell;
};

struct CellList {
  CellGrid g;
  int* count = nullptr;             // [ncell]
  int* start = nullptr;             // [ncell + 1]
  int* cellof = nullptr;            // [max_atoms]
  int* slot = nullptr;              // [max_atoms]
  int* sorted = nullptr;            // [max_atoms] atom indices grouped by cell
};

__device__ __forceinline__ void frac(const CellGrid& g, float x, float y, float z, float& s0,
                                     float& s1, float& s2) {
  s0 = x * g.Ci[0] + y * g.Ci[3] + z * g.Ci[6];
  s1 = x * g.Ci[1] + y * g.Ci[4] + z * g.Ci[7];
  s2 = x * g.Ci[2] + y * g.Ci[5] + z * g.Ci[8];
}

// Cell of a point (wrapped into the cell; NaN coordinates land in cell 0 of an axis).
__device__ __forceinline__ void cell_of(const CellGrid& g, float x, float y, float z, int (&c)[3]) {
  float s[3];
  frac(g, x, y, z, s[0], s[1], s[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float t = s[a] - floorf(s[a]);
    const int k = int(t * float(g.nc[a]));
    c[a] = (k < 0) ? 0 : ((k >= g.nc[a]) ? g.nc[a] - 1 : k);
  }
}

// Minimum-image displacement through fractional coordinates.
__device__ __forceinline__ float3 min_image(const CellGrid& g, float dx, float dy, float dz) {
  float f0, f1, f2;
  frac(g, dx, dy, dz, f0, f1, f2);
  f0 -= rintf(f0);
  f1 -= rintf(f1);
  f2 -= rintf(f2);
  return make_float3(f0 * g.C[0] + f1 * g.C[3] + f2 * g.C[6],
                     f0 * g.C[1] + f1 * g.C[4] + f2 * g.C[7],
                     f0 * g.C[2] + f1 * g.C[5] + f2 * g.C[8]);
}

// Neighbour cell number `o` (0 .. min(nc, 3) - 1) along an axis of a cell c.
__device__ __forceinline__ int neighbour_cell(int c, int o, int nc) {
  return (nc >= 3) ? (c + o - 1 + nc) % nc : o;
}

__global__ void k_cell_clear(int* count, int ncell) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncell; c += gridDim.x * blockDim.x)
    count[c] = 0;
}

__global__ void k_cell_count(int n, const float* pos, CellGrid g, int* count, int* cellof,
                             int* slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c[3];
  cell_of(g, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], c);
  const int cell = (c[0] * g.nc[1] + c[1]) * g.nc[2] + c[2];
  cellof[i] = cell;
  slot[i] = atomicAdd(&count[cell], 1);
}

// exclusive scan of the cell counts (one workgroup of 1024)
__global__ void __launch_bounds__(1024) k_cell_scan(const int* count, int* start, int ncell) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int seg = (ncell + 1023) / 1024;
  const int s0 = min(t * seg, ncell), s1 = min(s0 + seg, ncell);
  int acc = 0;
  for (int c = s0; c < s1; ++c) acc += count[c];
  part[t] = acc;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = (t >= o) ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - acc;
  for (int c = s0; c < s1; ++c) { start[c] = run; run += count[c]; }
  if (t == 1023) start[ncell] = part[1023];
}

__global__ void k_cell_fill(int n, const int* cellof, const int* slot, const int* start,
                            int* sorted) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) sorted[start[cellof[i]] + slot[i]] = i;
}

inline int cell_blocks(int m, int t) { return m > 0 ? (m + t - 1) / t : 1; }

// Grid of cells for a cell (host box, rows are lattice vectors) and cutoff, and
// its device arrays.  PME_EINVAL for a singular cell or a cutoff not below half
// the smallest perpendicular width.
inline int setup_cells(CellList& cl, const double* C, double rc, int max_atoms) {
  const double det = C[0] * (C[4] * C[8] - C[5] * C[7]) - C[1] * (C[3] * C[8] - C[5] * C[6]) +
                     C[2] * (C[3] * C[7] - C[4] * C[6]);
  if (!isfinite(det) || fabs(det) < 1e-12) return PME_EINVAL;
  double Ci[9];
  Ci[0] = (C[4] * C[8] - C[5] * C[7]) / det; Ci[1] = (C[2] * C[7] - C[1] * C[8]) / det;
  Ci[2] = (C[1] * C[5] - C[2] * C[4]) / det; Ci[3] = (C[5] * C[6] - C[3] * C[8]) / det;
  Ci[4] = (C[0] * C[8] - C[2] * C[6]) / det; Ci[5] = (C[2] * C[3] - C[0] * C[5]) / det;
  Ci[6] = (C[3] * C[7] - C[4] * C[6]) / det; Ci[7] = (C[1] * C[6] - C[0] * C[7]) / det;
  Ci[8] = (C[0] * C[4] - C[1] * C[3]) / det;
  // perpendicular widths w_a = 1 / |column a of C^-1|
  double w[3];
  for (int a = 0; a < 3; ++a)
    w[a] = 1.0 / sqrt(Ci[a] * Ci[a] + Ci[3 + a] * Ci[3 + a] + Ci[6 + a] * Ci[6 + a]);
  if (!(rc > 0.0) || !isfinite(rc) || rc >= 0.5 * fmin(w[0], fmin(w[1], w[2]))) return PME_EINVAL;
  long ncell = 1;
  for (int a = 0; a < 3; ++a) {
    int k = int(floor(w[a] / rc));
    if (k < 1) k = 1;
    if (k > 128) k = 128;
    cl.g.nc[a] = k;
    ncell *= k;
  }
  cl.g.ncell = int(ncell);
  for (int k = 0; k < 9; ++k) { cl.g.C[k] = float(C[k]); cl.g.Ci[k] = float(Ci[k]); }
  const size_t m = size_t(max_atoms);
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t r) { if (r != hipSuccess && e == hipSuccess) e = r; };
  ok(hipMalloc(&cl.count, sizeof(int) * ncell));
  ok(hipMalloc(&cl.start, sizeof(int) * (ncell + 1)));
  ok(hipMalloc(&cl.cellof, sizeof(int) * m));
  ok(hipMalloc(&cl.slot, sizeof(int) * m));
  ok(hipMalloc(&cl.sorted, sizeof(int) * m));
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? PME_ENOMEM : PME_EHIP;
  return PME_OK;
}

inline void free_cells(CellList& cl) {
  void* ptrs[] = {cl.count, cl.start, cl.cellof, cl.slot, cl.sorted};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  cl = CellList();
}

// Cell list of the current positions (4 launches on `s`).
inline hipError_t build_cells(const CellList& cl, hipStream_t s, int n, const float* pos) {
  const CellGrid& g = cl.g;
  hipLaunchKernelGGL(k_cell_clear, dim3(cell_blocks(g.ncell, 256)), dim3(256), 0, s, cl.count,
                     g.ncell);
  if (n > 0)
    hipLaunchKernelGGL(k_cell_count, dim3(cell_blocks(n, 256)), dim3(256), 0, s, n, pos, g,
                       cl.count, cl.cellof, cl.slot);
  hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, s, cl.count, cl.start, g.ncell);
  if (n > 0)
    hipLaunchKernelGGL(k_cell_fill, dim3(cell_blocks(n, 256)), dim3(256), 0, s, n, cl.cellof,
                       cl.slot, cl.start, cl.sorted);
  return hipGetLastError();
}

}  // namespace
