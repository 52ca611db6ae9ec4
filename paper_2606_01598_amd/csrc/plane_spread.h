// Pieces shared by the x-plane spreads (Sec. 2.3.2, Eq. charge_dipole_assign): the
// plane spread fused with the slab transform (fft.hip, k_spread_slab) and the band
// spread (band.hip, k_spread_band).  A workgroup of either scans the slot counts of
// the bins whose atoms can reach its plane (or band), maps scanned slots to records,
// and adds each reaching atom's p x p footprint in its x-plane into 64-bit
// fixed-point LDS words with the tile spread's expressions, so that every word equals
// the tile spread's.
#pragma once

#include "kernels.h"
#include "pme_common.h"

namespace pme {

// The slot counts of the scanned bins into s_off and the bins into s_bin (bin_of(e) is
// the e-th scanned bin); entry nscan is the overflow list (pseudo-bin -1).
template <class BinOf>
__device__ __forceinline__ void load_slot_counts(int nscan, BinOf bin_of, const int* count,
                                                 int cap, const int* ovf_count, int* s_off,
                                                 int* s_bin) {
  for (int e = threadIdx.x; e < nscan; e += blockDim.x) {
    const int bin = bin_of(e);
    s_bin[e] = bin;
    s_off[e] = min(count[bin], cap);
  }
  if (threadIdx.x == 0) {
    s_bin[nscan] = -1;
    s_off[nscan] = *ovf_count;
  }
}

// After a barrier that follows load_slot_counts: the exclusive scan of s_off[0..nscan]
// in place over the workgroup (consecutive segments per thread, wavefront prefix sums,
// then the wavefronts' totals; s_off[nscan + 1] is the total), then the item -> bin
// map when the total fits it.  Ends with a barrier; returns whether the map was made.
__device__ __forceinline__ bool scan_slot_counts(int nscan, int* s_off, int* s_wsum,
                                                 uint16_t* s_map, int map_cap, int& total) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  {
    const int len = nscan + 1;
    const int seg = (len + nthr - 1) / nthr;
    const int s0 = min(tid * seg, len), s1 = min(s0 + seg, len);
    int acc = 0;
    for (int e = s0; e < s1; ++e) acc += s_off[e];
    const int lane = tid & 63, wave = tid >> 6;
    int incl = acc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += s_wsum[w];
    int run = before + incl - acc;
    for (int e = s0; e < s1; ++e) { const int v = s_off[e]; s_off[e] = run; run += v; }
    if (tid == nthr - 1) s_off[len] = before + incl;
  }
  __syncthreads();
  total = s_off[nscan + 1];
  const bool mapped = total <= map_cap;
  if (mapped)
    for (int e = tid; e <= nscan; e += nthr)
      for (int k = s_off[e]; k < s_off[e + 1]; ++k) s_map[k] = uint16_t(e);
  __syncthreads();
  return mapped;
}

// Record index of scanned slot `it`: the bin is the last one whose offset is <= it.
__device__ __forceinline__ size_t scanned_record(int it, bool mapped, int nscan, const int* s_off,
                                                 const int* s_bin, const uint16_t* s_map, int cap,
                                                 long long ovf_base) {
  int lb = 0;
  if (mapped) {
    lb = s_map[it];
  } else {
    int hb = nscan;
    while (lb < hb) {
      const int mid = (lb + hb + 1) >> 1;
      if (s_off[mid] <= it) lb = mid; else hb = mid - 1;
    }
  }
  const int bin = s_bin[lb];
  const int slot = it - s_off[lb];
  return (bin >= 0) ? size_t(bin) * cap + slot : size_t(ovf_base) + slot;
}

// One atom's footprint in x-plane X: record ri's weights and coefficients with the tile
// spread's arithmetic, and its P x P words added at row rows(b_y, iy) (skipped from
// row_limit on) and padded column b_z + iz of `plane` (rows of PZ words).  DEG 1 takes the
// forward coefficients from a forward record, or with TREC forms q and J mu from a
// tangent record; DEG 2 forms the ten tangent coefficients.  s_J holds J (DEG 2 or
// TREC), s_cw the whole-number spline pieces, scale the fixed-point unit.
template <int P, int DEG, bool TREC, class Rows>
__device__ __forceinline__ void add_atom_plane(const float* rec, size_t ri, const float* s_J,
                                               const float* s_cw, int X, int Nx, float scale,
                                               unsigned long long* plane, int PZ, Rows rows,
                                               int row_limit) {
  static_assert(!TREC || DEG == 1, "tangent records serve the forward density");
  constexpr int NC = (DEG == 1) ? 4 : 10;
  constexpr int D = (DEG == 1) ? 1 : 2;       // highest weight derivative needed
  constexpr int lo = (P - 1) / 2;
  const float4* r = reinterpret_cast<const float4*>(rec + ri * kRecWords);
  const float4 h = r[0];
  const float4 c0v = r[1];
  float co[NC];
  if constexpr (DEG == 2) {
    const float4 c1v = r[2];
    const float* f = rec + ri * kRecWords;   // v_mu
    float Jt[3][3];
#pragma unroll
    for (int i = 0; i < 9; ++i) Jt[i / 3][i % 3] = s_J[i];
    tangent_coeffs(Jt, c0v.x, make_float3(c0v.y, c0v.z, c0v.w), c1v.x,
                   make_float3(c1v.y, c1v.z, c1v.w), make_float3(f[12], f[13], f[14]), co);
  } else if constexpr (TREC) {
    float Jt[3][3];
#pragma unroll
    for (int i = 0; i < 9; ++i) Jt[i / 3][i % 3] = s_J[i];
    const float3 d = jmul(Jt, make_float3(c0v.y, c0v.z, c0v.w));
    co[0] = c0v.x; co[1] = d.x; co[2] = d.y; co[3] = d.z;
  } else {
    co[0] = c0v.x; co[1] = c0v.y; co[2] = c0v.z; co[3] = c0v.w;
  }
  const int pk = __float_as_int(h.w);
  const int by = (pk >> 10) & 1023, bz = (pk >> 20) & 1023;
  int ix = X - (pk & 1023) + lo;
  ix += (ix < 0) ? Nx : 0;
  ix -= (ix >= Nx) ? Nx : 0;
  // this plane's x weights (whole-number, times the fixed-point unit): the column ix
  // of spline_weights_whole, with the same Horner steps
  float x[D + 1];
  weight_at_lds<P, D>(s_cw, ix, h.x, x);
#pragma unroll
  for (int d = 0; d <= D; ++d) x[d] *= scale;
  // this x-plane's coefficients of the (y, z) derivative monomials
  float ax0, az1, az2 = 0.f, ay1, ay2 = 0.f, ayz = 0.f;
  if (DEG == 1) {
    ax0 = co[0] * x[0] + co[1] * x[1];   // W_y W_z
    ay1 = co[2] * x[0];                  // W_y' W_z
    az1 = co[3] * x[0];                  // W_y W_z'
  } else {
    ax0 = co[0] * x[0] + co[1] * x[1] + co[4] * x[2];
    ay1 = co[2] * x[0] + co[7] * x[1];
    az1 = co[3] * x[0] + co[8] * x[1];
    ay2 = co[5] * x[0];
    az2 = co[6] * x[0];
    ayz = co[9] * x[0];
  }
  float wy[D + 1][P], wz[D + 1][P];
  spline_weights_whole<P, D>(h.y, wy);
  spline_weights_whole<P, D>(h.z, wz);
#pragma unroll
  for (int iy = 0; iy < P; ++iy) {
    const int rr = rows(by, iy);
    if (rr >= row_limit) continue;
    const float y0 = wy[0][iy], y1 = wy[1][iy];
    float c0 = ax0 * y0 + ay1 * y1, c1 = az1 * y0, c2 = 0.f;
    if (D == 2) {
      const float y2 = wy[2][iy];
      c0 += ay2 * y2;
      c1 += ayz * y1;
      c2 = az2 * y0;
    }
    unsigned long long* row = plane + rr * PZ + bz;
#pragma unroll
    for (int iz = 0; iz < P; ++iz) {
      float v = c0 * wz[0][iz] + c1 * wz[1][iz];
      if (D == 2) v += c2 * wz[2][iz];
      atomicAdd(row + iz, to_fixed(v));
    }
  }
}

}  // namespace pme
