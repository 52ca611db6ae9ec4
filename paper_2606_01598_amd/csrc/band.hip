// Band spread: the density (Sec. 2.3.2, Eq. charge_dipole_assign) or the tangent
// density of the Hessian-vector product, for meshes whose padded y-z plane does
// not fit in LDS beside the slab transform (so no plane spread fused with it).
//
// One workgroup owns a band of y-rows [Y0, Y0 + rows) of one x-plane X.  It takes
// from the bins every atom whose stencil reaches the plane and the band, and adds
// the atom's p x p footprint in that plane, restricted to the band's rows, into an
// LDS band of rows x (N_z + p - 1) 64-bit fixed-point words: a stencil point (j, k)
// of an atom anchored at (b_y, b_z) lands in the row of mesh row b_y - lo + j and
// the padded column b_z + k, so no z stencil wraps inside the band.  The write-back
// folds the extra columns into their periodic images and stores the band's rows of
// rho with plain coalesced stores.
//
// Rows are owned, not shared: an atom near a band edge adds in each band only the
// rows that band owns, so the mesh needs no clearing and no global atomics.  Every
// contribution is the tile spread's own fixed-point word (the same expressions, the
// same tables, the same scale), and 64-bit integer sums do not depend on their
// order, so rho equals the tile spread's bit for bit.
//
// Against the owner-computes tiles this spends a workgroup's lanes on stencil
// points that are all inside the band except in the p - 1 edge rows, and makes each
// atom's weights once per plane and band instead of once per tile.
//
// TREC: the density from the tangent records (q and mu; q and J mu are formed here,
// with the same expressions as the forward binning), so that pme_step bins once.
#include "kernels.h"
#include "pme_common.h"
#include "plane_spread.h"

namespace pme {
namespace {

struct BandArgs {
  int N[3], B[3], nb[3];
  int cap;
  const int* count;
  const int* ovf_count;
  const unsigned* cmax;
  const float* rec;
  long long ovf_base;      // record index of the overflow list
  int PZ;                  // padded row length N_z + p - 1
  int rows;                // rows per band (the last band of a plane may have fewer)
  int nband;               // bands per plane
  int nscan_max;           // bins a band may scan
  int map_cap;             // slots of the item -> bin map
  int hits_cap;            // entries of the hit list (>= kFusedSlotsPerThread blockDim)
  float* rho;
};

// The bins along one axis whose anchors lie in the cyclic range [first, first + len):
// from bin k0 on, n of them (all of them when the range covers the axis).
__device__ __forceinline__ void bin_run(int first, int len, int N, int B, int nb, int& k0,
                                        int& n) {
  if (len >= N) {
    k0 = 0;
    n = nb;
    return;
  }
  const int a = wrapn(first, N), b = wrapn(first + len - 1, N);
  k0 = a / B;
  const int k1 = b / B;
  if (a + len - 1 < N) n = k1 - k0 + 1;
  else n = (k1 < k0) ? nb - k0 + k1 + 1 : nb;
  n = min(n, nb);
}

template <int P, int DEG, bool TREC>
__global__ void __launch_bounds__(kSlabThreads) k_spread_band(BandArgs a, const double* box) {
  static_assert(!TREC || DEG == 1, "tangent records serve the forward density");
  constexpr int lo = (P - 1) / 2;
  extern __shared__ unsigned long long band[];
  const int tid = threadIdx.x;
  const int nthr = int(blockDim.x);
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int X = item / a.nband;
  const int Y0 = (item - X * a.nband) * a.rows;
  const int Ny = a.N[1], Nz = a.N[2];
  const int nrows = min(a.rows, Ny - Y0);
  // LDS: the band | bin offsets and bins of the scan | item map | hit list
  int* s_off = reinterpret_cast<int*>(band + size_t(a.rows) * a.PZ);
  int* s_bin = s_off + a.nscan_max + 2;
  uint16_t* s_map = reinterpret_cast<uint16_t*>(s_bin + a.nscan_max + 2);
  int* s_hits = reinterpret_cast<int*>(s_map + a.map_cap);
  __shared__ float s_J[(DEG == 2 || TREC) ? 9 : 1];
  __shared__ int s_nh;
  __shared__ float s_cw[4 * P * P];           // whole-number spline pieces (x weights)
  __shared__ int s_wsum[kSlabThreads / 64];   // per-wavefront sums of the scan
  constexpr int kTab = spline_offset(P);
  if (tid < 4 * P * P) s_cw[tid] = c_spline_whole.coef[kTab + tid];
  if ((DEG == 2 || TREC) && tid == 0) {
    float J[3][3];
    jacobian(cell_from_box(box), a.N, J);
#pragma unroll
    for (int i = 0; i < 9; ++i) s_J[i] = J[i / 3][i % 3];
  }
  // the bins whose anchors reach the plane (x anchors X + lo - P + 1 .. X + lo) and
  // the band (y anchors Y0 + lo - P + 1 .. Y0 + nrows - 1 + lo), every z bin
  int kx0, nlx, ky0, nly;
  bin_run(X + lo - P + 1, P, a.N[0], a.B[0], a.nb[0], kx0, nlx);
  bin_run(Y0 + lo - P + 1, nrows + P - 1, Ny, a.B[1], a.nb[1], ky0, nly);
  const int nbz = a.nb[2];
  const int nyz = nly * nbz;
  const int nscan = nlx * nyz;                // <= a.nscan_max (host guarantees)
  load_slot_counts(
      nscan,
      [&](int e) {
        const int li = e / nyz;
        const int r = e - li * nyz;
        const int yi = r / nbz;
        return (((kx0 + li) % a.nb[0]) * a.nb[1] + (ky0 + yi) % a.nb[1]) * nbz + (r - yi * nbz);
      },
      a.count, a.cap, a.ovf_count, s_off, s_bin);
  if (tid == 0) s_nh = 0;
  // the fixed-point unit of the tile spread (the same bound and the same scale)
  constexpr float kWhole3 = float(spline_norm(P)) * float(spline_norm(P)) * float(spline_norm(P));
  float scale = 1.0f;
  {
    const float cm = __uint_as_float(*a.cmax);
    if (cm > 0.0f && isfinite(cm)) scale = ldexpf(1.0f, 31 - (ilogbf(8.0f * cm * kWhole3) + 1));
  }
  const int bvol = nrows * a.PZ;
  for (int e = tid; e < bvol; e += nthr) band[e] = 0ull;
  __syncthreads();
  int total;
  const bool mapped = scan_slot_counts(nscan, s_off, s_wsum, s_map, a.map_cap, total);
  auto record_of = [&](int it) {
    return scanned_record(it, mapped, nscan, s_off, s_bin, s_map, a.cap, a.ovf_base);
  };
  // the first stencil row of an anchor relative to the band (mod N_y)
  auto row_rel = [&](int by) {
    int t = by - lo - Y0;
    t += (t < 0) ? Ny : 0;
    t += (t < 0) ? Ny : 0;
    t -= (t >= Ny) ? Ny : 0;
    return t;
  };
  // one atom: its footprint in the plane, in the band's rows (stencil row iy of an atom
  // anchored at b_y lies on mesh row b_y - lo + iy)
  auto add_atom = [&](size_t ri) {
    add_atom_plane<P, DEG, TREC>(a.rec, ri, s_J, s_cw, X, a.N[0], scale, band, a.PZ,
                                 [&](int by, int iy) {
                                   const int rr = row_rel(by) + iy;
                                   return rr - ((rr >= Ny) ? Ny : 0);
                                 },
                                 nrows);
  };

  // rounds of kFusedSlotsPerThread scanned slots per thread (their anchor words
  // loaded together): the atoms whose stencil covers the plane and the band are
  // listed; the list is drained (one atom per thread) when another round might not
  // fit and after the last round
  constexpr int U = kFusedSlotsPerThread;
  for (int r0 = 0; r0 < total; r0 += U * nthr) {
    size_t ri[U];
    int pk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int it = r0 + u * nthr + tid;
      ri[u] = (it < total) ? record_of(it) : size_t(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      pk[u] = (r0 + u * nthr + tid < total) ? __float_as_int(a.rec[ri[u] * kRecWords + 3]) : -1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      bool hit = false;
      if (pk[u] >= 0) {
        int d = X - (pk[u] & 1023) + lo;
        d += (d < 0) ? a.N[0] : 0;
        d -= (d >= a.N[0]) ? a.N[0] : 0;
        const int t = row_rel((pk[u] >> 10) & 1023);
        hit = d < P && (t < nrows || t + P - 1 >= Ny);
      }
      const int k = wave_compact(hit, &s_nh);
      if (hit) s_hits[k] = int(ri[u]);
    }
    __syncthreads();
    const int nh = s_nh;
    __syncthreads();   // every thread has read the count before it changes
    if (nh + U * nthr > a.hits_cap || r0 + U * nthr >= total) {
      for (int e = tid; e < nh; e += nthr) add_atom(size_t(uint32_t(s_hits[e])));
      if (tid == 0) s_nh = 0;
      __syncthreads();
    }
  }
  // write-back: each row's extra columns folded into their periodic images
  const double inv_scale = 1.0 / (double(scale) * double(kWhole3));
  float* out = a.rho + (size_t(X) * Ny + Y0) * Nz;
  const int nout = nrows * Nz;
  for (int e = tid; e < nout; e += nthr) {
    const int rr = e / Nz, z = e - rr * Nz;
    const unsigned long long* row = band + size_t(rr) * a.PZ;
    const int pz = z + lo;
    unsigned long long acc = row[pz];
    if (pz + Nz < a.PZ) acc += row[pz + Nz];
    if (pz >= Nz) acc += row[pz - Nz];
    out[e] = from_fixed((long long)acc, inv_scale);
  }
}

}  // namespace

hipError_t launch_spread_band(const DevPlan& d, hipStream_t s, int set, bool tangent,
                              const double* box, const LaunchEvents* ev, const RecordSource* from) {
  if (!d.band || (from && (tangent || !from->d || !from->cmax))) return hipErrorInvalidValue;
  BandArgs a;
  for (int k = 0; k < 3; ++k) { a.N[k] = d.N[k]; a.B[k] = d.B[k]; a.nb[k] = d.nb[k]; }
  // the bins (same geometry in both views of a plan) and the scale
  const DevPlan& r = from ? *from->d : d;
  const int rs = from ? from->set : set;
  a.cap = r.cap;
  a.count = r.count[rs]; a.ovf_count = r.ovf_count[rs];
  a.cmax = from ? from->cmax : d.cmax[set];
  a.rec = r.rec; a.ovf_base = r.ovf_base;
  a.PZ = d.N[2] + d.p - 1;
  a.rows = d.band_rows;
  a.nband = (d.N[1] + d.band_rows - 1) / d.band_rows;
  a.nscan_max = d.band_nscan;
  a.map_cap = kFusedMap;
  a.hits_cap = kBandHits;
  a.rho = d.rho;
  const dim3 g(d.N[0] * a.nband), b(kSlabThreads);
  const size_t sh = d.band_lds;
#define PME_B(P)                                                              \
  case P:                                                                     \
    if (tangent) launch_k(ev, k_spread_band<P, 2, false>, g, b, sh, s, a, box); \
    else if (from) launch_k(ev, k_spread_band<P, 1, true>, g, b, sh, s, a, box); \
    else launch_k(ev, k_spread_band<P, 1, false>, g, b, sh, s, a, box);        \
    break;
  switch (d.p) {
    PME_B(1) PME_B(2) PME_B(3) PME_B(4) PME_B(5) PME_B(6) PME_B(7)
    default: return hipErrorInvalidValue;
  }
#undef PME_B
  return hipGetLastError();
}

hipError_t enable_band_lds() {
  const void* fns[] = {
#define PME_B(P)                                                   \
  reinterpret_cast<const void*>(k_spread_band<P, 1, false>),       \
      reinterpret_cast<const void*>(k_spread_band<P, 1, true>),    \
      reinterpret_cast<const void*>(k_spread_band<P, 2, false>),
      PME_B(1) PME_B(2) PME_B(3) PME_B(4) PME_B(5) PME_B(6) PME_B(7)
#undef PME_B
  };
  for (const void* f : fns) {
    const hipError_t e =
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kSlabLdsMax);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace pme
