// Charge + dipole assignment onto the mesh (Sec. 2.3.2, Eq. charge_dipole_assign)
// and the tangent density of the Hessian-vector product.
//
// Two kernels:
//  * k_bin: one thread per atom computes its fractional coordinates, stencil
//    anchor b and offset f (Sec. 2.3.2), and the monomial coefficients of what it
//    assigns, c_abc, such that the value it adds at stencil point (i, j, k) is
//        sum_abc c_abc W_x^(a)[i] W_y^(b)[j] W_z^(c)[k]
//    (forward: c_000 = q, c_100..c_001 = N_a (mu . C^-1[:,a]); tangent: degree <= 2,
//    see tangent_coefs).  It files a 16-word record into a fixed-capacity bin of
//    B_x x B_y x B_z anchors (overflow goes to a list) and, for the forward,
//    block partial sums of q^2 and |mu|^2 for the self terms (Eqs. self_q, self_mu).
//  * k_spread: one workgroup owns one mesh tile.  It scans the bins whose anchors
//    can reach the tile, stages the overlapping atoms' weights in LDS, accumulates
//    their contributions with LDS float adds, and writes the tile back with plain
//    coalesced stores.  Halo contributions are computed by every tile they touch
//    instead of being flushed with global atomics, so the mesh needs no clearing
//    and no global read-modify-write.
#include "kernels.h"
#include "pme_common.h"

namespace pme {
namespace {

constexpr int kRecW = 16;   // record words: f[3], packed base, coefs[<=10], pad

struct BinArgs {
  int n;
  const float* pos;
  const float* q;
  const float* mu;
  const double* box;
  const float* v_pos;
  const float* v_q;
  const float* v_mu;
  int N[3];
  int B[3];
  int nb[3];
  int cap;
  int* count;
  int* ovf_count;
  float* rec;
  float* ovf_rec;
  double* spart;
  int* status;
};

__device__ __forceinline__ float3 ld3(const float* p, int i) {
  return p ? make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]) : make_float3(0.f, 0.f, 0.f);
}

// d = J v  (x-space components of a Cartesian vector)
__device__ __forceinline__ float3 jmul(const float (&J)[3][3], float3 v) {
  return make_float3(J[0][0] * v.x + J[0][1] * v.y + J[0][2] * v.z,
                     J[1][0] * v.x + J[1][1] * v.y + J[1][2] * v.z,
                     J[2][0] * v.x + J[2][1] * v.y + J[2][2] * v.z);
}

template <int P, bool TANGENT>
__global__ void __launch_bounds__(256) k_bin(BinArgs a) {
  __shared__ double red[8];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const Cell c = cell_from_box(a.box);
  double sq = 0.0, smu = 0.0;
  if (i < a.n) {
    int base[3];
    float f[3];
    const bool ok = atom_stencil<P>(a.pos, i, c, a.N, base, f);
    const float q = a.q ? a.q[i] : 0.0f;
    const float3 mu = ld3(a.mu, i);
    sq = double(q) * q;
    smu = double(mu.x) * mu.x + double(mu.y) * mu.y + double(mu.z) * mu.z;
    if (!ok) {
      atomicOr(a.status, 1);
    } else {
      float J[3][3];
      jacobian(c, a.N, J);
      const float3 d = jmul(J, mu);
      float co[10];
      int nc;
      if (!TANGENT) {
        co[0] = q; co[1] = d.x; co[2] = d.y; co[3] = d.z;
        nc = 4;
      } else {
        // rho_dot = v_q W + w.grad_x W + d^T (grad_x grad_x W) v,
        // w = J (v_mu + q v_r), v = J v_r, d = J mu
        const float vq = a.v_q ? a.v_q[i] : 0.0f;
        const float3 vr = ld3(a.v_pos, i);
        const float3 vm = ld3(a.v_mu, i);
        const float3 w = jmul(J, make_float3(vm.x + q * vr.x, vm.y + q * vr.y, vm.z + q * vr.z));
        const float3 v = jmul(J, vr);
        co[0] = vq;
        co[1] = w.x; co[2] = w.y; co[3] = w.z;
        co[4] = d.x * v.x; co[5] = d.y * v.y; co[6] = d.z * v.z;     // 200 020 002
        co[7] = d.x * v.y + d.y * v.x;                               // 110
        co[8] = d.x * v.z + d.z * v.x;                               // 101
        co[9] = d.y * v.z + d.z * v.y;                               // 011
        nc = 10;
      }
      const int bin = ((base[0] / a.B[0]) * a.nb[1] + base[1] / a.B[1]) * a.nb[2] + base[2] / a.B[2];
      const int slot = atomicAdd(&a.count[bin], 1);
      float* dst;
      if (slot < a.cap) {
        dst = a.rec + (size_t(bin) * a.cap + slot) * kRecW;
      } else {
        const int o = atomicAdd(a.ovf_count, 1);
        dst = a.ovf_rec + size_t(o) * kRecW;
      }
      float4* d4 = reinterpret_cast<float4*>(dst);
      d4[0] = make_float4(f[0], f[1], f[2],
                          __int_as_float(base[0] | (base[1] << 10) | (base[2] << 20)));
      d4[1] = make_float4(co[0], co[1], co[2], co[3]);
      if (nc == 10) {
        d4[2] = make_float4(co[4], co[5], co[6], co[7]);
        d4[3] = make_float4(co[8], co[9], 0.f, 0.f);
      }
    }
  }
  if (!TANGENT && a.spart) {
    const double s1 = block_sum(sq, red);
    const double s2 = block_sum(smu, red);
    if (threadIdx.x == 0) {
      a.spart[2 * blockIdx.x] = s1;
      a.spart[2 * blockIdx.x + 1] = s2;
    }
  }
}

struct SpreadArgs {
  int N[3];
  int B[3];
  int nb[3];
  int cap;
  const int* count;
  const int* ovf_count;
  const float* rec;
  const float* ovf_rec;
  int T[3];
  int nt[3];
  float* rho;
};

constexpr int kTileMax = 1024;

// Bitmask of the stencil points j whose wrapped mesh index falls in [t0, t0+T),
// and the tile-local coordinate of each.
template <int P>
__device__ __forceinline__ int axis_overlap(int b, int t0, int T, int N, int (&loc)[P]) {
  constexpr int lo = (P - 1) / 2;
  int mask = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int l = wrapn(b - lo + j, N) - t0;
    loc[j] = l;
    if (l >= 0 && l < T) mask |= 1 << j;
  }
  return mask;
}

template <int P, int DEG>
__global__ void __launch_bounds__(256) k_spread(SpreadArgs a) {
  constexpr int NC = (DEG == 1) ? 4 : 10;
  constexpr int D = DEG;                    // highest weight derivative needed
  constexpr int lo = (P - 1) / 2;
  // staged atom: weights w[axis][d][j], coefs, base, masks
  constexpr int kEnt = 3 * (D + 1) * P + NC + 2;
  __shared__ float s_tile[kTileMax];
  __shared__ int s_off[kMaxBinRange + 2];
  __shared__ int s_bin[kMaxBinRange + 1];
  __shared__ float s_list[kListCap * kEnt];
  __shared__ int s_nlist;
  __shared__ int s_part[256];

  const int tid = threadIdx.x;
  int tcoord[3];
  {
    int t = blockIdx.x;
    tcoord[2] = t % a.nt[2]; t /= a.nt[2];
    tcoord[1] = t % a.nt[1];
    tcoord[0] = t / a.nt[1];
  }
  int t0[3], T[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    t0[ax] = tcoord[ax] * a.T[ax];
    T[ax] = min(a.T[ax], a.N[ax] - t0[ax]);
  }
  const int tvol = T[0] * T[1] * T[2];
  for (int e = tid; e < tvol; e += 256) s_tile[e] = 0.0f;

  // bins whose anchors b can reach the tile: b in [t0 + lo - P + 1, t0 + T - 1 + lo]
  int kmin[3], nk[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int bmin = t0[ax] + lo - P + 1, bmax = t0[ax] + T[ax] - 1 + lo;
    const int k0 = (bmin >= 0) ? bmin / a.B[ax] : -((-bmin + a.B[ax] - 1) / a.B[ax]);
    const int k1 = (bmax >= 0) ? bmax / a.B[ax] : -((-bmax + a.B[ax] - 1) / a.B[ax]);
    nk[ax] = k1 - k0 + 1;
    kmin[ax] = k0;
    if (nk[ax] >= a.nb[ax]) { nk[ax] = a.nb[ax]; kmin[ax] = 0; }
  }
  const int nbr = nk[0] * nk[1] * nk[2];     // <= kMaxBinRange (host guarantees)
  for (int e = tid; e < nbr; e += 256) {
    const int kz = e % nk[2], ky = (e / nk[2]) % nk[1], kx = e / (nk[1] * nk[2]);
    int bx = (kmin[0] + kx) % a.nb[0]; bx += (bx < 0) ? a.nb[0] : 0;
    int by = (kmin[1] + ky) % a.nb[1]; by += (by < 0) ? a.nb[1] : 0;
    int bz = (kmin[2] + kz) % a.nb[2]; bz += (bz < 0) ? a.nb[2] : 0;
    const int bin = (bx * a.nb[1] + by) * a.nb[2] + bz;
    s_bin[e] = bin;
    s_off[e] = min(a.count[bin], a.cap);
  }
  if (tid == 0) {
    s_bin[nbr] = -1;                           // pseudo-bin: the overflow list
    s_off[nbr] = *a.ovf_count;
    s_nlist = 0;
  }
  __syncthreads();
  // exclusive scan of s_off[0..nbr]: each thread scans a contiguous segment
  {
    const int len = nbr + 1;
    const int seg = (len + 255) / 256;
    const int s0 = min(tid * seg, len), s1 = min(s0 + seg, len);
    int acc = 0;
    for (int e = s0; e < s1; ++e) acc += s_off[e];
    s_part[tid] = acc;
    __syncthreads();
    if (tid == 0) {
      int run = 0;
      for (int w = 0; w < 256; ++w) { const int v = s_part[w]; s_part[w] = run; run += v; }
    }
    __syncthreads();
    int run = s_part[tid];
    for (int e = s0; e < s1; ++e) { const int v = s_off[e]; s_off[e] = run; run += v; }
    if (tid == 255) s_off[len] = run;
    __syncthreads();
  }
  const int total = s_off[nbr + 1];

  for (int r0 = 0; r0 < total; r0 += kListCap) {
    // stage overlapping atoms of this round
    const int item = r0 + tid;
    if (tid < kListCap && item < total) {
      int lo_i = 0, hi_i = nbr;                 // largest bin index with s_off <= item
      while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i + 1) >> 1;
        if (s_off[mid] <= item) lo_i = mid; else hi_i = mid - 1;
      }
      const int bin = s_bin[lo_i];
      const int slot = item - s_off[lo_i];
      const float* src = (bin >= 0) ? a.rec + (size_t(bin) * a.cap + slot) * kRecW
                                    : a.ovf_rec + size_t(slot) * kRecW;
      const float4 h = reinterpret_cast<const float4*>(src)[0];
      const int pk = __float_as_int(h.w);
      const int b[3] = {pk & 1023, (pk >> 10) & 1023, (pk >> 20) & 1023};
      int lx[P], ly[P], lz[P];
      const int mx = axis_overlap<P>(b[0], t0[0], T[0], a.N[0], lx);
      const int my = axis_overlap<P>(b[1], t0[1], T[1], a.N[1], ly);
      const int mz = axis_overlap<P>(b[2], t0[2], T[2], a.N[2], lz);
      if (mx && my && mz) {
        const int e = atomicAdd(&s_nlist, 1);
        float* ent = s_list + e * kEnt;
        const float fr[3] = {h.x, h.y, h.z};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          float w[D + 1][P];
          spline_weights<P, D>(fr[ax], w);
#pragma unroll
          for (int d = 0; d <= D; ++d)
#pragma unroll
            for (int j = 0; j < P; ++j) ent[(ax * (D + 1) + d) * P + j] = w[d][j];
        }
        const float4* s4 = reinterpret_cast<const float4*>(src) + 1;
        float co[12];
        const float4 c0 = s4[0];
        co[0] = c0.x; co[1] = c0.y; co[2] = c0.z; co[3] = c0.w;
        if (NC == 10) {
          const float4 c1 = s4[1], c2 = s4[2];
          co[4] = c1.x; co[5] = c1.y; co[6] = c1.z; co[7] = c1.w;
          co[8] = c2.x; co[9] = c2.y;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) ent[3 * (D + 1) * P + k] = co[k];
        ent[3 * (D + 1) * P + NC] = __int_as_float(pk);
        ent[3 * (D + 1) * P + NC + 1] = __int_as_float(mx | (my << 8) | (mz << 16));
      }
    }
    __syncthreads();
    // accumulate: one task per (atom, x-point, y-point) column of the stencil
    const int nl = s_nlist;
    for (int t = tid; t < nl * P * P; t += 256) {
      const int e = t / (P * P), cc = t - e * (P * P);
      const int ix = cc / P, iy = cc - ix * P;
      const float* ent = s_list + e * kEnt;
      const int masks = __float_as_int(ent[3 * (D + 1) * P + NC + 1]);
      if (!((masks >> ix) & 1) || !((masks >> (8 + iy)) & 1)) continue;
      const int pk = __float_as_int(ent[3 * (D + 1) * P + NC]);
      const int mz = (masks >> 16) & 255;
      const float* wx = ent;                       // wx[d*P + j]
      const float* wy = ent + (D + 1) * P;
      const float* wz = ent + 2 * (D + 1) * P;
      const float* co = ent + 3 * (D + 1) * P;
      float c0, c1, c2 = 0.0f;
      if (DEG == 1) {
        const float x0 = wx[ix], x1 = wx[P + ix], y0 = wy[iy], y1 = wy[P + iy];
        c0 = co[0] * x0 * y0 + co[1] * x1 * y0 + co[2] * x0 * y1;
        c1 = co[3] * x0 * y0;
      } else {
        const float x0 = wx[ix], x1 = wx[P + ix], x2 = wx[2 * P + ix];
        const float y0 = wy[iy], y1 = wy[P + iy], y2 = wy[2 * P + iy];
        c0 = co[0] * x0 * y0 + co[1] * x1 * y0 + co[2] * x0 * y1 + co[4] * x2 * y0 +
             co[5] * x0 * y2 + co[7] * x1 * y1;
        c1 = co[3] * x0 * y0 + co[8] * x1 * y0 + co[9] * x0 * y1;
        c2 = co[6] * x0 * y0;
      }
      int lxy;
      {
        const int bx = pk & 1023, by = (pk >> 10) & 1023, bz = (pk >> 20) & 1023;
        int m = wrapn(bx - lo + ix, a.N[0]) - t0[0];
        int n = wrapn(by - lo + iy, a.N[1]) - t0[1];
        lxy = (m * T[1] + n) * T[2];
        int zb = bz - lo;
#pragma unroll
        for (int iz = 0; iz < P; ++iz) {
          if (!((mz >> iz) & 1)) continue;
          const int lz = wrapn(zb + iz, a.N[2]) - t0[2];
          float v = c0 * wz[iz] + c1 * wz[P + iz];
          if (DEG == 2) v += c2 * wz[2 * P + iz];
          atomicAdd(&s_tile[lxy + lz], v);
        }
      }
    }
    __syncthreads();
    if (tid == 0) s_nlist = 0;
    __syncthreads();
  }

  // write the tile (z rows contiguous)
  for (int e = tid; e < tvol; e += 256) {
    const int lz = e % T[2], ly = (e / T[2]) % T[1], lx = e / (T[1] * T[2]);
    a.rho[(size_t(t0[0] + lx) * a.N[1] + (t0[1] + ly)) * a.N[2] + t0[2] + lz] = s_tile[e];
  }
}

template <bool TANGENT>
hipError_t bin_dispatch(int p, dim3 g, hipStream_t s, const BinArgs& a) {
  switch (p) {
    case 1: hipLaunchKernelGGL((k_bin<1, TANGENT>), g, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_bin<2, TANGENT>), g, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_bin<3, TANGENT>), g, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_bin<4, TANGENT>), g, dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_bin<5, TANGENT>), g, dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_bin<6, TANGENT>), g, dim3(256), 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_bin<7, TANGENT>), g, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int DEG>
hipError_t spread_dispatch(int p, dim3 g, hipStream_t s, const SpreadArgs& a) {
  switch (p) {
    case 1: hipLaunchKernelGGL((k_spread<1, DEG>), g, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_spread<2, DEG>), g, dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_spread<3, DEG>), g, dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_spread<4, DEG>), g, dim3(256), 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_spread<5, DEG>), g, dim3(256), 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_spread<6, DEG>), g, dim3(256), 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_spread<7, DEG>), g, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bin(const DevPlan& d, hipStream_t s, int n, const float* pos, const float* q,
                      const float* mu, const double* box, const float* v_pos, const float* v_q,
                      const float* v_mu, bool tangent, bool self_sums) {
  BinArgs a;
  a.n = n; a.pos = pos; a.q = q; a.mu = mu; a.box = box;
  a.v_pos = v_pos; a.v_q = v_q; a.v_mu = v_mu;
  for (int k = 0; k < 3; ++k) { a.N[k] = d.N[k]; a.B[k] = d.B[k]; a.nb[k] = d.nb[k]; }
  a.cap = d.cap; a.count = d.count; a.ovf_count = d.ovf_count;
  a.rec = d.rec; a.ovf_rec = d.ovf_rec;
  a.spart = self_sums ? d.spart : nullptr;
  a.status = d.status;
  const dim3 g(bin_blocks(n));
  return tangent ? bin_dispatch<true>(d.p, g, s, a) : bin_dispatch<false>(d.p, g, s, a);
}

hipError_t launch_spread(const DevPlan& d, hipStream_t s, bool tangent) {
  SpreadArgs a;
  for (int k = 0; k < 3; ++k) {
    a.N[k] = d.N[k]; a.B[k] = d.B[k]; a.nb[k] = d.nb[k]; a.T[k] = d.T[k]; a.nt[k] = d.nt[k];
  }
  a.cap = d.cap; a.count = d.count; a.ovf_count = d.ovf_count;
  a.rec = d.rec; a.ovf_rec = d.ovf_rec; a.rho = d.rho;
  const dim3 g(d.nt[0] * d.nt[1] * d.nt[2]);
  return tangent ? spread_dispatch<2>(d.p, g, s, a) : spread_dispatch<1>(d.p, g, s, a);
}

}  // namespace pme
