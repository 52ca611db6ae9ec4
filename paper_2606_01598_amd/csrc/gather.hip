// Gradient gather (Eqs. energy_recip, self_q, self_mu, E_lr_total, forces) and
// the Hessian-vector product gather.
//
// One workgroup per mesh tile: it stages the potential (and the tangent
// potential) over the tile plus the stencil halo in LDS, takes the atoms whose
// stencil anchor lies in the tile from the bins, and gives each atom p lanes of a
// wavefront (one x-plane of the stencil each).  The lanes' partial stencil sums are
// combined with wavefront shuffles.  The gathers are the last readers of the atom
// bins of its counter set; the next binning clears that set.
//
// For atom i with stencil weights W (and x-space derivatives d_a W), the
// derivatives of E^lr = (1/2V) rho^T K rho + E_self are stencil sums of the
// potential phi = K rho:
//     dE/dq_i  = (1/V) sum W phi                       - 2a/sqrt(pi) q_i
//     dE/dmu_i = (1/V) J^T sum grad_x W phi            - 4a^3/(3 sqrt(pi)) mu_i
//     dE/dr_i  = (1/V) J^T [q_i sum grad_x W phi + (sum grad_x grad_x W phi) J mu_i]
// with J[a][b] = N_a (C^-1)[b][a].  Sums are separable: z partials per stencil
// column, then y, then x, so each of the p^3 points costs a few FMAs.
//
// The Hessian-vector product with cotangents (v_r, v_q, v_mu) also needs the
// tangent potential psi = K rho_dot (rho_dot spread by the tangent records):
//     q_bar  = (1/V)(P0 + S1 . v)                           - 2a/sqrt(pi) v_q
//     mu_bar = (1/V) J^T (P1 + S2 v)                        - 4a^3/(3 sqrt(pi)) v_mu
//     r_bar  = (1/V) J^T [q P1 + P2 d + v_q S1 + S2 w + S3(d, v, .)]
// where P_k are the order-k derivative sums of psi, S_k those of phi,
// d = J mu, v = J v_r, w = J (v_mu + q v_r).
//
// The quadrupole forward (second moments Theta, Q = J Theta J^T) adds
//     dE/dq_i     += 2a^3/(3 sqrt(pi)) tr Theta_i
//     dE/dTheta_i  = (1/2V) J^T S_2 J + d/dTheta [2a^3/(3 sqrt(pi)) q tr Theta
//                    - a^5/(5 sqrt(pi)) (tr^2 Theta + 2 Theta:Theta)]
//     dE/dr_i     += (1/V) J^T (1/2) S_3 : Q
// (Theta gradients of the six stored entries xx yy zz xy xz yz).
#include <vector>

#include "kernels.h"
#include "pme_common.h"

namespace pme {
namespace {

struct GArgs {
  int n;
  const float* pos;
  const float* q;
  const float* mu;
  const double* box;
  int N[3];
  const float* phi;
  const float* psi;
  const float* v_pos;
  const float* v_q;
  const float* v_mu;
  float* o_pos;
  float* o_q;
  float* o_mu;
  // Hessian-vector gather only: the forward outputs of the same atoms as well (the
  // stencil sums of phi it forms include those of the gradient); null to skip
  float* f_pos;
  float* f_q;
  float* f_mu;
  double* energy;
  const double* epart;
  int n_epart;
  const double* spart;
  int n_spart;
  double alpha;
  double prefactor;
  // quadrupole forward: second moments, their gradient, the block sums of the
  // Theta self terms (2 per binning block) and a^5 / (5 sqrt(pi))
  const float* theta;
  float* o_theta;
  const double* spart_th;
  float cth;
  // float constants of the outputs, made on the host: the prefactor, the self-term
  // factors 2 alpha / sqrt(pi) and 4 alpha^3 / (3 sqrt(pi))
  float pf, cq, cm;
  // cell gradient (forward gather, VIR variant): 9 partials per tile,
  // sum_i s_i (x) N (q_i G_i + H_i J mu_i) + (mu_i C^-1) (x) N G_i, s_i = r_i C^-1
  double* vpart;
  int B[3];
  int nb[3];
  int cap;
  const int* count;
  const int* ovf_count;
  const float* rec;
  long long ovf_base;      // record index of the overflow list
  int T[3];
  int nt[3];
  int off;                 // batches: offset of the box's atoms in the packed arrays
};


__device__ void finalize_energy(const GArgs& a, const Cell& c) {
  __shared__ double red[8];
  double e = 0.0, s1 = 0.0, s2 = 0.0;
  for (int k = threadIdx.x; k < a.n_epart; k += blockDim.x) e += a.epart[k];
  for (int k = threadIdx.x; k < a.n_spart; k += blockDim.x) {
    s1 += a.spart[2 * k];
    s2 += a.spart[2 * k + 1];
  }
  e = block_sum(e, red);
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    const double sp = sqrt(M_PI);
    a.energy[0] = a.prefactor * e / (2.0 * c.vol);
    a.energy[1] = -a.prefactor * a.alpha / sp * s1;
    a.energy[2] = -a.prefactor * 2.0 * a.alpha * a.alpha * a.alpha / (3.0 * sp) * s2;
  }
  if (a.spart_th) {
    double s3 = 0.0, s4 = 0.0;
    for (int k = threadIdx.x; k < a.n_spart; k += blockDim.x) {
      s3 += a.spart_th[2 * k];
      s4 += a.spart_th[2 * k + 1];
    }
    s3 = block_sum(s3, red);
    s4 = block_sum(s4, red);
    if (threadIdx.x == 0) {
      const double sp = sqrt(M_PI), a3 = a.alpha * a.alpha * a.alpha;
      a.energy[3] = a.prefactor * (2.0 * a3 / (3.0 * sp) * s3 - a3 * a.alpha * a.alpha / (5.0 * sp) * s4);
    }
  }
}

// J^T u
__device__ __forceinline__ float3 jtmul(const float (&J)[3][3], float3 u) {
  return make_float3(J[0][0] * u.x + J[1][0] * u.y + J[2][0] * u.z,
                     J[0][1] * u.x + J[1][1] * u.y + J[2][1] * u.z,
                     J[0][2] * u.x + J[1][2] * u.y + J[2][2] * u.z);
}
__device__ __forceinline__ float3 ld3(const float* p, int i) {
  return p ? make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]) : make_float3(0.f, 0.f, 0.f);
}
__device__ __forceinline__ void st3(float* p, int i, float3 v) {
  if (p) { p[3 * i] = v.x; p[3 * i + 1] = v.y; p[3 * i + 2] = v.z; }
}

// Sum over the P consecutive lanes of a group; the total lands on the group's first lane.
template <int P>
__device__ __forceinline__ float group_sum(float v, int ix) {
#pragma unroll
  for (int off = 1; off < P; off <<= 1) {
    const float o = __shfl_down(v, off, 64);
    if (ix + off < P) v += o;
  }
  return v;
}

// ceil(2^32 / d) as 0xffffffff / d + 1 (a 32-bit division; d = 1 passes through)
__device__ __forceinline__ FastDiv make_fastdiv(int d) {
  FastDiv f;
  f.d = uint32_t(d);
  f.m = d <= 1 ? 0u : 0xffffffffu / uint32_t(d) + 1u;
  return f;
}

// One tile of either gather.
//  1. One round trip: every thread loads the record of one slot of the tile's own
//     bins speculatively (slot e is slot e mod cap of own bin e / cap; it is used only
//     if it is occupied), the own-bin counts, the overflow count and the field
//     region(s) over the tile plus the stencil halo.
//  2. Rounds of up to 256 slots: occupied slots are compacted into an LDS queue
//     (the next round's records are loaded meanwhile) and the queue is processed
//     with p lanes per atom.
//  3. Overflow records whose anchor lies in the tile, the same way.
// Queue entries: the anchor header and, forward: q, mu, atom; Hessian-vector
// product: q, mu, v_q, v_r, v_mu, atom (the tangent record carries them).

// What the queue needs of a record: the anchor header and, forward: q, mu, atom;
// Hessian-vector product: (q, mu), (v_q, v_r), (v_mu, atom).
template <bool HVP>
struct RecRegs {
  float4 h, r1, r2, r3;
};
template <>
struct RecRegs<false> {
  float4 h, qm;
  float4 sa;   // unwrapped fractional position, atom index (bits)
};

template <bool HVP>
__device__ __forceinline__ RecRegs<HVP> load_rec(const float* rec, size_t ri) {
  const float4* r = reinterpret_cast<const float4*>(rec + ri * kRecWords);
  RecRegs<HVP> o;
  if constexpr (HVP) {
    o.h = r[0];
    o.r1 = r[1];
    o.r2 = r[2];
    o.r3 = r[3];
  } else {
    const float* f = rec + ri * kRecWords;
    o.h = r[0];
    o.qm = make_float4(f[4], f[8], f[9], f[10]);
    o.sa = r[3];
  }
  return o;
}

template <int P, bool HVP, bool DUAL = false, bool VIR = false, bool QUAD = false>
__device__ __forceinline__ void gather_tile(const GArgs& a, const int tile) {
  extern __shared__ float sm[];
  // records of four float4 (Hessian-vector product, quadrupole forward)
  constexpr bool R4 = HVP || QUAD;
  // the queue holds kGatherQueue atoms; a round's compacted records beyond that are
  // processed in further chunks, reloaded from the records
  __shared__ float4 s_h[kGatherQueue];
  __shared__ float4 s_qm[kGatherQueue];              // q, mu (quadrupole: q, J mu)
  __shared__ float4 s_v1[R4 ? kGatherQueue : 1];     // v_q, v_r (quadrupole: c_200 .. c_110)
  __shared__ float4 s_v2[R4 ? kGatherQueue : 1];     // v_mu, atom (quadrupole: c_101 c_011 - atom)
  __shared__ int s_atom[R4 ? 1 : kGatherQueue];      // forward
  __shared__ float4 s_sa[VIR ? kGatherQueue : 1];    // VIR: unwrapped fractional position
  __shared__ int s_n;
  __shared__ float s_coef[4 * P * P];       // pieces of N_P and their derivatives
  constexpr int lo = (P - 1) / 2;
  constexpr int APW = 64 / P;
  const int tid = threadIdx.x;
  if (tid == 0) s_n = 0;
  // the spline table is loaded now and stored in LDS after the field region, so that
  // no barrier waits for it
  static_assert(4 * P * P <= 256, "one coefficient per thread");
  const float coef = tid < 4 * P * P ? c_spline.coef[spline_offset(P) + tid] : 0.0f;
  const Cell c = cell_from_box(a.box);
  if (tile == 0 && a.energy) finalize_energy(a, c);
  int t0[3], T[3], E[3];
  {
    int t = tile;
    const int tz = t % a.nt[2];
    t /= a.nt[2];
    const int ty = t % a.nt[1];
    const int tx = t / a.nt[1];
    const int tc[3] = {tx, ty, tz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      t0[ax] = tc[ax] * a.T[ax];
      T[ax] = min(a.T[ax], a.N[ax] - t0[ax]);
      E[ax] = T[ax] + P - 1;
    }
  }
  int nbo[3], kb0[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    nbo[ax] = T[ax] / a.B[ax];
    kb0[ax] = t0[ax] / a.B[ax];
  }
  const int nown = nbo[0] * nbo[1] * nbo[2];
  const int cap = a.cap;
  const int nslot = nown * cap;
  auto own_bin = [&](int j) {
    const int kz = j % nbo[2], ky = (j / nbo[2]) % nbo[1], kx = j / (nbo[1] * nbo[2]);
    return ((kb0[0] + kx) * a.nb[1] + kb0[1] + ky) * a.nb[2] + kb0[2] + kz;
  };
  auto slot_rec = [&](int e) {
    const int j = e / cap;
    return load_rec<R4>(a.rec, size_t(own_bin(j)) * cap + (e - j * cap));
  };
  // 1. records of the first 256 slots, their bins' counts and the field region in
  // flight together (nslot >= cap > 0: a tile holds whole bins; slots past the end
  // load the last one again and are not used)
  int ec = min(tid, nslot - 1);
  RecRegs<R4> cur = slot_rec(ec);
  int cnt = a.count[own_bin(ec / cap)];
  const int novf = *a.ovf_count;
  const int EV = E[0] * E[1] * E[2];
  // global offsets of the region's rows (ex, ey) and wrapped z coordinates, made
  // once, after the field region in LDS: a region element then costs two LDS reads
  const int nrow = E[0] * E[1];
  int* s_row = reinterpret_cast<int*>(sm + (HVP ? 2 : 1) * EV);
  int* s_zo = s_row + nrow;
  {
    const bool small = (a.N[0] < P) || (a.N[1] < P) || (a.N[2] < P);
    auto wrap = [&](int m, int N) {
      return small ? wrapn(m, N) : ((m < 0) ? m + N : ((m >= N) ? m - N : m));
    };
    const FastDiv d1 = make_fastdiv(E[1]);
    for (int r = tid; r < nrow; r += blockDim.x) {
      const int ex = int(fdiv(uint32_t(r), d1)), ey = r - ex * E[1];
      s_row[r] = (wrap(t0[0] - lo + ex, a.N[0]) * a.N[1] + wrap(t0[1] - lo + ey, a.N[1])) * a.N[2];
    }
    for (int z = tid; z < E[2]; z += blockDim.x) s_zo[z] = wrap(t0[2] - lo + z, a.N[2]);
  }
  __syncthreads();
  {
    const FastDiv d2 = make_fastdiv(E[2]);
    constexpr int U = 16;   // loads kept in flight per thread
    for (int e0 = tid; e0 < EV; e0 += U * blockDim.x) {
      float vphi[U], vpsi[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * blockDim.x;
        const int ec = min(e, EV - 1);
        const int r = int(fdiv(uint32_t(ec), d2));
        const uint32_t g = uint32_t(s_row[r] + s_zo[ec - r * E[2]]);
        vphi[u] = a.phi[g];
        if (HVP) vpsi[u] = a.psi[g];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * blockDim.x;
        if (e < EV) {
          sm[e] = vphi[u];
          if (HVP) sm[EV + e] = vpsi[u];
        }
      }
    }
  }
  if (tid < 4 * P * P) s_coef[tid] = coef;
  // cell and prefactor constants are uniform: kept in scalar registers
  float J[3][3];
  jacobian(c, a.N, J);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) J[i][j] = uniform(J[i][j]);
  const float iv = uniform(float(1.0 / c.vol));
  const float pf = a.pf, cq = a.cq, cm = a.cm;
  // VIR: C^-1 in float and the per-thread sums of the atoms this thread finishes
  float ci[9], vg[9];
  if constexpr (VIR) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      ci[k] = float(c.inv[k]);
      vg[k] = 0.0f;
    }
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int gslot = lane / P, ix = lane - gslot * P;

  auto put = [&](int k, const RecRegs<R4>& r) {
    s_h[k] = r.h;
    if constexpr (R4) {
      s_qm[k] = r.r1;
      s_v1[k] = r.r2;
      s_v2[k] = r.r3;
    } else {
      s_qm[k] = r.qm;
      s_atom[k] = __float_as_int(r.sa.w);
      if constexpr (VIR) s_sa[k] = r.sa;
    }
  };
  // compacted index of a valid record (-1 otherwise); the first kGatherQueue are queued
  auto enqueue = [&](bool valid, const RecRegs<R4>& r) {
    const int k = wave_compact(valid, &s_n);
    if (valid && k < kGatherQueue) put(k, r);
    return k;
  };
  auto process = [&](int nq) {
    for (int b0 = 0; b0 < nq; b0 += 4 * APW) {
      const int slot = b0 + wave * APW + gslot;
      const bool active = (gslot < APW) && (slot < nq);
      // a wavefront with no atom in this pass skips it (its lanes would only sum zeros)
      if (__ballot(active) == 0ull) continue;
      if constexpr (QUAD) {
        // per-lane partial sums of the lane's x-plane, summed over the atom's lanes:
        // S_0, S_1, S_2 (200 020 002 110 101 011) and the pre-J position gradient
        float oq = 0, og[3] = {0, 0, 0}, oh[6] = {0, 0, 0, 0, 0, 0}, op[3] = {0, 0, 0};
        if (active) {
          const float4 h = s_h[slot];
          const int pk = __float_as_int(h.w);
          const int lx = (pk & 1023) - t0[0] + ix;
          const int yb = ((pk >> 10) & 1023) - t0[1], zb = ((pk >> 20) & 1023) - t0[2];
          float wz[4][P], wx[4];
          spline_weights<P, 3>(h.z, wz);
          weight_at_lds<P, 3>(s_coef, ix, h.x, wx);
          const float* plane = sm + (lx * E[1] + yb) * E[2] + zb;
          float Ys[4][4];
#pragma unroll
          for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int z = 0; z < 4; ++z) Ys[y][z] = 0.0f;
#pragma unroll
          for (int iy = 0; iy < P; ++iy) {
            float zs[4] = {0, 0, 0, 0};
#pragma unroll
            for (int iz = 0; iz < P; ++iz) {
              const float v = plane[iy * E[2] + iz];
#pragma unroll
              for (int k = 0; k < 4; ++k) zs[k] = fmaf(v, wz[k][iz], zs[k]);
            }
            float wy[4];
            spline_weight_at<P, 3>(iy, h.y, wy);
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
              for (int k = 0; k + b < 4; ++k) Ys[b][k] = fmaf(wy[b], zs[k], Ys[b][k]);
          }
          // S(x, y, z) = sum W^(x) W^(y) W^(z) phi over the lane's plane, x + y + z <= 3
          auto S = [&](int x, int y, int z) { return wx[x] * Ys[y][z]; };
          const float4 c0 = s_qm[slot], c1 = s_v1[slot], c2 = s_v2[slot];
          const float q = c0.x;
          const float d[3] = {c0.y, c0.z, c0.w};
          // second-order monomials and their coefficients (1/2) Q_aa, Q_ab
          constexpr int mono[6][3] = {{2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
          const float cm2[6] = {c1.x, c1.y, c1.z, c1.w, c2.x, c2.y};
          oq = S(0, 0, 0);
#pragma unroll
          for (int m = 0; m < 6; ++m) oh[m] = S(mono[m][0], mono[m][1], mono[m][2]);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int e[3] = {c == 0, c == 1, c == 2};
            og[c] = S(e[0], e[1], e[2]);
            float v = q * og[c];
#pragma unroll
            for (int b = 0; b < 3; ++b) v = fmaf(S(e[0] + (b == 0), e[1] + (b == 1), e[2] + (b == 2)), d[b], v);
#pragma unroll
            for (int m = 0; m < 6; ++m)
              v = fmaf(S(mono[m][0] + e[0], mono[m][1] + e[1], mono[m][2] + e[2]), cm2[m], v);
            op[c] = v;
          }
        }
        oq = group_sum<P>(oq, ix);
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          og[x] = group_sum<P>(og[x], ix);
          op[x] = group_sum<P>(op[x], ix);
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) oh[m] = group_sum<P>(oh[m], ix);
        if (active && ix == 0) {
          const int i = __float_as_int(s_v2[slot].w);
          const float q = s_qm[slot].x;
          const float3 mu = ld3(a.mu, i);
          float th[6] = {0, 0, 0, 0, 0, 0};
          if (a.theta)
#pragma unroll
            for (int k = 0; k < 6; ++k) th[k] = a.theta[6 * i + k];
          const float tr = th[0] + th[1] + th[2];
          const float c1 = 0.5f * cm, c2 = a.cth;
          if (a.o_q) a.o_q[i] = pf * (oq * iv - cq * q + c1 * tr);
          if (a.o_mu) {
            const float3 g = jtmul(J, make_float3(og[0], og[1], og[2]));
            st3(a.o_mu, i, make_float3(pf * (g.x * iv - cm * mu.x), pf * (g.y * iv - cm * mu.y),
                                       pf * (g.z * iv - cm * mu.z)));
          }
          if (a.o_pos) {
            const float3 g = jtmul(J, make_float3(op[0], op[1], op[2]));
            st3(a.o_pos, i, make_float3(pf * iv * g.x, pf * iv * g.y, pf * iv * g.z));
          }
          if (a.o_theta) {
            // G = (1/2V) J^T H J with H the symmetric matrix of the second-order sums
            const float H[3][3] = {{oh[0], oh[3], oh[4]}, {oh[3], oh[1], oh[5]}, {oh[4], oh[5], oh[2]}};
            float HJ[3][3];
#pragma unroll
            for (int x = 0; x < 3; ++x)
#pragma unroll
              for (int b = 0; b < 3; ++b) HJ[x][b] = H[x][0] * J[0][b] + H[x][1] * J[1][b] + H[x][2] * J[2][b];
            auto G = [&](int u, int b) {
              return 0.5f * iv * (J[0][u] * HJ[0][b] + J[1][u] * HJ[1][b] + J[2][u] * HJ[2][b]);
            };
            const float sd = c1 * q - 2.0f * c2 * tr;
            float* o = a.o_theta + 6 * i;
            o[0] = pf * (G(0, 0) + sd - 4.0f * c2 * th[0]);
            o[1] = pf * (G(1, 1) + sd - 4.0f * c2 * th[1]);
            o[2] = pf * (G(2, 2) + sd - 4.0f * c2 * th[2]);
            o[3] = pf * (2.0f * G(0, 1) - 8.0f * c2 * th[3]);
            o[4] = pf * (2.0f * G(0, 2) - 8.0f * c2 * th[4]);
            o[5] = pf * (2.0f * G(1, 2) - 8.0f * c2 * th[5]);
          }
        }
      } else if (!HVP) {
        // per-lane partial outputs (linear in the phi sums), summed over the atom's
        // lanes: dE/dq, the pre-J dipole gradient G, the pre-J position gradient
        float oq = 0, og[3] = {0, 0, 0}, op[3] = {0, 0, 0};
        if (active) {
          const float4 h = s_h[slot];
          const int pk = __float_as_int(h.w);
          const int lx = (pk & 1023) - t0[0] + ix;
          const int yb = ((pk >> 10) & 1023) - t0[1], zb = ((pk >> 20) & 1023) - t0[2];
          // y weights are made per row (fewer live registers), z weights once
          float wz[3][P], wx[3];
          spline_weights<P, 2>(h.z, wz);
          weight_at_lds<P, 2>(s_coef, ix, h.x, wx);
          const float* plane = sm + (lx * E[1] + yb) * E[2] + zb;
          float Y00 = 0, Y01 = 0, Y02 = 0, Y10 = 0, Y11 = 0, Y20 = 0;
#pragma unroll
          for (int iy = 0; iy < P; ++iy) {
            const float* row = plane + iy * E[2];
            float z0 = 0, z1 = 0, z2 = 0;
#pragma unroll
            for (int iz = 0; iz < P; ++iz) {
              const float v = row[iz];
              z0 = fmaf(v, wz[0][iz], z0);
              z1 = fmaf(v, wz[1][iz], z1);
              z2 = fmaf(v, wz[2][iz], z2);
            }
            float wy[3];
            spline_weight_at<P, 2>(iy, h.y, wy);
            Y00 = fmaf(wy[0], z0, Y00);
            Y01 = fmaf(wy[0], z1, Y01);
            Y02 = fmaf(wy[0], z2, Y02);
            Y10 = fmaf(wy[1], z0, Y10);
            Y11 = fmaf(wy[1], z1, Y11);
            Y20 = fmaf(wy[2], z0, Y20);
          }
          const float S000 = wx[0] * Y00, S001 = wx[0] * Y01, S002 = wx[0] * Y02;
          const float S010 = wx[0] * Y10, S011 = wx[0] * Y11, S020 = wx[0] * Y20;
          const float S100 = wx[1] * Y00, S101 = wx[1] * Y01, S110 = wx[1] * Y10;
          const float S200 = wx[2] * Y00;
          const float4 qmv = s_qm[slot];
          const float q = qmv.x;
          const float3 d = jmul(J, make_float3(qmv.y, qmv.z, qmv.w));
          oq = S000;
          og[0] = S100; og[1] = S010; og[2] = S001;
          op[0] = q * S100 + S200 * d.x + S110 * d.y + S101 * d.z;
          op[1] = q * S010 + S110 * d.x + S020 * d.y + S011 * d.z;
          op[2] = q * S001 + S101 * d.x + S011 * d.y + S002 * d.z;
        }
        oq = group_sum<P>(oq, ix);
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          og[x] = group_sum<P>(og[x], ix);
          op[x] = group_sum<P>(op[x], ix);
        }
        if (active && ix == 0) {
          const int i = s_atom[slot];
          const float4 qmv = s_qm[slot];
          const float q = qmv.x;
          const float3 mu = make_float3(qmv.y, qmv.z, qmv.w);
          if (a.o_q) a.o_q[i] = pf * (oq * iv - cq * q);
          if (a.o_mu) {
            const float3 g = jtmul(J, make_float3(og[0], og[1], og[2]));
            st3(a.o_mu, i, make_float3(pf * (g.x * iv - cm * mu.x), pf * (g.y * iv - cm * mu.y),
                                       pf * (g.z * iv - cm * mu.z)));
          }
          if (a.o_pos) {
            const float3 g = jtmul(J, make_float3(op[0], op[1], op[2]));
            st3(a.o_pos, i, make_float3(pf * iv * g.x, pf * iv * g.y, pf * iv * g.z));
          }
          if constexpr (VIR) {
            // unwrapped fractional position (from the caller's position, by the
            // binning) and the dipole times C^-1
            const float4 sa = s_sa[slot];
            const float sf[3] = {sa.x, sa.y, sa.z};
            float mc[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) mc[b] = mu.x * ci[b] + mu.y * ci[3 + b] + mu.z * ci[6 + b];
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
              for (int x = 0; x < 3; ++x)
                vg[3 * b + x] += float(a.N[x]) * (sf[b] * op[x] + mc[b] * og[x]);
          }
        }
      } else {
        // DUAL: the forward outputs too (a compile-time switch: the two epilogues
        // merged under a run-time flag need far more registers)
        constexpr bool dual = DUAL;
        // per-lane partial outputs, linear in the phi sums S_abc (a+b+c <= 3) and
        // the psi sums Q_abc (a+b+c <= 2) of the lane's x-plane, summed over the
        // atom's lanes: the pre-J Hessian-vector products (q, mu, r) and, with the
        // forward outputs, dE/dq and the pre-J dipole and position gradients
        float oq = 0, om[3] = {0, 0, 0}, op[3] = {0, 0, 0};
        float fq = 0, fm[3] = {0, 0, 0}, fp[3] = {0, 0, 0};
        float S[4][4][4];
        float Q[3][3][3];
        if (active) {
          {
            const float4 h = s_h[slot];
            const int pk = __float_as_int(h.w);
            const int lx = (pk & 1023) - t0[0] + ix;
            const int yb = ((pk >> 10) & 1023) - t0[1], zb = ((pk >> 20) & 1023) - t0[2];
            // y weights are made per row (fewer live registers), z weights once
            float wz[4][P], wx[4];
            spline_weights<P, 3>(h.z, wz);
            weight_at_lds<P, 3>(s_coef, ix, h.x, wx);
            const float* pphi = sm + (lx * E[1] + yb) * E[2] + zb;
            const float* ppsi = pphi + EV;
            float Ys[4][4], Yq[3][3];
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
              for (int z = 0; z < 4; ++z) Ys[y][z] = 0.0f;
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
              for (int z = 0; z < 3; ++z) Yq[y][z] = 0.0f;
#pragma unroll
            for (int iy = 0; iy < P; ++iy) {
              float zs[4] = {0, 0, 0, 0}, zq[3] = {0, 0, 0};
#pragma unroll
              for (int iz = 0; iz < P; ++iz) {
                const float v = pphi[iy * E[2] + iz], u = ppsi[iy * E[2] + iz];
#pragma unroll
                for (int k = 0; k < 4; ++k) zs[k] = fmaf(v, wz[k][iz], zs[k]);
#pragma unroll
                for (int k = 0; k < 3; ++k) zq[k] = fmaf(u, wz[k][iz], zq[k]);
              }
              float wy[4];
              spline_weight_at<P, 3>(iy, h.y, wy);
#pragma unroll
              for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int k = 0; k + b < 4; ++k) Ys[b][k] = fmaf(wy[b], zs[k], Ys[b][k]);
#pragma unroll
              for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int k = 0; k + b < 3; ++k) Yq[b][k] = fmaf(wy[b], zq[k], Yq[b][k]);
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int b = 0; b + x < 4; ++b)
#pragma unroll
                for (int k = 0; k + b + x < 4; ++k) S[x][b][k] = wx[x] * Ys[b][k];
#pragma unroll
            for (int x = 0; x < 3; ++x)
#pragma unroll
              for (int b = 0; b + x < 3; ++b)
#pragma unroll
                for (int k = 0; k + b + x < 3; ++k) Q[x][b][k] = wx[x] * Yq[b][k];
          }
        }
        if (active) {
          const float4 qm = s_qm[slot], e1 = s_v1[slot], e2 = s_v2[slot];
          const float q = qm.x, vq = e1.x;
          const float3 vr = make_float3(e1.y, e1.z, e1.w);
          const float3 d3 = jmul(J, make_float3(qm.y, qm.z, qm.w));
          const float3 v3 = jmul(J, vr);
          const float3 w3 = jmul(J, make_float3(e2.x + q * vr.x, e2.y + q * vr.y, e2.z + q * vr.z));
          const float d[3] = {d3.x, d3.y, d3.z}, v[3] = {v3.x, v3.y, v3.z};
          const float w[3] = {w3.x, w3.y, w3.z};
          float S1[3], P1[3], S2[3][3], P2[3][3];
#pragma unroll
          for (int x = 0; x < 3; ++x) {
            const int ex[3] = {x == 0, x == 1, x == 2};
            S1[x] = S[ex[0]][ex[1]][ex[2]];
            P1[x] = Q[ex[0]][ex[1]][ex[2]];
#pragma unroll
            for (int y = 0; y < 3; ++y) {
              const int e0 = ex[0] + (y == 0), e1i = ex[1] + (y == 1), e2i = ex[2] + (y == 2);
              S2[x][y] = S[e0][e1i][e2i];
              P2[x][y] = Q[e0][e1i][e2i];
            }
          }
          float T3[3] = {0, 0, 0};   // S3(d, v, .)
#pragma unroll
          for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
              for (int z = 0; z < 3; ++z) {
                const int e0 = (x == 0) + (y == 0) + (z == 0);
                const int e1i = (x == 1) + (y == 1) + (z == 1);
                const int e2i = (x == 2) + (y == 2) + (z == 2);
                T3[z] = fmaf(d[x] * v[y], S[e0][e1i][e2i], T3[z]);
              }
          oq = Q[0][0][0] + S1[0] * v[0] + S1[1] * v[1] + S1[2] * v[2];
#pragma unroll
          for (int x = 0; x < 3; ++x) {
            om[x] = P1[x] + S2[x][0] * v[0] + S2[x][1] * v[1] + S2[x][2] * v[2];
            op[x] = q * P1[x] + P2[x][0] * d[0] + P2[x][1] * d[1] + P2[x][2] * d[2] +
                    vq * S1[x] + S2[x][0] * w[0] + S2[x][1] * w[1] + S2[x][2] * w[2] + T3[x];
          }
          if (dual) {
            fq = S[0][0][0];
#pragma unroll
            for (int x = 0; x < 3; ++x) {
              fm[x] = S1[x];
              fp[x] = q * S1[x] + S2[x][0] * d[0] + S2[x][1] * d[1] + S2[x][2] * d[2];
            }
          }
        }
        oq = group_sum<P>(oq, ix);
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          om[x] = group_sum<P>(om[x], ix);
          op[x] = group_sum<P>(op[x], ix);
        }
        if (dual) {
          fq = group_sum<P>(fq, ix);
#pragma unroll
          for (int x = 0; x < 3; ++x) {
            fm[x] = group_sum<P>(fm[x], ix);
            fp[x] = group_sum<P>(fp[x], ix);
          }
        }
        if (active && ix == 0) {
          const float4 qm = s_qm[slot], e1 = s_v1[slot], e2 = s_v2[slot];
          const int i = __float_as_int(e2.w);
          const float q = qm.x, vq = e1.x;
          const float3 mu = make_float3(qm.y, qm.z, qm.w);
          const float3 vm = make_float3(e2.x, e2.y, e2.z);
          if (a.o_q) a.o_q[i] = pf * (oq * iv - cq * vq);
          if (a.o_mu) {
            const float3 g = jtmul(J, make_float3(om[0], om[1], om[2]));
            st3(a.o_mu, i, make_float3(pf * (g.x * iv - cm * vm.x), pf * (g.y * iv - cm * vm.y),
                                       pf * (g.z * iv - cm * vm.z)));
          }
          if (a.o_pos) {
            const float3 g = jtmul(J, make_float3(op[0], op[1], op[2]));
            st3(a.o_pos, i, make_float3(pf * iv * g.x, pf * iv * g.y, pf * iv * g.z));
          }
          if (dual) {
            // gradient of E^lr from the same phi sums
            if (a.f_q) a.f_q[i] = pf * (fq * iv - cq * q);
            if (a.f_mu) {
              const float3 g = jtmul(J, make_float3(fm[0], fm[1], fm[2]));
              st3(a.f_mu, i, make_float3(pf * (g.x * iv - cm * mu.x), pf * (g.y * iv - cm * mu.y),
                                         pf * (g.z * iv - cm * mu.z)));
            }
            if (a.f_pos) {
              const float3 g = jtmul(J, make_float3(fp[0], fp[1], fp[2]));
              st3(a.f_pos, i, make_float3(pf * iv * g.x, pf * iv * g.y, pf * iv * g.z));
            }
          }
        }
      }
    }
  };

  // 2. rounds of 256 own-bin slots, then of 256 overflow records (those anchored in
  // the tile are owned); one round is compacted into the queue while the previous
  // one has been processed, so that no record registers live across the stencil work
  // the queue of a round in chunks of kGatherQueue: chunks after the first reload
  // their records (record index ri) from global memory
  auto drain = [&](int k, uint32_t ri) {
    const int nv = s_n;
    process(min(nv, kGatherQueue));
    for (int c0 = kGatherQueue; c0 < nv; c0 += kGatherQueue) {
      __syncthreads();   // the queue has been read
      if (k >= c0 && k < c0 + kGatherQueue) put(k - c0, load_rec<R4>(a.rec, ri));
      __syncthreads();
      process(min(kGatherQueue, nv - c0));
    }
  };
  int kq = enqueue(tid < nslot && ec % cap < cnt, cur);
  uint32_t rq = uint32_t(own_bin(ec / cap) * cap + (ec - (ec / cap) * cap));
  __syncthreads();
  const int nrs = (nslot + 255) >> 8;
  const int nr = nrs + ((novf + 255) >> 8);
  for (int r = 0;;) {
    drain(kq, rq);
    if (++r >= nr) break;
    __syncthreads();   // the queue has been read
    if (tid == 0) s_n = 0;
    bool valid = false;
    RecRegs<R4> rec;
    if (r < nrs) {
      const int e = r * 256 + tid;
      ec = min(e, nslot - 1);
      rec = slot_rec(ec);
      cnt = a.count[own_bin(ec / cap)];
      valid = e < nslot && ec % cap < cnt;
      rq = uint32_t(own_bin(ec / cap) * cap + (ec - (ec / cap) * cap));
    } else {
      const int o = (r - nrs) * 256 + tid;
      if (o < novf) {
        rq = uint32_t(a.ovf_base + o);
        rec = load_rec<R4>(a.rec, rq);
        const int pk = __float_as_int(rec.h.w);
        const int b0 = pk & 1023, b1 = (pk >> 10) & 1023, b2 = (pk >> 20) & 1023;
        valid = b0 >= t0[0] && b0 < t0[0] + T[0] && b1 >= t0[1] && b1 < t0[1] + T[1] &&
                b2 >= t0[2] && b2 < t0[2] + T[2];
      }
    }
    __syncthreads();   // s_n is cleared
    kq = enqueue(valid, rec);
    __syncthreads();
  }
  if constexpr (VIR) {
    __shared__ double vred[16 * 9];
    double v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = vg[k];
    block_sums<9>(v, vred);
    if (tid == 0)
#pragma unroll
      for (int k = 0; k < 9; ++k) a.vpart[9 * tile + k] = v[k];
  }
}

template <int P, bool VIR = false>
__device__ __forceinline__ void gather_body(const GArgs& a, const int tile) {
  gather_tile<P, false, false, VIR>(a, tile);
}

template <int P, bool DUAL = false>
__device__ __forceinline__ void gather_hvp_body(const GArgs& a, const int tile) {
  gather_tile<P, true, DUAL>(a, tile);
}

template <int P, bool VIR>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(P >= 7 && VIR ? 3 : (P >= 6 ? 4 : 5))))
k_gather(GArgs a) {
  gather_body<P, VIR>(a, xcd_item(blockIdx.x, gridDim.x));
}

// Cell gradient from E_recip and the partials (one workgroup):
//   dE/dC = -E_recip C^-T + (pf/V) C^-T T - (pf/V) (P + Q) C^-T
// with T the k-space sums of the x pass and P + Q the per-atom sums of the gather.
__global__ void __launch_bounds__(256) k_cell_grad(const double* box, const double* energy,
                                                   const double* xpart, int nx,
                                                   const double* gpart, int ng, double pf,
                                                   double* out) {
  __shared__ double red[16 * 9];
  double t[6] = {0, 0, 0, 0, 0, 0}, m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = threadIdx.x; k < nx; k += blockDim.x)
    for (int c = 0; c < 6; ++c) t[c] += xpart[6 * k + c];
  for (int k = threadIdx.x; k < ng; k += blockDim.x)
    for (int c = 0; c < 9; ++c) m[c] += gpart[9 * k + c];
  block_sums<6>(t, red);
  block_sums<9>(m, red);
  if (threadIdx.x == 0) {
    const Cell cl = cell_from_box(box);
    const double e = energy[0], s = cl.ok ? pf / cl.vol : 0.0;
    const double T[3][3] = {{t[0], t[3], t[4]}, {t[3], t[1], t[5]}, {t[4], t[5], t[2]}};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        // (C^-T)[a][b] = (C^-1)[b][a] = inv[3 b + a]
        double g = -e * cl.inv[3 * b + a];
        for (int c = 0; c < 3; ++c)
          g += s * (cl.inv[3 * c + a] * T[c][b] - m[3 * a + c] * cl.inv[3 * b + c]);
        out[3 * a + b] = g;
      }
  }
}

template <int P, bool DUAL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P >= 7 ? 3 : 4)))
k_gather_hvp(GArgs a) {
  gather_hvp_body<P, DUAL>(a, xcd_item(blockIdx.x, gridDim.x));
}

template <int P>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P >= 7 ? 3 : 4)))
k_gather_quad(GArgs a) {
  gather_tile<P, false, false, false, true>(a, xcd_item(blockIdx.x, gridDim.x));
}

// Batched gathers: work item (box, tile), per-box argument templates completed
// with the call's packed arrays; workgroups loop over the items.
template <int P, bool HVP>
__global__ void __launch_bounds__(256) k_gather_batch(const GArgs* args, const int2* items, int n,
                                                      BatchIO io) {
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = items[it];
    GArgs a = args[w.x];
    const size_t o = size_t(a.off);
    a.pos = io.pos + 3 * o;
    a.q = io.q ? io.q + o : nullptr;
    a.mu = io.mu ? io.mu + 3 * o : nullptr;
    a.box = io.box + 9 * w.x;
    a.v_pos = io.v_pos ? io.v_pos + 3 * o : nullptr;
    a.v_q = io.v_q ? io.v_q + o : nullptr;
    a.v_mu = io.v_mu ? io.v_mu + 3 * o : nullptr;
    a.o_pos = io.o_pos ? io.o_pos + 3 * o : nullptr;
    a.o_q = io.o_q ? io.o_q + o : nullptr;
    a.o_mu = io.o_mu ? io.o_mu + 3 * o : nullptr;
    a.energy = io.energy ? io.energy + 3 * w.x : nullptr;
    if (HVP) gather_hvp_body<P>(a, w.y);
    else gather_body<P>(a, w.y);
    __syncthreads();
  }
}

template <bool HVP>
hipError_t gather_dispatch(int p, dim3 g, size_t sh, hipStream_t s, const GArgs& a,
                           const LaunchEvents* ev, bool dual = false) {
#define PME_G(P)                                                                  \
  case P:                                                                         \
    if (HVP && dual) launch_k(ev, k_gather_hvp<P, true>, g, dim3(256), sh, s, a);     \
    else if (HVP) launch_k(ev, k_gather_hvp<P, false>, g, dim3(256), sh, s, a);       \
    else if (a.vpart) launch_k(ev, k_gather<P, true>, g, dim3(256), sh, s, a);        \
    else launch_k(ev, k_gather<P, false>, g, dim3(256), sh, s, a);                    \
    break;
  switch (p) {
    PME_G(1) PME_G(2) PME_G(3) PME_G(4) PME_G(5) PME_G(6) PME_G(7)
    default: return hipErrorInvalidValue;
  }
#undef PME_G
  return hipGetLastError();
}

GArgs base_args(const DevPlan& d, int set, int n, const float* pos, const float* q,
                const float* mu, const double* box) {
  GArgs a{};
  a.off = 0;
  a.n = n; a.pos = pos; a.q = q; a.mu = mu; a.box = box;
  for (int k = 0; k < 3; ++k) {
    a.N[k] = d.N[k]; a.B[k] = d.B[k]; a.nb[k] = d.nb[k]; a.T[k] = d.T[k]; a.nt[k] = d.nt[k];
  }
  a.phi = d.phi;
  a.alpha = d.alpha; a.prefactor = d.prefactor;
  a.pf = float(d.prefactor);
  a.cq = float(2.0 * d.alpha / sqrt(M_PI));
  a.cm = float(4.0 * d.alpha * d.alpha * d.alpha / (3.0 * sqrt(M_PI)));
  a.cap = d.cap; a.count = d.count[set]; a.ovf_count = d.ovf_count[set];
  a.rec = d.rec; a.ovf_base = d.ovf_base;
  return a;
}

// the field region(s) over a tile plus its stencil halo, then the row offsets and
// wrapped z coordinates of the region
size_t region_bytes(const DevPlan& d, int fields) {
  const size_t e0 = d.T[0] + d.p - 1, e1 = d.T[1] + d.p - 1, e2 = d.T[2] + d.p - 1;
  return sizeof(float) * size_t(fields) * e0 * e1 * e2 + sizeof(int) * (e0 * e1 + e2);
}

template <bool HVP>
hipError_t gather_batch_dispatch(int p, dim3 g, size_t sh, hipStream_t s, const GArgs* args,
                                 const int2* it, int n, const BatchIO& io) {
  switch (p) {
    case 1: hipLaunchKernelGGL((k_gather_batch<1, HVP>), g, dim3(256), sh, s, args, it, n, io); break;
    case 2: hipLaunchKernelGGL((k_gather_batch<2, HVP>), g, dim3(256), sh, s, args, it, n, io); break;
    case 3: hipLaunchKernelGGL((k_gather_batch<3, HVP>), g, dim3(256), sh, s, args, it, n, io); break;
    case 4: hipLaunchKernelGGL((k_gather_batch<4, HVP>), g, dim3(256), sh, s, args, it, n, io); break;
    case 5: hipLaunchKernelGGL((k_gather_batch<5, HVP>), g, dim3(256), sh, s, args, it, n, io); break;
    case 6: hipLaunchKernelGGL((k_gather_batch<6, HVP>), g, dim3(256), sh, s, args, it, n, io); break;
    case 7: hipLaunchKernelGGL((k_gather_batch<7, HVP>), g, dim3(256), sh, s, args, it, n, io); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t enable_gather_lds() {
  const void* fns[] = {
#define PME_G(P)                                                                             \
  reinterpret_cast<const void*>(k_gather<P, false>),                                         \
      reinterpret_cast<const void*>(k_gather<P, true>),                                     \
      reinterpret_cast<const void*>(k_gather_hvp<P, false>),                                \
      reinterpret_cast<const void*>(k_gather_hvp<P, true>),                                 \
      reinterpret_cast<const void*>(k_gather_quad<P>),                                      \
      reinterpret_cast<const void*>(k_gather_batch<P, false>),                               \
      reinterpret_cast<const void*>(k_gather_batch<P, true>),
      PME_G(1) PME_G(2) PME_G(3) PME_G(4) PME_G(5) PME_G(6) PME_G(7)
#undef PME_G
  };
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kGatherLds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t gather_batch_build(const DevPlan* plans, const int* n, const int* off, int nbox,
                              GatherBatch& t) {
  t = GatherBatch();
  t.p = nbox > 0 ? plans[0].p : 0;
  std::vector<GArgs> ga(nbox);
  std::vector<int2> items;
  for (int b = 0; b < nbox; ++b) {
    const DevPlan& d = plans[b];
    const int nt = d.nt[0] * d.nt[1] * d.nt[2];
    for (int k = 0; k < nt; ++k) items.push_back(make_int2(b, k));
    for (int h = 0; h < 2; ++h)
      if (region_bytes(d, h + 1) > t.lds[h]) t.lds[h] = region_bytes(d, h + 1);
  }
  hipError_t e = hipSuccess;
  for (int set = 0; set < 2 && e == hipSuccess; ++set) {
    for (int b = 0; b < nbox; ++b) {
      const DevPlan& d = plans[b];
      GArgs a = base_args(d, set, n[b], nullptr, nullptr, nullptr, nullptr);
      a.off = off[b];
      a.psi = d.rho;
      a.epart = d.epart; a.n_epart = fftx_blocks(d);
      a.spart = d.spart; a.n_spart = bin_blocks(n[b]);
      ga[b] = a;
    }
    e = upload(&t.g[set], ga.data(), sizeof(GArgs) * nbox);
  }
  if (e == hipSuccess)
    e = upload(reinterpret_cast<void**>(&t.items), items.data(), sizeof(int2) * items.size());
  t.n_items = int(items.size());
  return e;
}

void gather_batch_free(GatherBatch& t) {
  void* ptrs[] = {t.g[0], t.g[1], t.items};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  t = GatherBatch();
}

hipError_t launch_gather_batch(const GatherBatch& t, hipStream_t s, int set, bool hvp,
                               const BatchIO& io) {
  const GArgs* args = static_cast<const GArgs*>(t.g[set]);
  const dim3 g(t.n_items < 2048 ? (t.n_items > 0 ? t.n_items : 1) : 2048);
  return hvp ? gather_batch_dispatch<true>(t.p, g, t.lds[1], s, args, t.items, t.n_items, io)
             : gather_batch_dispatch<false>(t.p, g, t.lds[0], s, args, t.items, t.n_items, io);
}

hipError_t launch_gather(const DevPlan& d, hipStream_t s, int set, int n, const float* pos,
                         const float* q, const float* mu, const double* box, double* energy,
                         float* dE_dpos, float* dE_dq, float* dE_dmu, int n_spart,
                         const LaunchEvents* ev, double* vpart) {
  GArgs a = base_args(d, set, n, pos, q, mu, box);
  a.o_pos = dE_dpos; a.o_q = dE_dq; a.o_mu = dE_dmu;
  a.energy = energy; a.epart = d.epart; a.n_epart = fftx_blocks(d);
  a.spart = d.spart; a.n_spart = n_spart;
  a.vpart = vpart;
  return gather_dispatch<false>(d.p, dim3(d.nt[0] * d.nt[1] * d.nt[2]), region_bytes(d, 1), s, a,
                                ev);
}

hipError_t launch_gather_quad(const DevPlan& d, hipStream_t s, int set, int n, const float* pos,
                              const float* q, const float* mu, const float* theta,
                              const double* box, double* energy, float* dE_dpos, float* dE_dq,
                              float* dE_dmu, float* dE_dtheta, const LaunchEvents* ev) {
  GArgs a = base_args(d, set, n, pos, q, mu, box);
  a.theta = theta;
  a.o_pos = dE_dpos; a.o_q = dE_dq; a.o_mu = dE_dmu; a.o_theta = dE_dtheta;
  a.energy = energy; a.epart = d.epart; a.n_epart = fftx_blocks(d);
  a.spart = d.spart; a.n_spart = bin_blocks(n);
  a.spart_th = energy ? d.spart + 2 * bin_blocks(n) : nullptr;
  a.cth = float(pow(d.alpha, 5) / (5.0 * sqrt(M_PI)));
  const dim3 g(d.nt[0] * d.nt[1] * d.nt[2]);
  const size_t sh = region_bytes(d, 1);
  switch (d.p) {
    case 1: launch_k(ev, k_gather_quad<1>, g, dim3(256), sh, s, a); break;
    case 2: launch_k(ev, k_gather_quad<2>, g, dim3(256), sh, s, a); break;
    case 3: launch_k(ev, k_gather_quad<3>, g, dim3(256), sh, s, a); break;
    case 4: launch_k(ev, k_gather_quad<4>, g, dim3(256), sh, s, a); break;
    case 5: launch_k(ev, k_gather_quad<5>, g, dim3(256), sh, s, a); break;
    case 6: launch_k(ev, k_gather_quad<6>, g, dim3(256), sh, s, a); break;
    case 7: launch_k(ev, k_gather_quad<7>, g, dim3(256), sh, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cell_grad(const DevPlan& d, hipStream_t s, const double* box,
                            const double* energy, double* dE_dbox) {
  const int nx = fftx_blocks(d);
  hipLaunchKernelGGL(k_cell_grad, dim3(1), dim3(256), 0, s, box, energy, d.vpart, nx,
                     d.vpart + 6 * nx, d.nt[0] * d.nt[1] * d.nt[2], d.prefactor, dE_dbox);
  return hipGetLastError();
}

hipError_t launch_gather_hvp(const DevPlan& d, hipStream_t s, int set, int n, const float* pos,
                             const float* q, const float* mu, const double* box,
                             const float* v_pos, const float* v_q, const float* v_mu,
                             float* g_pos, float* g_q, float* g_mu, const LaunchEvents* ev,
                             const GatherForward* fwd) {
  GArgs a = base_args(d, set, n, pos, q, mu, box);
  a.psi = d.rho;
  a.v_pos = v_pos; a.v_q = v_q; a.v_mu = v_mu;
  a.o_pos = g_pos; a.o_q = g_q; a.o_mu = g_mu;
  if (fwd) {
    a.f_pos = fwd->dE_dpos; a.f_q = fwd->dE_dq; a.f_mu = fwd->dE_dmu;
    a.energy = fwd->energy; a.epart = d.epart; a.n_epart = fftx_blocks(d);
    a.spart = d.spart; a.n_spart = fwd->n_spart;
  }
  const bool dual = a.f_pos || a.f_q || a.f_mu;
  return gather_dispatch<true>(d.p, dim3(d.nt[0] * d.nt[1] * d.nt[2]), region_bytes(d, 2), s, a,
                               ev, dual);
}

}  // namespace pme
