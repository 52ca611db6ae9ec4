// Gradient gather (Eqs. energy_recip, self_q, self_mu, E_lr_total, forces) and
// the Hessian-vector product gather.
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
  double* energy;
  const double* epart;
  int n_epart;
  const double* spart;
  int n_spart;
  double alpha;
  double prefactor;
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
}

__device__ __forceinline__ float3 jmul(const float (&J)[3][3], float3 v) {
  return make_float3(J[0][0] * v.x + J[0][1] * v.y + J[0][2] * v.z,
                     J[1][0] * v.x + J[1][1] * v.y + J[1][2] * v.z,
                     J[2][0] * v.x + J[2][1] * v.y + J[2][2] * v.z);
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

template <int P>
__global__ void __launch_bounds__(256) k_gather(GArgs a) {
  constexpr int lo = (P - 1) / 2;
  const Cell c = cell_from_box(a.box);
  if (blockIdx.x == 0 && a.energy) finalize_energy(a, c);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  int base[3];
  float f[3];
  const bool ok = atom_stencil<P>(a.pos, i, c, a.N, base, f);
  if (!ok) {
    const float nan = __int_as_float(0x7fc00000);
    st3(a.o_pos, i, make_float3(nan, nan, nan));
    st3(a.o_mu, i, make_float3(nan, nan, nan));
    if (a.o_q) a.o_q[i] = nan;
    return;
  }
  float wy[3][P], wz[3][P];
  spline_weights<P, 2>(f[1], wy);
  spline_weights<P, 2>(f[2], wz);
  const int Ny = a.N[1], Nz = a.N[2];
  int zi[P];
#pragma unroll
  for (int k = 0; k < P; ++k) zi[k] = wrapn(base[2] - lo + k, Nz);
  // S: 000, 100, 010, 001, 200, 020, 002, 110, 101, 011
  float S000 = 0, S100 = 0, S010 = 0, S001 = 0, S200 = 0, S020 = 0, S002 = 0, S110 = 0, S101 = 0,
        S011 = 0;
#pragma unroll 1
  for (int ix = 0; ix < P; ++ix) {
    float wx[3];
    spline_weight_at<P, 2>(ix, f[0], wx);
    const int mx = wrapn(base[0] - lo + ix, a.N[0]);
    float Y00 = 0, Y01 = 0, Y02 = 0, Y10 = 0, Y11 = 0, Y20 = 0;
#pragma unroll
    for (int iy = 0; iy < P; ++iy) {
      const int my = wrapn(base[1] - lo + iy, Ny);
      const float* row = a.phi + (size_t(mx) * Ny + my) * Nz;
      float z0 = 0, z1 = 0, z2 = 0;
#pragma unroll
      for (int iz = 0; iz < P; ++iz) {
        const float v = row[zi[iz]];
        z0 = fmaf(v, wz[0][iz], z0);
        z1 = fmaf(v, wz[1][iz], z1);
        z2 = fmaf(v, wz[2][iz], z2);
      }
      Y00 = fmaf(wy[0][iy], z0, Y00);
      Y01 = fmaf(wy[0][iy], z1, Y01);
      Y02 = fmaf(wy[0][iy], z2, Y02);
      Y10 = fmaf(wy[1][iy], z0, Y10);
      Y11 = fmaf(wy[1][iy], z1, Y11);
      Y20 = fmaf(wy[2][iy], z0, Y20);
    }
    S000 = fmaf(wx[0], Y00, S000);
    S001 = fmaf(wx[0], Y01, S001);
    S002 = fmaf(wx[0], Y02, S002);
    S010 = fmaf(wx[0], Y10, S010);
    S011 = fmaf(wx[0], Y11, S011);
    S020 = fmaf(wx[0], Y20, S020);
    S100 = fmaf(wx[1], Y00, S100);
    S101 = fmaf(wx[1], Y01, S101);
    S110 = fmaf(wx[1], Y10, S110);
    S200 = fmaf(wx[2], Y00, S200);
  }
  float J[3][3];
  jacobian(c, a.N, J);
  const float iv = float(1.0 / c.vol);
  const float pf = float(a.prefactor);
  const float q = a.q ? a.q[i] : 0.0f;
  const float3 mu = ld3(a.mu, i);
  const float3 d = jmul(J, mu);
  const float3 G = make_float3(S100, S010, S001);
  const float3 Hd = make_float3(S200 * d.x + S110 * d.y + S101 * d.z,
                                S110 * d.x + S020 * d.y + S011 * d.z,
                                S101 * d.x + S011 * d.y + S002 * d.z);
  const float cq = float(2.0 * a.alpha / sqrt(M_PI));
  const float cm = float(4.0 * a.alpha * a.alpha * a.alpha / (3.0 * sqrt(M_PI)));
  if (a.o_q) a.o_q[i] = pf * (S000 * iv - cq * q);
  if (a.o_mu) {
    const float3 g = jtmul(J, G);
    st3(a.o_mu, i, make_float3(pf * (g.x * iv - cm * mu.x), pf * (g.y * iv - cm * mu.y),
                               pf * (g.z * iv - cm * mu.z)));
  }
  if (a.o_pos) {
    const float3 g = jtmul(J, make_float3(q * G.x + Hd.x, q * G.y + Hd.y, q * G.z + Hd.z));
    st3(a.o_pos, i, make_float3(pf * iv * g.x, pf * iv * g.y, pf * iv * g.z));
  }
}

template <int P>
__global__ void __launch_bounds__(256) k_gather_hvp(GArgs a) {
  constexpr int lo = (P - 1) / 2;
  const Cell c = cell_from_box(a.box);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  int base[3];
  float f[3];
  const bool ok = atom_stencil<P>(a.pos, i, c, a.N, base, f);
  if (!ok) {
    const float nan = __int_as_float(0x7fc00000);
    st3(a.o_pos, i, make_float3(nan, nan, nan));
    st3(a.o_mu, i, make_float3(nan, nan, nan));
    if (a.o_q) a.o_q[i] = nan;
    return;
  }
  float wy[4][P], wz[4][P];
  spline_weights<P, 3>(f[1], wy);
  spline_weights<P, 3>(f[2], wz);
  const int Ny = a.N[1], Nz = a.N[2];
  int zi[P];
#pragma unroll
  for (int k = 0; k < P; ++k) zi[k] = wrapn(base[2] - lo + k, Nz);
  // phi sums S_abc, 1 <= a+b+c <= 3; psi sums P_abc, a+b+c <= 2
  float S[4][4][4];
  float Q[3][3][3];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int z = 0; z < 4; ++z) S[x][y][z] = 0.0f;
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
      for (int z = 0; z < 3; ++z) Q[x][y][z] = 0.0f;
#pragma unroll 1
  for (int ix = 0; ix < P; ++ix) {
    float wx[4];
    spline_weight_at<P, 3>(ix, f[0], wx);
    const int mx = wrapn(base[0] - lo + ix, a.N[0]);
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
      const int my = wrapn(base[1] - lo + iy, Ny);
      const size_t roff = (size_t(mx) * Ny + my) * Nz;
      const float* rphi = a.phi + roff;
      const float* rpsi = a.psi + roff;
      float zs[4] = {0, 0, 0, 0}, zq[3] = {0, 0, 0};
#pragma unroll
      for (int iz = 0; iz < P; ++iz) {
        const float v = rphi[zi[iz]], u = rpsi[zi[iz]];
#pragma unroll
        for (int k = 0; k < 4; ++k) zs[k] = fmaf(v, wz[k][iz], zs[k]);
#pragma unroll
        for (int k = 0; k < 3; ++k) zq[k] = fmaf(u, wz[k][iz], zq[k]);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int k = 0; k + b < 4; ++k) Ys[b][k] = fmaf(wy[b][iy], zs[k], Ys[b][k]);
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int k = 0; k + b < 3; ++k) Yq[b][k] = fmaf(wy[b][iy], zq[k], Yq[b][k]);
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int b = 0; b + x < 4; ++b)
#pragma unroll
        for (int k = 0; k + b + x < 4; ++k) S[x][b][k] = fmaf(wx[x], Ys[b][k], S[x][b][k]);
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int b = 0; b + x < 3; ++b)
#pragma unroll
        for (int k = 0; k + b + x < 3; ++k) Q[x][b][k] = fmaf(wx[x], Yq[b][k], Q[x][b][k]);
  }
  float J[3][3];
  jacobian(c, a.N, J);
  const float iv = float(1.0 / c.vol);
  const float pf = float(a.prefactor);
  const float q = a.q ? a.q[i] : 0.0f;
  const float3 mu = ld3(a.mu, i);
  const float vq = a.v_q ? a.v_q[i] : 0.0f;
  const float3 vr = ld3(a.v_pos, i);
  const float3 vm = ld3(a.v_mu, i);
  const float3 d3 = jmul(J, mu);
  const float3 v3 = jmul(J, vr);
  const float3 w3 = jmul(J, make_float3(vm.x + q * vr.x, vm.y + q * vr.y, vm.z + q * vr.z));
  const float d[3] = {d3.x, d3.y, d3.z}, v[3] = {v3.x, v3.y, v3.z}, w[3] = {w3.x, w3.y, w3.z};
  // index helpers: unit multi-indices
  float S1[3], P1[3], S2[3][3], P2[3][3];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    const int ex[3] = {x == 0, x == 1, x == 2};
    S1[x] = S[ex[0]][ex[1]][ex[2]];
    P1[x] = Q[ex[0]][ex[1]][ex[2]];
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      const int e0 = ex[0] + (y == 0), e1 = ex[1] + (y == 1), e2 = ex[2] + (y == 2);
      S2[x][y] = S[e0][e1][e2];
      P2[x][y] = Q[e0][e1][e2];
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
        const int e1 = (x == 1) + (y == 1) + (z == 1);
        const int e2 = (x == 2) + (y == 2) + (z == 2);
        T3[z] = fmaf(d[x] * v[y], S[e0][e1][e2], T3[z]);
      }
  const float P0 = Q[0][0][0];
  const float cq = float(2.0 * a.alpha / sqrt(M_PI));
  const float cm = float(4.0 * a.alpha * a.alpha * a.alpha / (3.0 * sqrt(M_PI)));
  if (a.o_q) {
    const float s = P0 + S1[0] * v[0] + S1[1] * v[1] + S1[2] * v[2];
    a.o_q[i] = pf * (s * iv - cq * vq);
  }
  if (a.o_mu) {
    float u[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) u[x] = P1[x] + S2[x][0] * v[0] + S2[x][1] * v[1] + S2[x][2] * v[2];
    const float3 g = jtmul(J, make_float3(u[0], u[1], u[2]));
    st3(a.o_mu, i, make_float3(pf * (g.x * iv - cm * vm.x), pf * (g.y * iv - cm * vm.y),
                               pf * (g.z * iv - cm * vm.z)));
  }
  if (a.o_pos) {
    float u[3];
#pragma unroll
    for (int x = 0; x < 3; ++x)
      u[x] = q * P1[x] + P2[x][0] * d[0] + P2[x][1] * d[1] + P2[x][2] * d[2] + vq * S1[x] +
             S2[x][0] * w[0] + S2[x][1] * w[1] + S2[x][2] * w[2] + T3[x];
    const float3 g = jtmul(J, make_float3(u[0], u[1], u[2]));
    st3(a.o_pos, i, make_float3(pf * iv * g.x, pf * iv * g.y, pf * iv * g.z));
  }
}

template <bool HVP>
hipError_t gather_dispatch(int p, dim3 g, hipStream_t s, const GArgs& a) {
#define PME_G(P)                                                                  \
  case P:                                                                         \
    if (HVP) hipLaunchKernelGGL(k_gather_hvp<P>, g, dim3(256), 0, s, a);          \
    else hipLaunchKernelGGL(k_gather<P>, g, dim3(256), 0, s, a);                   \
    break;
  switch (p) {
    PME_G(1) PME_G(2) PME_G(3) PME_G(4) PME_G(5) PME_G(6) PME_G(7)
    default: return hipErrorInvalidValue;
  }
#undef PME_G
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gather(const DevPlan& d, hipStream_t s, int n, const float* pos,
                         const float* q, const float* mu, const double* box, double* energy,
                         float* dE_dpos, float* dE_dq, float* dE_dmu, int n_spart) {
  GArgs a{};
  a.n = n; a.pos = pos; a.q = q; a.mu = mu; a.box = box;
  for (int k = 0; k < 3; ++k) a.N[k] = d.N[k];
  a.phi = d.phi;
  a.o_pos = dE_dpos; a.o_q = dE_dq; a.o_mu = dE_dmu;
  a.energy = energy; a.epart = d.epart; a.n_epart = fftx_blocks(d);
  a.spart = d.spart; a.n_spart = n_spart;
  a.alpha = d.alpha; a.prefactor = d.prefactor;
  return gather_dispatch<false>(d.p, dim3(bin_blocks(n)), s, a);
}

hipError_t launch_gather_hvp(const DevPlan& d, hipStream_t s, int n, const float* pos,
                             const float* q, const float* mu, const double* box,
                             const float* v_pos, const float* v_q, const float* v_mu,
                             float* g_pos, float* g_q, float* g_mu) {
  if (n == 0) return hipSuccess;
  GArgs a{};
  a.n = n; a.pos = pos; a.q = q; a.mu = mu; a.box = box;
  for (int k = 0; k < 3; ++k) a.N[k] = d.N[k];
  a.phi = d.phi; a.psi = d.rho;
  a.v_pos = v_pos; a.v_q = v_q; a.v_mu = v_mu;
  a.o_pos = g_pos; a.o_q = g_q; a.o_mu = g_mu;
  a.alpha = d.alpha; a.prefactor = d.prefactor;
  return gather_dispatch<true>(d.p, dim3(bin_blocks(n)), s, a);
}

}  // namespace pme
