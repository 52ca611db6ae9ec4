// Thole-damped polarizable point-charge model: cell list, real-space pair
// kernels and the preconditioned-conjugate-gradient induced-dipole solve whose
// matrix-vector product is the PME Hessian (pme_backward) plus the real-space
// dipole tensor.  The model and its conventions are documented in pol.h.
//
// Pair kernels give 16 lanes to an atom; the lanes split the atoms of the
// neighbouring cells and combine their partial sums with wavefront shuffles.
// The screened functions follow the recursion of the explicit Ewald sum,
//     B0 = erfc(a r)/r,  B_l = [(2l-1) B_{l-1} + (2a^2)^l exp(-a^2 r^2)/(a sqrt(pi))] / r^2,
// and the damped B_l^t keep grad B_l^t = -R B_{l+1}^t, so every gradient has the
// undamped form with B -> B^t.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "../../include/pol.h"
#include "cells.h"
#include "kernels.h"

namespace {

constexpr int kLanes = 16;          // lanes per atom in the pair kernels
constexpr int kPairThreads = 256;

enum PairMode { kEnergyGrad = 0, kMuGrad = 1, kMixed = 2, kHvp = 3 };

struct PairArgs {
  int n;
  const float* pos;
  const float* q;
  const float* mu;
  const float* pol;
  const float* vpos;
  const float* vq;   // charge and dipole tangents (kHvp)
  const float* vmu;
  CellGrid g;
  const int* start;
  const int* sorted;
  float alpha;
  float rc2;
  float A;
  float pf;
  float* o_pos;      // dE/dr
  float* o_q;        // dE/dq (or the q row of the Hessian product)
  float* o_mu;       // dE/dmu (or the mixed block, or the mu row)
  double* epart;     // [blocks] energy partials
};

__device__ __forceinline__ float3 ld3(const float* p, int i) {
  return p ? make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]) : make_float3(0.f, 0.f, 0.f);
}
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

__device__ __forceinline__ float lane_sum(float v) {
#pragma unroll
  for (int o = kLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kLanes);
  return v;
}

template <int MODE>
__global__ void __launch_bounds__(kPairThreads) k_pair(PairArgs a) {
  __shared__ double red[kPairThreads / kLanes];
  const int lane = threadIdx.x % kLanes;
  const int slot = threadIdx.x / kLanes;
  const int i = blockIdx.x * (kPairThreads / kLanes) + slot;
  const bool live = i < a.n;
  const int ii = live ? i : 0;
  const float3 pi = ld3(a.pos, ii);
  const float qi = a.q ? a.q[ii] : 0.0f;
  const float3 mi = ld3(a.mu, ii);
  const float ai = a.pol[ii];
  const float3 vi =
      (MODE == kMixed || MODE == kHvp) ? ld3(a.vpos, ii) : make_float3(0.f, 0.f, 0.f);
  int c[3], no[3];
  cell_of(a.g, pi.x, pi.y, pi.z, c);
#pragma unroll
  for (int d = 0; d < 3; ++d) no[d] = a.g.nc[d] < 3 ? a.g.nc[d] : 3;
  const float sqpi = 1.7724538509055159f;
  const float t2 = 2.0f * a.alpha * a.alpha;
  float e = 0.f, gx = 0.f, gy = 0.f, gz = 0.f, mx = 0.f, my = 0.f, mz = 0.f, gq = 0.f;
  if (live) {
    for (int ox = 0; ox < no[0]; ++ox)
      for (int oy = 0; oy < no[1]; ++oy)
        for (int oz = 0; oz < no[2]; ++oz) {
          const int cx = neighbour_cell(c[0], ox, a.g.nc[0]);
          const int cy = neighbour_cell(c[1], oy, a.g.nc[1]);
          const int cz = neighbour_cell(c[2], oz, a.g.nc[2]);
          const int cell = (cx * a.g.nc[1] + cy) * a.g.nc[2] + cz;
          const int b0 = a.start[cell], b1 = a.start[cell + 1];
          for (int k = b0 + lane; k < b1; k += kLanes) {
            const int j = a.sorted[k];
            if (j == i) continue;
            const float3 pj = ld3(a.pos, j);
            const float3 R = min_image(a.g, pi.x - pj.x, pi.y - pj.y, pi.z - pj.z);
            const float r2 = dot3(R, R);
            if (r2 >= a.rc2 || r2 <= 0.0f) continue;
            const float r = sqrtf(r2), ir = 1.0f / r, ir2 = ir * ir;
            const float ar = a.alpha * r;
            const float gexp = expf(-ar * ar) / (a.alpha * sqpi);
            const float B0 = erfcf(ar) * ir;
            const float B1 = (B0 + t2 * gexp) * ir2;
            const float B2 = (3.0f * B1 + t2 * t2 * gexp) * ir2;
            const float B3 = (5.0f * B2 + t2 * t2 * t2 * gexp) * ir2;
            float B1t = B1, B2t = B2, B3t = B3;
            const float aj = a.pol[j];
            const float pp = ai * aj;
            if (a.A > 0.0f && pp > 0.0f) {
              const float au3 = a.A * r2 * r * rsqrtf(pp);
              const float ex = expf(-au3);
              const float ir3 = ir2 * ir;
              B1t = B1 - ex * ir3;
              B2t = B2 - 3.0f * (1.0f + au3) * ex * ir3 * ir2;
              B3t = B3 - 15.0f * (1.0f + au3 + 0.6f * au3 * au3) * ex * ir3 * ir2 * ir2;
            }
            const float qj = a.q ? a.q[j] : 0.0f;
            const float3 mj = ld3(a.mu, j);
            const float mjr = dot3(mj, R);
            if (MODE == kHvp) {
              // r column: d/dR of dE/dq_i and dE/dmu_i along w = v_i - v_j
              // (grad B0 = -R B1 undamped); (q, mu) columns: the bilinear
              // gradients with charges vq and dipoles vmu
              const float3 vj = ld3(a.vpos, j);
              const float3 w = make_float3(vi.x - vj.x, vi.y - vj.y, vi.z - vj.z);
              const float rw = dot3(R, w), mjw = dot3(mj, w);
              const float vqj = a.vq ? a.vq[j] : 0.0f;
              const float3 vmj = ld3(a.vmu, j);
              const float vmjr = dot3(vmj, R);
              gq += -qj * B1 * rw + B1t * mjw - mjr * B2t * rw + vqj * B0 + vmjr * B1t;
              const float cw = -qj * B1t - mjr * B2t;
              const float cR = qj * rw * B2t - mjw * B2t + rw * mjr * B3t - vqj * B1t -
                               vmjr * B2t;
              const float cm = -rw * B2t;
              mx += cw * w.x + cR * R.x + cm * mj.x + B1t * vmj.x;
              my += cw * w.y + cR * R.y + cm * mj.y + B1t * vmj.y;
              mz += cw * w.z + cR * R.z + cm * mj.z + B1t * vmj.z;
              continue;
            }
            if (MODE == kMixed) {
              const float3 vj = ld3(a.vpos, j);
              const float3 w = make_float3(vi.x - vj.x, vi.y - vj.y, vi.z - vj.z);
              const float rw = dot3(R, w), mjw = dot3(mj, w);
              const float cw = -qj * B1t - mjr * B2t;
              const float cR = qj * rw * B2t - mjw * B2t + rw * mjr * B3t;
              const float cm = -rw * B2t;
              mx += cw * w.x + cR * R.x + cm * mj.x;
              my += cw * w.y + cR * R.y + cm * mj.y;
              mz += cw * w.z + cR * R.z + cm * mj.z;
              continue;
            }
            // dE/dmu_i
            const float cRm = -qj * B1t - mjr * B2t;
            mx += cRm * R.x + B1t * mj.x;
            my += cRm * R.y + B1t * mj.y;
            mz += cRm * R.z + B1t * mj.z;
            if (MODE == kEnergyGrad) {
              gq += qj * B0 + mjr * B1t;
              const float mir = dot3(mi, R), mm = dot3(mi, mj);
              const float cross = qi * mjr - qj * mir;
              e += 0.5f * (qi * qj * B0 + cross * B1t + mm * B1t - mir * mjr * B2t);
              const float cR = -qi * qj * B1 - cross * B2t - mm * B2t + mir * mjr * B3t;
              gx += cR * R.x + B1t * (qi * mj.x - qj * mi.x) - B2t * (mi.x * mjr + mj.x * mir);
              gy += cR * R.y + B1t * (qi * mj.y - qj * mi.y) - B2t * (mi.y * mjr + mj.y * mir);
              gz += cR * R.z + B1t * (qi * mj.z - qj * mi.z) - B2t * (mi.z * mjr + mj.z * mir);
            }
          }
        }
  }
  mx = lane_sum(mx); my = lane_sum(my); mz = lane_sum(mz);
  if (MODE == kEnergyGrad || MODE == kHvp) gq = lane_sum(gq);
  if (MODE == kEnergyGrad) {
    e = lane_sum(e);
    gx = lane_sum(gx); gy = lane_sum(gy); gz = lane_sum(gz);
  }
  if (live && lane == 0) {
    if (a.o_mu) {
      a.o_mu[3 * i] = a.pf * mx;
      a.o_mu[3 * i + 1] = a.pf * my;
      a.o_mu[3 * i + 2] = a.pf * mz;
    }
    if ((MODE == kEnergyGrad || MODE == kHvp) && a.o_q) a.o_q[i] = a.pf * gq;
    if (MODE == kEnergyGrad && a.o_pos) {
      a.o_pos[3 * i] = a.pf * gx;
      a.o_pos[3 * i + 1] = a.pf * gy;
      a.o_pos[3 * i + 2] = a.pf * gz;
    }
  }
  if (MODE == kEnergyGrad && a.epart) {
    if (lane == 0) red[slot] = live ? double(e) : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int k = 0; k < kPairThreads / kLanes; ++k) sum += red[k];
      a.epart[blockIdx.x] = sum;
    }
  }
}

// energy = pf * sum of block partials (one workgroup)
__global__ void __launch_bounds__(256) k_energy_sum(const double* part, int nb, double pf,
                                                    double* energy) {
  __shared__ double red[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) s += part[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) energy[0] = pf * red[0];
}

// ---- PCG vector kernels (length m = 3n) ----

// Two dot products a.b and c.d in FP64 (one workgroup), into out[0], out[1].
__global__ void __launch_bounds__(1024) k_dot2(int m, const float* a, const float* b,
                                               const float* c, const float* d, double* out) {
  __shared__ double r0[1024], r1[1024];
  double s0 = 0.0, s1 = 0.0;
  for (int k = threadIdx.x; k < m; k += 1024) {
    s0 += double(a[k]) * b[k];
    s1 += double(c[k]) * d[k];
  }
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[0] = r0[0]; out[1] = r1[0]; }
}

// Av = (pf / a) v + g1 + g2
__global__ void k_matvec_sum(int m, float pf, const float* pol, const float* v, const float* g1,
                             const float* g2, float* Av) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) Av[k] = pf * v[k] / pol[k / 3] + g1[k] + g2[k];
}

// r = -(g1 + g2) - (warm ? Ax : 0); x = warm ? x : 0; z = (a / pf) r; p = z
__global__ void k_pcg_start(int m, float pf, const float* pol, const float* g1, const float* g2,
                            const float* Ax, float* x, float* r, float* z, float* p, int warm) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  float rk = -(g1[k] + g2[k]);
  if (warm) rk -= Ax[k];
  else x[k] = 0.0f;
  const float zk = pol[k / 3] / pf * rk;
  r[k] = rk;
  z[k] = zk;
  p[k] = zk;
}

// scal: [0] r.z  [1] z.z  [2] p.Ap  [3] (unused)  [4] new r.z  [5] new z.z
// alpha = r.z / p.Ap; x += alpha p; r -= alpha Ap; z = (a / pf) r
__global__ void k_pcg_step(int m, float pf, const float* pol, const double* scal, const float* p,
                           const float* Ap, float* x, float* r, float* z) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const double pap = scal[2];
  const float al = pap != 0.0 ? float(scal[0] / pap) : 0.0f;
  x[k] += al * p[k];
  const float rk = r[k] - al * Ap[k];
  r[k] = rk;
  z[k] = pol[k / 3] / pf * rk;
}

// beta = new r.z / r.z; p = z + beta p
__global__ void k_pcg_dir(int m, const double* scal, const float* z, float* p) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const float be = scal[0] != 0.0 ? float(scal[4] / scal[0]) : 0.0f;
  p[k] = z[k] + be * p[k];
}

// dU_dpos = g_pos + h_pos; dU_dmu = g_mu + h_mu + (pf / a) mu (each output optional)
__global__ void k_model_grads(int n, float pf, const float* pol, const float* mu,
                              const float* gp, const float* hp, const float* gm, const float* hm,
                              float* dpos, float* dmu) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 3 * n) return;
  if (dpos) dpos[k] = gp[k] + hp[k];
  if (dmu) dmu[k] = gm[k] + hm[k] + (mu ? pf * mu[k] / pol[k / 3] : 0.0f);
}

// dU_dq = g_q + h_q
__global__ void k_add(int m, const float* a, const float* b, float* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) out[k] = a[k] + b[k];
}

// energy = e_lr[0] + e_lr[1] + e_lr[2] + e_real + pf sum |mu|^2 / (2 a) (one workgroup)
__global__ void __launch_bounds__(256) k_model_energy(int n, double pf, const float* pol,
                                                      const float* mu, const double* e_lr,
                                                      const double* e_real, double* energy) {
  __shared__ double red[256];
  double s = 0.0;
  if (mu)
    for (int i = threadIdx.x; i < n; i += 256) {
      const double m2 = double(mu[3 * i]) * mu[3 * i] + double(mu[3 * i + 1]) * mu[3 * i + 1] +
                        double(mu[3 * i + 2]) * mu[3 * i + 2];
      s += m2 / (2.0 * double(pol[i]));
    }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) energy[0] = e_lr[0] + e_lr[1] + e_lr[2] + e_real[0] + pf * red[0];
}

__global__ void k_copy_scal(double* scal) {
  if (threadIdx.x == 0) { scal[0] = scal[4]; scal[1] = scal[5]; }
}

}  // namespace

struct pol_plan_s {
  pol_desc_t desc;
  CellList cells;
  double* epart = nullptr;
  double* scal = nullptr;
  float* vec = nullptr;      // 8 work vectors of 3 max_atoms floats
};

namespace {

thread_local char g_pol_err[256] = "";

int pol_hip_fail(hipError_t e) {
  snprintf(g_pol_err, sizeof(g_pol_err), "%s", hipGetErrorString(e));
  return PME_EHIP;
}

void pol_free(pol_plan_s* p) {
  free_cells(p->cells);
  void* ptrs[] = {p->epart, p->scal, p->vec};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
}

inline int blocks_for(int m, int t) { return cell_blocks(m, t); }

PairArgs pair_args(const pol_plan_s* pl, int n, const float* pos, const float* q, const float* mu,
                   const float* pol) {
  PairArgs a;
  a.n = n; a.pos = pos; a.q = q; a.mu = mu; a.pol = pol;
  a.vpos = nullptr; a.vq = nullptr; a.vmu = nullptr;
  a.g = pl->cells.g;
  a.start = pl->cells.start; a.sorted = pl->cells.sorted;
  a.alpha = float(pl->desc.alpha);
  a.rc2 = float(pl->desc.cutoff * pl->desc.cutoff);
  a.A = float(pl->desc.thole_a);
  a.pf = float(pl->desc.prefactor);
  a.o_pos = nullptr; a.o_q = nullptr; a.o_mu = nullptr; a.epart = nullptr;
  return a;
}

int pair_blocks(int n) { return blocks_for(n, kPairThreads / kLanes); }

// dE_real/dmu only (dipole field of mu and q)
hipError_t real_mu_grad(pol_plan_s* pl, hipStream_t s, int n, const float* pos, const float* q,
                        const float* mu, const float* pol, float* out) {
  hipError_t e = build_cells(pl->cells, s, n, pos);
  if (e != hipSuccess) return e;
  PairArgs a = pair_args(pl, n, pos, q, mu, pol);
  a.o_mu = out;
  hipLaunchKernelGGL(k_pair<kMuGrad>, dim3(pair_blocks(n)), dim3(kPairThreads), 0, s, a);
  return hipGetLastError();
}

bool check_common(const pol_plan_s* pl, int n, const float* pos, const float* pol) {
  return pl && n >= 0 && n <= pl->desc.max_atoms && (n == 0 || (pos && pol));
}

}  // namespace

extern "C" {

int pol_plan_create(const pol_desc_t* desc, pol_plan_t* out) {
  if (!desc || !out) return PME_EINVAL;
  *out = nullptr;
  if (desc->max_atoms < 1 || (desc->flags & ~(POL_F_WARM_START | POL_F_FIXED_ITERS)))
    return PME_EINVAL;
  if (!(desc->alpha > 0.0) || !isfinite(desc->alpha) || !(desc->thole_a >= 0.0) ||
      !isfinite(desc->thole_a) || !isfinite(desc->prefactor) || desc->prefactor == 0.0)
    return PME_EALPHA;
  pol_plan_s* pl = new (std::nothrow) pol_plan_s();
  if (!pl) return PME_ENOMEM;
  pl->desc = *desc;
  int rc0 = setup_cells(pl->cells, desc->box, desc->cutoff, desc->max_atoms);
  if (rc0 != PME_OK) {
    pol_free(pl);
    return rc0;
  }
  const size_t m = size_t(desc->max_atoms);
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t r) { if (r != hipSuccess && e == hipSuccess) e = r; };
  ok(hipMalloc(&pl->epart, sizeof(double) * pair_blocks(int(m))));
  ok(hipMalloc(&pl->scal, sizeof(double) * 8));
  ok(hipMalloc(&pl->vec, sizeof(float) * 8 * 3 * m));
  if (e != hipSuccess) {
    pol_free(pl);
    return e == hipErrorOutOfMemory ? PME_ENOMEM : pol_hip_fail(e);
  }
  *out = pl;
  return PME_OK;
}

void pol_plan_destroy(pol_plan_t plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  pol_free(plan);
}

int pol_real(pol_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
             const float* mu, const float* pol, double* energy, float* dE_dpos, float* dE_dq,
             float* dE_dmu) {
  if (!check_common(plan, n, pos, pol)) return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = build_cells(plan->cells, s, n, pos);
  if (e != hipSuccess) return pol_hip_fail(e);
  PairArgs a = pair_args(plan, n, pos, q, mu, pol);
  a.o_pos = dE_dpos;
  a.o_q = dE_dq;
  a.o_mu = dE_dmu;
  a.epart = energy ? plan->epart : nullptr;
  const int nb = pair_blocks(n);
  if (n > 0) hipLaunchKernelGGL(k_pair<kEnergyGrad>, dim3(nb), dim3(kPairThreads), 0, s, a);
  if (energy) {
    if (n > 0)
      hipLaunchKernelGGL(k_energy_sum, dim3(1), dim3(256), 0, s, plan->epart, nb,
                         plan->desc.prefactor, energy);
    else
      hipLaunchKernelGGL(k_energy_sum, dim3(1), dim3(256), 0, s, plan->epart, 0,
                         plan->desc.prefactor, energy);
  }
  e = hipGetLastError();
  return e == hipSuccess ? PME_OK : pol_hip_fail(e);
}

int pol_real_mixed(pol_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                   const float* mu, const float* pol, const float* v_pos, float* g_mu) {
  if (!check_common(plan, n, pos, pol) || !g_mu || (n > 0 && !v_pos)) return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = build_cells(plan->cells, s, n, pos);
  if (e != hipSuccess) return pol_hip_fail(e);
  PairArgs a = pair_args(plan, n, pos, q, mu, pol);
  a.vpos = v_pos;
  a.o_mu = g_mu;
  if (n > 0)
    hipLaunchKernelGGL(k_pair<kMixed>, dim3(pair_blocks(n)), dim3(kPairThreads), 0, s, a);
  e = hipGetLastError();
  return e == hipSuccess ? PME_OK : pol_hip_fail(e);
}

int pol_model(pol_plan_t plan, pme_plan_t pme, void* stream, int32_t n, const float* pos,
              const float* q, const float* mu, const float* pol, const double* box,
              double* energy, float* dU_dpos, float* dU_dq, float* dU_dmu) {
  if (!check_common(plan, n, pos, pol) || !pme || !box) return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t stride = size_t(3) * plan->desc.max_atoms;
  float* gp = plan->vec + 4 * stride;     // PME gradients
  float* gm = plan->vec + 5 * stride;
  float* hp = plan->vec + 6 * stride;     // real-space gradients
  float* hm = plan->vec + 7 * stride;
  float* gq = plan->vec;                  // charge gradients (PME, real space)
  float* hq = plan->vec + stride;
  double* e_lr = plan->scal;              // [0..2]
  double* e_re = plan->scal + 3;
  int rc = pme_forward(pme, stream, n, pos, q, mu, box, energy ? e_lr : nullptr,
                       dU_dpos ? gp : nullptr, dU_dq ? gq : nullptr, dU_dmu ? gm : nullptr);
  if (rc != PME_OK) return rc;
  if ((rc = pol_real(plan, stream, n, pos, q, mu, pol, energy ? e_re : nullptr,
                     dU_dpos ? hp : nullptr, dU_dq ? hq : nullptr,
                     dU_dmu ? hm : nullptr)) != PME_OK)
    return rc;
  if (n > 0 && (dU_dpos || dU_dmu))
    hipLaunchKernelGGL(k_model_grads, dim3(blocks_for(3 * n, 256)), dim3(256), 0, s, n,
                       float(plan->desc.prefactor), pol, mu, gp, hp, gm, hm, dU_dpos, dU_dmu);
  if (n > 0 && dU_dq)
    hipLaunchKernelGGL(k_add, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, gq, hq, dU_dq);
  if (energy)
    hipLaunchKernelGGL(k_model_energy, dim3(1), dim3(256), 0, s, n, plan->desc.prefactor, pol,
                       mu, e_lr, e_re, energy);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? PME_OK : pol_hip_fail(e);
}

int pol_model_hvp(pol_plan_t plan, pme_plan_t pme, void* stream, int32_t n, const float* pos,
                  const float* q, const float* mu, const float* pol, const double* box,
                  const float* v_pos, const float* v_q, const float* v_mu, float* g_q,
                  float* g_mu) {
  if (!check_common(plan, n, pos, pol) || !pme || !box || !g_q || !g_mu) return PME_EINVAL;
  if (n == 0) return PME_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t stride = size_t(3) * plan->desc.max_atoms;
  float* lq = plan->vec;                  // PME rows
  float* lm = plan->vec + 4 * stride;
  float* rq = plan->vec + stride;         // real-space rows
  float* rm = plan->vec + 5 * stride;
  int rc = pme_backward(pme, stream, n, pos, q, mu, box, v_pos, v_q, v_mu, nullptr, lq, lm);
  if (rc != PME_OK) return rc;
  hipError_t e = build_cells(plan->cells, s, n, pos);
  if (e != hipSuccess) return pol_hip_fail(e);
  PairArgs a = pair_args(plan, n, pos, q, mu, pol);
  a.vpos = v_pos; a.vq = v_q; a.vmu = v_mu;
  a.o_q = rq;
  a.o_mu = rm;
  hipLaunchKernelGGL(k_pair<kHvp>, dim3(pair_blocks(n)), dim3(kPairThreads), 0, s, a);
  // mu row: the polarization term adds (pf / a) v_mu (k_model_grads with mu = v_mu)
  hipLaunchKernelGGL(k_model_grads, dim3(blocks_for(3 * n, 256)), dim3(256), 0, s, n,
                     float(plan->desc.prefactor), pol, v_mu, lm, rm, lm, rm, nullptr, g_mu);
  hipLaunchKernelGGL(k_add, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, lq, rq, g_q);
  e = hipGetLastError();
  return e == hipSuccess ? PME_OK : pol_hip_fail(e);
}

int pol_scf(pol_plan_t plan, pme_plan_t pme, void* stream, int32_t n, const float* pos,
            const float* q, const float* pol, const double* box, double tol, int32_t max_iter,
            float* mu, int32_t* iters, double* resid) {
  if (!check_common(plan, n, pos, pol) || !pme || !box || !mu || max_iter < 0 || !(tol >= 0.0))
    return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int m = 3 * n;
  const size_t stride = size_t(3) * plan->desc.max_atoms;
  float* g1 = plan->vec;
  float* g2 = g1 + stride;
  float* r = g2 + stride;
  float* z = r + stride;
  float* p = z + stride;
  float* Ap = p + stride;
  double* scal = plan->scal;
  const float pf = float(plan->desc.prefactor);
  const bool warm = (plan->desc.flags & POL_F_WARM_START) != 0;
  const bool fixed = (plan->desc.flags & POL_F_FIXED_ITERS) != 0;
  const int vb = blocks_for(m, 256);
  int rc;
  hipError_t e;
  if (iters) *iters = 0;
  if (resid) *resid = 0.0;
  if (n == 0) return PME_OK;
  // A v = (pf / a) v + H_pme v + H_real v
  auto matvec = [&](const float* v, float* out) -> int {
    int rr = pme_backward(pme, stream, n, pos, q, nullptr, box, nullptr, nullptr, v, nullptr,
                          nullptr, g1);
    if (rr != PME_OK) return rr;
    hipError_t he = real_mu_grad(plan, s, n, pos, nullptr, v, pol, g2);
    if (he != hipSuccess) return pol_hip_fail(he);
    hipLaunchKernelGGL(k_matvec_sum, dim3(vb), dim3(256), 0, s, m, pf, pol, v, g1, g2, out);
    he = hipGetLastError();
    return he == hipSuccess ? PME_OK : pol_hip_fail(he);
  };
  if (warm && (rc = matvec(mu, Ap)) != PME_OK) return rc;
  // right-hand side: -(dE_lr/dmu + dE_real/dmu) at mu = 0 (charges only)
  if ((rc = pme_forward(pme, stream, n, pos, q, nullptr, box, nullptr, nullptr, nullptr, g1)) !=
      PME_OK)
    return rc;
  if ((e = real_mu_grad(plan, s, n, pos, q, nullptr, pol, g2)) != hipSuccess)
    return pol_hip_fail(e);
  hipLaunchKernelGGL(k_pcg_start, dim3(vb), dim3(256), 0, s, m, pf, pol, g1, g2, Ap, mu, r, z, p,
                     warm ? 1 : 0);
  hipLaunchKernelGGL(k_dot2, dim3(1), dim3(1024), 0, s, m, r, z, z, z, scal);
  int it = 0;
  double rms = 0.0;
  for (;;) {
    if (fixed) {
      // no host round trip: exactly max_iter iterations (capturable)
      if (it >= max_iter) {
        rms = -1.0;
        break;
      }
    } else {
      double h[2];
      if ((e = hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, s)) != hipSuccess ||
          (e = hipStreamSynchronize(s)) != hipSuccess)
        return pol_hip_fail(e);
      rms = sqrt(fmax(h[1], 0.0) / double(m));
      if (!isfinite(rms)) return PME_ENONFINITE;
      if (rms < tol || it >= max_iter) break;
    }
    if ((rc = matvec(p, Ap)) != PME_OK) return rc;
    hipLaunchKernelGGL(k_dot2, dim3(1), dim3(1024), 0, s, m, p, Ap, p, p, scal + 2);
    hipLaunchKernelGGL(k_pcg_step, dim3(vb), dim3(256), 0, s, m, pf, pol, scal, p, Ap, mu, r, z);
    hipLaunchKernelGGL(k_dot2, dim3(1), dim3(1024), 0, s, m, r, z, z, z, scal + 4);
    hipLaunchKernelGGL(k_pcg_dir, dim3(vb), dim3(256), 0, s, m, scal, z, p);
    hipLaunchKernelGGL(k_copy_scal, dim3(1), dim3(64), 0, s, scal);
    if ((e = hipGetLastError()) != hipSuccess) return pol_hip_fail(e);
    ++it;
  }
  if (iters) *iters = it;
  if (resid) *resid = rms;
  return PME_OK;
}

}  // extern "C"
