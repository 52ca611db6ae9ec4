// Learned dipole head: local features, the SiLU MLP forward and backward, the
// training loss against the polarizable teacher and Adam (definitions in dip.h).
//
// Features give 16 lanes to an atom over the cell list of cells.h and combine the
// lanes' sums with shuffles.  The MLP runs 16 atoms per 64-thread workgroup with
// the weights staged in LDS (transposed, padded rows): a thread owns one hidden
// unit and loops over the workgroup's atoms.  Parameter gradients are summed per
// workgroup, then over workgroups in a fixed order.
#include <math.h>
#include <stdio.h>

#include <new>

#include "../../include/dip.h"
#include "cells.h"

namespace {

constexpr int NR = 8, NS = 2, NCH = DIP_NCH, NF = DIP_NFEAT, HID = DIP_HIDDEN;
constexpr int NP = DIP_NPARAM;
constexpr int oW1 = 0, ob1 = oW1 + HID * NF, oW2 = ob1 + HID, ob2 = oW2 + HID * HID;
constexpr int oW3 = ob2 + HID, ob3 = oW3 + NCH * HID;
static_assert(ob3 + NCH == NP, "parameter layout");
static_assert(NCH == NR * NS && NF == 2 * NCH + NS, "feature layout");

constexpr int kLanes = 16;
constexpr int kFeatThreads = 256;
constexpr int kAtoms = 16;            // atoms per MLP workgroup
constexpr int kMlpThreads = 64;
constexpr int HP = HID + 1;           // padded LDS row of 64

__device__ __forceinline__ float lane_sum(float v) {
#pragma unroll
  for (int o = kLanes / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kLanes);
  return v;
}

struct FeatArgs {
  int n;
  const float* pos;
  const float* q;
  CellGrid g;
  const int* start;
  const int* sorted;
  float rc;
  float* feat;
  float* vec;
};

__global__ void __launch_bounds__(kFeatThreads) k_features(FeatArgs a) {
  const int lane = threadIdx.x % kLanes;
  const int i = blockIdx.x * (kFeatThreads / kLanes) + threadIdx.x / kLanes;
  const bool live = i < a.n;
  const int ii = live ? i : 0;
  const float px = a.pos[3 * ii], py = a.pos[3 * ii + 1], pz = a.pos[3 * ii + 2];
  // per species s (A: cation neighbours, B: anion neighbours) and radial k
  float gA[NR], gB[NR], vA[NR][3], vB[NR][3];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    gA[k] = gB[k] = 0.0f;
    vA[k][0] = vA[k][1] = vA[k][2] = vB[k][0] = vB[k][1] = vB[k][2] = 0.0f;
  }
  const float rc2 = a.rc * a.rc, irc = 1.0f / a.rc;
  const float norm = sqrtf(2.0f * irc);
  if (live) {
    int c[3], no[3];
    cell_of(a.g, px, py, pz, c);
#pragma unroll
    for (int d = 0; d < 3; ++d) no[d] = a.g.nc[d] < 3 ? a.g.nc[d] : 3;
    for (int ox = 0; ox < no[0]; ++ox)
      for (int oy = 0; oy < no[1]; ++oy)
        for (int oz = 0; oz < no[2]; ++oz) {
          const int cell = (neighbour_cell(c[0], ox, a.g.nc[0]) * a.g.nc[1] +
                            neighbour_cell(c[1], oy, a.g.nc[1])) * a.g.nc[2] +
                           neighbour_cell(c[2], oz, a.g.nc[2]);
          for (int kk = a.start[cell] + lane; kk < a.start[cell + 1]; kk += kLanes) {
            const int j = a.sorted[kk];
            if (j == i) continue;
            const float3 R = min_image(a.g, px - a.pos[3 * j], py - a.pos[3 * j + 1],
                                       pz - a.pos[3 * j + 2]);
            const float r2 = R.x * R.x + R.y * R.y + R.z * R.z;
            if (r2 >= rc2 || r2 <= 0.0f) continue;
            const float r = sqrtf(r2), ir = 1.0f / r, x = r * irc;
            const float x2 = x * x, x5 = x2 * x2 * x;
            const float env = 1.0f - 21.0f * x5 + 35.0f * x5 * x - 15.0f * x5 * x2;
            const float pref = norm * ir * env;
            const float qj = a.q[j];
            const bool cat = qj > 0.0f;
            const float ux = R.x * ir, uy = R.y * ir, uz = R.z * ir;
            // sin((k+1) t) by the Chebyshev recurrence from sin t, cos t
            float sn, cs;
            sincosf(float(M_PI) * x, &sn, &cs);
            float s_prev = 0.0f, s_cur = sn;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
              const float Rk = pref * s_cur;
              const float qR = qj * Rk;
              if (cat) {
                gA[k] += Rk;
                vA[k][0] += qR * ux; vA[k][1] += qR * uy; vA[k][2] += qR * uz;
              } else {
                gB[k] += Rk;
                vB[k][0] += qR * ux; vB[k][1] += qR * uy; vB[k][2] += qR * uz;
              }
              const float s_next = 2.0f * cs * s_cur - s_prev;
              s_prev = s_cur;
              s_cur = s_next;
            }
          }
        }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    gA[k] = lane_sum(gA[k]);
    gB[k] = lane_sum(gB[k]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      vA[k][d] = lane_sum(vA[k][d]);
      vB[k][d] = lane_sum(vB[k][d]);
    }
  }
  if (live && lane == 0) {
    float* f = a.feat + size_t(i) * NF;
    float* v = a.vec + size_t(i) * NCH * 3;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      f[k] = gA[k];
      f[NR + k] = gB[k];
      f[NCH + k] = vA[k][0] * vA[k][0] + vA[k][1] * vA[k][1] + vA[k][2] * vA[k][2];
      f[NCH + NR + k] = vB[k][0] * vB[k][0] + vB[k][1] * vB[k][1] + vB[k][2] * vB[k][2];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        v[3 * k + d] = vA[k][d];
        v[3 * (NR + k) + d] = vB[k][d];
      }
    }
    const float qi = a.q[i];
    f[2 * NCH] = qi > 0.0f ? 1.0f : 0.0f;
    f[2 * NCH + 1] = qi > 0.0f ? 0.0f : 1.0f;
  }
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// LDS of one MLP workgroup
struct MlpLds {
  float W1T[NF][HP];     // W1T[k][o] = W1[o][k]
  float W2T[HID][HP];    // W2T[k][o] = W2[o][k]
  float W3[NCH][HP];
  float b1[HID], b2[HID], b3[NCH];
  float x[kAtoms][NF + 1];
  float z1[kAtoms][HP], h1[kAtoms][HP];
  float z2[kAtoms][HP], h2[kAtoms][HP];
  float w[kAtoms][NCH + 1];
  float V[kAtoms][NCH * 3 + 1];
};

// Stage the weights and the workgroup's inputs, run the network; leaves z1, h1,
// z2, h2 and w in LDS.
__device__ void mlp_eval(MlpLds& L, const float* P, const float* feat, const float* vec, int a0,
                         int na) {
  const int t = threadIdx.x;
  for (int e = t; e < HID * NF; e += kMlpThreads) {
    const int o = e / NF, k = e - o * NF;
    L.W1T[k][o] = P[oW1 + e];
  }
  for (int e = t; e < HID * HID; e += kMlpThreads) {
    const int o = e / HID, k = e - o * HID;
    L.W2T[k][o] = P[oW2 + e];
  }
  for (int e = t; e < NCH * HID; e += kMlpThreads) {
    const int c = e / HID, k = e - c * HID;
    L.W3[c][k] = P[oW3 + e];
  }
  L.b1[t] = P[ob1 + t];
  L.b2[t] = P[ob2 + t];
  if (t < NCH) L.b3[t] = P[ob3 + t];
  for (int e = t; e < kAtoms * NF; e += kMlpThreads) {
    const int a = e / NF, k = e - a * NF;
    L.x[a][k] = (a < na) ? feat[size_t(a0 + a) * NF + k] : 0.0f;
  }
  for (int e = t; e < kAtoms * NCH * 3; e += kMlpThreads) {
    const int a = e / (NCH * 3), k = e - a * NCH * 3;
    L.V[a][k] = (a < na) ? vec[size_t(a0 + a) * NCH * 3 + k] : 0.0f;
  }
  __syncthreads();
  // layer 1: thread t is hidden unit t
  for (int a = 0; a < kAtoms; ++a) {
    float z = L.b1[t];
#pragma unroll
    for (int k = 0; k < NF; ++k) z += L.W1T[k][t] * L.x[a][k];
    L.z1[a][t] = z;
    L.h1[a][t] = silu(z);
  }
  __syncthreads();
  for (int a = 0; a < kAtoms; ++a) {
    float z = L.b2[t];
#pragma unroll 8
    for (int k = 0; k < HID; ++k) z += L.W2T[k][t] * L.h1[a][k];
    L.z2[a][t] = z;
    L.h2[a][t] = silu(z);
  }
  __syncthreads();
  // layer 3: 16 atoms x 16 outputs, four per thread
  for (int e = t; e < kAtoms * NCH; e += kMlpThreads) {
    const int a = e / NCH, c = e - a * NCH;
    float z = L.b3[c];
#pragma unroll 8
    for (int k = 0; k < HID; ++k) z += L.W3[c][k] * L.h2[a][k];
    L.w[a][c] = z;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kMlpThreads) k_mlp_forward(int n, const float* P,
                                                             const float* feat, const float* vec,
                                                             float* mu) {
  __shared__ MlpLds L;
  const int a0 = blockIdx.x * kAtoms;
  const int na = min(kAtoms, n - a0);
  mlp_eval(L, P, feat, vec, a0, na);
  const int t = threadIdx.x;
  if (t < 3 * kAtoms) {
    const int a = t / 3, d = t - 3 * a;
    if (a < na) {
      float m = 0.0f;
#pragma unroll
      for (int c = 0; c < NCH; ++c) m += L.w[a][c] * L.V[a][3 * c + d];
      mu[size_t(a0 + a) * 3 + d] = m;
    }
  }
}

// Per-workgroup parameter gradient partials (part[block][NP]).
__global__ void __launch_bounds__(kMlpThreads) k_mlp_backward(int n, const float* P,
                                                              const float* feat, const float* vec,
                                                              const float* g0, const float* g1,
                                                              const float* g2, float* part) {
  __shared__ MlpLds L;
  __shared__ float gw[kAtoms][NCH + 1];
  __shared__ float gz2[kAtoms][HP];
  __shared__ float gz1[kAtoms][HP];
  const int a0 = blockIdx.x * kAtoms;
  const int na = min(kAtoms, n - a0);
  mlp_eval(L, P, feat, vec, a0, na);
  const int t = threadIdx.x;
  // dL/dw_c = dL/dmu . V_c
  for (int e = t; e < kAtoms * NCH; e += kMlpThreads) {
    const int a = e / NCH, c = e - a * NCH;
    float s = 0.0f;
    if (a < na) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const size_t k = size_t(a0 + a) * 3 + d;
        const float g = (g0 ? g0[k] : 0.0f) + (g1 ? g1[k] : 0.0f) + (g2 ? g2[k] : 0.0f);
        s += g * L.V[a][3 * c + d];
      }
    }
    gw[a][c] = s;
  }
  __syncthreads();
  for (int a = 0; a < kAtoms; ++a) {
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < NCH; ++c) s += L.W3[c][t] * gw[a][c];
    gz2[a][t] = s * dsilu(L.z2[a][t]);
  }
  __syncthreads();
  for (int a = 0; a < kAtoms; ++a) {
    float s = 0.0f;
#pragma unroll 8
    for (int k = 0; k < HID; ++k) s += L.W2T[t][k] * gz2[a][k];   // W2[k][t]
    gz1[a][t] = s * dsilu(L.z1[a][t]);
  }
  __syncthreads();
  float* out = part + size_t(blockIdx.x) * NP;
  // thread t owns row t of W1, W2 and b1, b2, column t of W3, and b3[t] (t < 16)
  for (int k = 0; k < NF; ++k) {
    float s = 0.0f;
    for (int a = 0; a < kAtoms; ++a) s += gz1[a][t] * L.x[a][k];
    out[oW1 + t * NF + k] = s;
  }
  for (int k = 0; k < HID; ++k) {
    float s = 0.0f;
    for (int a = 0; a < kAtoms; ++a) s += gz2[a][t] * L.h1[a][k];
    out[oW2 + t * HID + k] = s;
  }
  for (int c = 0; c < NCH; ++c) {
    float s = 0.0f;
    for (int a = 0; a < kAtoms; ++a) s += gw[a][c] * L.h2[a][t];
    out[oW3 + c * HID + t] = s;
  }
  float sb1 = 0.0f, sb2 = 0.0f;
  for (int a = 0; a < kAtoms; ++a) {
    sb1 += gz1[a][t];
    sb2 += gz2[a][t];
  }
  out[ob1 + t] = sb1;
  out[ob2 + t] = sb2;
  if (t < NCH) {
    float s = 0.0f;
    for (int a = 0; a < kAtoms; ++a) s += gw[a][t];
    out[ob3 + t] = s;
  }
}

// Feature cotangents of the position vector-Jacobian product for dL/dmu = u:
// fbar[i] = [dL/dG_i (16) | dL/dV_i (16 x 3)], with dL/dw_c = u . V_c run back through
// the network to its inputs and dL/dV_c = w_c u + 2 (dL/dx_{16+c}) V_c.
__global__ void __launch_bounds__(kMlpThreads) k_mlp_input_grad(int n, const float* P,
                                                                const float* feat,
                                                                const float* vec, const float* u,
                                                                float* fbar) {
  __shared__ MlpLds L;
  __shared__ float gw[kAtoms][NCH + 1];
  __shared__ float gz2[kAtoms][HP];   // later the input gradient (first 2 NCH inputs)
  __shared__ float gz1[kAtoms][HP];
  const int a0 = blockIdx.x * kAtoms;
  const int na = min(kAtoms, n - a0);
  mlp_eval(L, P, feat, vec, a0, na);
  const int t = threadIdx.x;
  for (int e = t; e < kAtoms * NCH; e += kMlpThreads) {
    const int a = e / NCH, c = e - a * NCH;
    float s = 0.0f;
    if (a < na)
#pragma unroll
      for (int d = 0; d < 3; ++d) s += u[size_t(a0 + a) * 3 + d] * L.V[a][3 * c + d];
    gw[a][c] = s;
  }
  __syncthreads();
  for (int a = 0; a < kAtoms; ++a) {
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < NCH; ++c) s += L.W3[c][t] * gw[a][c];
    gz2[a][t] = s * dsilu(L.z2[a][t]);
  }
  __syncthreads();
  for (int a = 0; a < kAtoms; ++a) {
    float s = 0.0f;
#pragma unroll 8
    for (int k = 0; k < HID; ++k) s += L.W2T[t][k] * gz2[a][k];   // W2[k][t]
    gz1[a][t] = s * dsilu(L.z1[a][t]);
  }
  __syncthreads();
  // dL/dx_k = sum_o gz1[o] W1[o][k] for the inputs G and |V|^2 (the species one-hot
  // does not move)
  for (int e = t; e < kAtoms * 2 * NCH; e += kMlpThreads) {
    const int a = e / (2 * NCH), k = e - a * 2 * NCH;
    float s = 0.0f;
#pragma unroll 8
    for (int o = 0; o < HID; ++o) s += gz1[a][o] * L.W1T[k][o];
    gz2[a][k] = s;
  }
  __syncthreads();
  for (int e = t; e < kAtoms * 4 * NCH; e += kMlpThreads) {
    const int a = e / (4 * NCH), k = e - a * 4 * NCH;
    if (a >= na) continue;
    float v;
    if (k < NCH) {
      v = gz2[a][k];
    } else {
      const int c = (k - NCH) / 3, d = (k - NCH) - 3 * c;
      v = L.w[a][c] * u[size_t(a0 + a) * 3 + d] + 2.0f * gz2[a][NCH + c] * L.V[a][3 * c + d];
    }
    fbar[size_t(a0 + a) * 4 * NCH + k] = v;
  }
}

struct VjpArgs {
  int n;
  const float* pos;
  const float* q;
  CellGrid g;
  const int* start;
  const int* sorted;
  float rc;
  const float* fbar;   // [n][64] feature cotangents
  const float* base;   // [n][3] added to the output, or NULL
  float* g_pos;        // [n][3] out
};

// d/dR of the features of the centre atom of a pair (R = r_c - r_o, neighbour o
// with charge qo) contracted with the cotangents cg[k], cv[k][3] of the neighbour's
// species: sum_k cg R_k' u + qo [R_k' (cv.u) u + R_k / r (cv - (cv.u) u)].
__device__ __forceinline__ float3 pair_vjp(const float* cg, const float* cv, float qo, float ux,
                                           float uy, float uz, const float (&Rk)[NR],
                                           const float (&dR)[NR], float ir) {
  float fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const float vx = cv[3 * k], vy = cv[3 * k + 1], vz = cv[3 * k + 2];
    const float cu = vx * ux + vy * uy + vz * uz;
    const float a = cg[k] * dR[k] + qo * (dR[k] - Rk[k] * ir) * cu;
    const float b = qo * Rk[k] * ir;
    fx += a * ux + b * vx;
    fy += a * uy + b * vy;
    fz += a * uz + b * vz;
  }
  return make_float3(fx, fy, fz);
}

// g_i = sum_j [d/dr_i of the features of i, with i's cotangents] + [d/dr_i of the
// features of j, with j's cotangents]: the pair (i, j) is visited from i only, so
// no atomics are needed.  16 lanes per atom as in k_features.
__global__ void __launch_bounds__(kFeatThreads) k_features_vjp(VjpArgs a) {
  __shared__ float s_f[kFeatThreads / kLanes][4 * NCH];
  const int lane = threadIdx.x % kLanes;
  const int slot = threadIdx.x / kLanes;
  const int i = blockIdx.x * (kFeatThreads / kLanes) + slot;
  const bool live = i < a.n;
  const int ii = live ? i : 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s_f[slot][lane + kLanes * k] = a.fbar[size_t(ii) * 4 * NCH + lane + kLanes * k];
  __syncthreads();
  const float px = a.pos[3 * ii], py = a.pos[3 * ii + 1], pz = a.pos[3 * ii + 2];
  const float qi = a.q[ii];
  const int si = qi > 0.0f ? 0 : 1;
  const float rc2 = a.rc * a.rc, irc = 1.0f / a.rc;
  const float norm = sqrtf(2.0f * irc);
  const float kpi = float(M_PI) * irc;
  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
  if (live) {
    int c[3], no[3];
    cell_of(a.g, px, py, pz, c);
#pragma unroll
    for (int d = 0; d < 3; ++d) no[d] = a.g.nc[d] < 3 ? a.g.nc[d] : 3;
    for (int ox = 0; ox < no[0]; ++ox)
      for (int oy = 0; oy < no[1]; ++oy)
        for (int oz = 0; oz < no[2]; ++oz) {
          const int cell = (neighbour_cell(c[0], ox, a.g.nc[0]) * a.g.nc[1] +
                            neighbour_cell(c[1], oy, a.g.nc[1])) * a.g.nc[2] +
                           neighbour_cell(c[2], oz, a.g.nc[2]);
          for (int kk = a.start[cell] + lane; kk < a.start[cell + 1]; kk += kLanes) {
            const int j = a.sorted[kk];
            if (j == i) continue;
            const float3 R = min_image(a.g, px - a.pos[3 * j], py - a.pos[3 * j + 1],
                                       pz - a.pos[3 * j + 2]);
            const float r2 = R.x * R.x + R.y * R.y + R.z * R.z;
            if (r2 >= rc2 || r2 <= 0.0f) continue;
            const float r = sqrtf(r2), ir = 1.0f / r, x = r * irc;
            const float x2 = x * x, x4 = x2 * x2, x5 = x4 * x;
            const float env = 1.0f - 21.0f * x5 + 35.0f * x5 * x - 15.0f * x5 * x2;
            const float denv = (-105.0f * x4 + 210.0f * x5 - 105.0f * x5 * x) * irc;
            const float ux = R.x * ir, uy = R.y * ir, uz = R.z * ir;
            // R_k = norm sin(k pi x) env / r and its r-derivative, sin and cos of
            // (k+1) pi x by the Chebyshev recurrences
            float sn, cs;
            sincosf(float(M_PI) * x, &sn, &cs);
            float Rk[NR], dR[NR];
            float s_prev = 0.0f, s_cur = sn, c_prev = 1.0f, c_cur = cs;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
              Rk[k] = norm * s_cur * env * ir;
              dR[k] = norm * ((k + 1) * kpi * c_cur * env * ir - s_cur * env * ir * ir +
                              s_cur * ir * denv);
              const float s_next = 2.0f * cs * s_cur - s_prev;
              const float c_next = 2.0f * cs * c_cur - c_prev;
              s_prev = s_cur;
              s_cur = s_next;
              c_prev = c_cur;
              c_cur = c_next;
            }
            const float qj = a.q[j];
            const int sj = qj > 0.0f ? 0 : 1;
            // features of i (neighbour j of species sj), R_ij = R
            const float* fi = s_f[slot];
            const float3 f1 = pair_vjp(fi + sj * NR, fi + NCH + 3 * sj * NR, qj, ux, uy, uz, Rk,
                                       dR, ir);
            // features of j (neighbour i of species si), R_ji = -R
            const float* fj = a.fbar + size_t(j) * 4 * NCH;
            const float3 f2 = pair_vjp(fj + si * NR, fj + NCH + 3 * si * NR, qi, -ux, -uy, -uz,
                                       Rk, dR, ir);
            gx += f1.x - f2.x;
            gy += f1.y - f2.y;
            gz += f1.z - f2.z;
          }
        }
  }
  gx = lane_sum(gx);
  gy = lane_sum(gy);
  gz = lane_sum(gz);
  if (live && lane == 0) {
    if (a.base) {
      gx += a.base[3 * i];
      gy += a.base[3 * i + 1];
      gz += a.base[3 * i + 2];
    }
    a.g_pos[3 * i] = gx;
    a.g_pos[3 * i + 1] = gy;
    a.g_pos[3 * i + 2] = gz;
  }
}

// ---- Charge head, feature tangents and the dual (forward-mode) networks ----
//
// The charge head c_i = w2 . silu(W1 x_i + b1) runs 16 atoms per 64-thread
// workgroup with a thread per hidden unit; the output sums over the hidden units
// are wavefront butterflies (every lane ends with the same bits).  Centring uses
// means from k_means, one workgroup reducing in a fixed order in FP64.

constexpr int NQP = DIP_NQPARAM;
constexpr int oQW1 = 0, oQb1 = HID * NF, oQw2 = oQb1 + HID;
static_assert(oQw2 + HID == NQP, "charge head layout");
constexpr int kAtomsD = 8;            // atoms per tile of the dual dipole network
constexpr int kGradBlocks = 512;      // cap on the workgroups of the parameter gradients

__device__ __forceinline__ float d2silu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f - s) * (2.0f + z * (1.0f - 2.0f * s));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// rows [a0, a0 + na) of a [n][W] array into LDS rows of stride LD (zeros past na
// or for a NULL source)
template <int ROWS, int W, int LD>
__device__ __forceinline__ void stage_rows(float (&dst)[ROWS][LD], const float* src, int a0,
                                           int na) {
  for (int e = threadIdx.x; e < ROWS * W; e += kMlpThreads) {
    const int a = e / W, k = e - a * W;
    dst[a][k] = (src && a < na) ? src[size_t(a0 + a) * W + k] : 0.0f;
  }
}

struct QLds {
  float W1T[NF][HP];     // W1T[k][o] = W1q[o][k]
  float b1[HID], w2[HID];
  float x[kAtoms][NF + 1];
  float xd[kAtoms][NF + 1];
  float s[kAtoms][HP];
  float gx[kAtoms][2 * NCH + 1];
};

__device__ void q_stage_weights(QLds& L, const float* P) {
  const int t = threadIdx.x;
  for (int e = t; e < HID * NF; e += kMlpThreads) {
    const int o = e / NF, k = e - o * NF;
    L.W1T[k][o] = P[oQW1 + e];
  }
  L.b1[t] = P[oQb1 + t];
  L.w2[t] = P[oQw2 + t];
}

// c and its tangent c_dot along feat_dot (uncentred), one 16-atom tile per workgroup
__global__ void __launch_bounds__(kMlpThreads) k_qhead_forward(int n, const float* P,
                                                               const float* feat,
                                                               const float* feat_dot, float* c,
                                                               float* cd) {
  __shared__ QLds L;
  const int a0 = blockIdx.x * kAtoms;
  const int na = min(kAtoms, n - a0);
  const int t = threadIdx.x;
  q_stage_weights(L, P);
  stage_rows<kAtoms, NF, NF + 1>(L.x, feat, a0, na);
  stage_rows<kAtoms, NF, NF + 1>(L.xd, feat_dot, a0, na);
  __syncthreads();
  for (int a = 0; a < kAtoms; ++a) {
    float z = L.b1[t], zd = 0.0f;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      z += L.W1T[k][t] * L.x[a][k];
      zd += L.W1T[k][t] * L.xd[a][k];
    }
    const float s = wave_sum(L.w2[t] * silu(z));
    const float sd = wave_sum(L.w2[t] * dsilu(z) * zd);
    if (t == 0 && a < na) {
      c[a0 + a] = s;
      cd[a0 + a] = sd;
    }
  }
}

// out[0] = mean of (a0 + a1), out[1] = mean of b (NULL arrays are zero); one workgroup
__global__ void __launch_bounds__(1024) k_means(int n, const float* a0, const float* a1,
                                                const float* b, double* out) {
  __shared__ double r0[1024], r1[1024];
  double s0 = 0.0, s1 = 0.0;
  for (int k = threadIdx.x; k < n; k += 1024) {
    s0 += double(a0 ? a0[k] : 0.0f) + double(a1 ? a1[k] : 0.0f);
    s1 += double(b ? b[k] : 0.0f);
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
  if (threadIdx.x == 0) {
    out[0] = n > 0 ? r0[0] / n : 0.0;
    out[1] = n > 0 ? r1[0] / n : 0.0;
  }
}

// q = z + c - mean c; q_dot = c_dot - mean c_dot (either output may be NULL)
__global__ void k_qcentre(int n, const float* z, const float* c, const float* cd,
                          const double* mean, float* q, float* qd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (q) q[i] = z[i] + (c[i] - float(mean[0]));
  if (qd) qd[i] = cd[i] - float(mean[1]);
}

// Feature cotangents of the charge head for a charge cotangent g (centred with
// mean[1]): dL/dx = sum_o (g - mean) w2_o silu'(z_o) W1q[o][:], mapped to
// fbar = [dL/dG (16) | dL/dV (16 x 3)] with dL/dV_c = 2 (dL/dx_{16+c}) V_c; added
// to fbar when `accumulate`.
__global__ void __launch_bounds__(kMlpThreads) k_qhead_input_grad(int n, const float* P,
                                                                  const float* feat,
                                                                  const float* vec,
                                                                  const float* g,
                                                                  const double* mean,
                                                                  float* fbar, int accumulate) {
  __shared__ QLds L;
  const int a0 = blockIdx.x * kAtoms;
  const int na = min(kAtoms, n - a0);
  const int t = threadIdx.x;
  q_stage_weights(L, P);
  stage_rows<kAtoms, NF, NF + 1>(L.x, feat, a0, na);
  __syncthreads();
  const float gm = float(mean[1]);
  for (int a = 0; a < kAtoms; ++a) {
    float z = L.b1[t];
#pragma unroll
    for (int k = 0; k < NF; ++k) z += L.W1T[k][t] * L.x[a][k];
    const float ga = a < na ? g[a0 + a] - gm : 0.0f;
    L.s[a][t] = ga * L.w2[t] * dsilu(z);
  }
  __syncthreads();
  for (int e = t; e < kAtoms * 2 * NCH; e += kMlpThreads) {
    const int a = e / (2 * NCH), k = e - a * 2 * NCH;
    float s = 0.0f;
#pragma unroll 8
    for (int o = 0; o < HID; ++o) s += L.s[a][o] * L.W1T[k][o];
    L.gx[a][k] = s;
  }
  __syncthreads();
  for (int e = t; e < kAtoms * 4 * NCH; e += kMlpThreads) {
    const int a = e / (4 * NCH), k = e - a * 4 * NCH;
    if (a >= na) continue;
    float v;
    if (k < NCH) {
      v = L.gx[a][k];
    } else {
      const int c = (k - NCH) / 3, d = (k - NCH) - 3 * c;
      v = 2.0f * L.gx[a][NCH + c] * vec[size_t(a0 + a) * NCH * 3 + 3 * c + d];
    }
    float* f = fbar + size_t(a0 + a) * 4 * NCH + k;
    *f = accumulate ? *f + v : v;
  }
}

// Charge-head parameter gradient from cotangents (g_q0 + g_q1 - mean[0]) on c and
// (cq - mean[1]) on c_dot; the workgroup walks tiles blockIdx.x, + gridDim.x, ...
// and keeps its thread's row of W1q, b1q[t] and w2q[t] in registers.
__global__ void __launch_bounds__(kMlpThreads) k_qhead_backward(int n, const float* P,
                                                                const float* feat,
                                                                const float* feat_dot,
                                                                const float* g_q0,
                                                                const float* g_q1,
                                                                const float* cq,
                                                                const double* mean,
                                                                float* part) {
  __shared__ QLds L;
  const int t = threadIdx.x;
  q_stage_weights(L, P);
  const float m0 = float(mean[0]), m1 = float(mean[1]);
  float aW[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) aW[k] = 0.0f;
  float ab = 0.0f, aw2 = 0.0f;
  const int tiles = (n + kAtoms - 1) / kAtoms;
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int a0 = tile * kAtoms;
    const int na = min(kAtoms, n - a0);
    __syncthreads();   // the previous tile's reads of x, xd are done
    stage_rows<kAtoms, NF, NF + 1>(L.x, feat, a0, na);
    stage_rows<kAtoms, NF, NF + 1>(L.xd, feat_dot, a0, na);
    __syncthreads();
    for (int a = 0; a < na; ++a) {
      float z = L.b1[t], zd = 0.0f;
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        z += L.W1T[k][t] * L.x[a][k];
        zd += L.W1T[k][t] * L.xd[a][k];
      }
      const size_t i = size_t(a0 + a);
      const float gc = (g_q0 ? g_q0[i] : 0.0f) + (g_q1 ? g_q1[i] : 0.0f) - m0;
      const float gcd = (cq ? cq[i] : 0.0f) - m1;
      const float ds = dsilu(z);
      aw2 += gc * silu(z) + gcd * ds * zd;
      const float gh = gc * L.w2[t], ghd = gcd * L.w2[t];
      const float gz = gh * ds + ghd * d2silu(z) * zd;
      const float gzd = ghd * ds;
      ab += gz;
#pragma unroll
      for (int k = 0; k < NF; ++k) aW[k] += gz * L.x[a][k] + gzd * L.xd[a][k];
    }
  }
  float* out = part + size_t(blockIdx.x) * NQP;
#pragma unroll
  for (int k = 0; k < NF; ++k) out[oQW1 + t * NF + k] = aW[k];
  out[oQb1 + t] = ab;
  out[oQw2 + t] = aw2;
}

struct FeatJvpArgs {
  int n;
  const float* pos;
  const float* q;
  CellGrid g;
  const int* start;
  const int* sorted;
  float rc;
  const float* vec;    // [n][16][3] features of dip_features
  const float* v;      // [n][3] position tangent
  float* feat_dot;     // [n][34]
  float* vec_dot;      // [n][16][3]
};

// Directional derivative of the features along v; 16 lanes per atom as in
// k_features.  Pair R = r_i - r_j, w = v_i - v_j, u = R/r, r_dot = u . w:
//   G_dot += R_k' r_dot,  V_dot += q_j [R_k' r_dot u + R_k/r (w - r_dot u)].
__global__ void __launch_bounds__(kFeatThreads) k_features_jvp(FeatJvpArgs a) {
  const int lane = threadIdx.x % kLanes;
  const int i = blockIdx.x * (kFeatThreads / kLanes) + threadIdx.x / kLanes;
  const bool live = i < a.n;
  const int ii = live ? i : 0;
  const float px = a.pos[3 * ii], py = a.pos[3 * ii + 1], pz = a.pos[3 * ii + 2];
  const float vix = a.v[3 * ii], viy = a.v[3 * ii + 1], viz = a.v[3 * ii + 2];
  float gA[NR], gB[NR], vA[NR][3], vB[NR][3];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    gA[k] = gB[k] = 0.0f;
    vA[k][0] = vA[k][1] = vA[k][2] = vB[k][0] = vB[k][1] = vB[k][2] = 0.0f;
  }
  const float rc2 = a.rc * a.rc, irc = 1.0f / a.rc;
  const float norm = sqrtf(2.0f * irc);
  const float kpi = float(M_PI) * irc;
  if (live) {
    int c[3], no[3];
    cell_of(a.g, px, py, pz, c);
#pragma unroll
    for (int d = 0; d < 3; ++d) no[d] = a.g.nc[d] < 3 ? a.g.nc[d] : 3;
    for (int ox = 0; ox < no[0]; ++ox)
      for (int oy = 0; oy < no[1]; ++oy)
        for (int oz = 0; oz < no[2]; ++oz) {
          const int cell = (neighbour_cell(c[0], ox, a.g.nc[0]) * a.g.nc[1] +
                            neighbour_cell(c[1], oy, a.g.nc[1])) * a.g.nc[2] +
                           neighbour_cell(c[2], oz, a.g.nc[2]);
          for (int kk = a.start[cell] + lane; kk < a.start[cell + 1]; kk += kLanes) {
            const int j = a.sorted[kk];
            if (j == i) continue;
            const float3 R = min_image(a.g, px - a.pos[3 * j], py - a.pos[3 * j + 1],
                                       pz - a.pos[3 * j + 2]);
            const float r2 = R.x * R.x + R.y * R.y + R.z * R.z;
            if (r2 >= rc2 || r2 <= 0.0f) continue;
            const float r = sqrtf(r2), ir = 1.0f / r, x = r * irc;
            const float x2 = x * x, x4 = x2 * x2, x5 = x4 * x;
            const float env = 1.0f - 21.0f * x5 + 35.0f * x5 * x - 15.0f * x5 * x2;
            const float denv = (-105.0f * x4 + 210.0f * x5 - 105.0f * x5 * x) * irc;
            const float ux = R.x * ir, uy = R.y * ir, uz = R.z * ir;
            const float wx = vix - a.v[3 * j], wy = viy - a.v[3 * j + 1],
                        wz = viz - a.v[3 * j + 2];
            const float rd = ux * wx + uy * wy + uz * wz;
            const float px_ = wx - rd * ux, py_ = wy - rd * uy, pz_ = wz - rd * uz;
            const float qj = a.q[j];
            const bool cat = qj > 0.0f;
            float sn, cs;
            sincosf(float(M_PI) * x, &sn, &cs);
            float s_prev = 0.0f, s_cur = sn, c_prev = 1.0f, c_cur = cs;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
              const float Rk = norm * s_cur * env * ir;
              const float dR = norm * ((k + 1) * kpi * c_cur * env * ir - s_cur * env * ir * ir +
                                       s_cur * ir * denv);
              const float gd = dR * rd;
              const float au = qj * gd, ap = qj * Rk * ir;
              if (cat) {
                gA[k] += gd;
                vA[k][0] += au * ux + ap * px_;
                vA[k][1] += au * uy + ap * py_;
                vA[k][2] += au * uz + ap * pz_;
              } else {
                gB[k] += gd;
                vB[k][0] += au * ux + ap * px_;
                vB[k][1] += au * uy + ap * py_;
                vB[k][2] += au * uz + ap * pz_;
              }
              const float s_next = 2.0f * cs * s_cur - s_prev;
              const float c_next = 2.0f * cs * c_cur - c_prev;
              s_prev = s_cur;
              s_cur = s_next;
              c_prev = c_cur;
              c_cur = c_next;
            }
          }
        }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    gA[k] = lane_sum(gA[k]);
    gB[k] = lane_sum(gB[k]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      vA[k][d] = lane_sum(vA[k][d]);
      vB[k][d] = lane_sum(vB[k][d]);
    }
  }
  if (live && lane == 0) {
    float* f = a.feat_dot + size_t(i) * NF;
    float* vd = a.vec_dot + size_t(i) * NCH * 3;
    const float* V = a.vec + size_t(i) * NCH * 3;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      f[k] = gA[k];
      f[NR + k] = gB[k];
      f[NCH + k] = 2.0f * (V[3 * k] * vA[k][0] + V[3 * k + 1] * vA[k][1] + V[3 * k + 2] * vA[k][2]);
      const float* W = V + 3 * NR;
      f[NCH + NR + k] =
          2.0f * (W[3 * k] * vB[k][0] + W[3 * k + 1] * vB[k][1] + W[3 * k + 2] * vB[k][2]);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        vd[3 * k + d] = vA[k][d];
        vd[3 * (NR + k) + d] = vB[k][d];
      }
    }
    f[2 * NCH] = 0.0f;
    f[2 * NCH + 1] = 0.0f;
  }
}

// LDS of the dual dipole network: the weights once per workgroup, and per tile
// the primal and tangent activations of kAtomsD atoms
struct DualLds {
  float W1T[NF][HP];
  float W2T[HID][HP];
  float W3[NCH][HP];
  float b1[HID], b2[HID], b3[NCH];
  float x[kAtomsD][NF + 1], xd[kAtomsD][NF + 1];
  float z1[kAtomsD][HP], z1d[kAtomsD][HP], h1[kAtomsD][HP], h1d[kAtomsD][HP];
  float z2[kAtomsD][HP], z2d[kAtomsD][HP], h2[kAtomsD][HP], h2d[kAtomsD][HP];
  float w[kAtomsD][NCH + 1], wd[kAtomsD][NCH + 1];
  float V[kAtomsD][NCH * 3 + 1], Vd[kAtomsD][NCH * 3 + 1];
};

__device__ void dual_stage_weights(DualLds& L, const float* P) {
  const int t = threadIdx.x;
  for (int e = t; e < HID * NF; e += kMlpThreads) {
    const int o = e / NF, k = e - o * NF;
    L.W1T[k][o] = P[oW1 + e];
  }
  for (int e = t; e < HID * HID; e += kMlpThreads) {
    const int o = e / HID, k = e - o * HID;
    L.W2T[k][o] = P[oW2 + e];
  }
  for (int e = t; e < NCH * HID; e += kMlpThreads) {
    const int c = e / HID, k = e - c * HID;
    L.W3[c][k] = P[oW3 + e];
  }
  L.b1[t] = P[ob1 + t];
  L.b2[t] = P[ob2 + t];
  if (t < NCH) L.b3[t] = P[ob3 + t];
}

// One tile through the network in forward mode (weights already staged); leaves
// every activation and its tangent in LDS.
__device__ void dual_eval(DualLds& L, const float* feat, const float* vec, const float* feat_dot,
                          const float* vec_dot, int a0, int na) {
  const int t = threadIdx.x;
  stage_rows<kAtomsD, NF, NF + 1>(L.x, feat, a0, na);
  stage_rows<kAtomsD, NF, NF + 1>(L.xd, feat_dot, a0, na);
  stage_rows<kAtomsD, NCH * 3, NCH * 3 + 1>(L.V, vec, a0, na);
  stage_rows<kAtomsD, NCH * 3, NCH * 3 + 1>(L.Vd, vec_dot, a0, na);
  __syncthreads();
  for (int a = 0; a < kAtomsD; ++a) {
    float z = L.b1[t], zd = 0.0f;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      z += L.W1T[k][t] * L.x[a][k];
      zd += L.W1T[k][t] * L.xd[a][k];
    }
    L.z1[a][t] = z;
    L.z1d[a][t] = zd;
    L.h1[a][t] = silu(z);
    L.h1d[a][t] = dsilu(z) * zd;
  }
  __syncthreads();
  for (int a = 0; a < kAtomsD; ++a) {
    float z = L.b2[t], zd = 0.0f;
#pragma unroll 8
    for (int k = 0; k < HID; ++k) {
      z += L.W2T[k][t] * L.h1[a][k];
      zd += L.W2T[k][t] * L.h1d[a][k];
    }
    L.z2[a][t] = z;
    L.z2d[a][t] = zd;
    L.h2[a][t] = silu(z);
    L.h2d[a][t] = dsilu(z) * zd;
  }
  __syncthreads();
  for (int e = t; e < kAtomsD * NCH; e += kMlpThreads) {
    const int a = e / NCH, c = e - a * NCH;
    float z = L.b3[c], zd = 0.0f;
#pragma unroll 8
    for (int k = 0; k < HID; ++k) {
      z += L.W3[c][k] * L.h2[a][k];
      zd += L.W3[c][k] * L.h2d[a][k];
    }
    L.w[a][c] = z;
    L.wd[a][c] = zd;
  }
  __syncthreads();
}

// mu = sum_c w_c V_c and mu_dot = sum_c (wd_c V_c + w_c Vd_c), one tile per workgroup
__global__ void __launch_bounds__(kMlpThreads) k_mlp_jvp_forward(int n, const float* P,
                                                                 const float* feat,
                                                                 const float* vec,
                                                                 const float* feat_dot,
                                                                 const float* vec_dot, float* mu,
                                                                 float* mud) {
  __shared__ DualLds L;
  const int a0 = blockIdx.x * kAtomsD;
  const int na = min(kAtomsD, n - a0);
  dual_stage_weights(L, P);
  dual_eval(L, feat, vec, feat_dot, vec_dot, a0, na);
  const int t = threadIdx.x;
  if (t < 3 * kAtomsD) {
    const int a = t / 3, d = t - 3 * a;
    if (a < na) {
      float m = 0.0f, md = 0.0f;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        m += L.w[a][c] * L.V[a][3 * c + d];
        md += L.wd[a][c] * L.V[a][3 * c + d] + L.w[a][c] * L.Vd[a][3 * c + d];
      }
      if (mu) mu[size_t(a0 + a) * 3 + d] = m;
      if (mud) mud[size_t(a0 + a) * 3 + d] = md;
    }
  }
}

// Dipole-head parameter gradient through the dual network: cotangents
// gw_c = (g_mu0 + g_mu1) . V_c + u . Vd_c on w and gwd_c = u . V_c on wd, run back
// through both the primal and the tangent activations (silu'' couples them).  The
// workgroup walks tiles blockIdx.x, + gridDim.x, ...; thread t keeps row t of W1
// and W2, column t of W3 and its biases in registers and writes them once to its
// partial row.
__global__ void __launch_bounds__(kMlpThreads) k_mlp_jvp_backward(
    int n, const float* P, const float* feat, const float* vec, const float* feat_dot,
    const float* vec_dot, const float* g_mu0, const float* g_mu1, const float* u, float* part) {
  __shared__ DualLds L;
  __shared__ float gw[kAtomsD][NCH + 1], gwd[kAtomsD][NCH + 1];
  __shared__ float gz2[kAtomsD][HP], gz2d[kAtomsD][HP];
  __shared__ float gz1[kAtomsD][HP], gz1d[kAtomsD][HP];
  const int t = threadIdx.x;
  dual_stage_weights(L, P);
  float aW1[NF], aW2[HID], aW3[NCH];
#pragma unroll
  for (int k = 0; k < NF; ++k) aW1[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < HID; ++k) aW2[k] = 0.0f;
#pragma unroll
  for (int c = 0; c < NCH; ++c) aW3[c] = 0.0f;
  float ab1 = 0.0f, ab2 = 0.0f, ab3 = 0.0f;
  const int tiles = (n + kAtomsD - 1) / kAtomsD;
  for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int a0 = tile * kAtomsD;
    const int na = min(kAtomsD, n - a0);
    __syncthreads();   // the previous tile is done with the LDS
    dual_eval(L, feat, vec, feat_dot, vec_dot, a0, na);
    for (int e = t; e < kAtomsD * NCH; e += kMlpThreads) {
      const int a = e / NCH, c = e - a * NCH;
      float s = 0.0f, sd = 0.0f;
      if (a < na) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const size_t k = size_t(a0 + a) * 3 + d;
          const float g = (g_mu0 ? g_mu0[k] : 0.0f) + (g_mu1 ? g_mu1[k] : 0.0f);
          const float uk = u ? u[k] : 0.0f;
          s += g * L.V[a][3 * c + d] + uk * L.Vd[a][3 * c + d];
          sd += uk * L.V[a][3 * c + d];
        }
      }
      gw[a][c] = s;
      gwd[a][c] = sd;
    }
    __syncthreads();
    for (int a = 0; a < kAtomsD; ++a) {
      float s = 0.0f, sd = 0.0f;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        s += L.W3[c][t] * gw[a][c];
        sd += L.W3[c][t] * gwd[a][c];
      }
      const float z = L.z2[a][t];
      const float ds = dsilu(z);
      gz2[a][t] = s * ds + sd * d2silu(z) * L.z2d[a][t];
      gz2d[a][t] = sd * ds;
    }
    __syncthreads();
    for (int a = 0; a < kAtomsD; ++a) {
      float s = 0.0f, sd = 0.0f;
#pragma unroll 8
      for (int k = 0; k < HID; ++k) {
        s += L.W2T[t][k] * gz2[a][k];      // W2[k][t]
        sd += L.W2T[t][k] * gz2d[a][k];
      }
      const float z = L.z1[a][t];
      const float ds = dsilu(z);
      gz1[a][t] = s * ds + sd * d2silu(z) * L.z1d[a][t];
      gz1d[a][t] = sd * ds;
    }
    __syncthreads();
    for (int a = 0; a < kAtomsD; ++a) {
      const float g1 = gz1[a][t], g1d = gz1d[a][t];
      const float g2 = gz2[a][t], g2d = gz2d[a][t];
#pragma unroll
      for (int k = 0; k < NF; ++k) aW1[k] += g1 * L.x[a][k] + g1d * L.xd[a][k];
#pragma unroll
      for (int k = 0; k < HID; ++k) aW2[k] += g2 * L.h1[a][k] + g2d * L.h1d[a][k];
      const float h = L.h2[a][t], hd = L.h2d[a][t];
#pragma unroll
      for (int c = 0; c < NCH; ++c) aW3[c] += gw[a][c] * h + gwd[a][c] * hd;
      ab1 += g1;
      ab2 += g2;
      if (t < NCH) ab3 += gw[a][t];
    }
  }
  float* out = part + size_t(blockIdx.x) * NP;
#pragma unroll
  for (int k = 0; k < NF; ++k) out[oW1 + t * NF + k] = aW1[k];
#pragma unroll
  for (int k = 0; k < HID; ++k) out[oW2 + t * HID + k] = aW2[k];
#pragma unroll
  for (int c = 0; c < NCH; ++c) out[oW3 + c * HID + t] = aW3[c];
  out[ob1 + t] = ab1;
  out[ob2 + t] = ab2;
  if (t < NCH) out[ob3 + t] = ab3;
}

// g[p] = sum over nb partial rows of width `width` in row order
__global__ void k_rows_reduce(int nb, int width, const float* part, float* g) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= width) return;
  float s = 0.0f;
  for (int b = 0; b < nb; ++b) s += part[size_t(b) * width + p];
  g[p] = s;
}

__global__ void __launch_bounds__(1024) k_loss(int n, const double* Us, const double* Ut,
                                               const float* ds, const float* dt, const float* mu,
                                               const float* mut, const float* dmu,
                                               const float* dq, double lE, double lF, double lmu,
                                               double* loss, float* vpos, float* gmu, float* gq) {
  __shared__ double rF[1024], rM[1024];
  const int m = 3 * n;
  const double dE = (n > 0) ? (Us[0] - Ut[0]) / double(n) : 0.0;
  const double cE = (n > 0) ? 2.0 * lE * dE / double(n) : 0.0;
  const double inv = (m > 0) ? 1.0 / double(m) : 0.0;
  double sF = 0.0, sM = 0.0;
  for (int k = threadIdx.x; k < m; k += 1024) {
    const float dF = ds[k] - dt[k];
    const float dM = mut ? mu[k] - mut[k] : 0.0f;
    sF += double(dF) * dF;
    sM += double(dM) * dM;
    vpos[k] = float(2.0 * lF * inv) * dF;
    gmu[k] = float(cE) * dmu[k] + float(2.0 * lmu * inv) * dM;
    if (gq && k < n) gq[k] = float(cE) * dq[k];
  }
  rF[threadIdx.x] = sF;
  rM[threadIdx.x] = sM;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      rF[threadIdx.x] += rF[threadIdx.x + o];
      rM[threadIdx.x] += rM[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = lE * dE * dE + lF * rF[0] * inv + lmu * rM[0] * inv;
}

__global__ void k_adam(int count, float lr, float b1, float b2, float eps, float c1, float c2,
                       float* p, const float* g, float* m, float* v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

thread_local char g_dip_err[256] = "";

int dip_fail(hipError_t e) {
  snprintf(g_dip_err, sizeof(g_dip_err), "%s", hipGetErrorString(e));
  return PME_EHIP;
}

inline int mlp_blocks(int n) { return n > 0 ? (n + kAtoms - 1) / kAtoms : 1; }

}  // namespace

inline int grad_blocks(int n, int per) {
  const int tiles = n > 0 ? (n + per - 1) / per : 1;
  return tiles < kGradBlocks ? tiles : kGradBlocks;
}

struct dip_plan_s {
  dip_desc_t desc;
  CellList cells;
  float* part = nullptr;     // [mlp blocks][NP]
  float* fbar = nullptr;     // [max_atoms][64] feature cotangents (position VJP)
  float* dpart = nullptr;    // [grad_blocks(max_atoms, kAtomsD)][NP] dual-network partials
  float* qpart = nullptr;    // [grad_blocks(max_atoms, kAtoms)][NQP] charge-head partials
  float* qbuf = nullptr;     // [2][max_atoms] charge-head outputs c, c_dot
  double* means = nullptr;   // [2]
};

extern "C" {

int dip_plan_create(const dip_desc_t* desc, dip_plan_t* out) {
  if (!desc || !out) return PME_EINVAL;
  *out = nullptr;
  if (desc->max_atoms < 1 || desc->flags != 0) return PME_EINVAL;
  dip_plan_s* pl = new (std::nothrow) dip_plan_s();
  if (!pl) return PME_ENOMEM;
  pl->desc = *desc;
  int rc = setup_cells(pl->cells, desc->box, desc->cutoff, desc->max_atoms);
  hipError_t e = hipSuccess;
  if (rc == PME_OK)
    e = hipMalloc(&pl->part, sizeof(float) * size_t(mlp_blocks(desc->max_atoms)) * NP);
  if (rc == PME_OK && e == hipSuccess)
    e = hipMalloc(&pl->fbar, sizeof(float) * size_t(desc->max_atoms) * 4 * NCH);
  if (rc == PME_OK && e == hipSuccess)
    e = hipMalloc(&pl->dpart, sizeof(float) * size_t(grad_blocks(desc->max_atoms, kAtomsD)) * NP);
  if (rc == PME_OK && e == hipSuccess)
    e = hipMalloc(&pl->qpart, sizeof(float) * size_t(grad_blocks(desc->max_atoms, kAtoms)) * NQP);
  if (rc == PME_OK && e == hipSuccess)
    e = hipMalloc(&pl->qbuf, sizeof(float) * 2 * size_t(desc->max_atoms));
  if (rc == PME_OK && e == hipSuccess) e = hipMalloc(&pl->means, sizeof(double) * 2);
  if (rc != PME_OK || e != hipSuccess) {
    free_cells(pl->cells);
    void* ptrs[] = {pl->part, pl->fbar, pl->dpart, pl->qpart, pl->qbuf, pl->means};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
    delete pl;
    return rc != PME_OK ? rc : (e == hipErrorOutOfMemory ? PME_ENOMEM : dip_fail(e));
  }
  *out = pl;
  return PME_OK;
}

void dip_plan_destroy(dip_plan_t plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  free_cells(plan->cells);
  void* ptrs[] = {plan->part, plan->fbar, plan->dpart, plan->qpart, plan->qbuf, plan->means};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete plan;
}

int dip_features(dip_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                 float* feat, float* vec) {
  if (!plan || n < 0 || n > plan->desc.max_atoms || (n > 0 && (!pos || !q || !feat || !vec)))
    return PME_EINVAL;
  if (n == 0) return PME_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = build_cells(plan->cells, s, n, pos);
  if (e != hipSuccess) return dip_fail(e);
  FeatArgs a;
  a.n = n; a.pos = pos; a.q = q; a.g = plan->cells.g;
  a.start = plan->cells.start; a.sorted = plan->cells.sorted;
  a.rc = float(plan->desc.cutoff); a.feat = feat; a.vec = vec;
  const int per = kFeatThreads / kLanes;
  hipLaunchKernelGGL(k_features, dim3((n + per - 1) / per), dim3(kFeatThreads), 0, s, a);
  e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_forward(dip_plan_t plan, void* stream, int32_t n, const float* params, const float* feat,
                const float* vec, float* mu) {
  if (!plan || n < 0 || n > plan->desc.max_atoms || (n > 0 && (!params || !feat || !vec || !mu)))
    return PME_EINVAL;
  if (n == 0) return PME_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_mlp_forward, dim3(mlp_blocks(n)), dim3(kMlpThreads), 0, s, n, params,
                     feat, vec, mu);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_backward(dip_plan_t plan, void* stream, int32_t n, const float* params, const float* feat,
                 const float* vec, const float* g_mu0, const float* g_mu1, const float* g_mu2,
                 float* g_params) {
  if (!plan || n < 0 || n > plan->desc.max_atoms || !g_params ||
      (n > 0 && (!params || !feat || !vec)))
    return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = n > 0 ? mlp_blocks(n) : 0;
  if (n > 0)
    hipLaunchKernelGGL(k_mlp_backward, dim3(nb), dim3(kMlpThreads), 0, s, n, params, feat, vec,
                       g_mu0, g_mu1, g_mu2, plan->part);
  hipLaunchKernelGGL(k_rows_reduce, dim3((NP + 255) / 256), dim3(256), 0, s, nb, NP, plan->part,
                     g_params);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_position_vjp(dip_plan_t plan, void* stream, int32_t n, const float* params,
                     const float* qparams, const float* pos, const float* q, const float* feat,
                     const float* vec, const float* u, const float* c, const float* base,
                     float* g_pos) {
  if (!plan || n < 0 || n > plan->desc.max_atoms || (u && !params) || (c && !qparams) ||
      (n > 0 && ((!u && !c) || !pos || !q || !feat || !vec || !g_pos)))
    return PME_EINVAL;
  if (n == 0) return PME_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = build_cells(plan->cells, s, n, pos);
  if (e != hipSuccess) return dip_fail(e);
  if (u)
    hipLaunchKernelGGL(k_mlp_input_grad, dim3(mlp_blocks(n)), dim3(kMlpThreads), 0, s, n, params,
                       feat, vec, u, plan->fbar);
  if (c) {
    hipLaunchKernelGGL(k_means, dim3(1), dim3(1024), 0, s, n, nullptr, nullptr, c, plan->means);
    hipLaunchKernelGGL(k_qhead_input_grad, dim3(mlp_blocks(n)), dim3(kMlpThreads), 0, s, n,
                       qparams, feat, vec, c, plan->means, plan->fbar, u ? 1 : 0);
  }
  VjpArgs a;
  a.n = n; a.pos = pos; a.q = q; a.g = plan->cells.g;
  a.start = plan->cells.start; a.sorted = plan->cells.sorted;
  a.rc = float(plan->desc.cutoff); a.fbar = plan->fbar; a.base = base; a.g_pos = g_pos;
  const int per = kFeatThreads / kLanes;
  hipLaunchKernelGGL(k_features_vjp, dim3((n + per - 1) / per), dim3(kFeatThreads), 0, s, a);
  e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_features_jvp(dip_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                     const float* vec, const float* v, float* feat_dot, float* vec_dot) {
  if (!plan || n < 0 || n > plan->desc.max_atoms ||
      (n > 0 && (!pos || !q || !vec || !v || !feat_dot || !vec_dot)))
    return PME_EINVAL;
  if (n == 0) return PME_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = build_cells(plan->cells, s, n, pos);
  if (e != hipSuccess) return dip_fail(e);
  FeatJvpArgs a;
  a.n = n; a.pos = pos; a.q = q; a.g = plan->cells.g;
  a.start = plan->cells.start; a.sorted = plan->cells.sorted;
  a.rc = float(plan->desc.cutoff); a.vec = vec; a.v = v;
  a.feat_dot = feat_dot; a.vec_dot = vec_dot;
  const int per = kFeatThreads / kLanes;
  hipLaunchKernelGGL(k_features_jvp, dim3((n + per - 1) / per), dim3(kFeatThreads), 0, s, a);
  e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_charges(dip_plan_t plan, void* stream, int32_t n, const float* qparams, const float* z,
                const float* feat, const float* feat_dot, float* q, float* q_dot) {
  if (!plan || n < 0 || n > plan->desc.max_atoms ||
      (n > 0 && ((!q && !q_dot) || !qparams || !z || !feat)))
    return PME_EINVAL;
  if (n == 0) return PME_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* c = plan->qbuf;
  float* cd = plan->qbuf + plan->desc.max_atoms;
  hipLaunchKernelGGL(k_qhead_forward, dim3(mlp_blocks(n)), dim3(kMlpThreads), 0, s, n, qparams,
                     feat, feat_dot, c, cd);
  hipLaunchKernelGGL(k_means, dim3(1), dim3(1024), 0, s, n, c, nullptr, cd, plan->means);
  hipLaunchKernelGGL(k_qcentre, dim3((n + 255) / 256), dim3(256), 0, s, n, z, c, cd, plan->means,
                     q, q_dot);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_forward_jvp(dip_plan_t plan, void* stream, int32_t n, const float* params,
                    const float* feat, const float* vec, const float* feat_dot,
                    const float* vec_dot, float* mu, float* mu_dot) {
  if (!plan || n < 0 || n > plan->desc.max_atoms ||
      (n > 0 && ((!mu && !mu_dot) || !params || !feat || !vec)))
    return PME_EINVAL;
  if (n == 0) return PME_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_mlp_jvp_forward, dim3((n + kAtomsD - 1) / kAtomsD), dim3(kMlpThreads), 0,
                     s, n, params, feat, vec, feat_dot, vec_dot, mu, mu_dot);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_backward_jvp(dip_plan_t plan, void* stream, int32_t n, const float* params,
                     const float* qparams, const float* feat, const float* vec,
                     const float* feat_dot, const float* vec_dot, const float* g_mu0,
                     const float* g_mu1, const float* u, const float* g_q0, const float* g_q1,
                     const float* c, float* g_params, float* g_qparams) {
  if (!plan || n < 0 || n > plan->desc.max_atoms || (!g_params && !g_qparams) ||
      (g_params && !params) || (g_qparams && !qparams) || (n > 0 && (!feat || !vec)))
    return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (g_params) {
    const int nb = grad_blocks(n, kAtomsD);
    if (n > 0)
      hipLaunchKernelGGL(k_mlp_jvp_backward, dim3(nb), dim3(kMlpThreads), 0, s, n, params, feat,
                         vec, feat_dot, vec_dot, g_mu0, g_mu1, u, plan->dpart);
    hipLaunchKernelGGL(k_rows_reduce, dim3((NP + 255) / 256), dim3(256), 0, s, n > 0 ? nb : 0,
                       NP, plan->dpart, g_params);
  }
  if (g_qparams) {
    const int nb = grad_blocks(n, kAtoms);
    if (n > 0) {
      hipLaunchKernelGGL(k_means, dim3(1), dim3(1024), 0, s, n, g_q0, g_q1, c, plan->means);
      hipLaunchKernelGGL(k_qhead_backward, dim3(nb), dim3(kMlpThreads), 0, s, n, qparams, feat,
                         feat_dot, g_q0, g_q1, c, plan->means, plan->qpart);
    }
    hipLaunchKernelGGL(k_rows_reduce, dim3((NQP + 255) / 256), dim3(256), 0, s, n > 0 ? nb : 0,
                       NQP, plan->qpart, g_qparams);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_loss(dip_plan_t plan, void* stream, int32_t n, const double* U_s, const double* U_t,
             const float* dUdr_s, const float* dUdr_t, const float* mu, const float* mu_t,
             const float* dUdmu_s, const float* dUdq_s, double lE, double lF, double lmu,
             double* loss, float* v_pos, float* g_mu, float* g_q) {
  if (!plan || n < 0 || n > plan->desc.max_atoms || !U_s || !U_t || !loss ||
      (n > 0 && (!dUdr_s || !dUdr_t || !mu || !dUdmu_s || !v_pos || !g_mu)) ||
      (lmu != 0.0 && !mu_t) || (!g_q != !dUdq_s))
    return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(1024), 0, s, n, U_s, U_t, dUdr_s, dUdr_t, mu, mu_t,
                     dUdmu_s, dUdq_s, lE, lF, lmu, loss, v_pos, g_mu, g_q);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_adam(void* stream, int32_t count, int32_t t, double lr, double beta1, double beta2,
             double eps, float* params, const float* grad, float* m, float* v) {
  if (count < 0 || t < 1 || !params || !grad || !m || !v) return PME_EINVAL;
  if (count == 0) return PME_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const float c1 = float(1.0 - pow(beta1, double(t))), c2 = float(1.0 - pow(beta2, double(t)));
  hipLaunchKernelGGL(k_adam, dim3((count + 255) / 256), dim3(256), 0, s, count, float(lr),
                     float(beta1), float(beta2), float(eps), c1, c2, params, grad, m, v);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

}  // extern "C"
