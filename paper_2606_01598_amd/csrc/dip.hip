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
    a.g_pos[3 * i] = gx;
    a.g_pos[3 * i + 1] = gy;
    a.g_pos[3 * i + 2] = gz;
  }
}

__global__ void k_param_reduce(int nb, const float* part, float* g) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  float s = 0.0f;
  for (int b = 0; b < nb; ++b) s += part[size_t(b) * NP + p];
  g[p] = s;
}

__global__ void __launch_bounds__(1024) k_loss(int n, const double* Us, const double* Ut,
                                               const float* ds, const float* dt, const float* mu,
                                               const float* mut, const float* dmu, double lE,
                                               double lF, double lmu, double* loss, float* vpos,
                                               float* gmu) {
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

struct dip_plan_s {
  dip_desc_t desc;
  CellList cells;
  float* part = nullptr;     // [mlp blocks][NP]
  float* fbar = nullptr;     // [max_atoms][64] feature cotangents (position VJP)
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
  if (rc != PME_OK || e != hipSuccess) {
    free_cells(pl->cells);
    if (pl->part) (void)hipFree(pl->part);
    if (pl->fbar) (void)hipFree(pl->fbar);
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
  if (plan->part) (void)hipFree(plan->part);
  if (plan->fbar) (void)hipFree(plan->fbar);
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
  hipLaunchKernelGGL(k_param_reduce, dim3((NP + 255) / 256), dim3(256), 0, s, nb, plan->part,
                     g_params);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_position_vjp(dip_plan_t plan, void* stream, int32_t n, const float* params,
                     const float* pos, const float* q, const float* feat, const float* vec,
                     const float* u, float* g_pos) {
  if (!plan || n < 0 || n > plan->desc.max_atoms ||
      (n > 0 && (!params || !pos || !q || !feat || !vec || !u || !g_pos)))
    return PME_EINVAL;
  if (n == 0) return PME_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = build_cells(plan->cells, s, n, pos);
  if (e != hipSuccess) return dip_fail(e);
  hipLaunchKernelGGL(k_mlp_input_grad, dim3(mlp_blocks(n)), dim3(kMlpThreads), 0, s, n, params,
                     feat, vec, u, plan->fbar);
  VjpArgs a;
  a.n = n; a.pos = pos; a.q = q; a.g = plan->cells.g;
  a.start = plan->cells.start; a.sorted = plan->cells.sorted;
  a.rc = float(plan->desc.cutoff); a.fbar = plan->fbar; a.g_pos = g_pos;
  const int per = kFeatThreads / kLanes;
  hipLaunchKernelGGL(k_features_vjp, dim3((n + per - 1) / per), dim3(kFeatThreads), 0, s, a);
  e = hipGetLastError();
  return e == hipSuccess ? PME_OK : dip_fail(e);
}

int dip_loss(dip_plan_t plan, void* stream, int32_t n, const double* U_s, const double* U_t,
             const float* dUdr_s, const float* dUdr_t, const float* mu, const float* mu_t,
             const float* dUdmu_s, double lE, double lF, double lmu, double* loss, float* v_pos,
             float* g_mu) {
  if (!plan || n < 0 || n > plan->desc.max_atoms || !U_s || !U_t || !loss ||
      (n > 0 && (!dUdr_s || !dUdr_t || !mu || !dUdmu_s || !v_pos || !g_mu)) ||
      (lmu != 0.0 && !mu_t))
    return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(1024), 0, s, n, U_s, U_t, dUdr_s, dUdr_t, mu, mu_t,
                     dUdmu_s, lE, lF, lmu, loss, v_pos, g_mu);
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
