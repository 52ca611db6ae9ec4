// Shared device-side definitions of the PME kernels (gfx950).
//
// * B-spline assignment weights (Sec. 2.3.2, Eq. w3d): W^(p) is the centered
//   cardinal B-spline M_p(t) = N_p(t + p/2), N_p the cardinal B-spline on
//   [0, p].  On each unit interval N_p is a polynomial; its pieces follow from
//   the recursion N_p(s) = [s N_{p-1}(s) + (p - s) N_{p-1}(s - 1)] / (p - 1),
//   evaluated here at compile time into per-piece coefficient tables, with the
//   derivative tables folded in (coefficient * k!/(k-d)!).
// * Stencil convention: for an atom at mesh coordinate x the anchor is
//   b = floor(x) (even p) or floor(x + 1/2) (odd p, the round() of the paper),
//   f = x + delta - b in [0, 1), and stencil point j = 0..p-1 sits at mesh
//   index b - floor((p-1)/2) + j with weight N_p(f + p - 1 - j), i.e. the
//   polynomial piece p-1-j evaluated at f.
// * Cell geometry (Sec. 2.3.1) is recomputed in FP64 from the device box in
//   every kernel, so a captured graph can be replayed with a new box.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PME_MAX_ORDER 7

namespace pme {

// ---------------------------------------------------------------------------
// compile-time spline tables
// ---------------------------------------------------------------------------
struct SplineTables {
  // coef[off(p) + (d*p + piece)*p + k]: k-th coefficient of the d-th derivative
  // of piece `piece` of N_p, as a polynomial in f (powers f^(k-d), k >= d).
  float coef[4 * (1 + 4 + 9 + 16 + 25 + 36 + 49)];
};

constexpr int spline_offset(int p) {
  int off = 0;
  for (int q = 1; q < p; ++q) off += 4 * q * q;
  return off;
}

// (p - 1)!: the tables with `whole` set hold (p - 1)! N_p, whose coefficients are
// integers (exact in float).
constexpr int spline_norm(int p) {
  int f = 1;
  for (int k = 2; k < p; ++k) f *= k;
  return f;
}

constexpr SplineTables make_spline_tables(bool whole = false) {
  SplineTables t{};
  double a[PME_MAX_ORDER][PME_MAX_ORDER] = {};   // pieces of N_p, a[piece][power]
  double b[PME_MAX_ORDER][PME_MAX_ORDER] = {};
  a[0][0] = 1.0;                                  // N_1 = 1 on [0, 1)
  for (int p = 1; p <= PME_MAX_ORDER; ++p) {
    if (p > 1) {
      for (int j = 0; j < PME_MAX_ORDER; ++j)
        for (int k = 0; k < PME_MAX_ORDER; ++k) b[j][k] = 0.0;
      for (int j = 0; j < p; ++j) {
        if (j < p - 1)                       // (j + f) * piece j of N_{p-1}
          for (int k = 0; k < p - 1; ++k) {
            b[j][k] += j * a[j][k];
            b[j][k + 1] += a[j][k];
          }
        if (j >= 1)                          // (p - j - f) * piece j-1 of N_{p-1}
          for (int k = 0; k < p - 1; ++k) {
            b[j][k] += (p - j) * a[j - 1][k];
            b[j][k + 1] -= a[j - 1][k];
          }
      }
      for (int j = 0; j < p; ++j)
        for (int k = 0; k < p; ++k) a[j][k] = b[j][k] / (p - 1);
    }
    const int off = spline_offset(p);
    for (int d = 0; d < 4; ++d)
      for (int pc = 0; pc < p; ++pc)
        for (int k = 0; k < p; ++k) {
          double fall = 1.0;
          for (int m = 0; m < d; ++m) fall *= (k - m);
          double v = (k >= d) ? a[pc][k] * fall : 0.0;
          if (whole) {
            // an integer up to rounding in the recursion: take the nearest one
            v *= spline_norm(p);
            v = double(static_cast<long long>(v + (v >= 0.0 ? 0.5 : -0.5)));
          }
          t.coef[off + (d * p + pc) * p + k] = float(v);
        }
  }
  return t;
}

static __constant__ SplineTables c_spline = make_spline_tables();
// (p - 1)! times the same: the spread accumulates with these, whose coefficients
// are exact, and divides the sums by ((p - 1)!)^3 in double precision.  The rounded
// coefficients of c_spline make the weights of a stencil sum to 1 + O(2e-8) on
// average (a bias, not noise), which would scale the density and the k-space
// energy of Eq. energy_recip alike.
static __constant__ SplineTables c_spline_whole = make_spline_tables(true);

// w[d][j], d = 0..D: d-th derivative (w.r.t. the mesh coordinate) of the weight of
// stencil point j.
template <int P, int D>
__device__ __forceinline__ void spline_weights(float f, float (&w)[D + 1][P]) {
  constexpr int off = spline_offset(P);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int pc = P - 1 - j;
#pragma unroll
    for (int d = 0; d <= D; ++d) {
      if (d > P - 1) {
        w[d][j] = 0.0f;
        continue;
      }
      const float* c = &c_spline.coef[off + (d * P + pc) * P];
      float acc = c[P - 1];
#pragma unroll
      for (int k = P - 2; k >= d; --k) acc = fmaf(acc, f, c[k]);
      w[d][j] = acc;
    }
  }
}

// spline_weights times (p - 1)! from the integer tables.
template <int P, int D>
__device__ __forceinline__ void spline_weights_whole(float f, float (&w)[D + 1][P]) {
  constexpr int off = spline_offset(P);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int pc = P - 1 - j;
#pragma unroll
    for (int d = 0; d <= D; ++d) {
      if (d > P - 1) {
        w[d][j] = 0.0f;
        continue;
      }
      const float* c = &c_spline_whole.coef[off + (d * P + pc) * P];
      float acc = c[P - 1];
#pragma unroll
      for (int k = P - 2; k >= d; --k) acc = fmaf(acc, f, c[k]);
      w[d][j] = acc;
    }
  }
}

// Weights of one stencil point j (runtime, wave-uniform) for derivative orders 0..D.
template <int P, int D>
__device__ __forceinline__ void spline_weight_at(int j, float f, float (&w)[D + 1]) {
  constexpr int off = spline_offset(P);
  const int pc = P - 1 - j;
#pragma unroll
  for (int d = 0; d <= D; ++d) {
    if (d > P - 1) {
      w[d] = 0.0f;
      continue;
    }
    const float* c = &c_spline.coef[off + (d * P + pc) * P];
    float acc = c[P - 1];
#pragma unroll
    for (int k = P - 2; k >= d; --k) acc = fmaf(acc, f, c[k]);
    w[d] = acc;
  }
}

// A value the caller knows to be the same in every lane, moved to a scalar register.
__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// ---------------------------------------------------------------------------
// cell geometry
// ---------------------------------------------------------------------------
struct Cell {
  double inv[9];   // C^-1, row-major: inv[3*b + a] = (C^-1)[b][a]
  double vol;      // |det C|
  bool ok;         // finite and non-singular
};

__device__ __forceinline__ Cell cell_from_box(const double* __restrict__ box) {
  Cell c;
  const double a00 = box[0], a01 = box[1], a02 = box[2];
  const double a10 = box[3], a11 = box[4], a12 = box[5];
  const double a20 = box[6], a21 = box[7], a22 = box[8];
  const double c00 = a11 * a22 - a12 * a21, c01 = a02 * a21 - a01 * a22, c02 = a01 * a12 - a02 * a11;
  const double c10 = a12 * a20 - a10 * a22, c11 = a00 * a22 - a02 * a20, c12 = a02 * a10 - a00 * a12;
  const double c20 = a10 * a21 - a11 * a20, c21 = a01 * a20 - a00 * a21, c22 = a00 * a11 - a01 * a10;
  const double det = a00 * c00 + a01 * c10 + a02 * c20;
  c.ok = isfinite(det) && det != 0.0;
  const double id = c.ok ? 1.0 / det : 0.0;
  c.inv[0] = c00 * id; c.inv[1] = c01 * id; c.inv[2] = c02 * id;
  c.inv[3] = c10 * id; c.inv[4] = c11 * id; c.inv[5] = c12 * id;
  c.inv[6] = c20 * id; c.inv[7] = c21 * id; c.inv[8] = c22 * id;
  c.vol = fabs(det);
  return c;
}

// J[a][b] = d x_a / d r_b = N_a (C^-1)[b][a]  (float, row-major)
__device__ __forceinline__ void jacobian(const Cell& c, const int (&N)[3], float (&J)[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) J[a][b] = float(N[a] * c.inv[3 * b + a]);
}

// Stencil anchor and offset of one atom along the three axes.  Returns false for a
// non-finite position.  base[a] in [0, N_a), f[a] in [0, 1).
template <int P>
__device__ __forceinline__ bool atom_stencil(float3 r, const Cell& c, const int (&N)[3],
                                             int (&base)[3], float (&f)[3]) {
  const double r0 = r.x, r1 = r.y, r2 = r.z;
  bool ok = isfinite(r0) && isfinite(r1) && isfinite(r2) && c.ok;
  constexpr double delta = (P & 1) ? 0.5 : 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double s = r0 * c.inv[a] + r1 * c.inv[3 + a] + r2 * c.inv[6 + a];
    s -= floor(s);
    double x = s * N[a] + delta;
    double fb = floor(x);
    int b = ok ? int(fb) : 0;
    float fr = ok ? float(x - fb) : 0.0f;
    if (fr >= 1.0f) { fr = 0.0f; b += 1; }
    if (b >= N[a]) b -= N[a];
    if (b < 0) b += N[a];
    if (b < 0 || b >= N[a]) { b = 0; ok = false; }
    base[a] = b;
    f[a] = fr;
  }
  return ok;
}

// d = J v  (x-space components of a Cartesian vector)
__device__ __forceinline__ float3 jmul(const float (&J)[3][3], float3 v) {
  return make_float3(J[0][0] * v.x + J[0][1] * v.y + J[0][2] * v.z,
                     J[1][0] * v.x + J[1][1] * v.y + J[1][2] * v.z,
                     J[2][0] * v.x + J[2][1] * v.y + J[2][2] * v.z);
}

// Coefficients of the tangent density of the Hessian-vector product:
// rho_dot = v_q W + w.grad_x W + d^T (grad_x grad_x W) v with d = J mu,
// v = J v_r, w = J (v_mu + q v_r); monomials 000, 100, 010, 001, 200, 020, 002,
// 110, 101, 011.
__device__ __forceinline__ void tangent_coeffs(const float (&J)[3][3], float q, float3 mu, float vq,
                                               float3 vr, float3 vm, float (&co)[10]) {
  const float3 d = jmul(J, mu);
  const float3 w = jmul(J, make_float3(vm.x + q * vr.x, vm.y + q * vr.y, vm.z + q * vr.z));
  const float3 v = jmul(J, vr);
  co[0] = vq;
  co[1] = w.x; co[2] = w.y; co[3] = w.z;
  co[4] = d.x * v.x; co[5] = d.y * v.y; co[6] = d.z * v.z;
  co[7] = d.x * v.y + d.y * v.x;
  co[8] = d.x * v.z + d.z * v.x;
  co[9] = d.y * v.z + d.z * v.y;
}

// A contribution of magnitude below 2^31 as a 64-bit fixed-point word: rounded to
// the nearest 32-bit integer, ties up (floor(v + 1/2), one conversion instruction)
// and sign-extended.  The rounding moves a contribution by at most half a unit,
// 2^-31 of the largest possible one, with no bias but at exact ties.
__device__ __forceinline__ unsigned long long to_fixed(float v) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
  return (unsigned long long)(long long)r;
}

// A 64-bit fixed-point sum as a float: hi * 2^32 + lo in double precision (exact
// below 2^53), scaled by inv_scale and rounded once to float.
__device__ __forceinline__ float from_fixed(long long v, double inv_scale) {
  const double vd = fma(double(int(v >> 32)), 4294967296.0, double(uint32_t(v)));
  return float(vd * inv_scale);
}

// Weights of stencil point j (lane-dependent) for derivative orders 0..D, from an LDS
// copy of the coefficients of N_P (or of its whole-number table); the same Horner
// steps as spline_weights, so the values are the same bit for bit (an indexed
// constant table would be hoisted into registers for the whole kernel).
template <int P, int D>
__device__ __forceinline__ void weight_at_lds(const float* tab, int j, float f, float (&w)[D + 1]) {
  const int pc = P - 1 - j;
#pragma unroll
  for (int d = 0; d <= D; ++d) {
    if (d > P - 1) {
      w[d] = 0.0f;
      continue;
    }
    const float* c = &tab[(d * P + pc) * P];
    float acc = c[P - 1];
#pragma unroll
    for (int k = P - 2; k >= d; --k) acc = fmaf(acc, f, c[k]);
    w[d] = acc;
  }
}

// m mod N in [0, N) for any int m
__device__ __forceinline__ int wrapn(int m, int N) {
  m %= N;
  return (m < 0) ? m + N : m;
}

// Stream compaction within a wavefront: every lane calls it; lanes with pred get
// consecutive slots of *counter (one LDS atomic per wavefront), others get -1.
__device__ __forceinline__ int wave_compact(bool pred, int* counter) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return -1;
  const int leader = __ffsll((long long)m) - 1;
  // set lanes below this one (mbcnt: no per-lane mask register)
  const int below = int(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
  int base = 0;
  if (int(threadIdx.x & 63) == leader) base = atomicAdd(counter, __popcll(m));
  base = __builtin_amdgcn_readlane(base, leader);
  return pred ? base + below : -1;
}

// Work item of workgroup b of a G-workgroup launch, chosen so that the workgroups
// one XCD receives take a contiguous range of items.  The GPU hands workgroups to
// its 8 XCDs in turn (b mod 8), and each XCD has its own L2: with tiles numbered
// along the mesh, a contiguous range is a compact block of neighbouring tiles whose
// halos and records that XCD's L2 then serves.  A bijection of [0, G).
__device__ __forceinline__ int xcd_item(int b, int G) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, per = G / kXcd, rem = G % kXcd;
  return x * per + min(x, rem) + b / kXcd;
}

// block-wide sum of a double (blockDim.x a multiple of 64, at most 1024)
__device__ __forceinline__ double block_sum(double v, double* scratch) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < int(blockDim.x >> 6); ++w) s += scratch[w];
  __syncthreads();
  return s;   // valid in thread 0
}

// block-wide sums of K doubles with one pair of barriers (blockDim.x a multiple of
// 64, at most 1024; scratch holds 16 K doubles); the sums land in v of thread 0
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_down(v[k], o, 64);
    if (lane == 0) scratch[wid * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < int(blockDim.x >> 6); ++w) s += scratch[w * K + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

}  // namespace pme
