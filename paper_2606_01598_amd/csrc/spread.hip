// Charge + dipole assignment onto the mesh (Sec. 2.3.2, Eq. charge_dipole_assign)
// and the tangent density of the Hessian-vector product.
//
// Two kernels:
//  * k_bin: one thread per atom computes its fractional coordinates, stencil
//    anchor b and offset f (Sec. 2.3.2), and the monomial coefficients of what it
//    assigns, c_abc, such that the value it adds at stencil point (i, j, k) is
//        sum_abc c_abc W_x^(a)[i] W_y^(b)[j] W_z^(c)[k]
//    (forward: c_000 = q, c_100..c_001 = N_a (mu . C^-1[:,a]); tangent and the
//    quadrupole forward: degree <= 2).
//    It files a 16-word record into a fixed-capacity bin of B_x x B_y x B_z anchors
//    (overflow goes to a list), reduces the largest coefficient sum (the fixed-point
//    scale of the spread) and, for the forward, block partial sums of q^2 and |mu|^2
//    for the self terms (Eqs. self_q, self_mu).  It also clears the other counter set.
//  * k_spread: one workgroup owns one mesh tile.  It enumerates the occupied record
//    slots of the bins whose anchors can reach the tile, stages the overlapping
//    atoms' weights in LDS, accumulates their contributions into an LDS tile in
//    64-bit fixed point with integer LDS adds (exact and order independent; LDS
//    float atomics are slow on gfx950), and writes the tile back with plain
//    coalesced stores.  Halo contributions are computed by every tile they touch
//    instead of being flushed with global atomics, so the mesh needs no clearing
//    and no global read-modify-write.
//
// Record layout (16 words): f_x f_y f_z anchor | forward: q d_x d_y d_z, tangent: q mu |
// forward: mu -, tangent: v_q v_r | forward: s (= r C^-1, unwrapped) atom, tangent: v_mu atom.
// Quadrupole forward: f anchor | q d | c_200 c_020 c_002 c_110 | c_101 c_011 - atom, the
// second-order coefficients those of (1/2) Q : grad_x grad_x W with Q = J Theta J^T.
#include <vector>

#include "kernels.h"
#include "pme_common.h"

namespace pme {
namespace {

struct BinArgs {
  int n;
  const float* pos;
  const float* q;
  const float* mu;
  const double* box;
  const float* v_pos;
  const float* v_q;
  const float* v_mu;
  const float* theta;  // quadrupole forward: second moments (xx yy zz xy xz yz)
  int N[3];
  int B[3];
  int nb[3];
  int cap;
  int* count;          // this binning's counters
  int* ovf_count;
  unsigned* cmax;
  int* count_other;    // the other set, cleared here
  int* ovf_other;
  unsigned* cmax_other;
  // tangent binning of a concurrent step: also the largest forward coefficient sum
  // |q| + |J mu|_1 (the forward plane spread reads these records), and its other set
  unsigned* cmax_fwd;
  unsigned* cmax_fwd_other;
  int nbins;
  float* rec;
  long long ovf_base;      // record index of the overflow list
  double* spart;
  double* spart_th;    // quadrupole forward: block sums of q tr(Theta), tr^2 + 2 Theta:Theta
  int* status;
  int nblk;            // workgroups of this binning (bin_blocks(n))
  int off;             // batches: offset of the box's atoms in the packed arrays
};

__device__ __forceinline__ float3 ld3(const float* p, int i) {
  return p ? make_float3(p[3 * i], p[3 * i + 1], p[3 * i + 2]) : make_float3(0.f, 0.f, 0.f);
}

// Second-order coefficients of the quadrupole density (1/2) Q : grad_x grad_x W,
// Q = J Theta J^T: monomials 200, 020, 002 take Q_aa / 2, 110, 101, 011 take Q_ab.
__device__ __forceinline__ void quad_coeffs(const float (&J)[3][3], const float (&th)[6],
                                            float* co) {
  const float T[3][3] = {{th[0], th[3], th[4]}, {th[3], th[1], th[5]}, {th[4], th[5], th[2]}};
  float JT[3][3];   // J Theta
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) JT[a][b] = J[a][0] * T[0][b] + J[a][1] * T[1][b] + J[a][2] * T[2][b];
  auto Q = [&](int a, int b) { return JT[a][0] * J[b][0] + JT[a][1] * J[b][1] + JT[a][2] * J[b][2]; };
  co[0] = 0.5f * Q(0, 0); co[1] = 0.5f * Q(1, 1); co[2] = 0.5f * Q(2, 2);
  co[3] = Q(0, 1); co[4] = Q(0, 2); co[5] = Q(1, 2);
}

template <int P, bool TANGENT, bool QUAD = false>
__device__ __forceinline__ void bin_body(const BinArgs& a, const int blk) {
  __shared__ double red[8];
  __shared__ unsigned s_wmax[8];
  const int i = blk * 256 + threadIdx.x;
  const bool live = i < a.n;
  // every per-atom input is loaded first, so that their latencies overlap with
  // each other and with the cell algebra
  const float3 zero3 = make_float3(0.f, 0.f, 0.f);
  const float3 r = live ? ld3(a.pos, i) : zero3;
  const float q = (live && a.q) ? a.q[i] : 0.0f;
  const float3 mu = live ? ld3(a.mu, i) : zero3;
  float vq = 0.0f;
  float3 vr = zero3, vm = zero3;
  if (TANGENT && live) {
    vq = a.v_q ? a.v_q[i] : 0.0f;
    vr = ld3(a.v_pos, i);
    vm = ld3(a.v_mu, i);
  }
  float th[6] = {0, 0, 0, 0, 0, 0};
  if (QUAD && live && a.theta) {
#pragma unroll
    for (int k = 0; k < 6; ++k) th[k] = a.theta[6 * i + k];
  }
  const Cell c = cell_from_box(a.box);
  double sq = 0.0, smu = 0.0, sqt = 0.0, stt = 0.0;
  float amax = 0.0f, fmax = 0.0f;
  if (live) {
    int base[3];
    float f[3];
    const bool ok = atom_stencil<P>(r, c, a.N, base, f);
    sq = double(q) * q;
    smu = double(mu.x) * mu.x + double(mu.y) * mu.y + double(mu.z) * mu.z;
    if (QUAD && a.theta) {
      const double tr = double(th[0]) + th[1] + th[2];
      sqt = double(q) * tr;
      stt = tr * tr + 2.0 * (double(th[0]) * th[0] + double(th[1]) * th[1] + double(th[2]) * th[2]) +
            4.0 * (double(th[3]) * th[3] + double(th[4]) * th[4] + double(th[5]) * th[5]);
    }
    if (!ok) {
      atomicOr(a.status, 1);
    } else {
      // the slot is reserved first: the coefficients are formed while it returns
      const int bin = ((base[0] / a.B[0]) * a.nb[1] + base[1] / a.B[1]) * a.nb[2] + base[2] / a.B[2];
      const int slot = atomicAdd(&a.count[bin], 1);
      float J[3][3];
      jacobian(c, a.N, J);
      const float3 d = jmul(J, mu);
      float co[10];
      if (!TANGENT) {
        co[0] = q; co[1] = d.x; co[2] = d.y; co[3] = d.z;
        if (QUAD) quad_coeffs(J, th, co + 4);
      } else {
        tangent_coeffs(J, q, mu, vq, vr, vm, co);
      }
      constexpr int nc = (TANGENT || QUAD) ? 10 : 4;
#pragma unroll
      for (int k = 0; k < nc; ++k) amax += fabsf(co[k]);
      if (!isfinite(amax)) {
        atomicOr(a.status, 1);
        amax = 0.0f;
      }
      if (TANGENT && a.cmax_fwd) {
        // the forward binning's sum of the same atom (q, J mu)
        const float c4[4] = {q, d.x, d.y, d.z};
#pragma unroll
        for (int k = 0; k < 4; ++k) fmax += fabsf(c4[k]);
        if (!isfinite(fmax)) fmax = 0.0f;
      }
      // every atom takes one slot of its bin or of the overflow list (which holds
      // max_atoms records)
      const size_t ri = (slot < a.cap) ? size_t(bin) * a.cap + slot
                                       : size_t(a.ovf_base) + atomicAdd(a.ovf_count, 1);
      float4* d4 = reinterpret_cast<float4*>(a.rec + ri * kRecWords);
      d4[0] = make_float4(f[0], f[1], f[2],
                          __int_as_float(base[0] | (base[1] << 10) | (base[2] << 20)));
      if (TANGENT) {
        // the raw inputs: the spread rebuilds the coefficients, and the gather of the
        // Hessian-vector product needs no per-atom loads of its own
        d4[1] = make_float4(q, mu.x, mu.y, mu.z);
        d4[2] = make_float4(vq, vr.x, vr.y, vr.z);
        d4[3] = make_float4(vm.x, vm.y, vm.z, __int_as_float(i));
      } else if (QUAD) {
        d4[1] = make_float4(co[0], co[1], co[2], co[3]);
        d4[2] = make_float4(co[4], co[5], co[6], co[7]);
        d4[3] = make_float4(co[8], co[9], 0.0f, __int_as_float(i));
      } else {
        // and the unwrapped fractional position r C^-1 (its image matters to the
        // cell gradient, which the forward gather forms when asked)
        const double r0 = r.x, r1 = r.y, r2 = r.z;
        float sf[3];
#pragma unroll
        for (int b = 0; b < 3; ++b)
          sf[b] = float(r0 * c.inv[b] + r1 * c.inv[3 + b] + r2 * c.inv[6 + b]);
        d4[1] = make_float4(co[0], co[1], co[2], co[3]);
        d4[2] = make_float4(mu.x, mu.y, mu.z, 0.f);
        d4[3] = make_float4(sf[0], sf[1], sf[2], __int_as_float(i));
      }
    }
  }
  // clear the other counter set for the next binning
  for (int e = blk * 256 + threadIdx.x; e < a.nbins; e += a.nblk * 256) a.count_other[e] = 0;
  if (blk == 0 && threadIdx.x == 0) {
    *a.ovf_other = 0;
    *a.cmax_other = 0u;
    if (TANGENT && a.cmax_fwd_other) *a.cmax_fwd_other = 0u;
  }
  // the largest coefficient sum: wavefront maxima, then the workgroup's (the sums
  // are non-negative, so their float bits order as unsigned integers)
  unsigned um = __float_as_uint(amax);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) um = max(um, unsigned(__shfl_xor(int(um), o, 64)));
  if ((threadIdx.x & 63) == 0) s_wmax[threadIdx.x >> 6] = um;
  if (TANGENT && a.cmax_fwd) {
    unsigned uf = __float_as_uint(fmax);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) uf = max(uf, unsigned(__shfl_xor(int(uf), o, 64)));
    if ((threadIdx.x & 63) == 0) s_wmax[4 + (threadIdx.x >> 6)] = uf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned m = max(max(s_wmax[0], s_wmax[1]), max(s_wmax[2], s_wmax[3]));
    if (m) atomicMax(a.cmax, m);
    if (TANGENT && a.cmax_fwd) {
      const unsigned mf = max(max(s_wmax[4], s_wmax[5]), max(s_wmax[6], s_wmax[7]));
      if (mf) atomicMax(a.cmax_fwd, mf);
    }
  }
  if (a.spart) {
    const double s1 = block_sum(sq, red);
    const double s2 = block_sum(smu, red);
    if (threadIdx.x == 0) {
      a.spart[2 * blk] = s1;
      a.spart[2 * blk + 1] = s2;
    }
    if (QUAD && a.spart_th) {
      const double s3 = block_sum(sqt, red);
      const double s4 = block_sum(stt, red);
      if (threadIdx.x == 0) {
        a.spart_th[2 * blk] = s3;
        a.spart_th[2 * blk + 1] = s4;
      }
    }
  }
}

template <int P, bool TANGENT, bool QUAD = false>
__global__ void __launch_bounds__(256) k_bin(BinArgs a) {
  bin_body<P, TANGENT, QUAD>(a, blockIdx.x);
}

// Batched binning: work item (box, workgroup of the box), per-box argument
// templates in device memory completed with the call's packed arrays; workgroups
// loop over the items.
template <int P, bool TANGENT>
__global__ void __launch_bounds__(256) k_bin_batch(const BinArgs* args, const int2* items,
                                                   int nitems, BatchIO io, int self_sums) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    BinArgs a = args[w.x];
    const int o = a.off;
    a.pos = io.pos + 3 * size_t(o);
    a.q = io.q ? io.q + o : nullptr;
    a.mu = io.mu ? io.mu + 3 * size_t(o) : nullptr;
    a.box = io.box + 9 * w.x;
    a.v_pos = io.v_pos ? io.v_pos + 3 * size_t(o) : nullptr;
    a.v_q = io.v_q ? io.v_q + o : nullptr;
    a.v_mu = io.v_mu ? io.v_mu + 3 * size_t(o) : nullptr;
    if (!self_sums) a.spart = nullptr;
    bin_body<P, TANGENT>(a, w.y);
    __syncthreads();
  }
}

struct ClearItem {
  int* count;
  int nbins;
  int* ovf_count;
  unsigned* cmax;
};

// one workgroup per box: zero counter set 0
__global__ void __launch_bounds__(256) k_clear_batch(const ClearItem* items, int nbox) {
  for (int b = blockIdx.x; b < nbox; b += gridDim.x) {
    const ClearItem c = items[b];
    for (int e = threadIdx.x; e < c.nbins; e += 256) c.count[e] = 0;
    if (threadIdx.x == 0) {
      *c.ovf_count = 0;
      *c.cmax = 0u;
    }
  }
}

struct SpreadArgs {
  int N[3];
  int B[3];
  int nb[3];
  int cap;
  int ch;                  // records staged per round (<= 256)
  int nbr_max;             // largest scanned bin range of a tile
  int tile_words;          // largest padded tile T_x T_y (T_z + 1)
  const int* count;
  const int* ovf_count;
  const unsigned* cmax;
  const float* rec;
  long long ovf_base;      // record index of the overflow list
  int T[3];
  int nt[3];
  int rel;                 // 1: N[a] >= T[a] + p - 1 on every axis (tile-relative offsets)
  float* rho;
};

// m mod N for m in [-N, 2N)
__device__ __forceinline__ int wrap1(int m, int N) {
  return (m < 0) ? m + N : ((m >= N) ? m - N : m);
}

// Does the stencil of an atom anchored at b reach the tile [t0, t0+T) along one axis?
template <int P>
__device__ __forceinline__ bool axis_hits(int b, int t0, int T, int N) {
  constexpr int lo = (P - 1) / 2;
  if (N < P) return true;                       // the stencil covers every residue
  const int m0 = b - lo, m1 = m0 + P - 1;
  const int e = t0 + T;
  return (m1 >= t0 && m0 < e) || (m1 - N >= t0 && m0 - N < e) || (m1 + N >= t0 && m0 + N < e);
}

// Tile-local coordinate of each stencil point (-1 outside the tile), packed as bytes.
template <int P>
__device__ __forceinline__ void axis_locs(int b, int t0, int T, int N, int& w0, int& w1) {
  constexpr int lo = (P - 1) / 2;
  uint32_t p0 = 0, p1 = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int m = (N >= P) ? wrap1(b - lo + j, N) : wrapn(b - lo + j, N);
    const int l = m - t0;
    const uint32_t byte = (l >= 0 && l < T) ? uint32_t(l) : 0xffu;
    if (j < 4) p0 |= byte << (8 * j); else p1 |= byte << (8 * (j - 4));
  }
  w0 = int(p0);
  w1 = int(p1);
}

// Tile-relative position of an atom's first stencil point along one axis, wrapped
// into [-(P-1), N-(P-1)): stencil point j lies in the tile [t0, t0+T) iff
// 0 <= d + j < T.  Exact when N >= T + P - 1 (no other periodic image of the
// stencil reaches the tile); the stencil reaches the tile iff d < T.
template <int P>
__device__ __forceinline__ int axis_rel(int b, int t0, int N) {
  int d = b - (P - 1) / 2 - t0;
  d += (d < -(P - 1)) ? N : 0;
  d -= (d >= N - (P - 1)) ? N : 0;
  return d;
}

// axis_locs from the tile-relative position d (same packed bytes)
template <int P>
__device__ __forceinline__ void rel_locs(int d, int T, int& w0, int& w1) {
  uint32_t p0 = 0, p1 = 0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int l = d + j;
    const uint32_t byte = (uint32_t(l) < uint32_t(T)) ? uint32_t(l) : 0xffu;
    if (j < 4) p0 |= byte << (8 * j); else p1 |= byte << (8 * (j - 4));
  }
  w0 = int(p0);
  w1 = int(p1);
}

__device__ __forceinline__ int loc_of(int w0, int w1, int j) {
  const int w = (j < 4) ? w0 : w1;
  return int(int8_t((w >> (8 * (j & 3))) & 0xff));
}

template <int P, int DEG>
__device__ __forceinline__ void spread_body(const SpreadArgs& a, const int tile_id,
                                            const double* box) {
  // DEG 1: forward (q, mu); 2: tangent density; 3: quadrupole forward (the
  // coefficients of degree <= 2 come with the record)
  constexpr int NC = (DEG == 1) ? 4 : 10;
  constexpr int D = (DEG == 1) ? 1 : 2;       // highest weight derivative needed
  constexpr int NW = 3 * (D + 1) * P;         // weights w[axis][d][j]
  constexpr int ES = spread_entry_words(P, D);
  constexpr int lo = (P - 1) / 2;
  const int CH = a.ch;                        // records staged per round
  // dynamic LDS, sized by the host (spread_lds_bytes): the fixed-point tile, the
  // scanned bin range, the staged entries and the task list
  extern __shared__ unsigned long long s_dyn[];
  unsigned long long* s_tile = s_dyn;
  int* s_off = reinterpret_cast<int*>(s_tile + a.tile_words);
  int* s_bin = s_off + a.nbr_max + 2;
  uint16_t* s_map = reinterpret_cast<uint16_t*>(s_bin + a.nbr_max + 2);
  float* s_ent = reinterpret_cast<float*>(s_map + kSpreadMap);
  uint16_t* s_task = reinterpret_cast<uint16_t*>(s_ent + CH * ES);
  __shared__ int s_nr[2], s_ntask;

  const int tid = threadIdx.x;
  // tangent records: the Jacobian rebuilds their coefficients at staging; it is
  // kept in LDS, where it takes no registers across the accumulation
  __shared__ float s_J[DEG == 2 ? 9 : 1];
  if (DEG == 2 && tid == 0) {
    float J[3][3];
    jacobian(cell_from_box(box), a.N, J);
#pragma unroll
    for (int i = 0; i < 9; ++i) s_J[i] = J[i / 3][i % 3];
  }
  int t0[3], T[3];
  {
    int t = tile_id;
    const int tz = t % a.nt[2];
    t /= a.nt[2];
    const int ty = t % a.nt[1];
    const int tx = t / a.nt[1];
    const int tc[3] = {tx, ty, tz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      t0[ax] = tc[ax] * a.T[ax];
      T[ax] = min(a.T[ax], a.N[ax] - t0[ax]);
    }
  }
  // bins whose anchors can reach the tile: b in [t0 + lo - P + 1, t0 + T - 1 + lo]
  int kmin[3], nk[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int bmin = t0[ax] + lo - P + 1, bmax = t0[ax] + T[ax] - 1 + lo;
    const int B = a.B[ax];
    const int k0 = (bmin >= 0) ? bmin / B : -((-bmin + B - 1) / B);
    const int k1 = (bmax >= 0) ? bmax / B : -((-bmax + B - 1) / B);
    nk[ax] = k1 - k0 + 1;
    kmin[ax] = k0;
    if (nk[ax] >= a.nb[ax]) { nk[ax] = a.nb[ax]; kmin[ax] = 0; }
  }
  const int nbr = nk[0] * nk[1] * nk[2];      // <= a.nbr_max (host guarantees)
  for (int e = tid; e < nbr; e += 256) {
    const int kz = e % nk[2], ky = (e / nk[2]) % nk[1], kx = e / (nk[1] * nk[2]);
    const int bx = wrapn(kmin[0] + kx, a.nb[0]);
    const int by = wrapn(kmin[1] + ky, a.nb[1]);
    const int bz = wrapn(kmin[2] + kz, a.nb[2]);
    const int bin = (bx * a.nb[1] + by) * a.nb[2] + bz;
    s_bin[e] = bin;
    s_off[e] = min(a.count[bin], a.cap);
  }
  if (tid == 0) {
    s_bin[nbr] = -1;                          // pseudo-bin: the overflow list
    s_off[nbr] = *a.ovf_count;
    s_nr[0] = 0;
    s_ntask = 0;
  }
  // each contribution is bounded by 8 sum_k |c_k| <= 8 cmax with normalised weights;
  // the staged weights are the whole-number ones ((P-1)! times larger per axis), so
  // the bound is 8 cmax ((P-1)!)^3: scale it below 2^31
  constexpr float kWhole3 = float(spline_norm(P)) * float(spline_norm(P)) * float(spline_norm(P));
  float scale = 1.0f;
  {
    const float cm = __uint_as_float(*a.cmax);
    if (cm > 0.0f && isfinite(cm)) scale = ldexpf(1.0f, 31 - (ilogbf(8.0f * cm * kWhole3) + 1));
  }
  const int TZP = T[2] + 1;                   // padded z stride; column T_z is scratch
  const int tpad = T[0] * T[1] * TZP;
  for (int e = tid; e < tpad; e += 256) s_tile[e] = 0ull;
  __syncthreads();
  // exclusive scan of the occupied slot counts (wavefront 0)
  if (tid < 64) {
    const int len = nbr + 1;
    const int seg = (len + 63) / 64;
    const int s0 = min(tid * seg, len), s1 = min(s0 + seg, len);
    int acc = 0;
    for (int e = s0; e < s1; ++e) acc += s_off[e];
    int incl = acc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o, 64);
      if (tid >= o) incl += v;
    }
    int run = incl - acc;
    for (int e = s0; e < s1; ++e) { const int v = s_off[e]; s_off[e] = run; run += v; }
    if (tid == 63) s_off[len] = incl;
  }
  __syncthreads();
  const int total = s_off[nbr + 1];
  const bool mapped = total <= kSpreadMap;
  if (mapped)
    for (int e = tid; e <= nbr; e += 256)
      for (int k = s_off[e]; k < s_off[e + 1]; ++k) s_map[k] = uint16_t(e);
  __syncthreads();

  // record of scanned slot `item`: the bin is the last one whose offset is <= item
  auto fetch = [&](int item, float4& h, float4& c0v, float4& c1v, float4& c2v) {
    int lo_i = 0;
    if (mapped) {
      lo_i = s_map[item];
    } else {
      int hi_i = nbr;
      while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i + 1) >> 1;
        if (s_off[mid] <= item) lo_i = mid; else hi_i = mid - 1;
      }
    }
    const int bin = s_bin[lo_i];
    const int slot = item - s_off[lo_i];
    const size_t ri = (bin >= 0) ? size_t(bin) * a.cap + slot : size_t(a.ovf_base) + slot;
    const float4* r = reinterpret_cast<const float4*>(a.rec + ri * kRecWords);
    h = r[0];
    c0v = r[1];
    if (NC == 10) {
      c1v = r[2];
      const float* f = a.rec + ri * kRecWords;   // v_mu; the atom index is not needed here
      c2v = make_float4(f[12], f[13], f[14], 0.0f);
    }
  };
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 h = z4, c0v = z4, c1v = z4, c2v = z4;
  if (tid < total) fetch(tid, h, c0v, c1v, c2v);

  // rounds of 256 scanned records (one per thread); the hits of a round (about a
  // third of them) are staged and accumulated in sub-rounds of at most CH entries
  // (the hit counter of round r is s_nr[r & 1]; the other one is cleared once every
  // thread has passed the round's first barrier, i.e. has read it in round r - 1)
  for (int r0 = 0, rr = 0; r0 < total; r0 += 256, ++rr) {
    // the next round's record is loaded now and used after this round's
    // accumulation (barriers do not wait for global loads)
    float4 nh = z4, nc0 = z4, nc1 = z4, nc2 = z4;
    if (r0 + 256 + tid < total) fetch(r0 + 256 + tid, nh, nc0, nc1, nc2);
    __syncthreads();
    if (tid == 0) s_nr[(rr + 1) & 1] = 0;
    // 1. keep the records whose stencil reaches the tile; stage their weights,
    //    tile-local coordinates and coefficients, and one task per stencil x-plane
    //    that lies in the tile
    bool hit = false;
    if (r0 + tid < total && a.rel) {
      const int pk = __float_as_int(h.w);
      hit = axis_rel<P>(pk & 1023, t0[0], a.N[0]) < T[0] &&
            axis_rel<P>((pk >> 10) & 1023, t0[1], a.N[1]) < T[1] &&
            axis_rel<P>((pk >> 20) & 1023, t0[2], a.N[2]) < T[2];
    } else if (r0 + tid < total) {
      int lw[3][2];
      const int pk = __float_as_int(h.w);
      const int b[3] = {pk & 1023, (pk >> 10) & 1023, (pk >> 20) & 1023};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) axis_locs<P>(b[ax], t0[ax], T[ax], a.N[ax], lw[ax][0], lw[ax][1]);
      // a byte is 0xff where the stencil point lies outside the tile
      auto any_in = [](int w0, int w1) {
        const uint32_t u0 = uint32_t(w0), u1 = uint32_t(w1) | (P <= 4 ? 0xffffffffu : 0u);
        const uint32_t m0 = (P >= 4) ? 0xffffffffu : ((1u << (8 * P)) - 1u);
        const uint32_t m1 = (P > 4) ? ((P == 8) ? 0xffffffffu : ((1u << (8 * (P - 4))) - 1u)) : 0u;
        return ((u0 & m0) != (0xffffffffu & m0)) || ((u1 & m1) != (0xffffffffu & m1));
      };
      hit = any_in(lw[0][0], lw[0][1]) && any_in(lw[1][0], lw[1][1]) && any_in(lw[2][0], lw[2][1]);
    }
    const int k = wave_compact(hit, &s_nr[rr & 1]);
    __syncthreads();
    const int nhit = s_nr[rr & 1];
    for (int base = 0; base < nhit; base += CH) {
      if (hit && k >= base && k < base + CH) {
        const int ke = k - base;
        float* ent = s_ent + ke * ES;
        int lw[3][2];   // made again from the anchor: not held in registers across sub-rounds
        {
          int pk = __float_as_int(h.w);
          asm volatile("" : "+v"(pk));   // opaque here, so that this is not hoisted out of the loop
          const int b[3] = {pk & 1023, (pk >> 10) & 1023, (pk >> 20) & 1023};
          if (a.rel) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
              rel_locs<P>(axis_rel<P>(b[ax], t0[ax], a.N[ax]), T[ax], lw[ax][0], lw[ax][1]);
          } else {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
              axis_locs<P>(b[ax], t0[ax], T[ax], a.N[ax], lw[ax][0], lw[ax][1]);
          }
        }
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          ent[NW + NC + 2 * ax] = __int_as_float(lw[ax][0]);
          ent[NW + NC + 2 * ax + 1] = __int_as_float(lw[ax][1]);
        }
        ent[NW + NC + 6] = h.x; ent[NW + NC + 7] = h.y; ent[NW + NC + 8] = h.z;
        if (DEG == 2) {
          // tangent records carry q, mu, v_q, v_r, v_mu
          float co[10];
          float Jt[3][3];
#pragma unroll
          for (int i = 0; i < 9; ++i) Jt[i / 3][i % 3] = s_J[i];
          tangent_coeffs(Jt, c0v.x, make_float3(c0v.y, c0v.z, c0v.w), c1v.x,
                         make_float3(c1v.y, c1v.z, c1v.w), make_float3(c2v.x, c2v.y, c2v.z), co);
#pragma unroll
          for (int k = 0; k < 10; ++k) ent[NW + k] = co[k];
        } else if (DEG == 3) {
          // quadrupole records carry the ten coefficients
          ent[NW + 0] = c0v.x; ent[NW + 1] = c0v.y; ent[NW + 2] = c0v.z; ent[NW + 3] = c0v.w;
          ent[NW + 4] = c1v.x; ent[NW + 5] = c1v.y; ent[NW + 6] = c1v.z; ent[NW + 7] = c1v.w;
          ent[NW + 8] = c2v.x; ent[NW + 9] = c2v.y;
        } else {
          ent[NW + 0] = c0v.x; ent[NW + 1] = c0v.y; ent[NW + 2] = c0v.z; ent[NW + 3] = c0v.w;
        }
        int nx = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) nx += (loc_of(lw[0][0], lw[0][1], j) >= 0) ? 1 : 0;
        int t = atomicAdd(&s_ntask, nx);
#pragma unroll
        for (int j = 0; j < P; ++j)
          if (loc_of(lw[0][0], lw[0][1], j) >= 0) s_task[t++] = uint16_t((ke << 3) | j);
      }

      __syncthreads();
      const int ntask = s_ntask;
      // weights: one thread per (entry, axis); the x weights carry the fixed-point unit
      {
        const int nent = min(CH, nhit - base);
        for (int t = tid; t < 3 * nent; t += 256) {
          const int e = t / 3, ax = t - 3 * e;
          float* ent = s_ent + e * ES;
          float w[D + 1][P];
          spline_weights_whole<P, D>(ent[NW + NC + 6 + ax], w);
          const float sc = (ax == 0) ? scale : 1.0f;
#pragma unroll
          for (int d = 0; d <= D; ++d)
#pragma unroll
            for (int j = 0; j < P; ++j) ent[(ax * (D + 1) + d) * P + j] = w[d][j] * sc;
        }
      }
      __syncthreads();
      if (tid == 0) s_ntask = 0;   // every thread has read it before the barrier above
      // 2. accumulate: one task per (atom, in-tile x-plane of its stencil); stencil
      //    points outside the tile along z go to the scratch column T_z of their row
      for (int t = tid; t < ntask; t += 256) {
        const int task = s_task[t];
        const int e = task >> 3, ix = task & 7;
        const float* ent = s_ent + e * ES;
        const int lx = loc_of(__float_as_int(ent[NW + NC]), __float_as_int(ent[NW + NC + 1]), ix);
        const int ly0 = __float_as_int(ent[NW + NC + 2]), ly1 = __float_as_int(ent[NW + NC + 3]);
        const int lz0 = __float_as_int(ent[NW + NC + 4]), lz1 = __float_as_int(ent[NW + NC + 5]);
        float wz[D + 1][P];
        int zi[P];
#pragma unroll
        for (int d = 0; d <= D; ++d)
#pragma unroll
          for (int j = 0; j < P; ++j) wz[d][j] = ent[(2 * (D + 1) + d) * P + j];
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const int l = loc_of(lz0, lz1, j);
          zi[j] = (l >= 0) ? l : T[2];
        }
        float x[D + 1];
#pragma unroll
        for (int d = 0; d <= D; ++d) x[d] = ent[d * P + ix];   // pre-scaled by the fixed-point unit
        float co[NC];
#pragma unroll
        for (int kk = 0; kk < NC; ++kk) co[kk] = ent[NW + kk];
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
        const int rowx = lx * T[1];
#pragma unroll
        for (int iy = 0; iy < P; ++iy) {
          const int ly = loc_of(ly0, ly1, iy);
          if (ly < 0) continue;
          const float y0 = ent[(D + 1) * P + iy], y1 = ent[(D + 1) * P + P + iy];
          float c0 = ax0 * y0 + ay1 * y1, c1 = az1 * y0, c2 = 0.f;
          if (D == 2) {
            const float y2 = ent[(D + 1) * P + 2 * P + iy];
            c0 += ay2 * y2;
            c1 += ayz * y1;
            c2 = az2 * y0;
          }
          unsigned long long* row = s_tile + (rowx + ly) * TZP;
#pragma unroll
          for (int iz = 0; iz < P; ++iz) {
            float v = c0 * wz[0][iz] + c1 * wz[1][iz];
            if (D == 2) v += c2 * wz[2][iz];
            atomicAdd(row + zi[iz], to_fixed(v));
          }
        }
      }
      __syncthreads();
    }
    h = nh; c0v = nc0; c1v = nc1; c2v = nc2;
  }

  // 3. write the tile back (plain stores; every point is owned by this tile)
  // the fixed-point unit and the whole-number weights undone in one double factor
  const double inv_scale = 1.0 / (double(scale) * double(kWhole3));
  const int tvol = T[0] * T[1] * T[2];
  // tile extents are uniform: the multiply-high divisors are made once
  const uint32_t tz = uint32_t(__builtin_amdgcn_readfirstlane(T[2]));
  const uint32_t ty = uint32_t(__builtin_amdgcn_readfirstlane(T[1]));
  const FastDiv dz{tz, tz <= 1 ? 0u : uint32_t(__builtin_amdgcn_readfirstlane(int(0xffffffffu / tz + 1u)))};
  const FastDiv dy{ty, ty <= 1 ? 0u : uint32_t(__builtin_amdgcn_readfirstlane(int(0xffffffffu / ty + 1u)))};
#pragma unroll 1
  for (int e = tid; e < tvol; e += 256) {
    const int r = int(fdiv(uint32_t(e), dz)), lz = e - r * T[2];
    const int lx = int(fdiv(uint32_t(r), dy)), ly = r - lx * T[1];
    // the 64-bit sum as hi * 2^32 + lo in double precision (exact below 2^53),
    // then rounded once to float
    const long long v = (long long)s_tile[r * TZP + lz];
    const double vd = fma(double(int(v >> 32)), 4294967296.0, double(uint32_t(v)));
    a.rho[(size_t(t0[0] + lx) * a.N[1] + (t0[1] + ly)) * a.N[2] + t0[2] + lz] =
        float(vd * inv_scale);
  }
}

template <int P, int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
k_spread(SpreadArgs a, const double* box) {
  spread_body<P, DEG>(a, xcd_item(blockIdx.x, gridDim.x), box);
}

// Batched spread: work item (box, tile of the box).
template <int P, int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
k_spread_batch(const SpreadArgs* args, const int2* items, int nitems, const double* box) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    spread_body<P, DEG>(args[w.x], w.y, box + 9 * w.x);
    __syncthreads();
  }
}

template <bool TANGENT, bool QUAD = false>
hipError_t bin_dispatch(int p, dim3 g, hipStream_t s, const BinArgs& a, const LaunchEvents* ev) {
  switch (p) {
    case 1: launch_k(ev, k_bin<1, TANGENT, QUAD>, g, dim3(256), 0, s, a); break;
    case 2: launch_k(ev, k_bin<2, TANGENT, QUAD>, g, dim3(256), 0, s, a); break;
    case 3: launch_k(ev, k_bin<3, TANGENT, QUAD>, g, dim3(256), 0, s, a); break;
    case 4: launch_k(ev, k_bin<4, TANGENT, QUAD>, g, dim3(256), 0, s, a); break;
    case 5: launch_k(ev, k_bin<5, TANGENT, QUAD>, g, dim3(256), 0, s, a); break;
    case 6: launch_k(ev, k_bin<6, TANGENT, QUAD>, g, dim3(256), 0, s, a); break;
    case 7: launch_k(ev, k_bin<7, TANGENT, QUAD>, g, dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int DEG>
hipError_t spread_dispatch(int p, dim3 g, size_t sh, hipStream_t s, const SpreadArgs& a,
                           const double* box, const LaunchEvents* ev) {
  switch (p) {
    case 1: launch_k(ev, k_spread<1, DEG>, g, dim3(256), sh, s, a, box); break;
    case 2: launch_k(ev, k_spread<2, DEG>, g, dim3(256), sh, s, a, box); break;
    case 3: launch_k(ev, k_spread<3, DEG>, g, dim3(256), sh, s, a, box); break;
    case 4: launch_k(ev, k_spread<4, DEG>, g, dim3(256), sh, s, a, box); break;
    case 5: launch_k(ev, k_spread<5, DEG>, g, dim3(256), sh, s, a, box); break;
    case 6: launch_k(ev, k_spread<6, DEG>, g, dim3(256), sh, s, a, box); break;
    case 7: launch_k(ev, k_spread<7, DEG>, g, dim3(256), sh, s, a, box); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

namespace {

BinArgs make_bin_args(const DevPlan& d, int set, int n, const float* pos, const float* q,
                      const float* mu, const double* box, const float* v_pos, const float* v_q,
                      const float* v_mu, bool self_sums) {
  BinArgs a;
  a.n = n; a.pos = pos; a.q = q; a.mu = mu; a.box = box;
  a.v_pos = v_pos; a.v_q = v_q; a.v_mu = v_mu;
  a.theta = nullptr;
  a.spart_th = nullptr;
  for (int k = 0; k < 3; ++k) { a.N[k] = d.N[k]; a.B[k] = d.B[k]; a.nb[k] = d.nb[k]; }
  a.cap = d.cap;
  a.count = d.count[set]; a.ovf_count = d.ovf_count[set]; a.cmax = d.cmax[set];
  a.count_other = d.count[1 - set]; a.ovf_other = d.ovf_count[1 - set];
  a.cmax_other = d.cmax[1 - set];
  a.cmax_fwd = nullptr;
  a.cmax_fwd_other = nullptr;
  a.nbins = d.nb[0] * d.nb[1] * d.nb[2];
  a.rec = d.rec; a.ovf_base = d.ovf_base;
  a.spart = self_sums ? d.spart : nullptr;
  a.status = d.status;
  a.nblk = bin_blocks(n);
  a.off = 0;
  return a;
}

SpreadArgs make_spread_args(const DevPlan& d, int set, bool tangent) {
  SpreadArgs a;
  for (int k = 0; k < 3; ++k) {
    a.N[k] = d.N[k]; a.B[k] = d.B[k]; a.nb[k] = d.nb[k]; a.T[k] = d.T[k]; a.nt[k] = d.nt[k];
  }
  a.cap = d.cap;
  a.count = d.count[set]; a.ovf_count = d.ovf_count[set]; a.cmax = d.cmax[set];
  a.rec = d.rec; a.ovf_base = d.ovf_base; a.rho = d.rho;
  a.ch = d.spread_ch[tangent ? 1 : 0];
  a.nbr_max = d.nbr_max;
  a.tile_words = d.T[0] * d.T[1] * (d.T[2] + 1);
  a.rel = 1;
  for (int k = 0; k < 3; ++k)
    if (d.N[k] < d.T[k] + d.p - 1) a.rel = 0;
  return a;
}

size_t spread_lds(const DevPlan& d, bool tangent) {
  const SpreadArgs a = make_spread_args(d, 0, tangent);
  return spread_lds_bytes(a.tile_words, a.nbr_max, a.ch, d.p, tangent ? 2 : 1);
}

template <bool TANGENT>
hipError_t bin_batch_dispatch(int p, dim3 g, hipStream_t s, const BinArgs* args, const int2* it,
                              int n, const BatchIO& io, int ss) {
  switch (p) {
    case 1: hipLaunchKernelGGL((k_bin_batch<1, TANGENT>), g, dim3(256), 0, s, args, it, n, io, ss); break;
    case 2: hipLaunchKernelGGL((k_bin_batch<2, TANGENT>), g, dim3(256), 0, s, args, it, n, io, ss); break;
    case 3: hipLaunchKernelGGL((k_bin_batch<3, TANGENT>), g, dim3(256), 0, s, args, it, n, io, ss); break;
    case 4: hipLaunchKernelGGL((k_bin_batch<4, TANGENT>), g, dim3(256), 0, s, args, it, n, io, ss); break;
    case 5: hipLaunchKernelGGL((k_bin_batch<5, TANGENT>), g, dim3(256), 0, s, args, it, n, io, ss); break;
    case 6: hipLaunchKernelGGL((k_bin_batch<6, TANGENT>), g, dim3(256), 0, s, args, it, n, io, ss); break;
    case 7: hipLaunchKernelGGL((k_bin_batch<7, TANGENT>), g, dim3(256), 0, s, args, it, n, io, ss); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int DEG>
hipError_t spread_batch_dispatch(int p, dim3 g, size_t sh, hipStream_t s, const SpreadArgs* args,
                                 const int2* it, int n, const double* box) {
  switch (p) {
    case 1: hipLaunchKernelGGL((k_spread_batch<1, DEG>), g, dim3(256), sh, s, args, it, n, box); break;
    case 2: hipLaunchKernelGGL((k_spread_batch<2, DEG>), g, dim3(256), sh, s, args, it, n, box); break;
    case 3: hipLaunchKernelGGL((k_spread_batch<3, DEG>), g, dim3(256), sh, s, args, it, n, box); break;
    case 4: hipLaunchKernelGGL((k_spread_batch<4, DEG>), g, dim3(256), sh, s, args, it, n, box); break;
    case 5: hipLaunchKernelGGL((k_spread_batch<5, DEG>), g, dim3(256), sh, s, args, it, n, box); break;
    case 6: hipLaunchKernelGGL((k_spread_batch<6, DEG>), g, dim3(256), sh, s, args, it, n, box); break;
    case 7: hipLaunchKernelGGL((k_spread_batch<7, DEG>), g, dim3(256), sh, s, args, it, n, box); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// grid of a batched launch: every work item, up to a few workgroups per CU
inline dim3 batch_grid(int items, int cap) { return dim3(items < cap ? (items > 0 ? items : 1) : cap); }

}  // namespace

hipError_t enable_spread_lds() {
  const void* fns[] = {
#define PME_S(P)                                                               \
  reinterpret_cast<const void*>(k_spread<P, 1>), reinterpret_cast<const void*>(k_spread<P, 2>), \
      reinterpret_cast<const void*>(k_spread<P, 3>),                           \
      reinterpret_cast<const void*>(k_spread_batch<P, 1>),                     \
      reinterpret_cast<const void*>(k_spread_batch<P, 2>),
      PME_S(1) PME_S(2) PME_S(3) PME_S(4) PME_S(5) PME_S(6) PME_S(7)
#undef PME_S
  };
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kBigLds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t upload(void** dst, const void* src, size_t bytes) {
  *dst = nullptr;
  hipError_t e = hipMalloc(dst, bytes ? bytes : 1);
  if (e != hipSuccess) return e;
  return bytes ? hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
}

hipError_t launch_bin(const DevPlan& d, hipStream_t s, int set, int n, const float* pos,
                      const float* q, const float* mu, const double* box, const float* v_pos,
                      const float* v_q, const float* v_mu, bool tangent, bool self_sums,
                      const LaunchEvents* ev, bool fwd_max) {
  BinArgs a = make_bin_args(d, set, n, pos, q, mu, box, v_pos, v_q, v_mu, self_sums);
  if (tangent && fwd_max) {
    if (!d.cmax_fwd[0] || !d.cmax_fwd[1]) return hipErrorInvalidValue;
    a.cmax_fwd = d.cmax_fwd[set];
    a.cmax_fwd_other = d.cmax_fwd[1 - set];
  }
  const dim3 g(bin_blocks(n));
  return tangent ? bin_dispatch<true>(d.p, g, s, a, ev) : bin_dispatch<false>(d.p, g, s, a, ev);
}

hipError_t launch_bin_quad(const DevPlan& d, hipStream_t s, int set, int n, const float* pos,
                           const float* q, const float* mu, const float* theta, const double* box,
                           bool self_sums, const LaunchEvents* ev) {
  BinArgs a = make_bin_args(d, set, n, pos, q, mu, box, nullptr, nullptr, nullptr, self_sums);
  a.theta = theta;
  a.spart_th = self_sums ? d.spart + 2 * bin_blocks(n) : nullptr;
  return bin_dispatch<false, true>(d.p, dim3(bin_blocks(n)), s, a, ev);
}

hipError_t launch_spread_quad(const DevPlan& d, hipStream_t s, int set, const double* box,
                              const LaunchEvents* ev) {
  // the entries of the tangent spread (coefficients of degree <= 2)
  const SpreadArgs a = make_spread_args(d, set, true);
  const size_t sh = spread_lds(d, true);
  return spread_dispatch<3>(d.p, dim3(d.nt[0] * d.nt[1] * d.nt[2]), sh, s, a, box, ev);
}

hipError_t launch_spread(const DevPlan& d, hipStream_t s, int set, bool tangent,
                         const double* box, const LaunchEvents* ev) {
  if (d.band) return launch_spread_band(d, s, set, tangent, box, ev);
  const SpreadArgs a = make_spread_args(d, set, tangent);
  const size_t sh = spread_lds(d, tangent);
  const dim3 g(d.nt[0] * d.nt[1] * d.nt[2]);
  return tangent ? spread_dispatch<2>(d.p, g, sh, s, a, box, ev)
                 : spread_dispatch<1>(d.p, g, sh, s, a, box, ev);
}

hipError_t spread_batch_build(const DevPlan* plans, const int* n, const int* off, int nbox,
                              SpreadBatch& t) {
  t = SpreadBatch();
  t.nbox = nbox;
  t.p = nbox > 0 ? plans[0].p : 0;
  std::vector<BinArgs> ba(nbox);
  std::vector<SpreadArgs> sa(nbox);
  std::vector<ClearItem> ci(nbox);
  std::vector<int2> bitems, titems;
  for (int b = 0; b < nbox; ++b) {
    const DevPlan& d = plans[b];
    for (int k = 0; k < bin_blocks(n[b]); ++k) bitems.push_back(make_int2(b, k));
    const int nt = d.nt[0] * d.nt[1] * d.nt[2];
    for (int k = 0; k < nt; ++k) titems.push_back(make_int2(b, k));
    for (int tg = 0; tg < 2; ++tg) {
      const size_t l = spread_lds(d, tg == 1);
      if (l > t.lds[tg]) t.lds[tg] = l;
    }
    ci[b].count = d.count[0];
    ci[b].nbins = d.nb[0] * d.nb[1] * d.nb[2];
    ci[b].ovf_count = d.ovf_count[0];
    ci[b].cmax = d.cmax[0];
  }
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t r) { if (r != hipSuccess && e == hipSuccess) e = r; };
  for (int tg = 0; tg < 2; ++tg)
    for (int set = 0; set < 2; ++set) {
      for (int b = 0; b < nbox; ++b) {
        ba[b] = make_bin_args(plans[b], set, n[b], nullptr, nullptr, nullptr, nullptr, nullptr,
                              nullptr, nullptr, tg == 0);
        ba[b].off = off[b];
        sa[b] = make_spread_args(plans[b], set, tg == 1);
      }
      ok(upload(&t.bin[tg][set], ba.data(), sizeof(BinArgs) * nbox));
      ok(upload(&t.spread[tg][set], sa.data(), sizeof(SpreadArgs) * nbox));
    }
  ok(upload(&t.clear, ci.data(), sizeof(ClearItem) * nbox));
  ok(upload(reinterpret_cast<void**>(&t.bin_items), bitems.data(), sizeof(int2) * bitems.size()));
  ok(upload(reinterpret_cast<void**>(&t.tile_items), titems.data(), sizeof(int2) * titems.size()));
  t.n_bin_items = int(bitems.size());
  t.n_tile_items = int(titems.size());
  return e;
}

void spread_batch_free(SpreadBatch& t) {
  for (int tg = 0; tg < 2; ++tg)
    for (int set = 0; set < 2; ++set) {
      if (t.bin[tg][set]) (void)hipFree(t.bin[tg][set]);
      if (t.spread[tg][set]) (void)hipFree(t.spread[tg][set]);
    }
  if (t.clear) (void)hipFree(t.clear);
  if (t.bin_items) (void)hipFree(t.bin_items);
  if (t.tile_items) (void)hipFree(t.tile_items);
  t = SpreadBatch();
}

hipError_t launch_clear_batch(const SpreadBatch& t, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_batch, batch_grid(t.nbox, 1024), dim3(256), 0, s,
                     static_cast<const ClearItem*>(t.clear), t.nbox);
  return hipGetLastError();
}

hipError_t launch_bin_batch(const SpreadBatch& t, hipStream_t s, int set, bool tangent,
                            const BatchIO& io, bool self_sums) {
  const BinArgs* args = static_cast<const BinArgs*>(t.bin[tangent ? 1 : 0][set]);
  const dim3 g = batch_grid(t.n_bin_items, 2048);
  return tangent ? bin_batch_dispatch<true>(t.p, g, s, args, t.bin_items, t.n_bin_items, io, 0)
                 : bin_batch_dispatch<false>(t.p, g, s, args, t.bin_items, t.n_bin_items, io,
                                             self_sums ? 1 : 0);
}

hipError_t launch_spread_batch(const SpreadBatch& t, hipStream_t s, int set, bool tangent,
                               const double* box) {
  const SpreadArgs* args = static_cast<const SpreadArgs*>(t.spread[tangent ? 1 : 0][set]);
  const dim3 g = batch_grid(t.n_tile_items, 1280);
  const size_t sh = t.lds[tangent ? 1 : 0];
  return tangent ? spread_batch_dispatch<2>(t.p, g, sh, s, args, t.tile_items, t.n_tile_items, box)
                 : spread_batch_dispatch<1>(t.p, g, sh, s, args, t.tile_items, t.n_tile_items,
                                            box);
}

}  // namespace pme
