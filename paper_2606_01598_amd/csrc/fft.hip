// The mesh operator K of Secs. 2.3.3-2.3.4: real-to-complex 3D DFT of the density
// (Eq. fft), multiplication by g(k) = G(k) C(n) (Eqs. green, influence,
// potential_k) and the unnormalised complex-to-real inverse (Eq. ifft), plus the
// k-space form of the reciprocal energy (Eq. energy_recip):
//     E_recip = (1/2V) sum_n rho phi = (1/2V) sum_k g(k) |rho~(k)|^2.
//
// LDS-staged passes over the half spectrum spec[x][y][kz], kz < N_z/2+1.  When a
// y-z plane of the half spectrum fits in LDS (slab mode) there are three:
//   slab fwd  one x-plane per workgroup: z R2C (two real rows packed into one
//             complex pencil) then y FFT, in LDS
//   x         fused forward FFT along x, x g(k), energy partial, inverse FFT along x
//   slab inv  y inverse FFT then z C2R (two Hermitian rows unpacked into one
//             complex pencil), in LDS
// Otherwise five pencil passes: z R2C, y fwd, x fused, y inv, z C2R.
// Each 1D transform is a mixed-radix (2, 3, 4, 5, 6, 8, 10) Stockham autosort over
// LDS ping-pong buffers; twiddles come from a per-axis table staged into LDS.
//
// Readings: signed frequency indices in fftfreq order (Nyquist at -N/2); the
// Nyquist bins of a non-orthogonal cell use the mean of g over the bin and its
// Hermitian partner, which makes the half-spectrum product equal the real part of
// the full complex product (the real-to-complex semantics).
#include <vector>

#include "../../include/pme.h"
#include "fft_radix.h"
#include "kernels.h"
#include "pme_common.h"
#include "plane_spread.h"

namespace pme {
namespace {

// Transform npen pencils (stride ps) held in x by stages [s0, s1) of the plan (all
// by default); returns the buffer holding the result.
__device__ __forceinline__ float2* lds_fft(float2* x, float2* y, int npen, int ps, const AxisPlan& ax,
                           const float2* tw, float s, int s0 = 0, int s1 = -1) {
  if (s1 < 0) s1 = ax.nst;
  for (int sti = s0; sti < s1; ++sti) {
    const FFTStage& st = ax.st[sti];
    const int total = npen * st.NR;
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int pen = int(fdiv(uint32_t(t), st.nr));
      const int j = t - pen * st.NR;
      const int jq = int(fdiv(uint32_t(j), st.ns));
      const int k = j - jq * st.Ns;
      const float2* in = x + pen * ps;
      float2* out = y + pen * ps;
      switch (st.R) {
#define PME_R(R) \
  case R: stockham_butterfly<R>(in, out, j, k, jq, st.Ns, st.NR, st.step, tw, s); break;
        PME_R(2) PME_R(3) PME_R(4) PME_R(5) PME_R(6) PME_R(8) PME_R(10)
#undef PME_R
        default: break;
      }
    }
    __syncthreads();
    float2* t = x; x = y; y = t;
  }
  return x;
}

// Twiddle table held in registers between its load and its LDS store, so that its
// loads are in flight together with the data loads (N <= 1024).
template <int NT>
struct Twiddles {
  static constexpr int U = (1024 + NT - 1) / NT;
  float2 v[U];
  __device__ __forceinline__ void load(const float2* src, int N) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = threadIdx.x + u * NT;
      if (t < N) v[u] = src[t];
    }
  }
  __device__ __forceinline__ void store(float2* dst, int N) const {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = threadIdx.x + u * NT;
      if (t < N) dst[t] = v[u];
    }
  }
};

// Global -> LDS copy with U loads in flight per thread before the LDS stores.
template <int U, class T, class Ld, class St>
__device__ __forceinline__ void staged_copy(int total, Ld ld, St st) {
  for (int e0 = threadIdx.x; e0 < total; e0 += U * blockDim.x) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * blockDim.x;
      if (e < total) v[u] = ld(e);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * blockDim.x;
      if (e < total) st(e, v[u]);
    }
  }
}

struct ZArgs {
  AxisPlan ax;
  const float2* tw;
  int rows;        // N_x N_y
  int H;
  int rp;          // rows per block (even)
  FastDiv nd;      // division by N_z
  const float* src;
  float2* spec;
  float* dst;
};

// z pass, real to complex
__global__ void __launch_bounds__(kFFTThreads) k_fftz_r2c(ZArgs a) {
  extern __shared__ float2 sm[];
  const int N = a.ax.N, H = a.H;
  float2* tw = sm;
  float2* X = tw + N;
  float2* Y = X + (a.rp / 2) * N;
  const int r0 = blockIdx.x * a.rp;
  Twiddles<kFFTThreads> twr;
  twr.load(a.tw, N);
  const int np = a.rp / 2;
  staged_copy<16, float2>(
      np * N,
      [&](int e) {
        const int c = int(fdiv(uint32_t(e), a.nd)), m = e - c * N;
        const int ra = r0 + 2 * c, rb = ra + 1;
        return make_float2(ra < a.rows ? a.src[size_t(ra) * N + m] : 0.0f,
                           rb < a.rows ? a.src[size_t(rb) * N + m] : 0.0f);
      },
      [&](int e, float2 v) { X[e] = v; });
  twr.store(tw, N);
  __syncthreads();
  const float2* Z = lds_fft(X, Y, np, N, a.ax, tw, -1.0f);
  for (int e = threadIdx.x; e < a.rp * H; e += blockDim.x) {
    const int rr = e / H, k = e - rr * H;
    const int row = r0 + rr;
    if (row >= a.rows) continue;
    const int c = rr >> 1;
    const float2 zk = Z[c * N + k];
    const float2 zn = Z[c * N + (k ? N - k : 0)];
    float2 v;
    if ((rr & 1) == 0) v = make_float2(0.5f * (zk.x + zn.x), 0.5f * (zk.y - zn.y));
    else v = make_float2(0.5f * (zk.y + zn.y), -0.5f * (zk.x - zn.x));
    a.spec[size_t(row) * H + k] = v;
  }
}

// z pass, complex to real
__global__ void __launch_bounds__(kFFTThreads) k_fftz_c2r(ZArgs a) {
  extern __shared__ float2 sm[];
  const int N = a.ax.N, H = a.H;
  float2* tw = sm;
  float2* S = tw + N;
  float2* X = S + a.rp * H;
  float2* Y = X + (a.rp / 2) * N;
  const int r0 = blockIdx.x * a.rp;
  Twiddles<kFFTThreads> twr;
  twr.load(a.tw, N);
  const int nvalid = min(a.rp, a.rows - r0) * H;
  staged_copy<16, float2>(
      a.rp * H, [&](int e) { return e < nvalid ? a.spec[size_t(r0) * H + e] : make_float2(0.f, 0.f); },
      [&](int e, float2 v) { S[e] = v; });
  twr.store(tw, N);
  __syncthreads();
  const int np = a.rp / 2;
  const bool even = (N & 1) == 0;
  for (int e = threadIdx.x; e < np * N; e += blockDim.x) {
    const int c = e / N, m = e - c * N;
    float2 A, B;
    if (m < H) {
      A = S[(2 * c) * H + m];
      B = S[(2 * c + 1) * H + m];
    } else {
      A = S[(2 * c) * H + N - m];
      B = S[(2 * c + 1) * H + N - m];
      A.y = -A.y;
      B.y = -B.y;
    }
    if (m == 0 || (even && m == N / 2)) { A.y = 0.0f; B.y = 0.0f; }
    X[e] = make_float2(A.x - B.y, A.y + B.x);
  }
  __syncthreads();
  const float2* Z = lds_fft(X, Y, np, N, a.ax, tw, +1.0f);
  for (int e = threadIdx.x; e < np * N; e += blockDim.x) {
    const int c = e / N, m = e - c * N;
    const int ra = r0 + 2 * c, rb = ra + 1;
    const float2 z = Z[e];
    if (ra < a.rows) a.dst[size_t(ra) * N + m] = z.x;
    if (rb < a.rows) a.dst[size_t(rb) * N + m] = z.y;
  }
}

struct SlabArgs {
  AxisPlan ay, az;
  const float2* twy;
  const float2* twz;
  int H;
  FastDiv nzd, hd;   // division by N_z and by H
  const float* src;  // real mesh (forward input)
  float2* spec;
  float* dst;        // real mesh (inverse output)
};

__device__ __forceinline__ void slab_layout(const SlabArgs& a, float2* sm, float2*& twz,
                                            float2*& twy, float2*& A, float2*& B) {
  const int Ny = a.ay.N, Nz = a.az.N;
  const int npairs = (Ny + 1) / 2;
  const int buf = max(npairs * Nz, a.H * (Ny + 1));
  twz = sm;
  twy = twz + Nz;
  A = twy + Ny;
  B = A + buf;
}

// forward slab: rho[x] -> z R2C -> y FFT -> spec[x].  Two real rows y = 2c, 2c+1 form
// one complex pencil; the first z stage reads them from global memory (when one
// round of the workgroup covers it) and the first y stage unpacks the two real
// transforms as it reads:
//   X_2c[k] = (Z[k] + conj Z[N-k]) / 2,  X_2c+1[k] = (Z[k] - conj Z[N-k]) / 2i.
// src(y, z) gives the plane's real value at (y, z); the twiddles are in tz and ty
// (stored to twz and twy before the first barrier); A and B hold max(npairs N_z,
// H (N_y + 1)) complex values each.
template <class Src>
__device__ __forceinline__ void slab_fwd_run(const SlabArgs& a, const int x, const Src& src,
                                             const Twiddles<kSlabThreads>& tz,
                                             const Twiddles<kSlabThreads>& ty, float2* twz,
                                             float2* twy, float2* A, float2* B) {
  const int Ny = a.ay.N, Nz = a.az.N, H = a.H;
  const int npairs = (Ny + 1) / 2;
  const FFTStage& z0 = a.az.st[0];
  float2* Z;
  if (npairs * z0.NR <= int(blockDim.x)) {
    const int t = threadIdx.x;
    if (t < npairs * z0.NR) {
      const int c = int(fdiv(uint32_t(t), z0.nr)), j = t - c * z0.NR;
      const bool odd_last = (2 * c + 1 >= Ny);   // odd row count: zero imaginary row
      float2* out = A + c * Nz;
      with_radix(z0.R, [&](auto rc) {
        constexpr int R = decltype(rc)::value;
        stockham_butterfly_io<R, false>(
            [&](int i) { return make_float2(src(2 * c, i), odd_last ? 0.0f : src(2 * c + 1, i)); },
            [&](int i, float2 v) { out[i] = v; }, j, 0, j, 1, z0.NR, z0.step, twz, -1.0f);
      });
    }
    tz.store(twz, Nz);
    ty.store(twy, Ny);
    __syncthreads();
    Z = lds_fft(A, B, npairs, Nz, a.az, twz, -1.0f, 1, -1);
  } else {
    float* Af = reinterpret_cast<float*>(A);
    staged_copy<12, float>(
        Ny * Nz,
        [&](int e) {
          const int y = int(fdiv(uint32_t(e), a.nzd));
          return src(y, e - y * Nz);
        },
        [&](int e, float v) {
          const int y = int(fdiv(uint32_t(e), a.nzd)), m = e - y * Nz;
          Af[2 * ((y >> 1) * Nz + m) + (y & 1)] = v;
        });
    if (Ny & 1)
      for (int m = threadIdx.x; m < Nz; m += blockDim.x) Af[2 * ((Ny >> 1) * Nz + m) + 1] = 0.0f;
    tz.store(twz, Nz);
    ty.store(twy, Ny);
    __syncthreads();
    Z = lds_fft(A, B, npairs, Nz, a.az, twz, -1.0f);
  }
  float2* O = (Z == A) ? B : A;
  const int ps = Ny + 1;
  {
    const FFTStage& y0 = a.ay.st[0];
    for (int t = threadIdx.x; t < H * y0.NR; t += blockDim.x) {
      const int k = int(fdiv(uint32_t(t), y0.nr)), j = t - k * y0.NR;
      const int kn = k ? Nz - k : 0;
      float2* out = O + k * ps;
      with_radix(y0.R, [&](auto rc) {
        constexpr int R = decltype(rc)::value;
        stockham_butterfly_io<R, false>(
            [&](int y) {
              const int c = y >> 1;
              const float2 zk = Z[c * Nz + k], zn = Z[c * Nz + kn];
              return ((y & 1) == 0) ? make_float2(0.5f * (zk.x + zn.x), 0.5f * (zk.y - zn.y))
                                    : make_float2(0.5f * (zk.y + zn.y), -0.5f * (zk.x - zn.x));
            },
            [&](int i, float2 v) { out[i] = v; }, j, 0, j, 1, y0.NR, y0.step, twy, -1.0f);
      });
    }
  }
  __syncthreads();
  float2* dst = a.spec + size_t(x) * Ny * H;
  const int ny = a.ay.nst;
  if (ny >= 2 && H * a.ay.st[ny - 1].NR <= int(blockDim.x)) {
    // last y stage writes the spectrum rows itself (kz fastest across lanes)
    const float2* Rin = lds_fft(O, Z, H, ps, a.ay, twy, -1.0f, 1, ny - 1);
    const FFTStage& yl = a.ay.st[ny - 1];
    const int t = threadIdx.x;
    if (t < H * yl.NR) {
      const int j = int(fdiv(uint32_t(t), a.hd)), k = t - j * H;
      const int jq = int(fdiv(uint32_t(j), yl.ns)), kk = j - jq * yl.Ns;
      const float2* in = Rin + k * ps;
      with_radix(yl.R, [&](auto rc) {
        constexpr int Rr = decltype(rc)::value;
        stockham_butterfly_io<Rr, true>([&](int i) { return in[i]; },
                                        [&](int y, float2 v) { dst[size_t(y) * H + k] = v; }, j, kk,
                                        jq, yl.Ns, yl.NR, yl.step, twy, -1.0f);
      });
    }
  } else {
    const float2* R = lds_fft(O, Z, H, ps, a.ay, twy, -1.0f, 1, -1);
    for (int e = threadIdx.x; e < Ny * H; e += blockDim.x) {
      const int y = int(fdiv(uint32_t(e), a.hd)), k = e - y * H;
      dst[e] = R[k * ps + y];
    }
  }
}

__device__ __forceinline__ void slab_fwd_body(const SlabArgs& a, const int x) {
  extern __shared__ float2 sm[];
  float2 *twz, *twy, *A, *B;
  slab_layout(a, sm, twz, twy, A, B);
  Twiddles<kSlabThreads> tz, ty;
  tz.load(a.twz, a.az.N);
  ty.load(a.twy, a.ay.N);
  const int Nz = a.az.N;
  const float* src = a.src + size_t(x) * a.ay.N * Nz;
  slab_fwd_run(a, x, [&](int y, int z) { return src[size_t(y) * Nz + z]; }, tz, ty, twz, twy, A, B);
}

// inverse slab: spec[x] -> y inverse FFT -> z C2R -> out[x].  The first y stage reads
// from global memory (when one round covers it); the first z stage packs two
// Hermitian rows into one complex pencil as it reads:
//   P[m] = X_2c[m] + i X_2c+1[m], X[m] = conj X[N-m] for m >= H.
__device__ __forceinline__ void slab_inv_body(const SlabArgs& a, const int x) {
  extern __shared__ float2 sm[];
  const int Ny = a.ay.N, Nz = a.az.N, H = a.H;
  const int npairs = (Ny + 1) / 2;
  float2 *twz, *twy, *A, *B;
  slab_layout(a, sm, twz, twy, A, B);
  Twiddles<kSlabThreads> tz, ty;
  tz.load(a.twz, Nz);
  ty.load(a.twy, Ny);
  const int ps = Ny + 1;
  const float2* src = a.spec + size_t(x) * Ny * H;
  const FFTStage& y0 = a.ay.st[0];
  float2* R;
  if (H * y0.NR <= int(blockDim.x)) {
    const int t = threadIdx.x;
    if (t < H * y0.NR) {
      // k fastest: consecutive lanes read consecutive kz of one spectrum row
      const int j = int(fdiv(uint32_t(t), a.hd)), k = t - j * H;
      float2* out = A + k * ps;
      with_radix(y0.R, [&](auto rc) {
        constexpr int Rr = decltype(rc)::value;
        stockham_butterfly_io<Rr, false>([&](int y) { return src[size_t(y) * H + k]; },
                                         [&](int i, float2 v) { out[i] = v; }, j, 0, j, 1, y0.NR,
                                         y0.step, twy, 1.0f);
      });
    }
    tz.store(twz, Nz);
    ty.store(twy, Ny);
    __syncthreads();
    R = lds_fft(A, B, H, ps, a.ay, twy, +1.0f, 1, -1);
  } else {
    staged_copy<12, float2>(
        Ny * H, [&](int e) { return src[e]; },
        [&](int e, float2 v) {
          const int y = int(fdiv(uint32_t(e), a.hd)), k = e - y * H;
          A[k * ps + y] = v;
        });
    tz.store(twz, Nz);
    ty.store(twy, Ny);
    __syncthreads();
    R = lds_fft(A, B, H, ps, a.ay, twy, +1.0f);
  }
  float2* O = (R == A) ? B : A;
  const bool even = (Nz & 1) == 0;
  {
    const FFTStage& z0 = a.az.st[0];
    for (int t = threadIdx.x; t < npairs * z0.NR; t += blockDim.x) {
      const int c = int(fdiv(uint32_t(t), z0.nr)), j = t - c * z0.NR;
      const int ya = 2 * c, yb = ya + 1;
      const bool hasb = yb < Ny;
      float2* out = O + c * Nz;
      with_radix(z0.R, [&](auto rc) {
        constexpr int Rr = decltype(rc)::value;
        stockham_butterfly_io<Rr, false>(
            [&](int m) {
              float2 Av, Bv;
              if (m < H) {
                Av = R[m * ps + ya];
                Bv = hasb ? R[m * ps + yb] : make_float2(0.f, 0.f);
              } else {
                Av = R[(Nz - m) * ps + ya];
                Bv = hasb ? R[(Nz - m) * ps + yb] : make_float2(0.f, 0.f);
                Av.y = -Av.y;
                Bv.y = -Bv.y;
              }
              if (m == 0 || (even && m == Nz / 2)) {
                Av.y = 0.0f;
                Bv.y = 0.0f;
              }
              return make_float2(Av.x - Bv.y, Av.y + Bv.x);
            },
            [&](int i, float2 v) { out[i] = v; }, j, 0, j, 1, z0.NR, z0.step, twz, 1.0f);
      });
    }
  }
  __syncthreads();
  float* dst = a.dst + size_t(x) * Ny * Nz;
  const int nz = a.az.nst;
  if (nz >= 2 && npairs * a.az.st[nz - 1].NR <= int(blockDim.x)) {
    // last z stage writes the two real rows of its pencil itself
    const float2* Zin = lds_fft(O, R, npairs, Nz, a.az, twz, +1.0f, 1, nz - 1);
    const FFTStage& zl = a.az.st[nz - 1];
    const int t = threadIdx.x;
    if (t < npairs * zl.NR) {
      const int c = int(fdiv(uint32_t(t), zl.nr)), j = t - c * zl.NR;
      const int jq = int(fdiv(uint32_t(j), zl.ns)), kk = j - jq * zl.Ns;
      const float2* in = Zin + c * Nz;
      float* ra = dst + size_t(2 * c) * Nz;
      float* rb = ra + Nz;
      const bool hasb = 2 * c + 1 < Ny;
      with_radix(zl.R, [&](auto rc) {
        constexpr int Rr = decltype(rc)::value;
        stockham_butterfly_io<Rr, true>(
            [&](int i) { return in[i]; },
            [&](int m, float2 v) {
              ra[m] = v.x;
              if (hasb) rb[m] = v.y;
            },
            j, kk, jq, zl.Ns, zl.NR, zl.step, twz, 1.0f);
      });
    }
  } else {
    const float2* Z = lds_fft(O, R, npairs, Nz, a.az, twz, +1.0f, 1, -1);
    for (int e = threadIdx.x; e < Ny * Nz; e += blockDim.x) {
      const int y = int(fdiv(uint32_t(e), a.nzd)), m = e - y * Nz;
      const float2 v = Z[(y >> 1) * Nz + m];
      dst[e] = (y & 1) ? v.y : v.x;
    }
  }
}

struct YArgs {
  AxisPlan ax;
  const float2* tw;
  int Ny, H, kt;
  FastDiv ktd;
  float2* spec;
  float sign;
};

// y pass: block = (x, tile of kz columns)
__global__ void __launch_bounds__(kFFTThreads) k_ffty(YArgs a) {
  extern __shared__ float2 sm[];
  const int N = a.ax.N, H = a.H, kt = a.kt;
  const int ps = N + 1;
  float2* tw = sm;
  float2* X = tw + N;
  float2* Y = X + kt * ps;
  const int ntk = (H + kt - 1) / kt;
  const int x = blockIdx.x / ntk, kz0 = (blockIdx.x - x * ntk) * kt;
  Twiddles<kFFTThreads> twr;
  twr.load(a.tw, N);
  float2* base = a.spec + size_t(x) * a.Ny * H;
  staged_copy<16, float2>(
      N * kt,
      [&](int e) {
        const int yy = int(fdiv(uint32_t(e), a.ktd)), l = e - yy * kt;
        const int kz = kz0 + l;
        return (kz < H) ? base[size_t(yy) * H + kz] : make_float2(0.f, 0.f);
      },
      [&](int e, float2 v) {
        const int yy = int(fdiv(uint32_t(e), a.ktd)), l = e - yy * kt;
        X[l * ps + yy] = v;
      });
  twr.store(tw, N);
  __syncthreads();
  const float2* Z = lds_fft(X, Y, kt, ps, a.ax, tw, a.sign);
  for (int e = threadIdx.x; e < N * kt; e += blockDim.x) {
    const int yy = e / kt, l = e - yy * kt;
    const int kz = kz0 + l;
    if (kz < H) base[size_t(yy) * H + kz] = Z[l * ps + yy];
  }
}

struct XArgs {
  AxisPlan ax;
  AxisPlan axi;    // the same radices in reverse order (inverse transform)
  const float2* tw;
  int N[3];
  int H, kt;
  FastDiv ktd;
  float2* spec;
  const double* box;
  const float* dcx;
  const float* dcy;
  const float* dcz;
  double alpha;
  double* epart;   // may be null
  // cell gradient (the VIR variant): per workgroup the six sums over its points of
  // w |rho~|^2 g (1/k^2 + 1/(4 alpha^2)) k_c k_d (cc, dd, ..: xx yy zz xy xz yz)
  double* vpart;
  // optimal influence (the OPT variant): aliasing weights [3][N_a] per axis
  const float* alx;
  const float* aly;
  const float* alz;
  // the per-workgroup cache of g and its keys (DevPlan::gcache, gkey; may be null)
  float* gcache;
  double* gkey;
};

__device__ __forceinline__ int signed_freq(int k, int N) { return (k >= (N + 1) / 2) ? k - N : k; }

// x pass fused with the influence function: forward FFT along x of kt half-spectrum
// lines (fixed y, consecutive kz), x g(k) (with the energy partial), inverse FFT.
//   g(k) = (4 pi / k^2) exp(-k^2 / (4 alpha^2)) dcx(kx) dcy(ky) dcz(kz),
//   k^2 = f^T M f, M = 4 pi^2 C^-1 C^-T (reciprocal metric), f = signed frequencies;
// g is 0 at k = 0; a Nyquist bin takes the mean of g over the bin and its Hermitian
// partner.  g depends on the box only (the mesh, order, alpha and influence are the
// plan's): a workgroup keeps its table in the plan's cache, with the box as key, and
// when the key equals the box it loads the table with the lines instead of making it.
// Otherwise g is tabulated while the line loads are in flight.  The product itself
// sits between the last forward and the first inverse stage, in registers (x_middle).
// MODE 0: the influence function of Eq. influence; 1: the same, also forming the
// cell-gradient partials; 2: the optimal influence function (aliasing sums).
template <int MODE = 0>
__device__ __forceinline__ void fftx_body(const XArgs& a, const int blk, const double* box,
                                          double* epart) {
  extern __shared__ float2 sm[];
  __shared__ double red[8];
  const int Nx = a.N[0], Ny = a.N[1], Nz = a.N[2], H = a.H, kt = a.kt;
  const int ps = Nx + 1;
  float2* tw = sm;
  float2* X = tw + Nx;
  float2* Y = X + kt * ps;
  float* s_g = reinterpret_cast<float*>(Y + kt * ps);   // g[l Nx + kx]
  constexpr bool VIR = MODE == 1, OPT = MODE == 2;
  float* s_dc = s_g + Nx * kt;                          // deconvolution: [Nx] x, [kt] z
  float* s_alx = s_dc + Nx + kt;                        // OPT: [3][Nx] x aliasing weights,
  float* s_alz = s_alx + 3 * Nx;                        //      [3][kt] z aliasing weights
  const int ntk = (H + kt - 1) / kt;
  const int y = blk / ntk, kz0 = (blk - y * ntk) * kt;
  // the x and z deconvolution factors of the workgroup's points, loaded before the
  // lines (waiting for them does not wait for the lines) and put in LDS before the
  // g table is made
  constexpr int DCU = 5;   // Nx + kt <= DCU blockDim (Nx <= 1024, kt <= 24)
  float dcv[DCU];
#pragma unroll
  for (int k = 0; k < DCU; ++k) {
    // unconditional loads from clamped addresses (straight-line code lets the later
    // wait count only these loads); entries past Nx + kt are not stored
    const int i = int(threadIdx.x) + k * int(blockDim.x);
    const float* src = (i < Nx) ? a.dcx + i : a.dcz + min(kz0 + max(i - Nx, 0), H - 1);
    dcv[k] = *src;
  }
  constexpr int ALU = OPT ? 13 : 1;   // 3 (Nx + kt) <= ALU blockDim
  float alv[ALU];
  if constexpr (OPT) {
#pragma unroll
    for (int k = 0; k < ALU; ++k) {
      const int i = int(threadIdx.x) + k * int(blockDim.x);
      const int j = max(i - 3 * Nx, 0);
      const int m = int(fdiv(uint32_t(j), a.ktd)), l = j - m * kt;
      const float* src = (i < 3 * Nx) ? a.alx + i
                                      : a.alz + min(m, 2) * Nz + min(kz0 + l, H - 1);
      alv[k] = *src;
    }
  }
  // the workgroup's cached g table, loaded before the lines whether or not its key
  // matches (the decision waits for the key; the loads need not)
  const int KN = Nx * kt;
  float* gblk = a.gcache ? a.gcache + size_t(blk) * KN : nullptr;
  constexpr int GU = 14;   // Nx kt <= GU blockDim (the plan bounds kt (Nx + 1) by 3500)
  float gv[GU];
  if (gblk) {
#pragma unroll
    for (int k = 0; k < GU; ++k) {
      const int e = int(threadIdx.x) + k * int(blockDim.x);
      gv[k] = (e < KN) ? gblk[e] : 0.0f;
    }
  }
  auto store_dc = [&]() {
#pragma unroll
    for (int k = 0; k < DCU; ++k) {
      const int i = int(threadIdx.x) + k * int(blockDim.x);
      if (i < Nx + kt) s_dc[i] = dcv[k];
    }
    if constexpr (OPT) {
#pragma unroll
      for (int k = 0; k < ALU; ++k) {
        const int i = int(threadIdx.x) + k * int(blockDim.x);
        if (i < 3 * (Nx + kt)) s_alx[i] = alv[k];
      }
    }
    __syncthreads();
  };
  Twiddles<kFFTThreads> twr;
  twr.load(a.tw, Nx);
  const size_t xstride = size_t(Ny) * H;
  float2* base = a.spec + size_t(y) * H;
  // g of the workgroup's points into LDS (issued while the line loads are in flight)
  auto gtable = [&]() {
    const Cell c = cell_from_box(box);
    // the reciprocal metric, 1/(4 alpha^2), k^2 and the exponent argument in double
    // precision, rounded once each to float: constants rounded to float would bias
    // every g(k) alike (about 1e-7 relative, which the near cancellation of E_recip
    // against the self terms would amplify in E^lr); a single rounding of k^2 and of
    // the argument is unbiased, and the exponential itself is evaluated in float
    double M[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        double m = 0.0;
#pragma unroll
        for (int g = 0; g < 3; ++g) m += c.inv[3 * g + p] * c.inv[3 * g + q];
        M[p][q] = 4.0 * M_PI * M_PI * m;
      }
    const double inv4a2 = 1.0 / (4.0 * a.alpha * a.alpha);
    const int fyi = signed_freq(y, Ny);
    const float fy = float(fyi);
    const bool nyq_y = ((Ny & 1) == 0) && (2 * fyi == -Ny);
    const float dcy = a.dcy[y];
    auto gk = [&](float px, float py, float pz) {
      const double x = px, y = py, z = pz;
      const double k2 = M[0][0] * x * x + M[1][1] * y * y + M[2][2] * z * z +
                        2.0 * (M[0][1] * x * y + M[0][2] * x * z + M[1][2] * y * z);
      return float(4.0 * M_PI / k2) * expf(-float(k2 * inv4a2));
    };
    float aly3[3] = {0.0f, 0.0f, 0.0f};
    if constexpr (OPT) {
#pragma unroll
      for (int m = 0; m < 3; ++m) aly3[m] = a.aly[m * Ny + y];
    }
    for (int e = threadIdx.x; e < Nx * kt; e += blockDim.x) {
      const int xx = int(fdiv(uint32_t(e), a.ktd)), l = e - xx * kt;
      const int kz = kz0 + l;
      float g = 0.0f;
      if (kz < H && (xx | y | kz) != 0) {
        const float fx = float(signed_freq(xx, Nx)), fz = float(signed_freq(kz, Nz));
        const bool nx = ((Nx & 1) == 0) && (2 * xx == Nx);
        const bool nz = ((Nz & 1) == 0) && (2 * kz == Nz);
        if constexpr (OPT) {
          // sum over the aliases f + m N of U^2 G; a partner frequency s f (s = -1 on
          // the flipped axes) takes the weight of alias -m of f, as sinc is even
          auto gopt = [&](int sx, int sy, int sz) {
            float num = 0.0f;
#pragma unroll
            for (int mx = -1; mx <= 1; ++mx) {
              const float ux = s_alx[(sx * mx + 1) * Nx + xx];
#pragma unroll
              for (int my = -1; my <= 1; ++my) {
                const float uxy = ux * aly3[sy * my + 1];
#pragma unroll
                for (int mz = -1; mz <= 1; ++mz) {
                  const float u2 = uxy * s_alz[(sz * mz + 1) * kt + l];
                  num = fmaf(u2, gk(float(sx) * fx + float(mx * Nx), float(sy) * fy + float(my * Ny),
                                    float(sz) * fz + float(mz * Nz)), num);
                }
              }
            }
            return num;
          };
          g = gopt(1, 1, 1);
          if (nx || nyq_y || nz) g = 0.5f * (g + gopt(nx ? 1 : -1, nyq_y ? 1 : -1, nz ? 1 : -1));
          g *= s_dc[xx] * dcy * s_dc[Nx + l];
        } else {
          g = gk(fx, fy, fz);
          if (nx || nyq_y || nz)   // Hermitian partner: the non-Nyquist components change sign
            g = 0.5f * (g + gk(nx ? fx : -fx, nyq_y ? fy : -fy, nz ? fz : -fz));
          g *= s_dc[xx] * dcy * s_dc[Nx + l];
        }
      }
      s_g[l * Nx + xx] = g;
      if (gblk) gblk[e] = g;
    }
  };
  // the g table into LDS: from the cache when the block's key is this box (a uniform
  // decision), else made (and cached with its key)
  auto gfill = [&]() {
    bool cached = gblk != nullptr;
    if (cached) {
      const double* key = a.gkey + size_t(blk) * 9;
#pragma unroll
      for (int k = 0; k < 9; ++k) cached = cached && key[k] == box[k];
    }
    if (cached) {
#pragma unroll
      for (int k = 0; k < GU; ++k) {
        const int e = int(threadIdx.x) + k * int(blockDim.x);
        if (e < KN) {
          const int xx = int(fdiv(uint32_t(e), a.ktd)), l = e - xx * kt;
          s_g[l * Nx + xx] = gv[k];
        }
      }
    } else {
      gtable();
      if (gblk && threadIdx.x < 9) a.gkey[size_t(blk) * 9 + threadIdx.x] = box[threadIdx.x];
    }
  };
  const int last = a.ax.nst - 1;
  // first forward stage reading the lines from global memory and last inverse stage
  // writing them back, when one round of the workgroup covers each (lanes: kz fastest)
  const bool fuse_io = last >= 1 && kt * a.ax.st[0].NR <= int(blockDim.x) &&
                       kt * a.axi.st[last].NR <= int(blockDim.x);
  float2* Z;
  if (fuse_io) {
    const FFTStage& x0 = a.ax.st[0];
    const int t = threadIdx.x;
    const bool act = t < kt * x0.NR;
    const int j = int(fdiv(uint32_t(t), a.ktd)), l = t - j * kt;
    const int kz = kz0 + l;
    with_radix(x0.R, [&](auto rc) {
      constexpr int Rr = decltype(rc)::value;
      float2 v[Rr];
      {
        // unconditional loads from clamped addresses: the waits before the g table
        // then count only the deconvolution loads issued before these
        const int jc = act ? j : 0, kc = (kz < H) ? kz : H - 1;
#pragma unroll
        for (int r = 0; r < Rr; ++r) v[r] = base[size_t(jc + r * x0.NR) * xstride + kc];
      }
      store_dc();
      gfill();
      if (act) {
        if (kz >= H) {
#pragma unroll
          for (int r = 0; r < Rr; ++r) v[r] = make_float2(0.f, 0.f);
        }
        Dft<Rr>::run(v, -1.0f);
        float2* out = X + l * ps;
#pragma unroll
        for (int r = 0; r < Rr; ++r) out[j * Rr + r] = v[r];
      }
    });
    twr.store(tw, Nx);
    __syncthreads();
    Z = lds_fft(X, Y, kt, ps, a.ax, tw, -1.0f, 1, last);
  } else {
    constexpr int U = 16;   // Nx kt <= U blockDim (the plan bounds kt (Nx + 1) by 3500)
    float2 lv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + u * kFFTThreads;
      if (e < Nx * kt) {
        const int xx = int(fdiv(uint32_t(e), a.ktd)), l = e - xx * kt;
        const int kz = kz0 + l;
        lv[u] = (kz < H) ? base[xx * xstride + kz] : make_float2(0.f, 0.f);
      }
    }
    store_dc();
    gfill();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + u * kFFTThreads;
      if (e < Nx * kt) {
        const int xx = int(fdiv(uint32_t(e), a.ktd)), l = e - xx * kt;
        X[l * ps + xx] = lv[u];
      }
    }
    twr.store(tw, Nx);
    __syncthreads();
    Z = lds_fft(X, Y, kt, ps, a.ax, tw, -1.0f, 0, last);
  }
  float2* W = (Z == X) ? Y : X;
  float e_acc = 0.0f;
  // cell gradient: w |v|^2 G(k) D(f) (1/k^2 + 1/(4 alpha^2)) k k^T with k = 2 pi C^-1 f,
  // the mean over a Nyquist bin and its Hermitian partner as for g (where a signed
  // frequency is -N/2 the partner keeps it and flips the others)
  float vacc[6] = {0, 0, 0, 0, 0, 0};
  float ci[9];
  if constexpr (VIR) {
    const Cell c = cell_from_box(box);
#pragma unroll
    for (int k = 0; k < 9; ++k) ci[k] = float(2.0 * M_PI * c.inv[k]);   // 2 pi (C^-1)[b][a]
  }
  const float inv4a2v = 1.0f / (4.0f * a.alpha * a.alpha);
  const int fyv = signed_freq(y, Ny);
  const bool nyq_yv = ((Ny & 1) == 0) && (2 * fyv == -Ny);
  auto vir_point = [&](int xx, int kz, int pen, float wv2, float gg) {
    const int fxi = signed_freq(xx, Nx), fzi = signed_freq(kz, Nz);
    if (kz >= H || (fxi | fyv | fzi) == 0) return;
    const bool nx = ((Nx & 1) == 0) && (2 * fxi == -Nx);
    const bool nz = ((Nz & 1) == 0) && (2 * kz == Nz);
    const bool nyq = nx || nyq_yv || nz;
    // off the Nyquist bins the tabulated g is this point's own; on them each of the
    // bin and its partner needs its own G(k)
    const float dc = nyq ? s_dc[xx] * a.dcy[y] * s_dc[Nx + pen] : 0.0f;
    auto add = [&](float fx, float fy, float fz, float scale) {
      const float k0 = ci[0] * fx + ci[1] * fy + ci[2] * fz;
      const float k1 = ci[3] * fx + ci[4] * fy + ci[5] * fz;
      const float k2c = ci[6] * fx + ci[7] * fy + ci[8] * fz;
      const float k2 = k0 * k0 + k1 * k1 + k2c * k2c;
      const float gk = nyq ? 4.0f * float(M_PI) / k2 * expf(-k2 * inv4a2v) * dc : gg;
      const float f = scale * gk * (1.0f / k2 + inv4a2v);
      vacc[0] = fmaf(f, k0 * k0, vacc[0]);
      vacc[1] = fmaf(f, k1 * k1, vacc[1]);
      vacc[2] = fmaf(f, k2c * k2c, vacc[2]);
      vacc[3] = fmaf(f, k0 * k1, vacc[3]);
      vacc[4] = fmaf(f, k0 * k2c, vacc[4]);
      vacc[5] = fmaf(f, k1 * k2c, vacc[5]);
    };
    const float fx = float(fxi), fy = float(fyv), fz = float(fzi);
    if (nyq) {
      add(fx, fy, fz, 0.5f * wv2);
      add(nx ? fx : -fx, nyq_yv ? fy : -fy, nz ? fz : -fz, 0.5f * wv2);
    } else {
      add(fx, fy, fz, wv2);
    }
  };
  {
    const FFTStage& st = a.ax.st[last];
    const int NR = st.NR;
    for (int t = threadIdx.x; t < kt * NR; t += blockDim.x) {
      const int pen = int(fdiv(uint32_t(t), st.nr));
      const int j = t - pen * NR;
      const float2* in = Z + pen * ps;
      float2* out = W + pen * ps;
      const float* gl = s_g + pen * Nx;
      const int kz = kz0 + pen;
      const float wgt = (kz == 0 || (((Nz & 1) == 0) && 2 * kz == Nz)) ? 1.0f : 2.0f;
      // g, and the energy partial wgt g |v|^2 of the value it scales
      auto gm = [&](int i, float2 v) -> float {
        const float gg = gl[i];
        if (epart) e_acc = fmaf(wgt * gg, v.x * v.x + v.y * v.y, e_acc);
        if constexpr (VIR) vir_point(i, kz, pen, wgt * (v.x * v.x + v.y * v.y), gg);
        return gg;
      };
      with_radix(st.R, [&](auto rc) { x_middle<decltype(rc)::value>(in, out, j, NR, tw, gm); });
    }
  }
  __syncthreads();
  if (fuse_io) {
    const float2* Rin = lds_fft(W, Z, kt, ps, a.axi, tw, +1.0f, 1, last);
    const FFTStage& xl = a.axi.st[last];
    const int t = threadIdx.x;
    if (t < kt * xl.NR) {
      const int j = int(fdiv(uint32_t(t), a.ktd)), l = t - j * kt;
      const int kz = kz0 + l;
      const int jq = int(fdiv(uint32_t(j), xl.ns)), kk = j - jq * xl.Ns;
      const float2* in = Rin + l * ps;
      with_radix(xl.R, [&](auto rc) {
        constexpr int Rr = decltype(rc)::value;
        stockham_butterfly_io<Rr, true>(
            [&](int i) { return in[i]; },
            [&](int i, float2 v) {
              if (kz < H) base[size_t(i) * xstride + kz] = v;
            },
            j, kk, jq, xl.Ns, xl.NR, xl.step, tw, 1.0f);
      });
    }
  } else {
    const float2* R = lds_fft(W, Z, kt, ps, a.axi, tw, +1.0f, 1, -1);
    for (int e = threadIdx.x; e < Nx * kt; e += blockDim.x) {
      const int xx = e / kt, l = e - xx * kt;
      const int kz = kz0 + l;
      if (kz < H) base[xx * xstride + kz] = R[l * ps + xx];
    }
  }
  if (epart) {
    const double s = block_sum(double(e_acc), red);
    if (threadIdx.x == 0) epart[blk] = s;
  }
  if constexpr (VIR) {
    __shared__ double vred[16 * 6];
    double v[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = vacc[k];
    block_sums<6>(v, vred);
    if (threadIdx.x == 0)
#pragma unroll
      for (int k = 0; k < 6; ++k) a.vpart[6 * blk + k] = v[k];
  }
}


__global__ void __launch_bounds__(kSlabThreads) k_slab_fwd(SlabArgs a) {
  slab_fwd_body(a, blockIdx.x);
}

__global__ void __launch_bounds__(kSlabThreads) k_slab_inv(SlabArgs a) {
  slab_inv_body(a, blockIdx.x);
}

template <int MODE>
__global__ void __launch_bounds__(kFFTThreads) k_fftx_fused(XArgs a) {
  fftx_body<MODE>(a, xcd_item(blockIdx.x, gridDim.x), a.box, a.epart);
}

// Batched passes: work item (box, x-plane) or (box, x-pass workgroup); per-box
// argument templates in device memory; workgroups loop over the items.
__global__ void __launch_bounds__(kSlabThreads) k_slab_fwd_batch(const SlabArgs* args,
                                                                 const int2* items, int n) {
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = items[it];
    slab_fwd_body(args[w.x], w.y);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kSlabThreads) k_slab_inv_batch(const SlabArgs* args,
                                                                 const int2* items, int n) {
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = items[it];
    slab_inv_body(args[w.x], w.y);
    __syncthreads();
  }
}

template <int MODE>
__global__ void __launch_bounds__(kFFTThreads) k_fftx_batch(const XArgs* args, const int2* items,
                                                            int n, const double* box, int energy) {
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = items[it];
    const XArgs& a = args[w.x];
    fftx_body<MODE>(a, w.y, box + 9 * w.x, energy ? a.epart : nullptr);
    __syncthreads();
  }
}

// Spread fused with the forward slab transform (Eq. charge_dipole_assign, then the
// z and y halves of Eq. fft): one workgroup per x-plane X.  It takes from the bins
// every atom whose stencil covers the plane (anchors b with X in [b - lo, b - lo +
// p - 1]: the bin layers along x that hold them, and the overflow list), adds the
// atom's p x p footprint in the plane into an LDS copy of the plane, and transforms
// the plane in place.  The plane carries p - 1 extra rows and columns, so that a
// stencil never wraps: padded point (b_y + j, b_z + k) holds stencil point (j, k)
// of an atom anchored at (b_y, b_z); the extra rows and columns are folded into
// their periodic images as the transform reads the plane.  Every contribution is
// the tile spread's own value and is added as the same 64-bit fixed-point word, so
// the plane's sums, and hence the spectrum, equal those of the tile spread followed
// by the slab transform bit for bit.
struct SpreadSlabArgs {
  SlabArgs sl;             // the plane's transform (sl.src unused)
  int N[3];
  int B[3];
  int nb[3];
  int cap;
  const int* count;
  const int* ovf_count;
  const unsigned* cmax;
  const float* rec;
  long long ovf_base;      // record index of the overflow list
  int PY, PZ;              // padded plane: N_y + p - 1 rows of N_z + p - 1 words
  int abuf;                // float2 words before the plane (the transform's first buffer)
  int nscan_max;           // bins a plane may scan
  int map_cap;             // slots of the item -> bin map
  int hits_cap;            // entries of the hit list (>= 2 kFusedSlotsPerThread blockDim)
};

// TREC: the records are tangent records (q, mu, v_q, v_r, v_mu) and the density is
// the forward one (DEG 1): its coefficients q, J mu are formed from them as the
// forward binning forms them.
template <int P, int DEG, bool TREC>
__device__ __forceinline__ void spread_slab_body(const SpreadSlabArgs& a, const int X,
                                                 const double* box) {
  static_assert(!TREC || DEG == 1, "tangent records serve the forward density");
  constexpr int lo = (P - 1) / 2;
  extern __shared__ float2 sm[];
  const int tid = threadIdx.x;
  const int nthr = int(blockDim.x);
  const int Ny = a.N[1], Nz = a.N[2];
  // LDS: twiddles | first transform buffer, which holds the scan, map and hit list
  // while atoms are added | the padded plane, later the second transform buffer
  float2* twz = sm;
  float2* twy = twz + Nz;
  float2* A = twy + Ny;
  unsigned long long* plane = reinterpret_cast<unsigned long long*>(A + a.abuf);
  float2* B = reinterpret_cast<float2*>(plane);
  int* s_off = reinterpret_cast<int*>(A);
  int* s_bin = s_off + a.nscan_max + 2;
  uint16_t* s_map = reinterpret_cast<uint16_t*>(s_bin + a.nscan_max + 2);
  int* s_hits = reinterpret_cast<int*>(s_map + a.map_cap);
  __shared__ float s_J[(DEG == 2 || TREC) ? 9 : 1];
  __shared__ int s_nh;
  __shared__ float s_cw[4 * P * P];           // whole-number spline pieces (x weights)
  __shared__ int s_wsum[kSlabThreads / 64];   // per-wavefront sums of the scan
  Twiddles<kSlabThreads> tz, ty;
  constexpr int kTab = spline_offset(P);
  if (tid < 4 * P * P) s_cw[tid] = c_spline_whole.coef[kTab + tid];
  tz.load(a.sl.twz, Nz);
  ty.load(a.sl.twy, Ny);
  if ((DEG == 2 || TREC) && tid == 0) {
    float J[3][3];
    jacobian(cell_from_box(box), a.N, J);
#pragma unroll
    for (int i = 0; i < 9; ++i) s_J[i] = J[i / 3][i % 3];
  }
  // the bin layers along x of the anchors X + lo - P + 1 .. X + lo (cyclic): from the
  // first anchor's layer on, nl of them
  const int b0 = wrapn(X + lo - P + 1, a.N[0]);
  const int k0 = b0 / a.B[0], k1 = wrapn(X + lo, a.N[0]) / a.B[0];
  int nl;
  if (b0 + P - 1 < a.N[0]) nl = k1 - k0 + 1;
  else nl = (k1 < k0) ? a.nb[0] - k0 + k1 + 1 : a.nb[0];
  nl = min(nl, a.nb[0]);
  const int nyz = a.nb[1] * a.nb[2];
  const int nscan = nl * nyz;                 // <= a.nscan_max (host guarantees)
  load_slot_counts(
      nscan,
      [&](int e) {
        const int li = e / nyz;
        return ((k0 + li) % a.nb[0]) * nyz + (e - li * nyz);
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
  const int pvol = a.PY * a.PZ;
  for (int e = tid; e < pvol; e += nthr) plane[e] = 0ull;
  __syncthreads();
  int total;
  const bool mapped = scan_slot_counts(nscan, s_off, s_wsum, s_map, a.map_cap, total);
  auto record_of = [&](int item) {
    return scanned_record(item, mapped, nscan, s_off, s_bin, s_map, a.cap, a.ovf_base);
  };
  // one atom: its footprint in the padded plane (stencil row iy of an atom anchored at
  // b_y in padded row b_y + iy)
  auto add_atom = [&](size_t ri) {
    add_atom_plane<P, DEG, TREC>(a.rec, ri, s_J, s_cw, X, a.N[0], scale, plane, a.PZ,
                                 [](int by, int iy) { return by + iy; }, 0x7fffffff);
  };

  // rounds of kSlotsPerThread scanned slots per thread (their anchor words loaded
  // together): the atoms whose stencil covers the plane are listed; the list is
  // drained (one atom per thread) when another round might not fit and after the
  // last round
  constexpr int U = kFusedSlotsPerThread;
  for (int r0 = 0; r0 < total; r0 += U * nthr) {
    size_t ri[U];
    int pk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int item = r0 + u * nthr + tid;
      ri[u] = (item < total) ? record_of(item) : size_t(0);
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
        hit = d < P;
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
  // the extra columns, then the extra rows, added into their periodic images: mesh
  // point (y, z) sits at padded (y + lo, z + lo), and padded column c < lo is column
  // c + N_z, column c >= lo + N_z is c - N_z (rows alike).  Each image word takes one
  // word per pass (N >= p keeps the two image ranges apart), and 64-bit sums do not
  // depend on their order.
  {
    constexpr int ne = P - 1;
    for (int e = tid; e < a.PY * ne; e += nthr) {
      const int py = e / ne, c = e - py * ne;
      const int src = (c < lo) ? c : c + Nz;
      unsigned long long* row = plane + py * a.PZ;
      row[(c < lo) ? src + Nz : src - Nz] += row[src];
    }
    __syncthreads();
    for (int e = tid; e < ne * Nz; e += nthr) {
      const int r = e / Nz, z = e - r * Nz + lo;
      const int src = (r < lo) ? r : r + Ny;
      plane[((r < lo) ? src + Ny : src - Ny) * a.PZ + z] += plane[src * a.PZ + z];
    }
    __syncthreads();
  }
  // the plane's value at (y, z)
  const double inv_scale = 1.0 / (double(scale) * double(kWhole3));
  auto value = [&](int y, int z) {
    return from_fixed((long long)plane[(y + lo) * a.PZ + z + lo], inv_scale);
  };
  slab_fwd_run(a.sl, X, value, tz, ty, twz, twy, A, B);
}

template <int P, int DEG, bool TREC>
__global__ void __launch_bounds__(kSlabThreads) k_spread_slab(SpreadSlabArgs a, const double* box) {
  spread_slab_body<P, DEG, TREC>(a, xcd_item(blockIdx.x, gridDim.x), box);
}

}  // namespace

namespace {

XArgs make_x_args(const DevPlan& d, const double* box, bool energy) {
  XArgs x;
  x.ax = d.ax[0]; x.tw = d.twiddle[0];
  reverse_plan(d.ax[0], x.axi);
  for (int k = 0; k < 3; ++k) x.N[k] = d.N[k];
  x.H = d.H; x.kt = d.ktile; x.ktd = make_fast_div(d.ktile); x.spec = d.spec; x.box = box;
  x.dcx = d.deconv[0]; x.dcy = d.deconv[1]; x.dcz = d.deconv[2];
  x.alpha = d.alpha;
  x.epart = energy ? d.epart : nullptr;
  x.vpart = nullptr;
  x.alx = d.alias[0]; x.aly = d.alias[1]; x.alz = d.alias[2];
  x.gcache = d.gcache; x.gkey = d.gkey;
  return x;
}

size_t x_lds(const DevPlan& d) {
  return sizeof(float2) * (d.N[0] + 2 * d.ktile * (d.N[0] + 1)) + sizeof(float) * d.N[0] * d.ktile +
         sizeof(float) * (d.N[0] + d.ktile) * (d.opt ? 4 : 1);
}

SlabArgs make_slab_args(const DevPlan& d, float* out) {
  SlabArgs sa;
  sa.ay = d.ax[1]; sa.az = d.ax[2]; sa.twy = d.twiddle[1]; sa.twz = d.twiddle[2];
  sa.H = d.H; sa.nzd = make_fast_div(d.N[2]); sa.hd = make_fast_div(d.H);
  sa.src = d.rho; sa.spec = d.spec; sa.dst = out;
  return sa;
}

inline dim3 fft_batch_grid(int items, int cap) {
  return dim3(items < cap ? (items > 0 ? items : 1) : cap);
}

}  // namespace

hipError_t fft_batch_build(const DevPlan* plans, int nbox, FFTBatch& t) {
  t = FFTBatch();
  std::vector<SlabArgs> s0(nbox), s1(nbox);
  std::vector<XArgs> xa(nbox);
  std::vector<int2> si, xi;
  t.opt = nbox > 0 && plans[0].opt;
  for (int b = 0; b < nbox; ++b) {
    const DevPlan& d = plans[b];
    if (!d.slab || d.opt != t.opt) return hipErrorInvalidValue;
    s0[b] = make_slab_args(d, d.phi);
    s1[b] = make_slab_args(d, d.rho);
    xa[b] = make_x_args(d, nullptr, true);
    for (int x = 0; x < d.N[0]; ++x) si.push_back(make_int2(b, x));
    for (int k = 0; k < fftx_blocks(d); ++k) xi.push_back(make_int2(b, k));
    if (d.slab_lds > t.slab_lds) t.slab_lds = d.slab_lds;
    if (x_lds(d) > t.x_lds) t.x_lds = x_lds(d);
  }
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t r) { if (r != hipSuccess && e == hipSuccess) e = r; };
  ok(upload(&t.slab[0], s0.data(), sizeof(SlabArgs) * nbox));
  ok(upload(&t.slab[1], s1.data(), sizeof(SlabArgs) * nbox));
  ok(upload(&t.x, xa.data(), sizeof(XArgs) * nbox));
  ok(upload(reinterpret_cast<void**>(&t.slab_items), si.data(), sizeof(int2) * si.size()));
  ok(upload(reinterpret_cast<void**>(&t.x_items), xi.data(), sizeof(int2) * xi.size()));
  t.n_slab_items = int(si.size());
  t.n_x_items = int(xi.size());
  if (e == hipSuccess) e = enable_slab_lds(t.slab_lds);
  return e;
}

void fft_batch_free(FFTBatch& t) {
  void* ptrs[] = {t.slab[0], t.slab[1], t.x, t.slab_items, t.x_items};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  t = FFTBatch();
}

hipError_t launch_convolve_batch(const FFTBatch& t, hipStream_t s, const double* box, bool to_phi,
                                 bool energy) {
  const SlabArgs* sa = static_cast<const SlabArgs*>(t.slab[to_phi ? 0 : 1]);
  hipLaunchKernelGGL(k_slab_fwd_batch, fft_batch_grid(t.n_slab_items, 512), dim3(kSlabThreads),
                     t.slab_lds, s, sa, t.slab_items, t.n_slab_items);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (t.opt)
    hipLaunchKernelGGL(k_fftx_batch<2>, fft_batch_grid(t.n_x_items, 2048), dim3(kFFTThreads),
                       t.x_lds, s, static_cast<const XArgs*>(t.x), t.x_items, t.n_x_items, box,
                       energy ? 1 : 0);
  else
    hipLaunchKernelGGL(k_fftx_batch<0>, fft_batch_grid(t.n_x_items, 2048), dim3(kFFTThreads),
                       t.x_lds, s, static_cast<const XArgs*>(t.x), t.x_items, t.n_x_items, box,
                       energy ? 1 : 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_slab_inv_batch, fft_batch_grid(t.n_slab_items, 512), dim3(kSlabThreads),
                     t.slab_lds, s, sa, t.slab_items, t.n_slab_items);
  return hipGetLastError();
}

hipError_t launch_convolve(const DevPlan& d, hipStream_t s, const double* box, float* out,
                           bool energy, KTimer* tm, double* vpart, bool from_spec) {
  hipError_t err;
  if (from_spec && !d.slab) return hipErrorInvalidValue;
  XArgs x = make_x_args(d, box, energy);
  x.vpart = vpart;
  const size_t xsh = x_lds(d);
  // timed kinds: a kind spanning two launches records its start with the first
  // and its stop with the second
  const LaunchEvents* er = (tm && !from_spec) ? tm->next(PME_K_FFT_R2C) : nullptr;
  const LaunchEvents* ex = tm ? tm->next(PME_K_FFT_X) : nullptr;
  const LaunchEvents* ei = tm ? tm->next(PME_K_FFT_C2R) : nullptr;
  LaunchEvents er0, er1, ei0, ei1;
  if (er) { er0.start = er->start; er1.stop = er->stop; }
  if (ei) { ei0.start = ei->start; ei1.stop = ei->stop; }

  if (d.slab) {
    const SlabArgs sa = make_slab_args(d, out);
    if (!from_spec) {
      launch_k(er, k_slab_fwd, dim3(d.N[0]), dim3(kSlabThreads), d.slab_lds, s, sa);
      if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    if (vpart) launch_k(ex, k_fftx_fused<1>, dim3(fftx_blocks(d)), dim3(kFFTThreads), xsh, s, x);
    else if (d.opt) launch_k(ex, k_fftx_fused<2>, dim3(fftx_blocks(d)), dim3(kFFTThreads), xsh, s, x);
    else launch_k(ex, k_fftx_fused<0>, dim3(fftx_blocks(d)), dim3(kFFTThreads), xsh, s, x);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    launch_k(ei, k_slab_inv, dim3(d.N[0]), dim3(kSlabThreads), d.slab_lds, s, sa);
    return hipGetLastError();
  }

  const int rows = d.N[0] * d.N[1];
  ZArgs z;
  z.ax = d.ax[2]; z.tw = d.twiddle[2]; z.rows = rows; z.H = d.H; z.rp = d.rows_per_block;
  z.src = d.rho; z.spec = d.spec; z.dst = out;
  z.nd = make_fast_div(d.N[2]);
  const int zb = fftz_blocks(d);
  const size_t zsh_f = sizeof(float2) * (d.N[2] + d.rows_per_block * d.N[2]);
  YArgs y;
  y.ax = d.ax[1]; y.tw = d.twiddle[1]; y.Ny = d.N[1]; y.H = d.H; y.kt = d.ytile; y.spec = d.spec;
  y.ktd = make_fast_div(d.ytile);
  const size_t ysh = sizeof(float2) * (d.N[1] + 2 * d.ytile * (d.N[1] + 1));

  launch_k(er ? &er0 : nullptr, k_fftz_r2c, dim3(zb), dim3(kFFTThreads), zsh_f, s, z);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  y.sign = -1.0f;
  launch_k(er ? &er1 : nullptr, k_ffty, dim3(ffty_blocks(d)), dim3(kFFTThreads), ysh, s, y);
  if ((err = hipGetLastError()) != hipSuccess) return err;

  if (vpart) launch_k(ex, k_fftx_fused<1>, dim3(fftx_blocks(d)), dim3(kFFTThreads), xsh, s, x);
  else if (d.opt) launch_k(ex, k_fftx_fused<2>, dim3(fftx_blocks(d)), dim3(kFFTThreads), xsh, s, x);
  else launch_k(ex, k_fftx_fused<0>, dim3(fftx_blocks(d)), dim3(kFFTThreads), xsh, s, x);
  if ((err = hipGetLastError()) != hipSuccess) return err;

  y.sign = +1.0f;
  launch_k(ei ? &ei0 : nullptr, k_ffty, dim3(ffty_blocks(d)), dim3(kFFTThreads), ysh, s, y);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  const size_t zsh_i = sizeof(float2) * (d.N[2] + d.rows_per_block * d.H + d.rows_per_block * d.N[2]);
  launch_k(ei ? &ei1 : nullptr, k_fftz_c2r, dim3(zb), dim3(kFFTThreads), zsh_i, s, z);
  return hipGetLastError();
}

hipError_t launch_spread_slab(const DevPlan& d, hipStream_t s, int set, bool tangent,
                              const double* box, const LaunchEvents* ev, const RecordSource* from) {
  if (!d.fused || (from && (tangent || !from->d || !from->cmax))) return hipErrorInvalidValue;
  SpreadSlabArgs a;
  a.sl = make_slab_args(d, nullptr);
  for (int k = 0; k < 3; ++k) { a.N[k] = d.N[k]; a.B[k] = d.B[k]; a.nb[k] = d.nb[k]; }
  // the bins (same geometry in both views of a plan) and the scale
  const DevPlan& r = from ? *from->d : d;
  const int rs = from ? from->set : set;
  a.cap = r.cap;
  a.count = r.count[rs]; a.ovf_count = r.ovf_count[rs];
  a.cmax = from ? from->cmax : d.cmax[set];
  a.rec = r.rec; a.ovf_base = r.ovf_base;
  a.PY = d.N[1] + d.p - 1;
  a.PZ = d.N[2] + d.p - 1;
  a.abuf = d.fused_abuf;
  a.nscan_max = d.fused_nscan;
  a.map_cap = kFusedMap;
  a.hits_cap = kFusedHits;
  const dim3 g(d.N[0]), b(kSlabThreads);
  const size_t sh = d.fused_lds;
#define PME_F(P)                                                                   \
  case P:                                                                          \
    if (tangent) launch_k(ev, k_spread_slab<P, 2, false>, g, b, sh, s, a, box);     \
    else if (from) launch_k(ev, k_spread_slab<P, 1, true>, g, b, sh, s, a, box);    \
    else launch_k(ev, k_spread_slab<P, 1, false>, g, b, sh, s, a, box);             \
    break;
  switch (d.p) {
    PME_F(1) PME_F(2) PME_F(3) PME_F(4) PME_F(5) PME_F(6) PME_F(7)
    default: return hipErrorInvalidValue;
  }
#undef PME_F
  return hipGetLastError();
}

hipError_t enable_slab_lds(size_t bytes) {
  // The limit is per kernel, not per plan: raise it to the largest slab any plan
  // may use, so that a later plan with smaller planes does not lower it.
  if (bytes > size_t(kSlabLdsMax)) return hipErrorInvalidValue;
  const void* fns[] = {reinterpret_cast<const void*>(k_slab_fwd),
                       reinterpret_cast<const void*>(k_slab_inv),
                       reinterpret_cast<const void*>(k_slab_fwd_batch),
                       reinterpret_cast<const void*>(k_slab_inv_batch),
#define PME_F(P)                                                   \
  reinterpret_cast<const void*>(k_spread_slab<P, 1, false>),       \
      reinterpret_cast<const void*>(k_spread_slab<P, 1, true>),    \
      reinterpret_cast<const void*>(k_spread_slab<P, 2, false>),
                       PME_F(1) PME_F(2) PME_F(3) PME_F(4) PME_F(5) PME_F(6) PME_F(7)
#undef PME_F
  };
  for (const void* f : fns) {
    const hipError_t e =
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kSlabLdsMax);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace pme
