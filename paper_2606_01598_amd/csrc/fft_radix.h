// Radix stages of the mesh FFT (the 3D DFT of Eq. fft and its inverse, Eq. ifft),
// written once for the device passes and for a host check of the same code.
//
// A length-N transform is a sequence of Stockham autosort stages, radix R_s each,
// N = prod R_s.  Stage s (Ns = product of the earlier radices) takes inputs
// in[j + r N/R], multiplies them by the twiddles w_N^{r k step}, k = j mod Ns,
// applies an R-point DFT and writes out[(j / Ns) Ns R + k + r Ns].  The R-point DFTs
// are done in registers: 2, 3, 4 and 5 directly, 6, 8 and 10 as R1 x R2
// Cooley-Tukey splits with compile-time internal twiddles.  Fewer, larger stages
// mean fewer LDS round trips and workgroup barriers per transform.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "kernels.h"

namespace pme {

// ---------------------------------------------------------------------------
// compile-time trigonometry (Taylor series on [-pi, pi]) for internal twiddles
// ---------------------------------------------------------------------------
constexpr double kTwoPi = 6.283185307179586476925286766559;

constexpr double ce_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 24; ++n) {
    term *= -x * x / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double ce_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 24; ++n) {
    term *= -x * x / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
// 2 pi m / R reduced to [-pi, pi]
constexpr double ce_angle(int m, int R) {
  m %= R;
  if (2 * m > R) m -= R;
  return kTwoPi * double(m) / double(R);
}

// A constant of the transform split into a float and the float of its remainder,
// so that x * (hi + lo) is formed with the constant accurate to about 2^-48.  A
// constant rounded to one float changes every product it forms in the same
// direction, so the transform would no longer preserve the norm on average
// (Parseval: sum |X|^2 = N sum |x|^2) but scale it by 1 + O(1e-8) per stage; the
// k-space energy sum of Eq. energy_recip would inherit that bias.
struct KConst {
  float hi, lo;
};
constexpr KConst kconst(double v) { return KConst{float(v), float(v - double(float(v)))}; }
// x * k
__host__ __device__ __forceinline__ float kmul(float x, KConst k) { return fmaf(x, k.hi, x * k.lo); }
// x * k + acc
__host__ __device__ __forceinline__ float kfma(float x, KConst k, float acc) {
  return fmaf(x, k.hi, fmaf(x, k.lo, acc));
}

__host__ __device__ __forceinline__ float2 c_add(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__host__ __device__ __forceinline__ float2 c_sub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
__host__ __device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// i s a (s = +-1)
__host__ __device__ __forceinline__ float2 c_imul(float2 a, float s) {
  return make_float2(-s * a.y, s * a.x);
}
// a e^{s 2 pi i M / R}
template <int R, int M>
__host__ __device__ __forceinline__ float2 c_twiddle(float2 a, float s) {
  constexpr KConst c = kconst(ce_cos(ce_angle(M, R)));
  constexpr KConst sn = kconst(ce_sin(ce_angle(M, R)));
  if constexpr (M % R == 0) {
    return a;
  } else if constexpr (c.lo == 0.0f && sn.lo == 0.0f) {
    // exact constants (quarter and half turns, 1/2 ...)
    const float ss = s * sn.hi;
    return make_float2(a.x * c.hi - a.y * ss, a.x * ss + a.y * c.hi);
  } else {
    // s = +-1: s * (a * sn) is exact
    return make_float2(kfma(a.x, c, -s * kmul(a.y, sn)), kfma(a.y, c, s * kmul(a.x, sn)));
  }
}

template <int... Is, class F>
__host__ __device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
// f(integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time
template <int N, class F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// In-place R-point DFT: v[k] <- sum_n v[n] e^{s 2 pi i n k / R}.
template <int R>
struct Dft;

template <>
struct Dft<2> {
  __host__ __device__ static __forceinline__ void run(float2 (&v)[2], float) {
    const float2 a = v[0], b = v[1];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, b);
  }
};

template <>
struct Dft<3> {
  __host__ __device__ static __forceinline__ void run(float2 (&v)[3], float s) {
    constexpr float c = -0.5f;
    constexpr KConst sn = kconst(0.86602540378443864676);
    const float2 t1 = c_add(v[1], v[2]);
    const float2 t2 = make_float2(v[0].x + c * t1.x, v[0].y + c * t1.y);
    const float2 d = c_sub(v[1], v[2]);
    const float2 t3 = c_imul(make_float2(kmul(d.x, sn), kmul(d.y, sn)), s);
    v[0] = c_add(v[0], t1);
    v[1] = c_add(t2, t3);
    v[2] = c_sub(t2, t3);
  }
};

template <>
struct Dft<4> {
  __host__ __device__ static __forceinline__ void run(float2 (&v)[4], float s) {
    const float2 a = c_add(v[0], v[2]), b = c_sub(v[0], v[2]);
    const float2 c = c_add(v[1], v[3]), d = c_imul(c_sub(v[1], v[3]), s);
    v[0] = c_add(a, c);
    v[1] = c_add(b, d);
    v[2] = c_sub(a, c);
    v[3] = c_sub(b, d);
  }
};

template <>
struct Dft<5> {
  __host__ __device__ static __forceinline__ void run(float2 (&v)[5], float s) {
    constexpr KConst c1 = kconst(0.30901699437494742410), c2 = kconst(-0.80901699437494742410);
    constexpr KConst s1 = kconst(0.95105651629515357212), s2 = kconst(0.58778525229247312917);
    const float2 t1 = c_add(v[1], v[4]), t2 = c_add(v[2], v[3]);
    const float2 t3 = c_sub(v[1], v[4]), t4 = c_sub(v[2], v[3]);
    const float2 a1 = make_float2(kfma(t1.x, c1, kfma(t2.x, c2, v[0].x)),
                                  kfma(t1.y, c1, kfma(t2.y, c2, v[0].y)));
    const float2 a2 = make_float2(kfma(t1.x, c2, kfma(t2.x, c1, v[0].x)),
                                  kfma(t1.y, c2, kfma(t2.y, c1, v[0].y)));
    const float2 b1 = c_imul(make_float2(kfma(t3.x, s1, kmul(t4.x, s2)),
                                         kfma(t3.y, s1, kmul(t4.y, s2))), s);
    const float2 b2 = c_imul(make_float2(kfma(t3.x, s2, -kmul(t4.x, s1)),
                                         kfma(t3.y, s2, -kmul(t4.y, s1))), s);
    v[0] = c_add(v[0], c_add(t1, t2));
    v[1] = c_add(a1, b1);
    v[4] = c_sub(a1, b1);
    v[2] = c_add(a2, b2);
    v[3] = c_sub(a2, b2);
  }
};

// R = R1 R2, n = R2 n1 + n2, k = k1 + R1 k2:
//   X[k1 + R1 k2] = sum_n2 w_R2^{n2 k2} w_R^{n2 k1} sum_n1 v[R2 n1 + n2] w_R1^{n1 k1}
template <int R1, int R2>
struct DftSplit {
  static constexpr int R = R1 * R2;
  __host__ __device__ static __forceinline__ void run(float2 (&v)[R], float s) {
    float2 y[R];   // y[n2 R1 + k1]
    static_for<R2>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      float2 t[R1];
      static_for<R1>([&](auto n1c) { t[decltype(n1c)::value] = v[R2 * decltype(n1c)::value + n2]; });
      Dft<R1>::run(t, s);
      static_for<R1>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        y[n2 * R1 + k1] = c_twiddle<R, n2 * k1>(t[k1], s);
      });
    });
    static_for<R1>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      float2 u[R2];
      static_for<R2>([&](auto n2c) { u[decltype(n2c)::value] = y[decltype(n2c)::value * R1 + k1]; });
      Dft<R2>::run(u, s);
      static_for<R2>([&](auto k2c) { v[k1 + R1 * decltype(k2c)::value] = u[decltype(k2c)::value]; });
    });
  }
};

template <>
struct Dft<6> : DftSplit<2, 3> {};
template <>
struct Dft<8> : DftSplit<2, 4> {};
template <>
struct Dft<10> : DftSplit<2, 5> {};

// Radices a stage may use, in the order the planner prefers at equal stage count.
constexpr int kRadices[] = {10, 8, 6, 5, 4, 3, 2};

// One radix-R Stockham butterfly (see the header comment) reading its inputs through
// ld(index in the pencil) and writing through st(index, value); the twiddle table
// holds e^{-2 pi i t / N}, t < N; s = -1 forward, +1 inverse.  TW = false for a first
// stage (Ns = 1, k = 0: no twiddles, the table need not be loaded yet).
template <int R, bool TW, class LD, class ST>
__host__ __device__ __forceinline__ void stockham_butterfly_io(LD&& ld, ST&& st, int j, int k,
                                                               int jq, int Ns, int NR, int step,
                                                               const float2* __restrict__ tw,
                                                               float s) {
  float2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = ld(j + r * NR);
  if constexpr (TW) {
    const int tstep = k * step;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      float2 w = tw[r * tstep];
      w.y *= -s;
      v[r] = c_mul(v[r], w);
    }
  }
  Dft<R>::run(v, s);
  const int base = jq * Ns * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) st(base + r * Ns, v[r]);
}

// The same from and to pencils in memory.
template <int R>
__host__ __device__ __forceinline__ void stockham_butterfly(const float2* __restrict__ in,
                                                            float2* __restrict__ out, int j, int k,
                                                            int jq, int Ns, int NR, int step,
                                                            const float2* __restrict__ tw, float s) {
  stockham_butterfly_io<R, true>([&](int i) { return in[i]; },
                                 [&](int i, float2 v) { out[i] = v; }, j, k, jq, Ns, NR, step, tw, s);
}

// f(integral_constant<int, R>) for the runtime radix R of a stage.
template <class F>
__host__ __device__ __forceinline__ void with_radix(int R, F&& f) {
  switch (R) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 10: f(std::integral_constant<int, 10>{}); break;
    default: break;
  }
}

// Last forward stage, x g(k) and first inverse stage of one butterfly, in registers.
// With the inverse planned in reverse radix order, the last forward stage of radix R
// (Ns = N/R, so k = j and the twiddle step is 1) reads and writes the elements
// j + r N/R, which are exactly the inputs of the first inverse stage (Ns = 1, no
// twiddles); the inverse stage then writes out[j R + r].
template <int R, class G>
__host__ __device__ __forceinline__ void x_middle(const float2* __restrict__ in, float2* __restrict__ out,
                                         int j, int NR, const float2* __restrict__ tw, G&& g) {
  float2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = in[j + r * NR];
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = c_mul(v[r], tw[r * j]);
  Dft<R>::run(v, -1.0f);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float f = g(j + r * NR, v[r]);
    v[r].x *= f;
    v[r].y *= f;
  }
  Dft<R>::run(v, 1.0f);
#pragma unroll
  for (int r = 0; r < R; ++r) out[j * R + r] = v[r];
}

// Host: n / d helper of the device index math (m = ceil(2^32 / d)).
inline FastDiv make_fast_div(int d) {
  FastDiv f;
  f.d = uint32_t(d);
  f.m = d <= 1 ? 0u : uint32_t(((1ull << 32) + uint64_t(d) - 1) / uint64_t(d));
  return f;
}

// Host: stage plan of a length-N transform with the fewest stages (ties: the
// smallest largest radix); false if N has a prime factor above 5.
inline bool radix_plan(int N, AxisPlan& ax) {
  constexpr int nr = int(sizeof(kRadices) / sizeof(kRadices[0]));
  int best[kMaxStages], nbest = kMaxStages + 1, bestmax = 1 << 30;
  int cur[kMaxStages];
  // depth-first over non-increasing radix sequences
  struct Search {
    int* best; int* nbest; int* bestmax; int* cur;
    void go(int n, int depth, int maxr_idx, int curmax) {
      if (n == 1) {
        if (depth < *nbest || (depth == *nbest && curmax < *bestmax)) {
          *nbest = depth;
          *bestmax = curmax;
          for (int i = 0; i < depth; ++i) best[i] = cur[i];
        }
        return;
      }
      if (depth >= kMaxStages || depth + 1 > *nbest) return;
      for (int i = maxr_idx; i < nr; ++i) {
        const int r = kRadices[i];
        if (n % r) continue;
        cur[depth] = r;
        go(n / r, depth + 1, i, curmax > r ? curmax : r);
      }
    }
  } search{best, &nbest, &bestmax, cur};
  if (N < 1) return false;
  search.go(N, 0, 0, 1);
  if (nbest > kMaxStages) return false;
  ax.N = N;
  ax.nst = 0;
  int Ns = 1;
  for (int i = 0; i < nbest; ++i) {
    const int r = best[i];
    FFTStage& st = ax.st[ax.nst++];
    st.R = r;
    st.Ns = Ns;
    st.NR = N / r;
    st.step = N / (Ns * r);
    st.ns = make_fast_div(Ns);
    st.nr = make_fast_div(N / r);
    Ns *= r;
  }
  return true;
}

// Host: the same stages in reverse order (used for the inverse of a pass that fuses
// the last forward stage with the first inverse one).
inline void reverse_plan(const AxisPlan& f, AxisPlan& r) {
  r.N = f.N;
  r.nst = f.nst;
  int Ns = 1;
  for (int i = 0; i < f.nst; ++i) {
    const int R = f.st[f.nst - 1 - i].R;
    FFTStage& st = r.st[i];
    st.R = R;
    st.Ns = Ns;
    st.NR = f.N / R;
    st.step = f.N / (Ns * R);
    st.ns = make_fast_div(Ns);
    st.nr = make_fast_div(f.N / R);
    Ns *= R;
  }
}

}  // namespace pme
