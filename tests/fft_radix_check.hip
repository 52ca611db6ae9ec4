// Host build of the FFT radix stages (csrc/fft_radix.h): the in-register R-point
// DFTs and whole Stockham transforms planned by radix_plan, against a direct
// double-precision DFT.  Built with hipcc --offload-host-only by
// test_fft_radix_cpu.py; prints one line per case:
//   dft R s err | plan N r1,r2,... | fft N s err | fused N err | noplan N
#include <math.h>
#include <stdio.h>

#include <random>
#include <vector>

#include "../paper_2606_01598_amd/csrc/fft_radix.h"

using pme::AxisPlan;

static double max_rel(const std::vector<float2>& a, const std::vector<double>& re,
                      const std::vector<double>& im) {
  double num = 0.0, den = 0.0;
  for (size_t i = 0; i < a.size(); ++i) {
    num = fmax(num, hypot(a[i].x - re[i], a[i].y - im[i]));
    den = fmax(den, hypot(re[i], im[i]));
  }
  return num / den;
}

static void direct_dft(const std::vector<float2>& x, double s, std::vector<double>& re,
                       std::vector<double>& im) {
  const int n = int(x.size());
  re.assign(n, 0.0);
  im.assign(n, 0.0);
  for (int k = 0; k < n; ++k)
    for (int t = 0; t < n; ++t) {
      const double a = s * 2.0 * M_PI * double((long(t) * k) % n) / n;
      re[k] += x[t].x * cos(a) - x[t].y * sin(a);
      im[k] += x[t].x * sin(a) + x[t].y * cos(a);
    }
}

template <int R>
static void check_dft(std::mt19937& g) {
  std::normal_distribution<float> nd;
  for (float s : {-1.0f, 1.0f}) {
    float2 v[R];
    std::vector<float2> x(R);
    for (int r = 0; r < R; ++r) x[r] = v[r] = make_float2(nd(g), nd(g));
    pme::Dft<R>::run(v, s);
    std::vector<double> re, im;
    direct_dft(x, s, re, im);
    printf("dft %d %d %.3e\n", R, int(s), max_rel(std::vector<float2>(v, v + R), re, im));
  }
}

// one pencil through stages [s0, s1) of a plan, as the device passes run them
static std::vector<float2> stockham(const AxisPlan& ax, std::vector<float2> x, float s,
                                    const std::vector<float2>& tw, int s0 = 0, int s1 = -1) {
  if (s1 < 0) s1 = ax.nst;
  std::vector<float2> y(x.size());
  for (int i = s0; i < s1; ++i) {
    const pme::FFTStage& st = ax.st[i];
    for (int j = 0; j < st.NR; ++j) {
      const int jq = j / st.Ns, k = j - jq * st.Ns;
      switch (st.R) {
#define PME_R(R) \
  case R: pme::stockham_butterfly<R>(x.data(), y.data(), j, k, jq, st.Ns, st.NR, st.step, tw.data(), s); break;
        PME_R(2) PME_R(3) PME_R(4) PME_R(5) PME_R(6) PME_R(8) PME_R(10)
#undef PME_R
        default: break;
      }
    }
    x.swap(y);
  }
  return x;
}

// the fused x pass on one line: forward stages but the last, the last forward stage
// with x g and the first inverse stage in registers (x_middle), the remaining stages
// of the reversed plan; equals IDFT(g DFT(x)) with the unnormalised inverse (N >= 2)
static std::vector<float2> fused_pass(const AxisPlan& ax, const std::vector<float2>& x,
                                      const std::vector<float>& g, const std::vector<float2>& tw) {
  AxisPlan axi;
  pme::reverse_plan(ax, axi);
  const int last = ax.nst - 1;
  std::vector<float2> z = stockham(ax, x, -1.0f, tw, 0, last);
  std::vector<float2> w(x.size());
  const int NR = ax.st[last].NR;
  auto gf = [&](int i, float2) { return g[i]; };
  for (int j = 0; j < NR; ++j) {
    switch (ax.st[last].R) {
#define PME_R(R) \
  case R: pme::x_middle<R>(z.data(), w.data(), j, NR, tw.data(), gf); break;
      PME_R(2) PME_R(3) PME_R(4) PME_R(5) PME_R(6) PME_R(8) PME_R(10)
#undef PME_R
      default: break;
    }
  }
  return stockham(axi, w, 1.0f, tw, 1, -1);
}

int main() {
  std::mt19937 g(7);
  check_dft<2>(g);
  check_dft<3>(g);
  check_dft<4>(g);
  check_dft<5>(g);
  check_dft<6>(g);
  check_dft<8>(g);
  check_dft<10>(g);
  std::normal_distribution<float> nd;
  for (int N : {1, 2, 12, 16, 30, 48, 60, 64, 80, 96, 100, 120, 128, 160, 200, 256, 320, 1000}) {
    AxisPlan ax;
    if (!pme::radix_plan(N, ax)) {
      printf("noplan %d\n", N);
      continue;
    }
    printf("plan %d", N);
    for (int i = 0; i < ax.nst; ++i) printf("%s%d", i ? "," : " ", ax.st[i].R);
    printf("\n");
    std::vector<float2> tw(N);
    for (int t = 0; t < N; ++t) {
      const double a = -2.0 * M_PI * double(t) / double(N);
      tw[t] = make_float2(float(cos(a)), float(sin(a)));
    }
    std::vector<float2> x(N);
    for (auto& v : x) v = make_float2(nd(g), nd(g));
    for (float s : {-1.0f, 1.0f}) {
      std::vector<double> re, im;
      direct_dft(x, s, re, im);
      printf("fft %d %d %.3e\n", N, int(s), max_rel(stockham(ax, x, s, tw), re, im));
    }
    if (ax.nst >= 1) {
      std::vector<float> g(N);
      for (int i = 0; i < N; ++i) g[i] = 1.0f + 0.5f * float(std::cos(0.37 * i));
      std::vector<double> re, im;
      direct_dft(x, -1.0, re, im);
      std::vector<float2> xg(N);
      for (int i = 0; i < N; ++i) xg[i] = make_float2(float(re[i] * g[i]), float(im[i] * g[i]));
      direct_dft(xg, 1.0, re, im);
      printf("fused %d %.3e\n", N, max_rel(fused_pass(ax, x, g, tw), re, im));
    }
  }
  for (int N : {7, 14, 22, 49}) {
    AxisPlan ax;
    if (!pme::radix_plan(N, ax)) printf("noplan %d\n", N);
  }
  return 0;
}
