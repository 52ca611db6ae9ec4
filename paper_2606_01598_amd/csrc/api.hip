// C ABI of the PME library: plan construction (Sec. 2.3.1 mesh helper, FFT radix
// plans, twiddles, the 1D deconvolution factors of Eqs. Bk and influence, atom
// bins and spread tiles), and the forward / backward call sequences.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/pme.h"
#include "fft_radix.h"
#include "kernels.h"

using pme::DevPlan;

// ---- table values shared by the host (plans) and the device (pme_forward_noalloc) ----
namespace {

__host__ __device__ double sinc(double x) { return x == 0.0 ? 1.0 : sin(M_PI * x) / (M_PI * x); }

// e^{-2 pi i t / N} as a float pair: among the pairs within 3 units in the last
// place of the rounded cosine and sine, the one whose squared modulus is closest to
// 1 (ties: closest to the exact values).  Rounding each component on its own leaves
// |w|^2 - 1 of order 1e-8 with a sign that does not average out over the few
// twiddles a short transform uses, so the transform would scale the norm of its
// output (and the k-space energy) by a small bias; the phase moves by at most a few
// units in the last place instead.
__host__ __device__ float2 twiddle(int t, int N) {
  const double ang = -2.0 * M_PI * double(t) / double(N);
  const double c0 = cos(ang), s0 = sin(ang);
  float2 best = make_float2(float(c0), float(s0));
  double score = 1e300;
  float c = float(c0);
  for (int i = 0; i < 3; ++i) c = nextafterf(c, -2.0f);
  for (int i = -3; i <= 3; ++i, c = nextafterf(c, 2.0f)) {
    float sv = float(s0);
    for (int k = 0; k < 3; ++k) sv = nextafterf(sv, -2.0f);
    for (int k = -3; k <= 3; ++k, sv = nextafterf(sv, 2.0f)) {
      const double m = fabs(double(c) * c + double(sv) * sv - 1.0);
      const double d = fabs(double(c) - c0) + fabs(double(sv) - s0);
      const double sc = m + 1e-3 * d;
      if (sc < score) {
        score = sc;
        best = make_float2(c, sv);
      }
    }
  }
  return best;
}

// Deconvolution factor |sinc(f/N)|^(-2 gamma p) of Eqs. Bk and influence at index t
// (signed frequency f = t - N [t >= ceil(N/2)]).
__host__ __device__ float deconv_factor(int t, int N, int p, double gamma) {
  const int f = (t >= (N + 1) / 2) ? t - N : t;
  const double b = pow(fabs(sinc(double(f) / N)), double(p));
  return float(pow(b, -2.0 * gamma));
}

}  // namespace



struct pme_plan_s {
  pme_desc_t desc;
  DevPlan d;
  int64_t bytes;
  int max_atoms;
  bool phi_valid;
  int64_t phi_id = 0;    // evaluation that wrote the kept phi (0: none)
  int64_t phi_gen = 0;   // last identifier handed out
  int set;        // counter set of the next binning (alternates)
  pme::KTimer timer;
  // PME_F_CONCURRENT: the cotangent chain's view of the plan (own records,
  // counters, density and spectrum; the rest shared with d), its stream and the
  // fork/join events
  bool concurrent = false;
  DevPlan dt;
  int tset = 0;
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr;
  hipEvent_t join = nullptr;
  hipEvent_t binned = nullptr;   // pme_step with plane spreads: the one binning is done
  // pme_step_capture: the capture stream, the graph of the captured steps and the
  // counter sets (set, tset) the graph starts from
  hipStream_t cap = nullptr;
  hipGraph_t sgraph = nullptr;
  hipGraphExec_t sexec = nullptr;
  int gset = 0, gtset = 0;
};

namespace pme {

constexpr size_t kTimerMaxEvents = 2 * 65536;

const LaunchEvents* KTimer::next(int k) {
  if (k != kind || capturing) return nullptr;
  while (used + 2 > ev.size()) {
    if (ev.size() >= kTimerMaxEvents) return nullptr;
    for (int i = 0; i < 512; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) break;
      ev.push_back(e);
    }
    if (used + 2 > ev.size()) return nullptr;
  }
  cur.start = ev[used];
  cur.stop = ev[used + 1];
  used += 2;
  return &cur;
}

}  // namespace pme

namespace {

thread_local char g_hip_err[256] = "";

int hip_fail(hipError_t e) {
  snprintf(g_hip_err, sizeof(g_hip_err), "%s", hipGetErrorString(e));
  return PME_EHIP;
}

// phi now holds the potential of a new evaluation (valid) or nothing reusable
void mark_phi(pme_plan_s* pl, bool valid) {
  pl->phi_valid = valid;
  pl->phi_id = valid ? ++pl->phi_gen : 0;
}

bool five_smooth(long m) {
  if (m < 1) return false;
  for (long f : {2L, 3L, 5L})
    while (m % f == 0) m /= f;
  return m == 1;
}

int pick_bin(int N) {
  for (int c : {4, 5, 3, 6, 2})
    if (N % c == 0) return c;
  return N;
}

// Default geometry of one axis: among atom-bin sizes B that divide N (in the
// order of pick_bin) and tiles T = k B that divide N as well, the T closest to
// the target within [target / 2, 2 target] (ties: the larger B, then the
// smaller T).  Tiles that divide the mesh leave no partial tiles at the edge,
// whose shorter work and uneven spread over the CUs cost the 100^3 mesh about 7 %
// of a step (8 x 8 x 16 with 4-point bins against 10 x 10 x 20 with 5-point
// bins).  Returns false when no such tile exists.
bool pick_dividing_tile(int N, int target, int& B, int& T) {
  int best = -1;
  for (int c : {4, 5, 3, 6, 2}) {
    if (N % c) continue;
    for (int t = c; t <= 2 * target && t <= N; t += c) {
      if (N % t || 2 * t < target) continue;
      const int d = t > target ? t - target : target - t;
      if (best < 0 || d < best || (d == best && c > B)) {
        best = d;
        B = c;
        T = t;
      }
    }
  }
  return best >= 0;
}





// Descriptor checks shared by every entry point that takes one.
int check_desc(const pme_desc_t& desc) {
  if (desc.order < 1 || desc.order > 7) return PME_EORDER;
  for (int a = 0; a < 3; ++a)
    if (desc.mesh[a] < 2 || desc.mesh[a] > 1024 || !five_smooth(desc.mesh[a])) return PME_EMESH;
  if (!(desc.alpha > 0.0) || !isfinite(desc.alpha) || !(desc.influence_power >= 0.0) ||
      !isfinite(desc.influence_power) || !isfinite(desc.prefactor))
    return PME_EALPHA;
  if (desc.max_atoms < 1 ||
      (desc.flags & ~(PME_F_KEEP_PHI | PME_F_CONCURRENT | PME_F_OPT_INFLUENCE |
                      PME_F_SEPARATE_SPREAD)))
    return PME_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (desc.tile[a] < 0 || desc.tile[a] > 1024) return PME_EINVAL;
  if (desc.fft_lines < 0 || desc.fft_lines > 1024) return PME_EINVAL;
  return PME_OK;
}

// Geometry of a plan (host only, nothing allocated): mesh and order, atom bins and
// their capacity, spread and gather tiles, spread staging, FFT layout.  `nbins`
// receives the number of atom bins.  PME_EMESH when no tile or FFT layout fits.
int plan_geometry(const pme_desc_t& desc, DevPlan& d, long& nbins_out) {
  const int p = desc.order;
  for (int a = 0; a < 3; ++a) d.N[a] = desc.mesh[a];
  d.H = d.N[2] / 2 + 1;
  d.p = p;
  d.alpha = desc.alpha;
  d.prefactor = desc.prefactor;
  d.opt = (desc.flags & PME_F_OPT_INFLUENCE) != 0;
  const long M = long(d.N[0]) * d.N[1] * d.N[2];

  // bins of B cells and mesh tiles of T = k B cells: by default tiles near
  // 8 x 8 x 16 that divide the mesh (pick_dividing_tile); a target the descriptor
  // sets is rounded to the first bin size that divides N, as are axes with no
  // dividing tile
  long nbins = 1;
  int target[3] = {8, 8, 16};
  const bool given = desc.tile[0] > 0 || desc.tile[1] > 0 || desc.tile[2] > 0;
  for (int a = 0; a < 3; ++a)
    if (desc.tile[a] > 0) target[a] = desc.tile[a];
  for (int a = 0; a < 3; ++a) {
    if (given || !pick_dividing_tile(d.N[a], target[a], d.B[a], d.T[a])) {
      d.B[a] = pick_bin(d.N[a]);
      int k = (target[a] + d.B[a] / 2) / d.B[a];
      if (k < 1) k = 1;
      if (k > d.N[a] / d.B[a]) k = d.N[a] / d.B[a];
      d.T[a] = k * d.B[a];
    }
    d.nb[a] = d.N[a] / d.B[a];
    nbins *= d.nb[a];
  }
  // shrink tiles until the spread tile, the scanned bin range, the gather's own
  // bins and its LDS field region fit their bounds
  for (;;) {
    long range = 1, own = 1, region = 2;
    for (int a = 0; a < 3; ++a) {
      long k = (d.T[a] + p - 1 + d.B[a] - 1) / d.B[a] + 1;
      range *= (k < d.nb[a] ? k : d.nb[a]);
      own *= d.T[a] / d.B[a];
      region *= d.T[a] + p - 1;
    }
    const long tpad = long(d.T[0]) * d.T[1] * (d.T[2] + 1);
    // two field regions and their row and z tables
    const long rows = long(d.T[0] + p - 1) * (d.T[1] + p - 1) + (d.T[2] + p - 1);
    if (range <= pme::kMaxBinRange && own <= 256 && tpad <= pme::kTileLds &&
        region * 4 + rows * 4 <= pme::kGatherLds &&
        long(pme::spread_lds_bytes(int(tpad), int(range), 64, p, 2)) <= pme::kBigLds)
      break;
    int big = 0;
    for (int a = 1; a < 3; ++a)
      if (d.T[a] / d.B[a] > d.T[big] / d.B[big]) big = a;
    if (d.T[big] == d.B[big]) return PME_EMESH;
    d.T[big] -= d.B[big];
  }
  for (int a = 0; a < 3; ++a) d.nt[a] = (d.N[a] + d.T[a] - 1) / d.T[a];
  {
    // spread staging: records per round such that five workgroups share a CU's
    // 160 KiB of LDS (all tiles of a 100^3 mesh resident at once; 1 KiB per
    // workgroup is left for static LDS and allocation granularity), at least 64
    long range = 1;
    for (int a = 0; a < 3; ++a) {
      long k = (d.T[a] + p - 1 + d.B[a] - 1) / d.B[a] + 1;
      range *= (k < d.nb[a] ? k : d.nb[a]);
    }
    d.nbr_max = int(range);
    const int tw = d.T[0] * d.T[1] * (d.T[2] + 1);
    for (int deg = 1; deg <= 2; ++deg) {
      const long fixed = long(pme::spread_lds_bytes(tw, d.nbr_max, 0, p, deg));
      const long per = 4L * pme::spread_entry_words(p, deg) + 2L * p;
      long ch = (32768 - 1024 - fixed) / per;
      if (ch > 256) ch = 256;
      if (ch < 64) ch = 64;
      d.spread_ch[deg - 1] = int(ch);
    }
  }
  {
    const double per_bin = double(desc.max_atoms) * d.B[0] * d.B[1] * d.B[2] / double(M);
    long cap = long(ceil(2.0 * per_bin)) + 8;
    if (cap > 64) cap = 64;
    d.cap = int(cap);
  }
  // FFT layout
  for (int a = 0; a < 3; ++a)
    if (!pme::radix_plan(d.N[a], d.ax[a])) return PME_EMESH;
  {
    // slab mode when a y-z plane of the half spectrum (two LDS buffers) fits
    const long npairs = (d.N[1] + 1) / 2;
    long buf = npairs * d.N[2];
    if (long(d.H) * (d.N[1] + 1) > buf) buf = long(d.H) * (d.N[1] + 1);
    const long slab_bytes = long(sizeof(float2)) * (2 * buf + d.N[1] + d.N[2]);
    d.slab = slab_bytes <= pme::kSlabLdsMax;
    d.slab_lds = size_t(slab_bytes);
    // spread fused with the forward slab transform: the padded plane (64-bit words)
    // after the first transform buffer, which also holds the bin scan, the item map
    // and the hit list while atoms are added; the second buffer overlaps the plane.
    // Every axis needs N >= p + B (a plane's anchors then lie in at most
    // (p - 1) / B + 2 bin layers and a padded row or column has one periodic image).
    d.fused = false;
    if (d.slab && !(desc.flags & PME_F_SEPARATE_SPREAD) && p <= 7) {
      bool ok = true;
      for (int a = 0; a < 3; ++a)
        if (d.N[a] < p + d.B[a]) ok = false;
      long layers = (p - 1) / d.B[0] + 2;
      if (layers > d.nb[0]) layers = d.nb[0];
      const long nscan = layers * d.nb[1] * d.nb[2];
      const long arrays = 8 * (nscan + 2) + 2L * pme::kFusedMap + 4L * pme::kFusedHits;
      const long abuf = buf > (arrays + 7) / 8 ? buf : (arrays + 7) / 8;
      const long pl = long(d.N[1] + p - 1) * (d.N[2] + p - 1);
      const long bytes = 8 * (d.N[1] + d.N[2] + abuf + (pl > buf ? pl : buf));
      if (ok && nscan < 65535 && bytes <= pme::kSlabLdsMax) {
        d.fused = true;
        d.fused_lds = size_t(bytes);
        d.fused_abuf = int(abuf);
        d.fused_nscan = int(nscan);
      }
    }
    // band spread where the plane spread is not fused with the transform: the most
    // rows per band (at most 64) whose band, scan arrays, item map and hit list fit
    // the slab LDS limit, then bands of equal height; worth it from 8 rows.  When
    // that grid is four or more rounds of workgroups deep, bands sized for two
    // workgroups per CU instead (one's latency phases overlap the other's adds)
    d.band = false;
    if (!d.fused && !(desc.flags & PME_F_SEPARATE_SPREAD) && p <= 7) {
      bool ok = true;
      for (int a = 0; a < 3; ++a)
        if (d.N[a] < p + d.B[a]) ok = false;
      const long PZ = d.N[2] + p - 1;
      const long lx = std::min<long>(d.nb[0], (p - 1) / d.B[0] + 2);
      auto scan_of = [&](long rows) {
        return lx * std::min<long>(d.nb[1], (rows + p - 2) / d.B[1] + 2) * d.nb[2];
      };
      auto bytes_of = [&](long rows) {
        return 8 * rows * PZ + 8 * (scan_of(rows) + 2) + 2L * pme::kFusedMap +
               4L * pme::kBandHits;
      };
      auto fit_rows = [&](long budget) {
        for (long rows = std::min(d.N[1], 64); rows >= 1; --rows)
          if (scan_of(rows) < 65535 && bytes_of(rows) <= budget) return rows;
        return 0L;
      };
      long fit = fit_rows(pme::kSlabLdsMax);
      if (fit && d.N[0] * ((d.N[1] + fit - 1) / fit) >= 4L * pme::kNumCUs) {
        const long fit2 = fit_rows(pme::kBandLdsPair);
        if (fit2 >= std::min(d.N[1], 8)) fit = fit2;
      }
      if (ok && fit >= std::min(d.N[1], 8)) {
        const long nband = (d.N[1] + fit - 1) / fit;
        const long rows = (d.N[1] + nband - 1) / nband;
        d.band = true;
        d.band_rows = int(rows);
        d.band_nscan = int(scan_of(rows));
        d.band_lds = size_t(bytes_of(rows));
      }
    }
    // pencil passes: about 1024 complex points per workgroup
    int pairs = (1024 + d.N[2] - 1) / d.N[2];
    if (pairs > 32) pairs = 32;
    d.rows_per_block = 2 * pairs;
    const int nmax = d.N[0] > d.N[1] ? d.N[0] : d.N[1];
    const int kt0 = nmax <= 64 ? 16 : (nmax <= 160 ? 24 : 4);
    int kt = desc.fft_lines > 0 ? desc.fft_lines : kt0;
    // the pencil y pass holds no g table: on meshes above 160 points it takes twice
    // the x pass's default lines (64-byte segments of its strided lines); on smaller
    // meshes, and with lines given in the descriptor, the x pass's
    int kty = desc.fft_lines > 0 ? desc.fft_lines : 2 * kt0;
    // LDS of a line workgroup within 56 KB: twiddles, two line buffers and (x pass)
    // the kt N_x table of g and the deconvolution factors:
    // 8 N + kt (16 (N + 1) + 4 N) + 4 (N + kt) bytes
    // (optimal influence: 12 (N + kt) more bytes of aliasing weights)
    const int extra = d.opt ? 3 * (nmax + 1) / 2 : 0;
    const int lds_cap = (7000 - nmax - (nmax + 1) / 2 - extra) /
                        (2 * (nmax + 1) + (nmax + 1) / 2 + 2 + (d.opt ? 2 : 0));
    if (kt > lds_cap) kt = lds_cap;
    if (kt < 1) kt = 1;
    if (kt > d.H) kt = d.H;
    // the y pass: twiddles and two line buffers within the same 56 KB
    const int ycap = (7000 - nmax) / (2 * (nmax + 1));
    if (kty > ycap) kty = ycap;
    if (kty < 1) kty = 1;
    if (kty > d.H) kty = d.H;
    // equal chunks of the H columns (no mostly-empty last chunk)
    const int nchunk = (d.H + kt - 1) / kt;
    kt = (d.H + nchunk - 1) / nchunk;
    d.ktile = kt;
    if (nmax <= 160 || desc.fft_lines > 0) {
      d.ytile = kt;
    } else {
      const int nchunk_y = (d.H + kty - 1) / kty;
      d.ytile = (d.H + nchunk_y - 1) / nchunk_y;
    }
  }
  nbins_out = nbins;
  return PME_OK;
}

template <class T>
hipError_t dev_alloc(T** p, size_t count, int64_t& bytes) {
  const size_t b = sizeof(T) * (count ? count : 1);
  bytes += int64_t(b);
  return hipMalloc(reinterpret_cast<void**>(p), b);
}

void drop_step_graph(pme_plan_s* pl) {
  if (pl->sexec) (void)hipGraphExecDestroy(pl->sexec);
  if (pl->sgraph) (void)hipGraphDestroy(pl->sgraph);
  pl->sexec = nullptr;
  pl->sgraph = nullptr;
}

void free_plan(pme_plan_s* pl) {
  drop_step_graph(pl);
  if (pl->cap) (void)hipStreamDestroy(pl->cap);
  for (hipEvent_t e : pl->timer.ev) (void)hipEventDestroy(e);
  if (pl->concurrent) {
    DevPlan& t = pl->dt;
    void* own[] = {t.count[0], t.count[1], t.ovf_count[0], t.ovf_count[1], t.cmax[0], t.cmax[1],
                   t.rec, t.rho, t.spec, t.cmax_fwd[0], t.cmax_fwd[1], t.gcache, t.gkey};
    for (void* p : own)
      if (p) (void)hipFree(p);
  }
  if (pl->fork) (void)hipEventDestroy(pl->fork);
  if (pl->join) (void)hipEventDestroy(pl->join);
  if (pl->binned) (void)hipEventDestroy(pl->binned);
  if (pl->aux) (void)hipStreamDestroy(pl->aux);
  DevPlan& d = pl->d;
  void* ptrs[] = {d.count[0], d.count[1], d.ovf_count[0], d.ovf_count[1], d.cmax[0],
                  d.cmax[1], d.rec, d.twiddle[0], d.twiddle[1], d.twiddle[2],
                  d.deconv[0], d.deconv[1], d.deconv[2], d.rho, d.spec, d.phi, d.epart,
                  d.spart, d.vpart, d.escr, d.status, d.alias[0], d.alias[1], d.alias[2],
                  d.gcache, d.gkey};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete pl;
}

}  // namespace

extern "C" {

const char* pme_strerror(int code) {
  switch (code) {
    case PME_OK: return "ok";
    case PME_EINVAL: return "invalid argument (NULL required pointer, n < 0 or bad flag)";
    case PME_EORDER: return "assignment order must be in 1..7";
    case PME_EMESH: return "mesh dimensions must be 5-smooth and within 2..1024";
    case PME_EALPHA: return "alpha must be > 0 and finite; gamma >= 0; prefactor finite";
    case PME_ECAPACITY: return "more atoms than the plan's max_atoms";
    case PME_ENOMEM: return "device allocation failed";
    case PME_EHIP: return "HIP runtime error";
    case PME_ENONFINITE: return "non-finite position or box seen on the device";
    case PME_ESCRATCH:
      return "workspace of pme_forward_noalloc exceeds its fixed scratch array "
             "(PME_NOALLOC_SCRATCH_BYTES per GPU)";
    default: return "unknown error";
  }
}

const char* pme_last_hip_error(void) { return g_hip_err; }

int pme_mesh_dims(const double box[9], double spacing, int strategy, int32_t out[3]) {
  if (!box || !out || !(spacing > 0.0) || !isfinite(spacing)) return PME_EINVAL;
  const double det = box[0] * (box[4] * box[8] - box[5] * box[7]) -
                     box[1] * (box[3] * box[8] - box[5] * box[6]) +
                     box[2] * (box[3] * box[7] - box[4] * box[6]);
  if (!isfinite(det) || det == 0.0) return PME_EINVAL;
  for (int a = 0; a < 3; ++a) {
    const double len = sqrt(box[3 * a] * box[3 * a] + box[3 * a + 1] * box[3 * a + 1] +
                            box[3 * a + 2] * box[3 * a + 2]);
    const double t = ceil(2.0 * len / spacing + 1.0);
    if (!(t < 1073741824.0)) return PME_EINVAL;
    long n = long(t);
    if (strategy == PME_MESH_POW2) {
      long m = 1;
      while (m < n) m <<= 1;
      n = m;
    } else if (strategy == PME_MESH_SMOOTH) {
      while (!five_smooth(n)) ++n;
    } else if (strategy != PME_MESH_CEIL) {
      return PME_EINVAL;
    }
    if (n > 1073741824L) return PME_EINVAL;
    out[a] = int32_t(n);
  }
  return PME_OK;
}

int pme_plan(const pme_desc_t* desc, pme_plan_t* out) {
  if (!desc || !out) return PME_EINVAL;
  *out = nullptr;
  {
    const int vc = check_desc(*desc);
    if (vc != PME_OK) return vc;
  }

  pme_plan_s* pl = new (std::nothrow) pme_plan_s();
  if (!pl) return PME_ENOMEM;
  memset(&pl->d, 0, sizeof(pl->d));
  pl->desc = *desc;
  pl->bytes = 0;
  pl->max_atoms = desc->max_atoms;
  pl->phi_valid = false;
  pl->set = 0;
  DevPlan& d = pl->d;
  long nbins = 0;
  const int p = desc->order;
  {
    const int gc = plan_geometry(*desc, d, nbins);
    if (gc != PME_OK) {
      free_plan(pl);
      return gc;
    }
  }
  const long M = long(d.N[0]) * d.N[1] * d.N[2];

  hipError_t e = hipSuccess;
  int64_t& by = pl->bytes;
  auto ok = [&](hipError_t r) { if (r != hipSuccess && e == hipSuccess) e = r; };
  for (int k = 0; k < 2; ++k) {
    ok(dev_alloc(&d.count[k], size_t(nbins), by));
    ok(dev_alloc(&d.ovf_count[k], 1, by));
    ok(dev_alloc(&d.cmax[k], 1, by));
  }
  // one allocation for the bins and the overflow list, so that kernels select a
  // record by index from a single base pointer
  d.ovf_base = (long long)nbins * d.cap;
  ok(dev_alloc(&d.rec, (size_t(d.ovf_base) + size_t(desc->max_atoms)) * 16, by));
  for (int a = 0; a < 3; ++a) {
    ok(dev_alloc(&d.twiddle[a], size_t(d.N[a]), by));
    ok(dev_alloc(&d.deconv[a], size_t(d.N[a]), by));
    if (d.opt) ok(dev_alloc(&d.alias[a], size_t(3 * d.N[a]), by));
  }
  // the x pass's g tables: where its workgroups fit in one round (at most four per
  // CU) the pass is latency-bound and loading a table beats making it; on larger
  // meshes the strided line traffic bounds it and the table's extra bytes cost more
  // than the arithmetic they save, except for the optimal influence function
  const size_t xblocks = size_t(pme::fftx_blocks(d));
  const bool gtables = d.opt || xblocks <= 1024;
  d.gcache = nullptr;
  d.gkey = nullptr;
  if (gtables) {
    ok(dev_alloc(&d.gcache, xblocks * d.N[0] * d.ktile, by));
    ok(dev_alloc(&d.gkey, 9 * xblocks, by));
  }
  ok(dev_alloc(&d.rho, size_t(M), by));
  ok(dev_alloc(&d.spec, size_t(d.N[0]) * d.N[1] * d.H, by));
  ok(dev_alloc(&d.phi, size_t(M), by));
  ok(dev_alloc(&d.epart, size_t(pme::fftx_blocks(d)), by));
  ok(dev_alloc(&d.spart, size_t(4 * pme::bin_blocks(desc->max_atoms)), by));
  ok(dev_alloc(&d.vpart, size_t(6 * pme::fftx_blocks(d) + 9 * d.nt[0] * d.nt[1] * d.nt[2]), by));
  ok(dev_alloc(&d.escr, 3, by));
  ok(dev_alloc(&d.status, 1, by));
  if (e != hipSuccess) {
    free_plan(pl);
    return e == hipErrorOutOfMemory ? PME_ENOMEM : hip_fail(e);
  }
  // tables (host FP64, stored FP32)
  for (int a = 0; a < 3; ++a) {
    const int N = d.N[a];
    float2* tw = new float2[N];
    float* dc = new float[N];
    for (int t = 0; t < N; ++t) {
      tw[t] = twiddle(t, N);
      dc[t] = deconv_factor(t, N, p, desc->influence_power);
    }
    if (d.opt) {
      // aliasing weights sinc^{2p}((f + m N)/N), m = -1, 0, 1, and the separable
      // denominator of the optimal influence function
      float* al = new float[3 * N];
      for (int t = 0; t < N; ++t) {
        const int f = (t >= (N + 1) / 2) ? t - N : t;
        double sum = 0.0;
        for (int m = -1; m <= 1; ++m) {
          const double u = pow(sinc(double(f + m * N) / N), 2.0 * p);
          al[(m + 1) * N + t] = float(u);
          sum += u;
        }
        dc[t] = float(1.0 / (sum * sum));
      }
      ok(hipMemcpy(d.alias[a], al, sizeof(float) * 3 * N, hipMemcpyHostToDevice));
      delete[] al;
    }
    ok(hipMemcpy(d.twiddle[a], tw, sizeof(float2) * N, hipMemcpyHostToDevice));
    ok(hipMemcpy(d.deconv[a], dc, sizeof(float) * N, hipMemcpyHostToDevice));
    delete[] tw;
    delete[] dc;
  }
  for (int k = 0; k < 2; ++k) {
    ok(hipMemset(d.count[k], 0, sizeof(int) * nbins));
    ok(hipMemset(d.ovf_count[k], 0, sizeof(int)));
    ok(hipMemset(d.cmax[k], 0, sizeof(unsigned)));
  }
  ok(hipMemset(d.status, 0, sizeof(int)));
  if (d.gkey) ok(hipMemset(d.gkey, 0xff, sizeof(double) * 9 * xblocks));   // NaN: none made yet
  ok(hipMemset(d.phi, 0, sizeof(float) * M));
  if (e == hipSuccess && (desc->flags & PME_F_CONCURRENT)) {
    pl->concurrent = true;
    DevPlan& t = pl->dt;
    t = d;
    t.count[0] = t.count[1] = nullptr;
    t.ovf_count[0] = t.ovf_count[1] = nullptr;
    t.cmax[0] = t.cmax[1] = nullptr;
    t.rec = nullptr;
    t.rho = nullptr;
    t.spec = nullptr;
    t.gcache = nullptr;
    t.gkey = nullptr;
    for (int k = 0; k < 2; ++k) {
      ok(dev_alloc(&t.count[k], size_t(nbins), by));
      ok(dev_alloc(&t.ovf_count[k], 1, by));
      ok(dev_alloc(&t.cmax[k], 1, by));
      ok(dev_alloc(&t.cmax_fwd[k], 1, by));
    }
    ok(dev_alloc(&t.rec, (size_t(t.ovf_base) + size_t(desc->max_atoms)) * 16, by));
    ok(dev_alloc(&t.rho, size_t(M), by));
    ok(dev_alloc(&t.spec, size_t(d.N[0]) * d.N[1] * d.H, by));
    // the cotangent chain's x passes keep their own g tables: the two chains' passes
    // run at the same time
    if (gtables) {
      ok(dev_alloc(&t.gcache, xblocks * d.N[0] * d.ktile, by));
      ok(dev_alloc(&t.gkey, 9 * xblocks, by));
      if (e == hipSuccess) ok(hipMemset(t.gkey, 0xff, sizeof(double) * 9 * xblocks));
    }
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
      ok(hipMemset(t.count[k], 0, sizeof(int) * nbins));
      ok(hipMemset(t.ovf_count[k], 0, sizeof(int)));
      ok(hipMemset(t.cmax[k], 0, sizeof(unsigned)));
      ok(hipMemset(t.cmax_fwd[k], 0, sizeof(unsigned)));
    }
    ok(hipStreamCreateWithFlags(&pl->aux, hipStreamNonBlocking));
    ok(hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming));
    ok(hipEventCreateWithFlags(&pl->join, hipEventDisableTiming));
    ok(hipEventCreateWithFlags(&pl->binned, hipEventDisableTiming));
  }
  if (d.slab) ok(pme::enable_slab_lds(d.slab_lds));
  if (d.band) ok(pme::enable_band_lds());
  ok(pme::enable_spread_lds());
  ok(pme::enable_gather_lds());
  ok(hipDeviceSynchronize());
  if (e != hipSuccess) {
    free_plan(pl);
    return hip_fail(e);
  }
  *out = pl;
  return PME_OK;
}

void pme_plan_destroy(pme_plan_t plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  free_plan(plan);
}

int64_t pme_plan_workspace_bytes(pme_plan_t plan) { return plan ? plan->bytes : 0; }

const float* pme_plan_phi(pme_plan_t plan) { return plan ? plan->d.phi : nullptr; }

int64_t pme_plan_phi_id(pme_plan_t plan) { return plan ? plan->phi_id : 0; }

int pme_plan_drop_phi(pme_plan_t plan) {
  if (!plan) return PME_EINVAL;
  mark_phi(plan, false);
  return PME_OK;
}
const float* pme_plan_rho(pme_plan_t plan) {
  return (plan && !plan->d.fused) ? plan->d.rho : nullptr;
}

int pme_plan_spread_kind(pme_plan_t plan) {
  if (!plan) return PME_EINVAL;
  return plan->d.fused ? PME_SPREAD_FUSED : (plan->d.band ? PME_SPREAD_BAND : PME_SPREAD_TILE);
}

}  // extern "C"

namespace {

// The density (or tangent density) of binning `set` and its potential into `out`:
// the fused plane spread and transform when the plan has it, else the tile spread
// and the slab or pencil transform.
hipError_t spread_convolve(const DevPlan& d, hipStream_t s, int set, bool tangent,
                           const double* box, float* out, bool energy, pme::KTimer& tm,
                           double* vpart = nullptr) {
  hipError_t e;
  const int kind = tangent ? PME_K_SPREAD_TANGENT : PME_K_SPREAD;
  if (d.fused) e = pme::launch_spread_slab(d, s, set, tangent, box, tm.next(kind));
  else e = pme::launch_spread(d, s, set, tangent, box, tm.next(kind));
  if (e != hipSuccess) return e;
  return pme::launch_convolve(d, s, box, out, energy, &tm, vpart, d.fused);
}

// pme_forward, and with dE_dbox the cell gradient: the x pass and the gather also
// form their partials of it and one workgroup assembles dE/dC after the gather
int forward_impl(pme_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                 const float* mu, const double* box, double* energy, float* dE_dpos,
                 float* dE_dq, float* dE_dmu, double* dE_dbox) {
  if (!plan || n < 0 || !box || (n > 0 && !pos)) return PME_EINVAL;
  if (n > plan->max_atoms) return PME_ECAPACITY;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevPlan& d = plan->d;
  pme::KTimer& tm = plan->timer;
  hipError_t e;
  if (dE_dbox && !energy) energy = d.escr;
  double* vpart = dE_dbox ? d.vpart : nullptr;
  mark_phi(plan, false);
  const int set = plan->set;
  plan->set ^= 1;
  if ((e = pme::launch_bin(d, s, set, n, pos, q, mu, box, nullptr, nullptr, nullptr, false,
                           energy != nullptr, tm.next(PME_K_BIN))) != hipSuccess)
    return hip_fail(e);
  if ((e = spread_convolve(d, s, set, false, box, d.phi, energy != nullptr, tm, vpart)) !=
      hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_gather(d, s, set, n, pos, q, mu, box, energy, dE_dpos, dE_dq, dE_dmu,
                              pme::bin_blocks(n), tm.next(PME_K_GATHER),
                              vpart ? vpart + 6 * pme::fftx_blocks(d) : nullptr)) != hipSuccess)
    return hip_fail(e);
  if (dE_dbox && (e = pme::launch_cell_grad(d, s, box, energy, dE_dbox)) != hipSuccess)
    return hip_fail(e);
  mark_phi(plan, true);
  return PME_OK;
}

}  // namespace

extern "C" {

int pme_forward(pme_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                const float* mu, const double* box, double* energy, float* dE_dpos,
                float* dE_dq, float* dE_dmu) {
  return forward_impl(plan, stream, n, pos, q, mu, box, energy, dE_dpos, dE_dq, dE_dmu, nullptr);
}

int pme_forward_cell(pme_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                     const float* mu, const double* box, double* energy, float* dE_dpos,
                     float* dE_dq, float* dE_dmu, double* dE_dbox) {
  if (!dE_dbox || (plan && plan->d.opt)) return PME_EINVAL;
  return forward_impl(plan, stream, n, pos, q, mu, box, energy, dE_dpos, dE_dq, dE_dmu, dE_dbox);
}

int pme_forward_quad(pme_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                     const float* mu, const float* theta, const double* box, double* energy,
                     float* dE_dpos, float* dE_dq, float* dE_dmu, float* dE_dtheta) {
  if (!plan || n < 0 || !box || (n > 0 && !pos) || plan->d.p < 4) return PME_EINVAL;
  if (n > plan->max_atoms) return PME_ECAPACITY;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevPlan& d = plan->d;
  pme::KTimer& tm = plan->timer;
  hipError_t e;
  // phi of this call is not the one a following pme_backward may reuse
  mark_phi(plan, false);
  const int set = plan->set;
  plan->set ^= 1;
  if ((e = pme::launch_bin_quad(d, s, set, n, pos, q, mu, theta, box, energy != nullptr,
                                tm.next(PME_K_BIN))) != hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_spread_quad(d, s, set, box, tm.next(PME_K_SPREAD))) != hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_convolve(d, s, box, d.phi, energy != nullptr, &tm)) != hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_gather_quad(d, s, set, n, pos, q, mu, theta, box, energy, dE_dpos, dE_dq,
                                   dE_dmu, dE_dtheta, tm.next(PME_K_GATHER))) != hipSuccess)
    return hip_fail(e);
  return PME_OK;
}

int pme_backward(pme_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
                 const float* mu, const double* box, const float* v_pos, const float* v_q,
                 const float* v_mu, float* g_pos, float* g_q, float* g_mu) {
  if (!plan || n < 0 || !box || (n > 0 && !pos)) return PME_EINVAL;
  if (n > plan->max_atoms) return PME_ECAPACITY;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevPlan& d = plan->d;
  pme::KTimer& tm = plan->timer;
  hipError_t e;
  if (!((plan->desc.flags & PME_F_KEEP_PHI) && plan->phi_valid)) {
    const int set = plan->set;
    plan->set ^= 1;
    if ((e = pme::launch_bin(d, s, set, n, pos, q, mu, box, nullptr, nullptr, nullptr, false,
                             false, tm.next(PME_K_BIN))) != hipSuccess)
      return hip_fail(e);
    if ((e = spread_convolve(d, s, set, false, box, d.phi, false, tm)) != hipSuccess)
      return hip_fail(e);
    mark_phi(plan, true);
  }
  const int set = plan->set;
  plan->set ^= 1;
  if ((e = pme::launch_bin(d, s, set, n, pos, q, mu, box, v_pos, v_q, v_mu, true, false,
                           tm.next(PME_K_BIN_TANGENT))) != hipSuccess)
    return hip_fail(e);
  if ((e = spread_convolve(d, s, set, true, box, d.rho, false, tm)) != hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_gather_hvp(d, s, set, n, pos, q, mu, box, v_pos, v_q, v_mu, g_pos, g_q,
                                  g_mu, tm.next(PME_K_GATHER_HVP))) != hipSuccess)
    return hip_fail(e);
  return PME_OK;
}

int pme_step(pme_plan_t plan, void* stream, int32_t n, const float* pos, const float* q,
             const float* mu, const double* box, double* energy, float* dE_dpos, float* dE_dq,
             float* dE_dmu, const float* v_pos, const float* v_q, const float* v_mu, float* g_pos,
             float* g_q, float* g_mu) {
  if (!plan || n < 0 || !box || (n > 0 && !pos)) return PME_EINVAL;
  if (n > plan->max_atoms) return PME_ECAPACITY;
  if (!plan->concurrent) {
    const int32_t flags = plan->desc.flags;
    plan->desc.flags |= PME_F_KEEP_PHI;   // the backward reuses this forward's phi
    int r = pme_forward(plan, stream, n, pos, q, mu, box, energy, dE_dpos, dE_dq, dE_dmu);
    if (r == PME_OK)
      r = pme_backward(plan, stream, n, pos, q, mu, box, v_pos, v_q, v_mu, g_pos, g_q, g_mu);
    plan->desc.flags = flags;
    return r;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipStream_t s2 = plan->aux;
  const DevPlan& d = plan->d;
  const DevPlan& dt = plan->dt;
  pme::KTimer& tm = plan->timer;
  hipError_t e;
  mark_phi(plan, false);
  if (d.fused || d.band) {
    // One binning for both densities and the gather: the cotangent binning (its
    // records carry q and mu; it also forms the forward coefficients' largest sum and
    // the self-term sums) on the second stream, then the cotangent chain there; the
    // forward plane or band spread reads the same records once they are written.
    const int tset = plan->tset;
    plan->tset ^= 1;
    if ((e = hipEventRecord(plan->fork, s)) != hipSuccess) return hip_fail(e);
    if ((e = hipStreamWaitEvent(s2, plan->fork, 0)) != hipSuccess) return hip_fail(e);
    if ((e = pme::launch_bin(dt, s2, tset, n, pos, q, mu, box, v_pos, v_q, v_mu, true,
                             energy != nullptr, tm.next(PME_K_BIN_TANGENT), true)) != hipSuccess)
      return hip_fail(e);
    if ((e = hipEventRecord(plan->binned, s2)) != hipSuccess) return hip_fail(e);
    if ((e = spread_convolve(dt, s2, tset, true, box, dt.rho, false, tm)) != hipSuccess)
      return hip_fail(e);
    if ((e = hipStreamWaitEvent(s, plan->binned, 0)) != hipSuccess) return hip_fail(e);
    const pme::RecordSource src{&dt, tset, dt.cmax_fwd[tset]};
    e = d.fused ? pme::launch_spread_slab(d, s, 0, false, box, tm.next(PME_K_SPREAD), &src)
                : pme::launch_spread_band(d, s, 0, false, box, tm.next(PME_K_SPREAD), &src);
    if (e != hipSuccess) return hip_fail(e);
    if ((e = pme::launch_convolve(d, s, box, d.phi, energy != nullptr, &tm, nullptr, d.fused)) !=
        hipSuccess)
      return hip_fail(e);
    if ((e = hipEventRecord(plan->join, s2)) != hipSuccess) return hip_fail(e);
    if ((e = hipStreamWaitEvent(s, plan->join, 0)) != hipSuccess) return hip_fail(e);
    const pme::GatherForward fwd{energy, dE_dpos, dE_dq, dE_dmu, pme::bin_blocks(n)};
    if ((e = pme::launch_gather_hvp(dt, s, tset, n, pos, q, mu, box, v_pos, v_q, v_mu, g_pos,
                                    g_q, g_mu, tm.next(PME_K_GATHER_HVP), &fwd)) != hipSuccess)
      return hip_fail(e);
    mark_phi(plan, true);
    return PME_OK;
  }
  const int set = plan->set;
  plan->set ^= 1;
  const int tset = plan->tset;
  plan->tset ^= 1;
  // cotangent chain on the second stream: binning, tangent density, its potential
  // (into dt.rho); it reads only inputs and the shared tables
  if ((e = hipEventRecord(plan->fork, s)) != hipSuccess) return hip_fail(e);
  if ((e = hipStreamWaitEvent(s2, plan->fork, 0)) != hipSuccess) return hip_fail(e);
  if ((e = pme::launch_bin(dt, s2, tset, n, pos, q, mu, box, v_pos, v_q, v_mu, true, false,
                           tm.next(PME_K_BIN_TANGENT))) != hipSuccess)
    return hip_fail(e);
  if ((e = spread_convolve(dt, s2, tset, true, box, dt.rho, false, tm)) != hipSuccess)
    return hip_fail(e);
  // forward chain on the caller's stream
  if ((e = pme::launch_bin(d, s, set, n, pos, q, mu, box, nullptr, nullptr, nullptr, false,
                           energy != nullptr, tm.next(PME_K_BIN))) != hipSuccess)
    return hip_fail(e);
  if ((e = spread_convolve(d, s, set, false, box, d.phi, energy != nullptr, tm)) != hipSuccess)
    return hip_fail(e);
  // join, then one gather over the cotangent chain's records (which carry q and mu)
  // forms H v and the forward outputs from phi and the tangent potential
  if ((e = hipEventRecord(plan->join, s2)) != hipSuccess) return hip_fail(e);
  if ((e = hipStreamWaitEvent(s, plan->join, 0)) != hipSuccess) return hip_fail(e);
  const pme::GatherForward fwd{energy, dE_dpos, dE_dq, dE_dmu, pme::bin_blocks(n)};
  if ((e = pme::launch_gather_hvp(dt, s, tset, n, pos, q, mu, box, v_pos, v_q, v_mu, g_pos, g_q,
                                  g_mu, tm.next(PME_K_GATHER_HVP), &fwd)) != hipSuccess)
    return hip_fail(e);
  mark_phi(plan, true);
  return PME_OK;
}

int pme_step_capture(pme_plan_t plan, int32_t steps, int32_t n, const float* pos, const float* q,
                     const float* mu, const double* box, double* energy, float* dE_dpos,
                     float* dE_dq, float* dE_dmu, const float* v_pos, const float* v_q,
                     const float* v_mu, float* g_pos, float* g_q, float* g_mu) {
  if (!plan || steps < 1 || n < 0 || !box || (n > 0 && !pos)) return PME_EINVAL;
  if (n > plan->max_atoms) return PME_ECAPACITY;
  drop_step_graph(plan);
  hipError_t e;
  if (!plan->cap && (e = hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(e);
  const int set0 = plan->set, tset0 = plan->tset;
  const bool phi0 = plan->phi_valid;
  const int64_t id0 = plan->phi_id;
  pme::KTimer& t = plan->timer;
  t.capturing = true;
  if ((e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
    t.capturing = false;
    return hip_fail(e);
  }
  int rc = PME_OK;
  for (int k = 0; k < steps && rc == PME_OK; ++k)
    rc = pme_step(plan, plan->cap, n, pos, q, mu, box, energy, dE_dpos, dE_dq, dE_dmu, v_pos, v_q,
                  v_mu, g_pos, g_q, g_mu);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(plan->cap, &g);
  t.capturing = false;
  // nothing ran: the host-side state is that of before the capture
  const bool parity = plan->set == set0 && plan->tset == tset0;
  plan->set = set0;
  plan->tset = tset0;
  plan->phi_valid = phi0;
  plan->phi_id = id0;
  if (rc != PME_OK || e != hipSuccess || !parity) {
    if (g) (void)hipGraphDestroy(g);
    if (rc != PME_OK) return rc;
    return e != hipSuccess ? hip_fail(e) : PME_EINVAL;
  }
  plan->sgraph = g;
  if ((e = hipGraphInstantiate(&plan->sexec, g, nullptr, nullptr, 0)) != hipSuccess) {
    drop_step_graph(plan);
    return hip_fail(e);
  }
  plan->gset = set0;
  plan->gtset = tset0;
  return PME_OK;
}

int pme_step_replay(pme_plan_t plan, void* stream) {
  if (!plan || !plan->sexec) return PME_EINVAL;
  // the graph bins into the counter sets it was captured with: calls made on the
  // plan since must have left the same ones next
  if (plan->set != plan->gset || plan->tset != plan->gtset) return PME_EINVAL;
  const hipError_t e = hipGraphLaunch(plan->sexec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  mark_phi(plan, true);
  return PME_OK;
}

int pme_plan_timer(pme_plan_t plan, int kind) {
  if (!plan || kind < PME_K_NONE || kind >= PME_K_COUNT) return PME_EINVAL;
  pme::KTimer& t = plan->timer;
  t.kind = kind;
  t.used = 0;
  if (kind != PME_K_NONE && t.ev.empty()) {
    for (int i = 0; i < 512; ++i) {
      hipEvent_t ev;
      const hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) return hip_fail(e);
      t.ev.push_back(ev);
    }
  }
  return PME_OK;
}

int pme_plan_timer_read(pme_plan_t plan, int64_t* launches, double* total_ms) {
  if (!plan) return PME_EINVAL;
  pme::KTimer& t = plan->timer;
  double sum = 0.0;
  int64_t count = 0;
  for (size_t i = 0; i + 1 < t.used; i += 2) {
    hipError_t e = hipEventSynchronize(t.ev[i + 1]);
    if (e != hipSuccess) return hip_fail(e);
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1])) != hipSuccess) return hip_fail(e);
    sum += ms;
    ++count;
  }
  if (launches) *launches = count;
  if (total_ms) *total_ms = sum;
  t.used = 0;
  return PME_OK;
}

int pme_status(pme_plan_t plan, void* stream) {
  if (!plan) return PME_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e);
  int flag = 0;
  if ((e = hipMemcpy(&flag, plan->d.status, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e);
  if (flag) {
    if ((e = hipMemset(plan->d.status, 0, sizeof(int))) != hipSuccess) return hip_fail(e);
    return PME_ENONFINITE;
  }
  return PME_OK;
}

}  // extern "C"

// ---- batches ------------------------------------------------------------

struct pme_batch_s {
  int nbox = 0;
  std::vector<pme_plan_s*> plans;
  std::vector<int> n, off;
  pme::SpreadBatch sp;
  pme::FFTBatch ff;
  pme::GatherBatch ga;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int next_set = 1;     // counter set of the next backward (alternates after a forward)
};

namespace {

void free_batch(pme_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  pme::spread_batch_free(b->sp);
  pme::fft_batch_free(b->ff);
  pme::gather_batch_free(b->ga);
  for (pme_plan_s* p : b->plans)
    if (p) free_plan(p);
  delete b;
}

// forward of every box: counters of set 0 cleared, binning (set 0), spread,
// convolution with energy, gather; backward: set 1
int batch_forward(pme_batch_s* b, hipStream_t s, const pme::BatchIO& io) {
  hipError_t e;
  if ((e = pme::launch_clear_batch(b->sp, s)) != hipSuccess) return hip_fail(e);
  if ((e = pme::launch_bin_batch(b->sp, s, 0, false, io, io.energy != nullptr)) != hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_spread_batch(b->sp, s, 0, false, io.box)) != hipSuccess) return hip_fail(e);
  if ((e = pme::launch_convolve_batch(b->ff, s, io.box, true, io.energy != nullptr)) !=
      hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_gather_batch(b->ga, s, 0, false, io)) != hipSuccess) return hip_fail(e);
  return PME_OK;
}

// Hessian-vector product of every box; `set` alternates 1, 0, 1, ... over the
// backward calls that follow one forward
int batch_backward(pme_batch_s* b, hipStream_t s, int set, const pme::BatchIO& io) {
  hipError_t e;
  if ((e = pme::launch_bin_batch(b->sp, s, set, true, io, false)) != hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_spread_batch(b->sp, s, set, true, io.box)) != hipSuccess) return hip_fail(e);
  if ((e = pme::launch_convolve_batch(b->ff, s, io.box, false, false)) != hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_gather_batch(b->ga, s, set, true, io)) != hipSuccess) return hip_fail(e);
  return PME_OK;
}

pme::BatchIO fwd_io(const float* pos, const float* q, const float* mu, const double* box,
                    double* energy, float* gp, float* gq, float* gm) {
  pme::BatchIO io;
  io.pos = pos; io.q = q; io.mu = mu; io.box = box; io.energy = energy;
  io.o_pos = gp; io.o_q = gq; io.o_mu = gm;
  return io;
}

pme::BatchIO bwd_io(const float* pos, const float* q, const float* mu, const double* box,
                    const float* vp, const float* vq, const float* vm, float* gp, float* gq,
                    float* gm) {
  pme::BatchIO io = fwd_io(pos, q, mu, box, nullptr, gp, gq, gm);
  io.v_pos = vp; io.v_q = vq; io.v_mu = vm;
  return io;
}

}  // namespace

extern "C" {

int pme_batch_plan(const pme_desc_t* descs, int32_t nbox, const int32_t* n_atoms,
                     pme_batch_t* out) {
  if (!descs || !n_atoms || !out || nbox < 1) return PME_EINVAL;
  *out = nullptr;
  for (int b = 0; b < nbox; ++b) {
    if (n_atoms[b] < 0) return PME_EINVAL;
    if (descs[b].order != descs[0].order) return PME_EORDER;
    if ((descs[b].flags ^ descs[0].flags) & PME_F_OPT_INFLUENCE) return PME_EINVAL;
  }
  pme_batch_s* bt = new (std::nothrow) pme_batch_s();
  if (!bt) return PME_ENOMEM;
  bt->nbox = nbox;
  bt->plans.assign(nbox, nullptr);
  bt->n.resize(nbox);
  bt->off.resize(nbox);
  long long acc = 0;
  std::vector<DevPlan> dp(nbox);
  for (int b = 0; b < nbox; ++b) {
    pme_desc_t d = descs[b];
    d.flags = PME_F_KEEP_PHI | (descs[0].flags & PME_F_OPT_INFLUENCE);
    d.max_atoms = n_atoms[b] > 0 ? n_atoms[b] : 1;
    const int rc = pme_plan(&d, &bt->plans[b]);
    if (rc != PME_OK) {
      free_batch(bt);
      return rc;
    }
    if (!bt->plans[b]->d.slab) {
      free_batch(bt);
      return PME_EMESH;
    }
    bt->n[b] = n_atoms[b];
    bt->off[b] = int(acc);
    acc += n_atoms[b];
    if (acc > 0x7fffffffLL) {
      free_batch(bt);
      return PME_EINVAL;
    }
    dp[b] = bt->plans[b]->d;
  }
  hipError_t e = pme::spread_batch_build(dp.data(), bt->n.data(), bt->off.data(), nbox, bt->sp);
  if (e == hipSuccess) e = pme::fft_batch_build(dp.data(), nbox, bt->ff);
  if (e == hipSuccess)
    e = pme::gather_batch_build(dp.data(), bt->n.data(), bt->off.data(), nbox, bt->ga);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&bt->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_batch(bt);
    return e == hipErrorOutOfMemory ? PME_ENOMEM : hip_fail(e);
  }
  *out = bt;
  return PME_OK;
}

void pme_batch_destroy(pme_batch_t batch) {
  if (!batch) return;
  (void)hipDeviceSynchronize();
  free_batch(batch);
}

int pme_batch_forward(pme_batch_t batch, void* stream, const float* pos, const float* q,
                      const float* mu, const double* box, double* energy, float* dE_dpos,
                      float* dE_dq, float* dE_dmu) {
  if (!batch || !box || !pos) return PME_EINVAL;
  batch->next_set = 1;
  return batch_forward(batch, static_cast<hipStream_t>(stream),
                       fwd_io(pos, q, mu, box, energy, dE_dpos, dE_dq, dE_dmu));
}

int pme_batch_backward(pme_batch_t batch, void* stream, const float* pos, const float* q,
                       const float* mu, const double* box, const float* v_pos, const float* v_q,
                       const float* v_mu, float* g_pos, float* g_q, float* g_mu) {
  if (!batch || !box || !pos) return PME_EINVAL;
  const int set = batch->next_set;
  batch->next_set ^= 1;
  return batch_backward(batch, static_cast<hipStream_t>(stream), set,
                        bwd_io(pos, q, mu, box, v_pos, v_q, v_mu, g_pos, g_q, g_mu));
}

int pme_batch_graph_capture(pme_batch_t batch, const pme_batch_step_t* st) {
  if (!batch || !st || !st->pos || !st->box) return PME_EINVAL;
  if (batch->exec) { (void)hipGraphExecDestroy(batch->exec); batch->exec = nullptr; }
  if (batch->graph) { (void)hipGraphDestroy(batch->graph); batch->graph = nullptr; }
  hipStream_t s = batch->cap;
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e);
  int rc = batch_forward(batch, s, fwd_io(st->pos, st->q, st->mu, st->box, st->energy,
                                          st->dE_dpos, st->dE_dq, st->dE_dmu));
  if (rc == PME_OK)
    rc = batch_backward(batch, s, 1, bwd_io(st->pos, st->q, st->mu, st->box, st->v_pos, st->v_q,
                                            st->v_mu, st->g_pos, st->g_q, st->g_mu));
  if (rc == PME_OK)
    rc = batch_backward(batch, s, 0, bwd_io(st->pos, st->q, st->mu, st->box, st->vf_pos, nullptr,
                                            nullptr, st->gf_pos, st->gf_q, st->gf_mu));
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(s, &g);
  if (rc != PME_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e);
  batch->graph = g;
  e = hipGraphInstantiate(&batch->exec, g, nullptr, nullptr, 0);
  return e == hipSuccess ? PME_OK : hip_fail(e);
}

int pme_batch_graph_launch(pme_batch_t batch, void* stream) {
  if (!batch || !batch->exec) return PME_EINVAL;
  const hipError_t e = hipGraphLaunch(batch->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PME_OK : hip_fail(e);
}

int pme_batch_status(pme_batch_t batch, void* stream) {
  if (!batch) return PME_EINVAL;
  int worst = PME_OK;
  for (pme_plan_s* p : batch->plans) {
    const int rc = pme_status(p, stream);
    if (rc != PME_OK && worst == PME_OK) worst = rc;
  }
  return worst;
}

}  // extern "C"

// ---- pme_forward without allocation --------------------------------------
//
// Every workspace of the forward (atom bins and records, counters, density,
// spectrum, potential, twiddle and deconvolution tables, energy partials) is
// carved from one fixed device array per GPU.  The array's name is a host-side
// stand-in: host code uses only the device address that hipGetSymbolAddress
// returns for the current device, kept per device.

namespace {

constexpr size_t kScratchBytes = size_t(PME_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device: looked up once per device
// (with that device current), together with the dynamic LDS limits the kernels
// need, which pme_plan sets for plans.
int scratch_address(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= kMaxDevices) return PME_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return hip_fail(e);
    if (!p) return PME_EHIP;
    if ((e = pme::enable_slab_lds(pme::kSlabLdsMax)) != hipSuccess) return hip_fail(e);
    if ((e = pme::enable_band_lds()) != hipSuccess) return hip_fail(e);
    if ((e = pme::enable_spread_lds()) != hipSuccess) return hip_fail(e);
    if ((e = pme::enable_gather_lds()) != hipSuccess) return hip_fail(e);
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return PME_OK;
}

struct TableArgs {
  int N[3];
  int p;
  double gamma;
  float2* tw[3];
  float* dc[3];
};

// The per-axis twiddle and deconvolution tables, one thread per entry (the same
// values pme_plan computes on the host).
__global__ void __launch_bounds__(256) k_tables(TableArgs a) {
  int i = blockIdx.x * 256 + threadIdx.x;
  for (int ax = 0; ax < 3; ++ax) {
    if (i < a.N[ax]) {
      a.tw[ax][i] = twiddle(i, a.N[ax]);
      a.dc[ax][i] = deconv_factor(i, a.N[ax], a.p, a.gamma);
      return;
    }
    i -= a.N[ax];
  }
}

__global__ void __launch_bounds__(256) k_zero(int* p, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}

}  // namespace

extern "C" {

int pme_forward_noalloc(const pme_desc_t* desc, void* stream, int32_t n, const float* pos,
                        const float* q, const float* mu, const double* box, double* energy,
                        float* dE_dpos, float* dE_dq, float* dE_dmu) {
  if (!desc || n < 0 || !box || (n > 0 && !pos)) return PME_EINVAL;
  pme_desc_t dd = *desc;
  dd.max_atoms = n > 0 ? n : 1;       // the workspaces are sized for this call
  {
    const int vc = check_desc(dd);
    if (vc != PME_OK) return vc;
  }
  if (dd.flags & PME_F_OPT_INFLUENCE) return PME_EINVAL;
  DevPlan d;
  memset(&d, 0, sizeof(d));
  long nbins = 0;
  {
    const int gc = plan_geometry(dd, d, nbins);
    if (gc != PME_OK) return gc;
  }
  const long M = long(d.N[0]) * d.N[1] * d.N[2];
  d.ovf_base = (long long)nbins * d.cap;
  // layout of the scratch array (256-byte aligned pieces)
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const int nzero = int(2 * nbins + 5);   // both counter sets, overflow counts, cmax, status
  const size_t o_zero = take(sizeof(int) * size_t(nzero));
  const size_t o_rec = take(sizeof(float) * 16 * (size_t(d.ovf_base) + size_t(dd.max_atoms)));
  size_t o_tw[3], o_dc[3];
  for (int a = 0; a < 3; ++a) {
    o_tw[a] = take(sizeof(float2) * size_t(d.N[a]));
    o_dc[a] = take(sizeof(float) * size_t(d.N[a]));
  }
  const size_t o_rho = take(sizeof(float) * size_t(M));
  const size_t o_phi = take(sizeof(float) * size_t(M));
  const size_t o_spec = take(sizeof(float2) * size_t(d.N[0]) * d.N[1] * d.H);
  const size_t o_epart = take(sizeof(double) * size_t(pme::fftx_blocks(d)));
  const size_t o_spart = take(sizeof(double) * 4 * size_t(pme::bin_blocks(dd.max_atoms)));
  if (off > kScratchBytes) return PME_ESCRATCH;

  unsigned char* base = nullptr;
  {
    const int rc = scratch_address(&base);
    if (rc != PME_OK) return rc;
  }
  int* zero = reinterpret_cast<int*>(base + o_zero);
  d.count[0] = zero;
  d.count[1] = zero + nbins;
  d.ovf_count[0] = zero + 2 * nbins;
  d.ovf_count[1] = zero + 2 * nbins + 1;
  d.cmax[0] = reinterpret_cast<unsigned*>(zero + 2 * nbins + 2);
  d.cmax[1] = reinterpret_cast<unsigned*>(zero + 2 * nbins + 3);
  d.status = zero + 2 * nbins + 4;
  d.rec = reinterpret_cast<float*>(base + o_rec);
  TableArgs ta;
  ta.p = d.p;
  ta.gamma = dd.influence_power;
  for (int a = 0; a < 3; ++a) {
    d.twiddle[a] = reinterpret_cast<float2*>(base + o_tw[a]);
    d.deconv[a] = reinterpret_cast<float*>(base + o_dc[a]);
    ta.N[a] = d.N[a];
    ta.tw[a] = d.twiddle[a];
    ta.dc[a] = d.deconv[a];
  }
  d.rho = reinterpret_cast<float*>(base + o_rho);
  d.phi = reinterpret_cast<float*>(base + o_phi);
  d.spec = reinterpret_cast<float2*>(base + o_spec);
  d.epart = reinterpret_cast<double*>(base + o_epart);
  d.spart = reinterpret_cast<double*>(base + o_spart);

  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  hipLaunchKernelGGL(k_zero, dim3((nzero + 255) / 256), dim3(256), 0, s, zero, nzero);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e);
  hipLaunchKernelGGL(k_tables, dim3((d.N[0] + d.N[1] + d.N[2] + 255) / 256), dim3(256), 0, s, ta);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e);
  // the forward of pme_forward with counter set 0
  if ((e = pme::launch_bin(d, s, 0, n, pos, q, mu, box, nullptr, nullptr, nullptr, false,
                           energy != nullptr, nullptr)) != hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_spread(d, s, 0, false, box, nullptr)) != hipSuccess) return hip_fail(e);
  if ((e = pme::launch_convolve(d, s, box, d.phi, energy != nullptr, nullptr)) != hipSuccess)
    return hip_fail(e);
  if ((e = pme::launch_gather(d, s, 0, n, pos, q, mu, box, energy, dE_dpos, dE_dq, dE_dmu,
                              pme::bin_blocks(n), nullptr)) != hipSuccess)
    return hip_fail(e);
  return PME_OK;
}

}  // extern "C"
