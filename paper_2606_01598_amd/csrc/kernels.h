// Host-side launchers of the PME kernels and the plan data they read.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace pme {

constexpr int kMaxStages = 16;
constexpr int kMaxBinRange = 2048;   // bins a spread tile may scan (LDS count array)
constexpr int kTileLds = 8192;       // max padded spread-tile points: T_x T_y (T_z + 1)
constexpr int kBigLds = 150 * 1024;  // dynamic LDS limit of the spread kernels
constexpr int kGatherQueue = 128;                      // atoms a gather queues at once
constexpr int kGatherStaticLds = 20 * 1024;            // bound on the gathers' static LDS
constexpr int kGatherLds = 160 * 1024 - kGatherStaticLds;  // their dynamic LDS limit

// LDS words of one staged spread entry: weights of three axes (derivative orders up
// to deg), the assignment coefficients, the tile-local stencil coordinates and the
// three fractional offsets; odd, so that consecutive entries start in different
// LDS banks.
constexpr int spread_entry_words(int p, int deg) {
  return (3 * (deg + 1) * p + (deg == 1 ? 4 : 10) + 9) | 1;
}
// Slots of the item -> bin map of a spread workgroup (larger scanned ranges fall
// back to a binary search).
constexpr int kSpreadMap = 1024;
// Dynamic LDS of a spread workgroup staging `ch` entries per round.
inline size_t spread_lds_bytes(int tile_words, int nbr_max, int ch, int p, int deg) {
  return size_t(8) * tile_words + size_t(8) * (nbr_max + 2) + size_t(2) * kSpreadMap +
         size_t(4) * ch * spread_entry_words(p, deg) + size_t(2) * ch * p;
}
constexpr int kRecWords = 16;        // words per atom record

// n / d for 0 <= n < 2^17 and 1 <= d <= 4096 by a multiply-high:
// m = ceil(2^32 / d) (d = 1 is passed through).
struct FastDiv {
  uint32_t d;
  uint32_t m;
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
  return f.d == 1 ? n : __umulhi(n, f.m);
}

struct FFTStage {          // one Stockham stage: radix R after Ns = product of earlier radices
  int R;
  int Ns;
  int NR;                  // N / R
  int step;                // N / (Ns R): twiddle stride
  FastDiv ns;
  FastDiv nr;
};

struct AxisPlan {          // 1D mixed-radix FFT of length N
  int N;
  int nst;
  FFTStage st[kMaxStages];
};

constexpr int kFFTThreads = 256;    // pencil-pass workgroup
constexpr int kSlabThreads = 1024;  // slab-pass workgroup (one x-plane)
constexpr int kSlabLdsMax = 160 * 1024 - 2048;
constexpr int kFusedMap = 4096;     // item -> bin map slots of a fused spread-slab workgroup
constexpr int kFusedSlotsPerThread = 4;   // scanned slots per thread and round
constexpr int kFusedHits = 2 * kFusedSlotsPerThread * kSlabThreads;   // its hit list (two rounds)
constexpr int kBandHits = kFusedSlotsPerThread * kSlabThreads;       // band spread's (one round)
constexpr int kBandLdsPair = 78 * 1024;   // band workgroup's LDS budget, two per CU
constexpr int kNumCUs = 256;               // compute units of the MI355X

struct DevPlan {
  int N[3];                // mesh dims
  int H;                   // N_z/2 + 1 (half spectrum along z)
  int p;                   // assignment order
  double alpha;
  double prefactor;
  // atom bins: bins of B[a] mesh cells along axis a (B[a] divides N[a])
  int B[3];
  int nb[3];
  int cap;                 // records per bin
  int nbr_max;             // largest bin range a spread tile scans
  int spread_ch[2];        // records staged per round by the forward / tangent spread
  // two counter sets used alternately by successive binnings; a binning clears the
  // other set, so no kernel has to clear the set it reads
  int* count[2];           // [nbins] atoms per bin
  int* ovf_count[2];       // [1] atoms in the overflow list
  unsigned* cmax[2];       // [1] max over atoms of sum |assignment coefficients| (float bits)
  float* rec;              // [(nbins * cap + max_atoms) * 16] records (16 words each):
                           // the bins, then the overflow list
  long long ovf_base;      // record index of the overflow list (nbins * cap)
  // mesh tiles shared by the spread and the gathers (T[a] a multiple of B[a])
  int T[3];
  int nt[3];
  // FFT
  AxisPlan ax[3];
  float2* twiddle[3];      // e^{-2 pi i t / N_a}, t < N_a
  float* deconv[3];        // |sinc(f/N_a)|^{-2 gamma p}, signed f; with the optimal
                           // influence 1 / (sum_m sinc^{2p}((f + m N_a)/N_a))^2
  bool opt;                // optimal influence function (aliasing sums)
  float* alias[3];         // optimal influence: [3][N_a] sinc^{2p}((f + m N_a)/N_a), m = -1, 0, 1
  // the x pass's g tables, one block per x-pass workgroup ([fftx_blocks][N_x kt], in
  // the order the workgroup makes them), and the box each block was made for
  // ([fftx_blocks][9], NaN until made): a workgroup reads its block when the key
  // equals the caller's box, else it makes the table and stores both
  float* gcache;
  double* gkey;
  bool slab;               // y-z planes transformed in LDS (z and y passes fused)
  size_t slab_lds;         // dynamic LDS bytes of a slab workgroup
  // spread fused with the forward slab transform (one x-plane per workgroup), when
  // the padded plane fits in LDS beside a transform buffer
  bool fused;
  size_t fused_lds;        // its dynamic LDS bytes
  int fused_abuf;          // float2 words before the plane
  int fused_nscan;         // bins a plane may scan
  // band spread (meshes without the fused plane spread): one workgroup per band of
  // band_rows y-rows of an x-plane, the band in LDS (band_rows x (N_z + p - 1) words)
  bool band;
  int band_rows;
  int band_nscan;          // bins a band may scan
  size_t band_lds;         // its dynamic LDS bytes
  int rows_per_block;      // z-pass rows per block (even)
  int ktile;               // half-spectrum z columns per x-pass block
  int ytile;               // half-spectrum z columns per y-pass block (pencil layout)
  // meshes
  float* rho;              // [M] density (also the tangent density / its potential)
  float2* spec;            // [N_x N_y H]
  float* phi;              // [M]
  // reductions
  double* epart;           // [x-pass blocks]
  double* spart;           // [4 * bin blocks]: q^2, |mu|^2 per block (then, quadrupole
                           // forward: q tr Theta, tr^2 Theta + 2 Theta:Theta)
  double* vpart;           // cell gradient: [6 per x-pass block] then [9 per tile]
  double* escr;            // [3] energy of a cell-gradient call that asks for none
  int* status;             // bit 0: non-finite input seen
  // the cotangent view of a concurrent plan: the largest forward coefficient sum of
  // each counter set's records, for the forward plane spread of pme_step
  unsigned* cmax_fwd[2];
};

// Events into which a launch records its kernel's own begin and end timestamps
// (hipExtLaunchKernel); null members are not recorded.
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};

// Without events the plain launch is used (it can be captured into a HIP graph).
template <class F, class... A>
inline void launch_k(const LaunchEvents* ev, F kernel, dim3 g, dim3 b, size_t sh, hipStream_t s,
                     A... args) {
  if (ev) {
    hipExtLaunchKernelGGL(kernel, g, b, uint32_t(sh), s, ev->start, ev->stop, 0u, args...);
  } else {
    hipLaunchKernelGGL(kernel, g, b, uint32_t(sh), s, args...);
  }
}

// Launch timer (host side): hands out event pairs for the launches of one kernel
// kind.
struct KTimer {
  int kind = -1;
  std::vector<hipEvent_t> ev;   // start/stop pairs
  size_t used = 0;              // events handed out since the last read
  LaunchEvents cur;
  // launches being captured into a HIP graph are not timed (events recorded by
  // graph nodes cannot be read back here)
  bool capturing = false;
  // Events for the next launch of kind k, or nullptr when k is not being timed.
  const LaunchEvents* next(int k);
};

// ---- batches of boxes (one launch per kernel kind for all boxes) ----

// Per-call arrays of a batch: the atoms of box b occupy [off_b, off_b + n_b) of the
// packed per-atom arrays, cells are [nbox][9] and energies [nbox][3].
struct BatchIO {
  const float* pos = nullptr;
  const float* q = nullptr;
  const float* mu = nullptr;
  const double* box = nullptr;
  const float* v_pos = nullptr;
  const float* v_q = nullptr;
  const float* v_mu = nullptr;
  double* energy = nullptr;
  float* o_pos = nullptr;
  float* o_q = nullptr;
  float* o_mu = nullptr;
};

// Device tables of a batch: per-box argument templates (indexed by box) and the
// (box, work item) lists of each batched kernel.
struct SpreadBatch {
  int p = 0;
  void* bin[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};      // [tangent][set]
  void* spread[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [tangent][set]
  void* clear = nullptr;                                            // set-0 counters per box
  int2* bin_items = nullptr;
  int n_bin_items = 0;
  int2* tile_items = nullptr;
  int n_tile_items = 0;
  int nbox = 0;
  size_t lds[2] = {0, 0};                                           // spread LDS [tangent]
};
struct FFTBatch {
  void* slab[2] = {nullptr, nullptr};   // potential into phi / into rho
  void* x = nullptr;
  int2* slab_items = nullptr;
  int n_slab_items = 0;
  int2* x_items = nullptr;
  int n_x_items = 0;
  size_t slab_lds = 0, x_lds = 0;
  bool opt = false;                     // every box with the optimal influence function
};
struct GatherBatch {
  int p = 0;
  void* g[2] = {nullptr, nullptr};      // [set]
  int2* items = nullptr;
  int n_items = 0;
  size_t lds[2] = {0, 0};               // [hvp]
};

// Build the tables of boxes `plans[0..nbox)` with n[b] atoms at offsets off[b]
// (all plans of one order, slab FFT layout).
hipError_t spread_batch_build(const DevPlan* plans, const int* n, const int* off, int nbox,
                              SpreadBatch& t);
void spread_batch_free(SpreadBatch& t);
hipError_t fft_batch_build(const DevPlan* plans, int nbox, FFTBatch& t);
void fft_batch_free(FFTBatch& t);
hipError_t gather_batch_build(const DevPlan* plans, const int* n, const int* off, int nbox,
                              GatherBatch& t);
void gather_batch_free(GatherBatch& t);
// Clear counter set 0 of every box (the first binning of a batch step uses it).
hipError_t launch_clear_batch(const SpreadBatch& t, hipStream_t s);
hipError_t launch_bin_batch(const SpreadBatch& t, hipStream_t s, int set, bool tangent,
                            const BatchIO& io, bool self_sums);
hipError_t launch_spread_batch(const SpreadBatch& t, hipStream_t s, int set, bool tangent,
                               const double* box);
hipError_t launch_convolve_batch(const FFTBatch& t, hipStream_t s, const double* box, bool to_phi,
                                 bool energy);
hipError_t launch_gather_batch(const GatherBatch& t, hipStream_t s, int set, bool hvp,
                               const BatchIO& io);
// Upload `count` bytes of host data to a new device array.
hipError_t upload(void** dst, const void* src, size_t bytes);

inline int fftx_blocks(const DevPlan& d) { return d.N[1] * ((d.H + d.ktile - 1) / d.ktile); }
inline int ffty_blocks(const DevPlan& d) { return d.N[0] * ((d.H + d.ytile - 1) / d.ytile); }
inline int fftz_blocks(const DevPlan& d) {
  const int rows = d.N[0] * d.N[1];
  return (rows + d.rows_per_block - 1) / d.rows_per_block;
}
inline int bin_blocks(int n) { return n > 0 ? (n + 255) / 256 : 1; }

// Binning: stencil anchor, bin slot, per-atom record (forward: q and the x-space
// dipole; tangent: the 10 monomial coefficients of the tangent density).
// fwd_max (tangent binning of a concurrent step): also the largest forward
// coefficient sum into d.cmax_fwd[set], so that the forward plane spread can read
// these records.
hipError_t launch_bin(const DevPlan& d, hipStream_t s, int set, int n, const float* pos,
                      const float* q, const float* mu, const double* box, const float* v_pos,
                      const float* v_q, const float* v_mu, bool tangent, bool self_sums,
                      const LaunchEvents* ev, bool fwd_max = false);
// Owner-computes spread of the binned records (counter set `set`) into d.rho.
hipError_t launch_spread(const DevPlan& d, hipStream_t s, int set, bool tangent,
                         const double* box, const LaunchEvents* ev);
// Quadrupole forward: binning with the ten coefficients of q, J mu and
// (1/2) J Theta J^T in the records (self sums of Theta after the 2 n_blocks of q, mu),
// and their spread into d.rho.
hipError_t launch_bin_quad(const DevPlan& d, hipStream_t s, int set, int n, const float* pos,
                           const float* q, const float* mu, const float* theta, const double* box,
                           bool self_sums, const LaunchEvents* ev);
hipError_t launch_spread_quad(const DevPlan& d, hipStream_t s, int set, const double* box,
                              const LaunchEvents* ev);
// Quadrupole forward gather: E^lr (energy[0..3]: recip, self q, self mu, self Theta)
// and its gradients in r, q, mu and the six stored Theta entries.
hipError_t launch_gather_quad(const DevPlan& d, hipStream_t s, int set, int n, const float* pos,
                              const float* q, const float* mu, const float* theta,
                              const double* box, double* energy, float* dE_dpos, float* dE_dq,
                              float* dE_dmu, float* dE_dtheta, const LaunchEvents* ev);
// rho -> spec -> (x g) -> out, the mesh operator K; energy partials when wanted, and
// with vpart the six k-space partials of the cell gradient per x-pass workgroup.
// from_spec: the spectrum is already there (the fused spread wrote it); only the
// x pass and the inverse slab transform run
hipError_t launch_convolve(const DevPlan& d, hipStream_t s, const double* box, float* out,
                           bool energy, KTimer* tm, double* vpart = nullptr,
                           bool from_spec = false);
// Spread fused with the forward slab transform (d.fused): writes d.spec directly.
// from: the binned records and fixed-point scale to read instead of d's own (the
// forward density of pme_step from the cotangent binning: tangent records, which
// carry q and mu, and its cmax_fwd)
struct RecordSource {
  const DevPlan* d;   // counts, records, overflow list
  int set;
  const unsigned* cmax;
};
hipError_t launch_spread_slab(const DevPlan& d, hipStream_t s, int set, bool tangent,
                              const double* box, const LaunchEvents* ev,
                              const RecordSource* from = nullptr);
// The band spread of binning `set` into d.rho (d.band plans); with `from`, the
// forward density from another view's tangent records (as launch_spread_slab).
hipError_t launch_spread_band(const DevPlan& d, hipStream_t s, int set, bool tangent,
                              const double* box, const LaunchEvents* ev,
                              const RecordSource* from = nullptr);
hipError_t enable_band_lds();
// Raise the dynamic LDS limit of the spread (kBigLds) and gather (kGatherLds) kernels.
hipError_t enable_spread_lds();
hipError_t enable_gather_lds();
// Allow slab workgroups up to kSlabLdsMax of dynamic LDS (above the 64 KiB
// default); `bytes`, the need of the calling plan, must not exceed it.
hipError_t enable_slab_lds(size_t bytes);
// Gradient gather (+ energy finalisation) over the atoms binned in counter set `set`.
hipError_t launch_gather(const DevPlan& d, hipStream_t s, int set, int n, const float* pos,
                         const float* q, const float* mu, const double* box, double* energy,
                         float* dE_dpos, float* dE_dq, float* dE_dmu, int n_spart,
                         const LaunchEvents* ev, double* vpart = nullptr);
// Cell gradient dE^lr/dC (row-major like the box) from E_recip (energy[0]) and the
// partials of the x pass (vpart, 6 per block) and of the gather (9 per tile after them).
hipError_t launch_cell_grad(const DevPlan& d, hipStream_t s, const double* box,
                            const double* energy, double* dE_dbox);
// Hessian-vector product gather from phi (d.phi) and psi (d.rho).
// Forward outputs a Hessian-vector gather may form as well (same atoms, same phi).
struct GatherForward {
  double* energy;
  float* dE_dpos;
  float* dE_dq;
  float* dE_dmu;
  int n_spart;   // self-term partial sums written by the forward binning
};
hipError_t launch_gather_hvp(const DevPlan& d, hipStream_t s, int set, int n, const float* pos,
                             const float* q, const float* mu, const double* box,
                             const float* v_pos, const float* v_q, const float* v_mu,
                             float* g_pos, float* g_q, float* g_mu, const LaunchEvents* ev,
                             const GatherForward* fwd = nullptr);

}  // namespace pme
