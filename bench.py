"""Throughput of the PME hot path on one MI355X.

One step = pme_forward (E^lr, dE/dr, dE/dq, dE/dmu) + pme_backward (Hessian-vector
product with generic cotangents v_r, v_q, v_mu), inputs resident in HBM, on the
32,000-ion molten-salt box (L = 100.006 A, mesh 100^3, p = 6, alpha = 0.30 1/A).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 32k|8k|128k|1m]

Prints one JSON line.  Work is fixed per GPU ("weak" scaling); only N = 1 runs.

Besides the whole-step rate the line carries
  * "kernels_us": the average launch duration of every kernel kind over a short
    pass after the warm-up, from HIP events that the launches themselves stamp
    with their kernel's begin and end (pme_plan_timer);
  * "roofline": the dominant kernel (largest time per step), timed the same way
    over the timed region itself, against the HBM peak, with its
    algorithmic bytes per launch (ALG_BYTES below) and, when a counter summary
    for the current sources exists, its measured HBM traffic per launch;
  * "cpu_baseline": the FP64 oracle timed on the host cores on a bounded sample.

Counter summary (traffic):
    rocprofv3 --pmc FETCH_SIZE -d D1 -o run -- python bench.py --steps 3 --warmup 2 \\
        --cpu-baseline 0 --copy-calibration 1
    rocprofv3 --pmc WRITE_SIZE -d D2 -o run -- python bench.py (same arguments)
    python bench.py --traffic-summary D1/run_counter_collection.csv \\
        D2/run_counter_collection.csv
writes profiles/<kernel>_<workload>_traffic.txt, which the next bench run reads.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (n_ions, seed, mesh, order, alpha)
    "32k": (32000, 3, (100, 100, 100), 6, 0.30),
    "8k": (8000, 2, (64, 64, 64), 6, 0.30),
    "128k": (128000, 4, (160, 160, 160), 6, 0.30),
    "1m": (1000000, 5, (320, 320, 320), 6, 0.30),
}

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
COPY_BYTES = 256 << 20         # calibration copy for the byte counters

# Kernel symbol (as a profiler prints it) of each launch-timer kind, slab FFT layout.
KERNEL_SYMBOL = {
    "bin": "k_bin<6, false, false>", "bin_tangent": "k_bin<6, true, false>",
    "spread": "k_spread<6, 1>", "spread_tangent": "k_spread<6, 2>",
    "fft_r2c": "k_slab_fwd", "fft_x": "k_fftx_fused<0>", "fft_c2r": "k_slab_inv",
    "gather": "k_gather<6, false>", "gather_hvp": "k_gather_hvp<6, false>",
}


# The spread kinds where the spread is fused with the forward slab transform (one
# x-plane per workgroup; the default on meshes whose padded plane fits in LDS)
FUSED_SYMBOL = {"spread": "k_spread_slab<6, 1, false>", "spread_tangent": "k_spread_slab<6, 2, false>"}
# under pme_step's concurrent chains the forward plane spread takes the tangent records
FUSED_STEP_SPREAD = "k_spread_slab<6, 1, true>"
# ... and where a plan spreads by bands of y-rows of each x-plane (meshes whose
# padded plane does not fit in LDS beside the slab transform)
BAND_SYMBOL = {"spread": "k_spread_band<6, 1, false>", "spread_tangent": "k_spread_band<6, 2, false>"}
BAND_STEP_SPREAD = "k_spread_band<6, 1, true>"


# The transform kinds of a pencil-layout plan (a y-z plane of the half spectrum too
# large for LDS): each spans two launches (the z pass and a y pass)
PENCIL_SYMBOL = {"fft_r2c": "k_fftz_r2c+k_ffty", "fft_c2r": "k_ffty+k_fftz_c2r"}
SLAB_LDS_MAX = 160 * 1024 - 2048     # kSlabLdsMax of the library


def is_slab(mesh) -> bool:
    """Whether the library transforms this mesh by y-z planes in LDS (its slab test)."""
    ny, nz = mesh[1], mesh[2]
    h = nz // 2 + 1
    buf = max((ny + 1) // 2 * nz, h * (ny + 1))
    return 8 * (2 * buf + ny + nz) <= SLAB_LDS_MAX


def kernel_symbol(kind: str, step: bool = False, fused: bool = False, band: bool = False,
                  slab: bool = True) -> str:
    """Profiler name of a timer kind's kernel; under pme_step the Hessian-vector
    gather is the variant that also forms the forward outputs; with the fused
    plane spread the spread kinds name the fused kernel (whose forward variant reads
    the tangent records under pme_step)."""
    if kind == "gather_hvp" and step:
        return "k_gather_hvp<6, true>"
    if fused and kind == "spread" and step:
        return FUSED_STEP_SPREAD
    if fused and kind in FUSED_SYMBOL:
        return FUSED_SYMBOL[kind]
    if band and kind == "spread" and step:
        return BAND_STEP_SPREAD
    if band and kind in BAND_SYMBOL:
        return BAND_SYMBOL[kind]
    if not slab and kind in PENCIL_SYMBOL:
        return PENCIL_SYMBOL[kind]
    return KERNEL_SYMBOL[kind]


def spec_bytes(mesh) -> int:
    """Bytes of the half spectrum (complex float, N_x N_y (N_z/2 + 1))."""
    return 8 * mesh[0] * mesh[1] * (mesh[2] // 2 + 1)


def alg_bytes(kind: str, n: int, m: int, step: bool = True, spec: int = 0) -> int:
    """Algorithmic HBM bytes of one launch: the method's arrays (FP32) that the
    step must read or write, split over the kernels that perform the method's
    steps (the binning is part of the spread step, Eq. charge_dipole_assign):
      bin            (charged to the spread)                     0
      spread         pos, q, mu in; rho out                      28 n + 4 M
      spread_tangent pos, q, mu, v_pos, v_q, v_mu in; rho_dot out  56 n + 4 M
      fft_r2c        density in                                  4 M
      fft_x          (intermediate spectrum only)                0
      fft_c2r        potential out                               4 M
      gather         pos, q, mu in; 3 gradients out; phi in      56 n + 4 M
      gather_hvp     6 inputs in; 3 outputs; phi and psi in      84 n + 8 M
                     (pme_step: also the 3 gradients out        112 n + 8 M)
    A pme_forward + pme_backward step sums to 224 B per atom + 36 B per mesh point;
    a pme_step (one gather for both) to 196 B per atom + 32 B per mesh point.
    With the spread fused with the forward slab transform (spec = the half
    spectrum's bytes, 8 N_x N_y (N_z/2 + 1)), the density never leaves the
    workgroup: the fused kernel reads the atom inputs and writes the spectrum,
      spread         28 n + spec,   spread_tangent   56 n + spec,
    and the step model is unchanged up to the spectrum's size against 4 M.
    """
    table = {"bin": 0, "bin_tangent": 0, "spread": 28 * n + (spec or 4 * m),
             "spread_tangent": 56 * n + (spec or 4 * m), "fft_r2c": 4 * m, "fft_x": 0,
             "fft_c2r": 4 * m, "gather": 56 * n + 4 * m,
             "gather_hvp": (112 if step else 84) * n + 8 * m}
    return table[kind]


def step_bytes(n: int, m: int, step: bool = True) -> int:
    return 196 * n + 32 * m if step else 224 * n + 36 * m


# the sources each timer kind's kernel is compiled from (a traffic summary holds
# only while they are unchanged)
KERNEL_SOURCES = {
    "bin": ("spread.hip",), "bin_tangent": ("spread.hip",),
    "spread": ("spread.hip", "band.hip", "fft.hip", "fft_radix.h"),
    "spread_tangent": ("spread.hip", "band.hip", "fft.hip", "fft_radix.h"), "fft_r2c": ("fft.hip", "fft_radix.h"),
    "fft_x": ("fft.hip", "fft_radix.h"), "fft_c2r": ("fft.hip", "fft_radix.h"),
    "gather": ("gather.hip",), "gather_hvp": ("gather.hip",),
}


# sources of the learned-head, teacher and probe calls: no PME step kernel is built from them
NON_PME_SOURCES = ("cells.h", "dip.hip", "pol.hip", "probe.hip")


def source_digest(kind: str = None) -> str:
    """Digest of the HIP sources of the PME path (all of them, or those of one kernel
    kind together with the shared headers): a summary is valid only for the kernels
    it was measured on."""
    csrc = os.path.join(ROOT, "paper_2606_01598_amd", "csrc")
    if kind is None:
        files = sorted(f for f in glob.glob(os.path.join(csrc, "*"))
                       if os.path.basename(f) not in NON_PME_SOURCES)
    else:
        files = [os.path.join(csrc, f) for f in
                 sorted(set(KERNEL_SOURCES[kind]) | {"kernels.h", "pme_common.h"})]
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="32k", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-baseline", type=int, default=1,
                    help="0 skips the oracle timing on the host")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--breakdown-steps", type=int, default=10)
    ap.add_argument("--sequential", type=int, default=0,
                    help="1: pme_forward then pme_backward on one stream instead of pme_step "
                         "with the cotangent chain on a second stream")
    ap.add_argument("--graph", type=int, default=1,
                    help="1: the timed steps are captured into one HIP graph (pme_step_capture) "
                         "and replayed once, after one untimed replay; 0: eager calls")
    ap.add_argument("--replays", type=int, default=200,
                    help="single replays of a two-step graph timed one by one (median, p10, p90)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="1 also runs a device copy of 256 MiB (byte-counter calibration)")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the counter summary of the dominant kernel and exit")
    ap.add_argument("--kernel", default=None, help="kernel kind for --traffic-summary")
    ap.add_argument("--counter-summary", nargs="+", default=None, metavar="DIR",
                    help="write profiles/kernels_<workload>_counters.txt from rocprofv3 counter "
                         "directories (one per COUNTER_PASSES entry) and exit")
    ap.add_argument("--counter-step", type=int, default=0,
                    help="with --counter-summary: passes over the concurrent pme_step "
                         "(profiles/kernels_<workload>_step_counters.txt)")
    ap.add_argument("--kernel-stats", default=None, metavar="STATS_CSV",
                    help="write profiles/<workload> kernel-statistics summary from a "
                         "rocprofv3 --stats kernel_stats.csv")
    ap.add_argument("--bench-line", default=None, metavar="LOG",
                    help="with --kernel-stats: a log holding the JSON line of the same bench "
                         "command run without the profiler; its kernels_us are listed beside "
                         "the profiler's averages")
    ap.add_argument("--sweep-summary", nargs="+", default=None, metavar="LOG",
                    help="write profiles/pme_sweep_molten_sizes.txt from the JSON lines of "
                         "bench runs at several workloads and exit")
    ap.add_argument("--cell", type=int, default=1,
                    help="1 adds the cell-gradient leg (pme_forward_cell against pme_forward)")
    ap.add_argument("--influence", type=int, default=1,
                    help="1 adds the optimal-influence leg (pme_step with each influence function)")
    ap.add_argument("--quad", type=int, default=1,
                    help="1 adds the quadrupole leg (pme_forward_quad against pme_forward)")
    ap.add_argument("--influence-compare", type=int, default=0,
                    help="1: write the accuracy-per-mesh-point comparison of the influence "
                         "functions against Ewald and exit")
    ap.add_argument("--batched", type=int, default=1,
                    help="1 adds the batched-graph leg (64 boxes, one HIP graph per step)")
    ap.add_argument("--learned", type=int, default=1,
                    help="1 adds the learned-dipole leg (SCF teacher vs trained network)")
    ap.add_argument("--separate-spread", type=int, default=0,
                    help="1: plans spread by mesh tiles and transform in a separate pass "
                         "(PME_F_SEPARATE_SPREAD) instead of the fused plane spread")
    ap.add_argument("--halo-probe", type=int, default=0,
                    help="1: time the global-memory combination of the overlapping per-tile "
                         "regions of a scatter-once spread (pme_halo_probe: 64-bit atomics, or "
                         "contiguous region blocks and a fold) on the 100^3 and 320^3 meshes, "
                         "print one JSON line per tile shape, then exit")
    ap.add_argument("--halo-summary", nargs=2, default=None, metavar=("TRACE_CSV", "LOG"),
                    help="summarise a rocprofv3 kernel trace of --halo-probe 1 and the JSON "
                         "lines of an unprofiled run (LOG), then exit")
    ap.add_argument("--crossover", type=int, default=0,
                    help="1: time explicit Ewald and PME (oracles on the host, PME on the GPU) "
                         "for 128..8192 ions and print one JSON line per size, then exit")
    return ap.parse_args(argv)


def main(argv=None):
    args = _args(argv)
    if args.traffic_summary:
        return traffic_summary(args)
    if args.kernel_stats:
        return kernel_stats_summary(args)
    if args.counter_summary:
        return counter_summary(args)
    if args.sweep_summary:
        return sweep_summary(args.sweep_summary)
    if args.halo_summary:
        return halo_summary(*args.halo_summary)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        return 2
    if args.halo_probe:
        return halo_probe()
    if args.crossover:
        return crossover()
    if args.influence_compare:
        return influence_compare()
    import torch

    import synth
    from paper_2606_01598_amd import _lib
    from paper_2606_01598_amd.pme import Plan

    n, seed, mesh, p, alpha = WORKLOADS[args.workload]
    m = mesh[0] * mesh[1] * mesh[2]
    frame = synth.molten_box(n, seed)
    dev = torch.device("cuda", 0)
    pos = torch.tensor(frame.pos, dtype=torch.float32, device=dev)
    q = torch.tensor(frame.q, dtype=torch.float32, device=dev)
    mu = torch.tensor(frame.mu, dtype=torch.float32, device=dev)
    box = torch.tensor(frame.box, dtype=torch.float64, device=dev)
    v = synth.random_cotangents(n, 11, scale_r=0.1)
    vr, vq, vm = (torch.tensor(x, dtype=torch.float32, device=dev) for x in v)
    plan = Plan(mesh, p, alpha, max_atoms=n, keep_phi=True, concurrent=not args.sequential,
                separate_spread=bool(args.separate_spread))
    fo = {"energy": torch.empty(3, dtype=torch.float64, device=dev),
          "dE_dpos": torch.empty(n, 3, device=dev), "dE_dq": torch.empty(n, device=dev),
          "dE_dmu": torch.empty(n, 3, device=dev)}
    bo = {"g_pos": torch.empty(n, 3, device=dev), "g_q": torch.empty(n, device=dev),
          "g_mu": torch.empty(n, 3, device=dev)}
    so = {**fo, **bo}

    def step():
        if args.sequential:
            plan.forward(pos, q, mu, box, out=fo)
            plan.backward(pos, q, mu, box, vr, vq, vm, out=bo)
        else:
            plan.step(pos, q, mu, box, vr, vq, vm, out=so)

    for _ in range(args.warmup):
        step()
    plan.status()
    torch.cuda.synchronize()

    # per-kind launch durations (short pass, one kind at a time)
    kernels_us, per_step_us = {}, {}
    for kind in _lib.KERNEL_KINDS:
        plan.timer(kind)
        for _ in range(args.breakdown_steps):
            step()
        launches, ms = plan.timer_read()
        if launches:
            kernels_us[kind] = round(1e3 * ms / launches, 3)
            per_step_us[kind] = 1e3 * ms / args.breakdown_steps
    plan.timer(None)
    # the fused plane spread performs the forward slab transform: no r2c launches
    fused = "fft_r2c" not in kernels_us
    spec = spec_bytes(mesh) if fused else 0
    dominant = max((k for k in per_step_us if alg_bytes(k, n, m, not args.sequential, spec) > 0),
                   key=lambda k: per_step_us[k])

    # eager timed region: K steps, the dominant kernel's launches bracketed by HIP events
    args.steps += args.steps % 2          # the graph needs an even count (set parity)
    plan.timer(dominant)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, dom_ms = plan.timer_read()
    plan.timer(None)
    eager_ms = (t1 - t0) * 1e3 / args.steps
    if args.graph:
        # the same K steps captured into one HIP graph (launches in a graph cannot be
        # timed by events here): one untimed replay, then the timed one
        plan.step_capture(args.steps, pos, q, mu, box, vr, vq, vm, out=so)
        plan.step_replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step_replay()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    plan.timer(None)
    plan.status()
    ms = (t1 - t0) * 1e3 / args.steps
    value = n * args.steps / (t1 - t0) / 1e6
    replays = None
    if args.graph and args.replays > 0:
        # distribution over single replays of a two-step graph (HIP events around each)
        plan.step_capture(2, pos, q, mu, box, vr, vq, vm, out=so)
        for _ in range(5):
            plan.step_replay()
        per = [t / 2 for t in device_ms(plan.step_replay, args.replays)]
        plan.status()
        replays = {"replays": args.replays, "steps_per_replay": 2,
                   "ms_per_step_median": round(pct(per, 0.5), 5),
                   "ms_per_step_p10": round(pct(per, 0.1), 5),
                   "ms_per_step_p90": round(pct(per, 0.9), 5),
                   "note": "HIP events around each replay of a captured two-step graph"}

    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    dur_s = dom_ms / launches / 1e3
    ab = alg_bytes(dominant, n, m, not args.sequential, spec)
    achieved = ab / dur_s / 1e9
    traffic = read_traffic(dominant, args.workload)
    band = plan.spread_kind == "band"
    sym = kernel_symbol(dominant, not args.sequential, fused, band, is_slab(mesh))
    rp_us = read_kernel_stats(args.workload + ("_sequential" if args.sequential else ""), sym)
    copy_bw = copy_bandwidth(dev)
    lds = lds_peak(dev)
    lds_bytes = read_lds_bytes(args.workload, sym)
    line = {
        "metric": "PME q+mu fwd+bwd Matom-steps/s @32k atoms",
        "value": value,
        "unit": "Matom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"molten-salt box, {n} ions (+-1 e, mu ~ N(0, 0.1^2) e*A), "
                               f"cubic L={frame.box[0, 0]:.3f} A, mesh {mesh[0]}x{mesh[1]}x{mesh[2]}, "
                               f"p={p}, alpha={alpha}, forward + Hessian-vector product",
                   "atoms": n, "mesh": list(mesh), "order": p, "alpha": alpha,
                   "call": "pme_forward; pme_backward" if args.sequential else
                           "pme_step (cotangent chain on a second stream)",
                   "launch": ("the timed steps captured into one HIP graph (pme_step_capture), "
                              "replayed once" if args.graph else "eager calls")},
        "eager": {"ms_per_step": round(eager_ms, 6), "value": round(n / eager_ms / 1e3, 3),
                  "note": "the same K steps as eager calls, timed just before; the roofline "
                          "launch durations are timed over this pass"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                     "traffic": traffic, "kernel": sym, "kind": dominant,
                     "alg_bytes_per_launch": ab, "avg_launch_us": round(dur_s * 1e6, 3),
                     "launches": launches,
                     "rocprof_avg_us": rp_us,
                     "frac_rocprof": (round(ab / (rp_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 6)
                                      if rp_us else None),
                     "frac_of_copy": round(achieved / copy_bw["GBps"], 6),
                     "copy": copy_bw,
                     "lds": {"bytes_per_launch": lds_bytes,
                             "GBps": round(lds_bytes / dur_s / 1e9, 1) if lds_bytes else None,
                             "peak_read_b128_GBps": lds["read_b128_GBps"],
                             "peak_atomic_add_u64_GBps": lds["atomic_add_u64_GBps"],
                             "frac_of_read_peak": (round(lds_bytes / dur_s / 1e9 /
                                                         lds["read_b128_GBps"], 6)
                                                   if lds_bytes else None)}},
        "replays": replays,
        "kernels_us": kernels_us,
        "spread": ("fused with the forward slab transform (one x-plane per workgroup)" if fused
                   else ("bands of y-rows of each x-plane, separate transform" if band
                         else "mesh tiles, separate transform")),
        "step_model_bytes": step_bytes(n, m, not args.sequential),
    }
    if args.cell:
        line["cell_gradient"] = cell_leg(pos, q, mu, box, mesh, p, alpha, n)
    if args.influence:
        line["optimal_influence"] = influence_leg(pos, q, mu, box, mesh, p, alpha, n, vr, vq, vm)
    if args.quad:
        line["quadrupole"] = quad_leg(pos, q, mu, box, mesh, p, alpha, n)
    if args.batched:
        line["batched"] = batched_leg()
    if args.learned:
        line["learned_dipole"] = learned_leg()
    if args.cpu_baseline and args.workload == "32k":
        line["cpu_baseline"] = cpu_baseline(frame, mesh, p, alpha, v, args.cpu_steps)
    print(json.dumps(line), flush=True)
    return 0


def _median_ms(fn, reps):
    import torch
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    times.sort()
    return times[len(times) // 2]


def cell_leg(pos, q, mu, box, mesh, p, alpha, n, reps=50):
    """The cell gradient dE^lr/dC (pme_forward_cell) on the benchmark workload: the
    forward call with and without it, median of ``reps`` timed calls each (inputs
    resident in HBM), and the launch-timer durations of the kernel variants that
    form its partials."""
    import torch

    from paper_2606_01598_amd.pme import Plan
    plan = Plan(mesh, p, alpha, max_atoms=n)
    dev = pos.device
    fo = {"energy": torch.empty(3, dtype=torch.float64, device=dev),
          "dE_dpos": torch.empty(n, 3, device=dev), "dE_dq": torch.empty(n, device=dev),
          "dE_dmu": torch.empty(n, 3, device=dev),
          "dE_dbox": torch.empty(3, 3, dtype=torch.float64, device=dev)}
    plain = {k: v for k, v in fo.items() if k != "dE_dbox"}
    for _ in range(10):
        plan.forward(pos, q, mu, box, out=plain)
        plan.forward(pos, q, mu, box, out=fo, cell=True)
    plan.status()
    t_plain = _median_ms(lambda: plan.forward(pos, q, mu, box, out=plain), reps)
    t_cell = _median_ms(lambda: plan.forward(pos, q, mu, box, out=fo, cell=True), reps)
    kern = {}
    for kind in ("fft_x", "gather"):
        for cell in (False, True):
            plan.timer(kind)
            for _ in range(10):
                plan.forward(pos, q, mu, box, out=fo if cell else plain, cell=cell)
            k, ms = plan.timer_read()
            kern[f"{kind}{'_cell' if cell else ''}"] = round(1e3 * ms / max(k, 1), 3)
    plan.timer(None)
    plan.status()
    return {"workload": "the benchmark box, pme_forward vs pme_forward_cell",
            "forward_ms": round(t_plain, 4), "forward_cell_ms": round(t_cell, 4),
            "overhead_ms": round(t_cell - t_plain, 4), "kernels_us": kern}


def quad_leg(pos, q, mu, box, mesh, p, alpha, n, reps=50):
    """The quadrupole channel (pme_forward_quad) on the benchmark workload with seeded
    second moments: the forward call with and without it, median of ``reps`` timed
    calls each (inputs resident in HBM), and the launch-timer durations of the
    binning, spread and gather variants it uses."""
    import torch

    import synth
    from paper_2606_01598_amd.pme import Plan
    plan = Plan(mesh, p, alpha, max_atoms=n)
    dev = pos.device
    th = torch.tensor(synth.random_quadrupoles(n, 27), dtype=torch.float32, device=dev)
    fo = {"energy": torch.empty(4, dtype=torch.float64, device=dev),
          "dE_dpos": torch.empty(n, 3, device=dev), "dE_dq": torch.empty(n, device=dev),
          "dE_dmu": torch.empty(n, 3, device=dev), "dE_dtheta": torch.empty(n, 6, device=dev)}
    plain = {k: v for k, v in fo.items() if k not in ("dE_dtheta", "energy")}
    plain["energy"] = torch.empty(3, dtype=torch.float64, device=dev)
    for _ in range(10):
        plan.forward(pos, q, mu, box, out=plain)
        plan.forward(pos, q, mu, box, out=fo, theta=th)
    plan.status()
    t_plain = _median_ms(lambda: plan.forward(pos, q, mu, box, out=plain), reps)
    t_quad = _median_ms(lambda: plan.forward(pos, q, mu, box, out=fo, theta=th), reps)
    kern = {}
    for kind in ("bin", "spread", "gather"):
        for quad in (False, True):
            plan.timer(kind)
            for _ in range(10):
                if quad:
                    plan.forward(pos, q, mu, box, out=fo, theta=th)
                else:
                    plan.forward(pos, q, mu, box, out=plain)
            k, ms = plan.timer_read()
            kern[f"{kind}{'_quad' if quad else ''}"] = round(1e3 * ms / max(k, 1), 3)
    plan.timer(None)
    plan.status()
    return {"workload": "the benchmark box with seeded second moments Theta, pme_forward vs "
                        "pme_forward_quad",
            "forward_ms": round(t_plain, 4), "forward_quad_ms": round(t_quad, 4),
            "quad_atom_steps_per_s": round(n / (t_quad * 1e-3), 1), "kernels_us": kern}


def influence_leg(pos, q, mu, box, mesh, p, alpha, n, vr, vq, vm, reps=50):
    """pme_step (concurrent chains) on the benchmark workload with the optimal
    influence function against the deconvolution: median step time of each and the
    x-pass launch duration (where the two differ)."""
    import torch

    from paper_2606_01598_amd.pme import Plan
    res = {"workload": "the benchmark box, pme_step with each influence function"}
    for opt in (False, True):
        plan = Plan(mesh, p, alpha, max_atoms=n, concurrent=True, optimal_influence=opt)
        for _ in range(10):
            plan.step(pos, q, mu, box, vr, vq, vm)
        plan.status()
        t = _median_ms(lambda: plan.step(pos, q, mu, box, vr, vq, vm), reps)
        plan.timer("fft_x")
        for _ in range(10):
            plan.step(pos, q, mu, box, vr, vq, vm)
        k, ms = plan.timer_read()
        plan.timer(None)
        plan.status()
        key = "optimal" if opt else "deconvolution"
        res[f"{key}_step_ms"] = round(t, 4)
        res[f"{key}_fft_x_us"] = round(1e3 * ms / max(k, 1), 3)
    return res


def influence_compare(out_path=None):
    """Accuracy per mesh point of the two influence functions: RMS force error of the
    GPU PME (forward) against the FP64 explicit Ewald long-range forces on the host,
    for molten-salt boxes of 512 ions (three configurations) over meshes from 3 A to
    1 A, p = 4 and 6, alpha = 0.45 / A.  Writes profiles/influence_accuracy_molten512.txt."""
    import numpy as np
    import torch

    import synth
    from oracle import ewald as oew
    from paper_2606_01598_amd.pme import Plan

    dev = torch.device("cuda", 0)
    rows = []
    a = 0.45
    frames = [synth.molten_box(512, 30 + s) for s in range(3)]
    refs = [oew.ewald_long_range(f.pos, f.q, f.mu, f.box, a)[1] for f in frames]
    L = frames[0].box[0, 0]
    for p in (4, 6):
        for m in (8, 10, 12, 16, 20, 24):
            errs = {}
            for opt in (False, True):
                e = []
                for f, gref in zip(frames, refs):
                    plan = Plan((m, m, m), p, a, max_atoms=f.n, optimal_influence=opt)
                    t = lambda x: torch.tensor(x, dtype=torch.float32, device=dev)
                    out = plan.forward(t(f.pos), t(f.q), t(f.mu),
                                       torch.tensor(f.box, dtype=torch.float64, device=dev))
                    g = out["dE_dpos"].double().cpu().numpy()
                    e.append(float(np.sqrt(np.mean((g - gref) ** 2) / np.mean(gref ** 2))))
                errs[opt] = float(np.mean(e))
            rows.append((p, m, L / m, errs[False], errs[True]))
    lines = [
        "# Accuracy per mesh point of the influence functions: mean over 3 molten-salt",
        "# boxes of 512 ions (L = %.2f A) of ||F_PME - F_Ewald||_rms / ||F_Ewald||_rms," % L,
        "# F_PME from the GPU (forward), F_Ewald the FP64 explicit Ewald long-range force",
        "# (oracle, host); alpha = 0.45 / A",
        "# command: python -u bench.py --influence-compare 1",
        f"# source digest of the PME sources in paper_2606_01598_amd/csrc (bench.source_digest): {source_digest()}",
        "",
        f"{'p':>3s} {'mesh':>5s} {'h (A)':>7s} {'deconvolution':>14s} {'optimal':>10s} {'ratio':>7s}",
    ]
    for p, m, h, e0, e1 in rows:
        lines.append(f"{p:3d} {m:5d} {h:7.3f} {e0:14.3e} {e1:10.3e} {e1 / e0:7.3f}")
    out = out_path or os.path.join(ROOT, "profiles", "influence_accuracy_molten512.txt")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(open(out).read())
    return 0


def batched_leg(n_boxes=64, seed=6, reps=20):
    """64 molten-salt boxes, atom counts log-uniform in [64, 4096], meshes of about
    1 A (16..64 per side), p = 6, alpha = 0.30: one training step (forward,
    Hessian-vector product, force-loss double backward) as one replay of a HIP
    graph over the batch, against 64 sequential un-graphed single-box plans doing
    the same three calls.  Tiles and FFT lines per workgroup come from the
    autotuner."""
    import tempfile

    import numpy as np
    import torch

    import synth
    from paper_2606_01598_amd import autotune
    from paper_2606_01598_amd.batch import Batch
    from paper_2606_01598_amd.pme import Plan

    dev = torch.device("cuda", 0)
    frames, meshes = synth.batch_boxes(n_boxes, seed)
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
    boxes = []
    for b, f in enumerate(frames):
        vr, vq, vm = synth.random_cotangents(f.n, 300 + b, scale_r=0.1)
        vf = synth.random_cotangents(f.n, 600 + b, scale_r=0.1)[0]
        boxes.append({"mesh": meshes[b], "pos": t(f.pos), "q": t(f.q), "mu": t(f.mu),
                      "box": torch.tensor(f.box, dtype=torch.float64, device=dev),
                      "v": [t(vr), t(vq), t(vm)], "vf": t(vf)})
    cache = os.path.join(tempfile.gettempdir(), "pme_bench_tiles.json")
    t0 = time.perf_counter()
    cfgs, timed = autotune.tune(boxes, 6, 0.30, cache_path=cache, steps=2,
                                candidates=((8, 8, 16), (8, 16, 16), (16, 16, 16)),
                                lines=(8, 16, 32))
    tune_s = time.perf_counter() - t0
    tiles = [c.tile for c in cfgs]
    lines = [c.fft_lines for c in cfgs]
    plans = [Plan(b["mesh"], 6, 0.30, max_atoms=b["pos"].shape[0], tile=tiles[k],
                  fft_lines=lines[k] or None)
             for k, b in enumerate(boxes)]
    outs = []

    def sequential():
        outs.clear()
        for pl, b in zip(plans, boxes):
            o = pl.forward(b["pos"], b["q"], b["mu"], b["box"])
            g = pl.backward(b["pos"], b["q"], b["mu"], b["box"], *b["v"])
            gf = pl.backward(b["pos"], b["q"], b["mu"], b["box"], b["vf"], None, None)
            outs.append((o, g, gf))

    for _ in range(2):
        sequential()
    seq_ms = _median_ms(sequential, 5)
    cat = lambda k: torch.cat([b[k] for b in boxes]).contiguous()
    pos, q, mu = cat("pos"), cat("q"), cat("mu")
    box = torch.stack([b["box"] for b in boxes]).contiguous()
    vr = torch.cat([b["v"][0] for b in boxes]); vq = torch.cat([b["v"][1] for b in boxes])
    vm = torch.cat([b["v"][2] for b in boxes]); vf = cat("vf")
    bt = Batch(meshes, [f.n for f in frames], 6, 0.30, tiles=tiles, fft_lines=lines)
    N, B = bt.total, bt.nbox
    emp = lambda *sh: torch.empty(*sh, dtype=torch.float32, device=dev)
    step = {"pos": pos, "q": q, "mu": mu, "box": box,
            "energy": torch.empty(B, 3, dtype=torch.float64, device=dev),
            "dE_dpos": emp(N, 3), "dE_dq": emp(N), "dE_dmu": emp(N, 3), "v_pos": vr, "v_q": vq,
            "v_mu": vm, "g_pos": emp(N, 3), "g_q": emp(N), "g_mu": emp(N, 3), "vf_pos": vf,
            "gf_pos": emp(N, 3), "gf_q": emp(N), "gf_mu": emp(N, 3)}
    bt.capture(step)
    for _ in range(3):
        bt.replay()
    graph_ms = _median_ms(bt.replay, reps)
    bt.status()
    # largest relative difference between the sequential and the graph results
    worst = 0.0
    for k, (o, g, gf) in enumerate(outs):
        s0, s1 = int(bt.offsets[k]), int(bt.offsets[k + 1])
        pairs = [(step["energy"][k], o["energy"]), (step["dE_dpos"][s0:s1], o["dE_dpos"]),
                 (step["g_pos"][s0:s1], g["g_pos"]), (step["gf_pos"][s0:s1], gf["g_pos"]),
                 (step["g_mu"][s0:s1], g["g_mu"])]
        for x, y in pairs:
            den = float(y.abs().max().clamp_min(1e-30))
            worst = max(worst, float((x - y).abs().max()) / den)
    return {"workload": f"{B} molten-salt boxes, {N} ions in all (64..4096 per box, log-uniform), "
                        "meshes 16..64 at ~1 A, p=6, alpha=0.3; forward + H v + force-loss H v",
            "graph_ms": round(graph_ms, 4), "sequential_ms": round(seq_ms, 4),
            "speedup": round(seq_ms / graph_ms, 3),
            "graph_Matom_steps_per_s": round(N / graph_ms / 1e3, 3),
            "max_rel_diff": worst, "autotune_keys_timed": timed, "autotune_s": round(tune_s, 2),
            "autotune_choices": sorted({f"{c.tile[0]}x{c.tile[1]}x{c.tile[2]}/lines {c.fft_lines}"
                                        for c in cfgs})}


def _thole_frame(seed: int):
    """A 4096-ion box of the learned-head workload (module-level: worker processes
    draw the boxes in parallel)."""
    import synth
    return synth.molten_box(4096, seed)


def learned_leg(n_train=256, n_val=32, epochs=12, workers=8):
    """4096-ion boxes of the Thole-damped polarizable model (polarizabilities
    0.15 / 3.5 A^3, L = 50.4 A, mesh 50^3, p = 6, alpha = 0.30, r_c = 10 A): the
    self-consistent dipoles by PCG to 1e-6 e*A (the teacher) against the trained
    dipole network (features + network + one model evaluation).  Training boxes
    seeds 1000.., held-out boxes seeds 2000.. (256 / 32); Adam with a linear warmup
    and exponential decay.  Reports force and dipole errors on the held-out boxes
    (absolute and relative to the teacher's RMS), the same force error with the
    dipoles left at zero, and times per box both as host-driven calls and replayed
    from HIP graphs (the SCF with a fixed iteration count, the network path)."""
    import multiprocessing as mp

    import numpy as np
    import torch

    import synth
    from paper_2606_01598_amd.dip import DipPlan, Trainer
    from paper_2606_01598_amd.pme import Plan
    from paper_2606_01598_amd.pol import PolPlan

    dev = torch.device("cuda", 0)
    n = 4096
    L = synth.molten_side(n)
    box_np = np.eye(3) * L
    box = torch.tensor(box_np, dtype=torch.float64, device=dev)
    mesh, p, alpha, rc = (50, 50, 50), 6, 0.30, 10.0
    pme = Plan(mesh, p, alpha, max_atoms=n, keep_phi=True)
    polp = PolPlan(box_np, alpha, rc, max_atoms=n)
    dip = DipPlan(box_np, n, cutoff=5.0)
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
    seeds = [1000 + k for k in range(n_train)] + [2000 + k for k in range(n_val)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        frames = pool.map(_thole_frame, seeds, chunksize=8)
    gen_s = time.perf_counter() - t0
    data, scf_ms, iters = [], [], []
    for k, f in enumerate(frames):
        pos, q, a = t(f.pos), t(f.q), t(np.where(f.q > 0, 0.15, 3.5))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mu, it, res = polp.scf(pme, pos, q, a, box, tol=1e-6, max_iter=300)
        o = polp.model(pme, pos, q, mu, a, box, dU_dmu=False)
        torch.cuda.synchronize()
        scf_ms.append((time.perf_counter() - t1) * 1e3)
        iters.append(it)
        feat, vec = dip.features(pos, q)
        data.append({"pos": pos, "q": q, "pol": a, "feat": feat, "vec": vec, "U": o["energy"],
                     "dUdr": o["dU_dpos"], "mu": mu})
    train, val = data[:n_train], data[n_train:]
    steps = epochs * n_train

    def fit(charge_head, conservative):
        trn = Trainer(dip, polp, pme, box, synth.mlp_init(7), lr=3e-3, lE=1.0, lF=1.0,
                      warmup=max(1, steps // 20), decay=0.1, decay_steps=steps,
                      qtheta0=synth.charge_head_init(8) if charge_head else None,
                      conservative=conservative)
        order = np.random.default_rng(5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(epochs):
            for k in order.permutation(n_train):
                trn.step(train[k])
        torch.cuda.synchronize()
        return trn, time.perf_counter() - t0

    tr, train_s = fit(False, False)

    def errors(mu, b):
        s = polp.model(pme, b["pos"], b["q"], mu, b["pol"], box, energy=False, dU_dmu=False)
        df = float(torch.sqrt(torch.mean((s["dU_dpos"] - b["dUdr"]) ** 2)))
        ref = float(torch.sqrt(torch.mean(b["dUdr"] ** 2)))
        dm = float(torch.sqrt(torch.mean(torch.sum((mu - b["mu"]) ** 2, dim=1))))
        mref = float(torch.sqrt(torch.mean(torch.sum(b["mu"] ** 2, dim=1))))
        return df, ref, dm, mref

    zero = torch.zeros(n, 3, dtype=torch.float32, device=dev)
    e_nn = np.array([errors(tr.predict(b["feat"], b["vec"]), b) for b in val])
    e_zero = np.array([errors(zero, b) for b in val])

    # the charge head and training on conservative forces: the same schedule, the
    # forces each model is trained on (conservative -dU(r, q(r), mu(r))/dr or the
    # Hellmann-Feynman -dU/dr at the predicted charges and dipoles) on held-out boxes
    heads = {}
    for name, ch, cons in (("hf_charge", True, False), ("conservative", False, True),
                           ("conservative_charge", True, True)):
        trn, secs = fit(ch, cons)
        ev = [trn.evaluate(b) for b in val]
        df = np.array([float(torch.sqrt(torch.mean((o["dU_dpos"] - b["dUdr"]) ** 2)))
                       / float(torch.sqrt(torch.mean(b["dUdr"] ** 2))) for o, b in zip(ev, val)])
        dq = [float(torch.sqrt(torch.mean((o["q"] - b["q"]) ** 2))) for o, b in zip(ev, val)]
        heads[name] = {"force_rel": float(df.mean()), "charge_rms_shift": float(np.mean(dq)),
                       "train_ms_per_step": round(secs * 1e3 / steps, 4)}
    b = val[0]

    def infer():
        feat, vec = dip.features(b["pos"], b["q"])
        mu = dip.forward(tr.theta, feat, vec)
        return polp.model(pme, b["pos"], b["q"], mu, b["pol"], box, dU_dmu=False)

    def infer_conservative():
        # the conservative student force: dU/dr plus the position vector-Jacobian
        # product of the dipole head with dU/dmu
        feat, vec = dip.features(b["pos"], b["q"])
        mu = dip.forward(tr.theta, feat, vec)
        s = polp.model(pme, b["pos"], b["q"], mu, b["pol"], box)
        return dip.position_vjp(tr.theta, b["pos"], b["q"], feat, vec, s["dU_dmu"],
                                base=s["dU_dpos"])

    for _ in range(3):
        infer()
        infer_conservative()
    nn_ms = _median_ms(infer, 20)
    cons_ms = _median_ms(infer_conservative, 20)
    scf_med = float(np.median(scf_ms[n_train:]))

    # HIP graphs: plans of their own (a captured call sequence leaves the plans'
    # host-side counter sets as if it had run: an even number of binnings per graph)
    k_fix = int(max(iters[n_train:]))
    k_fix += k_fix % 2                       # 1 + k_fix + 1 binnings per captured solve
    pme_g = Plan(mesh, p, alpha, max_atoms=n, keep_phi=True)
    pol_g = PolPlan(box_np, alpha, rc, max_atoms=n, fixed_iters=True)
    mu_g = torch.zeros(n, 3, dtype=torch.float32, device=dev)

    def scf_fixed():
        pol_g.scf(pme_g, b["pos"], b["q"], b["pol"], box, max_iter=k_fix, mu=mu_g)
        return pol_g.model(pme_g, b["pos"], b["q"], mu_g, b["pol"], box)

    def nn_twice():
        o = None
        for _ in range(2):
            feat, vec = dip.features(b["pos"], b["q"])
            mu = dip.forward(tr.theta, feat, vec)
            o = pol_g.model(pme_g, b["pos"], b["q"], mu, b["pol"], box, dU_dmu=False)
        return o

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ref_scf = {k: v.clone() for k, v in scf_fixed().items()}
        ref_nn = nn_twice()["dU_dpos"].clone()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g_scf, g_nn = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_scf):
        out_scf = scf_fixed()
    with torch.cuda.graph(g_nn):
        out_nn = nn_twice()
    diffs = []
    for _ in range(3):
        g_scf.replay()
        torch.cuda.synchronize()
        g_nn.replay()
        torch.cuda.synchronize()
        diffs.append(max(float((out_scf["dU_dpos"] - ref_scf["dU_dpos"]).abs().max()),
                         float((out_nn["dU_dpos"] - ref_nn).abs().max())))
    scf_g = sorted(device_ms(g_scf.replay, 20))[10]
    nn_g = sorted(device_ms(g_nn.replay, 20))[10] / 2
    g_scf.replay()
    torch.cuda.synchronize()
    stat = float(torch.sqrt(torch.mean(out_scf["dU_dmu"] ** 2)))
    f_fix = float(torch.sqrt(torch.mean((out_scf["dU_dpos"] - b["dUdr"]) ** 2)))
    return {"workload": f"{n}-ion Thole boxes, L={L:.1f} A, mesh 50^3, p=6, alpha=0.3, r_c=10 A; "
                        f"{n_train} training boxes (seeds 1000..), {n_val} held-out boxes "
                        f"(seeds 2000..), {epochs} epochs, Adam lr 3e-3 with linear warmup over "
                        f"{tr.warmup} steps and exponential decay to 0.1 over {steps} steps",
            "scf_ms": round(scf_med, 3), "scf_iterations": int(np.median(iters)),
            "nn_ms": round(nn_ms, 4), "speedup": round(scf_med / nn_ms, 2),
            "graph": {"scf_ms": round(scf_g, 4), "scf_fixed_iterations": k_fix,
                      "nn_ms": round(nn_g, 4), "speedup": round(scf_g / nn_g, 2),
                      "scf_stationarity_rms_dU_dmu": stat,
                      "scf_force_rmse_vs_converged": f_fix,
                      "replay_max_abs_diff_vs_eager": max(diffs),
                      "note": "one replay per box: PCG with the held-out maximum iteration count "
                              "(rounded up to even) + the model evaluation, against features + "
                              "network + model evaluation (two per graph, halved)"},
            "nn_conservative_ms": round(cons_ms, 4),
            "force_rmse_nn": float(e_nn[:, 0].mean()),
            "force_rel_nn": float((e_nn[:, 0] / e_nn[:, 1]).mean()),
            "force_rmse_zero_dipoles": float(e_zero[:, 0].mean()),
            "force_rel_zero_dipoles": float((e_zero[:, 0] / e_zero[:, 1]).mean()),
            "dipole_rmse_nn": float(e_nn[:, 2].mean()),
            "dipole_rel_nn": float((e_nn[:, 2] / e_nn[:, 3]).mean()),
            "force_unit": "e^2/A^2", "dipole_unit": "e*A",
            "train_s": round(train_s, 2), "train_ms_per_step": round(train_s * 1e3 / steps, 4),
            "heads": heads,
            "heads_note": "hf_charge: charge head + dipole head on Hellmann-Feynman forces; "
                          "conservative: dipole head on -dU(r, mu(r))/dr (second order); "
                          "conservative_charge: both heads on -dU(r, q(r), mu(r))/dr; "
                          "force_rel is the held-out force RMSE over the teacher's RMS force, "
                          "charge_rms_shift the RMS of q - formal charge",
            "generate_s": round(gen_s, 1)}


def _traffic_path(kind: str, workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"{kind}_{workload}_traffic.txt")


def read_traffic(kind: str, workload: str):
    """HBM bytes per launch of `kind` from its committed counter summary, or None
    when there is none or it was taken on other kernel sources."""
    path = _traffic_path(kind, workload)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for ln in fh:
            if ":" in ln:
                k, _, v = ln.partition(":")
                vals[k.strip()] = v.strip()
    if vals.get("sources") != source_digest(kind):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _counter_means(path: str, counter: str):
    """Mean per-dispatch value (KiB) of `counter` for every kernel in a rocprofv3
    counter-collection CSV.  For the copy kernel only the dispatches of the largest
    grid (the calibration copy) are kept."""
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") == counter:
                rows.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    copy_grid = max([g for k, g, _ in rows if "copyBuffer" in k], default=0)
    sums, cnt = {}, {}
    for k, g, v in rows:
        if "copyBuffer" in k and g != copy_grid:
            continue
        sums[k] = sums.get(k, 0.0) + v
        cnt[k] = cnt.get(k, 0) + 1
    return {k: (sums[k] / cnt[k], cnt[k]) for k in sums}


# bench.py flags of the counter passes: a few steps (a profiler with counters slows
# every launch), no side legs, one breakdown step per kind, the copy calibration
PMC_FLAGS = ("--steps 3 --warmup 2 --cpu-baseline 0 --batched 0 --learned 0 "
             "--copy-calibration 1 --breakdown-steps 1")


def traffic_summary(args) -> int:
    fetch = _counter_means(args.traffic_summary[0], "FETCH_SIZE")
    write = _counter_means(args.traffic_summary[1], "WRITE_SIZE")
    kind = args.kernel or "spread_tangent"
    step = not args.sequential
    fused = any(kernel_symbol(kind, step, True) in k for k in fetch)
    band = not fused and any(kernel_symbol(kind, step, False, True) in k for k in fetch)
    sym = kernel_symbol(kind, not args.sequential, fused, band)

    def find(table, key):
        hits = [k for k in table if key in k]
        if not hits:
            raise SystemExit(f"no dispatch of {key} in the counter file")
        return hits[0]

    copy_f = find(fetch, "copyBuffer")
    copy_w = find(write, "copyBuffer")
    # KiB read / written per copy dispatch vs the bytes it moves
    f_scale = COPY_BYTES / (fetch[copy_f][0] * 1024.0)
    w_scale = COPY_BYTES / (write[copy_w][0] * 1024.0)
    kf = find(fetch, sym)
    kw = find(write, sym)
    fb = fetch[kf][0] * 1024.0 * f_scale
    wb = write[kw][0] * 1024.0 * w_scale
    n, _, mesh, _, _ = WORKLOADS[args.workload]
    m = mesh[0] * mesh[1] * mesh[2]
    out = _traffic_path(kind, args.workload)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as fh:
        fh.write(f"# HBM traffic of {sym} ({kind}), workload {args.workload}\n")
        fh.write("# commands (from the repository root):\n")
        flags = COUNTER_FLAGS if args.sequential else STEP_COUNTER_FLAGS
        seq = " --sequential 1" if args.sequential else ""
        for ctr, d in (("FETCH_SIZE", "<D1>"), ("WRITE_SIZE", "<D2>")):
            fh.write(f"#   rocprofv3 --pmc {ctr} --output-format csv -d {d} -o run -- "
                     f"python -u bench.py {flags} --workload {args.workload}\n")
        fh.write("#   python bench.py --traffic-summary <D1>/run_counter_collection.csv "
                 f"<D2>/run_counter_collection.csv --kernel {kind} --workload {args.workload}"
                 f"{seq}\n")
        fh.write(f"# sources: digest of {', '.join(sorted(set(KERNEL_SOURCES[kind]) | {'kernels.h', 'pme_common.h'}))} "
                 f"(bench.source_digest('{kind}'))\n")
        fh.write(f"sources: {source_digest(kind)}\n")
        fh.write(f"kernel: {kf}\n")
        fh.write(f"dispatches: {fetch[kf][1]} (FETCH_SIZE), {write[kw][1]} (WRITE_SIZE)\n")
        fh.write(f"fetch_kib_per_dispatch: {fetch[kf][0]:.1f}\n")
        fh.write(f"write_kib_per_dispatch: {write[kw][0]:.1f}\n")
        fh.write(f"copy_kernel: {copy_f}\n")
        fh.write(f"copy_fetch_kib: {fetch[copy_f][0]:.1f} for {COPY_BYTES} bytes read "
                 f"(scale {f_scale:.4f})\n")
        fh.write(f"copy_write_kib: {write[copy_w][0]:.1f} for {COPY_BYTES} bytes written "
                 f"(scale {w_scale:.4f})\n")
        fh.write(f"fetch_bytes_per_launch: {fb:.0f}\n")
        fh.write(f"write_bytes_per_launch: {wb:.0f}\n")
        fh.write(f"traffic_bytes_per_launch: {fb + wb:.0f}\n")
        fh.write(f"alg_bytes_per_launch: {alg_bytes(kind, n, m, True, spec_bytes(mesh) if fused else 0)}\n")
    print(open(out).read())
    return 0


# counter passes of the per-kernel summary (one rocprofv3 run each; every pass stays
# within the per-block counter limits)
COUNTER_PASSES = (
    "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR "
    "SQ_WAVE_CYCLES SQ_BUSY_CYCLES",
    "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_LDS "
    "SQ_WAIT_INST_ANY SQ_INSTS_LDS_ATOMIC SQ_LDS_IDX_ACTIVE SQ_INSTS_BRANCH",
    "SQ_INSTS_LDS_LOAD_BANDWIDTH SQ_INSTS_LDS_STORE_BANDWIDTH SQ_INSTS_LDS_ATOMIC_BANDWIDTH "
    "SQ_INSTS_VALU_FMA_F32 SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_CVT GRBM_GUI_ACTIVE",
    "FETCH_SIZE",
    "WRITE_SIZE",
)
COUNTER_FLAGS = ("--steps 3 --warmup 2 --cpu-baseline 0 --batched 0 --learned 0 --cell 0 "
                 "--influence 0 --quad 0 --copy-calibration 1 --breakdown-steps 1 --sequential 1 "
                 "--graph 0 --replays 0")
# the same passes over the concurrent pme_step (its kernel variants: the forward
# spread from the tangent records, the gather that also forms the forward outputs)
STEP_COUNTER_FLAGS = COUNTER_FLAGS.replace(" --sequential 1", "")


def _pass_rows(path):
    """{kernel: {counter: mean per dispatch}} and {kernel: (grid, wg, lds, vgpr)} of a
    rocprofv3 counter-collection CSV (the calibration copy: its largest grid only)."""
    vals, meta = {}, {}
    rows = list(csv.DictReader(open(path)))
    copy_grid = max([int(r["Grid_Size"]) for r in rows if "copyBuffer" in r["Kernel_Name"]],
                    default=0)
    for r in rows:
        k = r["Kernel_Name"].replace("void ", "").replace("pme::(anonymous namespace)::", "")
        k = k.replace("(anonymous namespace)::", "").split("(")[0]
        if "copyBuffer" in k and int(r["Grid_Size"]) != copy_grid:
            continue
        vals.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        meta[k] = (int(r["Grid_Size"]), int(r["Workgroup_Size"]), int(r["LDS_Block_Size"]),
                   int(r.get("VGPR_Count") or r.get("Arch_VGPR_Count") or 0))
    return ({k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in vals.items()}, meta)


def counter_summary(args) -> int:
    """profiles/kernels_<workload>_counters.txt: per-kernel instruction mix, LDS
    traffic and bank conflicts, occupancy and HBM bytes of the two-call step, from the
    rocprofv3 counter passes in the directories given (one per COUNTER_PASSES entry)."""
    merged, meta = {}, {}
    for d in args.counter_summary:
        v, m = _pass_rows(os.path.join(d, "run_counter_collection.csv"))
        for k, cs in v.items():
            merged.setdefault(k, {}).update(cs)
        meta.update(m)
    copy = next(k for k in merged if "copyBuffer" in k)
    f_scale = COPY_BYTES / (merged[copy]["FETCH_SIZE"] * 1024.0)
    w_scale = COPY_BYTES / (merged[copy]["WRITE_SIZE"] * 1024.0)
    n, _, mesh, p, _ = WORKLOADS[args.workload]
    step = bool(args.counter_step)
    out = os.path.join(ROOT, "profiles", f"kernels_{args.workload}{'_step' if step else ''}_counters.txt")
    flags = STEP_COUNTER_FLAGS if step else COUNTER_FLAGS
    call = ("concurrent pme_step (under the counters each kernel runs alone on the GPU)" if step
            else "two-call step (pme_forward; pme_backward, each kernel alone on the GPU)")
    lines = [
        f"# rocprofv3 counters of the PME kernels, {call},",
        f"# {n}-ion molten-salt box, mesh {mesh[0]}^3, p = {p}, one MI355X",
        "# commands (repository root), one run per counter pass:",
    ]
    for i, ps in enumerate(COUNTER_PASSES):
        lines.append(f"#   rocprofv3 --pmc {ps} --output-format csv -d <D{i + 1}> -o run -- "
                     f"python -u bench.py {flags} --workload {args.workload}")
    lines += [
        "#   python bench.py --counter-summary <D1> <D2> <D3> <D4> <D5> --workload " + args.workload
        + (" --counter-step 1" if step else ""),
        "# per wave: instructions issued per wavefront (SQ_INSTS_* / SQ_WAVES);",
        "# lds_bytes = 64 * (SQ_INSTS_LDS_{LOAD,STORE,ATOMIC}_BANDWIDTH) per launch;",
        "# bank_conflict = SQ_LDS_BANK_CONFLICT / (SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT)",
        "#   (stall cycles per LDS access cycle);",
        "# occupancy = 400 SQ_WAVE_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs) / 256 CUs / 32 waves (%);",
        "# hbm = FETCH_SIZE, WRITE_SIZE scaled by a 256 MiB device copy in the same run "
        f"(x {f_scale:.3f}, x {w_scale:.3f});",
        "# vgpr, lds_alloc: per workitem registers and LDS bytes per workgroup of the dispatch.",
        f"# source digest of the PME sources in paper_2606_01598_amd/csrc (bench.source_digest): {source_digest()}",
        "",
        f"{'kernel':28s} {'grid':>8s} {'wg':>5s} {'vgpr':>5s} {'lds_alloc':>9s} {'waves':>7s} "
        f"{'valu/w':>7s} {'salu/w':>7s} {'lds/w':>6s} {'ldsat/w':>7s} {'vmem/w':>7s} "
        f"{'lds_MB':>7s} {'bank_cf':>7s} {'occ%':>5s} {'hbm_MB':>7s}",
    ]
    lds_lines = []
    order = [KERNEL_SYMBOL[k] for k in ("bin", "bin_tangent", "spread", "spread_tangent")]
    order += [FUSED_SYMBOL[k] for k in ("spread", "spread_tangent")]
    order += [BAND_SYMBOL[k] for k in ("spread", "spread_tangent")]
    order += [FUSED_STEP_SPREAD, BAND_STEP_SPREAD]
    order += [KERNEL_SYMBOL[k] for k in ("fft_r2c", "fft_x", "fft_c2r", "gather", "gather_hvp")]
    order += ["k_gather_hvp<6, true>"]
    for k in order:
        if k not in merged:
            continue
        c = merged[k]
        grid, wg, lds_alloc, vgpr = meta[k]
        waves = max(c.get("SQ_WAVES", 0.0), 1.0)
        pw = lambda name: c.get(name, float("nan")) / waves
        lds_b = 64.0 * sum(c.get(x, 0.0) for x in ("SQ_INSTS_LDS_LOAD_BANDWIDTH",
                                                   "SQ_INSTS_LDS_STORE_BANDWIDTH",
                                                   "SQ_INSTS_LDS_ATOMIC_BANDWIDTH"))
        act = c.get("SQ_LDS_IDX_ACTIVE", 0.0)
        cf = c.get("SQ_LDS_BANK_CONFLICT", 0.0)
        bank = cf / (act - cf) if act > cf else float("nan")
        gui = c.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
        occ = 400.0 * c.get("SQ_WAVE_CYCLES", 0.0) / gui / 256 / 32 if gui else float("nan")
        hbm = c.get("FETCH_SIZE", 0.0) * 1024 * f_scale + c.get("WRITE_SIZE", 0.0) * 1024 * w_scale
        lines.append(f"{k[:28]:28s} {grid:8d} {wg:5d} {vgpr:5d} {lds_alloc:9d} {int(waves):7d} "
                     f"{pw('SQ_INSTS_VALU'):7.0f} {pw('SQ_INSTS_SALU'):7.0f} "
                     f"{pw('SQ_INSTS_LDS'):6.0f} {pw('SQ_INSTS_LDS_ATOMIC'):7.1f} "
                     f"{pw('SQ_INSTS_VMEM_RD') + pw('SQ_INSTS_VMEM_WR'):7.1f} {lds_b / 1e6:7.2f} "
                     f"{bank:7.3f} {occ:5.1f} {hbm / 1e6:7.2f}")
        lds_lines.append(f"lds_bytes_per_launch {k} {lds_b:.0f}")
    lines += ["", "# LDS bytes per launch (read by bench.py for the roofline's LDS figure):"]
    lines += lds_lines
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(open(out).read())
    return 0


def kernel_stats_summary(args) -> int:
    """profiles/pme_step_<workload>[_sequential]_kernel_stats.txt from rocprofv3's
    kernel_stats.csv, with bench.py's own launch timer beside it when --bench-line
    names the log of the same command run without the profiler."""
    rows = []
    with open(args.kernel_stats) as fh:
        for r in csv.DictReader(fh):
            name = r["Name"].replace("void ", "").replace("pme::(anonymous namespace)::", "")
            name = name.replace("(anonymous namespace)::", "")
            name = name.split("(")[0] if "(" in name else name
            rows.append((name, int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    rows.sort(key=lambda x: -x[5])
    bench_us, bench_val = {}, None
    if args.bench_line:
        with open(args.bench_line) as fh:
            for ln in fh:
                if ln.startswith("{") and '"kernels_us"' in ln:
                    d = json.loads(ln)
                    step = "pme_step" in d["config"].get("call", "")
                    fz = "fft_r2c" not in d["kernels_us"]
                    bd = d.get("spread", "").startswith("bands")
                    bench_us = {kernel_symbol(k, step, fz, bd): v for k, v in d["kernels_us"].items()}
                    bench_val = (d["value"], d["unit"], d["roofline"]["kernel"],
                                 d["roofline"]["avg_launch_us"])
                    break
    suffix = "_sequential" if args.sequential else ""
    out = os.path.join(ROOT, "profiles", f"pme_step_{args.workload}{suffix}_kernel_stats.txt")
    n, _, mesh, p, _ = WORKLOADS[args.workload]
    call = "pme_forward; pme_backward" if args.sequential else "pme_step (concurrent chains)"
    seq = " --sequential 1" if args.sequential else ""
    # off the benchmark workload the unprofiled run skips the host baseline and the
    # side legs, as the profiled one does
    extra = "" if args.workload == "32k" else (" --steps 20 --warmup 5 --cpu-baseline 0 "
                                               "--batched 0 --learned 0")
    lines = [
        f"# rocprofv3 kernel statistics: PME forward + Hessian-vector product ({call}),",
        f"# {n}-ion molten-salt box, mesh {mesh[0]}^3, p = {p}, one MI355X",
        "# commands (from the repository root):",
        "#   rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- \\",
        f"#       python -u bench.py --steps 20 --warmup 5 --cpu-baseline 0 --batched 0 "
        f"--learned 0 --workload {args.workload}{seq}",
        f"#   python -u bench.py --workload {args.workload}{seq}{extra} > <log>   (no profiler)",
        f"#   python bench.py --kernel-stats <dir>/run_kernel_stats.csv --bench-line <log> "
        f"--workload {args.workload}{seq}",
        "# (5 warm-up, 10 per kernel kind breakdown and 20 eager timed steps, then twice",
        "#  20 steps replayed from one HIP graph; copyBuffer and fillBuffer are input uploads;",
        "#  the default legs add their kernel variants: cell gradient k_fftx_fused<1>,",
        "#  k_gather<p, true>, k_cell_grad; optimal influence k_fftx_fused<2>; quadrupole",
        "#  k_bin<p, false, true>, k_spread<p, 3>, k_gather_quad<p>)",
        f"# source digest of the PME sources in paper_2606_01598_amd/csrc (bench.source_digest): {source_digest()}",
    ]
    if bench_val:
        lines.append(f"# bench_us: bench.py's launch timer without the profiler (kernels_us); "
                     f"that run: {bench_val[0]:.1f} {bench_val[1]}, roofline kernel "
                     f"{bench_val[2]} at {bench_val[3]:.2f} us per launch")
    if not args.sequential:
        lines += [
            "# Under the profiler every launch is issued some 10-15 us later than without it,",
            "# so the cotangent chain (second stream) and the forward chain run mostly one",
            "# after the other and each kernel has the GPU to itself.  Without the profiler",
            "# the two chains overlap and the kernels that share CUs take longer (bench_us);",
            "# the sequential-call summary has no overlap to lose and agrees with its timer.",
        ]
    lines += ["", f"{'kernel':40s} {'calls':>7s} {'avg_us':>8s} {'min_us':>8s} {'max_us':>8s} "
              f"{'pct':>6s} {'bench_us':>9s}"]
    for name, calls, avg, mn, mx, pct in rows:
        b = bench_us.get(name)
        bs = f"{b:9.2f}" if b is not None else f"{'':9s}"
        lines.append(f"{name[:40]:40s} {calls:7d} {avg:8.2f} {mn:8.2f} {mx:8.2f} {pct:6.2f} {bs}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(open(out).read())
    return 0


def sweep_summary(logs) -> int:
    """profiles/pme_sweep_molten_sizes.txt from bench JSON lines at several sizes."""
    res = []
    for path in logs:
        with open(path) as fh:
            for ln in fh:
                if ln.startswith("{") and '"kernels_us"' in ln:
                    res.append(json.loads(ln))
                    break
    res.sort(key=lambda d: d["config"]["atoms"])
    kinds = [k for k in KERNEL_SYMBOL if any(k in d["kernels_us"] for d in res)]
    lines = [
        "# PME forward + Hessian-vector product across sizes (molten-salt boxes at the",
        "# density of molten NaCl, mesh ~1 A, p = 6, alpha = 0.30), one MI355X, pme_step",
        "# with the cotangent chain on a second stream, the timed steps replayed from one",
        "# HIP graph (the bench default; ms/step and Matom-steps/s are of that replay)",
        "# commands (repository root):",
        "#   python -u bench.py --workload 8k   --batched 0 --learned 0 --cpu-baseline 0 "
        "--steps 100 --warmup 10",
        "#   python -u bench.py --workload 32k  (the default bench run)",
        "#   python -u bench.py --workload 128k --batched 0 --learned 0 --cpu-baseline 0 "
        "--steps 100 --warmup 10",
        "#   python -u bench.py --workload 1m   --batched 0 --learned 0 --cpu-baseline 0 "
        "--steps 10 --warmup 3 --breakdown-steps 2",
        "#   python bench.py --sweep-summary <log 8k> <log 32k> <log 128k> <log 1m>",
        f"# model bytes per step: {step_bytes(1, 0)} B per atom + {step_bytes(0, 1)} B per "
        f"mesh point; HBM peak {HBM_PEAK_GBS:.0f} GB/s",
        f"# source digest of the PME sources in paper_2606_01598_amd/csrc (bench.source_digest): {source_digest()}",
        "",
        f"{'atoms':>8s} {'mesh':>5s} {'ms/step':>9s} {'Matom-steps/s':>14s} {'model GB/s':>11s} "
        f"{'% HBM':>6s}  dominant kernel (us/launch, % HBM of its algorithmic bytes)",
    ]
    for d in res:
        c, r = d["config"], d["roofline"]
        n, mesh = c["atoms"], c["mesh"]
        m = mesh[0] * mesh[1] * mesh[2]
        gbs = step_bytes(n, m) / (d["ms_per_step"] * 1e-3) / 1e9
        sym = kernel_symbol(r["kind"], True, "fft_r2c" not in d["kernels_us"],
                            d.get("spread", "").startswith("bands"), is_slab(mesh))
        lines.append(f"{n:8d} {mesh[0]:5d} {d['ms_per_step']:9.4f} {d['value']:14.2f} "
                     f"{gbs:11.1f} {100 * gbs / HBM_PEAK_GBS:6.2f}  {sym} "
                     f"{r['avg_launch_us']:.1f} us, {100 * r['frac']:.2f}%")
    lines += ["", "per-kernel average launch durations (us, the bench's breakdown pass):",
              f"{'atoms':>8s} " + " ".join(f"{k:>14s}" for k in kinds)]
    for d in res:
        lines.append(f"{d['config']['atoms']:8d} " +
                     " ".join(f"{d['kernels_us'].get(k, float('nan')):14.2f}" for k in kinds))
    out = os.path.join(ROOT, "profiles", "pme_sweep_molten_sizes.txt")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(open(out).read())
    return 0


def crossover(sizes=(128, 512, 1024, 2048, 4096), alpha=0.30):
    """Explicit Ewald against PME for replicated-density molten-salt boxes: the
    FP64 Ewald oracle at a matched accuracy (erfc(alpha r_c) = 1e-6, k_c =
    2 alpha sqrt(ln 1e6)), the FP64 PME oracle and the GPU PME (forward only, mesh
    ~1 A, p = 6), energy and gradients.  One JSON line per size."""
    import numpy as np
    import torch

    import synth
    from oracle import ewald as oew
    from oracle import pme as opme
    from paper_2606_01598_amd.pme import Plan

    dev = torch.device("cuda", 0)
    for n in sizes:
        f = synth.molten_box(n, 40 + n)
        L = f.box[0, 0]
        m = synth.nearest_smooth(L)
        mesh = (m, m, m)
        t0 = time.perf_counter()
        ew = oew.ewald(f.pos, f.q, f.mu, f.box, alpha, eps=1e-6)
        t_ew = time.perf_counter() - t0
        t0 = time.perf_counter()
        pm = opme.forward(f.pos, f.q, f.mu, f.box, mesh, 6, alpha)
        t_pm = time.perf_counter() - t0
        t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
        plan = Plan(mesh, 6, alpha, max_atoms=n)
        pos, q, mu = t(f.pos), t(f.q), t(f.mu)
        box = torch.tensor(f.box, dtype=torch.float64, device=dev)
        for _ in range(5):
            plan.forward(pos, q, mu, box)
        gpu_ms = _median_ms(lambda: plan.forward(pos, q, mu, box), 20)
        err = abs(pm.energy - ew.long_range) / abs(ew.long_range)
        print(json.dumps({"atoms": n, "L": round(L, 3), "mesh": m, "ewald_cpu_s": round(t_ew, 4),
                          "pme_cpu_s": round(t_pm, 4), "pme_gpu_ms": round(gpu_ms, 4),
                          "ewald_over_pme_cpu": round(t_ew / t_pm, 3),
                          "pme_vs_ewald_rel_energy_diff": err}), flush=True)
    return 0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(frame, mesh, p, alpha, v, steps, runs=3):
    """The FP64 oracle (forward + HVP) timed on the host cores: the median of `runs`
    runs of `steps` full steps each."""
    from oracle import pme as opme
    threads = 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([1] + [int(i.get("num_threads", 1)) for i in threadpool_info()])
    except Exception:
        threads = int(os.environ.get("OMP_NUM_THREADS", "1"))
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        for _ in range(steps):
            opme.forward(frame.pos, frame.q, frame.mu, frame.box, mesh, p, alpha)
            opme.hvp(frame.pos, frame.q, frame.mu, frame.box, mesh, p, alpha, *v)
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[len(times) // 2]
    return {"value": frame.n * steps / dt / 1e6, "unit": "Matom-steps/s", "cores": threads,
            "kind": "oracle", "cpu": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"median of {runs} runs of {steps} full forward+HVP steps of the same "
                      f"{frame.n}-ion workload ({dt:.2f} s per run; the DFT matrix products "
                      f"use {threads} BLAS threads, the spread and gather loops one)"}


def device_ms(fn, reps):
    """Per-call durations (ms) of fn() on the current stream, from HIP events
    recorded around each call."""
    import torch
    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
    return out


def pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(round(q * (len(xs) - 1))))]


def copy_bandwidth(dev):
    """Device-to-device copy of 256 MiB (bytes read + written per second): the
    achievable HBM bandwidth beside the 8 TB/s datasheet peak."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ms = sorted(device_ms(lambda: dst.copy_(src), 10))[5]
    del src, dst
    return {"bytes": 2 * COPY_BYTES, "ms": round(ms, 4), "GBps": round(2 * COPY_BYTES / ms / 1e6, 1)}


def halo_probe() -> int:
    """Cost of combining the overlapping (T + p - 1)^3 regions of a scatter-once
    spread in global memory (pme_halo_probe), p = 6: 64-bit atomic adds into the
    mesh, or contiguous region blocks written and then folded per mesh point.  Both
    combinations are exact; the line says whether the fold equals the atomic sum."""
    import ctypes

    import torch

    from paper_2606_01598_amd import _lib
    lib = _lib.load()
    dev = torch.device("cuda", 0)
    p = 6
    cases = (("32k", 100, (10, 10, 20)), ("32k", 100, (10, 10, 10)),
             ("1m", 320, (8, 8, 16)), ("1m", 320, (16, 16, 16)))
    stream = lambda: ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for workload, n, tile in cases:
        N = (ctypes.c_int32 * 3)(n, n, n)
        T = (ctypes.c_int32 * 3)(*tile)
        tiles = (n // tile[0]) * (n // tile[1]) * (n // tile[2])
        vol = (tile[0] + p - 1) * (tile[1] + p - 1) * (tile[2] + p - 1)
        regions = torch.empty(tiles * vol, dtype=torch.int64, device=dev)
        mesh64 = torch.zeros(n ** 3, dtype=torch.int64, device=dev)
        mesh32 = torch.empty(n ** 3, dtype=torch.float32, device=dev)

        def launch(kind, mesh):
            _lib.check(lib.pme_halo_probe(stream(), kind, N, T, p, ctypes.c_void_p(regions.data_ptr()),
                                          ctypes.c_void_p(mesh.data_ptr())))

        def timed(kind, mesh, clear):
            out = []
            for _ in range(12):
                if clear:
                    mesh.zero_()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                launch(kind, mesh)
                b.record()
                b.synchronize()
                out.append(a.elapsed_time(b) * 1e3)
            return sorted(out[2:])[5]

        atomic_us = timed(_lib.PME_PROBE_HALO_ATOMIC, mesh64, True)
        write_us = timed(_lib.PME_PROBE_HALO_WRITE, mesh64, False)
        fold_us = timed(_lib.PME_PROBE_HALO_FOLD, mesh32, False)
        mesh64.zero_()
        launch(_lib.PME_PROBE_HALO_ATOMIC, mesh64)
        launch(_lib.PME_PROBE_HALO_WRITE, mesh64)
        launch(_lib.PME_PROBE_HALO_FOLD, mesh32)
        torch.cuda.synchronize()
        exact = (int(mesh64.sum()) == tiles * vol) and bool(torch.equal(mesh32, mesh64.float()))
        print(json.dumps({"halo_probe": {
            "workload": workload, "mesh": [n, n, n], "tile": list(tile), "p": p, "tiles": tiles,
            "region_points": tiles * vol, "region_over_mesh": round(tiles * vol / n ** 3, 3),
            "atomic_us": round(atomic_us, 1),
            "atomic_G_per_s": round(tiles * vol / atomic_us / 1e3, 1),
            "write_us": round(write_us, 1), "fold_us": round(fold_us, 1),
            "write_plus_fold_us": round(write_us + fold_us, 1), "exact": exact}}), flush=True)
        del regions, mesh64, mesh32
        torch.cuda.empty_cache()
    return 0


def halo_summary(trace_csv: str, log: str) -> int:
    """Per-configuration median kernel durations of the halo probe from a rocprofv3
    kernel trace (a configuration is told apart by its grid), beside the event
    timings of an unprofiled run."""
    import csv
    cases = []
    with open(log) as fh:
        for ln in fh:
            if ln.startswith("{") and "halo_probe" in ln:
                cases.append(json.loads(ln)["halo_probe"])
    # the probe launches, per configuration in order, 12 timed atomic, write and fold
    # launches each and then one of each for the exactness check: 39 launches
    seq = []
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"]
            if "k_halo_" not in name:
                continue
            kind = "atomic" if "<true>" in name else ("write" if "<false>" in name else "fold")
            seq.append((int(r["Start_Timestamp"]), kind,
                        (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
    seq.sort()
    print("# rocprofv3 median kernel durations (us) of pme_halo_probe, p = 6; event timings of an")
    print("# unprofiled run in brackets (one launch between two events, launch overhead included)")
    print(f"{'mesh':>6} {'tile':>10} {'tiles':>6} {'region/mesh':>11} {'atomic':>16} {'G atomics/s':>11} "
          f"{'write':>14} {'fold':>14} {'write+fold':>10} exact")
    for ci, c in enumerate(cases):
        n = c["mesh"][0]
        block = seq[39 * ci: 39 * (ci + 1)]
        med = {}
        for kind in ("atomic", "write", "fold"):
            v = sorted(d for _, k, d in block if k == kind)
            med[kind] = v[len(v) // 2] if v else float("nan")
        tile = "x".join(str(t) for t in c["tile"])
        print(f"{n:>5}^3 {tile:>10} {c['tiles']:>6} {c['region_over_mesh']:>11.3f} "
              f"{med['atomic']:>7.1f} [{c['atomic_us']:>6.1f}] {c['region_points'] / med['atomic'] / 1e3:>11.1f} "
              f"{med['write']:>6.1f} [{c['write_us']:>5.1f}] {med['fold']:>6.1f} [{c['fold_us']:>5.1f}] "
              f"{med['write'] + med['fold']:>10.1f} {c['exact']}")
    return 0


def lds_peak(dev):
    """LDS bandwidth of the GPU from the library's probe (pme_lds_probe): conflict-
    free 16-byte reads and 64-bit atomic adds, 8 workgroups per CU."""
    import ctypes

    import torch

    from paper_2606_01598_amd import _lib
    lib = _lib.load()
    nblocks, iters = 256 * 8, 4096
    out = torch.empty(nblocks, dtype=torch.float32, device=dev)
    res = {}
    for kind, name, width in ((_lib.PME_PROBE_LDS_READ, "read_b128", 16),
                              (_lib.PME_PROBE_LDS_ATOMIC, "atomic_add_u64", 8)):
        def run():
            _lib.check(lib.pme_lds_probe(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                         kind, iters, nblocks, ctypes.c_void_p(out.data_ptr())))
        run()
        ms = sorted(device_ms(run, 5))[2]
        res[name + "_GBps"] = round(nblocks * 256 * iters * width / ms / 1e6, 1)
    return res


def read_kernel_stats(workload: str, symbol: str):
    """rocprofv3 average duration (us) of `symbol` from the committed kernel-statistics
    summary of the workload, when it was taken on the current sources; else None."""
    path = os.path.join(ROOT, "profiles", f"pme_step_{workload}_kernel_stats.txt")
    if not os.path.exists(path):
        return None
    digest, avg = None, None
    with open(path) as fh:
        for ln in fh:
            if "source digest" in ln:
                digest = ln.rsplit(":", 1)[1].strip()
            elif ln.startswith(symbol[:40]) and not ln.startswith("#"):
                avg = float(ln[40:].split()[1])
    return avg if digest == source_digest() else None


def read_lds_bytes(workload: str, symbol: str):
    """LDS bytes per launch of `symbol` from the committed counter summaries of the
    workload (two-call step, then concurrent step), when taken on the current sources;
    else None."""
    for name in (f"kernels_{workload}_counters.txt", f"kernels_{workload}_step_counters.txt"):
        path = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(path):
            continue
        digest, val = None, None
        with open(path) as fh:
            for ln in fh:
                if "source digest" in ln:
                    digest = ln.rsplit(":", 1)[1].strip()
                elif ln.startswith("lds_bytes_per_launch " + symbol + " "):
                    val = float(ln.rsplit(None, 1)[1])
        if val is not None and digest == source_digest():
            return val
    return None


if __name__ == "__main__":
    sys.exit(main())
