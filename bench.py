"""Benchmark: spin-update attempts/s of the REWL hot path on one MI355X.

Headline workload: bcc L=32 (65,536 spins per configuration, held in HBM),
eight coupling shells (z = 112), 128 windows x 8 walkers, the learned
proposal (a network trained on the device, by the library's own kernels, on
about 1e7 (local field, spin) records harvested from the plain walk of the
same workload), FP32 energy changes with FP64 energy / ln g / bins, run by
the persistent batched kernel.

One step = one round of the whole hot path for every walker, in one
persistent launch: 1e4 trial moves per walker (Philox draws, MLP inference
on MFMA, vMF mixture draw, local field, dE, bin, q-ratio acceptance, ln g / H
update), the resync when due, the flatness test with the ln f update, and
the replica-exchange step.  Inputs are resident in HBM before the timed
region; set-up (drive into the windows, harvest, training, autotuning) is
outside it.

Beside the headline (under `extra`): the bcc L=8 four-shell workload (128
walkers, LDS-resident spins, uniform proposal), the 64 uneven instances in
the persistent kernel, the L=16 eight-shell workload with both proposals,
and the shape of the paper's largest run.

Prints ONE JSON line (see the keys at the end of main()).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LDS_PEAK_GBS = 256 * 128 * 2.4          # 256 CUs x 128 B/clk x 2.4 GHz = 78643 GB/s
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
MLP_FLOP_PER_ATTEMPT = 2 * (4 * 64 + 64 * 64 + 64 * 12)    # one 4-64-64-12 evaluation = 10,240

# HBM bytes per launch of a benchmark kernel, from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a plain copy of
# known size; keyed by (kernel sources digest, workload, residency): a changed
# kernel reports null until measured again.
MEASURED_TRAFFIC = {
    # profiles/sweep_fast_c2_fp32_counters.md: FETCH 1355.0 KiB x 2.00 + WRITE 2754.5 KiB x 1.00
    ("60a24928d224d1fc", "c2", "lds"): 5595648,
    # profiles/persistent_c5_fp32_learned_counters.md: FETCH 24,162,000 KiB x 2.00 + WRITE 650,540 KiB x 1.00
    ("d6d81c611cdab2a8", "c5", "hbm"): 50149928960,
}
# Instruction mix of the same launches (SQ counters, one rocprofv3 --pmc pass,
# per trial move): the second axis next to the bandwidth fraction, since a
# lone wavefront per walker is bound by its serial issue chain.
MEASURED_ISSUE = {
    # profiles/sweep_fast_c2_fp32_counters.md
    ("60a24928d224d1fc", "c2", "lds"): {"valu_insts_per_attempt": 69.5,
                                        "salu_insts_per_attempt": 25.7,
                                        "lds_insts_per_attempt": 5.1,
                                        "wave_clk_per_attempt": 845},
    # profiles/persistent_c5_fp32_learned_counters.md
    ("d6d81c611cdab2a8", "c5", "hbm"): {"valu_insts_per_attempt": 202.7,
                                        "salu_insts_per_attempt": 35.3,
                                        "vmem_insts_per_attempt": 3.57,
                                        "lds_insts_per_attempt": 2.6,
                                        "wave_clk_per_attempt": 2534,
                                        "wait_fraction": 0.46,
                                        "l2_misses_per_attempt": 38.7},
}
KERNEL_SOURCES = ["rewl_kernels.hip", "rewl_device.h", "rewl_internal.h", "rewl_mlp_device.h"]
SHELL_COUNTS = [8, 6, 12, 24, 8, 6, 24, 24]


def kernel_digest():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1411_4212_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _shape_key(t):
    """Name of an autotuner trial: walkers per block, residency, grid cap."""
    k = "%dx%s" % (t["walkers_per_block"], "lds" if t["residency"] == 1 else "hbm")
    return k + ("/grid%d" % t["max_blocks"] if t.get("max_blocks") else "")


def bytes_per_attempt(z, mode="fp32_de"):
    """Algorithmic bytes of one trial move: z neighbour spins and the site's
    own spin (3 components each), ln g read at the proposed bin, and the
    ln g + H update of the current bin (read + write): 644 B for z = 50 and
    1388 B for z = 112 in FP32."""
    s = 12 if mode == "fp32_de" else 24
    return z * s + s + 8 + (8 + 4) * 2


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, seconds, theta=None, walkers_per_window=None):
    """The oracle as it stands, on the host cores, on a bounded sample:
    whole segments of the same workload (lattice, couplings, windows,
    schedule, proposal) until `seconds` have elapsed, optionally with fewer
    walkers per window (the walkers are independent within a segment, so
    the rate per core does not depend on their number)."""
    import oracle
    from oracle.build import build_oracle
    build_oracle()
    threads = min(os.cpu_count() or 1, 64)
    lat = cfg["lattice"]
    win = list(cfg["windows"])
    if walkers_per_window:
        win[5] = walkers_per_window
    o = oracle.Oracle(L=lat[1], J=lat[2])
    o.set_windows(*win)
    o.set_schedule(*cfg["schedule"])
    o.set_threads(threads)
    if theta is not None:
        o.set_proposal(theta)
    from paper_1411_4212_amd.workloads import init_spins
    o.init(cfg["seed"], init_spins(cfg))
    W = o.W
    seg = cfg["schedule"][4]
    t0 = time.perf_counter()
    segs = 0
    while time.perf_counter() - t0 < seconds:
        o.run(1)
        segs += 1
    dt = time.perf_counter() - t0
    return {"value": segs * seg * W / dt, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "%d segments x %d walkers (%d windows x %d) x %d moves of the same workload, "
                      "%s proposal (FP64 oracle, %.1f s)"
                      % (segs, W, win[3], win[5], seg, "learned" if theta is not None else "uniform", dt)}


def _timed(r, fn, torch):
    torch.cuda.synchronize()
    a0, _ = r.total_attempts()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    a1, _ = r.total_attempts()
    return (a1 - a0) / dt, dt


def trained_network(r, torch, segments=1, every_k=1, epochs=2, seed=5):
    """Harvest (x, S_i) records of the plain walk of run `r` for `segments`
    segments (every `every_k`-th move), train the learned proposal on them
    with the library's kernels, switch harvesting off; returns (params,
    number of records, seconds spent)."""
    from paper_1411_4212_amd import learned, rewl
    t0 = time.perf_counter()
    seg = r.seg_len
    r.set_harvest(segments * seg // every_k + 1, every_k)
    r.run(segments)
    recs = r.harvested()
    rewl.rewl_set_harvest(r.ctx, None, 0, 0)
    params = learned.init_params(3, recs.device)
    learned.train(recs, params, epochs=epochs, batch=4096, lr=2e-3, seed=seed)
    torch.cuda.synchronize()
    n = int(recs.shape[0])
    del recs
    r.harvest_buf = None
    torch.cuda.empty_cache()
    return params, n, time.perf_counter() - t0


def c2_measurement(torch, workloads, Run, steps, warmup):
    """The bcc L=8 four-shell workload (128 walkers, LDS-resident spins,
    uniform proposal) with launch-per-segment sweeps, LDS roofline."""
    cfg = workloads.c2()
    lat = cfg["lattice"]
    zsum = sum(SHELL_COUNTS[:len(lat[2])])
    r = Run([dict(lattice=lat, windows=cfg["windows"], schedule=cfg["schedule"])], mode="fp32_de")
    r.init(cfg["seed"])
    r.autotune(segments=2)
    lc = r.launch()
    for _ in range(warmup):
        r.sweep()
        r.exchange()
    stream = r.stream
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    a0, _ = r.total_attempts()
    t0 = time.perf_counter()
    for k in range(steps):
        evs[k][0].record(stream)
        r.sweep()
        evs[k][1].record(stream)
        r.exchange()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    a1, _ = r.total_attempts()
    avg = sum(s.elapsed_time(e) for s, e in evs) / steps / 1e3
    in_lds = bool(lc["spins_in_lds"])
    bpa = bytes_per_attempt(zsum)
    achieved = bpa * r.n_walkers * cfg["schedule"][4] / avg / 1e9
    peak = LDS_PEAK_GBS if in_lds else HBM_PEAK_GBS
    digest = kernel_digest()
    res = "lds" if in_lds else "hbm"
    r.close()
    log("bench: c2 %.3e attempts/s, sweep %.3f ms" % ((a1 - a0) / wall, avg * 1e3))
    return {"workload": "bcc L=8 (1024 spins), 4 shells (z=50), 16 windows x 8 walkers, 2000 bins, "
                        "uniform proposal, launch per segment",
            "walkers": 128, "attempts_per_s": (a1 - a0) / wall, "ms_per_step": wall / steps * 1e3,
            "roofline": {"bound": res, "achieved": achieved, "peak": peak, "unit": "GB/s",
                         "frac": achieved / peak, "bytes_per_attempt": bpa,
                         "traffic": MEASURED_TRAFFIC.get((digest, "c2", res)),
                         "issue": MEASURED_ISSUE.get((digest, "c2", res)),
                         "kernel": "sweep_fast_kernel (fp32_de)", "avg_launch_ms": avg * 1e3,
                         "walkers_per_block": lc["walkers_per_block"]}}


def extra_measurements(torch, workloads, Run):
    """The same kernels on other workloads, each with an autotuned launch
    shape: the 64 uneven instances in the persistent kernel, the L=16
    eight-shell workload (1024 walkers) with the uniform and with the learned
    proposal (trained on its own plain walk), the shape of the paper's
    largest run (L=40, 893 windows x 1 walker, two shells), and the walk over
    the magnetisation M_z on bcc L=8."""
    out = {}
    cfgs = workloads.batched(64)
    r = Run([dict(lattice=c["lattice"], windows=c["windows"], schedule=c["schedule"]) for c in cfgs],
            mode="fp32_de")
    r.init(cfgs[0]["seed"])
    trials = r.autotune(segments=1, persistent=True)
    lc = r.launch()
    rate, dt = _timed(r, lambda: r.run_persistent(3), torch)
    out["batched_64_instances"] = {
        "walkers": r.n_walkers, "attempts_per_s": rate, "seconds": dt, "rounds": 3,
        "kernel": "persistent_kernel (fp32_de)", "walkers_per_block": lc["walkers_per_block"],
        "spins_in_lds": lc["spins_in_lds"],
        "grid_cap": r.grid_cap(),
        "autotune_ms_per_segment": {_shape_key(t): (round(t["ms_per_segment"], 3) if t["status"] == 0 else None)
                                    for t in trials}}
    r.close()
    log("bench: batched %.3e attempts/s" % rate)
    for name, wl, kinds in (("L16_8shell", workloads.c4(), ("uniform", "learned")),
                            ("L40_paper_shape_893x1", workloads.paper_l40(), ("uniform",))):
        for kind in kinds:
            r = Run([dict(lattice=wl["lattice"], windows=wl["windows"], schedule=wl["schedule"])], mode="fp32_de")
            r.seg_len = wl["schedule"][4]
            r.init(wl["seed"], workloads.init_spins(wl))
            info = {}
            if kind == "learned":
                params, nrec, secs = trained_network(r, torch, segments=1, every_k=1)
                r.set_proposal(params)
                info = {"network": "trained on %d records of the plain walk (%.2f s harvest + training)"
                                   % (nrec, secs)}
            r.autotune(segments=1)
            lc = r.launch()
            rate, dt = _timed(r, lambda: r.run(2), torch)
            out["%s_%s" % (name, kind)] = dict(
                walkers=r.n_walkers, attempts_per_s=rate, seconds=dt, segments=2, proposal=kind,
                walkers_per_block=lc["walkers_per_block"], spins_in_lds=lc["spins_in_lds"], **info)
            r.close()
            log("bench: %s %s %.3e attempts/s (%s)" % (name, kind, rate, "LDS" if lc["spins_in_lds"] else "HBM"))
    # the walk over the magnetisation M_z (generic sweep kernel): bcc L=8,
    # M_z in [-64, 64) on 64 bins (about +-3.5 standard deviations of the
    # infinite-temperature distribution), 8 windows x 8 walkers
    wl = dict(lattice=("bcc", 8, list(workloads.J_C2)), windows=(-64.0, 64.0, 64, 8, 0.75, 8),
              schedule=(4, 5, 1.0, 2.0 ** -20, 10000, 102400), coord="Mz")
    r = Run([wl], mode="fp32_de")
    r.init(11)
    lc = r.launch()
    rate, dt = _timed(r, lambda: r.run(4), torch)
    out["Mz_L8_uniform"] = dict(walkers=r.n_walkers, attempts_per_s=rate, seconds=dt, segments=4,
                                coordinate="M_z", kernel="sweep_kernel (fp32_de, generic)",
                                walkers_per_block=lc["walkers_per_block"], spins_in_lds=lc["spins_in_lds"])
    r.close()
    log("bench: Mz_L8 %.3e attempts/s" % rate)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shape instead of the autotuner's choice")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the workloads reported under 'extra'")
    ap.add_argument("--uniform", action="store_true",
                    help="headline workload with the uniform proposal (for comparison runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, copy a 256 MiB buffer 3 times (counter calibration)")
    ap.add_argument("--harvest-every", type=int, default=1,
                    help="record every k-th move of the plain walk for training (profiling runs use a "
                         "larger k: fewer training steps to count)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the REWL hot path here is single-GPU "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1411_4212_amd import workloads
    from paper_1411_4212_amd.rewl import Run

    cfg = workloads.c5()
    lat = cfg["lattice"]
    zsum = sum(SHELL_COUNTS[:len(lat[2])])
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log("bench: building run", cfg["name"])
    r = Run([dict(lattice=lat, windows=cfg["windows"], schedule=cfg["schedule"])], mode="fp32_de")
    r.seg_len = cfg["schedule"][4]
    t0 = time.perf_counter()
    r.init(cfg["seed"], workloads.init_spins(cfg))
    torch.cuda.synchronize()
    log("bench: walkers driven into their windows in %.1f s" % (time.perf_counter() - t0))
    net = None
    theta = None
    if not args.uniform:
        log("bench: harvest and training")
        params, nrec, secs = trained_network(r, torch, segments=1, every_k=args.harvest_every)
        r.set_proposal(params)
        theta = params.double().cpu().numpy()
        net = "trained on the device on %d (field, spin) records of the plain walk of this workload " \
              "(%.2f s harvest + training, not timed)" % (nrec, secs)
        log("bench:", net)
    # warm-up rounds first, so that the autotuner times the walk's steady
    # regime rather than its first rounds from freshly placed walkers
    log("bench: warmup", args.warmup)
    for _ in range(args.warmup):
        r.run_persistent(1)
    trials = []
    if not args.no_autotune:
        trials = r.autotune(segments=2, persistent=True)
    lc = r.launch()
    W = r.n_walkers
    seg = cfg["schedule"][4]
    log("bench: launch", lc, "grid cap", r.grid_cap())
    torch.cuda.synchronize()
    stream = r.stream
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    log("bench: timed steps", args.steps)
    a0, _ = r.total_attempts()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grid = 0
    for k in range(args.steps):
        evs[k][0].record(stream)
        grid = r.run_persistent(1)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("bench: timed steps done")
    a1, _ = r.total_attempts()
    attempts = a1 - a0
    wall = t1 - t0
    launch_ms = [s.elapsed_time(e) for s, e in evs]
    avg_launch_s = sum(launch_ms) / len(launch_ms) / 1e3
    per_launch_attempts = W * seg
    bpa = bytes_per_attempt(zsum)
    achieved = bpa * per_launch_attempts / avg_launch_s / 1e9
    rate = attempts / wall
    log("bench: %.3e attempts/s, persistent round %.3f ms avg" % (rate, avg_launch_s * 1e3))
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy calibration done (3 x 256 MiB)")
    acc = sum(r.walker(0, w)["accepts"] for w in range(W)) / max(1, sum(r.walker(0, w)["attempts"] for w in range(W)))
    grid_cap = r.grid_cap()
    r.close()
    digest = kernel_digest()
    res = "lds" if lc["spins_in_lds"] else "hbm"
    kname = "c5" if not args.uniform else "c5_uniform"
    traffic = MEASURED_TRAFFIC.get((digest, kname, res))
    issue = MEASURED_ISSUE.get((digest, kname, res))

    extra = {}
    if not args.no_extra:
        extra["c2_L8_uniform_lds"] = c2_measurement(torch, workloads, Run, 20, 3)
        extra.update(extra_measurements(torch, workloads, Run))

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(cfg, args.cpu_seconds, theta=theta, walkers_per_window=1)

    out = {
        "metric": "spin-update attempts/s",
        "value": rate,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: bcc L=%d (%d spins, in HBM), %d shells (z=%d), %d windows x %d walkers, "
                               "%d bins, %s proposal, persistent kernel, round of %d moves/walker"
                               % (cfg["name"], lat[1], 2 * lat[1] ** 3, len(lat[2]), zsum,
                                  cfg["windows"][3], cfg["windows"][5], cfg["windows"][2],
                                  "uniform" if args.uniform else "learned", seg),
                   "mode": "fp32_de", "walkers": W, "attempts_timed": attempts,
                   "network": net, "acceptance": acc,
                   "parallelism": "one wavefront per walker, single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch", "kernel_digest": digest,
                     "kernel": "persistent_kernel (fp32_de, %s, spins in %s)"
                               % ("uniform" if args.uniform else "learned", res.upper()),
                     "bytes_per_attempt": bpa, "attempts_per_launch": per_launch_attempts,
                     "walkers_per_block": lc["walkers_per_block"],
                     "avg_launch_ms": avg_launch_s * 1e3, "issue": issue,
                     "mfma_tflops": None if args.uniform else MLP_FLOP_PER_ATTEMPT * per_launch_attempts / avg_launch_s / 1e12,
                     "mfma_frac": None if args.uniform else MLP_FLOP_PER_ATTEMPT * per_launch_attempts / avg_launch_s / 1e12 / BF16_PEAK_TFLOPS,
                     "grid": grid, "grid_cap": grid_cap,
                     "autotune_ms_per_round": {_shape_key(t): (round(t["ms_per_segment"], 3) if t["status"] == 0 else None)
                                               for t in trials}},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
