"""Benchmark: spin-update attempts/s of the REWL hot path on one MI355X.

One step = one segment of the whole hot path for every walker: 1e4 trial
moves per walker (Philox draws, proposal, local field, dE, bin, acceptance,
ln g / H update), the resync when due, the flatness test with the ln f
update, and one replica-exchange step.  Inputs are resident in HBM before
the timed region.  Default workload: bcc L=8, four shells, 16 windows x 8
walkers (1024 spins each), FP32 energy changes with FP64 energy/ln g.

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

# HBM bytes per sweep launch of the benchmark workload, from two rocprofv3
# --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a
# plain copy of known size; keyed by the digest of the kernel sources they
# were taken on (a changed kernel reports null until measured again).
MEASURED_TRAFFIC = {
    # profiles/sweep_fast_c2_fp32_counters.md: FETCH 1355.0 KiB x 2.00 + WRITE 2754.5 KiB x 1.00
    ("60a24928d224d1fc", "fp32_de", "lds"): 5595648,
}
# Instruction mix of the same launches (SQ counters, one rocprofv3 --pmc pass,
# per trial move): the second axis next to the bandwidth fraction, since a
# lone wavefront per walker is bound by its serial issue chain, not by LDS.
MEASURED_ISSUE = {
    # profiles/sweep_fast_c2_fp32_counters.md
    ("60a24928d224d1fc", "fp32_de", "lds"): {"valu_insts_per_attempt": 69.5,
                                             "salu_insts_per_attempt": 25.7,
                                             "lds_insts_per_attempt": 5.1,
                                             "wave_clk_per_attempt": 845},
}
KERNEL_SOURCES = ["rewl_kernels.hip", "rewl_device.h", "rewl_internal.h", "rewl_mlp_device.h"]


def kernel_digest():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1411_4212_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_attempt(z, mode):
    """Algorithmic LDS bytes of one trial move: z neighbour spins and the
    site's own spin (3 components each), ln g read at the proposed bin, and
    the ln g + H update of the current bin (read + write)."""
    s = 12 if mode == "fp32_de" else 24
    return z * s + s + 8 + (8 + 4) * 2


def hbm_bytes_per_attempt(z, mode):
    """Algorithmic HBM bytes of one trial move when the configurations stay in
    HBM: the z neighbour spins and the site's own spin (3 components each);
    ln g and H stay in LDS for the segment."""
    s = 12 if mode == "fp32_de" else 24
    return (z + 1) * s


def cpu_baseline(cfg, seconds):
    """The oracle as it stands, on the host cores, on a bounded sample:
    whole segments of the same workload until `seconds` have elapsed."""
    import oracle
    from oracle.build import build_oracle
    build_oracle()
    threads = min(os.cpu_count() or 1, 64)
    lat = cfg["lattice"]
    o = oracle.Oracle(L=lat[1], J=lat[2])
    o.set_windows(*cfg["windows"])
    o.set_schedule(*cfg["schedule"])
    o.set_threads(threads)
    o.init(cfg["seed"])
    W = o.W
    seg = cfg["schedule"][4]
    t0 = time.perf_counter()
    segs = 0
    while time.perf_counter() - t0 < seconds:
        o.run(1)
        segs += 1
    dt = time.perf_counter() - t0
    return {"value": segs * seg * W / dt, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "sample": "%d segments x %d walkers x %d moves of the same workload (FP64 oracle, "
                      "%.1f s)" % (segs, W, seg, dt)}


def _timed(r, fn, torch):
    torch.cuda.synchronize()
    a0, _ = r.total_attempts()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    a1, _ = r.total_attempts()
    return (a1 - a0) / dt, dt


def extra_measurements(torch, workloads, Run):
    """The same kernels on workloads that fill the chip (reported beside the
    headline figure), each with an autotuned launch shape: the 64 uneven
    instances in the persistent kernel, the L=16 eight-shell workload (1024
    walkers) with the uniform and with the learned proposal, the L=32
    workload (1024 walkers, 65,536 spins each), and the shape of the paper's
    largest run (L=40, 893 windows x 1 walker, two shells)."""
    import numpy as np
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
        "autotune_ms_per_segment": {"%dx%s" % (t["walkers_per_block"], "lds" if t["residency"] == 1 else "hbm"):
                                    (round(t["ms_per_segment"], 3) if t["status"] == 0 else None) for t in trials}}
    r.close()
    log("bench: batched %.3e attempts/s" % rate)
    from paper_1411_4212_amd import learned
    for name, wl, kinds in (("L16_8shell", workloads.c4(), ("uniform", "learned")),
                            ("L32_8shell", workloads.c5(), ("uniform",)),
                            ("L40_paper_shape_893x1", workloads.paper_l40(), ("uniform",))):
        for kind in kinds:
            r = Run([dict(lattice=wl["lattice"], windows=wl["windows"], schedule=wl["schedule"])], mode="fp32_de")
            r.init(wl["seed"], workloads.init_spins(wl))
            if kind == "learned":
                r.set_proposal(learned.init_params(1, torch.device("cuda", 0)))
            r.autotune(segments=1)
            lc = r.launch()
            rate, dt = _timed(r, lambda: r.run(2), torch)
            z = {2: 14, 4: 50, 8: 112}[len(wl["lattice"][2])]
            out["%s_%s" % (name, kind)] = {
                "walkers": r.n_walkers, "attempts_per_s": rate, "seconds": dt, "segments": 2, "proposal": kind,
                "walkers_per_block": lc["walkers_per_block"], "spins_in_lds": lc["spins_in_lds"],
                # algorithmic gather bytes per attempt (z neighbour spins + own spin, 16 B each)
                # when the configurations are read from HBM
                "gather_GBs_if_hbm": None if lc["spins_in_lds"] else rate * (z + 1) * 16 / 1e9}
            r.close()
            log("bench: %s %s %.3e attempts/s (%s)" % (name, kind, rate, "LDS" if lc["spins_in_lds"] else "HBM"))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="fp32_de", choices=["fp32_de", "fp64", "fp64_det"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shape instead of the autotuner's choice")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the chip-filling workloads reported under 'extra'")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed region, copy a 256 MiB buffer 3 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the REWL hot path here is single-GPU "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1411_4212_amd import workloads
    from paper_1411_4212_amd.rewl import Run

    cfg = workloads.c2()
    lat = cfg["lattice"]
    z = [8, 6, 12, 24, 8, 6, 24, 24]
    zsum = sum(z[:len(lat[2])])
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log("bench: building run", cfg["name"], args.mode)
    r = Run([dict(lattice=lat, windows=cfg["windows"], schedule=cfg["schedule"])], mode=args.mode)
    r.init(cfg["seed"])
    if not args.no_autotune:
        # launch shape by the project's autotuner (the walk is restored after
        # every trial, so the timed steps start from the initialised state)
        r.autotune(segments=2)
    lc = r.launch()
    in_lds = bool(lc["spins_in_lds"])
    W = r.n_walkers
    seg = cfg["schedule"][4]
    log("bench: warmup", args.warmup, "launch", lc)
    for _ in range(args.warmup):
        r.sweep()
        r.exchange()
    torch.cuda.synchronize()
    a0, _ = r.total_attempts()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    log("bench: timed steps", args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        r.sweep()
        evs[k][1].record(stream)
        r.exchange()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    a1, _ = r.total_attempts()
    attempts = a1 - a0
    wall = t1 - t0
    sweep_ms = [s.elapsed_time(e) for s, e in evs]
    avg_sweep_s = sum(sweep_ms) / len(sweep_ms) / 1e3
    if in_lds:
        bpa, bound, peak = bytes_per_attempt(zsum, args.mode), "lds", LDS_PEAK_GBS
    else:
        bpa, bound, peak = hbm_bytes_per_attempt(zsum, args.mode), "hbm", HBM_PEAK_GBS
    per_launch_bytes = bpa * W * seg
    achieved = per_launch_bytes / avg_sweep_s / 1e9
    log("bench: %.3e attempts/s, sweep %.3f ms avg" % (attempts / wall, avg_sweep_s * 1e3))
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy calibration done (3 x 256 MiB)")
    digest = kernel_digest()
    traffic = MEASURED_TRAFFIC.get((digest, args.mode, "lds" if in_lds else "hbm"))
    issue = MEASURED_ISSUE.get((digest, args.mode, "lds" if in_lds else "hbm"))

    extra = None
    if not args.no_extra:
        extra = extra_measurements(torch, workloads, Run)

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(cfg, args.cpu_seconds)

    out = {
        "metric": "spin-update attempts/s",
        "value": attempts / wall,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32_de": "f32", "fp64": "f64", "fp64_det": "f64"}[args.mode],
        "data": "synthetic",
        "config": {"workload": "%s: bcc L=%d (%d spins), %d shells (z=%d), %d windows x %d walkers, "
                               "%d bins, segment %d moves/walker"
                               % (cfg["name"], lat[1], 2 * lat[1] ** 3, len(lat[2]), zsum,
                                  cfg["windows"][3], cfg["windows"][5], cfg["windows"][2], seg),
                   "mode": args.mode, "walkers": W, "attempts_timed": attempts,
                   "parallelism": "one wavefront per walker, single GPU"},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": "GB/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch", "kernel_digest": digest,
                     "kernel": "sweep_fast_kernel (%s)" % args.mode,
                     "bytes_per_attempt": bpa, "walkers_per_block": lc["walkers_per_block"],
                     "avg_launch_ms": avg_sweep_s * 1e3, "issue": issue},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
