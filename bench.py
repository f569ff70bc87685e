"""Benchmark: SU(2) checkerboard heat bath on one MI355X.

Workload (headline): 48^4 periodic lattice, beta = 6.0, hot start (Philox seed 3).
One step = one full sweep (8 checkerboard passes, Sec. 4 schedule) with the
mean plaquette fused into the sweep, the Polyakov loop measured after it, and
reunitarisation after every 10th sweep.  Throughput = link updates per second
(4 V per sweep) with the links resident in HBM.

The roofline object reports the dominant kernel (the heat-bath pass):
128 algorithmic bytes per link update (the pass reads U_nu, nu != mu, at both
parities plus the opposite-parity U_mu, 56 V bytes, and writes 8 V bytes, for
V/2 updates), divided by its average launch duration measured here with HIP
events on the lattice's stream.

cpu_baseline: the FP64 CPU oracle as it stands, timed on the host cores on a
bounded sample (one sweep of the same 48^4 lattice).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SU(2) link updates/sec + % HBM roofline, plain vs learned-proposal, 1 MI355X"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 128
DIMS = [48, 48, 48, 48]
BETA = 6.0
SEED = 3


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("su2_device.h", "su2_kernels.hip"):
        with open(os.path.join(ROOT, "paper_1010_1486_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per pass launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "pass_kernel_48x48x48x48_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_source_hash():
        return None
    return float(t.group(1))


def cpu_baseline(sample_sweeps=1):
    from oracle import su2_oracle as orc
    threads = orc.max_threads()
    U = orc.init(DIMS, 1, SEED)
    t0 = time.perf_counter()
    orc.sweeps(DIMS, U, sample_sweeps, 0, BETA, SEED, nthreads=threads, measure=True)
    dt = time.perf_counter() - t0
    V = int(np.prod(DIMS))
    return {"value": 4 * V * sample_sweeps / dt, "unit": "link updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sample_sweeps} FP64 sweep(s) + plaquette + Polyakov of the 48^4 "
                      f"beta=6.0 hot-start lattice, {threads} OpenMP threads, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--pass-launches", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--counters", action="store_true",
                    help="short program for rocprofv3 --pmc runs: 16 pass launches in sweep "
                         "order, then 4 plain device copies of the field size (339.7 MB) "
                         "that calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "t-slab decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1010_1486_amd as su2

    dev = torch.device("cuda:0")
    V = int(np.prod(DIMS))
    lat = su2.Lattice(DIMS, BETA, SEED, su2.SU2_HOT, device=dev)
    stream = lat.stream
    meas = su2.SU2_MEAS_PLAQ | su2.SU2_MEAS_POLY
    hist = torch.zeros((max(args.steps, args.warmup, 1), 3), dtype=torch.float64, device=dev)

    if args.counters:
        lat.heatbath_sweep(2)
        for i in range(16):
            lat.test_pass((i // 2) % 4, i % 2)
        x = torch.ones(su2.su2_links_bytes(DIMS) // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(4):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"counters_run": True, "pass_launches": 16, "copy_bytes": 4 * x.numel()}))
        lat.close()
        return

    print(f"[bench] warmup {args.warmup} sweeps on {DIMS}", file=sys.stderr, flush=True)
    lat.sweep_measure(args.warmup, reunit_every=10, meas=meas, hist=hist)
    torch.cuda.synchronize()

    print(f"[bench] timing {args.steps} sweeps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.sweep_measure(args.steps, reunit_every=10, meas=meas, hist=hist)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h = hist[:args.steps].cpu().numpy()

    # average launch duration of the pass kernel, HIP events on the lattice's stream
    print(f"[bench] timing {args.pass_launches} pass launches", file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(args.pass_launches):
            lat.test_pass((i // 2) % 4, i % 2)  # sweep order: mu outer, parity inner
        e1.record(stream)
    e1.synchronize()
    pass_ms = e0.elapsed_time(e1) / args.pass_launches
    achieved = BYTES_PER_UPDATE * (V // 2) / (pass_ms * 1e-3) / 1e9
    traffic = traffic_from_profile()

    value = 4 * V * args.steps / dt
    out = {
        "metric": METRIC, "value": value, "unit": "link updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "48^4 periodic, beta=6.0, hot start (Philox seed 3); step = 1 "
                               "heat-bath sweep (8 passes) + fused plaquette + Polyakov loop, "
                               "reunitarise every 10 sweeps",
                   "dims": DIMS, "beta": BETA, "links": 4 * V, "mode": "plain KP"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x copy "
                                     "calibration + WRITE_SIZE)",
                     "traffic_gbs": None if traffic is None else traffic / (pass_ms * 1e-3) / 1e9,
                     "kernel": "pass_kernel", "avg_launch_us": pass_ms * 1e3,
                     "bytes_per_update": BYTES_PER_UPDATE, "updates_per_launch": V // 2},
        "plaquette_mean_last_half": float(h[args.steps // 2:, 0].mean()),
    }
    lat.close()
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
