"""Benchmark: SU(2) checkerboard heat bath on one MI355X.

Workload (headline): 48^4 periodic lattice, beta = 6.0, hot start (Philox seed 3).
One step = one full sweep (8 checkerboard passes, Sec. 4 schedule) with the
mean plaquette of every sweep fused into its passes (the workload measures the
plaquette each sweep) and reunitarisation of every link in every 10th sweep,
fused into that sweep's passes (each link is reunitarised as it is stored; the
time of the same sweeps with a separate reunitarisation pass and plaquette is
reported beside it).  Throughput
= link updates per second (4 V per sweep) with the links resident in HBM.
Other workloads (4^4, beta scans, 32^3 x Nt with the Polyakov loop, the
batched learned-vs-plain comparison) are reported in the same JSON line.

The roofline object reports the dominant kernel (the heat-bath pass):
128 algorithmic bytes per link update (the pass reads U_nu, nu != mu, at both
parities plus the opposite-parity U_mu, 56 V bytes, and writes 8 V bytes, for
V/2 updates), divided by its average launch duration measured here with HIP
events on the lattice's stream.  floor_us is the duration of a streaming
kernel that moves exactly the same bytes without the stencil (each plane read
at the thread's own index), the practical bound for this traffic mix.

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
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 vector
BYTES_PER_UPDATE = 128
DIMS = [48, 48, 48, 48]
OR_WIDTH = 0.02  # noise half-width of the over-relaxed learned proposal
BETA = 6.0
SEED = 3


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("su2_device.h", "su2_kcommon.h", "su2_internal.h", "su2_kernels.hip"):
        with open(os.path.join(ROOT, "paper_1010_1486_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def f64_source_hash():
    h = hashlib.sha256()
    for f in ("su2_device.h", "su2_kcommon.h", "su2_internal.h", "su2_f64.hip"):
        with open(os.path.join(ROOT, "paper_1010_1486_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


F64_PROFILE = os.path.join(ROOT, "profiles", "pass64_kernel_48x48x48x48_counters.md")

SU3_BYTES_PER_UPDATE = 432  # 9 links of 48 B: 8 read (7 neighbours' classes + the link), 1 written
SU3_PROFILE = os.path.join(ROOT, "profiles", "su3_pass_kernel_48x48x48x48.md")


def su3_source_hash():
    h = hashlib.sha256()
    for f in ("su2_device.h", "su2_kcommon.h", "su2_internal.h", "su3_internal.h",
              "su3_kernels.hip"):
        with open(os.path.join(ROOT, "paper_1010_1486_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_value(path, key, source_hash, key_name="kernel_source_hash"):
    """A figure from a committed rocprofv3 summary, if it was taken on the
    current kernel source (else None)."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(key_name + r":\s*([0-9a-f]+)", text)
    t = re.search(key + r":\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != source_hash:
        return None
    return float(t.group(1))


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


def tau_int(x, c=6.0):
    """Integrated autocorrelation time, Madras-Sokal automatic window."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    x = x - x.mean()
    var = x.var()
    if var == 0 or n < 8:
        return 0.5
    f = np.fft.rfft(x, 2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n] / (var * np.arange(n, 0, -1))
    tau = 0.5
    for w in range(1, n):
        tau += acf[w]
        if w >= c * tau:
            break
    return max(tau, 0.5)


def tau_int_err(tau, n, c=6.0):
    """Madras-Sokal error of an integrated autocorrelation time measured with
    window c tau on n samples: tau sqrt(2 (2 W + 1) / n), W = c tau."""
    return tau * np.sqrt(2.0 * (2.0 * c * tau + 1.0) / n)


def jackknife_mean(x):
    """Mean over the replicas and its leave-one-out (jackknife) error."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    loo = (x.sum() - x) / (n - 1)
    return float(x.mean()), float(np.sqrt((n - 1) / n * ((loo - loo.mean()) ** 2).sum()))


def learned_vs_plain(su2, torch, dev, sweeps=2000, therm=300, chunk=50, with_cpu=True):
    """64 replicas, L = 8 + 2 (r mod 7) (8^4 .. 20^4), beta uniform in [1.8, 3.0]
    (seeded), hot start; the learned proposal is trained on the GPU on 1e7
    exact-sampler draws (alpha log-uniform in [0.5, 30]).  Each mode: autotuned
    launch, then graph-captured chunks of batched sweeps with the plaquette
    and the Polyakov loop measured every sweep.  Effective rate = sweeps/s /
    (2 tau_int(P)), averaged over the replicas (and the same with tau_int of
    the absolute Polyakov loop, the long-distance observable).  The untrained network (identity spline, i.e. a uniform
    proposal) runs the same protocol for comparison, and so does the trained
    flow used over-relaxed (proposal -g(x_old) + noise in the flow coordinate,
    noise half-width OR_WIDTH, and without noise), which anticorrelates
    successive plaquettes.  The baselines without learning are the plain heat
    bath and the heat bath followed by 1 or 3 microcanonical over-relaxation
    sweeps (compound sweeps; rates count every link update, tau_int counts
    compound sweeps).  Error bars: tau_int and the effective rates as means
    over the replicas with jackknife errors; the ratio to the plain heat bath
    as the replica-paired mean ratio with its jackknife error; per replica the
    Madras-Sokal error of tau_int as well."""
    n = 64
    L = [8 + 2 * (r % 7) for r in range(n)]
    dims = [[l] * 4 for l in L]
    betas = np.random.default_rng(5).uniform(1.8, 3.0, n)
    links = 4 * sum(l ** 4 for l in L)
    side = torch.cuda.Stream(device=dev)
    out = {"workload": "64 replicas L=8+2(r mod 7), beta~U[1.8,3.0] (seed 5), hot start; "
                       f"{therm} thermalisation + {sweeps} measured sweeps per mode",
           "links_per_sweep": links}
    with torch.cuda.stream(side):
        net = su2.NN(seed=5)
        t0 = time.perf_counter()
        net.sample_data(10_000_000, 0.5, 30.0, seed=5)
        hist = net.train(20000, 16384, 3e-3, lr_end=1e-5)
        net.build_table()
        torch.cuda.synchronize()
        out["training"] = {"samples": 10_000_000, "steps": 20000, "batch": 16384,
                           "lr": "cosine 3e-3 -> 1e-5",
                           "seconds": time.perf_counter() - t0,
                           "nll_first_100": float(hist[:100].mean()),
                           "nll_last_100": float(hist[-100:].mean())}
        untrained = su2.NN(seed=5)  # identity spline: the uniform proposal
        untrained.build_table()
        eff_r, eff_l = {}, {}
        for name, mode, proposal, width, n_or in (
                ("plain", su2.SU2_KP, net, -1.0, 0),
                ("plain_overrelaxed", su2.SU2_KP_OR, net, -1.0, 1),
                ("plain_overrelaxed3", su2.SU2_KP_OR, net, -1.0, 3),
                ("learned", su2.SU2_LEARNED, net, -1.0, 0),
                ("learned_untrained", su2.SU2_LEARNED, untrained, -1.0, 0),
                ("learned_overrelaxed", su2.SU2_LEARNED, net, OR_WIDTH, 0),
                ("learned_reflection", su2.SU2_LEARNED, net, 0.0, 0)):
            b = su2.Batch(dims, betas, [1] * n, seed=5, device=dev)
            b.set_proposal(proposal)
            b.set_overrelax(width)
            b.set_hb_overrelax(n_or)
            tuned_us = b.autotune(None, mode)
            launch = b.launch()
            b.sweep(therm, mode)
            b.accept_stats(reset=True)
            h = torch.zeros((sweeps, n, 3), dtype=torch.float64, device=dev)
            b.capture(chunk, mode, meas=su2.SU2_MEAS_PLAQ | su2.SU2_MEAS_POLY, hist=h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.replay(sweeps // chunk)
            b.synchronize()
            dt = time.perf_counter() - t0
            prop, acc = b.accept_stats()
            hh = h.cpu().numpy()
            P, AL = hh[:, :, 0], hh[:, :, 2]
            taus = np.array([tau_int(P[:, r]) for r in range(n)])
            taus_l = np.array([tau_int(AL[:, r]) for r in range(n)])
            sps = sweeps / dt  # (compound) sweeps per second
            # bytes per update: the heat bath 128; the learned and over-relaxation
            # updates also read the old link (144)
            bpu = ((128 + 144 * n_or) / (1 + n_or) if mode == su2.SU2_KP_OR else
                   (128 if mode == su2.SU2_KP else 144))
            ups = links * (1 + n_or) * sps
            gbs = bpu * ups / 1e9
            eff_r[name] = sps / (2 * taus)
            eff_l[name] = sps / (2 * taus_l)
            tau_m, tau_e = jackknife_mean(taus)
            eff_m, eff_e = jackknife_mean(eff_r[name])
            taul_m, taul_e = jackknife_mean(taus_l)
            out[name] = {"link_updates_per_s": ups, "sweeps_per_s": sps,
                         "algorithmic_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                         "bytes_per_update": bpu,
                         "overrelax_width": None if width < 0 else width,
                         "or_sweeps_per_heatbath": n_or if mode == su2.SU2_KP_OR else None,
                         "launch": launch, "tuned_us_per_sweep": tuned_us,
                         "tau_int_plaquette_mean": tau_m, "tau_int_plaquette_err": tau_e,
                         "tau_int_madras_sokal_err_per_replica_mean":
                             float(np.mean(tau_int_err(taus, sweeps))),
                         "effective_sweeps_per_s": eff_m, "effective_sweeps_per_s_err": eff_e,
                         "tau_int_abs_polyakov_mean": taul_m,
                         "tau_int_abs_polyakov_err": taul_e,
                         "acceptance": (float(acc.sum() / prop.sum()) if prop.sum() else None),
                         "mean_plaquette": float(P.mean())}
            if name != "plain":
                r_m, r_e = jackknife_mean(eff_r[name] / eff_r["plain"])
                out[name]["effective_over_plain"] = r_m
                out[name]["effective_over_plain_err"] = r_e
                r_m, r_e = jackknife_mean(eff_l[name] / eff_l["plain"])
                out[name]["effective_over_plain_abs_polyakov"] = r_m
                out[name]["effective_over_plain_abs_polyakov_err"] = r_e
            b.close()
        net.close()
        untrained.close()
    torch.cuda.synchronize()
    out["learned_over_plain_updates"] = (out["learned"]["link_updates_per_s"] /
                                         out["plain"]["link_updates_per_s"])
    out["learned_over_plain_effective"] = (out["learned"]["effective_sweeps_per_s"] /
                                           out["plain"]["effective_sweeps_per_s"])
    if with_cpu:
        out["oracle"] = {"plain_link_updates_per_s": oracle_rate([20] * 4, 1, 2.3),
                         "plain_threads": oracle_threads(),
                         "learned_link_updates_per_s": oracle_learned_rate([12] * 4, 2.3),
                         "learned_threads": 1,
                         "sample": "one sweep of a 20^4 replica (heat bath, all threads); one "
                                   "sweep of learned passes on a 12^4 lattice (one thread)"}
    out["overrelaxed_over_plain_effective"] = (
        out["learned_overrelaxed"]["effective_sweeps_per_s"] /
        out["plain"]["effective_sweeps_per_s"])
    # the fair comparison of the over-relaxed learned form: against the heat
    # bath with the standard over-relaxation (replica-paired ratio)
    for base in ("plain_overrelaxed", "plain_overrelaxed3"):
        r_m, r_e = jackknife_mean(eff_r["learned_overrelaxed"] / eff_r[base])
        out[f"learned_overrelaxed_over_{base}_effective"] = r_m
        out[f"learned_overrelaxed_over_{base}_effective_err"] = r_e
    return out


def run_batch(su2, torch, dev, dims, betas, starts, seed, therm, sweeps, meas, reunit,
              chunk=50):
    """Autotuned batch: `therm` sweeps, then `sweeps` measured sweeps replayed as
    graph-captured chunks; returns (seconds of the measured part, history, the
    autotuned launch).  When the autotuner picks per-pass launches, the
    reunitarisation is fused into the passes (launch["reunit_fused"])."""
    b = su2.Batch(dims, betas, starts, seed=seed, device=dev)
    b.autotune(None, su2.SU2_KP)
    launch = b.launch()
    launch["reunit_fused"] = bool(reunit > 0 and not launch["flags"] & 8)
    b.set_reunit_fused(launch["reunit_fused"])
    b.sweep_measure(therm, reunit_every=reunit, meas=meas)
    h = torch.zeros((sweeps, len(dims), 3), dtype=torch.float64, device=dev)
    b.capture(chunk, su2.SU2_KP, reunit_every=reunit, meas=meas, hist=h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.replay(sweeps // chunk)
    b.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    return dt, h.cpu().numpy(), launch


def step_bytes(volumes, polyakov, reunit):
    """Algorithmic HBM bytes of one sweep over lattices of these volumes:
    8 passes x 64 V, plus 16 V for the Polyakov loop, plus 128 V per separate
    reunitarisation (amortised; reunit 0 when there is none or it is fused
    into the passes); the plaquette is fused into the passes."""
    V = float(sum(volumes))
    return V * (512.0 + (16.0 if polyakov else 0.0) + (128.0 / reunit if reunit else 0.0))


def oracle_threads():
    from oracle import su2_oracle as orc
    return orc.max_threads()


def oracle_learned_rate(dims, beta, seed=5):
    """The oracle's learned (independence) Metropolis passes on one lattice:
    link updates/s on one thread (its learned pass is serial)."""
    from oracle import su2_oracle as orc
    from oracle import nn_oracle
    p = np.zeros(nn_oracle.NPARAM, dtype=np.float32)
    p[2624:] = nn_oracle.identity_raw_bias()
    table = orc.nn_table(p)
    U = orc.init(dims, 1, seed)
    t0 = time.perf_counter()
    for mu in range(4):
        for par in range(2):
            orc.learned_pass(dims, U, table, mu, par, 0, beta, seed)
    return 4 * int(np.prod(dims)) / (time.perf_counter() - t0)


def oracle_rate(dims, sweeps, beta):
    from oracle import su2_oracle as orc
    U = orc.init(dims, 1, 1)
    t0 = time.perf_counter()
    orc.sweeps(dims, U, sweeps, 0, beta, 1, reunit_every=10, nthreads=orc.max_threads(),
               measure=True)
    return 4 * int(np.prod(dims)) * sweeps / (time.perf_counter() - t0)


def other_configs(su2, torch, dev, with_cpu):
    """The remaining workloads, each at its full protocol: link updates/s,
    algorithmic GB/s and fraction of the 8 TB/s HBM peak, ensemble means, and
    the oracle's rate on a few sweeps of the same lattice (host threads)."""
    out = {}
    PL = su2.SU2_MEAS_PLAQ
    # 4^4, beta 2.3, hot start (seed 1), 100 sweeps, plaquette every sweep
    dims = [4, 4, 4, 4]
    with su2.Lattice(dims, 2.3, 1, su2.SU2_HOT, device=dev) as lat:
        lat.sweep_measure(10, meas=PL)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = lat.sweep_measure(100, meas=PL)
        torch.cuda.synchronize()
        dt_direct = time.perf_counter() - t0
        with su2.Lattice(dims, 2.3, 1, su2.SU2_HOT, device=dev) as lg:
            hg = torch.zeros((200, 3), dtype=torch.float64, device=dev)
            lg.capture(100, meas=PL, hist=hg)
            lg.replay(1)
            lg.synchronize()
            t0 = time.perf_counter()
            lg.replay(1)
            lg.synchronize()
            dt_graph = time.perf_counter() - t0
    n = 4 * 256 * 100
    out["4^4"] = {"workload": "4^4, beta 2.3, hot start seed 1, 100 sweeps, plaquette every sweep "
                              "(latency-bound; not a roofline point)",
                  "link_updates_per_s_direct": n / dt_direct,
                  "link_updates_per_s_graph": n / dt_graph,
                  "us_per_sweep_graph": 1e6 * dt_graph / 100,
                  "algorithmic_gbs": step_bytes([256], False, 0) * 100 / dt_graph / 1e9,
                  "hbm_frac": step_bytes([256], False, 0) * 100 / dt_graph / 1e9 / HBM_PEAK_GBS,
                  "mean_plaquette": float(h.cpu().numpy()[:, 0].mean())}
    if with_cpu:
        out["4^4"]["oracle_link_updates_per_s"] = oracle_rate(dims, 100, 2.3)
        out["4^4"]["oracle_threads"] = oracle_threads()
    # beta scan 1.5..3.0 on 16^4 and 24^4, cold + hot, 500 + 1000 sweeps, reunit 10
    betas = np.round(np.arange(1.5, 3.0001, 0.1), 2)
    for L in (16, 24):
        d = [[L] * 4] * (2 * len(betas))
        starts = [0] * len(betas) + [1] * len(betas)
        dt, h, launch = run_batch(su2, torch, dev, d, np.concatenate([betas, betas]), starts, 1000,
                             500, 1000, PL, 10)
        vols = [L ** 4] * len(d)
        ups = 4 * sum(vols) * 1000 / dt
        gbs = step_bytes(vols, False, 0 if launch["reunit_fused"] else 10) * 1000 / dt / 1e9
        P = h[:, :, 0].mean(axis=0)
        key = f"beta_scan_{L}^4"
        out[key] = {"workload": f"{len(d)} chains of {L}^4 (beta 1.5..3.0 step 0.1, cold and hot), "
                                "500 + 1000 sweeps, reunitarise every 10, plaquette every sweep; "
                                "one batch, graph-captured chunks of 50 sweeps",
                    "link_updates_per_s": ups, "algorithmic_gbs": gbs,
                    "hbm_frac": gbs / HBM_PEAK_GBS, "launch": launch,
                    "mean_plaquette_by_beta": [round(float(0.5 * (P[i] + P[i + len(betas)])), 6)
                                               for i in range(len(betas))]}
        if with_cpu:
            out[key]["oracle_link_updates_per_s"] = oracle_rate([L] * 4, 2, 2.3)
            out[key]["oracle_threads"] = oracle_threads()
    # 32^3 x Nt, Nt in {4, 6, 8}, beta 2.00..2.60 step 0.05, cold, 5000 sweeps
    betas = np.round(np.arange(2.0, 2.6001, 0.05), 2)
    nts = (4, 6, 8)
    d = [[32, 32, 32, nt] for nt in nts for _ in betas]
    dt, h, launch = run_batch(su2, torch, dev, d, np.concatenate([betas] * 3), 0, 4000, 0, 5000,
                         PL | su2.SU2_MEAS_POLY, 10)
    vols = [32 ** 3 * x[3] for x in d]
    ups = 4 * sum(vols) * 5000 / dt
    gbs = step_bytes(vols, True, 0 if launch["reunit_fused"] else 10) * 5000 / dt / 1e9
    absL = np.abs(h[1000:, :, 1]).mean(axis=0)
    out["polyakov_32^3xNt"] = {
        "workload": f"{len(d)} chains of 32^3 x Nt (Nt 4, 6, 8; beta 2.00..2.60 step 0.05), "
                    "cold start, 5000 sweeps, plaquette and Polyakov loop every sweep, "
                    "reunitarise every 10; one batch, graph-captured chunks of 50 sweeps",
        "link_updates_per_s": ups, "algorithmic_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
        "launch": launch,
        "mean_abs_polyakov_by_nt": {str(nt): [round(float(x), 5) for x in
                                              absL[k * len(betas):(k + 1) * len(betas)]]
                                    for k, nt in enumerate(nts)}}
    if with_cpu:
        out["polyakov_32^3xNt"]["oracle_threads"] = oracle_threads()
        out["polyakov_32^3xNt"]["oracle_link_updates_per_s"] = oracle_rate([32, 32, 32, 4], 2,
                                                                           2.3)
    return out


def _beta_scan(L):
    b = np.round(np.arange(1.5, 3.0001, 0.1), 2)
    return [[L] * 4] * (2 * len(b)), np.concatenate([b, b]), [0] * len(b) + [1] * len(b)


def _polyakov_grid():
    b = np.round(np.arange(2.0, 2.6001, 0.05), 2)
    return [[32, 32, 32, nt] for nt in (4, 6, 8) for _ in b], np.concatenate([b] * 3), 0


def _replicas64():
    L = [8 + 2 * (r % 7) for r in range(64)]
    return [[l] * 4 for l in L], np.random.default_rng(5).uniform(1.8, 3.0, 64), 1


COUNTER_WORKLOADS = ("headline", "beta16", "beta24", "polyakov", "replicas64", "replicas64_learned",
                     "su3", "plaquette", "fp64", "wilson")


def counters_run(su2, torch, dev, lat, name):
    """Counter runs: the workload with its autotuned launch, then the pass
    launches whose counters are read (the last `pass_launches` pass_kernel
    dispatches of the run), each updating `updates_per_launch` links."""
    if name == "headline":
        lat.autotune(None, su2.SU2_KP)
        lat.heatbath_sweep(2)
        for i in range(16):
            lat.test_pass((i // 2) % 4, i % 2)
        torch.cuda.synchronize()
        return {"pass_launches": 16, "updates_per_launch": int(np.prod(DIMS)) // 2}
    if name == "plaquette":  # the standalone plaquette kernel on the 48^4 field
        lat.heatbath_sweep(2)
        for _ in range(8):
            lat.plaquette()
        torch.cuda.synchronize()
        return {"plaquette_launches": 8, "sites_per_launch": int(np.prod(DIMS))}
    if name == "wilson":  # W(R, T) for R, T <= 4 on the 48^4 field
        lat.heatbath_sweep(2)
        for _ in range(2):
            lat.wilson_loops(4, 4)
        torch.cuda.synchronize()
        return {"wilson_launches": 2, "sites_per_launch": int(np.prod(DIMS))}
    if name == "fp64":  # the FP64-link pass at 48^4 in its autotuned launch
        with su2.Lattice64(DIMS, BETA, SEED, su2.SU2_HOT, device=dev) as l64:
            l64.autotune(None, su2.SU2_KP)
            l64.heatbath_sweep(2)
            for i in range(16):
                l64.test_pass((i // 2) % 4, i % 2)
            l64.synchronize()
        return {"pass_launches": 16, "updates_per_launch": int(np.prod(DIMS)) // 2}
    if name == "su3":
        with su2.Lattice3(DIMS, BETA, SEED, su2.SU2_HOT, device=dev) as l3:
            l3.heatbath_sweep(2)
            for i in range(16):
                l3.test_pass((i // 2) % 4, i % 2)
            l3.synchronize()
        return {"pass_launches": 16, "updates_per_launch": int(np.prod(DIMS)) // 2}
    dims, betas, starts = {"beta16": lambda: _beta_scan(16), "beta24": lambda: _beta_scan(24),
                           "polyakov": _polyakov_grid, "replicas64": _replicas64,
                           "replicas64_learned": _replicas64}[name]()
    learned = name.endswith("learned")
    mode = su2.SU2_LEARNED if learned else su2.SU2_KP
    meas = su2.SU2_MEAS_PLAQ | (su2.SU2_MEAS_POLY if name == "polyakov" else 0)
    with torch.cuda.stream(torch.cuda.Stream(device=dev)):
        net = None
        if learned:
            net = su2.NN(seed=5)
            net.sample_data(2_000_000, 0.5, 30.0, seed=5)
            net.train(4000, 16384, 3e-3, lr_end=1e-5)
            net.build_table()
        b = su2.Batch(dims, betas, starts, seed=5, device=dev)
        if net is not None:
            b.set_proposal(net)
        b.autotune(None, mode)
        lc = b.launch()
        if lc["flags"] & 8:  # the work queue won: read the pass kernel in its per-pass launch
            b.set_launch(256, 1 | 4, 8, 8, 0)
        b.sweep_measure(20, mode, reunit_every=10, meas=meas)
        b.sweep_measure(8, mode, reunit_every=0, meas=meas)
        b.synchronize()
        b.close()
        if net is not None:
            net.close()
    torch.cuda.synchronize()
    return {"pass_launches": 64, "updates_per_launch": sum(int(np.prod(d)) for d in dims) // 2}


def fp64_run(su2, torch, dev, steps=100, launches=80):
    """The 48^4 headline workload with FP64 links and staples (the paper's
    next step): autotuned launch, `steps` sweeps with the fused plaquette and
    reunitarisation every 10, the pass kernel's average launch over
    `launches` launches (256 algorithmic bytes per update: the FP32 pass's
    seven reads and one write of 32-byte links), and the FP32-vs-FP64
    difference of the plaquette and Polyakov loop after one sweep from the
    same FP64 hot start."""
    V = int(np.prod(DIMS))
    out = {"workload": "48^4, beta=6.0, hot start (Philox seed 3), FP64 links and staples; "
                       "step = 1 sweep + fused plaquette, reunitarise every 10"}
    with su2.Lattice64(DIMS, BETA, SEED, su2.SU2_HOT, device=dev) as lat:
        start = lat.get_links()
        with su2.Lattice(DIMS, BETA, SEED, su2.SU2_COLD, device=dev) as l32:
            l32.set_links(start.astype(np.float32))
            l32.heatbath_sweep(1)
            lat.heatbath_sweep(1)
            out["fp32_minus_fp64_after_one_sweep"] = {
                "plaquette": l32.plaquette() - lat.plaquette(),
                "polyakov_signed": l32.polyakov()[0] - lat.polyakov()[0]}
        del start
        out["autotuned_us_per_sweep"] = lat.autotune(None, su2.SU2_KP)
        out["launch"] = lat.launch()
        hist = torch.zeros((steps, 3), dtype=torch.float64, device=dev)
        lat.sweep_measure(10, reunit_every=10, meas=su2.SU2_MEAS_PLAQ, hist=hist)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.sweep_measure(steps, reunit_every=10, meas=su2.SU2_MEAS_PLAQ, hist=hist)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stream = lat.stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(launches):
            lat.test_pass((i // 2) % 4, i % 2)
        e1.record(stream)
        e1.synchronize()
        pass_ms = e0.elapsed_time(e1) / launches
    gbs = 256 * (V // 2) / (pass_ms * 1e-3) / 1e9
    traffic = profile_value(F64_PROFILE, "hbm_bytes_per_launch", f64_source_hash(),
                            key_name="f64_source_hash")
    out.update({"link_updates_per_s": 4 * V * steps / dt, "ms_per_sweep": 1e3 * dt / steps,
                "pass_avg_launch_us": pass_ms * 1e3, "bytes_per_update": 256,
                "pass_algorithmic_gbs": gbs, "pass_hbm_frac": gbs / HBM_PEAK_GBS,
                "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                             "kernel": "pass64_kernel"},
                "mean_plaquette": float(hist.cpu().numpy()[:, 0].mean())})
    return out


def su3_run(su2, torch, dev, steps=100, launches=80, with_cpu=True):
    """SU(3) (Cabibbo-Marinari subgroups on the SU(2) sampler) on the 48^4
    lattice at beta = 6.0 from a hot start: `steps` sweeps with the fused
    plaquette and reunitarisation every 10 after 10 warm-up sweeps, and the
    pass kernel's average launch over `launches` launches.  Algorithmic bytes
    per update: 432 (nine 48-byte links: the updated link read and written,
    the opposite-parity U_mu and U_nu, nu != mu, at both parities read).  The
    ALU side of the roofline: VALU instructions per update from the committed
    counter profile, against 256 CUs x 4 SIMDs issuing one 64-lane FP32 VALU
    instruction per 4 cycles at 2.4 GHz (packed FP32 is not used)."""
    V = int(np.prod(DIMS))
    out = {"workload": "SU(3) 48^4, beta=6.0, hot start (Philox seed 3); step = 1 sweep "
                       "(8 passes, 3 SU(2) subgroup heat-bath draws per link) + fused "
                       "plaquette, reunitarise every 10"}
    side = torch.cuda.Stream(device=dev)  # graph capture needs a non-null stream
    with torch.cuda.stream(side), su2.Lattice3(DIMS, BETA, SEED, su2.SU2_HOT, device=dev) as lat:
        lat.heatbath_sweep(10, reunit_every=10, history=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = lat.heatbath_sweep(steps, reunit_every=10, history=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # the same sweeps as graph replays of one reunitarisation period
        graph_ms = None
        if lat.sweep % 10 == 0:
            reps = max(1, steps // 10)
            hg = torch.zeros(10 * (reps + 1), dtype=torch.float64, device=dev)
            lat.capture(10, reunit_every=10, hist=hg)
            lat.replay(1)
            lat.synchronize()
            t0 = time.perf_counter()
            lat.replay(reps)
            lat.synchronize()
            graph_ms = 1e3 * (time.perf_counter() - t0) / (10 * reps)
        stream = lat.stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(launches):
            lat.test_pass((i // 2) % 4, i % 2)
        e1.record(stream)
        e1.synchronize()
        pass_ms = e0.elapsed_time(e1) / launches
        e0.record(stream)
        for i in range(launches):
            lat.test_or_pass((i // 2) % 4, i % 2)
        e1.record(stream)
        e1.synchronize()
        or_ms = e0.elapsed_time(e1) / launches
        poly = lat.polyakov()
    gbs = SU3_BYTES_PER_UPDATE * (V // 2) / (pass_ms * 1e-3) / 1e9
    h_ = su3_source_hash()
    traffic = profile_value(SU3_PROFILE, "hbm_bytes_per_launch", h_)
    valu = profile_value(SU3_PROFILE, "valu_instructions_per_update", h_)
    # one wave64 VALU instruction per SIMD per 4 cycles: 256 * 4 * 2.4e9 / 4 per s
    valu_peak = 256 * 4 * 2.4e9 / 4 * 64  # lane-instructions per second
    out.update({
        "link_updates_per_s": 4 * V * steps / dt, "ms_per_sweep": 1e3 * dt / steps,
        "graph_ms_per_sweep": graph_ms,
        "graph_link_updates_per_s": None if graph_ms is None else 4 * V / (graph_ms * 1e-3),
        "pass_avg_launch_us": pass_ms * 1e3, "updates_per_launch": V // 2,
        "overrelaxation_pass_avg_launch_us": or_ms * 1e3,
        "mean_plaquette": float(np.mean(h)), "polyakov": poly,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_update": SU3_BYTES_PER_UPDATE, "kernel": "su3_pass_kernel"},
        "alu": None if valu is None else {
            "bound": "alu", "valu_instructions_per_update": valu,
            "achieved": valu * (V // 2) / (pass_ms * 1e-3), "peak": valu_peak,
            "unit": "VALU lane-instructions/s",
            "frac": valu * (V // 2) / (pass_ms * 1e-3) / valu_peak}})
    if with_cpu:
        out["cpu_baseline"] = su3_oracle_rate()
    out["small_lattice_graph"] = su3_small_graph(su2, torch, dev)
    out["small_lattice_batch"] = su3_small_batch(su2, torch, dev)
    return out


def su3_small_graph(su2, torch, dev, dims=(16, 16, 16, 4), sweeps=200):
    """A launch-bound SU(3) lattice (16^3 x 4, beta 5.7, hot start, reunitarise
    every 10): sweeps enqueued directly against the same sweeps replayed from a
    graph of one reunitarisation period (su3_capture_sweeps)."""
    V = int(np.prod(dims))
    side = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(side), su2.Lattice3(list(dims), 5.7, 9, su2.SU2_HOT, device=dev) as lat:
        lat.heatbath_sweep(10, reunit_every=10)
        lat.synchronize()
        t0 = time.perf_counter()
        lat.heatbath_sweep(sweeps, reunit_every=10)
        lat.synchronize()
        direct = (time.perf_counter() - t0) / sweeps
        lat.capture(10, reunit_every=10)
        lat.replay(1)
        lat.synchronize()
        t0 = time.perf_counter()
        lat.replay(sweeps // 10)
        lat.synchronize()
        graph = (time.perf_counter() - t0) / (10 * (sweeps // 10))
    return {"workload": f"SU(3) {dims[0]}^3 x {dims[3]}, beta 5.7, hot start, {sweeps} sweeps, "
                        "reunitarise every 10",
            "us_per_sweep_direct": 1e6 * direct, "us_per_sweep_graph": 1e6 * graph,
            "link_updates_per_s_direct": 4 * V / direct,
            "link_updates_per_s_graph": 4 * V / graph}


SU3_SCAN_BETAS = [round(5.40 + 0.05 * i, 2) for i in range(13)]


def su3_polyakov_scan(su2, torch, dev, dims=(16, 16, 16, 4), therm=300, nmeas=300, every=2):
    """The SU(3) counterpart of the Polyakov-loop scan: 16^3 x 4 from a cold
    start at 13 couplings 5.40..6.00 run as one batch (replica r at coupling
    r), `therm` sweeps, then the Polyakov loop (and the fused plaquette) every
    `every` sweeps for `nmeas` measurements.  beta_c is where <|L|> rises most
    (the same estimator as for SU(2))."""
    nb = len(SU3_SCAN_BETAS)
    t0 = time.perf_counter()
    with su2.Batch3(list(dims), SU3_SCAN_BETAS, 9000, su2.SU2_COLD, device=dev) as b:
        b.heatbath_sweep(therm, reunit_every=10)
        absL, plaq = np.zeros((nmeas, nb)), np.zeros((nmeas, nb))
        for m in range(nmeas):
            plaq[m] = b.heatbath_sweep(every, reunit_every=10, history=True)[-1]
            pl = b.polyakov()
            absL[m] = np.hypot(pl[:, 0], pl[:, 1])
    dt = time.perf_counter() - t0
    rows = []
    for i, beta in enumerate(SU3_SCAN_BETAS):
        a = absL[:, i]
        rows.append({"beta": beta, "mean_abs_polyakov": float(np.mean(a)),
                     "err_abs_polyakov": float(np.std(a, ddof=1) * np.sqrt(2 * tau_int(a) / len(a))),
                     "mean_plaquette": float(np.mean(plaq[:, i]))})
    absl = [r["mean_abs_polyakov"] for r in rows]
    V = int(np.prod(dims))
    return {"workload": f"SU(3) {dims[0]}^3 x {dims[3]}, cold start, {nb} couplings "
                        f"{SU3_SCAN_BETAS[0]}..{SU3_SCAN_BETAS[-1]} as one batch, {therm} + "
                        f"{nmeas} x {every} sweeps, |mean Polyakov loop| every measurement",
            "by_beta": rows, "beta_c": beta_c(SU3_SCAN_BETAS, absl),
            "link_updates_per_s": 4 * V * nb * (therm + nmeas * every) / dt}


def su3_small_batch(su2, torch, dev, dims=(16, 16, 16, 4), n=64, sweeps=100):
    """64 replicas of the launch-bound 16^3 x 4 lattice (beta 5.7, hot start,
    reunitarise every 10) as one SU(3) batch: one launch per pass for all of
    them, against the single lattice's graph-replayed sweeps."""
    V = int(np.prod(dims))
    with su2.Batch3(list(dims), [5.7] * n, 9, su2.SU2_HOT, device=dev) as b:
        b.heatbath_sweep(10, reunit_every=10)
        b.synchronize()
        t0 = time.perf_counter()
        b.heatbath_sweep(sweeps, reunit_every=10)
        b.synchronize()
        dt = (time.perf_counter() - t0) / sweeps
        plaq = b.plaquette()
    return {"workload": f"SU(3) {n} replicas of {dims[0]}^3 x {dims[3]}, beta 5.7, hot start, "
                        f"{sweeps} sweeps, reunitarise every 10, one batch",
            "us_per_sweep_all_replicas": 1e6 * dt, "link_updates_per_s": 4 * V * n / dt,
            "plaquette_mean_over_replicas": float(np.mean(plaq))}


def su3_overrelaxation_gain(su2, torch, dev, dims=(16, 16, 16, 4), beta=5.69, budget=6000,
                           n_or=3, therm=300):
    """Heat bath alone against one heat-bath sweep followed by `n_or`
    over-relaxation sweeps, at equal numbers of sweeps (`budget`), near the
    N_t = 4 deconfinement coupling where the Polyakov loop decorrelates
    slowly: tau_int of |mean Polyakov loop| and of the plaquette (measured after
    every group) and the effective rate groups/s / (2 tau)."""
    out = {"workload": f"SU(3) {dims[0]}^3 x {dims[3]}, beta {beta}, cold start, {therm} "
                       f"thermalisation groups, {budget} sweeps each way"}
    for nor in (0, n_or):
        with su2.Lattice3(list(dims), beta, 5, su2.SU2_COLD, device=dev) as lat:
            for _ in range(therm):
                lat.heatbath_sweep(1, reunit_every=10)
                if nor:
                    lat.overrelax(nor)
            groups = budget // (1 + nor)
            L, P = [], []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(groups):
                h = lat.heatbath_sweep(1, reunit_every=10, history=True)
                if nor:
                    lat.overrelax(nor)
                re, im, _ = lat.polyakov()
                L.append(abs(complex(re, im)))
                P.append(h[0])
            dt = time.perf_counter() - t0
        tl, tp = tau_int(np.array(L)), tau_int(np.array(P))
        out[f"hb+{nor}or"] = {"groups": groups, "seconds": dt, "mean_abs_polyakov": float(np.mean(L)),
                              "tau_int_abs_polyakov": tl, "tau_int_plaquette": tp,
                              "effective_rate_polyakov": groups / dt / (2 * tl),
                              "effective_rate_plaquette": groups / dt / (2 * tp)}
    a, b = out["hb+0or"], out[f"hb+{n_or}or"]
    # wall clock on this small, launch-bound lattice
    out["gain_polyakov"] = b["effective_rate_polyakov"] / a["effective_rate_polyakov"]
    out["gain_plaquette"] = b["effective_rate_plaquette"] / a["effective_rate_plaquette"]
    # per sweep of work: at 48^4 an over-relaxation pass costs what a heat-bath pass
    # costs (both move the same bytes), so this is the gain where the passes are HBM-bound
    out["gain_per_sweep_polyakov"] = a["tau_int_abs_polyakov"] / ((1 + n_or) * b["tau_int_abs_polyakov"])
    out["gain_per_sweep_plaquette"] = a["tau_int_plaquette"] / ((1 + n_or) * b["tau_int_plaquette"])
    return out


def su3_oracle_rate(L=24, beta=BETA):
    """The FP64 SU(3) oracle as it stands: one sweep of an L^4 hot start on all
    host threads, and one pass single-threaded (link updates per second)."""
    from oracle import su2_oracle as o2, su3_oracle as o3
    dims = [L] * 4
    U = o3.init(dims, 1, SEED)
    n = oracle_threads()
    t0 = time.perf_counter()
    o3.sweeps(dims, U, 1, 0, beta, SEED, nthreads=n)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    o3.pass_(dims, U, 0, 0, 1, beta, SEED, nthreads=1)
    d1 = time.perf_counter() - t0
    V = o2.volume(dims)
    return {"value": 4 * V / dt, "unit": "link updates/s", "cores": n, "kind": "oracle",
            "sample": f"one SU(3) sweep of a {L}^4 hot start at beta {beta} (4 x {V} updates)",
            "single_thread_value": (V // 2) / d1}


def creutz(W, R):
    """chi(R, R) = -ln[W(R,R) W(R-1,R-1) / (W(R,R-1) W(R-1,R))], W(0, .) = 1."""
    w = lambda r, t: 1.0 if r == 0 or t == 0 else W[r - 1, t - 1]
    return -np.log(w(R, R) * w(R - 1, R - 1) / (w(R, R - 1) * w(R - 1, R)))


POLYAKOV_BETAS = tuple(np.round(np.arange(2.0, 2.6001, 0.05), 2))


def beta_c(betas, absL):
    """Deconfinement coupling of one N_t from <|L|>(beta): the midpoint of the
    beta interval over which <|L|> rises most."""
    betas, absL = np.asarray(betas, float), np.asarray(absL, float)
    k = int(np.argmax(np.diff(absL)))
    return 0.5 * (betas[k] + betas[k + 1])


def t_over_tc(betas_sigma, sigma, bc, betas):
    """T/Tc = a(beta_c)/a(beta) at fixed N_t, with a ~ sqrt(sigma a^2): the
    string tension in lattice units, interpolated linearly in ln(sigma a^2)
    between the measured couplings."""
    ls = np.log(np.asarray(sigma, float))
    f = lambda b: np.interp(b, betas_sigma, ls)
    return np.exp(0.5 * (f(bc) - f(np.asarray(betas, float))))


def scale_setting(su2, torch, dev, betas=POLYAKOV_BETAS, therm=300, nmeas=40, every=5):
    """Wilson loops W(R,T), R, T <= 4, on thermalised 16^4 lattices (hot start,
    seed 1000 + i) at the couplings of the Polyakov workload, measured every
    `every` sweeps; the Creutz ratios chi(2,2), chi(3,3), chi(4,4) (the string
    tension sigma a^2 in lattice units: the scale the T/Tc axis of the
    Polyakov loop needs), and the time of one W(4,4) measurement on the 48^4
    headline lattice."""
    out = {"workload": f"16^4, beta {list(betas)}, hot start, {therm} thermalisation sweeps, "
                       f"{nmeas} measurements of W(R,T) (R,T <= 4) every {every} sweeps"}
    rows = []
    for i, beta in enumerate(betas):
        with su2.Lattice([16] * 4, beta, 1000 + i, su2.SU2_HOT, device=dev) as lat:
            lat.sweep_measure(therm, reunit_every=10, meas=su2.SU2_MEAS_PLAQ)
            W = []
            for k in range(nmeas):
                lat.sweep_measure(every, reunit_every=10, meas=su2.SU2_MEAS_PLAQ)
                W.append(lat.wilson_loops(4, 4))
        W = np.array(W)
        mean = W.mean(axis=0)
        with np.errstate(invalid="ignore", divide="ignore"):
            chis = {f"chi_{R}{R}": float(creutz(mean, R)) for R in (2, 3, 4)}
        # jackknife error of the Creutz ratios
        with np.errstate(invalid="ignore", divide="ignore"):
            jk = np.array([[creutz((W.sum(axis=0) - W[j]) / (len(W) - 1), R) for R in (2, 3, 4)]
                           for j in range(len(W))])
        err = np.sqrt((len(W) - 1) * jk.var(axis=0))
        rows.append({"beta": float(beta), "W": np.round(mean, 7).tolist(), **chis,
                     **{f"chi_{R}{R}_err": float(e) for R, e in zip((2, 3, 4), err)}})
    out["by_beta"] = rows
    with su2.Lattice(DIMS, BETA, SEED, su2.SU2_HOT, device=dev) as lat:
        lat.wilson_loops(4, 4)
        t0 = time.perf_counter()
        for _ in range(5):
            lat.wilson_loops(4, 4)
        dt = (time.perf_counter() - t0) / 5
    out["wilson_4x4_48^4_ms"] = 1e3 * dt
    # per site and ordered plane (R, T <= 4): 72 quaternion products (16 FMA each), 16
    # four-term dot products, 40 link loads of 16 B; 12 ordered planes per site
    V = int(np.prod(DIMS))
    flop = 12 * (72 * 16 + 16 * 4) * 2 * V
    gathered = 12 * 40 * 16 * V
    out["wilson_4x4_48^4"] = {
        "fp32_tflops": flop / dt / 1e12, "fp32_frac": flop / dt / 1e12 / FP32_PEAK_TFLOPS,
        "gathered_bytes_per_site": 12 * 40 * 16, "gathered_tbs": gathered / dt / 1e12,
        "hbm_algorithmic_frac": 64 * V / dt / 1e9 / HBM_PEAK_GBS,
        "note": "one thread per site and plane; the links of each stage of the loop lines "
                "are gathered together (480 16-byte gathers per site, served by L1/L2)"}
    return out


def cpu_baseline(sample_sweeps=5):
    from oracle import su2_oracle as orc
    threads = orc.max_threads()
    V = int(np.prod(DIMS))
    rates = {}
    for nt, ns in ((threads, sample_sweeps), (1, 1)):
        U = orc.init(DIMS, 1, SEED)
        t0 = time.perf_counter()
        orc.sweeps(DIMS, U, ns, 0, BETA, SEED, nthreads=nt, measure=True)
        dt = time.perf_counter() - t0
        rates[nt] = (4 * V * ns / dt, dt)
    return {"value": rates[threads][0], "unit": "link updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sample_sweeps} FP64 sweep(s) + plaquette + Polyakov of the 48^4 "
                      f"beta=6.0 hot-start lattice, {threads} OpenMP threads, "
                      f"{rates[threads][1]:.1f} s",
            "single_thread": {"value": rates[1][0], "cores": 1,
                              "sample": f"the same sweep on 1 thread, {rates[1][1]:.1f} s"},
            "host": host_cpu()}


def host_cpu():
    """CPU model and logical CPUs of the host the oracle ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--pass-launches", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the batched plain-vs-learned comparison")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-link workload")
    ap.add_argument("--no-wilson", action="store_true", help="skip the Wilson-loop workload")
    ap.add_argument("--no-su3", action="store_true", help="skip the SU(3) workload")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 4^4, beta-scan and Polyakov workloads")
    ap.add_argument("--counters", nargs="?", const="headline", default=None,
                    choices=list(COUNTER_WORKLOADS),
                    help="short program for rocprofv3 --pmc runs: the workload's autotuned "
                         "launch, then its last pass launches (16 for the 48^4 headline, 8 "
                         "sweeps otherwise), then 4 plain device copies of 339.7 MB that "
                         "calibrate FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "t-slab decomposition is designed but not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1010_1486_amd as su2

    dev = torch.device("cuda:0")
    V = int(np.prod(DIMS))
    side = torch.cuda.Stream(device=dev)  # graph capture needs a non-null stream
    with torch.cuda.stream(side):
        lat = su2.Lattice(DIMS, BETA, SEED, su2.SU2_HOT, device=dev)
    lat.set_reunit_fused(True)
    stream = lat.stream
    meas = su2.SU2_MEAS_PLAQ
    hist = torch.zeros((max(args.steps, args.warmup, 1), 3), dtype=torch.float64, device=dev)

    if args.counters:
        info = counters_run(su2, torch, dev, lat, args.counters)
        x = torch.ones(su2.su2_links_bytes(DIMS) // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(4):
            y.copy_(x)
        torch.cuda.synchronize()
        info.update({"counters_run": args.counters, "copy_bytes": 4 * x.numel()})
        print(json.dumps(info))
        lat.close()
        return

    tuned_us = lat.autotune(None, su2.SU2_KP)
    print(f"[bench] autotuned launch: {tuned_us:.1f} us per sweep", file=sys.stderr, flush=True)
    print(f"[bench] warmup {args.warmup} sweeps on {DIMS}", file=sys.stderr, flush=True)
    lat.sweep_measure(args.warmup, reunit_every=10, meas=meas, hist=hist)
    torch.cuda.synchronize()

    # the timed sweeps replay a captured graph of one reunitarisation period
    # (10 sweeps: 80 passes with the fused plaquette, the last sweep's passes
    # reunitarising the links they store, the end-of-sweep bookkeeping); a
    # remainder below 10 runs as direct launches
    chunk = 10
    pad = (-lat.sweep) % chunk
    if pad:
        lat.sweep_measure(pad, reunit_every=10, meas=meas, hist=hist)
    full, rem = divmod(args.steps, chunk)
    hist_g = torch.zeros((max(full * chunk, 1), 3), dtype=torch.float64, device=dev)
    if full:
        lat.capture(chunk, su2.SU2_KP, reunit_every=10, meas=meas, hist=hist_g)
    print(f"[bench] timing {args.steps} sweeps ({full} graph replays of {chunk}, {rem} direct)",
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        g0.record(stream)
        if full:
            lat.replay(full)
        if rem:
            lat.sweep_measure(rem, reunit_every=10, meas=meas, hist=hist)
        g1.record(stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    gpu_us_per_sweep = g0.elapsed_time(g1) * 1e3 / args.steps
    h = np.concatenate([hist_g[:full * chunk].cpu().numpy(), hist[:rem].cpu().numpy()])

    # the same sweeps with the reunitarisation as a separate pass over the
    # field followed by a standalone plaquette (graph replays of 10 sweeps)
    lat.set_reunit_fused(False)
    pad = (-lat.sweep) % chunk
    if pad:
        lat.sweep_measure(pad, reunit_every=10, meas=meas, hist=hist)
    nrep_s = 10
    hist_s = torch.zeros(((nrep_s + 1) * chunk, 3), dtype=torch.float64, device=dev)
    lat.capture(chunk, su2.SU2_KP, reunit_every=10, meas=meas, hist=hist_s)
    lat.replay(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.replay(nrep_s)
    torch.cuda.synchronize()
    sep_us_per_sweep = (time.perf_counter() - t0) * 1e6 / (nrep_s * chunk)
    lat.set_reunit_fused(True)

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
    # bandwidth floor: the same bytes per launch without the stencil
    out_buf = torch.empty(2 * V, dtype=torch.float32, device=dev)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for i in range(args.pass_launches):
            lat.test_stream_pass((i // 2) % 4, i % 2, out_buf)
        e1.record(stream)
    e1.synchronize()
    floor_ms = e0.elapsed_time(e1) / args.pass_launches
    del out_buf
    achieved = BYTES_PER_UPDATE * (V // 2) / (pass_ms * 1e-3) / 1e9
    traffic = traffic_from_profile()

    value = 4 * V * args.steps / dt
    out = {
        "metric": METRIC, "value": value, "unit": "link updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "48^4 periodic, beta=6.0, hot start (Philox seed 3); step = 1 "
                               "heat-bath sweep (8 passes) + fused plaquette, "
                               "reunitarise every 10 sweeps (fused into that sweep's passes)",
                   "dims": DIMS, "beta": BETA, "links": 4 * V, "mode": "plain KP"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x copy "
                                     "calibration + WRITE_SIZE)",
                     "traffic_gbs": None if traffic is None else traffic / (pass_ms * 1e-3) / 1e9,
                     "kernel": "pass_kernel", "avg_launch_us": pass_ms * 1e3,
                     "bytes_per_update": BYTES_PER_UPDATE, "updates_per_launch": V // 2,
                     "floor_us": floor_ms * 1e3,
                     "floor_gbs": BYTES_PER_UPDATE * (V // 2) / (floor_ms * 1e-3) / 1e9,
                     "frac_of_floor": floor_ms / pass_ms},
        "plaquette_mean_last_half": float(h[args.steps // 2:, 0].mean()),
        "timed_sweeps": {"graph_replays": full, "sweeps_per_replay": chunk, "direct_sweeps": rem,
                         "wall_us_per_sweep": 1e6 * dt / args.steps,
                         "gpu_event_us_per_sweep": gpu_us_per_sweep,
                         "pass_kernels_us_per_sweep": 8 * pass_ms * 1e3,
                         "wall_over_pass_kernels": 1e6 * dt / args.steps / (8 * pass_ms * 1e3),
                         "reunitarisation": "fused into the passes of every 10th sweep",
                         "separate_reunitarisation_wall_us_per_sweep": sep_us_per_sweep},
        "autotuned_us_per_sweep": tuned_us,
        "launch": lat.launch(),
    }
    # the same workload from a cold start, in the same launch
    launch = lat.launch()
    lat.close()
    with su2.Lattice(DIMS, BETA, SEED, su2.SU2_COLD, device=dev) as cold:
        cold.set_reunit_fused(True)
        cold.set_launch(launch["block"], launch["flags"], launch["tile_z"], launch["tile_t"],
                        launch["grid_cap"])
        cold.sweep_measure(args.warmup, reunit_every=10, meas=meas, hist=hist)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cold.sweep_measure(args.steps, reunit_every=10, meas=meas, hist=hist)
        torch.cuda.synchronize()
        dc = time.perf_counter() - t0
        hc = hist[:args.steps].cpu().numpy()
    out["cold_start"] = {"workload": "48^4, beta=6.0, cold start; same step and launch as the "
                                     "headline", "link_updates_per_s": 4 * V * args.steps / dc,
                         "ms_per_step": 1e3 * dc / args.steps,
                         "plaquette_mean_last_half": float(hc[args.steps // 2:, 0].mean())}
    if not args.no_configs:
        print("[bench] other workloads", file=sys.stderr, flush=True)
        with torch.cuda.stream(torch.cuda.Stream(device=dev)):  # graphs need a non-null stream
            out["other_configs"] = other_configs(su2, torch, dev, not args.no_cpu_baseline)
        torch.cuda.synchronize()
    if not args.no_fp64:
        print("[bench] FP64 links", file=sys.stderr, flush=True)
        out["fp64"] = fp64_run(su2, torch, dev)
    if not args.no_su3:
        print("[bench] SU(3) subgroup heat bath", file=sys.stderr, flush=True)
        out["su3"] = su3_run(su2, torch, dev, with_cpu=not args.no_cpu_baseline)
        out["su3"]["polyakov_scan_nt4"] = su3_polyakov_scan(su2, torch, dev)
        out["su3"]["overrelaxation"] = su3_overrelaxation_gain(su2, torch, dev)
    if not args.no_wilson:
        print("[bench] Wilson loops and Creutz ratios", file=sys.stderr, flush=True)
        out["scale_setting"] = scale_setting(su2, torch, dev)
    if "scale_setting" in out and "other_configs" in out:
        ss = out["scale_setting"]["by_beta"]
        bs = [r["beta"] for r in ss]
        sig = [r["chi_22"] for r in ss]
        pol = out["other_configs"]["polyakov_32^3xNt"]["mean_abs_polyakov_by_nt"]
        tt = {"scale": "sigma a^2 from the Creutz ratio chi(2,2) on 16^4, interpolated in "
                       "ln(sigma a^2); beta_c per N_t where <|L|> rises most",
              "by_nt": {}}
        for nt, absL in pol.items():
            bc = beta_c(POLYAKOV_BETAS, absL)
            x = t_over_tc(bs, sig, bc, POLYAKOV_BETAS)
            tt["by_nt"][nt] = {"beta_c": bc, "T_over_Tc": np.round(x, 4).tolist(),
                               "mean_abs_polyakov": absL}
        out["polyakov_vs_T_over_Tc"] = tt
    if not args.no_learned:
        print("[bench] batched plain vs learned proposal", file=sys.stderr, flush=True)
        out["learned_vs_plain"] = learned_vs_plain(su2, torch, dev,
                                                   with_cpu=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
