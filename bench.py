"""Throughput of plain parallel tempering on one MI355X.

Workload (the large plain-PT configuration): N = 256 modes, 8 disorder
samples (random frequencies, frequency-matched terms, Gaussian couplings of
variance N/c), 40 temperatures geometric in [0.25, 1.5], 2 replicas (640
copies), FP32 fields and energy changes, FP64 energy recomputation every 100
sweeps, a swap round and a measurement after every sweep.  A step is one
recomputation interval: 100 sweeps of every copy (N/2 two-mode updates each),
each followed by its swap round and measurement, then the FP64
recomputation -- every part of the path.  Inputs are synthetic and already
resident in HBM when timing starts.

Prints one JSON line.  ``value`` = mode-updates/s (N mode-updates per copy
per sweep) over the timed steps.  ``roofline`` describes the sweep kernel:
``achieved`` = algorithmic bytes per launch (every list entry a step
streams: 6.25 B in the chunked layout, 25 B per chunk of 4 entries sharing
their partner mode; 8 B in the packed one) over its mean duration measured
with HIP events on the context's stream; ``traffic`` = the fabric bytes per
launch from the committed rocprofv3 counters of this kernel source;
``frac`` = traffic per second over the published 8 TB/s HBM peak, and
``peak`` = that peak scaled by algorithmic / fabric bytes, so that
achieved / peak = frac (fabric bytes include Infinity-Cache hits: the HBM
share is at most frac).  The list-stream probe (rlpt_stream_lists: the
sweep's grid and reads with no arithmetic) is timed beside it.
``cpu_baseline`` times the CPU FP64 oracle on a bounded slice of the same
workload (sample 0, all 80 copies, whole sweeps for ~10 s).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SEED_BASE = 2511135080 + 400  # disorder seed of sample mu: SEED_BASE + mu
HBM_PEAK_GBS = 8000.0
LDS_PEAK_GBS = 128 * 256 * 2.4  # 128 B per clock per CU, 256 CUs, 2.4 GHz
METRIC = "mode-updates/s + τ_int-corrected sweeps/s (learned vs plain PT), N=256, 1 GPU"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_n256_traffic.json")
BATCHED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batched_traffic.json")
# the sweep kernel and the host code that lays out its launch (tiles, item order)
KERNEL_SRC = [os.path.join(ROOT, "paper_2511_13508_amd", "csrc", f) for f in ("kernels.hip", "api.cpp")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sha() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for_current_kernel(launch_bytes_alg: float, path: str = TRAFFIC_FILE):
    """HBM bytes per sweep launch from committed rocprofv3 counters, if they
    were taken on the current kernel source; else None."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_sha():
        return None
    return t.get("hbm_bytes_per_launch")


PROFILE_CMDS = {
    "kt": "rocprofv3 --kernel-trace --stats -f csv -d {OUT}/kt -o kt -- python bench.py --steps 20 --warmup 5 "
          "--tau-sweeps 0 --no-cpu-baseline --no-cached",
    "kta": "rocprofv3 --kernel-trace --stats -f csv -d {OUT}/kta -o kta -- python bench.py --steps 1 "
           "--warmup 3 --tau-sweeps 100 --no-cpu-baseline --no-n64 --no-batched",
    "ktb": "rocprofv3 --kernel-trace --stats -f csv -d {OUT}/ktb -o ktb -- python bench.py --workload batched "
           "--steps 5",
    "ktl": "rocprofv3 --kernel-trace --stats -f csv -d {OUT}/ktl -o ktl -- python bench.py --workload learned64 "
           "--steps 20",
    "pmc64": "rocprofv3 --pmc SQ_WAVES SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAIT_INST_LDS SQ_INSTS_VALU SQ_WAVE_CYCLES "
             "SQ_BUSY_CYCLES SQ_INSTS_SALU --kernel-include-regex 'k_sweep<' -f csv -d {OUT}/pmc64 -o pmc -- "
             "python bench.py --workload n64",
    "sq256": "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_BUSY_CYCLES SQ_WAVE_CYCLES "
             "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS GRBM_GUI_ACTIVE --kernel-include-regex 'k_sweep<|k_stream_lists' "
             "-f csv -d {OUT}/sq256 -o pmc -- python bench.py --sweeps-per-step 1 --steps 4 --warmup 2 "
             "--tau-sweeps 0 --no-cpu-baseline --no-cached",
    "pmc": "rocprofv3 --pmc {C} --kernel-include-regex 'k_sweep<|k_stream_lists' -f csv -d {OUT}/pmc_{C} -o pmc -- "
           "python bench.py --sweeps-per-step 1 --steps 4 --warmup 2 --tau-sweeps 0 --no-cpu-baseline --no-cached",
    "cal": "rocprofv3 --pmc {C} -f csv -d {OUT}/cal_{C} -o cal -- python bench.py --copy-calibration",
    "pmcb": "rocprofv3 --pmc {C} --kernel-include-regex 'k_sweep<' -f csv -d {OUT}/pmcb_{C} -o pmc -- python bench.py "
            "--workload batched --batched-launches-only",
}


def summarize_profiles(d):
    """Turn the rocprofv3 CSVs of the commands above (written under directory d,
    run from the repository root) into the summaries under profiles/."""
    import csv

    def cmd(tag, counter=""):
        return PROFILE_CMDS[tag].format(OUT=os.path.relpath(d, ROOT) if os.path.isabs(d) else d, C=counter)

    def rows(path):
        with open(path) as f:
            return list(csv.DictReader(f))

    def mean_counter(path, kernel_pred):
        vals = [float(r["Counter_Value"]) for r in rows(path) if kernel_pred(r["Kernel_Name"])]
        return sum(vals) / len(vals), len(vals)

    lines = []
    have_headline = all(os.path.exists(os.path.join(d, x)) for x in ("kt", "pmc_FETCH_SIZE", "pmc_WRITE_SIZE",
                                                                    "cal_FETCH_SIZE", "cal_WRITE_SIZE"))
    is_sweep = lambda n: "k_sweep<" in n  # noqa: E731
    is_ceiling = lambda n: "k_stream_lists" in n  # noqa: E731
    is_copy = lambda n: "copyBuffer" in n  # noqa: E731
    if have_headline:
        stats = rows(os.path.join(d, "kt", "kt_kernel_stats.csv"))
        lines = ["# rocprofv3 kernel statistics, headline N=256 workload (8 samples x 40 T x 2 replicas, streaming sweep, "
                 "per-copy pairs); k_stream_lists is the list-stream ceiling the bench measures beside it",
                 "# command (from the repository root):",
                 "#   " + cmd("kt"), "",
                 f"{'kernel':<60} {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}"]
        for r in stats:
            name = r["Name"].replace("rlpt::(anonymous namespace)::", "")[:60]
            lines.append(f"{name:<60} {int(r['Calls']):>6} {float(r['AverageNs']) / 1e3:>10.1f} "
                         f"{float(r['MinNs']) / 1e3:>10.1f} {float(r['MaxNs']) / 1e3:>10.1f} {float(r['Percentage']):>6.2f}")
        avg_ns = {}
        for tag, pred in (("k_sweep", is_sweep), ("k_stream_lists", is_ceiling)):
            hit = [r for r in stats if pred(r["Name"])]
            if hit:
                avg_ns[tag] = float(hit[0]["AverageNs"])
        cal_f, _ = mean_counter(os.path.join(d, "cal_FETCH_SIZE", "cal_counter_collection.csv"), is_copy)
        cal_w, _ = mean_counter(os.path.join(d, "cal_WRITE_SIZE", "cal_counter_collection.csv"), is_copy)
        copy_bytes = 512 * 1024 * 1024
        f_scale, w_scale = copy_bytes / (cal_f * 1024), copy_bytes / (cal_w * 1024)
        traffic = {"kernel": "k_sweep<float, 256>", "kernel_source_sha": kernel_sha(),
                   "copy_kernel_fetch_kib": cal_f, "copy_kernel_write_kib": cal_w, "copy_bytes": copy_bytes,
                   "fetch_scale": f_scale, "write_scale": w_scale,
                   "commands": [cmd("pmc", "FETCH_SIZE"), cmd("pmc", "WRITE_SIZE"), cmd("cal", "FETCH_SIZE"),
                                cmd("cal", "WRITE_SIZE")]}
        lines += ["", "# fabric traffic per dispatch (rocprofv3 --pmc, one counter per run; FETCH_SIZE counts every L2 "
                      "miss, whether the Infinity Cache or HBM serves it):"]
        for tag, pred in (("k_sweep", is_sweep), ("k_stream_lists", is_ceiling)):
            try:
                fetch_kib, nf = mean_counter(os.path.join(d, "pmc_FETCH_SIZE", "pmc_counter_collection.csv"), pred)
                write_kib, nw = mean_counter(os.path.join(d, "pmc_WRITE_SIZE", "pmc_counter_collection.csv"), pred)
            except ZeroDivisionError:
                continue
            hbm = fetch_kib * 1024 * f_scale + write_kib * 1024 * w_scale
            key = "" if tag == "k_sweep" else "ceiling_"
            traffic.update({key + "fetch_kib_per_dispatch": fetch_kib, key + "write_kib_per_dispatch": write_kib,
                            key + "dispatches": [nf, nw], key + "hbm_bytes_per_launch": hbm,
                            key + "avg_duration_ns_kernel_trace": avg_ns.get(tag)})
            lines.append(f"#   {tag}: FETCH_SIZE {fetch_kib:.0f} KiB x {f_scale:.4f} (copy-kernel scale) + WRITE_SIZE "
                         f"{write_kib:.0f} KiB x {w_scale:.4f} = {hbm / 1e9:.3f} GB per launch"
                         + (f"; over the kernel-trace average {avg_ns[tag] / 1e6:.3f} ms: {hbm / avg_ns[tag]:.0f} GB/s"
                            if tag in avg_ns else ""))
        os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
        with open(os.path.join(ROOT, "profiles", "sweep_n256_kernel_stats.txt"), "w") as f:
            f.write("\n".join(lines) + "\n")
    if all(os.path.exists(os.path.join(d, x)) for x in ("pmcb_FETCH_SIZE", "pmcb_WRITE_SIZE", "cal_FETCH_SIZE",
                                                        "cal_WRITE_SIZE")):
        cal_f, _ = mean_counter(os.path.join(d, "cal_FETCH_SIZE", "cal_counter_collection.csv"), is_copy)
        cal_w, _ = mean_counter(os.path.join(d, "cal_WRITE_SIZE", "cal_counter_collection.csv"), is_copy)
        copy_bytes = 512 * 1024 * 1024
        f_scale, w_scale = copy_bytes / (cal_f * 1024), copy_bytes / (cal_w * 1024)
        fetch_kib, nf = mean_counter(os.path.join(d, "pmcb_FETCH_SIZE", "pmc_counter_collection.csv"), is_sweep)
        write_kib, nw = mean_counter(os.path.join(d, "pmcb_WRITE_SIZE", "pmc_counter_collection.csv"), is_sweep)
        tb = {"kernel": "k_sweep, batched uneven-N launch (built-in tiles)", "kernel_source_sha": kernel_sha(),
              "fetch_kib_per_dispatch": fetch_kib, "write_kib_per_dispatch": write_kib, "dispatches": [nf, nw],
              "fetch_scale": f_scale, "write_scale": w_scale,
              "hbm_bytes_per_launch": fetch_kib * 1024 * f_scale + write_kib * 1024 * w_scale,
              "commands": [cmd("pmcb", "FETCH_SIZE"), cmd("pmcb", "WRITE_SIZE"), cmd("cal", "FETCH_SIZE"),
                           cmd("cal", "WRITE_SIZE")]}
        with open(BATCHED_TRAFFIC_FILE, "w") as f:
            json.dump(tb, f, indent=1)
    sq = os.path.join(d, "sq256", "pmc_counter_collection.csv")
    if os.path.exists(sq):
        rs = rows(sq)
        bl = ["# rocprofv3 SQ counters, headline N=256 workload: the sweep kernel and the list-stream ceiling kernel "
              "(same grid, tile and list reads, no arithmetic), mean per dispatch",
              "# command (from the repository root):", "#   " + cmd("sq256"), ""]
        for tag, pred in (("k_sweep", is_sweep), ("k_stream_lists", is_ceiling)):
            acc = {}
            for r in rs:
                if pred(r["Kernel_Name"]):
                    acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            if not acc:
                continue
            bl.append(f"# {tag}")
            for k in sorted(acc):
                bl.append(f"{k:<24} {sum(acc[k]) / len(acc[k]):>16.1f}   ({len(acc[k])} dispatches)")
            bl.append("")
        with open(os.path.join(ROOT, "profiles", "sweep_n256_sq_counters.txt"), "w") as f:
            f.write("\n".join(bl) + "\n")
    other = (("kta", "bench_all_kernel_stats.txt",
              "N=256 bench with every variant after 300 warm-up sweeps: streaming and cached-field sweeps, shared "
              "pairs, learned proposal (harvest, training, moves), the sparse N=1024 run and the IPR comparison "
              "(k_sweep<float, 256, 2> here also covers the shared-pair and small-N IPR launches)"),
             ("ktb", "batched_kernel_stats.txt",
              "batched uneven-N workload (N in {32,48,64,96,128} x 32 samples x 32 T x 2 replicas, 10-sweep "
              "HIP-graph segments, built-in then tuned tiles, autotuner trials)"),
             ("ktl", "learned_n64_kernel_stats.txt",
              "learned-proposal comparison at N=64 (8 samples x 24 T x 2 replicas): plain run, harvest of 10^5 "
              "pairs per network, training (MFMA bfloat16 GEMMs), learned run with one round per sweep, "
              "100-sweep HIP-graph segments"))
    for tag, fname, title in other:
        path = os.path.join(d, tag, tag + "_kernel_stats.csv")
        if not os.path.exists(path):
            continue
        bl = ["# rocprofv3 kernel statistics, " + title, "# command (from the repository root):",
              "#   " + cmd(tag), "",
              f"{'kernel':<60} {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}"]
        for r in rows(path):
            name = r["Name"].replace("rlpt::(anonymous namespace)::", "")[:60]
            bl.append(f"{name:<60} {int(r['Calls']):>6} {float(r['AverageNs']) / 1e3:>10.1f} "
                      f"{float(r['MinNs']) / 1e3:>10.1f} {float(r['MaxNs']) / 1e3:>10.1f} {float(r['Percentage']):>6.2f}")
        with open(os.path.join(ROOT, "profiles", fname), "w") as f:
            f.write("\n".join(bl) + "\n")
    pmc64 = os.path.join(d, "pmc64", "pmc_counter_collection.csv")
    if os.path.exists(pmc64):
        # the run also sweeps N = 32 ... 128 for the latency floor: keep the
        # N = 64 kernel variant, the one with the most dispatches
        rs = rows(pmc64)
        counts = {}
        for r in rs:
            counts[r["Kernel_Name"]] = counts.get(r["Kernel_Name"], 0) + 1
        top = max(counts, key=counts.get)
        acc = {}
        for r in rs:
            if r["Kernel_Name"] == top:
                acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        kname = top.replace("rlpt::(anonymous namespace)::", "")[:70]
        bl = ["# rocprofv3 SQ counters of the sweep kernel, N=64 configuration (8 samples x 24 T x 2 replicas, 384 "
              "copies, 512 threads per copy), mean per dispatch; the N=64 point of the latency-floor run (same "
              "kernel, tile and size) is included, the other N of that run are not",
              "# command (from the repository root):", "#   " + cmd("pmc64"), f"# kernel: {kname}", ""]
        for k in sorted(acc):
            bl.append(f"{k:<24} {sum(acc[k]) / len(acc[k]):>16.1f}   ({len(acc[k])} dispatches)")
        with open(os.path.join(ROOT, "profiles", "sweep_n64_sq_counters.txt"), "w") as f:
            f.write("\n".join(bl) + "\n")
    if have_headline:
        with open(TRAFFIC_FILE, "w") as f:
            json.dump(traffic, f, indent=1)
        print("\n".join(lines))


def cpu_baseline(N, temps, n_reps, budget_s, n_threads):
    """The oracle on the host: whole sweeps of sample 0 for about budget_s on
    n_threads threads, then the same on one thread (one copy per thread, so
    the 1-thread figure is the per-core rate)."""
    from oracle import oracle as O
    og = O.Graph(N, SEED_BASE + 0)

    def rate(threads, budget):
        pt = O.PT(og, temps, n_reps=n_reps, run_seed=1, sample=0, swap_interval=1, resync_interval=100,
                  measure_start=0, measure_interval=1, n_bins=100, n_threads=threads)
        t0 = time.perf_counter()
        sweeps = 0
        while time.perf_counter() - t0 < budget:
            pt.run(1)
            sweeps += 1
        el = time.perf_counter() - t0
        return N * pt.R * sweeps / el, f"{pt.R} copies x {sweeps} whole sweeps", el

    v, what, el = rate(n_threads, budget_s)
    v1, what1, el1 = rate(1, budget_s / 2)
    return {"value": v, "unit": "mode-updates/s", "cores": n_threads, "kind": "oracle",
            "sample": f"sample 0 of the workload: {what} (N={N}, {og.n_terms} terms), FP64, {el:.1f} s",
            "value_1_core": v1, "sample_1_core": f"{what1}, {el1:.1f} s",
            "cpu_model": cpu_model(), "cpus_available": len(os.sched_getaffinity(0)), "nproc": os.cpu_count()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def batched(args, short=False):
    """The batched uneven-N configuration: N in {32, 48, 64, 96, 128} x 32
    samples x 32 temperatures x 2 replicas in one launch per sweep, a segment of
    10 sweeps captured in a HIP graph and replayed; built-in tiles versus tiles
    chosen by the autotuner.  Returns its own result (not the headline);
    short: 500 sweeps per rate instead of the step count's."""
    import torch
    from paper_2511_13508_amd import rlpt

    Ns, per_N, T, reps = [32, 48, 64, 96, 128], 32, 32, 2
    temps = 0.3 * (1.5 / 0.3) ** (np.arange(T) / (T - 1))
    log("building 160 graphs")
    graphs = [rlpt.Graph(N, 2511135080 + 200 + 1000 * i + m) for i, N in enumerate(Ns) for m in range(per_N)]
    copies = len(graphs) * T * reps
    mode_updates_per_sweep = sum(g.N for g in graphs) * T * reps
    kw = dict(n_temps=T, n_reps=reps, precision=rlpt.FP32, swap_interval=1, resync_interval=0, measure_start=0,
              measure_interval=10, n_bins=100)

    # algorithmic bytes of one sweep launch: every copy streams, per two-mode
    # step, the lists of j and k (all lists chunked here: 6.25 B per entry)
    infos = [g.info() for g in graphs]
    bytes_per_sweep = sum(reps * T * inf["deg_sum"] * 6.25 for inf in infos)

    if getattr(args, "batched_launches_only", False):
        # only the mixed launch with built-in tiles, 20 eager sweeps (the counters' run)
        rlpt.tune_clear()
        ctx = rlpt.Context(graphs, temps, **kw)
        ctx.init(1)
        ctx.sweep(20)
        torch.cuda.synchronize()
        ctx.check()
        ctx.close()
        return {"batched_launches_only": 20}

    def rate(gs, ctx_kw, segments):
        """mode-updates/s of 10-sweep HIP-graph segments, then the sweep kernel's
        mean launch time from HIP events over 20 eager sweeps"""
        ctx = rlpt.Context(gs, temps, **ctx_kw)
        ctx.init(1)
        ctx.run_graph(10, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.run_graph(10, segments)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.sweep_timing(True)
        ctx.sweep(20)
        torch.cuda.synchronize()
        ctx.check()
        kms, launches = ctx.sweep_time()
        tile = ctx.tile()
        ceil_ms = ctx.stream_lists(5) if len(gs) == len(graphs) else None
        ctx.close()
        return sum(g.N for g in gs) * T * reps * segments * 10 / el, (kms / launches, ceil_ms), tile

    segs = 50 if short else max(args.sweeps // 10, 1)

    def run(tag):
        v, (ms, ceil_ms), (block, cp) = rate(graphs, kw, segs)
        tile = {int(N): int(cp[i * per_N]) for i, N in enumerate(Ns)}
        log(f"{tag}: {v:.4g} mode-updates/s, block {block}, copies per block {tile}")
        return v, block, tile, ms, ceil_ms

    rlpt.tune_clear()
    v0, b0, t0_, ms0, _ = run("built-in tiles")
    # each N class alone (its 32 samples in a launch of their own, built-in tile)
    alone = {}
    for i, N in enumerate(Ns):
        vN, (msN, _), _ = rate(graphs[i * per_N:(i + 1) * per_N], kw, segs)
        alone[N] = {"mode_updates_per_s": vN, "ms_per_launch": msN,
                    "share_of_mixed_mode_updates": N * per_N / sum(g.N for g in graphs)}
        log(f"N={N} alone: {vN:.4g} mode-updates/s, {msN:.3f} ms per sweep launch")
    log("autotuning")
    t_tune = time.perf_counter()
    n_trials = rlpt.autotune(graphs, temps, sweeps_per_trial=10, **kw)
    t_tune = time.perf_counter() - t_tune
    v1, b1, t1_, ms1, ceil1 = run("tuned tiles")
    # the tuner times every trial on the whole launch: per N, the trial of the chosen tile
    per_N = {}
    for e in rlpt.tune_entries():
        N = e["n_modes"]
        if e["block_threads"] == b1 and e["copies_per_block"] == t1_[N]:
            per_N[N] = {"copies_per_block": t1_[N], "launch_ms_per_sweep": e["ms_per_sweep"]}
    # roofline of the built-in tiles' launch (the configuration whose fabric bytes are committed)
    traffic_b = traffic_for_current_kernel(bytes_per_sweep, BATCHED_TRAFFIC_FILE)
    roof_b = {"bound": "hbm", "kernel": "k_sweep (one launch for every N, built-in tiles)", "unit": "GB/s",
              "algorithmic_bytes_per_launch": bytes_per_sweep, "ms_per_launch": ms0,
              "achieved": bytes_per_sweep / ms0 / 1e6, "hbm_peak_published": HBM_PEAK_GBS,
              "frac_of_hbm_peak": bytes_per_sweep / ms0 / 1e6 / HBM_PEAK_GBS, "traffic": traffic_b,
              "ms_per_launch_tuned_tiles": ms1,
              "list_stream_probe_ms": ceil1, "sweep_over_probe_time_tuned": ms1 / ceil1}
    if traffic_b:
        roof_b.update({"peak": HBM_PEAK_GBS * bytes_per_sweep / traffic_b,
                       "frac": traffic_b / ms0 / 1e6 / HBM_PEAK_GBS, "traffic_GBps": traffic_b / ms0 / 1e6,
                       "peak_kind": "published HBM peak x algorithmic / fabric bytes (profiles/batched_traffic.json)"})
    else:
        roof_b.update({"peak": bytes_per_sweep / ceil1 / 1e6, "frac": ceil1 / ms1,
                       "peak_kind": "measured list-stream probe of the tuned launch (no committed counters)"})
    out = {"metric": "aggregate mode-updates/s, batched uneven N (one launch per sweep, HIP graph)",
           "value": v1, "unit": "mode-updates/s", "untuned_value": v0, "tuned_vs_untuned": v1 / v0,
           "copies": copies, "sweeps": segs * 10, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batched uneven N: N in {32,48,64,96,128} x 32 samples x 32 temperatures x "
                                  "2 replicas, FP32, 10-sweep HIP-graph segments"},
           "roofline": roof_b,
           "per_N_alone": alone,
           "tile_builtin": {"block": b0, "copies_per_block": t0_}, "tile_tuned": {"block": b1, "copies_per_block": t1_},
           "autotune": {"trials": n_trials, "seconds": t_tune,
                        "method": "per workgroup size, each N's copies per workgroup timed on the whole launch "
                                  "with the other N at their current choice", "chosen_trials": per_N}}
    log(f"batched: {v1:.4g} mode-updates/s tuned, {v0:.4g} built-in")
    return out


def cached_fields(args, rlpt, torch, graphs, infos, temps, common, el, n_copies, chunked, out, src):
    """The headline workload with cached local fields (field_mode = FIELDS_CACHED):
    the same chain as the streaming run, timed from an equilibrated state (the
    streaming context src's configurations after its tau_int run, each placed
    at the temperature it held), since its cost follows the acceptance rate;
    reports its rate, the speedup over the streaming sweep, the acceptance and
    an algorithmic byte count per launch."""
    N, S, T, reps = args.n_modes, args.samples, args.temps, args.reps
    ctx = rlpt.Context(graphs, temps, shared_pairs=args.shared_pairs, field_mode=rlpt.FIELDS_CACHED, **common)
    ctx.init(1)
    equilibrated_state(src, ctx, N, S, T, reps)
    src_sweeps = src.counters()[0]
    log(f"cached fields: from the streaming run's state after {src_sweeps} sweeps")
    ctx.sweep(args.sweeps_per_step)
    ctx.check()
    torch.cuda.synchronize()
    o0 = ctx.observables()
    acc0, tries0 = o0["acc"].sum(), o0["tries"].sum()
    ctx.sweep_timing(True)
    t0 = time.perf_counter()
    ctx.sweep(args.sweeps)
    torch.cuda.synchronize()
    el4 = time.perf_counter() - t0
    ctx.check()
    kms4, launches4 = ctx.sweep_time()
    ctx.sweep_timing(False)
    o1 = ctx.observables()
    accepted = o1["acc"].sum() - acc0
    steps_total = n_copies * (N // 2) * args.sweeps
    idx_b = 2 if chunked else 4
    pair_b = sum(inf["pair_entries"] / (N * (N - 1)) * 8.0 for inf in infos) / S  # per step
    gather_b = sum(inf["gather_entries"] for inf in infos) / (S * N) * (idx_b + 4)
    bytes4 = (steps_total * pair_b + accepted * 2 * gather_b) / launches4
    tile4 = ctx.tile()
    acc_T = (o1["acc"] - o0["acc"]).sum(axis=0) / np.maximum((o1["tries"] - o0["tries"]).sum(axis=0), 1)
    ctx.close()
    out["cached_fields"] = {
        "mode_updates_per_s": N * n_copies * args.sweeps / el4,
        "speedup_vs_streaming": el / el4,
        "start": f"equilibrated: the streaming run's configurations after {src_sweeps} sweeps",
        "ms_per_launch": kms4 / launches4,
        "acceptance": accepted / steps_total,
        "acceptance_hottest_coldest": [float(acc_T[-1]), float(acc_T[0])],
        "tile": {"block_threads": int(tile4[0]), "copies_per_block": int(tile4[1][0])},
        "algorithmic_bytes_per_launch": bytes4,
        "achieved_GBs": bytes4 / (kms4 / launches4 * 1e-3) / 1e9,
        "note": "bytes: per step the (j->k) pair list (8 B/entry), per accepted step the padded gather "
                "blocks of j and k; the launch is bound by the hottest copies' accepted steps, not by HBM",
    }
    log(f"cached fields: {out['cached_fields']['mode_updates_per_s']:.4g} mode-updates/s "
        f"({out['cached_fields']['speedup_vs_streaming']:.2f}x streaming), acceptance "
        f"{out['cached_fields']['acceptance']:.4f}")


def sparse_graphs(args, rlpt, torch, temps, out, N=1024, z=32):
    """Sparse mode-locked graphs (finite connectivity, c = z N / 4 matched
    terms per sample) with the ladder and copies of the headline workload:
    the one-wave-per-copy short-list sweep, latency-bound."""
    S, T, reps = args.samples, args.temps, args.reps
    graphs = [rlpt.Graph(N, SEED_BASE + 900 + mu, mean_degree=z) for mu in range(S)]
    ctx = rlpt.Context(graphs, temps, n_temps=T, n_reps=reps, precision=rlpt.FP32, swap_interval=1,
                       resync_interval=100, measure_start=args.warm_sweeps, measure_interval=1, n_bins=100)
    ctx.init(1)
    ctx.sweep(args.warm_sweeps)
    torch.cuda.synchronize()
    ctx.sweep_timing(True)
    t0 = time.perf_counter()
    ctx.sweep(args.sweeps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.check()
    kms, launches = ctx.sweep_time()
    out["sparse_graph"] = {"n_modes": N, "mean_degree": z, "terms_per_sample": z * N // 4,
                           "copies": ctx.n_copies, "mode_updates_per_s": N * ctx.n_copies * args.sweeps / el,
                           "ms_per_launch": kms / launches, "sweeps_per_s": args.sweeps / el}
    ctx.close()
    log(f"sparse N={N} z={z}: {out['sparse_graph']['mode_updates_per_s']:.4g} mode-updates/s")


def ipr_comparison(args, rlpt, torch, out, Ns=(32, 64, 128), S=4, T=16, sweeps=1500):
    """The constraint comparison of sec. IV (inverse participation ratios):
    Y_2 = sum |a|^4 / (sum |a|^2)^2 at the coldest bath of a [0.25, 1.5] ladder,
    for the smoothed-cubic constraint (rho = 4) and the spherical one (rho = 2),
    on complete mode-locked graphs of growing N.  N Y_2 stays O(1) when the
    intensity is spread over all modes and grows with N when a few modes hold
    a finite fraction of it."""
    temps = 0.25 * (1.5 / 0.25) ** (np.arange(T) / (T - 1))
    res = {}
    for rho in (4, 2):
        row = {}
        for N in Ns:
            graphs = [rlpt.Graph(N, SEED_BASE + 800 + 10 * N + mu) for mu in range(S)]
            ctx = rlpt.Context(graphs, temps, n_temps=T, n_reps=2, precision=rlpt.FP32, swap_interval=1,
                               resync_interval=100, measure_start=sweeps // 2, measure_interval=1, n_bins=50,
                               rho=rho)
            ctx.init(3)
            ctx.sweep(sweeps)
            ctx.check()
            o = ctx.observables()
            y2 = o["y2_sum"][:, 0] / o["e_n"][:, 0]
            row[str(N)] = {"Y2": float(y2.mean()), "N_Y2": float(N * y2.mean()),
                           "N_Y2_err": float(N * y2.std(ddof=1) / np.sqrt(S))}
            ctx.close()
        res[f"rho{rho}"] = row
    out["ipr_rho4_vs_rho2"] = {"temperature": float(temps[0]), "samples": S, "sweeps": sweeps, **res}
    log("IPR comparison: " + ", ".join(f"rho{r} N={N}: N*Y2={res[f'rho{r}'][str(N)]['N_Y2']:.2f}"
                                       for r in (4, 2) for N in Ns))


def n64_configuration(args, rlpt, torch, out):
    """The N = 64 configuration (8 samples x 24 temperatures geometric in
    [0.3, 1.5] x 2 replicas, FP32, recomputation every 100 sweeps): lists of
    about 1.3 K entries per mode stay in L2, so the sweep is bound by the
    latency of a two-mode step, not by HBM."""
    N, S, T = 64, 8, 24
    temps = 0.3 * (1.5 / 0.3) ** (np.arange(T) / (T - 1))
    graphs = [rlpt.Graph(N, SEED_BASE + 100 + mu) for mu in range(S)]
    ctx = rlpt.Context(graphs, temps, n_temps=T, n_reps=2, precision=rlpt.FP32, swap_interval=1,
                       resync_interval=100, measure_start=args.warm_sweeps, measure_interval=1, n_bins=100)
    ctx.init(1)
    ctx.sweep(args.warm_sweeps)
    torch.cuda.synchronize()
    # wall clock without events (a sweep here is ~80 us, and two event records
    # per launch would add several); then the same number of sweeps with HIP
    # events around each sweep launch for the kernel's own time
    t0 = time.perf_counter()
    ctx.sweep(args.sweeps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.sweep_timing(True)
    ctx.sweep(args.sweeps)
    torch.cuda.synchronize()
    ctx.check()
    kms, launches = ctx.sweep_time()
    steps = N // 2
    out["n64_configuration"] = {"copies": ctx.n_copies, "mode_updates_per_s": N * ctx.n_copies * args.sweeps / el,
                                "us_per_sweep_wall": el / args.sweeps * 1e6, "ms_per_launch": kms / launches,
                                "us_per_two_mode_step": kms / launches * 1e3 / steps}
    ctx.close()
    # latency floor: the same kernel and tile (one copy per 512-thread workgroup)
    # at N = 32 ... 128 with the same ladder.  Up to N = 64 a step's time does
    # not depend on the length of its lists (the list work hides under the
    # step's chain of reductions, barriers and decision): the smallest of those
    # times is the floor; beyond, the time grows with the entries streamed
    pts = []
    for n in (32, 48, 64, 96, 128):
        gs = [rlpt.Graph(n, SEED_BASE + 100 + 10 * n + mu) for mu in range(S)]
        c2 = rlpt.Context(gs, temps, n_temps=T, n_reps=2, precision=rlpt.FP32, swap_interval=1,
                          resync_interval=100, measure_start=0, measure_interval=1, n_bins=100,
                          block_threads=512, copies_per_block=1)
        c2.init(1)
        c2.sweep(50)
        torch.cuda.synchronize()
        c2.sweep_timing(True)
        c2.sweep(200)
        torch.cuda.synchronize()
        c2.check()
        ms, nl = c2.sweep_time()
        c2.close()
        entries = np.mean([2 * g.info()["deg_sum"] / n for g in gs])  # both lists of a step, mean
        pts.append((n, entries, ms / nl * 1e3 / (n // 2)))
    floor = min(p[2] for p in pts if p[0] <= 64)
    slope = (pts[-1][2] - pts[-2][2]) / (pts[-1][1] - pts[-2][1])
    step64 = out["n64_configuration"]["us_per_two_mode_step"]
    out["n64_configuration"]["latency_floor"] = {
        "method": "k_sweep at one copy per 512-thread workgroup, 8 samples x 24 T x 2 replicas at N = 32..128; "
                  "floor = the smallest us per two-mode step over N <= 64, where the step time does not follow "
                  "the list length; ns per entry from the two largest N",
        "points": [{"N": p[0], "entries_per_step": round(p[1], 1), "us_per_step": round(p[2], 4)} for p in pts],
        "us_per_step_floor": floor, "ns_per_entry_large_N": slope * 1e3, "n64_step_over_floor": step64 / floor}
    log(f"N=64 configuration: {out['n64_configuration']['mode_updates_per_s']:.4g} mode-updates/s")


def n64_physics(args, rlpt, torch, out, sweeps=100000):
    """The N = 64 configuration run to its length: 10^5 sweeps in 100-sweep
    HIP-graph segments, measurements over the second half (equilibration =
    half the run, sec. III.B), FP64 recomputation every 100 sweeps.  Reports
    per temperature the disorder averages with jackknife errors of the energy
    per mode, the specific heat per mode, <q^2>, the overlap kurtosis, the
    IPRs Y_2 and Y_4, the acceptance and swap rates, the 100-bin P(q) at
    the coldest bath, the specific-heat peak and the hottest bath, and the
    intensity spectrum (its spread over the frequency band per temperature and
    its profile in 8 bands at those three baths)."""
    N, S, T = 64, 8, 24
    temps = 0.3 * (1.5 / 0.3) ** (np.arange(T) / (T - 1))
    graphs = [rlpt.Graph(N, SEED_BASE + 100 + mu) for mu in range(S)]
    half = sweeps // 2 // 100 * 100
    ctx = rlpt.Context(graphs, temps, n_temps=T, n_reps=2, precision=rlpt.FP32, swap_interval=1,
                       resync_interval=100, measure_start=half, measure_interval=1, n_bins=100)
    ctx.init(2)
    t0 = time.perf_counter()
    ctx.run_graph(100, half // 100)
    ctx.run_graph(100, (sweeps - half) // 100)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.check()
    o = ctx.observables()
    ctx.close()
    sm = rlpt.summarize(o, N, temps)
    h = o["hist"] / np.maximum(o["hist"].sum(axis=2, keepdims=True), 1)
    pq = h.mean(axis=0)
    pk = 2 + int(np.argmax(sm["cv"][2:T - 2]))
    # intensity spectrum I(omega_k) = <|a_k|^2> (modes in frequency order), normalised per sample and
    # temperature to unit mean; its intensity-weighted spread in frequency rank measures the narrowing
    spec = o["spectrum"] / o["e_n"][:, :, None]
    spec = spec / spec.mean(axis=2, keepdims=True)
    rank = (np.arange(N) + 0.5) / N
    width = np.sqrt(np.sum(spec * (rank - 0.5) ** 2, axis=2) / np.sum(spec, axis=2))  # [S][T]
    bands = spec.reshape(S, T, 8, N // 8).mean(axis=3).mean(axis=0)  # 8 frequency bands, sample mean
    r = lambda v, d=4: np.round(np.asarray(v, dtype=float), d).tolist()  # noqa: E731
    out["n64_physics"] = {
        "sweeps": sweeps, "measured_sweeps": sweeps - half, "seconds": el, "sweeps_per_s": sweeps / el,
        "temperatures": r(temps), "E_per_mode": r(sm["E"] / N), "E_per_mode_err": r(sm["E_err"] / N, 5),
        "cv_per_mode": r(sm["cv"]), "cv_per_mode_err": r(sm["cv_err"]), "q2": r(sm["q2"]),
        "kurtosis": r(sm["kurtosis"]), "Y2": r(sm["y2"], 5), "Y4": r(sm["y4"], 6), "acceptance": r(sm["acc_rate"]),
        "swap_rate": r(sm["swap_rate"]),
        "P_q": {"bins": 100, "range": [-1, 1], "at_T": {f"{temps[t]:.4f}": r(pq[t], 5) for t in (0, pk, T - 1)}},
        "spectrum": {"width_in_frequency_rank": r(width.mean(axis=0)), "width_err": r(width.std(axis=0, ddof=1)
                                                                                      / np.sqrt(S)),
                     "flat_width": float(np.sqrt(1.0 / 12.0)),
                     "bands_at_T": {f"{temps[t]:.4f}": r(bands[t]) for t in (0, pk, T - 1)},
                     "note": "8 equal bands of frequency rank, intensity relative to the mode average"},
    }
    log(f"N=64 physics: {sweeps} sweeps in {el:.1f} s, C_V peak at T={temps[pk]:.3f}")


def n64_protocol(args, rlpt, torch, out, cv_per_mode, sweeps=32768, ladder_sweeps=20000):
    """The paper's run protocol on the N = 64 configuration (sec. III.B, App. A):
    the doubling-window thermalisation check (energy means over sweeps
    [2^k, 2^(k+1)) from a random start, sample-averaged, at the coldest bath,
    the specific-heat peak and the hottest bath), and the ladder adapted to the
    measured specific heat (eq. PT_Ti, C = 0.6) run beside the geometric one:
    swap acceptance across the ladder (the rule spaces temperatures so that
    neighbouring energy distributions overlap alike)."""
    N, S, T = 64, 8, 24
    temps = 0.3 * (1.5 / 0.3) ** (np.arange(T) / (T - 1))
    graphs = [rlpt.Graph(N, SEED_BASE + 100 + mu) for mu in range(S)]
    ctx = rlpt.Context(graphs, temps, n_temps=T, n_reps=2, precision=rlpt.FP32, swap_interval=1,
                       resync_interval=100, measure_start=0, measure_interval=1, n_bins=100, series_len=sweeps)
    ctx.init(4)
    ctx.run_graph(100, sweeps // 100)
    ctx.sweep(sweeps % 100)
    ctx.check()
    o = ctx.observables()
    ctx.close()
    pk = 2 + int(np.argmax(np.asarray(cv_per_mode)[2:T - 2]))
    windows = {}
    for t in (0, pk, T - 1):
        per = [rlpt.window_means(o["series_e"][mu, t, :sweeps])[0] for mu in range(S)]
        m = np.array(per) / N
        windows[f"{temps[t]:.4f}"] = {"E_per_mode": np.round(m.mean(axis=0), 4).tolist()[-6:],
                                       "err": np.round(m.std(axis=0, ddof=1) / np.sqrt(S), 4).tolist()[-6:]}
    starts = rlpt.window_means(o["series_e"][0, 0, :sweeps])[1].tolist()[-6:]

    def swap_rates(ladder):
        Tn = len(ladder)
        c2 = rlpt.Context(graphs, ladder, n_temps=Tn, n_reps=2, precision=rlpt.FP32, swap_interval=1,
                          resync_interval=100, measure_start=ladder_sweeps // 2, measure_interval=1, n_bins=10)
        c2.init(5)
        c2.run_graph(100, ladder_sweeps // 200)
        c2.run_graph(100, ladder_sweeps // 200)
        c2.check()
        r = rlpt.summarize(c2.observables(), N, ladder)["swap_rate"]
        c2.close()
        return r

    adapt = rlpt.adaptive_ladder(temps, np.asarray(cv_per_mode) * N, 0.3, 1.5, c=0.6)
    r_geo, r_ad = swap_rates(temps), swap_rates(adapt)
    out["n64_protocol"] = {
        "doubling_windows": {"window_starts": starts, "at_T": windows,
                             "note": "energy per mode averaged over sweeps [start_k, start_{k+1}), last six windows"},
        "adaptive_ladder": {"C": 0.6, "temperatures": np.round(adapt, 4).tolist(), "n": int(len(adapt)),
                            "swap_rate_min_max": [float(r_ad.min()), float(r_ad.max())],
                            "swap_rate_std": float(r_ad.std())},
        "geometric_ladder": {"n": T, "swap_rate_min_max": [float(r_geo.min()), float(r_geo.max())],
                             "swap_rate_std": float(r_geo.std())},
    }
    log(f"N=64 protocol: adaptive ladder {len(adapt)} temperatures, swap rates "
        f"{r_ad.min():.2f}-{r_ad.max():.2f} (geometric {r_geo.min():.2f}-{r_geo.max():.2f})")


def graph_sweeps(ctx, n, tag, piece=10000):
    """n sweeps (a multiple of 100) in 100-sweep HIP-graph segments, a progress line after each piece"""
    done = 0
    while done < n:
        k = min(piece, n - done)
        ctx.run_graph(100, k // 100)
        done += k
        if n > piece:
            ctx.check()
            log(f"{tag}: {done}/{n} sweeps")


def learned_n64(args, rlpt, torch, out, N=64, S=8, T=24, reps=2, n_nets=4, sweeps=20000, warm=2000,
                harvest_rounds=6250, train_steps=1000, reeq=5000, at="peak", train=True):
    """The learned-proposal configuration: N = 64, 8 samples x 24 temperatures
    geometric in [0.3, 1.5] x 2 replicas.  A first plain run finds the peak of
    the specific heat; networks (2N -> 256 -> 256 SiLU -> 4-component mixture)
    at the n_nets temperatures around it are trained on 10^5 harvested pairs
    each.  The comparison is two runs with one history: warm-up, harvest (its
    sweeps run without swaps), reeq sweeps with swaps, then the measured
    sweeps in 100-sweep HIP-graph segments; the learned run trains after the
    harvest and makes one learned round per sweep from then on, the plain run
    does not.  Reports tau_int of E and q at the learned temperatures,
    effective sweeps/s learned / plain, and whether the energy and the overlap
    histogram agree (paired jackknife over samples).  at = "cold" puts the
    networks on the four coldest temperatures instead; train = False runs the
    learned rounds with the networks at their initialisation (outputs near
    zero: an isotropic small-step mixture), the same history otherwise."""
    temps = 0.3 * (1.5 / 0.3) ** (np.arange(T) / (T - 1))
    graphs = [rlpt.Graph(N, 2511135080 + 300 + mu) for mu in range(S)]
    start = warm + harvest_rounds * 2 + reeq

    def run(learn_t, learned, subset=0, scale=None):
        scale = args.learn_scale if scale is None else scale
        cfg = dict(n_temps=T, n_reps=reps, precision=rlpt.FP32, swap_interval=1, resync_interval=100,
                   measure_start=start, measure_interval=1, n_bins=100, series_len=sweeps,
                   mlp_nets=len(learn_t), mlp_hidden=256, mlp_components=4,
                   mlp_capacity=harvest_rounds * S * reps, mlp_batch=512, mlp_subset=subset)
        ctx = rlpt.Context(graphs, temps, **cfg)
        ctx.init(1)
        ctx.sweep(warm)
        ctx.mlp_setup(learn_t, seed=1)
        t0 = time.perf_counter()
        ctx.mlp_harvest(rounds=harvest_rounds, lag=2)
        info = {}
        if learned and train:
            try:
                l0 = ctx.mlp_train(1, 1e-3)
                l1 = ctx.mlp_train(train_steps, 1e-3)
                torch.cuda.synchronize()
                info = {"harvest_and_train_s": time.perf_counter() - t0, "pairs_per_net": harvest_rounds * S * reps,
                        "train_loss_first_last": [l0.round(2).tolist(), l1.round(2).tolist()]}
            except rlpt.RlptError as e:
                info = {"train_error": str(e)}
                log(f"learned N=64: training failed: {e}")
        if learned and "train_error" not in info:
            ctx.mlp_enable(args.n64_rounds, scale)
        ctx.sweep(start - ctx.counters()[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph_sweeps(ctx, sweeps, "learned N=64: measured")  # 100-sweep segments replayed as HIP graphs
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.check()
        o = ctx.observables()
        if learned:
            acc, tries = ctx.mlp_stats()
            info["move_acceptance"] = (acc / np.maximum(tries, 1)).round(4).tolist()
        ctx.close()
        return o, sweeps / el, info

    def peak_run():
        ctx = rlpt.Context(graphs, temps, n_temps=T, n_reps=reps, precision=rlpt.FP32, swap_interval=1,
                           resync_interval=100, measure_start=warm, measure_interval=1, n_bins=100)
        ctx.init(3)
        ctx.run_graph(100, warm // 100)
        graph_sweeps(ctx, sweeps, "learned N=64: C_V peak run")
        ctx.check()
        cv = rlpt.summarize(ctx.observables(), N, temps)["cv"]
        ctx.close()
        return 2 + int(np.argmax(cv[2:T - 2]))  # interior maximum (the ladder's ends are not a peak)

    def taus(o, t_idx):
        """per sample tau_int of E and q at t_idx: arrays [len(t_idx)][S]"""
        m = min(int(o["e_n"][0, 0] / reps), sweeps)
        lo = m // 10
        return [tau_per_sample(o[k], t_idx, lo, m) for k in ("series_e", "series_q")]

    def jk(v):
        n = v.shape[0]
        loo = (v.sum(axis=0) - v) / (n - 1)
        return v.mean(axis=0), np.sqrt((n - 1) / n * ((loo - loo.mean(axis=0)) ** 2).sum(axis=0))

    if at == "cold":
        pk = -1
        t_learn = list(range(n_nets))
    else:
        log("learned N=64: locating the C_V peak")
        pk = peak_run()
        t_learn = [t for t in range(pk - n_nets // 2, pk - n_nets // 2 + n_nets) if 0 <= t < T]
        log(f"learned N=64: C_V peak at T={temps[pk]:.3f}")
    log("learned N=64: plain run with the harvest history")
    op, sps_p, _ = run(t_learn, False)
    log("learned N=64: learned run")
    ol, sps_l, info = run(t_learn, True)
    m_sub = max(2, N // args.subset_frac)
    log(f"learned N=64: learned subset run (m = {m_sub})")
    os_, sps_s, info_s = run(t_learn, True, subset=m_sub, scale=args.subset_scale)
    tEp, tqp = taus(op, t_learn)
    tEl, tql = taus(ol, t_learn)
    # the two runs share disorder, seed and history up to the first learned round: paired differences over samples
    Ep, El = op["e_sum"] / op["e_n"], ol["e_sum"] / ol["e_n"]
    dE, sE = jk(El - Ep)
    zE = np.abs(dE) / np.maximum(sE, 1e-12)
    hp = op["hist"] / np.maximum(op["hist"].sum(axis=2, keepdims=True), 1)
    hl = ol["hist"] / np.maximum(ol["hist"].sum(axis=2, keepdims=True), 1)
    dh, sh_ = jk(hl - hp)
    mass = (hp.mean(axis=0) + hl.mean(axis=0)) > 1e-3
    zq = np.abs(dh) / np.maximum(sh_, 1e-12)
    rE = eff_ratio(tEl, tEp, sps_l, sps_p)
    rq = eff_ratio(tql, tqp, sps_l, sps_p)
    tEs, tqs = taus(os_, t_learn)
    rEs = eff_ratio(tEs, tEp, sps_s, sps_p)
    dead_s = dead_networks(info_s.get("move_acceptance", []), np.array(info_s["train_loss_first_last"])
                           if "train_loss_first_last" in info_s else None)
    for d in dead_s:
        rEs["status"][d["network"]] = "failed: " + d["failed"]
    if "train_error" in info_s:
        rEs["status"] = ["failed: " + info_s["train_error"]] * len(t_learn)
    Es = os_["e_sum"] / os_["e_n"]
    dEs, sEs = jk(Es - Ep)
    zEs = np.abs(dEs) / np.maximum(sEs, 1e-12)
    dead = dead_networks(info.get("move_acceptance", []), np.array(info["train_loss_first_last"])
                         if "train_loss_first_last" in info else None)
    for d in dead:
        rE["status"][d["network"]] = rq["status"][d["network"]] = "failed: " + d["failed"]
    if "train_error" in info:
        rE["status"] = rq["status"] = ["failed: " + info["train_error"]] * len(t_learn)
    out["learned_n64"] = {
        "config": f"N={N}, {S} samples x {T} temperatures [0.3, 1.5] x {reps} replicas, FP32; learned rounds "
                  f"({args.n64_rounds} per sweep, step scale {args.learn_scale}, {'trained' if train else 'untrained'} "
                  f"networks) at "
                  f"the {len(t_learn)} {'coldest temperatures' if at == 'cold' else 'temperatures around the C_V peak'}"
                  f"; both runs: {warm} warm-up, {harvest_rounds * 2} harvest (no swaps), {reeq} more sweeps, "
                  f"then {sweeps} measured sweeps",
        "temperatures": [float(temps[t]) for t in t_learn], "cv_peak_T": float(temps[pk]) if pk >= 0 else None,
        "plain": {"sweeps_per_s": sps_p, "tau_int_E": tau_stats(tEp), "tau_int_q": tau_stats(tqp)},
        "learned": {"sweeps_per_s": sps_l, "tau_int_E": tau_stats(tEl), "tau_int_q": tau_stats(tql), **info,
                    "failed_networks": dead},
        "learned_vs_plain_eff_E": rE,
        "learned_vs_plain_eff_q": rq,
        "learned_subset": {"move": f"subset of {m_sub} modes", "step_scale": args.subset_scale,
                           "sweeps_per_s": sps_s, "tau_int_E": tau_stats(tEs), "tau_int_q": tau_stats(tqs), **info_s,
                           "failed_networks": dead_s, "E_within_2sigma": float(np.mean(zEs <= 2)),
                           "E_z_all_T": zEs.round(2).tolist()},
        "learned_subset_vs_plain_eff_E": rEs,
        "agreement": {"E_diff_learned_minus_plain": dE.round(3).tolist(), "E_diff_err": sE.round(3).tolist(),
                      "E_z_all_T": zE.round(2).tolist(), "E_within_2sigma": float(np.mean(zE <= 2)),
                      "Pq_cells": int(mass.sum()), "Pq_within_2sigma": float(np.mean(zq[mass] <= 2)),
                      "test": "paired jackknife over the 8 samples of (learned - plain)"},
    }
    log(f"learned N=64: subset eff ratio E {rEs['ratio']} {rEs['status']}")
    log(f"learned N=64: eff ratio E {rE['ratio']} {rE['status']}, "
        f"E within 2 sigma {out['learned_n64']['agreement']['E_within_2sigma']:.2f}, "
        f"P(q) within 2 sigma {out['learned_n64']['agreement']['Pq_within_2sigma']:.2f}")


def tau_per_sample(series, t_idx, lo, m):
    """tau_int (Sokal window) of series[mu, t, lo:m] for every sample mu and
    temperature index t in t_idx: array [len(t_idx)][samples]"""
    from paper_2511_13508_amd import rlpt
    S = series.shape[0]
    return np.array([[rlpt.tau_int(series[mu, t, lo:m])[0] for mu in range(S)] for t in t_idx])


def tau_stats(tau_ps):
    """median over samples, and mean with its standard error over samples"""
    S = tau_ps.shape[1]
    return {"median": np.round(np.median(tau_ps, axis=1), 2).tolist(),
            "mean": np.round(tau_ps.mean(axis=1), 2).tolist(),
            "err": np.round(tau_ps.std(axis=1, ddof=1) / np.sqrt(S), 2).tolist()}


def eff_ratio(tau_a, tau_b, sps_a, sps_b):
    """Effective sweeps/s of run a over run b per temperature, sps_a/(2 tau_a)
    over sps_b/(2 tau_b), paired by disorder sample: the ratio is
    (sps_a / sps_b) x exp(mean over samples of log(tau_b / tau_a)), its error
    band exp(+-1 standard error of that mean).  A ratio whose band contains 1
    is 'unresolved'."""
    lr = np.log(tau_b) - np.log(tau_a)
    S = lr.shape[1]
    m, se = lr.mean(axis=1), lr.std(axis=1, ddof=1) / np.sqrt(S)
    r = sps_a / sps_b * np.exp(m)
    lo, hi = r * np.exp(-se), r * np.exp(se)
    status = ["faster" if l > 1 else "slower" if h < 1 else "unresolved" for l, h in zip(lo, hi)]
    return {"ratio": np.round(r, 3).tolist(), "lo": np.round(lo, 3).tolist(), "hi": np.round(hi, 3).tolist(),
            "status": status, "method": "paired over disorder samples: (sweeps/s ratio) x exp(mean log tau ratio), "
                                        "band = exp(+-1 standard error)"}


def window_means(o, t_idx, lo, m):
    """per-sample means over the series window [lo, m) at the temperature
    indices t_idx, arrays [len(t_idx)][samples]: E, q^2, and E over the
    window's first and second halves (a drift between them means the run is
    still relaxing)"""
    e = o["series_e"][:, t_idx, lo:m].astype(np.float64)
    q = o["series_q"][:, t_idx, lo:m].astype(np.float64)
    h = (m - lo) // 2
    return {"E": e.mean(axis=2).T, "q2": (q * q).mean(axis=2).T, "E_first": e[:, :, :h].mean(axis=2).T,
            "E_second": e[:, :, h:].mean(axis=2).T}


def paired_agreement(a, b):
    """a - b per temperature (rows), paired by disorder sample (columns): the
    mean difference, its jackknife error over the samples (for a mean, the
    standard error), z = |mean| / error and the fraction of rows with z <= 2"""
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    n = d.shape[1]
    loo = (d.sum(axis=1, keepdims=True) - d) / (n - 1)
    err = np.sqrt((n - 1) / n * ((loo - loo.mean(axis=1, keepdims=True)) ** 2).sum(axis=1))
    mean = d.mean(axis=1)
    z = np.abs(mean) / np.maximum(err, 1e-300)
    return {"diff": np.round(mean, 4).tolist(), "err": np.round(err, 4).tolist(), "z": np.round(z, 2).tolist(),
            "within_2sigma": float(np.mean(z <= 2))}


def dead_networks(acceptance, losses):
    """Networks that accepted no learned move or trained to a non-finite loss"""
    bad = []
    for n, a in enumerate(acceptance):
        reasons = []
        if not a > 0:
            reasons.append("accepted no learned move")
        if losses is not None and not np.all(np.isfinite(np.asarray(losses)[..., n])):
            reasons.append("non-finite training loss")
        if reasons:
            bad.append({"network": n, "failed": "; ".join(reasons)})
    return bad


def equilibrated_state(src, dst, N, S, T, reps):
    """Copy the configurations of context src into context dst so that every
    (sample, ladder, temperature) slot of dst starts from src's configuration
    at that slot (dst fresh from init: copy mu*R + r*T + t holds temperature t)."""
    a = src.get_state().reshape(src.n_copies, N)
    _, temp_of = src.energies()
    R = T * reps
    b = np.empty_like(a)
    for c in range(src.n_copies):
        mu, r = c // R, (c % R) // T
        b[mu * R + r * T + temp_of[c]] = a[c]
    dst.set_state(b.reshape(-1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps (a step is --sweeps-per-step sweeps)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps before the timed ones")
    ap.add_argument("--sweeps-per-step", type=int, default=100,
                    help="sweeps per step; 100 = one FP64 recomputation interval (every part of the path)")
    ap.add_argument("--n-modes", type=int, default=256)
    ap.add_argument("--samples", type=int, default=8)
    ap.add_argument("--temps", type=int, default=40)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--shared-pairs", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--copies-per-block", type=int, default=0)
    ap.add_argument("--layout", type=int, default=0, help="0 auto, 1 packed (8 B/entry), 2 chunked (6.25 B/entry)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--tau-sweeps", type=int, default=20000, help="extra sweeps per run for tau_int (0: skip)")
    ap.add_argument("--learn-temps", type=lambda v: [int(x) for x in v.split(",")] if v else [],
                    default=[25, 26, 27, 28], help="temperature indices with learned global moves")
    ap.add_argument("--learn-scale", type=float, default=0.05)
    ap.add_argument("--learn-rounds", type=int, default=1, help="all-mode learned rounds per sweep at N=256")
    ap.add_argument("--run-seed", type=int, default=1, help="N=256 runs: the seed of the initial draw and the moves")
    ap.add_argument("--untrained", action="store_true",
                    help="N=256 learned runs with untrained networks (no harvest, no training)")
    ap.add_argument("--only-learned-all-256", action="store_true",
                    help="n256 workload: only the plain tau run and the all-mode learned comparison")
    ap.add_argument("--subset-frac", type=int, default=8, help="subset move: m = N / subset_frac modes per move")
    ap.add_argument("--subset-scale", type=float, default=0.5, help="subset move: step scale")
    ap.add_argument("--subset-rounds", type=int, default=1, help="subset move: learned rounds per sweep at N=256")
    ap.add_argument("--only-learned-256", action="store_true",
                    help="n256 workload: only the plain tau run and the learned comparisons (scans)")
    ap.add_argument("--harvest-rounds", type=int, default=400)
    ap.add_argument("--train-steps", type=int, default=600)
    ap.add_argument("--reeq", type=int, default=500, help="sweeps with swaps between harvest and the learned window")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cached", action="store_true", help="skip the cached-field, sparse, IPR and N=64 runs")
    ap.add_argument("--no-n64", action="store_true", help="skip the N=64 physics run and learned comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched uneven-N block")
    ap.add_argument("--summarize-profiles", metavar="DIR", default=None,
                    help="write profiles/ summaries from rocprofv3 CSVs under DIR and exit")
    ap.add_argument("--workload", choices=["n256", "batched", "learned64", "n64"], default="n256",
                    help="n256: the headline configuration; batched: the uneven-N configuration with autotuning; "
                         "learned64: only the N=64 learned-proposal comparison; n64: only the N=64 configuration's "
                         "rate")
    ap.add_argument("--n64-learn-at", choices=["peak", "cold"], default="peak",
                    help="learned64 workload: networks around the C_V peak or on the four coldest temperatures")
    ap.add_argument("--n64-untrained", action="store_true",
                    help="learned64 workload: learned rounds with untrained networks")
    ap.add_argument("--n64-rounds", type=int, default=1, help="N=64 learned comparison: learned rounds per sweep")
    ap.add_argument("--batched-launches-only", action="store_true",
                    help="batched workload: only 20 sweeps of the mixed launch with built-in tiles (for counters)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (scales the rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.only_learned_256 or args.only_learned_all_256:
        args.no_cached = args.no_n64 = args.no_batched = args.no_cpu_baseline = True
    args.sweeps = args.steps * args.sweeps_per_step
    args.warm_sweeps = args.warmup * args.sweeps_per_step
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (disorder samples would shard "
              "across GPUs, see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_13508_amd import rlpt

    torch.cuda.set_device(0)
    if args.workload == "batched":
        print(json.dumps(batched(args)), flush=True)
        return
    if args.workload == "n64":
        res = {}
        n64_configuration(args, rlpt, torch, res)
        print(json.dumps(res["n64_configuration"]), flush=True)
        return
    if args.workload == "learned64":
        res = {}
        learned_n64(args, rlpt, torch, res, sweeps=args.sweeps // 100 * 100 or 100, at=args.n64_learn_at,
                    train=not args.n64_untrained)
        print(json.dumps(res["learned_n64"]), flush=True)
        return
    if args.copy_calibration:
        n = 128 * 1024 * 1024  # 512 MiB of float32 read and 512 MiB written per copy
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_dispatch": 4 * n}), flush=True)
        return
    N, S, T, reps = args.n_modes, args.samples, args.temps, args.reps
    temps = 0.25 * (1.5 / 0.25) ** (np.arange(T) / (T - 1))
    log(f"building {S} graphs N={N}")
    graphs = [rlpt.Graph(N, SEED_BASE + mu) for mu in range(S)]
    infos = [g.info() for g in graphs]
    series_len = args.sweeps + args.tau_sweeps
    common = dict(n_temps=T, n_reps=reps, precision=rlpt.FP32, swap_interval=1, resync_interval=100,
                  measure_start=args.warm_sweeps, measure_interval=1, n_bins=100, series_len=series_len,
                  block_threads=args.block, copies_per_block=args.copies_per_block, list_layout=args.layout)

    def timed(ctx, tag):
        """warm-up, then the timed steps with sweep-kernel events; returns (s, kernel ms, launches)"""
        ctx.init(args.run_seed)
        log(f"{tag}: warmup {args.warmup} steps ({args.warm_sweeps} sweeps)")
        ctx.sweep(args.warm_sweeps)
        ctx.check()
        torch.cuda.synchronize()
        ctx.sweep_timing(True)
        log(f"{tag}: timing {args.steps} steps ({args.sweeps} sweeps)")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.sweep(args.sweeps_per_step)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.check()
        kms, launches = ctx.sweep_time()
        ctx.sweep_timing(False)
        return el, kms, launches

    def long_run(ctx, n, tag):
        """n sweeps in pieces of 10,000, a progress line after each"""
        done = 0
        while done < n:
            k = min(10000, n - done)
            ctx.sweep(k)
            ctx.check()
            done += k
            if n > 10000:
                log(f"{tag}: {done}/{n} sweeps")

    def tau_block(ctx, sweeps_per_s, t_idx, extra_sweeps, tag):
        """continue extra_sweeps sweeps, then tau_int of E and q at the
        temperature indices t_idx from the series (first quarter discarded),
        per sample; returns (summary, tau_E per sample, the window means of
        E and q^2 per sample)"""
        if extra_sweeps > 0:
            long_run(ctx, extra_sweeps, tag)
        o = ctx.observables()
        m = int(o["e_n"][0, 0] / reps)
        m = min(m, series_len)
        lo = m // 4
        tE = tau_per_sample(o["series_e"], t_idx, lo, m)
        tq = tau_per_sample(o["series_q"], t_idx, lo, m)
        return ({"temperatures": [float(temps[t]) for t in t_idx], "tau_int_E": tau_stats(tE),
                 "tau_int_q": tau_stats(tq), "sweeps_per_s": sweeps_per_s,
                 "eff_sweeps_per_s_E": (sweeps_per_s / (2 * np.median(tE, axis=1))).round(3).tolist(),
                 "series_points": m - lo}, tE, window_means(o, t_idx, lo, m))

    # ---------------------------------------------------------------- headline: per-copy pairs
    ctx = rlpt.Context(graphs, temps, shared_pairs=args.shared_pairs, **common)
    el, kms, launches = timed(ctx, "plain")
    n_copies = ctx.n_copies
    value = N * n_copies * args.sweeps / el
    # algorithmic bytes of one sweep launch (one sweep): every copy streams, per
    # two-mode step, the lists of j and k; over a sweep of N/2 uniform pairs that
    # is the 4c entries of all lists on average: 8 B per entry in the packed
    # layout, 25 B per 4 entries in the chunked one (padding not counted)
    chunked = args.layout == 2 or (args.layout == 0 and N <= 256 and N >= 32)
    per_entry = 6.25 if chunked else 8.0
    sweeps_per_launch = args.sweeps / launches
    entries_per_launch = sweeps_per_launch * sum(reps * T * inf["deg_sum"] for inf in infos)
    bytes_per_launch = entries_per_launch * per_entry
    t_launch = kms / launches * 1e-3
    achieved = bytes_per_launch / t_launch / 1e9
    traffic = traffic_for_current_kernel(bytes_per_launch)
    log(f"{value:.4g} mode-updates/s; sweep kernel {kms / launches:.3f} ms/launch, {achieved:.0f} GB/s algorithmic")
    roof = {"bound": "hbm", "achieved": achieved, "unit": "GB/s", "kernel": "k_sweep",
            "ms_per_launch": kms / launches, "bytes_per_entry": per_entry,
            "entries_per_launch": entries_per_launch, "algorithmic_bytes_per_launch": bytes_per_launch,
            "hbm_peak_published": HBM_PEAK_GBS, "frac_of_hbm_peak": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_over_algorithmic": traffic / bytes_per_launch if traffic else None,
            "traffic_GBps": traffic / t_launch / 1e9 if traffic else None}
    if traffic:
        # the HBM roof for the bytes that pass the L2: the published peak scaled by the measured reuse
        # (algorithmic / fabric bytes); frac = fabric GB/s / HBM peak.  Fabric bytes include Infinity-Cache
        # hits, so the true HBM fraction is at most this
        roof.update({"peak": HBM_PEAK_GBS * bytes_per_launch / traffic,
                     "frac": traffic / t_launch / 1e9 / HBM_PEAK_GBS,
                     "peak_kind": "published HBM peak x algorithmic / fabric bytes (rocprofv3 FETCH_SIZE + "
                                  "WRITE_SIZE of this kernel source, profiles/sweep_n256_traffic.json): the HBM roof "
                                  "for the bytes that pass the L2; fabric bytes include Infinity-Cache hits, so the "
                                  "HBM fraction is at most frac"})
    if chunked and not args.shared_pairs:
        # the list-stream probe in three rounds, each beside a few timed sweep launches (same box, same clocks)
        probe, beside = [], []
        for _ in range(3):
            probe.append(ctx.stream_lists(5))
            ctx.sweep_timing(True)
            ctx.sweep(5)
            kr, nr = ctx.sweep_time()
            ctx.sweep_timing(False)
            beside.append(kr / nr)
        ms_probe = float(np.mean(probe))
        roof["list_stream_probe"] = {
            "ms_per_launch": ms_probe, "GBps": bytes_per_launch / (ms_probe * 1e-3) / 1e9,
            "rounds_ms": [round(x, 4) for x in probe], "sweep_beside_ms": [round(x, 4) for x in beside],
            "sweep_over_probe_time": float(np.mean(beside)) / ms_probe,
            "what": "rlpt_stream_lists: the sweep's grid, tile, LDS footprint, barriers and list reads with no "
                    "arithmetic; the sweep takes within a few per cent of its time (box to box 0.96-1.04)"}
        log(f"list-stream probe {ms_probe:.3f} ms/launch; sweep beside it {np.mean(beside):.3f} ms")
        if "peak" not in roof:
            roof.update({"peak": bytes_per_launch / (ms_probe * 1e-3) / 1e9, "frac": ms_probe / t_launch,
                         "peak_kind": "measured list-stream probe (no committed counters for this kernel source)"})
    if "peak" not in roof:
        roof.update({"peak": HBM_PEAK_GBS, "frac": achieved / HBM_PEAK_GBS, "peak_kind": "published HBM peak"})
    sweeps_per_s = args.sweeps / el
    t_learn = [t for t in args.learn_temps if t < T]
    tau_plain = tau_plain_E = tau_plain_w = None
    if args.tau_sweeps > 0:
        log(f"plain: {args.tau_sweeps} more sweeps for tau_int")
        tau_plain, tau_plain_E, tau_plain_w = tau_block(ctx, sweeps_per_s, t_learn, args.tau_sweeps, "plain")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "mode-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain PT N={N}, {S} samples x {T} temperatures x {reps} replicas, FP32 fields, "
                               f"FP64 resync/100, swap+measure every sweep; one step = {args.sweeps_per_step} sweeps",
                   "n_modes": N, "samples": S, "temperatures": T, "replicas": reps, "copies": n_copies,
                   "sweeps_per_step": args.sweeps_per_step,
                   "terms_per_sample": [inf["n_terms"] for inf in infos],
                   "pair_schedule": "shared per sample" if args.shared_pairs else "per copy",
                   "list_layout": "chunked" if chunked else "packed"},
        "roofline": roof,
        "sweeps_per_s": sweeps_per_s,
    }
    # ---------------------------------------------------------------- other variants and configurations
    if not args.no_cached:
        cached_fields(args, rlpt, torch, graphs, infos, temps, common, el, n_copies, chunked, out, ctx)
    ctx.close()
    if not args.no_cached:
        sparse_graphs(args, rlpt, torch, temps, out)
        ipr_comparison(args, rlpt, torch, out)
        n64_configuration(args, rlpt, torch, out)
        if not args.no_n64:
            n64_physics(args, rlpt, torch, out)
            n64_protocol(args, rlpt, torch, out, out["n64_physics"]["cv_per_mode"])
    if not args.no_batched and not args.no_cached:
        out["batched"] = batched(args, short=True)
        rlpt.tune_clear()  # the autotuner's registry would otherwise choose the later contexts' tiles
    if args.tau_sweeps > 0 and args.learn_temps and not args.no_n64:
        learned_n64(args, rlpt, torch, out)
        # the same comparison at the four coldest temperatures with untrained networks (isotropic small
        # steps), over 10^5 measured sweeps: where the pair moves freeze, global chart moves pay
        cold = {}
        learned_n64(args, rlpt, torch, cold, sweeps=100000, at="cold", train=False)
        out["learned_n64_cold_untrained"] = cold["learned_n64"]
    if args.tau_sweeps > 0:
        tau = {"observable": "E (energy of ladder 0 at each temperature); tau_int_q: overlap q of the two "
                             "replicas, same window", "estimator": "Sokal window c=6, per disorder sample",
               "plain": tau_plain}
        # ------------------------------------------------------------ shared pair schedule
        if not args.shared_pairs and not args.only_learned_256 and not args.only_learned_all_256:
            ctx = rlpt.Context(graphs, temps, shared_pairs=1, **common)
            el2, kms2, launches2 = timed(ctx, "shared pairs")
            tau["shared_pairs"], tE2, _ = tau_block(ctx, args.sweeps / el2, t_learn, args.tau_sweeps, "shared pairs")
            tau["shared_pairs"]["mode_updates_per_s"] = N * n_copies * args.sweeps / el2
            if chunked:
                # the copies of a sample share their lists through L2, so the binding roof is the LDS
                # gathers: per chunk of 4 entries one partner and 8 pair amplitudes, 9 x 8 B = 18 B per
                # entry; LDS peak = 128 B per clock per CU x 256 CUs x 2.4 GHz
                t2 = kms2 / launches2 * 1e-3
                lds_gbs = entries_per_launch * 18.0 / t2 / 1e9
                tau["shared_pairs"]["roofline"] = {
                    "bound": "lds", "achieved": lds_gbs, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                    "frac": lds_gbs / LDS_PEAK_GBS, "bytes_per_entry": 18.0, "ms_per_launch": kms2 / launches2,
                    "list_GBps_algorithmic": entries_per_launch * per_entry / t2 / 1e9}
            tau["shared_vs_plain_eff"] = eff_ratio(tE2, tau_plain_E, args.sweeps / el2, sweeps_per_s)
            ctx.close()
        # ------------------------------------------------------------ learned global moves
        def learned_256(subset, scale, tag, rounds=1):
            lcommon = dict(common, series_len=series_len + 2 * args.harvest_rounds + args.reeq)
            ctx = rlpt.Context(graphs, temps, shared_pairs=args.shared_pairs, mlp_nets=len(t_learn),
                               mlp_hidden=256, mlp_components=4, mlp_capacity=8192, mlp_batch=512,
                               mlp_subset=subset, **lcommon)
            ctx.init(args.run_seed)
            ctx.sweep(args.warm_sweeps)
            ctx.mlp_setup(t_learn, seed=1)
            t0 = time.perf_counter()
            losses, train_error = [], None
            if not args.untrained:
                log(f"{tag}: harvest and train")
                ctx.mlp_harvest(rounds=args.harvest_rounds, lag=2)
                try:
                    losses.append(ctx.mlp_train(1, 1e-3))
                    losses.append(ctx.mlp_train(args.train_steps, 1e-3))
                except rlpt.RlptError as e:
                    train_error = str(e)
                    log(f"{tag}: training failed: {e}")
            t_train = time.perf_counter() - t0
            if train_error is None:
                ctx.mlp_enable(rounds, scale)
            # the harvest ran without swaps: re-equilibrate with swaps and learned rounds before the window
            if not args.untrained:
                ctx.sweep(args.reeq)
            done = ctx.counters()[0]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.sweep(args.sweeps)
            torch.cuda.synchronize()
            el3 = time.perf_counter() - t0
            log(f"{tag}: {args.sweeps / el3:.1f} sweeps/s; tau_int run")
            # measurements started at the warm-up boundary: the series covers harvest + learned sweeps;
            # tau is taken over the learned part only
            long_run(ctx, args.tau_sweeps, tag)
            o = ctx.observables()
            m = min(int(o["e_n"][0, 0] / reps), series_len + 2 * args.harvest_rounds + args.reeq)
            lo = max(done - args.warm_sweeps, 0) + (m - max(done - args.warm_sweeps, 0)) // 4
            tEl = tau_per_sample(o["series_e"], t_learn, lo, m)
            tql = tau_per_sample(o["series_q"], t_learn, lo, m)
            wl = window_means(o, t_learn, lo, m)
            acc, tries = ctx.mlp_stats()
            acc_rate = acc / np.maximum(tries, 1)
            sps3 = args.sweeps / el3
            dead = dead_networks(acc_rate, np.array(losses) if losses else None)
            if train_error:
                dead.append({"network": "all", "failed": train_error})
            res = {"move": f"subset of {subset} modes" if subset else "all modes",
                   "networks": "untrained (outputs near 0: an isotropic small-step mixture)" if args.untrained
                   else "trained on harvested pairs", "temperatures":
                   [float(temps[t]) for t in t_learn], "tau_int_E": tau_stats(tEl), "tau_int_q": tau_stats(tql),
                   "sweeps_per_s": sps3, "series_points": m - lo, "move_acceptance": acc_rate.round(4).tolist(),
                   "step_scale": scale, "rounds_per_sweep": rounds,
                   "train_loss_first_last": [np.round(x, 2).tolist() for x in losses],
                   "harvest_and_train_s": t_train, "failed_networks": dead,
                   "agreement_with_plain": {
                       "E": paired_agreement(wl["E"], tau_plain_w["E"]),
                       "q2": paired_agreement(wl["q2"], tau_plain_w["q2"]),
                       "E_drift_plain": paired_agreement(tau_plain_w["E_second"], tau_plain_w["E_first"]),
                       "E_drift_learned": paired_agreement(wl["E_second"], wl["E_first"]),
                       "test": "window means of E and of q^2 per sample, learned - plain, paired jackknife over "
                               "the disorder samples; E_drift: second half of a run's window - first half"}}
            ctx.close()
            ratio = eff_ratio(tEl, tau_plain_E, sps3, sweeps_per_s)
            for d in dead:
                if isinstance(d["network"], int):
                    ratio["status"][d["network"]] = "failed: " + d["failed"]
                else:
                    ratio["status"] = ["failed: " + d["failed"]] * len(ratio["status"])
            log(f"{tag}: eff ratio {ratio['ratio']} {ratio['status']}; E within 2 sigma of plain "
                f"{res['agreement_with_plain']['E']['within_2sigma']:.2f}, q^2 "
                f"{res['agreement_with_plain']['q2']['within_2sigma']:.2f}; E drift over the window plain "
                f"{res['agreement_with_plain']['E_drift_plain']['diff']}, learned "
                f"{res['agreement_with_plain']['E_drift_learned']['diff']}")
            return res, ratio

        if t_learn and not args.only_learned_256:
            tau["learned"], tau["learned_vs_plain_eff"] = learned_256(0, args.learn_scale, "learned",
                                                                      args.learn_rounds)
        if t_learn and not args.only_learned_all_256:
            m_sub = max(2, N // args.subset_frac)
            tau["learned_subset"], tau["learned_subset_vs_plain_eff"] = learned_256(m_sub, args.subset_scale,
                                                                                   "learned subset",
                                                                                   args.subset_rounds)
        out["tau_int_corrected"] = tau
    if not args.no_cpu_baseline:
        try:
            nthr = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
        except (ValueError, AttributeError):
            nthr = os.cpu_count() or 1
        log(f"cpu baseline: oracle on {nthr} threads for ~{args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(N, temps, reps, args.cpu_seconds, nthr)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
