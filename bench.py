"""Benchmark: real-time factor and synaptic events/s of the full-scale cortical
microcircuit (77,169 neurons, ~3e8 synapses, dt = 0.1 ms) on one MI355X.

One benchmark "step" is one simulation step: Poisson drive, LIF update, spike
compaction and delivery of every spike's synaptic row, for the whole network.
Prints one JSON line.  Inputs are synthetic and seeded; the network is built and
uploaded before the timed region (the synapse store is resident in HBM).

    python bench.py [--gpus 1] [--steps 100000] [--warmup 1000]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DT_S = 1e-4
HBM_PEAK_GBS = 8000.0
METRIC = "real-time factor + synaptic events/s, full 77k-neuron microcircuit, 1 GPU"
WFMT = {"fp32": 0, "fp16": 1, "bf16": 2}
INIT_MODES = {"uniform": 0, "zero": 1, "relaxed": 2}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(seed, scale, conn, warm, steps, i_dc=None, single_steps=0, init_kw=None):
    """The oracle (FP32 mirror) on this host's cores, on a bounded sample of the
    same workload: same network, `steps` steps after `warm` untimed steps on
    every core, then (single_steps > 0) the next single_steps on one thread."""
    from oracle import oracle as O

    cores = O.max_threads()
    t = time.time()
    kw = dict(init_kw or {})
    params = O.default_params(**kw) if i_dc is None else O.default_params(poisson_on=False, i_dc=i_dc, **kw)
    net = O.OracleNet.build(seed, scale, conn.reshape(64), params)
    log(f"oracle build {time.time() - t:.1f}s ({cores} threads)")
    net.run(warm)
    net.spikes(clear=True)

    def timed(n):
        c0 = net.counters()
        t0 = time.perf_counter()
        net.run(n)
        wall = time.perf_counter() - t0
        net.spikes(clear=True)
        return wall, net.counters()["events"] - c0["events"]

    wall, ev = timed(steps)
    log(f"oracle {steps} steps in {wall:.2f}s on {cores} threads")
    out = {"value": round(steps * DT_S / wall, 6), "unit": "x real time (simulated s per wall s)",
           "events_per_s": round(ev / wall, 1), "cores": cores, "kind": "oracle",
           "sample": f"FP32-mirror oracle, same seeded network (scale {scale}), steps {warm}..{warm + steps} "
                     f"({steps * DT_S:.2f} s biological time) on {cores} threads, build excluded"}
    if single_steps:
        O.set_threads(1)
        wall1, ev1 = timed(single_steps)
        O.set_threads(cores)
        log(f"oracle {single_steps} steps in {wall1:.2f}s on 1 thread")
        out["single_thread"] = {"value": round(single_steps * DT_S / wall1, 6), "events_per_s": round(ev1 / wall1, 1),
                                "steps": [warm + steps, warm + steps + single_steps]}
    return out


def cpu_survey(conn, init_kw):
    """The oracle (FP32 mirror) on the 2 % network (10^4 steps), one 10 %
    instance of the batch workload and the full network (bounded samples after a
    warm-up), each on every core and on one thread: real-time factor and
    recurrent events/s.  Host model and core count are reported."""
    import platform

    from oracle import oracle as O
    cores = O.max_threads()
    model = ""
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        model = platform.processor()
    rows = []
    for name, seed, scale, warm, steps, steps1 in (("2 % (1,544 neurons)", 1, 0.02, 1000, 10000, 10000),
                                                   ("10 % instance of the batch (7,718 neurons)", 1000, 0.1, 1000, 5000, 2000),
                                                   ("full scale (77,169 neurons)", 1, 1.0, 1000, 3000, 200)):
        t = time.time()
        net = O.OracleNet.build(seed, scale, conn.reshape(64), O.default_params(**init_kw))
        build_s = time.time() - t
        net.run(warm)
        net.spikes(clear=True)
        row = {"workload": name, "scale": scale, "seed": seed, "build_s": round(build_s, 2)}
        for threads, n in ((cores, steps), (1, steps1)):
            O.set_threads(threads)
            c0 = net.counters()
            t0 = time.perf_counter()
            net.run(n)
            wall = time.perf_counter() - t0
            net.spikes(clear=True)
            ev = net.counters()["events"] - c0["events"]
            row[f"threads_{threads}"] = {"steps": n, "rtf": round(n * DT_S / wall, 5), "events_per_s": round(ev / wall, 1)}
            log(f"oracle {name}: {threads} threads, {n} steps in {wall:.2f}s -> RTF {n * DT_S / wall:.4f}")
        O.set_threads(cores)
        rows.append(row)
        del net
    return {"metric": "oracle (FP32 mirror) real-time factor on the host", "cores": cores, "cpu": model,
            "kind": "oracle", "rows": rows}


PHASES = (("update+publish", 0, 1), ("wait for all tiles", 3, 4),
          ("spike ids + sub-row entries", 4, 5), ("delivery", 5, 6))


def step_latency(net):
    """Per-step timing of the tiled kernel from its 100 MHz phase timestamps:
    phase means and the step period against the 100 us real-time deadline."""
    tr, launch = net.trace(launch=True)               # [steps, tiles, 8], [tiles, 4]
    tr = tr.astype(np.int64)
    if tr.shape[0] < 2:
        return None
    launch = launch.astype(np.int64)
    prologue = (launch[:, 1] - launch[:, 0]) * 0.01                       # us per tile
    epilogue = (launch[:, 3] - launch[:, 2]) * 0.01
    skew = (launch[:, 0].max() - launch[:, 0].min()) * 0.01
    log(f"  launch: prologue max {prologue.max():.2f} us, epilogue max {epilogue.max():.2f} us, "
        f"start skew over tiles {skew:.2f} us")
    if launch.shape[1] >= 7:
        for name, a, b in (("state stores + barrier", 2, 4), ("ring stores", 4, 5), ("counter atomics", 5, 6),
                           ("path counters, heads", 6, 3)):
            d = (launch[:, b] - launch[:, a]) * 0.01
            log(f"    epilogue {name:24s} mean {d.mean():7.3f} us  max {d.max():7.3f} us")
    tr[:, :, 5] = np.where(tr[:, :, 5] == 0, tr[:, :, 4], tr[:, :, 5])   # steps without spikes
    per = np.diff(tr[:, :, 0], axis=0).max(axis=1) * 0.01                # us, slowest tile
    phases = {}
    for name, a, b in PHASES:
        d = (tr[:, :, b] - tr[:, :, a]) * 0.01
        phases[name] = round(float(d.mean()), 3)
        log(f"  phase {name:30s} mean {d.mean():7.3f} us  p99 {np.percentile(d, 99):7.3f} us")
    log(f"  step period mean {per.mean():.3f} us, p50 {np.median(per):.3f}, p99 {np.percentile(per, 99):.3f}, "
        f"max {per.max():.3f}")
    return {"steps": int(tr.shape[0] - 1), "mean_us": round(float(per.mean()), 3),
            "p50_us": round(float(np.median(per)), 3), "p99_us": round(float(np.percentile(per, 99)), 3),
            "max_us": round(float(per.max()), 3), "deadline_us": 100.0,
            "frac_over_deadline": float((per > 100.0).mean()), "phases_us": phases,
            "launch_us": {"prologue_max": round(float(prologue.max()), 3), "epilogue_max": round(float(epilogue.max()), 3),
                          "start_skew": round(float(skew), 3)}}


# Workloads: (seeds, scales, default weight format, description)
CONFIGS = {
    "full": "one full-scale instance",
    "batch64": "64 independent instances at 10 % scale, seeds 1000..1063",
    "uneven32": "32 independent instances at scales drawn from U(0.05, 0.5), seeds 2000..2031, FP16 weights",
}


def workload(args):
    from synth_inputs import batch_scales

    if args.config == "batch64":
        return [1000 + j for j in range(64)], [0.1] * 64
    if args.config == "uneven32":
        return [2000 + j for j in range(32)], [float(x) for x in batch_scales(32, 0.05, 0.5, seed=777)]
    return [args.seed], [args.scale]


def delivery_microbench(net, info, args, conn_desc):
    """Delivery of forced spike lists (S neurons spiking at once, ids spread over
    the populations in proportion to their sizes) through mc_inject_spikes:
    algorithmic bytes = events x bytes per synapse record + S x tiles x 8 B of
    sub-row descriptors + the read-modify-write of the ring cells that receive
    events, over the HIP-event kernel time."""
    from synth_inputs import forced_spike_list

    import paper_1909_08665_amd as mc

    b_event = info["syn_bytes"]
    tiled = info["engine"] == 2 and info["lds_ring"] == 1
    n = info["n_neurons"]
    # the rate of whole-line reads at random places of a buffer as large as the
    # synapse store: what HBM gives reads at random places, beside the streaming
    # copy
    gather_gbs = mc.probe(mc.PROBE_HBM_GATHER, 2 << 30)[0]
    copy_gbs = mc.probe(mc.PROBE_HBM_COPY, 2 << 30)[0]
    log(f"D1 ceilings: random 128-byte line reads {gather_gbs:.0f} GB/s, streaming copy {copy_gbs:.0f} GB/s")
    rows = []
    for S in (25, 93, 1000, 4000, 20000, 77169):
        ids = forced_spike_list(S, args.scale, seed=S)
        net.inject_spikes(ids)                          # warm-up
        net.set_timing(True)
        reps, events = 0, 0
        while reps < 3 or (events < 3e9 and reps < 200):
            events += net.inject_spikes(ids)
            reps += 1
        ms, launches = net.timing()
        net.set_timing(False)
        per = ms / launches
        ev = events / reps
        ptr_bytes = S * info["n_tiles"] * 8 if tiled else S * 16
        # the staged ring's cells that received events, read and written back
        # (expected distinct cells hit by ev events; exact for uniform slots)
        cells = info["ring_depth"] * n
        ring_bytes = 8 * cells * -np.expm1(-ev / cells) if tiled else 0
        algo = ev * b_event + ptr_bytes + ring_bytes
        gbs = algo / (per * 1e-3) / 1e9
        rows.append({"spikes": S, "events": int(ev), "kernel_ms": round(per, 4), "GB_s": round(gbs, 1),
                     "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "frac_gather": round(gbs / gather_gbs, 4),
                     "events_per_s": round(ev / (per * 1e-3), 1)})
        log(f"D1 S={S:6d}: {ev:.3e} events in {per:.3f} ms -> {gbs:8.1f} GB/s ({gbs / HBM_PEAK_GBS:.1%} of HBM, "
            f"{gbs / gather_gbs:.1%} of the random-line rate), {ev / (per * 1e-3):.3e} events/s")
    return {"metric": "delivery microbenchmark (forced spike lists)", "unit": "GB/s", "dtype": "i32",
            "data": "synthetic", "ceilings_GB_s": {"random_line_reads": round(gather_gbs, 1),
                                                   "streaming_copy": round(copy_gbs, 1)},
            "config": {"workload": f"microcircuit scale {args.scale}, {args.wfmt.upper()} store, "
                                            f"{'tiled LDS-staged' if tiled else 'global-atomic'} delivery",
                                            "conn_table": conn_desc, "n_tiles": info["n_tiles"]},
            "rows": rows}


def probe_table():
    """Every ceiling mc_probe measures, at buffer sizes that sit in one XCD's
    L2 (1 MiB), in the Infinity Cache (64 MiB) and in HBM (2 GiB)."""
    import torch

    import paper_1909_08665_amd as mc

    out = {"metric": "memory-system ceilings (mc_probe)", "device": torch.cuda.get_device_name(0), "rows": []}
    rows = [("streaming copy, read + written", mc.PROBE_HBM_COPY, 2 << 30, "GB/s"),
            ("whole 128-byte lines at random places", mc.PROBE_HBM_GATHER, 2 << 30, "GB/s"),
            ("whole 128-byte lines at random places", mc.PROBE_HBM_GATHER, 64 << 20, "GB/s"),
            ("whole 128-byte lines at random places", mc.PROBE_HBM_GATHER, 1 << 20, "GB/s"),
            ("LDS int32 atomic add, random words", mc.PROBE_LDS_ATOMICS, 0, "atomics/s"),
            ("device int32 atomic add, random words", mc.PROBE_DEVICE_ATOMICS, 1 << 20, "atomics/s"),
            ("device int32 atomic add, random words", mc.PROBE_DEVICE_ATOMICS, 64 << 20, "atomics/s"),
            ("device int32 atomic add, random words", mc.PROBE_DEVICE_ATOMICS, 2 << 30, "atomics/s")]
    for name, kind, nbytes, unit in rows:
        rate, ms = mc.probe(kind, nbytes)
        out["rows"].append({"probe": name, "bytes": nbytes, "rate": round(rate, 1), "unit": unit,
                            "kernel_ms": round(ms, 4)})
        log(f"{name:40s} {nbytes / 2**20:8.0f} MiB: {rate:.4g} {unit} ({ms:.3f} ms)")
    return out


PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1909_08665_amd", "csrc", "kernels.hip")


def measured_traffic_per_launch(workload_key):
    """HBM bytes per timed launch of the dominant kernel, from a committed
    rocprofv3 record (FETCH_SIZE and WRITE_SIZE of the timed dispatches, each
    scaled by what the counter reads for a plain copy of known size) taken on
    exactly this workload, step count and warm-up, and on the kernel source
    built here; None when no such record exists."""
    import glob
    import hashlib
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(PROFILES, "*.md"))):
        for line in open(path):
            if not line.startswith("traffic-record:"):
                continue
            f = dict(x.strip().rsplit(" ", 1) for x in line.split(":", 1)[1].split(";"))
            if f.get("kernels.hip sha256") != sha or f.get("workload") != workload_key:
                continue
            total = float(f["fetch KiB"]) * float(f["fetch factor"]) + float(f["write KiB"]) * float(f["write factor"])
            return total * 1024 / float(f["launches"])
    return None


def stability_run(args, mc, conn):
    """Long full-scale run (hours of biological time) in 10 s windows: the
    per-population rate of every window, the fitted drift of each population's
    rate (per cent of its mean per hour, first window discarded), error flags,
    a checkpoint every 10 biological minutes, and at the end a bit-exact check
    that a fresh network resumed from the last checkpoint continues the run."""
    import tempfile

    from synth_inputs import FULL_SIZE, POP_NAMES
    win = 100000                                   # 10 s
    windows = max(2, int(round(args.stability * 3600 / 10)))
    net = mc.Network.build(args.seed, 1.0, conn, wfmt=WFMT[args.wfmt])
    sizes = np.array(FULL_SIZE, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)])
    rates = np.zeros((windows, 8))
    ckpt = os.path.join(tempfile.gettempdir(), f"mc_stability_{os.getpid()}.ckpt")
    ckpt_ms = []
    t0 = time.perf_counter()
    for w in range(windows):
        net.run(win)
        _, ids = net.spikes()
        pop = np.searchsorted(off, ids, side="right") - 1
        rates[w] = np.bincount(pop, minlength=8)[:8] / (sizes * win * DT_S)
        if (w + 1) % 60 == 0:
            tc = time.perf_counter()
            net.save(ckpt)
            ckpt_ms.append((time.perf_counter() - tc) * 1e3)
        if (w + 1) % 6 == 0:
            log(f"stability: {(w + 1) * 10 / 60:.0f} biological min, wall {time.perf_counter() - t0:.1f}s, "
                f"rates {np.round(rates[w], 3).tolist()}")
    wall = time.perf_counter() - t0
    c = net.counters()
    hours = (np.arange(1, windows) + 0.5) * 10 / 3600
    drift = {}
    for a, name in enumerate(POP_NAMES):
        r = rates[1:, a]
        slope = np.polyfit(hours, r, 1)[0] if len(r) > 1 else 0.0
        drift[name] = {"mean_hz": round(float(r.mean()), 4), "sd_hz": round(float(r.std()), 4),
                       "slope_pct_per_h": round(float(100 * slope / r.mean()), 3) if r.mean() > 0 else None}
    # resume check: continue 2000 steps, then replay them from the last checkpoint
    net.save(ckpt)
    net.run(2000)
    sa = net.spikes()
    fresh = mc.Network.build(args.seed, 1.0, conn, wfmt=WFMT[args.wfmt])
    fresh.load(ckpt)
    fresh.run(2000)
    sb = fresh.spikes()
    resumed = bool(np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1]))
    os.remove(ckpt)
    fresh.close()
    net.close()
    return {"metric": "stability (full scale, long run)", "unit": "x real time", "value": round(windows * win * DT_S / wall, 4),
            "data": "synthetic", "dtype": "f32",
            "config": {"workload": f"microcircuit scale 1.0, {args.wfmt.upper()} store, "
                                   f"{windows * 10 / 3600:g} h biological time in 10 s windows", "seed": args.seed},
            "steps": windows * win, "wall_s": round(wall, 2), "spikes": c["spikes"], "events": c["events"],
            "max_spikes_per_step": c["max_spikes_per_step"], "error_flags": "none: every mc_run returned MC_OK (a recorder overflow or a timed-out wait raises)",
            "drift": drift, "checkpoint_ms": [round(x, 1) for x in ckpt_ms], "resume_bit_exact": resumed,
            "window_rates_hz": np.round(rates, 4).tolist()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--config", choices=sorted(CONFIGS), default="full",
                    help="full: one full-scale instance; batch64: 64 instances at 10 %%; "
                         "uneven32: 32 instances at scales U(5 %%, 50 %%), FP16 weights")
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--wfmt", choices=sorted(WFMT), default=None)
    ap.add_argument("--engine", choices=["auto", "graph", "tiled"], default="auto")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--tune", action="store_true", help="run the autotuner before timing")
    ap.add_argument("--init", choices=sorted(INIT_MODES), default="relaxed",
                    help="initial state: relaxed (default; per-population steady-state moments of u and I, "
                         "as the paper starts from a relaxed state), uniform u in [0, theta), or all at rest")
    ap.add_argument("--device-build", action="store_true", help="draw and sort the synapse store on the GPU")
    ap.add_argument("--dc", action="store_true",
                    help="DC-input workload: no Poisson background, each population driven by the mean "
                         "current of its Poisson drive (stand-in amplitudes)")
    ap.add_argument("--step-budget", type=float, default=0, metavar="US",
                    help="lossy real-time mode: drop deliveries past US microseconds into a step (tiled engine)")
    ap.add_argument("--poll-delay", type=int, default=0,
                    help="tiled engine: sleep before polling, units of 64 clocks (-1 none, 0 library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-warm", type=int, default=1000)
    ap.add_argument("--cpu-steps", type=int, default=5000)
    ap.add_argument("--cpu-survey", action="store_true",
                    help="only time the oracle on the host: 2 %%, one 10 %% instance, full scale; all cores and one")
    ap.add_argument("--cpu-single-steps", type=int, default=300,
                    help="oracle steps timed on one thread after the multi-thread sample (0: none)")
    ap.add_argument("--d1", action="store_true",
                    help="delivery microbenchmark: inject forced spike lists of 25..77169 neurons")
    ap.add_argument("--probes", action="store_true",
                    help="only print the memory-system ceilings mc_probe measures on this device and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device twice (reference for HBM byte counters) and exit")
    ap.add_argument("--stability", type=float, default=0, metavar="HOURS",
                    help="long full-scale run of HOURS biological time: per-window rates, drift, checkpoints")
    ap.add_argument("--trace", type=int, default=0,
                    help="record per-step phase timestamps for the first K timed steps (tiled engine)")
    args = ap.parse_args()
    if args.wfmt is None:
        args.wfmt = "fp16" if args.config == "uneven32" else "fp32"

    if args.cpu_survey:
        from synth_inputs import relaxed_start, standin_conn_table
        kw = relaxed_start() if args.init == "relaxed" else {"init_mode": INIT_MODES[args.init]}
        print(json.dumps(cpu_survey(standin_conn_table(), kw)), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(independent instances would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1909_08665_amd as mc
    from synth_inputs import dc_standin_amplitudes, relaxed_start, standin_conn_table, standin_description

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.probes:
        print(json.dumps(probe_table()), flush=True)
        return
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "copies": 2}), flush=True)
        return
    conn = standin_conn_table()
    if args.stability:
        print(json.dumps(stability_run(args, mc, conn)), flush=True)
        return
    engine = {"auto": mc.ENGINE_AUTO, "graph": mc.ENGINE_GRAPH, "tiled": mc.ENGINE_TILED}[args.engine]

    seeds, scales = workload(args)
    n_inst = len(seeds)
    t = time.time()
    db = int(args.device_build)
    drive = dict(poisson_on=False, i_dc=dc_standin_amplitudes()) if args.dc else {}
    drive.update(relaxed_start() if args.init == "relaxed" else {"init_mode": INIT_MODES[args.init]})
    if n_inst == 1:
        net = mc.Network.build(seeds[0], scales[0], conn, wfmt=WFMT[args.wfmt], engine=engine, device_build=db, **drive)
    else:
        net = mc.Network.build_batch(seeds, scales, conn, wfmt=WFMT[args.wfmt], engine=engine, device_build=db,
                                     **drive)
    if args.tile:
        net.set_launch(engine=mc.ENGINE_TILED, tile=args.tile)
    if args.poll_delay:
        net.set_launch(poll_delay=args.poll_delay)
    if args.step_budget:
        net.set_step_budget(args.step_budget)
    info = net.info()
    n_neurons, n_syn = info["n_neurons"], info["n_synapses"]
    log(f"build+upload {time.time() - t:.1f}s: {n_inst} instance(s), {n_neurons} neurons, {n_syn} synapses")
    if args.tune:
        net.tune(500)
    info = net.info()
    log("launch", {k: info[k] for k in ("engine", "tile_neurons", "n_tiles", "ring_depth", "graph_chunk", "seg")})

    def drain_all():
        for j in range(n_inst):
            net.spikes(j)

    if args.d1:
        print(json.dumps(delivery_microbench(net, info, args, conn_desc=standin_description())), flush=True)
        net.close()
        return

    net.run(args.warmup)
    drain_all()
    if args.trace and info["engine"] == mc.ENGINE_TILED:
        net.set_trace(args.trace)
    c0 = net.counters()
    net.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.run(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms, launches = net.timing()
    c1 = net.counters()
    drain_all()
    events = c1["events"] - c0["events"]
    spikes = c1["spikes"] - c0["spikes"]
    rtf = n_inst * args.steps * DT_S / wall        # instance-seconds simulated per wall second
    log(f"{args.steps} steps in {wall:.3f}s: RTF {rtf:.2f}, {events / wall:.3e} events/s, "
        f"{spikes / args.steps:.1f} spikes/step")

    # Roofline of the dominant kernel: the algorithmic HBM bytes of the path
    # per unit of work -- per recurrent event the synapse's target, weight and
    # delay (4 + 4 + 1 B, or 4 + 2 + 1 B with a 16-bit weight), per spike its
    # 8-byte row pointer plus, in the tiled form, (T + 1) 4-byte sub-row
    # pointers of its instance's T tiles, and per neuron-step the state
    # traffic of the forms that keep it in HBM (graph: 26 B; tiled with the
    # ring in global memory: 8 B, the slot read and clear), and per launch of
    # the tiled kernel the rings and neuron state it loads at its start and
    # stores at its end (LDS ring: R x 4 B each way per neuron, a ring slice in
    # global memory: twice that; state 9 B each way) -- times the units one
    # launch processes, over its HIP-event-timed duration.  The bytes of the
    # store as actually laid out (packed records of syn_bytes, 8-byte sub-row
    # entries) are reported beside them.
    tiled = info["engine"] == mc.ENGINE_TILED
    b_event = 9 if args.wfmt == "fp32" else 7
    tiles_per_inst = info["n_tiles"] / n_inst if tiled else 0
    if tiled:
        per_spike = 8 + (tiles_per_inst + 1) * 4
        per_neuron_step = 0 if info["lds_ring"] else 8
        per_neuron_launch = 2 * 9 + (2 if info["lds_ring"] else 4) * info["ring_depth"] * 4
        stored_per_spike = 8 * tiles_per_inst
        kname = "k_tiled (persistent step kernel)"
    else:
        per_spike = 8
        per_neuron_step = 26
        per_neuron_launch = 0
        stored_per_spike = 16
        kname = "k_neuron + k_deliver (graph-captured step)"
    launch_bytes = launches * n_neurons * per_neuron_launch
    algo_bytes = events * b_event + spikes * per_spike + args.steps * n_neurons * per_neuron_step + launch_bytes
    stored_bytes = (events * info["syn_bytes"] + spikes * stored_per_spike + args.steps * n_neurons * per_neuron_step
                    + launch_bytes)
    avg_launch_ms = kernel_ms / max(1, launches)
    per_launch_s = max(1e-12, avg_launch_ms * 1e-3)
    achieved = algo_bytes / max(1, launches) / per_launch_s / 1e9 if kernel_ms > 0 else 0.0
    workload_key = (f"{args.config}/{args.wfmt}/scale={scales[0] if n_inst == 1 else 'batch'}/steps={args.steps}/"
                    f"warmup={args.warmup}/engine={'tiled' if tiled else 'graph'}/dc={int(args.dc)}/"
                    f"budget={args.step_budget:g}/init={args.init}")
    traffic = measured_traffic_per_launch(workload_key) if launches else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 6),
                "traffic": int(traffic) if traffic is not None else None, "kernel": kname,
                "launches": launches, "avg_launch_ms": round(avg_launch_ms, 4),
                "bytes_per_launch": int(algo_bytes / max(1, launches)),
                "stored_layout": {"bytes_per_launch": int(stored_bytes / max(1, launches)),
                                  "achieved": round(stored_bytes / max(1, launches) / per_launch_s / 1e9, 3)
                                  if kernel_ms > 0 else 0.0},
                "workload_key": workload_key}
    # Atomic throughput: every recurrent event is one int32 atomic add into a
    # ring slot -- LDS atomics when the tile rings sit in LDS; with the ring in
    # each workgroup's global slice, LDS atomics for the delays the LDS window
    # holds and workgroup-scope atomics into the slice for the others (the LDS
    # rate is then the ceiling: no form of the add is faster); device atomics in
    # the graph engine -- against the ceiling the probe measures on this device.
    atomics = None
    if kernel_ms > 0:
        if tiled and info["lds_ring"]:
            peak, akind = mc.probe(mc.PROBE_LDS_ATOMICS)[0], "LDS int32 atomic add (random words)"
        elif tiled:
            peak, akind = mc.probe(mc.PROBE_LDS_ATOMICS)[0], \
                "LDS (window) and workgroup-scope int32 atomic adds; peak: the LDS atomic rate"
        else:
            ring_bytes = info["ring_depth"] * n_neurons * 4
            peak, akind = mc.probe(mc.PROBE_DEVICE_ATOMICS, max(8192, ring_bytes))[0], \
                f"device int32 atomic add (random words of a {ring_bytes / 2**20:.0f} MiB buffer)"
        rate = events / max(1, launches) / per_launch_s
        atomics = {"achieved": round(rate, 1), "peak": round(peak, 1), "unit": "atomics/s",
                   "frac": round(rate / peak, 6) if peak else None, "kind": akind}

    latency = step_latency(net) if args.trace and tiled else None

    out = {
        "metric": METRIC,
        "value": round(rtf, 4),
        "unit": "x real time (simulated s per wall s)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"microcircuit scale {scales[0]} " if n_inst == 1 else CONFIGS[args.config] + " ")
                               + f"({n_neurons} neurons, {n_syn} synapses), {args.wfmt.upper()} weight store, "
                               f"{args.steps * DT_S:g} s biological time, "
                               + ("DC input (per population the mean current of its Poisson drive)"
                                  if args.dc else "Poisson background") + ", dt 0.1 ms",
                   "instances": n_inst, "seed": seeds[0] if n_inst == 1 else [seeds[0], seeds[-1]],
                   "conn_table": standin_description(),
                   "engine": "tiled" if tiled else "graph", "tile": info["tile_neurons"],
                   "n_tiles": info["n_tiles"], "ring_depth": info["ring_depth"],
                   "poll_delay": info["poll_delay"] if tiled else None,
                   "lds_window": info["lds_window"] if tiled else None},
        "events_per_s": round(events / wall, 1),
        **({"step_budget_us": args.step_budget,
            "dropped_events_frac": round((c1["dropped_events"] - c0["dropped_events"]) / max(1, events), 6)}
           if args.step_budget else {}),
        "spikes_per_step": round(spikes / args.steps, 3),
        "max_spikes_per_step": c1["max_spikes_per_step"],
        "context": {"paper_spinnaker_rtf": 1.0, "paper_spinnaker_events_per_s": 9.343e8},
        "roofline": roofline,
        "atomics": atomics,
    }
    if latency:
        out["step_latency"] = latency
    net.close()
    if not args.no_cpu_baseline:
        # one instance of the workload (the first) on the host cores, scaled to the batch
        cb = cpu_baseline(seeds[0], scales[0], conn, args.cpu_warm, args.cpu_steps,
                          i_dc=dc_standin_amplitudes() if args.dc else None, single_steps=args.cpu_single_steps,
                          init_kw={k: v for k, v in drive.items() if k.startswith("init_")})
        if n_inst > 1:
            cb["sample"] += f"; instance 0 of {n_inst} (per-instance rate)"
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
