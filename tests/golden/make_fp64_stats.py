"""Write tests/golden/fp64_stats_full.json: spike statistics of the oracle's
FP64 mode on the full-scale microcircuit (stand-in connection table), 10 s
biological time, first 1 s discarded (Sec. 2a / 4b of the paper).

Entries "<seed>" are the model (Poisson stream 0) for network seeds 1, 2, 3;
entries "1/stream<k>" are independent background realisations on the seed-1
network (the run-to-run spread of the model on that network); entries
"1/perturb<k>" keep stream 0 and make one neuron (id 7919 k mod N) spike in
the first step (initial u = theta + 1 mV): the smallest discrete change of a
run, the kind an FP32 rounding causes when it flips one threshold decision.
Their spread around entry "1" is what the divergence that follows does to the
statistics of a run with the same background input: the noise floor of an
FP32-versus-FP64 comparison.  (A sub-ulp change of the initial state alone
decays with tau_m before it flips any decision and leaves the run unchanged.)

Calls only oracle/ (and the seeded input generator).  ~3-7 min per run on 8
CPU cores:  python tests/golden/make_fp64_stats.py [seed[/stream<k>] ...]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from oracle.stats import population_stats           # noqa: E402
from synth_inputs import standin_conn_table, standin_description   # noqa: E402

STEPS, DISCARD = 100000, 10000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp64_stats_full.json")


def main(keys):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    conn = standin_conn_table()
    for key in keys:
        seed, _, var = key.partition("/")
        seed = int(seed)
        stream = int(var[len("stream"):]) if var.startswith("stream") else 0
        perturb = int(var[len("perturb"):]) if var.startswith("perturb") else 0
        t = time.time()
        net = O.OracleNet.build(seed, 1.0, conn.reshape(64), O.default_params(mode=O.FP64, pois_stream=stream))
        if perturb:
            u, _, _ = net.state()
            u[(7919 * perturb) % len(u)] = 15.0 + 1.0
            net.set_state(u=u)
        net.run(STEPS)
        st, ids = net.spikes()
        stats = population_stats(st, ids, net.pop_offsets, DISCARD, STEPS)
        data[key] = {"stats": stats, "counters": net.counters(), "steps": STEPS, "discard": DISCARD,
                     "seed": seed, "pois_stream": stream, "forced_first_spike": (7919 * perturb) % net.N if perturb else None, "conn_table": standin_description(), "mode": "FP64"}
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        print(f"{key}: {time.time() - t:.0f}s", {k: round(v['rate_hz'], 3) for k, v in stats.items()}, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["1", "2", "3", "1/stream1", "1/stream2", "1/stream3", "1/stream4",
                          "1/perturb1", "1/perturb2", "1/perturb3", "1/perturb4"])
