"""Write tests/golden/fp64_ensemble_full.json: spike statistics of the oracle's
FP64 mode on the full-scale microcircuit (stand-in connection table, seed 1),
10 s biological time, first 1 s discarded (Sec. 2a / 4b of the paper).

Chaotic dynamics make an FP32 run and an FP64 run of the same network diverge
spike by spike once one rounding flips one threshold decision, so they are
compared as ensembles.  Entry "perturb<k>" (k = 1..8) is the FP64 run in which
neuron (7919 k) mod N starts above threshold (initial u = theta + 1 mV) and so
spikes in the first step -- the smallest discrete change of a run; the test
gives the GPU runs exactly the same eight starts.  Entries "seed<s>" are the
unperturbed FP64 runs of the networks built from seeds 2 and 3 (the spread
between network realisations, reported only).

Calls only oracle/ (and the seeded input generator).  Several minutes per run
on 8 CPU cores:  python tests/golden/make_fp64_stats.py [key ...]
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
ENSEMBLE = 8
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp64_ensemble_full.json")


def perturbed_neuron(k, n):
    return (7919 * k) % n


def main(keys):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    conn = standin_conn_table()
    for key in keys:
        seed, k = 1, 0
        if key.startswith("perturb"):
            k = int(key[len("perturb"):])
        elif key.startswith("seed"):
            seed = int(key[len("seed"):])
        t = time.time()
        net = O.OracleNet.build(seed, 1.0, conn.reshape(64), O.default_params(mode=O.FP64))
        forced = None
        if k:
            u, _, _ = net.state()
            forced = perturbed_neuron(k, len(u))
            u[forced] = 15.0 + 1.0
            net.set_state(u=u)
        net.run(STEPS)
        st, ids = net.spikes()
        stats = population_stats(st, ids, net.pop_offsets, DISCARD, STEPS)
        data[key] = {"stats": stats, "counters": net.counters(), "steps": STEPS, "discard": DISCARD,
                     "seed": seed, "forced_first_spike": forced, "conn_table": standin_description(),
                     "mode": "FP64"}
        del net
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        print(f"{key}: {time.time() - t:.0f}s", {p: round(v["rate_hz"], 3) for p, v in stats.items()}, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or [f"perturb{k}" for k in range(1, ENSEMBLE + 1)] + ["seed2", "seed3"])
