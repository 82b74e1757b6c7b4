"""Write tests/golden/fp64_stats_full.json: spike statistics of the oracle's
FP64 mode on the full-scale microcircuit (stand-in connection table), 10 s
biological time, first 1 s discarded (Sec. 2a / 4b of the paper).

Entries "<seed>" are the model (Poisson stream 0) for network seeds 1, 2, 3;
entries "1/stream<k>" are independent background realisations on the seed-1
network (the noise floor of a comparison on that network).

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
        seed, _, stream = key.partition("/stream")
        seed, stream = int(seed), int(stream or 0)
        t = time.time()
        net = O.OracleNet.build(seed, 1.0, conn.reshape(64), O.default_params(mode=O.FP64, pois_stream=stream))
        net.run(STEPS)
        st, ids = net.spikes()
        stats = population_stats(st, ids, net.pop_offsets, DISCARD, STEPS)
        data[key] = {"stats": stats, "counters": net.counters(), "steps": STEPS, "discard": DISCARD,
                     "seed": seed, "pois_stream": stream, "conn_table": standin_description(), "mode": "FP64"}
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
        print(f"{key}: {time.time() - t:.0f}s", {k: round(v['rate_hz'], 3) for k, v in stats.items()}, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["1", "2", "3", "1/stream1", "1/stream2"])
