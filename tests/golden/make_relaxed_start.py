"""Write synth_inputs/relaxed_start.json: per-population moments of the steady
state of the full-scale microcircuit (stand-in connection table), the inputs of
the relaxed initial state (init_mode 2).

The paper starts its runs from membrane potentials chosen so that the first
steps already look like the steady state, instead of the transient a uniform
start gives (Sec. 4a); its values are not given.  Here they are measured: the
oracle (FP32 mirror) runs the network of seed 1 from the uniform start for
2 s, then the mean and standard deviation of u (neurons not refractory) and of
the synaptic current I of every population are averaged over forty snapshots
taken 3.7 ms apart (not a multiple of the network's oscillation period, so the
snapshots sample its phases).

Calls only oracle/ (and the seeded input generator):
    python tests/golden/make_relaxed_start.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                      # noqa: E402
from synth_inputs import standin_conn_table, standin_description   # noqa: E402

OUT = os.path.join(ROOT, "synth_inputs", "relaxed_start.json")
SETTLE, SNAPS, GAP = 20000, 40, 37


def main():
    net = O.OracleNet.build(1, 1.0, standin_conn_table().reshape(64))
    net.run(SETTLE)
    off = net.pop_offsets
    acc = {k: np.zeros(8) for k in ("u_mean", "u_sd", "i_mean", "i_sd")}
    for _ in range(SNAPS):
        net.run(GAP)
        net.spikes(clear=True)
        u, cur, refr = net.state()
        for a in range(8):
            sl = slice(off[a], off[a + 1])
            live = refr[sl] == 0
            acc["u_mean"][a] += u[sl][live].mean()
            acc["u_sd"][a] += u[sl][live].std()
            acc["i_mean"][a] += cur[sl].mean()
            acc["i_sd"][a] += cur[sl].std()
    out = {k: [round(float(v) / SNAPS, 4) for v in acc[k]] for k in acc}
    out["source"] = (f"oracle FP32 mirror, seed 1, full scale, {standin_description()}; "
                     f"moments averaged over {SNAPS} snapshots {GAP} steps apart after {SETTLE} steps")
    json.dump(out, open(OUT, "w"), indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
