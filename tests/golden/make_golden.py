"""Write tests/golden/oracle_optima.json: the CPU oracle's canonical optima
(Algorithm 1 with the exact keys of eqs. (12)-(20)) for full-size windows
whose oracle run is too slow to repeat inside a GPU test.

Calls only oracle/ and the seeded generator; run on the CPU:
    python tests/golden/make_golden.py
"""

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

# (config, window index): the smallest and a large window of the 640x480
# batch, the three smallest and the three largest windows of the 1280x720
# batch (with hot pixels; 4.8-4.9M events plus the hot pixels' ~230k), and
# extra 346x260 windows.
CASES = [("c3", 56), ("c3", 9), ("c3", 11), ("c5", 179), ("c5", 110), ("c5", 138),
         ("c5", 64), ("c5", 2), ("c5", 95),
         ("c2", 2), ("c2", 3), ("c2", 4), ("c2", 5)]


def solve(case):
    from oracle import oracle as O
    from synth import config_windows

    cfg, k = case
    w = config_windows(cfg, [k])[0]
    s = w.spec
    t0 = time.time()
    r = O.bnb(O.Events.of_window(w), s.d_lo, s.d_hi, s.eps)
    return {"config": cfg, "window": k, "n_events": w.n, "j_star": r.j_star, "K": str(r.K),
            "d_hat": r.d_hat, "L": r.L, "nodes_expanded": r.nodes_expanded, "oracle_seconds": time.time() - t0}


def main():
    from oracle import oracle as O

    O.build(force=False)
    with ProcessPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        rows = list(ex.map(solve, CASES))
    out = {"source": "oracle/ecmd_oracle.c orc_bnb (canonical optimum, gamma = 0)",
           "method": "Algorithm 1 with the bound of eqs. (15)-(20) on the fp32 warp of eq. (12)",
           "windows": rows}
    with open(os.path.join(HERE, "oracle_optima.json"), "w") as f:
        json.dump(out, f, indent=1)
    for r in rows:
        print(r, flush=True)


if __name__ == "__main__":
    main()
