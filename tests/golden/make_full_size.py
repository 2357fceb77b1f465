"""Write tests/golden/full_size.json: global energy, virial and interacting-pair count of every
full-size workload, from the FP64 brute-force oracle (all N^2 minimum-image pairs).

Calls only oracle/ (and the seeded input generators).  Usage:
    OMP_NUM_THREADS=6 python tests/golden/make_full_size.py [names...]
Each configuration is appended as soon as it finishes (minutes to about an hour each)."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1408_4599_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")
NAMES = ["c5_4site_200k", "c4_2cljq_500k", "c2_lj_1m", "c3_lj_slab_2m"]


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        if name in data:
            continue
        cfg = W.make(name)
        t = time.time()
        r = O.forces(cfg["model"], cfg["pos"], cfg["quat"], cfg["comp"], cfg["box"])
        data[name] = {"N": int(cfg["pos"].shape[0]), "U": r["U"], "W": r["W"], "Wd": [float(x) for x in r["Wd"]],
                      "npairs": r["npairs"], "oracle_seconds": time.time() - t, "threads": O.num_threads(),
                      "source": "oracle/oracle.c oracle_all (FP64, all pairs, minimum image)"}
        json.dump(data, open(OUT, "w"), indent=1)
        print(name, data[name], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or NAMES)
