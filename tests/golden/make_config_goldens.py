#!/usr/bin/env python3
"""Write the oracle's full DD, DR and RR counts of the small (10k + 10k) and
1M (1M + 1M) workloads into tests/golden/ -- test infrastructure.

The paper validates its GPU code by comparing the DR histogram with a CPU run
on the same galaxies (Sec. 2.2, CPU-GPU consistency); these files hold that
CPU side at the workloads' full sizes, so the GPU tests can compare the exact
launch the benchmark times with it bit for bit.

Only the CPU oracle (oracle/) and the seeded input generators (synth/) are
used: no value here comes from the GPU library.  Each file records the
SHA-256 of every input array (RA, Dec, edges, as little-endian binary64), so
a test can tell whether the generator on its machine still draws the same
catalogues; if not, the file does not apply and this script must be run again.

    python3 tests/golden/make_config_goldens.py small     # seconds
    python3 tests/golden/make_config_goldens.py 1m        # ~20-40 min on 8-16 cores
"""
from __future__ import annotations

import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

CONFIGS = {
    # name: (generator, golden file)
    "small": (lambda: synth.config_small(), "config_small_10k.json"),
    "1m": (lambda: synth.config_1m(), "config_1m.json"),
}


def sha256(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()


def input_hashes(c) -> dict:
    return {"D_ra": sha256(c["D"][0]), "D_dec": sha256(c["D"][1]), "R_ra": sha256(c["R"][0]),
            "R_dec": sha256(c["R"][1]), "edges": sha256(c["edges"])}


def golden_path(name: str) -> str:
    return os.path.join(HERE, CONFIGS[name][1])


def make(name: str) -> dict:
    c = CONFIGS[name][0]()
    D, R, e = c["D"], c["R"], c["edges"]
    out = {"workload": c["name"], "n_data": int(D[0].size), "n_random": int(R[0].size),
           "theta_edges_deg": [float(x) for x in e], "input_sha256": input_hashes(c)}
    times = {}
    counts = {}
    for key, kw in (("DD", {}), ("DR", {"B": R, "auto": False}), ("RR", None)):
        t = time.time()
        if kw is None:
            counts[key] = oracle.count(R, e)
        else:
            counts[key] = oracle.count(D, e, **kw)
        times[key] = round(time.time() - t, 1)
        print(f"{name} {key}: {times[key]} s", file=sys.stderr, flush=True)
    nD, nR = D[0].size, R[0].size
    assert int(counts["DD"].sum()) == nD * (nD - 1) // 2
    assert int(counts["DR"].sum()) == nD * nR
    assert int(counts["RR"].sum()) == nR * (nR - 1) // 2
    out["counts"] = {k: [int(x) for x in v] for k, v in counts.items()}
    out["oracle"] = {"threads": oracle.num_threads(), "seconds": times, "cpu": platform.processor() or "",
                     "command": f"python3 tests/golden/make_config_goldens.py {name}"}
    return out


def main(argv):
    names = argv[1:] or ["small"]
    for name in names:
        if name not in CONFIGS:
            raise SystemExit(f"unknown config {name!r}; choose from {sorted(CONFIGS)}")
        g = make(name)
        tmp = golden_path(name) + ".tmp"
        with open(tmp, "w") as f:
            json.dump(g, f, indent=1)
            f.write("\n")
        os.replace(tmp, golden_path(name))
        print(f"wrote {golden_path(name)}", file=sys.stderr)


if __name__ == "__main__":
    main(sys.argv)
