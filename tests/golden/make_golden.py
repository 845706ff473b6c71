"""Write the full-size parity fixtures from the oracle alone.

For configurations 2 (1,000,000 triangles, 1,000 steps) and 3 (10,000,000 triangles, 500
steps) this runs the FP64 CPU oracle from the seeded initial state and stores, in input order,
the final state of a seeded sample of cells plus whole-field summaries (time, dt statistics,
clamp count, wet-cell count, mass, maxima).  Only `gen` and `oracle` are used.

    python tests/golden/make_golden.py [2] [3]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import gen      # noqa: E402
import oracle   # noqa: E402

N_SAMPLES = 2048


def sample_ids(n_cells: int, cfg: int) -> np.ndarray:
    rng = np.random.default_rng([cfg, 99])
    return np.sort(rng.choice(n_cells, size=N_SAMPLES, replace=False))


def make(cfg: int) -> str:
    case = gen.config(cfg)
    t0 = time.time()
    mesh = oracle.Mesh(case.xy, case.tri, case.edge_tag)
    area = mesh.arrays()[2]
    rc, h, hu, hv, dts, st = oracle.run_case(case, mesh=mesh)
    el = time.time() - t0
    assert rc == 0, rc
    ids = sample_ids(case.n_cells, cfg)
    out = {
        "what": f"oracle state of configuration {cfg} after {case.steps} steps from its seeded "
                f"initial state (gen.config({cfg})), FP64",
        "made_by": "tests/golden/make_golden.py (gen + oracle only)",
        "n_cells": case.n_cells, "steps": case.steps,
        "t": st["t"], "dt_min": st["dt_min"], "dt_max": st["dt_max"], "dt_sum": st["dt_sum"],
        "dt_first": float(dts[0]), "dt_last": float(dts[-1]),
        "clamps": st["clamps"],
        "wet_cells": int((h > case.h_dry).sum()),
        "mass": float(np.dot(h, area)), "mass0": float(np.dot(case.h, area)),
        "max_h": float(np.abs(h).max()), "max_hu": float(np.abs(hu).max()),
        "max_hv": float(np.abs(hv).max()),
        "ids": ids.tolist(),
        "h": h[ids].tolist(), "hu": hu[ids].tolist(), "hv": hv[ids].tolist(),
        "oracle_seconds": el, "oracle_threads": oracle.threads(),
    }
    path = os.path.join(HERE, f"config{cfg}_final.json")
    with open(path, "w") as f:
        json.dump(out, f)
    return path


if __name__ == "__main__":
    for a in (sys.argv[1:] or ["2", "3"]):
        print(make(int(a)), flush=True)
