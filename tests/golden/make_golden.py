"""Write the stored expected values of the long slit runs.

Every number written here comes from the FP64 CPU oracle (``oracle/``) run on
the seeded inputs of ``paper_0712_2247_amd.workloads``; nothing comes from the
GPU library.  Usage:

    python tests/golden/make_golden.py slit_64   # 64x64x136 slit, 20000 steps
    python tests/golden/make_golden.py columns   # laterally uniform reductions

``slit_64`` runs the full three-dimensional 64x64x136 slit (sigma 8, eta 0.25,
tau 0.8, g 2e-6, +-0.5% noise; at eta 0.30 and above the scheme diverges) and stores the
layer profiles n(z), u(z) at several step counts, plus the total mass.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_0712_2247_amd import workloads  # noqa: E402


def _dump(path, obj):
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(obj, fh, indent=1)
    os.replace(tmp, path)


def slit_64(snapshots=(1000, 5000, 10000, 20000)):
    wl = workloads.slit_64_f32_stable()
    n, u = wl.fields()
    o = oracle.Oracle(**wl.params())
    o.init(n, u)
    out = {"workload": wl.name, "source": "oracle FP64, full 3-D grid",
           "threads": oracle.max_threads(), "snapshots": {}}
    path = os.path.join(HERE, "slit_64x64x136_eta0.25_profiles.json")
    done = 0
    t0 = time.time()
    for s in snapshots:
        o.step(s - done)
        done = s
        pn, pu = o.profiles()
        nn, _ = o.moments()
        out["snapshots"][str(s)] = {"n_z": pn.tolist(), "u_z": pu.tolist(),
                                    "mass": float(nn.sum())}
        out["seconds"] = time.time() - t0
        _dump(path, out)
        print(f"step {s}: {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "slit_64"
    if what == "slit_64":
        slit_64()
    else:
        raise SystemExit(f"unknown target {what}")
