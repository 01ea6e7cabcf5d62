"""Write the stored expected values of the full-size multi-step parity tests.

Runs the FP64 oracle (oracle/) on the named workloads (workloads/) and stores, per case,
the subspace sizes it chose, the energies and a seeded sample of the free DOFs of u and v
after the last step, with max |u| and max |v| over all DOFs (the normalisation of the
element-wise error).  Nothing here touches the HIP library.

Usage: python -m tests.golden.make_fullsize_golden [case ...]   (cases: c2dt1e-3 c3 c4)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.stepper import Propagator  # noqa: E402
from workloads import config  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLE = 2048

# name: (workload, overrides, steps, Krylov settings) - the launch settings the benchmark uses
CASES = {
    "c2dt1e-3": ("c2", dict(dt=1e-3), 1, dict(m_max=64, m_fixed=56, k_fixed=32)),
    "c3": ("c3", dict(dt=1e-4), 3, dict(m_max=64)),
    "c4": ("c4", dict(dt=1e-3), 3, dict(m_max=64)),
}


def path_of(case):
    return os.path.join(HERE, f"fullsize_{case}.json")


def make(case):
    name, over, steps, kw = CASES[case]
    p = config(name, **over)
    t0 = time.perf_counter()
    orc = Propagator(p, **kw)
    for i in range(steps):
        orc.step(p.dt)
        print(f"{case}: step {i + 1}/{steps} done, {time.perf_counter() - t0:.0f} s", flush=True)
    u, v = orc.u(), orc.v()
    rng = np.random.default_rng(1234)
    idx = np.sort(rng.choice(orc.free, size=min(N_SAMPLE, orc.N), replace=False))
    ke, se, we = orc.energies()
    rec = {
        "case": case, "workload": name, "overrides": over, "steps": steps, "krylov": kw,
        "n_nodes": int(p.n_nodes), "t": orc.t,
        "m_corr": [int(r["corr"]["m"][0]) for r in orc.log],
        "k_corr": [int(r["corr"]["k"]) for r in orc.log],
        "m_pred": [int(r["pred"]["m"][0]) for r in orc.log if "pred" in r],
        "energies": [ke, se, we],
        "max_abs_u": float(np.abs(u).max()), "max_abs_v": float(np.abs(v).max()),
        "dofs": idx.tolist(), "u": [float(a) for a in u[idx]], "v": [float(a) for a in v[idx]],
        "oracle_seconds": time.perf_counter() - t0,
    }
    with open(path_of(case), "w") as fh:
        json.dump(rec, fh, indent=0)
    print(f"wrote {path_of(case)}")


if __name__ == "__main__":
    for c in (sys.argv[1:] or sorted(CASES)):
        make(c)
