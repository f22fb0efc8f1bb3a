"""Write the stored oracle results that the GPU tests compare against when the oracle
itself would take too long inside a test.

Only the FP64 oracle (oracle/) and the workload descriptions (skyr_inputs) are used.

  cube_b4_128_oracle.json   the B = 4 cube (O_h rational map of Table RMA, Sec. 4.1,
                            profile pi exp(-r/1.5)) on 128^3 at h = 0.15, m = 1, relaxed by
                            the arrested Newton flow with the energy rule (Sec. 3), dt = 0.015,
                            until max|F| < 1e-4 or 5000 steps: steps, arrests, E_prev of the
                            flow state every 250 steps (the energy of the field one accepted
                            step before), and the observables of the final field.

usage: python tests/golden/make_oracle_goldens.py [--threads T]
(about 0.2 s per step on 8 host threads)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from skyr_inputs import CUBE_B4_128  # noqa: E402


def cube_b4_128(out_path: str, chunk: int = 250) -> dict:
    w = CUBE_B4_128
    n, h, m, dt, tol, cap = w["n"], w["h"], w["m"], w["dt"], w["tol"], w["steps"]
    lam = w["init"]["prof_lambda"]
    phi = oracle.init_product((n, n, n), h, [oracle.cube_b4(prof_a=math.pi, prof_lambda=lam)])
    vel = np.zeros_like(phi)
    st = oracle.AnfState.fresh()
    e_at = {}
    t0 = time.time()
    while st.steps < cap and not st.converged:
        target = min(cap, st.steps + chunk)
        phi, vel, st, _, _ = oracle.anf(phi, vel, h, m, dt, tol, target, st, rule="energy")
        if not st.converged:
            e_at[int(st.steps)] = float(st.E_prev)
        print(f"steps {st.steps} arrests {st.arrests} E {st.E:.12f} max|F| {st.max_force:.3e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    obs = oracle.observables(phi, h, m)
    res = {
        "workload": w["name"], "n": n, "h": h, "m": m, "dt": dt, "tol": tol, "max_steps": cap,
        "init": w["init"], "rule": "energy",
        "steps": int(st.steps), "arrests": int(st.arrests), "converged": bool(st.converged),
        "max_force": float(st.max_force), "E_flow": float(st.E),
        "observables": {k: float(v) for k, v in obs.items()},
        "E_prev_after_steps": {str(k): v for k, v in sorted(e_at.items())},
        "source": "python tests/golden/make_oracle_goldens.py (FP64 oracle)",
    }
    with open(out_path, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0, help="oracle threads (0: its default)")
    args = ap.parse_args()
    if args.threads:
        oracle.set_num_threads(args.threads)
    cube_b4_128(os.path.join(HERE, "cube_b4_128_oracle.json"))


if __name__ == "__main__":
    main()
