"""Writes the stored oracle results under tests/golden/ (calls only the oracle).

sphere16_oracle.json: the 16^3 two-phase sphere cube (backward Euler, dt=1e-3,
20 steps, rtol 1e-10, T=0 on z=0) run by the CPU oracle: per-step PCG
iteration counts and relative residuals, and the final field at a few nodes.
It guards the oracle against unnoticed changes; it is not a paper value.

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle  # noqa: E402
from paper_1905_07622_amd import workloads as wl  # noqa: E402

PROBE_NODES = [17 * 17 * 8 + 17 * 8 + 8, 17 * 17 * 16, 17 * 17 * 1 + 3, 4912, 2000]


def main():
    p = wl.two_phase_sphere_cube()
    out = oracle.run(p)
    data = dict(
        problem="two-phase sphere cube 16^3, theta=1, dt=1e-3, 20 steps, rtol=1e-10",
        iters=[int(v) for v in out["iters"]],
        relres=[float(v) for v in out["relres"]],
        probe_nodes=PROBE_NODES,
        T_final_probe=[float(out["T_final"][i]) for i in PROBE_NODES],
        T_final_l2=float((out["T_final"] ** 2).sum() ** 0.5),
    )
    with open(os.path.join(HERE, "sphere16_oracle.json"), "w") as f:
        json.dump(data, f, indent=1)


if __name__ == "__main__":
    main()
