"""The oracle reproduces its stored sphere-cube results (written by
tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np

from oracle import oracle
from paper_1905_07622_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sphere16_oracle.json")


def test_sphere_cube_matches_stored_oracle_results():
    with open(GOLDEN) as f:
        g = json.load(f)
    out = oracle.run(wl.two_phase_sphere_cube())
    assert list(out["iters"]) == g["iters"]
    np.testing.assert_allclose(out["relres"], g["relres"], rtol=1e-6)
    np.testing.assert_allclose(out["T_final"][g["probe_nodes"]], g["T_final_probe"], rtol=1e-12, atol=1e-14)
    assert abs(np.linalg.norm(out["T_final"]) - g["T_final_l2"]) < 1e-10 * g["T_final_l2"]
