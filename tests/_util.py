"""Shared helpers of the GPU parity tests (comparison and case naming)."""
import sys

import numpy as np
import scipy.sparse as sp

from oracle import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def abs_operator(prob, cm, ck):
    """|A| of the assembled operator as a scipy CSR (for elementwise error bounds)."""
    A = oracle.CSR(prob, cm, ck)
    rowptr, col, val = A.to_arrays()
    A.close()
    return sp.csr_matrix((np.abs(val), col, rowptr), shape=(prob.n_nodes, prob.n_nodes))


def assert_apply_close(y, prob, cm, ck, x, rel):
    """|y - A x| <= rel * (|A| |x|) elementwise, A x from the oracle's CSR."""
    ref = oracle.operator_apply(prob, cm, ck, x)
    bound = abs_operator(prob, cm, ck) @ np.abs(x)
    err = np.abs(np.asarray(y) - ref)
    worst = float(np.max(err / np.maximum(bound, 1e-300)))
    assert np.all(err <= rel * bound + 1e-300), f"worst relative error {worst:.3e} > {rel:.1e}"
    return worst


def to_np(a):
    if a is None:
        return None
    if type(a).__module__.startswith("torch"):
        return a.detach().cpu().numpy()
    return np.asarray(a)
