"""Host-side checks of the benchmark's byte model (no GPU)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def brute_share(iters, R):
    """Direction launches of iterations 0..it-1 whose previous iteration ended
    with a plain update (not a residual replacement at i mod R == 0)."""
    corr = total = 0
    for it in iters:
        for j in range(it):
            total += 1
            corr += j > 0 and (j - 1) % R != 0
    return corr / total if total else 0.0


@pytest.mark.parametrize("iters,R", [([27] * 5, 50), ([0, 1, 2, 3], 50), ([120, 51, 50, 49], 50),
                                     ([7, 8, 9], 3), ([], 50)])
def test_deferred_share_matches_enumeration(iters, R):
    assert bench.deferred_fraction(iters, R) == pytest.approx(brute_share(iters, R), abs=0)


def test_byte_model_per_node():
    N, E = 1000, 729
    ab0 = bench.algorithmic_bytes(N, E, 8, 0.0)
    ab1 = bench.algorithmic_bytes(N, E, 8, 1.0)
    assert ab0["gather"] == (5 * N + 2 * E) * 8
    assert ab1["gather"] - ab0["gather"] == 16 * N  # x read and written once
    assert ab0["update"] == ab1["update"] == 32 * N  # r, q, P^-1 read; r written


def test_byte_model_one_reduction():
    N, E = 1000, 729
    ab0 = bench.algorithmic_bytes(N, E, 8, 0.0, "one-reduction")
    ab1 = bench.algorithmic_bytes(N, E, 8, 1.0, "one-reduction")
    assert ab0["gather"] == (5 * N + 2 * E) * 8  # as the two-kernel direction kernel
    assert ab1["gather"] - ab0["gather"] == 32 * N  # + q read, r written, x read and written
    assert ab1["update"] == 0


def test_byte_model_one_kernel():
    """Both halves of the iteration in one launch: the two kernels' bytes
    minus q written and read and r and P^-1 read again (q, r and P^-1 at the
    own nodes stay on chip), so the direction kernel's bytes with r written
    in place of q; the deferred x as before."""
    N, E = 1000, 729
    for f in (0.0, 0.5, 1.0):
        two = bench.algorithmic_bytes(N, E, 8, f)
        one = bench.algorithmic_bytes(N, E, 8, f, "one-kernel")
        assert one["update"] == 0
        assert one["gather"] == two["gather"]
        assert one["gather"] == two["gather"] + two["update"] - 4 * N * 8
