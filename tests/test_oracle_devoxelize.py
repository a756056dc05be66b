"""Pins of the de-voxelisation oracle: per-element brute force over explicit
Python lists, hand cases (single slot, empty segment, ties), and central
finite differences of the forward for both reductions (max is linear away
from ties, so the difference quotient is exact there)."""

import numpy as np
import pytest

import oracle


def _case(seed, G=7, U=9, C=5, max_slots=4):
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, max_slots + 1, G)
    counts[0] = 0  # an empty segment
    offs = np.concatenate([[0], np.cumsum(counts)])
    vu = rng.integers(0, U, offs[-1])
    pred = rng.standard_normal((U, C))
    return offs, vu, pred


@pytest.mark.parametrize("reduce", ["max", "mean"])
def test_matches_per_element_brute_force(reduce):
    offs, vu, pred = _case(1)
    out, arg = oracle.devoxelize(offs, vu, pred, reduce)
    for g in range(offs.size - 1):
        slots = list(range(offs[g], offs[g + 1]))
        for c in range(pred.shape[1]):
            vals = [float(pred[vu[m], c]) for m in slots]
            if not vals:
                assert out[g, c] == 0.0
                if reduce == "max":
                    assert arg[g, c] == -1
            elif reduce == "max":
                assert out[g, c] == max(vals)
                assert arg[g, c] == slots[vals.index(max(vals))]  # first of any tie
            else:
                assert out[g, c] == pytest.approx(sum(vals) / len(vals), abs=1e-15)


def test_hand_cases():
    pred = np.array([[1.0, -2.0], [3.0, -2.0], [0.5, 7.0]])
    offs = np.array([0, 1, 1, 4])  # one slot, empty, three slots
    vu = np.array([2, 0, 1, 0])
    out, arg = oracle.devoxelize(offs, vu, pred, "max")
    np.testing.assert_array_equal(out, [[0.5, 7.0], [0.0, 0.0], [3.0, -2.0]])
    np.testing.assert_array_equal(arg, [[0, 0], [-1, -1], [2, 1]])  # -2 ties: first slot wins
    out_m, _ = oracle.devoxelize(offs, vu, pred, "mean")
    np.testing.assert_allclose(out_m[2], [5.0 / 3.0, -2.0])


@pytest.mark.parametrize("reduce", ["max", "mean"])
def test_backward_matches_finite_differences(reduce):
    offs, vu, pred = _case(2)
    U, C = pred.shape
    gout = np.random.default_rng(3).standard_normal((offs.size - 1, C))
    out, arg = oracle.devoxelize(offs, vu, pred, reduce)
    grad = oracle.devoxelize_backward(offs, vu, U, gout, reduce, arg)
    h = 1e-6
    for u in range(U):
        for c in range(C):
            p1, p0 = pred.copy(), pred.copy()
            p1[u, c] += h
            p0[u, c] -= h
            f1 = (oracle.devoxelize(offs, vu, p1, reduce)[0] * gout).sum()
            f0 = (oracle.devoxelize(offs, vu, p0, reduce)[0] * gout).sum()
            assert (f1 - f0) / (2 * h) == pytest.approx(grad[u, c], abs=1e-8)
