"""Host check of the width bracket in the GPU-side enumeration's adaptive filter.

For a candidate between the fixed cut and its q-point bound, the fused kernel
first forms the adaptive width from the per-mode projection table
P_g[d] = (v_g . b_d) * (1 / N_d) (pair differences of table entries) and keeps
or drops the candidate without the enumerator's own arithmetic unless |Delta|
falls inside a bracket around it: the norm of the nine pair projections must
lie within [n'(1 - 1e-13) - e, n'(1 + 1e-13) + e] of the table's norm n', with
e = 3e-12 max_{g,d} sum_k |v_gk b_dk| / N_d.  The enumerator forms each pair
projection as ((v_i - v_j) . b_d) / N_d, summed left to right.  This test
emulates both forms in double precision (the table with and without fused
multiply-adds) on random, nearly equal and large-but-close velocities, and
checks that the enumerator's norm always lies inside the bracket, so the
kernel's early decisions agree with the enumerator's.  The host enumerator's
order-4 adaptive filter takes the same early decisions from the same table
(formed without fused multiply-adds, pairs summed in slot order).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

REL = 1e-13


def fma(a, b, c):
    """Correctly rounded a * b + c."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def table(v, b, n, fused):
    out = []
    for d in range(3):
        if fused:
            s = fma(v[2], b[d, 2], fma(v[1], b[d, 1], v[0] * b[d, 0]))
        else:
            s = (v[0] * b[d, 0] + v[1] * b[d, 1]) + v[2] * b[d, 2]
        out.append(s * (1.0 / n[d]))
    return out


def enumerator_norm(vs, b, n):
    s2 = 0.0
    for i, j in ((0, 1), (0, 2), (1, 2)):
        w = [vs[i][k] - vs[j][k] for k in range(3)]
        for d in range(3):
            p = ((w[0] * b[d, 0] + w[1] * b[d, 1]) + w[2] * b[d, 2]) / n[d]
            s2 = s2 + p * p
    return math.sqrt(s2)


def table_norm(vs, b, n, fused):
    P = [table(v, b, n, fused) for v in vs]
    s2 = 0.0
    for i, j in ((0, 1), (0, 2), (1, 2)):
        for d in range(3):
            t = P[i][d] - P[j][d]
            s2 += t * t
    return math.sqrt(s2)


def bound_scale(vs, b, n):
    return max(sum(abs(v[k] * b[d, k]) for k in range(3)) / n[d] for v in vs for d in range(3))


@pytest.mark.parametrize("kind", ["random", "near_equal", "large_close", "zero_difference"])
def test_enumerator_width_inside_bracket(kind):
    rng = np.random.default_rng({"random": 1, "near_equal": 2, "large_close": 3, "zero_difference": 4}[kind])
    worst = 0.0
    for _ in range(400):
        b = rng.uniform(-2.0, 2.0, size=(3, 3))
        n = [float(x) for x in rng.choice([3, 4, 8, 16, 20, 32], size=3)]
        v0 = rng.uniform(-60.0, 60.0, size=3)
        if kind == "random":
            vs = [rng.uniform(-60.0, 60.0, size=3) for _ in range(3)]
        elif kind == "near_equal":
            vs = [v0 + rng.uniform(-1e-9, 1e-9, size=3) for _ in range(3)]
        elif kind == "large_close":
            vs = [v0 * 1e3 + rng.uniform(-1e-3, 1e-3, size=3) for _ in range(3)]
        else:
            vs = [v0.copy() for _ in range(3)]
        vs = [[float(x) for x in v] for v in vs]
        exact = enumerator_norm(vs, b, n)
        e = 3e-12 * bound_scale(vs, b, n)
        for fused in (False, True):
            nrm = table_norm(vs, b, n, fused)
            lo = nrm * (1.0 - REL) - e
            hi = nrm * (1.0 + REL) + e
            assert lo <= exact <= hi, (kind, fused, exact, nrm, e)
            worst = max(worst, abs(exact - nrm) / max(e, 1e-300))
    # the margin is generous: the observed difference stays far below it
    assert worst < 0.05
