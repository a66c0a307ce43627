"""Pins of the oracle's exact orientation predicate and E-F hit test.

The oracle's signs are checked against exact rational arithmetic
(``fractions``), on generic points and on points built on or one ulp away
from degeneracies, and its hit test against a crossing-point formulation of
the same definition.
"""
import numpy as np
import pytest

import oracle
from tests.exact_ref import adversarial_points, ef_hit_parametric, orient_exact, sign

pytestmark = pytest.mark.filterwarnings("ignore")


def test_sign_convention_front_is_right_hand_normal():
    a, b, c = (0, 0, 0), (1, 0, 0), (0, 1, 0)  # counter-clockwise seen from +z
    assert oracle.orient_sign(a, b, c, (0.2, 0.2, 1.0)) == 1
    assert oracle.orient_sign(a, b, c, (0.2, 0.2, -1.0)) == -1
    assert oracle.orient_sign(a, b, c, (5.0, -3.0, 0.0)) == 0


@pytest.mark.parametrize("seed", [0, 1])
def test_orient_matches_rationals_adversarial(seed):
    rng = np.random.default_rng(seed)
    pts = adversarial_points(rng, 600)
    zero = 0
    for a, b, c, p in pts:
        want = sign(orient_exact(a, b, c, p))
        zero += want == 0
        assert oracle.orient_sign(a, b, c, p) == want
        assert oracle.orient_sign_exact(a, b, c, p) == want
    assert zero > 100  # the set really exercises exact zeros


def test_orient_extreme_magnitudes():
    rng = np.random.default_rng(7)
    for scale in (2.0 ** -190, 2.0 ** -60, 1.0, 2.0 ** 60, 2.0 ** 190):
        for _ in range(50):
            a, b, c, p = rng.normal(size=(4, 3)) * scale
            assert oracle.orient_sign(a, b, c, p) == sign(orient_exact(a, b, c, p))


def test_orient_antisymmetry_and_cyclic():
    rng = np.random.default_rng(3)
    for a, b, c, p in adversarial_points(rng, 200):
        s = oracle.orient_sign(a, b, c, p)
        assert oracle.orient_sign(b, c, a, p) == s
        assert oracle.orient_sign(b, a, c, p) == -s


HAND = [
    # (p, q, a, b, c, expected)
    ("through interior", (0.2, 0.2, -1), (0.2, 0.2, 1), 1),
    ("reverse direction", (0.2, 0.2, 1), (0.2, 0.2, -1), 2),
    ("endpoint on plane", (0.2, 0.2, 0), (0.2, 0.2, 1), 0),
    ("coplanar edge", (-1, 0.2, 0), (2, 0.2, 0), 0),
    ("misses outside", (2, 2, -1), (2, 2, 1), 0),
    ("through a triangle edge", (0.5, 0.0, -1), (0.5, 0.0, 1), 1),
    ("through a triangle vertex", (0.0, 0.0, -1), (0.0, 0.0, 1), 1),
    ("through the hypotenuse", (0.5, 0.5, 1), (0.5, 0.5, -1), 2),
    ("just outside the hypotenuse", (0.5, 0.5 + 2.0 ** -40, 1), (0.5, 0.5 + 2.0 ** -40, -1), 0),
]


@pytest.mark.parametrize("name,p,q,expected", HAND, ids=[h[0] for h in HAND])
def test_hand_cases(name, p, q, expected):
    a, b, c = (0, 0, 0), (1, 0, 0), (0, 1, 0)
    assert oracle.ef_hit(p, q, a, b, c) == expected
    assert ef_hit_parametric(np.array(p, float), np.array(q, float), np.array(a, float),
                             np.array(b, float), np.array(c, float)) == expected


def test_zero_area_triangle_never_hits():
    a, b, c = (0, 0, 0), (1, 1, 1), (2, 2, 2)
    assert oracle.ef_hit((0.5, 0.6, -1), (0.5, 0.4, 2), a, b, c) == 0


def test_shared_edge_crossing_hits_both_faces():
    # two triangles sharing the edge (0,0,0)-(1,0,0); a segment through that edge
    a, b = (0, 0, 0), (1, 0, 0)
    c1, c2 = (0, 1, 0), (0, -1, 0)
    p, q = (0.5, 0, -1), (0.5, 0, 1)
    assert oracle.ef_hit(p, q, a, b, c1) == 1
    assert oracle.ef_hit(p, q, b, a, c2) == 1  # same orientation (+z front)


def test_hit_matches_parametric_random_snapped():
    rng = np.random.default_rng(11)
    n_hit = 0
    for _ in range(3000):
        P = rng.integers(-4, 5, (5, 3)).astype(float) / 4.0
        p, q, a, b, c = P
        want = ef_hit_parametric(p, q, a, b, c)
        n_hit += want != 0
        assert oracle.ef_hit(p, q, a, b, c) == want
    assert n_hit > 50
