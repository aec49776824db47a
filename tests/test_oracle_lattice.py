"""Pins of the oracle's lattice tables (paper Sec. 2, Fig. "lattice").

The velocity sets are checked against the vectors the paper's figure draws
(tests/golden/lattice_vectors.txt); the weights, which the paper does not
print, are pinned by the isotropy identities that determine them (exact
rational arithmetic): sum w = 1, sum w c = 0, sum w c c = delta/3,
sum w c c c = 0, sum w c c c c = (dd + dd + dd)/9, and the half-space sum
sum_{c.n = 1} w = 1/6 used by the Zou-He closure.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lattice_vectors.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        q, cx, cy, cz = map(int, line.split())
        out.setdefault(q, []).append((cx, cy, cz))
    return out


@pytest.mark.parametrize("q", [9, 19, 27])
def test_vectors_match_paper_figure(oracle_mod, q):
    c, _, _ = oracle_mod.tables(q)
    assert [tuple(v) for v in c.tolist()] == _golden()[q]


@pytest.mark.parametrize("q", [9, 19, 27])
def test_opposite_table(oracle_mod, q):
    c, _, opp = oracle_mod.tables(q)
    for i in range(q):
        assert tuple(c[opp[i]]) == tuple(-c[i])
    assert opp[0] == 0


@pytest.mark.parametrize("q", [9, 19, 27])
def test_isotropy_exact(oracle_mod, q):
    c, w, _ = oracle_mod.tables(q)
    D = 2 if q == 9 else 3
    W = [Fraction(x).limit_denominator(10000) for x in w]
    for x, fr in zip(w, W):
        assert float(fr) == x                     # weights are the doubles nearest the rationals
    assert sum(W) == 1
    d = lambda a, b: 1 if a == b else 0
    for a in range(D):
        assert sum(W[i] * c[i, a] for i in range(q)) == 0
        for b in range(D):
            assert sum(W[i] * c[i, a] * c[i, b] for i in range(q)) == Fraction(d(a, b), 3)
            for g in range(D):
                assert sum(W[i] * c[i, a] * c[i, b] * c[i, g] for i in range(q)) == 0
    for a, b, g, e in itertools.product(range(D), repeat=4):
        lhs = sum(W[i] * c[i, a] * c[i, b] * c[i, g] * c[i, e] for i in range(q))
        rhs = Fraction(d(a, b) * d(g, e) + d(a, g) * d(b, e) + d(a, e) * d(b, g), 9)
        assert lhs == rhs


@pytest.mark.parametrize("q", [9, 19, 27])
def test_half_space_weight(oracle_mod, q):
    c, w, _ = oracle_mod.tables(q)
    D = 2 if q == 9 else 3
    for a in range(D):
        for sgn in (1, -1):
            tot = sum(Fraction(w[i]).limit_denominator(10000) for i in range(q) if c[i, a] == sgn)
            assert tot == Fraction(1, 6)


def test_2d_lattice_has_no_z_component(oracle_mod):
    c, _, _ = oracle_mod.tables(9)
    assert np.all(c[:, 2] == 0)
