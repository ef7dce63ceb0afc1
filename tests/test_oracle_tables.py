"""The oracle's lattice tables against Table 1 and the paper's identities.

Pins: the Table 1 fixture (tests/golden/table1_weights.txt), the normalisations
eq. (weights_1) and eq. (weights_2), the claimed 8th-order isotropy
(section III), and the 12/7 surface-tension factor (section III) that follows
from the fourth moments.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from tests import paper_tables as T


def test_fixture_link_counts_match_figure():
    # Belt 1 has 8 speeds on levels 1, 2; belt 2 has 16 on levels 4, 5, 8.
    assert len(T.BELT1) == 8 and len(T.BELT2) == 16
    for level, (_, links) in T.P.items():
        assert sum(1 for c in T.BLOCK if T.c2(c) == level) == links


def test_normalisations_exact():
    # eq. (weights_1): sum w = 1 and sum p_s + sum p_m = 1 (with the rest link).
    assert T.W[0][0] + sum(T.w_of(c) for c in T.BELT1) == 1
    assert T.p_rest() == Fraction(247, 420)
    assert sum(T.p_of(c) for c in T.BLOCK) == Fraction(173, 420)
    # eq. (weights_2): second moments equal c_s^2 = 1/3 for both weight sets.
    assert sum(T.w_of(c) * c[0] ** 2 for c in T.BELT1) == T.CS2
    assert sum(T.p_of(c) * c[0] ** 2 for c in T.BLOCK) == T.CS2
    assert sum(T.p_of(c) * c[1] ** 2 for c in T.BLOCK) == T.CS2


def _mom(a, b):
    return sum(T.p_of(c) * c[0] ** a * c[1] ** b for c in T.BLOCK)


def test_isotropy_to_eighth_order():
    # Odd moments vanish by symmetry; even moments follow the isotropic
    # ratios of a 2D rank-2n tensor up to n = 4 (section III: 8th order).
    assert _mom(4, 0) == 3 * _mom(2, 2)
    assert _mom(6, 0) * 3 == _mom(4, 2) * 15
    assert _mom(8, 0) * 15 == _mom(6, 2) * 105
    assert _mom(8, 0) * 9 == _mom(4, 4) * 105
    # ... but not to 10th order.
    assert _mom(10, 0) * 105 != _mom(8, 2) * 945


def test_twelve_sevenths():
    # The fourth-order coefficient of the G2 force relative to c_s^4 is 12/7
    # (section III: C2 G <-> G1 + 12/7 G2); for the D2Q9 w it is 1.
    assert _mom(2, 2) / T.CS2 ** 2 == Fraction(12, 7)
    d2q9 = sum(T.w_of(c) * c[0] ** 2 * c[1] ** 2 for c in T.BELT1)
    assert d2q9 / T.CS2 ** 2 == 1


def test_oracle_d2q9_matches_fixture():
    cx, cy, w = O.d2q9()
    vecs = list(zip(cx.tolist(), cy.tolist()))
    assert vecs[0] == (0, 0) and sorted(vecs[1:]) == sorted(T.BELT1)
    assert w[0] == float(T.W[0][0])
    for (x, y), wi in zip(vecs[1:], w[1:]):
        assert wi == float(T.w_of((x, y)))


@pytest.mark.parametrize("G1,G2", [(1.0, 0.0), (0.0, 1.0)])
def test_oracle_link_table_unit_couplings(G1, G2):
    cx, cy, K, KE = O.tables(G1, G2)
    vecs = list(zip(cx.tolist(), cy.tolist()))
    assert sorted(vecs) == sorted(T.BLOCK)
    assert vecs[:8] == [tuple(v) for v in zip(*O.d2q9()[:2])][1:]
    for k, c in enumerate(vecs):
        assert K[k] == float(T.coupling(c, Fraction(int(G1)), Fraction(int(G2))))
        assert KE[1 + k] == K[k]
    rest = T.W[0][0] if G1 == 1.0 else T.p_rest()
    assert KE[0] == float(rest)


def test_oracle_link_table_general_couplings():
    G1, G2 = -5.444444444444445, 0.5444444444444445
    cx, cy, K, KE = O.tables(G1, G2)
    for k, c in enumerate(zip(cx.tolist(), cy.tolist())):
        exact = T.coupling(c, Fraction(G1), Fraction(G2))
        assert abs(K[k] - float(exact)) <= 4 * np.spacing(abs(float(exact)) + 1e-300)
    # Newton's third law: every link has its opposite with the same coupling.
    vecs = list(zip(cx.tolist(), cy.tolist()))
    for k, (x, y) in enumerate(vecs):
        assert K[vecs.index((-x, -y))] == K[k]
