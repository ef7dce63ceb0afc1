"""Exact lattice tables rebuilt from the paper's Table 1 fixture (tests only).

The links are enumerated from the two-belt figure caption (belt 1: the 8
speeds with |c|^2 in {1, 2}; belt 2: the 16 speeds with |c|^2 in {4, 5, 8}),
not copied from either implementation, and every weight is a Fraction.
"""
import os
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))


def load_golden():
    p, w, cs2 = {}, {}, None
    with open(os.path.join(HERE, "golden", "table1_weights.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            kind, c2, val, links = line.split()
            if kind == "p":
                p[int(c2)] = (Fraction(val), int(links))
            elif kind == "w":
                w[int(c2)] = (Fraction(val), int(links))
            elif kind == "cs2":
                cs2 = Fraction(val)
    return p, w, cs2


P, W, CS2 = load_golden()

# Every integer vector of the 5x5 block except the origin.
BLOCK = [(x, y) for y in range(-2, 3) for x in range(-2, 3) if (x, y) != (0, 0)]
BELT1 = [c for c in BLOCK if c[0] ** 2 + c[1] ** 2 in (1, 2)]
BELT2 = [c for c in BLOCK if c[0] ** 2 + c[1] ** 2 in (4, 5, 8)]


def c2(c):
    return c[0] ** 2 + c[1] ** 2


def p_of(c):
    return P[c2(c)][0]


def w_of(c):
    return W[c2(c)][0]


def p_rest():
    """Rest weight of the first belt implied by eq. (weights_1)."""
    return 1 - sum(p_of(c) for c in BLOCK)


def coupling(c, G1, G2):
    """Exact coupling of link c in eq. (FORCE) (G1, G2 Fractions or floats)."""
    if c in BELT1:
        return G1 * w_of(c) + G2 * p_of(c)
    return G2 * p_of(c)
