"""Pins of the oracle's Clebsch-Gordan coefficients (CPU only)."""
import itertools
import math

import pytest

from oracle.cg import cg


def test_known_values():
    r2 = 1 / math.sqrt(2)
    assert cg(1, 1, 1, -1, 0, 0) == pytest.approx(r2, abs=1e-15)
    assert cg(1, -1, 1, 1, 0, 0) == pytest.approx(-r2, abs=1e-15)
    assert cg(1, 1, 1, -1, 2, 0) == pytest.approx(r2, abs=1e-15)
    assert cg(2, 0, 2, 0, 0, 0) == pytest.approx(-1 / math.sqrt(3), abs=1e-15)
    assert cg(2, 0, 2, 0, 2, 0) == pytest.approx(0.0, abs=1e-15)
    assert cg(2, 0, 2, 0, 4, 0) == pytest.approx(math.sqrt(2 / 3), abs=1e-15)
    # stretched state
    for j1, j2 in ((7, 5), (3, 3), (11, 1)):
        assert cg(j1, j1, j2, j2, j1 + j2, j1 + j2) == pytest.approx(1.0, abs=1e-15)


def test_spin_half_coupling_closed_form():
    """<l m-1/2 1/2 1/2 | j=l+1/2 m> = sqrt((l+m+1/2)/(2l+1)) (textbook closed form)."""
    for l in range(0, 6):
        tl, tj = 2 * l, 2 * l + 1
        for tm in range(-tj + 2, tj + 1, 2):
            want = math.sqrt((l + tm / 2 + 0.5) / (2 * l + 1))
            assert cg(tl, tm - 1, 1, 1, tj, tm) == pytest.approx(want, abs=1e-14)


@pytest.mark.parametrize("tj1,tj2", [(1, 1), (5, 3), (7, 7), (3, 11), (5, 5)])
def test_orthogonality(tj1, tj2):
    """sum_{m1 m2} <j1 m1 j2 m2|J M><j1 m1 j2 m2|J' M> = delta_JJ' (and the column relation)."""
    Js = range(abs(tj1 - tj2), tj1 + tj2 + 1, 2)
    for tM in range(-(tj1 + tj2), tj1 + tj2 + 1, 2):
        pairs = [(m1, tM - m1) for m1 in range(-tj1, tj1 + 1, 2) if abs(tM - m1) <= tj2]
        for J, K in itertools.product(Js, Js):
            s = sum(cg(tj1, m1, tj2, m2, J, tM) * cg(tj1, m1, tj2, m2, K, tM) for m1, m2 in pairs)
            want = 1.0 if (J == K and abs(tM) <= J) else 0.0
            assert s == pytest.approx(want, abs=1e-13)
        for (a, b), (c, d) in itertools.product(pairs, pairs):
            s = sum(cg(tj1, a, tj2, b, J, tM) * cg(tj1, c, tj2, d, J, tM) for J in Js)
            assert s == pytest.approx(1.0 if (a, b) == (c, d) else 0.0, abs=1e-13)


def test_exchange_symmetry():
    for tj1, tj2 in ((5, 3), (7, 7), (1, 3)):
        for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
            for m1 in range(-tj1, tj1 + 1, 2):
                for m2 in range(-tj2, tj2 + 1, 2):
                    ph = (-1) ** ((tj1 + tj2 - tJ) // 2)
                    assert cg(tj2, m2, tj1, m1, tJ, m1 + m2) == pytest.approx(
                        ph * cg(tj1, m1, tj2, m2, tJ, m1 + m2), abs=1e-15)
