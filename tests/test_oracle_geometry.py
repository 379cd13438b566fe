"""Oracle site indexing against hand-worked values of eq. (lexi) / eq. (ipt) and bijection properties."""
import os

import numpy as np
import pytest

from oracle import geometry as geo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "index_points.txt")


def _rows():
    for line in open(GOLDEN):
        line = line.split("#")[0].split()
        if line:
            yield [int(v) for v in line]


@pytest.mark.parametrize("row", list(_rows()))
def test_golden_index_points(row):
    L, B, x = row[0:4], row[4:8], row[8:12]
    lam, par, xhat = row[12:15]
    assert int(geo.lex(x, L)) == lam
    assert int(geo.parity(x)) == par
    assert int(geo.ipt(x, L, B)) == xhat
    if B == L:
        assert int(geo.eo_index(x, L)) == xhat
    assert list(geo.coords(lam, L)) == x


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 6, 8), (8, 6, 4, 2), (6, 2, 2, 4)])
def test_lexi_and_eo_bijective(L):
    V = geo.volume(L)
    lam = np.arange(V)
    x = geo.coords(lam, L)
    assert np.array_equal(geo.lex(x, L), lam)
    xh = geo.eo_index(x, L)
    assert np.array_equal(np.sort(xh), lam)
    # even sites occupy [0, V/2), odd sites [V/2, V)
    assert np.all((xh < V // 2) == (geo.parity(x) == 0))
    # within a parity, EO order is ascending Lambda
    for p in (0, 1):
        s = geo.sites_of_parity(L, p)
        assert np.array_equal(geo.eo_index(geo.coords(s, L), L), np.arange(V // 2) + p * V // 2)


@pytest.mark.parametrize("L,B", [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 4, 4, 8), (4, 2, 4, 2)), ((4, 8, 4, 4), (4, 4, 2, 4))])
def test_ipt_blocked_bijective(L, B):
    V = geo.volume(L)
    x = geo.coords(np.arange(V), L)
    xh = geo.ipt(x, L, B)
    assert np.array_equal(np.sort(xh), np.arange(V))
    assert np.all((xh < V // 2) == (geo.parity(x) == 0))


def test_shift_wraps_and_inverts():
    L = (4, 2, 6, 4)
    lam = np.arange(geo.volume(L))
    for mu in range(4):
        fwd = geo.shift(lam, L, mu, 1)
        assert np.array_equal(geo.shift(fwd, L, mu, -1), lam)
        # a neighbour has the opposite parity (all extents even)
        assert np.all(geo.parity(geo.coords(fwd, L)) != geo.parity(geo.coords(lam, L)))
        # L_mu forward steps return to the start
        y = lam
        for _ in range(L[mu]):
            y = geo.shift(y, L, mu, 1)
        assert np.array_equal(y, lam)


def test_odd_extent_rejected():
    with pytest.raises(ValueError):
        geo.check_dims((4, 4, 4, 3))
