"""Pins of the oracle's openQxD storage (Sec. 4.1, Fig. gauge): the odd-point link storage holds
every link of the lattice exactly once, hand-checked slots on a small lattice, inverse maps."""
import numpy as np
import pytest

from oracle import geometry as geo
from oracle import openqxd as oq


def tagged_links(L):
    """U[lam, mu] = (1000 lam + mu) * identity: every link carries its own (site, direction)."""
    V = geo.volume(L)
    tag = (1000.0 * np.arange(V)[:, None] + np.arange(4)[None, :])
    return tag[..., None, None] * np.eye(3)[None, None], tag.copy()


@pytest.mark.parametrize("L,B", [((2, 2, 2, 2), (2, 2, 2, 2)), ((4, 2, 6, 4), (2, 2, 3, 2)),
                                 ((4, 4, 4, 4), (2, 2, 2, 2)), ((6, 4, 2, 8), (3, 4, 1, 4))])
def test_every_link_stored_once(L, B):
    U, th = tagged_links(L)
    u, a = oq.links_to_openqxd(U, th, L, B)
    tags = np.sort(u[:, :, 0, 0].real.ravel())
    assert np.array_equal(tags, np.sort(th.ravel()))
    assert np.array_equal(np.sort(a.ravel()), np.sort(th.ravel()))
    U2, th2 = oq.links_from_openqxd(u, a, L, B)
    assert np.array_equal(U2, U) and np.array_equal(th2, th)


def test_slots_by_hand():
    """4^4 with B = L: the odd point x = (0, 0, 0, 1) (Lambda 1) is the first odd point (ipt 128,
    position 0); slot 2 holds U_1(x) (tag 1001), slot 3 the link U_1(x - 1hat) from
    (0, 3, 0, 1), Lambda 3 * 16 + 1 = 49 (tag 49001); slot 6 U_3(x) (tag 1003), slot 7 the link
    U_3 of (0, 0, 0, 0) (tag 3)."""
    L = B = (4, 4, 4, 4)
    U, th = tagged_links(L)
    u, a = oq.links_to_openqxd(U, th, L, B)
    assert int(geo.ipt(np.array([0, 0, 0, 1]), L, B)) == 128
    assert a[0, 2] == 1001 and a[0, 3] == 49001 and a[0, 6] == 1003 and a[0, 7] == 3
    # slot 0: U_0(x); slot 1: U_0(x - 0hat) with x - 0hat = (3, 0, 0, 1), Lambda 3 * 64 + 1 = 193
    assert a[0, 0] == 1000 and a[0, 1] == 193000


def test_even_points_store_nothing_and_order_is_ipt():
    L, B = (4, 2, 6, 4), (2, 2, 3, 2)
    perm = oq.site_order(L, B)
    V = geo.volume(L)
    assert np.all(geo.parity(geo.coords(perm[: V // 2], L)) == 0)
    assert np.all(geo.parity(geo.coords(perm[V // 2:], L)) == 1)
    x = geo.coords(perm, L)
    assert np.array_equal(geo.ipt(x, L, B), np.arange(V))


def test_bad_blocks_rejected():
    with pytest.raises(ValueError):
        oq.site_order((4, 4, 4, 4), (3, 4, 4, 4))
    with pytest.raises(ValueError):
        oq.site_order((4, 4, 4, 6), (4, 4, 4, 3))
