"""Input generators: Philox4x32-10 known answers and properties of the synthetic fields."""
import numpy as np

import gen


def test_philox_known_answers():
    # Known-answer vectors of Philox4x32-10 published with the Random123 library (Salmon et al., SC'11)
    assert [int(v) for v in gen.philox4x32_10([0, 0, 0, 0], [0, 0])] == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    ff = 0xFFFFFFFF
    assert [int(v) for v in gen.philox4x32_10([ff] * 4, [ff] * 2)] == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]


def test_uniform_moments():
    u = gen.uniforms(200000, seed=5)
    assert 0.0 < u.min() and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.005 and abs(u.var() - 1.0 / 12) < 0.002


def test_su3_links_unitary_unit_det_and_spread():
    L = (4, 4, 2, 2)
    U = gen.su3_field(L, 0.5, 201)
    UUd = np.einsum("nmab,nmcb->nmac", U, U.conj())
    assert np.abs(UUd - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # exp(i eps H): the mean of Re tr U / 3 is below one and depends on eps
    tr = np.einsum("nmaa->nm", U).real.mean() / 3
    tr2 = np.einsum("nmaa->nm", gen.su3_field(L, 0.3, 201)).real.mean() / 3
    assert 0.5 < tr < tr2 < 1.0


def test_fields_are_seeded_and_layout_free():
    L = (2, 2, 2, 4)
    a, b = gen.su3_field(L, 0.5, 7), gen.su3_field(L, 0.5, 7)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, gen.su3_field(L, 0.5, 8))
    # a larger lattice shares its first sites' draws: fields are keyed by the site index only
    big = gen.su3_field((2, 2, 2, 8), 0.5, 7)
    assert np.array_equal(big[:16], a[:16])
    th = gen.u1_field(L, 0.3, 7)
    assert np.abs(th).max() < 0.3 and th.std() > 0.1
    s = gen.gaussian_spinor(L, 7)
    assert s.shape == (32, 4, 3) and abs(np.mean(np.abs(s) ** 2) - 2.0) < 0.5
