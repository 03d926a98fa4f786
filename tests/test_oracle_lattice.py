"""Pins for the oracle's lattice conventions (CPU)."""
import numpy as np
import pytest

from oracle import lattice as L


def test_clifford_algebra():
    g, g5 = L.gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2.0 * (mu == nu) * np.eye(4), atol=1e-15)
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=1e-15)
    for mu in range(4):
        assert np.allclose(g5 @ g[mu] + g[mu] @ g5, 0, atol=1e-15)


def test_lex_index_matches_c_order():
    dims = (4, 2, 6, 2)
    s = L.lex_site(dims)
    assert np.array_equal(s.ravel(), np.arange(L.volume(dims)))
    x, y, z, t = L.coords(dims)
    assert s[1, 2, 1, 3] == 3 + 4 * (1 + 2 * (2 + 6 * 1))


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 6, 8)])
def test_eo_tables_are_bijections(dims):
    ev, od = L.eo_tables(dims)
    V = L.volume(dims)
    both = np.concatenate([ev, od])
    assert np.array_equal(np.sort(both), np.arange(V))
    p = L.parity(dims).ravel()
    assert (p[ev] == 0).all() and (p[od] == 1).all()
    assert np.array_equal(ev >> 1, np.arange(V // 2))
    assert np.array_equal(od >> 1, np.arange(V // 2))


def test_neighbours_flip_parity():
    dims = (4, 4, 2, 6)
    p = L.parity(dims)
    for ax in range(4):
        assert ((np.roll(p, 1, axis=ax) + p) % 2 == 1).all()


def test_eo_roundtrip():
    dims = (4, 2, 2, 4)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((3, 4, 2, 2, 4, 4, 3)) + 0j
    e, o = L.to_eo(dims, f)
    assert np.array_equal(L.from_eo(dims, e, o), f)


def test_odd_extent_rejected():
    with pytest.raises(ValueError):
        L.check_dims((4, 4, 3, 4))
