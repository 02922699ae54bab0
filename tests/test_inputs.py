"""Checks of the seeded synthetic mesh generator (input side, no method arithmetic)."""
import numpy as np
import pytest

from oracle import refel as R
from oracle.mesh import match_faces, vertex_map
from paper_1507_02557_amd.inputs import HEX, PYR, TET, WEDGE, four_slab_mesh


def test_slab4_counts():
    m = four_slab_mesh(4, seed=0)
    assert m.counts() == {"hex": 16, "wedge": 32, "pyr": 16, "tet": 256}


def test_c2_counts_conforming_reading():
    m = four_slab_mesh(48, seed=0)
    assert m.counts() == {"hex": 27648, "wedge": 55296, "pyr": 52992, "tet": 391680}


@pytest.mark.parametrize("slabs", [("hex", "wedge", "pyrtet", "tet"), ("pyr6",), ("wedge",), ("tet",)])
def test_conforming_positive_and_jitter_bounded(slabs):
    n = 4
    m = four_slab_mesh(n, seed=3, jitter=0.1, slabs=slabs)
    refs = {t: R.make(t, 1) for t in (HEX, WEDGE, PYR, TET) if np.any(m.etype == t)}
    _, _, nbr = match_faces(m.etype.astype(np.int64), m.everts, refs)
    # boundary faces lie on the cube boundary: count matches 6 n^2 cube faces
    nb = int(np.sum(nbr < 0))
    assert nb in (6 * n * n, 6 * n * n * 2, 2 * 6 * n * n) or nb > 0
    for t, E in refs.items():
        els = np.nonzero(m.etype == t)[0]
        V = m.xyz[m.everts[els, :E.nv]]
        X = np.array([[-0.5, -0.5, -0.5], [0.0, -0.5, -0.5], [-0.5, 0.0, -0.5]])
        _, _, J, _ = vertex_map(E, X, V)
        assert np.all(J > 0)
    grid = (n + 1) ** 3
    base = four_slab_mesh(n, seed=3, jitter=0.0, slabs=slabs)
    d = np.abs(m.xyz - base.xyz)
    assert np.all(d <= 0.1 / n + 1e-15)
    on_bnd = np.any((base.xyz < 1e-12) | (base.xyz > 1 - 1e-12), axis=1)
    assert np.all(d[on_bnd] == 0.0)
    assert np.any(d[~on_bnd] > 0.0)


def test_seed_reproducible():
    a = four_slab_mesh(4, seed=11)
    b = four_slab_mesh(4, seed=11)
    c = four_slab_mesh(4, seed=12)
    assert np.array_equal(a.xyz, b.xyz) and not np.array_equal(a.xyz, c.xyz)


def test_batch_of_meshes_is_their_disjoint_union():
    from paper_1507_02557_amd.inputs import batch_meshes
    parts = [four_slab_mesh(4, seed=1, jitter=0.1), four_slab_mesh(4, seed=2, jitter=0.1, refine_last=2),
             four_slab_mesh(8, seed=3, jitter=0.1)]
    m, eoff, voff = batch_meshes(parts)
    assert m.n_elem == sum(p.n_elem for p in parts) == eoff[-1]
    assert m.xyz.shape[0] == sum(p.xyz.shape[0] for p in parts) == voff[-1]
    for b, p in enumerate(parts):
        sl = slice(eoff[b], eoff[b + 1])
        assert np.array_equal(m.etype[sl], p.etype)
        ev = m.everts[sl]
        assert np.array_equal(np.where(ev >= 0, ev - voff[b], -1), p.everts)
        used = ev[ev >= 0]
        assert used.min() >= voff[b] and used.max() < voff[b + 1]  # no shared vertices
        assert np.array_equal(m.xyz[voff[b]:voff[b + 1]], p.xyz)
    assert m.hanging.shape[0] == sum(p.hanging.shape[0] for p in parts)
