"""Face matching, canonical face frames and geometric factors (oracle side).

Face matching: every element face is keyed by the sorted global ids of its
vertices; two element faces with the same key form an interior face, a key
seen once is a boundary face, more than two is an error.

Canonical face frame: a triangle's canonical vertex order is its vertices
by ascending global id; a quadrilateral's starts at its smallest-id vertex,
continues to whichever of that vertex's two edge neighbours has the smaller
id, and goes round the cycle.  Face cubature points are placed in this frame,
so both elements sharing a face evaluate their traces at the same physical
points, in the same order.

Geometric factors follow the vertex map x(r,s,t) = sum_v N_v(r,s,t) x_v
(Section 2): F = dx/d(r,s,t), J = det F, G = F^{-1} = d(r,s,t)/dx.
"""
from __future__ import annotations

import numpy as np

from . import refel as R


def vertex_map(E, X, V):
    """Physical points and Jacobians of elements V (K, nv, 3) at reference points X (npts, 3).

    X may also be per-element (K, npts, 3).  Returns x (K, npts, 3),
    F (K, npts, 3, 3) with F[..., d, r] = dx_d/dxi_r, J (K, npts), G (K, npts, 3, 3)
    with G[..., r, d] = dxi_r/dx_d.
    """
    if X.ndim == 2:
        S, dS = E.shape(X)
        x = np.einsum("qv,kvd->kqd", S, V)
        F = np.einsum("rqv,kvd->kqdr", dS, V)
    else:
        K, npts, _ = X.shape
        S, dS = E.shape(X.reshape(-1, 3))
        S = S.reshape(K, npts, -1)
        dS = dS.reshape(3, K, npts, -1)
        x = np.einsum("kqv,kvd->kqd", S, V)
        F = np.einsum("rkqv,kvd->kqdr", dS, V)
    J = np.linalg.det(F)
    G = np.linalg.inv(F)
    return x, F, J, G


def match_faces(types, everts, refs):
    """Pair element faces by their vertex sets.

    ``types`` (n_elem,), ``everts`` (n_elem, 8); ``refs`` maps type -> RefElement.
    Slots are all (element, local face) pairs, ordered by element then face.
    Returns slot_elem, slot_face and the neighbour slot of every slot (-1 on
    the boundary).
    """
    nfaces = np.array([refs[int(t)].nfaces if int(t) in refs else 0 for t in range(4)])
    nf_e = nfaces[types.astype(np.int64)]
    first = np.concatenate([[0], np.cumsum(nf_e)])
    nslot = int(first[-1])
    slot_elem = np.repeat(np.arange(types.shape[0]), nf_e)
    slot_face = np.arange(nslot) - first[slot_elem]
    keys = -np.ones((nslot, 4), dtype=np.int64)
    for t, E in refs.items():
        els = np.nonzero(types == t)[0]
        for f, fv in enumerate(E.faces):
            g = np.sort(everts[els][:, list(fv)], axis=1)
            keys[first[els] + f, 4 - len(fv):] = g
    order = np.lexsort(keys.T[::-1])
    ks = keys[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    if np.any(same[1:] & same[:-1]):
        raise ValueError("non-manifold face shared by more than two elements")
    nbr = -np.ones(nslot, dtype=np.int64)
    i = np.nonzero(same)[0]
    nbr[order[i]] = order[i + 1]
    nbr[order[i + 1]] = order[i]
    return slot_elem, slot_face, nbr


def canonical_perm(gids):
    """Positions (in the face's local vertex list) of the canonical vertices c0..c_{nv-1}."""
    gids = list(gids)
    nv = len(gids)
    if nv == 3:
        return tuple(int(i) for i in np.argsort(gids))
    p = int(np.argmin(gids))
    prv, nxt = (p - 1) % 4, (p + 1) % 4
    if gids[nxt] < gids[prv]:
        return (p, nxt, (p + 2) % 4, prv)
    return (p, prv, (p + 2) % 4, nxt)


def nonconforming_faces(types, everts, refs, slot_elem, slot_face, nbr, hanging):
    """1:4 non-conforming triangular faces.

    ``hanging`` rows (v, a, b): vertex v is the midpoint of the edge (a, b).
    An unmatched triangular face (v0, v1, v2) whose three edge midpoints are
    all hanging vertices is a coarse face; its four sub-faces are the
    triangles of its midpoint subdivision,
      (v0, m01, m20), (v1, m12, m01), (v2, m20, m12), (m01, m12, m20),
    each of which must be an unmatched face of exactly one element.
    Returns a list of (coarse slot, [(fine slot, {vertex id: barycentric
    coordinates w.r.t. the coarse face's local vertices (v0, v1, v2)})] * 4).
    """
    hanging = np.asarray(hanging, dtype=np.int64).reshape(-1, 3)
    if hanging.shape[0] == 0:
        return []
    mid = {(min(a, b), max(a, b)): int(v) for v, a, b in hanging}
    first = {}
    free_tri = {}
    for s in np.nonzero(nbr < 0)[0]:
        e, f = int(slot_elem[s]), int(slot_face[s])
        fv = refs[int(types[e])].faces[f]
        if len(fv) != 3:
            continue
        g = tuple(int(everts[e, v]) for v in fv)
        first[s] = g
        free_tri[tuple(sorted(g))] = int(s)
    out = []
    used = set()
    for s, g in first.items():
        v0, v1, v2 = g
        m01 = mid.get((min(v0, v1), max(v0, v1)))
        m12 = mid.get((min(v1, v2), max(v1, v2)))
        m20 = mid.get((min(v2, v0), max(v2, v0)))
        if m01 is None or m12 is None or m20 is None:
            continue
        bary = {v0: np.array([1.0, 0.0, 0.0]), v1: np.array([0.0, 1.0, 0.0]), v2: np.array([0.0, 0.0, 1.0]),
                m01: np.array([0.5, 0.5, 0.0]), m12: np.array([0.0, 0.5, 0.5]), m20: np.array([0.5, 0.0, 0.5])}
        subs = []
        for tri in ((v0, m01, m20), (v1, m12, m01), (v2, m20, m12), (m01, m12, m20)):
            fs = free_tri.get(tuple(sorted(tri)))
            if fs is None or fs in used:
                raise ValueError("a sub-face of a refined triangular face has no element")
            used.add(fs)
            subs.append((fs, {v: bary[v] for v in tri}))
        out.append((int(s), subs))
    return out
