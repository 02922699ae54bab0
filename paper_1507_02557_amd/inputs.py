"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the discontinuous Galerkin method itself:
it builds vertex-mapped hybrid meshes (vertex coordinates plus element vertex
lists), draws the seeded vertex jitter, and evaluates closed-form initial and
exact fields at caller-supplied points.

Mesh construction ("four-slab" cube meshes)
-------------------------------------------
The unit cube is cut into n^3 cubes of side h = 1/n.  The x-layers of cubes
are grouped into four slabs; slab k covers layers
[round(k n / 4), round((k+1) n / 4)).  By default the slabs are, in x order:

* ``hex``    -- every cube is one hexahedron;
* ``wedge``  -- every cube is cut by the vertical plane through its
  (x0,y0)-(x1,y1) edge diagonal into two wedges (triangles in z = const
  planes, extruded along z); this is the cube subdivision into wedges used
  for the paper's single-type wedge meshes (Section 4.1);
* ``pyrtet`` -- every cube is cut into six pyramids with apex at the cube
  centre; the -x pyramid is kept, and so is the +x pyramid when the next
  cube in +x is also of this kind (so that x-interior faces stay conforming
  quadrilaterals); every other pyramid is cut into two tetrahedra along the
  diagonal of its base through the face's (min,min)-(max,max) corners;
* ``tet``    -- every cube is cut into the six Kuhn tetrahedra along its
  (x0,y0,z0)-(x1,y1,z1) diagonal.

``pyr6`` (all six pyramids kept) is also available for single-type pyramid
meshes, the subdivision of hexahedra into pyramids used in Section 4.1.

All choices above are conforming: every interior face is shared by exactly
two elements with the same vertex set.

Refined last slab (``refine_last=2``): the last slab, which must be of kind
``tet``, is built on a grid of half the spacing (every cube cut into eight,
each cut into its six Kuhn tetrahedra).  Its face with the previous slab is
then non-conforming 1:4: every triangle of the coarse side (the
(min,min)-(max,max) diagonal split of a coarse cube face) is the union of the
four triangles of its midpoint subdivision on the fine side, because the
fine Kuhn diagonals run the same way.  The fine grid points on that face
that are not coarse vertices are *hanging vertices*: each is the midpoint of
a coarse edge (a square edge or the square's diagonal), placed at the
midpoint of the two (jittered) coarse vertices and not jittered itself, so
the four fine triangles lie exactly in the plane of their coarse triangle.
``Mesh.hanging`` lists them as rows (vertex, parent a, parent b).  The fine
grid's own interior vertices are jittered by ``jitter * h / 2`` from the same
generator, drawn after the coarse vertices, in fine-grid id order.

Element-local vertex orders are those of the reference elements:

* hex   (r,s,t) in [-1,1]^3: 0(-1,-1,-1) 1(1,-1,-1) 2(1,1,-1) 3(-1,1,-1)
  4(-1,-1,1) 5(1,-1,1) 6(1,1,1) 7(-1,1,1)
* wedge (triangle in (r,t), extruded in s): 0(-1,-1,-1) 1(1,-1,-1)
  2(-1,-1,1) 3(-1,1,-1) 4(1,1,-1) 5(-1,1,1)
* pyramid (base t = -1, apex over (r,s) = (-1,-1)): 0(-1,-1,-1) 1(1,-1,-1)
  2(1,1,-1) 3(-1,1,-1) 4(-1,-1,1)
* tet: 0(-1,-1,-1) 1(1,-1,-1) 2(-1,1,-1) 3(-1,-1,1)

The generator orders each element's vertices so that the vertex map has a
positive Jacobian.

Jitter: every vertex strictly inside the unit cube (cube centres included) is
moved by an independent uniform displacement in [-j h, j h]^3 drawn from
``numpy.random.default_rng(seed)`` for all vertices in id order (boundary
vertices' draws are discarded).  Grid vertex (i,j,k) has id
i + (n+1)(j + (n+1)k); cube centres follow in order of creation.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

HEX, WEDGE, PYR, TET = 0, 1, 2, 3
NVERT = {HEX: 8, WEDGE: 6, PYR: 5, TET: 4}
TYPE_NAMES = {HEX: "hex", WEDGE: "wedge", PYR: "pyr", TET: "tet"}

BC_FREE_SURFACE = 0  # p = 0 on the boundary (the paper's boundary condition)
BC_RIGID_WALL = 1    # u . n = 0 on the boundary

DEFAULT_SLABS = ("hex", "wedge", "pyrtet", "tet")


@dataclass
class Mesh:
    """A vertex-mapped hybrid mesh: vertices plus element vertex lists."""

    xyz: np.ndarray            # (n_vert, 3) float64
    etype: np.ndarray          # (n_elem,) int8, HEX/WEDGE/PYR/TET
    everts: np.ndarray         # (n_elem, 8) int64, local vertex order, -1 padded
    kappa: np.ndarray          # (n_elem,) float64 bulk modulus
    rho: np.ndarray            # (n_elem,) float64 density
    n: int = 0
    info: dict = field(default_factory=dict)
    hanging: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), dtype=np.int64))
    # optional boundary condition per element and local face ([n_elem, 6],
    # -1: the solver's default, else 0 free surface / 1 rigid wall); only
    # boundary faces use it
    bc_face: np.ndarray | None = None

    @property
    def n_elem(self) -> int:
        return int(self.etype.shape[0])

    def counts(self) -> dict:
        return {TYPE_NAMES[t]: int(np.sum(self.etype == t)) for t in (HEX, WEDGE, PYR, TET)}

    def permuted(self, order) -> "Mesh":
        """The same mesh with element i of the result being element order[i]."""
        order = np.asarray(order, dtype=np.int64)
        if order.shape != (self.n_elem,) or not np.array_equal(np.sort(order), np.arange(self.n_elem)):
            raise ValueError("order must be a permutation of the elements")
        return Mesh(xyz=self.xyz, etype=self.etype[order], everts=self.everts[order], kappa=self.kappa[order],
                    rho=self.rho[order], n=self.n, info=dict(self.info), hanging=self.hanging,
                    bc_face=None if self.bc_face is None else np.asarray(self.bc_face)[order])

    def level_order(self, level) -> np.ndarray:
        """Element order that stores every type's elements finest level first
        (highest level number first, mesh order within a level)."""
        level = np.asarray(level, dtype=np.int64)
        return np.lexsort((np.arange(self.n_elem), -level, self.etype.astype(np.int64)))


def batch_meshes(meshes) -> tuple:
    """Disjoint union of several meshes (one batch of independent problems):
    vertex ids of mesh b are offset by the vertices before it, its elements
    follow those of the meshes before it.  Within each part the order of the
    global vertex ids is kept, so every face keeps its canonical frame.
    Returns (mesh, element offsets [B + 1], vertex offsets [B + 1])."""
    xyz, et, ev, ka, rh, hang, bcf = [], [], [], [], [], [], []
    voff, eoff = [0], [0]
    any_bc = any(m.bc_face is not None for m in meshes)
    for m in meshes:
        v0 = voff[-1]
        xyz.append(np.asarray(m.xyz, dtype=np.float64))
        et.append(np.asarray(m.etype, dtype=np.int8))
        e = np.asarray(m.everts, dtype=np.int64)
        ev.append(np.where(e >= 0, e + v0, -1))
        ka.append(np.asarray(m.kappa, dtype=np.float64))
        rh.append(np.asarray(m.rho, dtype=np.float64))
        h = np.asarray(m.hanging, dtype=np.int64).reshape(-1, 3)
        hang.append(h + v0)
        if any_bc:
            bcf.append(np.full((m.n_elem, 6), -1, dtype=np.int8) if m.bc_face is None
                       else np.asarray(m.bc_face, dtype=np.int8))
        voff.append(v0 + m.xyz.shape[0])
        eoff.append(eoff[-1] + m.n_elem)
    out = Mesh(xyz=np.concatenate(xyz), etype=np.concatenate(et), everts=np.concatenate(ev),
               kappa=np.concatenate(ka), rho=np.concatenate(rh), n=0, info={"batch": len(meshes)},
               hanging=np.concatenate(hang), bc_face=np.concatenate(bcf) if any_bc else None)
    return out, np.asarray(eoff, dtype=np.int64), np.asarray(voff, dtype=np.int64)


def _slab_of_layer(n: int, layer: int, nslab: int) -> int:
    for k in range(nslab):
        lo = int(round(k * n / nslab))
        hi = int(round((k + 1) * n / nslab))
        if lo <= layer < hi:
            return k
    return nslab - 1


def _det3(a, b, c) -> float:
    return float(np.dot(a, np.cross(b, c)))


def _orient(kind: int, v: list, P: np.ndarray) -> list:
    """Reorder vertices so that the reference-to-physical map has J > 0."""
    p = [P[i] for i in v]
    if kind == TET:
        if _det3(p[1] - p[0], p[2] - p[0], p[3] - p[0]) < 0:
            v = [v[0], v[1], v[3], v[2]]
    elif kind == PYR:
        if _det3(p[1] - p[0], p[3] - p[0], p[4] - p[0]) < 0:
            v = [v[0], v[3], v[2], v[1], v[4]]
    elif kind == WEDGE:
        # r along v0->v1, s along v0->v3, t along v0->v2
        if _det3(p[1] - p[0], p[3] - p[0], p[2] - p[0]) < 0:
            v = [v[0], v[2], v[1], v[3], v[5], v[4]]
    elif kind == HEX:
        if _det3(p[1] - p[0], p[3] - p[0], p[4] - p[0]) < 0:
            raise ValueError("hex construction produced a negative Jacobian")
    return v


def _orient_all(etype: np.ndarray, everts: np.ndarray, P: np.ndarray) -> None:
    """_orient applied to every element at once (in place), same tests."""
    def det(rows, i0, i1, i2, i3):
        v = everts[rows]
        p0 = P[v[:, i0]]
        a, b, c = P[v[:, i1]] - p0, P[v[:, i2]] - p0, P[v[:, i3]] - p0
        return np.einsum("ij,ij->i", a, np.cross(b, c))

    rows = np.nonzero(etype == TET)[0]
    flip = rows[det(rows, 0, 1, 2, 3) < 0]
    everts[flip, 2:4] = everts[flip][:, [3, 2]]
    rows = np.nonzero(etype == PYR)[0]
    flip = rows[det(rows, 0, 1, 3, 4) < 0]
    everts[flip, :5] = everts[flip][:, [0, 3, 2, 1, 4]]
    rows = np.nonzero(etype == WEDGE)[0]
    flip = rows[det(rows, 0, 1, 3, 2) < 0]
    everts[flip, :6] = everts[flip][:, [0, 2, 1, 3, 5, 4]]
    rows = np.nonzero(etype == HEX)[0]
    if np.any(det(rows, 0, 1, 3, 4) < 0):
        raise ValueError("hex construction produced a negative Jacobian")


def four_slab_mesh(n: int, seed: int = 0, jitter: float = 0.1,
                   slabs=DEFAULT_SLABS, kappa: float = 1.0, rho: float = 1.0, refine_last: int = 1) -> Mesh:
    """Build the four-slab hybrid cube mesh described in the module docstring.

    ``slabs`` lists the kind of each x-slab ("hex", "wedge", "pyrtet", "tet",
    "pyr6"); its length sets the number of slabs (a one-element list gives a
    single-type mesh).  ``refine_last=2`` builds the last slab (kind "tet", not
    the first slab) on the half-spacing grid with a 1:4 non-conforming face.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    slabs = tuple(slabs)
    nslab = len(slabs)
    if refine_last not in (1, 2):
        raise ValueError("refine_last must be 1 or 2")
    if refine_last == 2 and (slabs[-1] != "tet" or nslab < 2):
        raise ValueError("only a last slab of kind 'tet' after another slab can be refined")
    # first coarse layer of the refined slab (n: no refined slab)
    i_ref = int(round((nslab - 1) * n / nslab)) if refine_last == 2 else n
    if i_ref <= 0 or i_ref >= n + (refine_last == 1):
        raise ValueError("the refined slab must be non-empty and not the whole mesh")
    h = 1.0 / n
    n1 = n + 1

    def gid(i, j, k):
        return i + n1 * (j + n1 * k)

    # id order i fastest: flat index = i + n1*(j + n1*k)
    pts = np.empty((n1 ** 3, 3))
    kk, jj, ii = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    pts[:, 0] = (ii.ravel()) * h
    pts[:, 1] = (jj.ravel()) * h
    pts[:, 2] = (kk.ravel()) * h
    centres: list = []

    def centre_id(i, j, k):
        centres.append(((i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h))
        return n1 ** 3 + len(centres) - 1

    elems: list = []  # (type, [vertex ids])

    def kind_of(i):
        if i < 0 or i >= n:
            return None
        return slabs[_slab_of_layer(n, i, nslab)]

    for k in range(n):
        for j in range(n):
            for i in range(i_ref):
                kind = kind_of(i)
                c = [[[gid(i + a, j + b, k + d) for d in (0, 1)] for b in (0, 1)] for a in (0, 1)]
                # c[a][b][d]: corner at (x_i+a, y_j+b, z_k+d)
                if kind == "hex":
                    v = [c[0][0][0], c[1][0][0], c[1][1][0], c[0][1][0],
                         c[0][0][1], c[1][0][1], c[1][1][1], c[0][1][1]]
                    elems.append((HEX, None, v))
                elif kind == "wedge":
                    for tri in (((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1))):
                        bot = [c[a][b][0] for a, b in tri]
                        top = [c[a][b][1] for a, b in tri]
                        v = [bot[0], bot[1], bot[2], top[0], top[1], top[2]]
                        # reference order: 0,1,2 on s=-1 (triangle r,t), 3,4,5 on s=+1
                        elems.append((WEDGE, None, v))
                elif kind == "tet":
                    lo = np.array([i, j, k])
                    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
                        p = lo.copy()
                        v = [gid(*p)]
                        for ax in perm:
                            p[ax] += 1
                            v.append(gid(*p))
                        elems.append((TET, None, v))
                elif kind in ("pyrtet", "pyr6"):
                    cid = centre_id(i, j, k)
                    # six faces: (axis, side)
                    for ax in range(3):
                        for side in (0, 1):
                            # face corners in cyclic order in the two tangential axes
                            t1, t2 = [a for a in range(3) if a != ax]
                            cyc = []
                            for (u, w) in ((0, 0), (1, 0), (1, 1), (0, 1)):
                                idx = [0, 0, 0]
                                idx[ax] = side
                                idx[t1] = u
                                idx[t2] = w
                                cyc.append(c[idx[0]][idx[1]][idx[2]])
                            keep = False
                            if kind == "pyr6":
                                keep = True
                            elif ax == 0 and side == 0:
                                keep = True
                            elif ax == 0 and side == 1 and kind_of(i + 1) == "pyrtet":
                                keep = True
                            if keep:
                                elems.append((PYR, None, cyc + [cid]))
                            else:
                                # split along the (min,min)-(max,max) diagonal of the face
                                a0, a1, a2, a3 = cyc  # (0,0),(1,0),(1,1),(0,1)
                                elems.append((TET, None, [a0, a1, a2, cid]))
                                elems.append((TET, None, [a0, a2, a3, cid]))
                else:
                    raise ValueError(f"unknown slab kind {kind!r}")

    allpts = np.concatenate([pts, np.array(centres, dtype=np.float64).reshape(-1, 3)], axis=0)
    n_coarse = allpts.shape[0]
    hanging = np.zeros((0, 3), dtype=np.int64)
    if refine_last == 2:
        fine_pts, hanging, fine_elems = _refined_tet_slab(n, i_ref, gid, n_coarse)
        allpts = np.concatenate([allpts, fine_pts], axis=0)
        elems.extend(fine_elems)
    n_vert = allpts.shape[0]
    etype = np.array([t for t, _, _ in elems], dtype=np.int8)
    everts = -np.ones((len(elems), 8), dtype=np.int64)
    for kind, nv in ((HEX, 8), (WEDGE, 6), (PYR, 5), (TET, 4)):
        sel = np.nonzero(etype == kind)[0]
        if sel.size:
            everts[sel, :nv] = np.array([elems[e][2] for e in sel], dtype=np.int64)
    # orientation decisions use the unjittered positions
    _orient_all(etype, everts, allpts)

    rng = np.random.default_rng(seed)
    disp = rng.uniform(-jitter * h, jitter * h, size=(n_coarse, 3))
    if n_vert > n_coarse:
        disp = np.concatenate([disp, rng.uniform(-jitter * h / 2, jitter * h / 2, size=(n_vert - n_coarse, 3))])
    tol = 1e-12
    on_bnd = np.any((allpts < tol) | (allpts > 1.0 - tol), axis=1)
    disp[on_bnd] = 0.0
    if hanging.shape[0]:
        disp[hanging[:, 0]] = 0.0
    xyz = allpts + disp
    if hanging.shape[0]:
        # hanging vertices: midpoints of their (jittered) coarse edges
        xyz[hanging[:, 0]] = 0.5 * (xyz[hanging[:, 1]] + xyz[hanging[:, 2]])

    ne = etype.shape[0]
    return Mesh(xyz=xyz, etype=etype, everts=everts,
                kappa=np.full(ne, float(kappa)), rho=np.full(ne, float(rho)), n=n,
                info={"seed": seed, "jitter": jitter, "slabs": list(slabs), "refine_last": refine_last},
                hanging=hanging)


def _refined_tet_slab(n: int, i0: int, gid, id0: int):
    """Kuhn tetrahedra of the half-spacing grid over the coarse layers i0..n-1.

    Fine grid point (a, b, c), a in 0..2(n-i0), b, c in 0..2n, sits at
    ((i0 + a/2) h, b h/2, c h/2).  On the face a = 0, points with b and c even
    are the coarse vertices gid(i0, b/2, c/2); the others are hanging vertices
    (midpoints of a coarse square edge, or of its (min,min)-(max,max)
    diagonal when b and c are both odd).  Every other fine point is a new
    vertex, numbered from id0 in order a fastest, then b, then c.
    Returns (points, hanging rows (vertex, parent a, parent b), elements).
    """
    h = 1.0 / n
    na, nb = 2 * (n - i0), 2 * n
    ids = -np.ones((na + 1, nb + 1, nb + 1), dtype=np.int64)
    pts, hang = [], []
    nxt = id0
    for c in range(nb + 1):
        for b in range(nb + 1):
            for a in range(na + 1):
                if a == 0 and b % 2 == 0 and c % 2 == 0:
                    ids[a, b, c] = gid(i0, b // 2, c // 2)
                    continue
                ids[a, b, c] = nxt
                pts.append(((i0 + a / 2.0) * h, b * h / 2.0, c * h / 2.0))
                if a == 0:
                    if b % 2 and c % 2:
                        pa, pb = gid(i0, (b - 1) // 2, (c - 1) // 2), gid(i0, (b + 1) // 2, (c + 1) // 2)
                    elif b % 2:
                        pa, pb = gid(i0, (b - 1) // 2, c // 2), gid(i0, (b + 1) // 2, c // 2)
                    else:
                        pa, pb = gid(i0, b // 2, (c - 1) // 2), gid(i0, b // 2, (c + 1) // 2)
                    hang.append((nxt, pa, pb))
                nxt += 1
    elems = []
    perms = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
    for c in range(nb):
        for b in range(nb):
            for a in range(na):
                for perm in perms:
                    p = [a, b, c]
                    v = [int(ids[a, b, c])]
                    for ax in perm:
                        p[ax] += 1
                        v.append(int(ids[p[0], p[1], p[2]]))
                    elems.append((TET, None, v))
    return (np.array(pts, dtype=np.float64).reshape(-1, 3), np.array(hang, dtype=np.int64).reshape(-1, 3), elems)


# ---------------------------------------------------------------------------
# Closed-form fields (kappa = rho = 1); accept numpy arrays or torch tensors
# ---------------------------------------------------------------------------

def _xp(x):
    if type(x).__module__.startswith("torch"):
        import torch
        return torch
    return np


def standing_mode_rigid(x, y, z, t):
    """Rigid-wall (u.n = 0) resonant mode of p_t + div u = 0, u_t + grad p = 0.

    p = cos(pi x) cos(pi y) cos(pi z) cos(sqrt(3) pi t) and
    u_x = sin(pi x) cos(pi y) cos(pi z) sin(sqrt(3) pi t) / sqrt(3), cyclic.
    Returns (p, ux, uy, uz).
    """
    xp = _xp(x)
    pi = np.pi
    w = np.sqrt(3.0) * pi
    cx, cy, cz = xp.cos(pi * x), xp.cos(pi * y), xp.cos(pi * z)
    sx, sy, sz = xp.sin(pi * x), xp.sin(pi * y), xp.sin(pi * z)
    st = np.sin(w * t) / np.sqrt(3.0)
    return (cx * cy * cz * np.cos(w * t), sx * cy * cz * st, cx * sy * cz * st, cx * cy * sz * st)


def standing_mode_free(x, y, z, t):
    """Free-surface (p = 0) resonant cavity mode of Section 4.1.

    p = sin(pi x) sin(pi y) sin(pi z) cos(sqrt(3) pi t) and
    u_x = -cos(pi x) sin(pi y) sin(pi z) sin(sqrt(3) pi t) / sqrt(3), cyclic.
    Returns (p, ux, uy, uz).
    """
    xp = _xp(x)
    pi = np.pi
    w = np.sqrt(3.0) * pi
    cx, cy, cz = xp.cos(pi * x), xp.cos(pi * y), xp.cos(pi * z)
    sx, sy, sz = xp.sin(pi * x), xp.sin(pi * y), xp.sin(pi * z)
    st = -np.sin(w * t) / np.sqrt(3.0)
    return (sx * sy * sz * np.cos(w * t), cx * sy * sz * st, sx * cy * sz * st, sx * sy * cz * st)


def pulse_centre(seed: int) -> np.ndarray:
    """Centre of the Gaussian pressure pulse, uniform in [0.2, 0.8]^3 from the seed."""
    rng = np.random.default_rng(seed + 7919)
    return rng.uniform(0.2, 0.8, size=3)


def gaussian_pulse(x, y, z, centre, width: float = 0.05):
    """p = exp(-|x - x0|^2 / (2 width^2)), u = 0.  Returns (p, ux, uy, uz)."""
    xp = _xp(x)
    r2 = (x - float(centre[0])) ** 2 + (y - float(centre[1])) ** 2 + (z - float(centre[2])) ** 2
    p = xp.exp(-r2 / (2.0 * width * width))
    zero = xp.zeros_like(p)
    return (p, zero, zero.clone() if xp is not np else zero.copy(), zero.clone() if xp is not np else zero.copy())
