"""Pins of the oracle on meshes with a 1:4 non-conforming face (CPU).

The last slab of the four-slab mesh is built on the half-spacing grid, so
every coarse triangle on its face with the previous slab is the union of the
four triangles of its midpoint subdivision.  The oracle couples them by
evaluating the coarse trace at the fine face points and summing the coarse
face integral over the four sub-faces.  What fixes the result:

* geometry: hanging vertices are coarse-edge midpoints and the four fine
  triangles tile their coarse triangle (areas add up, points coplanar);
* consistency: constant states are steady, and on tetrahedral meshes (exact
  integration, polynomial traces) linear fields give the exact derivatives,
  with either boundary condition (a decoupled or mis-mapped interface gives
  a trace jump there);
* the semi-discrete energy identity (Section 3.1, eq. sym) with random
  materials, which fails if the sub-face weights, normals or pairing are wrong;
* the analytic standing mode, and h-convergence across the interface;
* the local time step of a coarse interface element, whose penalty maxima run
  over the fine neighbours found by brute force.
"""
import numpy as np
import pytest

from oracle import mesh as OM
from oracle import refel as R
from oracle.mrab import bin_levels
from oracle.solver import BC_FREE_SURFACE, BC_RIGID_WALL, Disc, lserk4_step
from oracle.tables import trace_constant
from paper_1507_02557_amd.inputs import TET, four_slab_mesh, standing_mode_rigid


def _tri_area(p):
    return 0.5 * np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[0]))


@pytest.mark.parametrize("n", [4, 8])
def test_refined_mesh_counts_and_hanging_vertices(n):
    m = four_slab_mesh(n, seed=3, jitter=0.1, refine_last=2)
    c = four_slab_mesh(n, seed=3, jitter=0.1).counts()
    nt = n - int(round(3 * n / 4))          # coarse layers of the tet slab
    assert m.counts()["tet"] == c["tet"] - 6 * nt * n * n + 48 * nt * n * n
    assert m.counts()["hex"] == c["hex"] and m.counts()["pyr"] == c["pyr"]
    assert m.hanging.shape == ((2 * n + 1) ** 2 - (n + 1) ** 2, 3)
    h = m.hanging
    assert np.allclose(m.xyz[h[:, 0]], 0.5 * (m.xyz[h[:, 1]] + m.xyz[h[:, 2]]), atol=1e-15)


def test_sub_faces_tile_their_coarse_triangle():
    m = four_slab_mesh(4, seed=1, jitter=0.1, refine_last=2)
    types = m.etype.astype(np.int64)
    refs = {t: R.make(t, 1) for t in np.unique(types)}
    se, sf, nbr = OM.match_faces(types, m.everts, refs)
    nc = OM.nonconforming_faces(types, m.everts, refs, se, sf, nbr, m.hanging)
    assert len(nc) == 2 * 4 * 4  # two coarse triangles per coarse cube face on the interface
    for s, subs in nc:
        e, f = se[s], sf[s]
        cv = m.everts[e, list(refs[int(types[e])].faces[f])]
        P = m.xyz[cv]
        nrm = np.cross(P[1] - P[0], P[2] - P[0])
        nrm /= np.linalg.norm(nrm)
        area = 0.0
        for fs, bary in subs:
            fe = se[fs]
            fv = m.everts[fe, list(refs[int(types[fe])].faces[sf[fs]])]
            Q = m.xyz[fv]
            assert np.max(np.abs((Q - P[0]) @ nrm)) < 1e-14      # in the coarse plane
            for v in fv:                                         # barycentrics reproduce the vertex
                assert np.allclose(bary[int(v)] @ P, m.xyz[v], atol=1e-15)
            area += _tri_area(Q)
        assert abs(area - _tri_area(P)) < 1e-14


def test_refined_constant_state_is_steady():
    for slabs, jit in ((("hex", "wedge", "pyrtet", "tet"), 0.0), (("tet", "tet"), 0.1)):
        d = Disc(four_slab_mesh(4, seed=0, jitter=jit, slabs=slabs, refine_last=2), 3)
        U = d.project(lambda x, y, z, t: (np.ones_like(x), 0 * x, 0 * x, 0 * x))
        Rr = d.rhs(U)
        assert max(np.abs(Rr[t]).max() for t in d.types) < 1e-10, slabs


@pytest.mark.parametrize("bc", [BC_RIGID_WALL, BC_FREE_SURFACE])
def test_refined_linear_fields_have_exact_derivatives(bc):
    """On jittered tetrahedra, p and u linear: rhs_p = -div u, rhs_u = -grad p in
    elements away from the domain boundary (there the mirror state makes a jump);
    the interface is interior, so a wrong coupling shows up there."""
    m = four_slab_mesh(4, seed=4, jitter=0.1, slabs=("tet", "tet"), refine_last=2)
    d = Disc(m, 2, bc=bc)
    f = lambda x, y, z, t: (1 + 2 * x - 3 * y + 0.5 * z, 0.3 + x - y, 2 * z - 0.5 * y, -x + 4 * y)
    U = d.project(f)
    Rr = d.rhs(U)[R.TET]
    sl = d.slot[R.TET]
    bnd = np.any((d.nbr[sl] < 0) & ~d.is_parent[sl], axis=1)   # a face on the domain boundary
    assert (~bnd).sum() > 500
    inner = Rr[~bnd]
    assert np.abs(inner[:, 0] + 0.5).max() < 1e-10   # -div u = -(1 - 0.5 + 0)
    assert np.abs(inner[:, 1] + 2.0).max() < 1e-10
    assert np.abs(inner[:, 2] - 3.0).max() < 1e-10
    assert np.abs(inner[:, 3] + 0.5).max() < 1e-10
    # interface elements of both sides are among them
    coarse = np.unique(d.slot_elem[np.nonzero(d.is_parent)[0]])
    fine = np.unique(np.concatenate(d.nc_groups))
    assert np.sum(~bnd[np.searchsorted(d.els[R.TET], coarse)]) >= 8
    assert np.sum(~bnd[np.searchsorted(d.els[R.TET], fine)]) >= 32


@pytest.mark.parametrize("bc", [BC_RIGID_WALL, BC_FREE_SURFACE])
def test_refined_energy_identity(bc):
    """sum_K (p^T M r_p / kappa + rho u^T M r_u) = -1/2 sum over face pairs of
    int tau_p [p]^2 + tau_u [u.n]^2 (sub-face pairs on the non-conforming face)
    plus the mirror-state boundary terms, random kappa, rho and state."""
    m = four_slab_mesh(4, seed=6, jitter=0.1, refine_last=2)
    rng = np.random.default_rng(8)
    m.kappa = rng.uniform(0.5, 2.0, m.n_elem)
    m.rho = rng.uniform(0.5, 2.0, m.n_elem)
    d = Disc(m, 2, bc=bc)
    assert d.is_parent.sum() == 32
    U = {t: rng.standard_normal(d.zeros()[t].shape) for t in d.types}
    Rr = d.rhs(U)
    lhs = 0.0
    for t in d.types:
        MR = d.mass_apply(t, Rr[t])
        lhs += float(np.sum(U[t][:, 0] * MR[:, 0] / d.kappa[d.els[t]][:, None]))
        lhs += float(np.sum(d.rho[d.els[t]][:, None, None] * U[t][:, 1:] * MR[:, 1:]))
    TR = d.traces(U)
    inner = d.nbr >= 0
    nb = TR[np.maximum(d.nbr, 0)]
    rc_o = d.rhoc[d.slot_elem]
    rc_n = np.where(inner, d.rhoc[d.slot_elem[np.maximum(d.nbr, 0)]], rc_o)
    avg = 0.5 * (rc_o + rc_n)
    jp = nb[..., 0] - TR[..., 0]
    un_o = np.einsum("kqd,kqd->kq", TR[..., 1:], d.nrm)
    un_n = np.einsum("kqd,kqd->kq", nb[..., 1:], d.nrm)
    w = d.wq * d.Js
    e_int = -0.25 * np.sum((w * (jp ** 2 / avg[:, None] + avg[:, None] * (un_n - un_o) ** 2))[inner])
    if bc == BC_RIGID_WALL:
        e_bnd = -np.sum((w * avg[:, None] * un_o ** 2)[~inner])
    else:
        e_bnd = -np.sum((w * TR[..., 0] ** 2 / avg[:, None])[~inner])
    assert abs(lhs - (e_int + e_bnd)) < 1e-11 * abs(e_int + e_bnd)


def test_refined_standing_mode():
    """100 LSERK4 steps of the rigid-wall standing mode on the refined n=4
    hybrid mesh, N=3: the error stays at the discretisation level of the
    conforming mesh (whose coarse tetrahedra it refines)."""
    m = four_slab_mesh(4, seed=0, jitter=0.1, refine_last=2)
    d = Disc(m, 3)
    dt = d.dt_min(0.5)
    U = d.project(standing_mode_rigid)
    for _ in range(100):
        U = lserk4_step(d, U, dt)
    err = d.l2_error(U, standing_mode_rigid, 100 * dt)
    d0 = Disc(four_slab_mesh(4, seed=0, jitter=0.1), 3)
    U0 = d0.project(standing_mode_rigid)
    for _ in range(100):
        U0 = lserk4_step(d0, U0, dt)
    err0 = d0.l2_error(U0, standing_mode_rigid, 100 * dt)
    assert err < err0, (err, err0)


def test_refined_convergence_rate():
    """Unjittered tetrahedral meshes with the refined slab, N=2, n = 4 -> 8:
    the error at t = 0.02 falls at a rate >= N + 1/2."""
    errs = []
    T = 0.02
    for n in (4, 8):
        d = Disc(four_slab_mesh(n, seed=0, jitter=0.0, slabs=("tet", "tet"), refine_last=2), 2)
        nst = int(np.ceil(T / d.dt_min(0.5)))
        U = d.project(standing_mode_rigid)
        for _ in range(nst):
            U = lserk4_step(d, U, T / nst)
        errs.append(d.l2_error(U, standing_mode_rigid, T))
    rate = np.log2(errs[0] / errs[1])
    assert rate > 2.5, (errs, rate)


def test_refined_time_step_of_a_coarse_interface_element():
    """dtau_K = C / (C_rhokappa C_T(N) C_J^K) for a coarse tetrahedron on the
    interface, with the penalty maxima over its conforming neighbours and the
    fine neighbours of its refined face, all found by brute force."""
    m = four_slab_mesh(4, seed=2, jitter=0.1, refine_last=2)
    rng = np.random.default_rng(11)
    m.kappa = rng.uniform(0.5, 2.0, m.n_elem)
    m.rho = rng.uniform(0.5, 2.0, m.n_elem)
    N = 2
    d = Disc(m, N)
    rc = np.sqrt(m.kappa * m.rho)
    tet_faces = R.make(R.TET, 1).faces
    checked = 0
    for s in np.nonzero(d.is_parent)[0][:6]:
        e = int(d.slot_elem[s])
        ev = [int(v) for v in m.everts[e, :4]]
        faces = [frozenset(ev[i] for i in f) for f in tet_faces]
        mids = {frozenset((int(a), int(b))): int(v) for v, a, b in m.hanging}
        avg = []
        for F in faces:
            # conforming neighbour: an element with the same three vertices
            nb = [k for k in range(m.n_elem) if k != e and F <= set(int(v) for v in m.everts[k] if v >= 0)]
            if nb:
                avg.append(0.5 * (rc[e] + rc[nb[0]]))
                continue
            Fl = sorted(F)
            pts = set(Fl) | {mids.get(frozenset((Fl[i], Fl[j]))) for i in range(3) for j in range(i + 1, 3)}
            fine = [k for k in range(m.n_elem)
                    if k != e and sum(int(v) in pts for v in m.everts[k] if v >= 0) == 3]
            if len(fine) == 4:                      # the refined face: its four fine neighbours
                avg.extend(0.5 * (rc[e] + rc[k]) for k in fine)
            else:                                   # domain boundary: own rho c
                assert not fine
                avg.append(rc[e])
        c_rk = max(max(1.0 / a for a in avg) * m.kappa[e], max(avg) / m.rho[e])
        P = m.xyz[ev]
        J = np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], 1)) / 8.0
        js = max(_tri_area(P[list(f)]) / 2.0 for f in tet_faces)   # J^s w.r.t. the area-2 reference face
        dt = 0.5 / (c_rk * trace_constant(R.TET, N) * js / J)
        k = int(np.nonzero(d.els[R.TET] == e)[0][0])
        assert abs(d.dt_elements(0.5)[R.TET][k] - dt) < 1e-12 * dt
        checked += 1
    assert checked == 6


def test_refined_levels_keep_sub_face_groups_together():
    d = Disc(four_slab_mesh(4, seed=0, jitter=0.1, refine_last=2), 2)
    lev, _ = bin_levels(d, 3)
    g = np.zeros(d.kappa.shape[0], dtype=np.int64)
    for t in d.types:
        g[d.els[t]] = lev[t]
    for grp in d.nc_groups:
        assert np.all(g[grp] == g[grp[0]])
    inner = d.nbr >= 0
    assert np.all(np.abs(g[d.slot_elem[inner]] - g[d.slot_elem[d.nbr[inner]]]) <= 1)
