"""Pins of the oracle's stable time step and energy against closed forms.

The local step of Section 3.4 (eq. dtK) is
    dtau_K = C / (C_rhokappa^K C_T(N) C_J^K),
    C_rhokappa^K = max(tau_p,K kappa_K, tau_u,K / rho_K)   (face maxima),
    C_J^K = ||J^s||_inf ||J^-1||_inf                       (hex, pyramid, tet).
The tests below build single elements whose J and J^s are known in closed
form (written out here from the element geometry, not from the oracle's
vertex maps) and compare with ``Disc.dt_elements``.  C_T(N) is the paper's
printed table (Appendix B, Table computedTrace).  The energy
E = 1/2 sum_K int_K (p^2 / kappa + rho |u|^2) is checked on states whose
integrals are known exactly.  A dense eigen-solve checks the real-part
bound of the spectrum (eq. bnd_re) that the time step is built from.
"""
import numpy as np
import pytest

from oracle import refel as R
from oracle.quad import gauss_legendre
from oracle.solver import Disc
from oracle.tables import COMPUTED_TRACE
from paper_1507_02557_amd.inputs import HEX, PYR, TET, WEDGE, Mesh, four_slab_mesh

CFL = 0.5


def _mesh(etype, verts, xyz, kappa=None, rho=None):
    n = len(verts)
    ev = -np.ones((n, 8), dtype=np.int64)
    for i, v in enumerate(verts):
        ev[i, : len(v)] = v
    return Mesh(xyz=np.asarray(xyz, dtype=np.float64), etype=np.asarray(etype, dtype=np.int8), everts=ev,
                kappa=np.ones(n) if kappa is None else np.asarray(kappa, float),
                rho=np.ones(n) if rho is None else np.asarray(rho, float))


def _dt_of(mesh, N, t):
    d = Disc(mesh, N)
    return d.dt_elements(CFL)[t]


def _tri_area(a, b, c):
    return 0.5 * np.linalg.norm(np.cross(np.asarray(b) - a, np.asarray(c) - a))


@pytest.mark.parametrize("N", [1, 3])
def test_dt_single_trapezoidal_hex(N):
    """x = (1+r)/2 (1 + (1+s)/2), y = (1+s)/2, z = (1+t)/2: dx/dxi is upper
    triangular with diagonal ((1 + (1+s)/2)/2, 1/2, 1/2), so
    J = (1 + (1+s)/2)/8 with minimum 1/8 on the face s = -1 (a vertex value).
    The face s = +1 (y = 1, x in [0, 2]) has J^s = 2/4 = 1/2, the largest of
    all faces (the slanted face r = +1 has sqrt(2)/4, the faces t = +-1 at
    most (1 + (1+s)/2)/4 < 1/2 at GL points).  C_J = (1/2) / (1/8) = 4; one
    element with kappa = rho = 1 has tau_p = tau_u = 1, C_rhokappa = 1."""
    xyz = [[0, 0, 0], [1, 0, 0], [2, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [2, 1, 1], [0, 1, 1]]
    m = _mesh([HEX], [list(range(8))], xyz)
    expect = CFL / (1.0 * COMPUTED_TRACE[HEX][N - 1] * 4.0)
    assert abs(_dt_of(m, N, R.HEX)[0] - expect) < 1e-13 * expect


@pytest.mark.parametrize("N", [1, 2, 4])
def test_dt_single_pyramid_with_trapezoidal_base(N):
    """Pyramid on a planar trapezoid.  With X(a, b) the bilinear base map,
    J(a, b) = det[X_a, X_b, (x_apex - X)/2] does not depend on the collapsed
    coordinate and is bilinear in (a, b), so its minimum is at a base vertex,
    where J_i = det[e_a, e_b, x_apex - x_i] / 8 with e_a, e_b the base edges
    along a and b at vertex i.  The base's J^s = |X_a x X_b| is linear in
    (a, b) (planar quadrilateral), taken at the GL points of the face rule;
    the triangles have J^s = area / reference area (2 or 2 sqrt 2)."""
    V = np.array([[0, 0, 0], [2, 0, 0], [1.5, 1, 0], [0.5, 1, 0], [0.3, 0.4, 1.2]], dtype=np.float64)
    m = _mesh([PYR], [list(range(5))], V)
    V0, V1, V2, V3, V4 = V
    ea = {0: V1 - V0, 1: V1 - V0, 2: V2 - V3, 3: V2 - V3}
    eb = {0: V3 - V0, 1: V2 - V1, 2: V2 - V1, 3: V3 - V0}
    Jv = [np.linalg.det(np.stack([ea[i], eb[i], V4 - V[i]], 1)) / 8.0 for i in range(4)]
    assert min(Jv) > 0
    x, _ = gauss_legendre(N + 1)
    js_base = 0.0
    for a in x:
        for b in x:
            Xa = 0.5 * ((1 - b) / 2 * (V1 - V0) + (1 + b) / 2 * (V2 - V3))
            Xb = 0.5 * ((1 - a) / 2 * (V3 - V0) + (1 + a) / 2 * (V2 - V1))
            js_base = max(js_base, np.linalg.norm(np.cross(Xa, Xb)))
    js_tri = max(_tri_area(V0, V1, V4) / 2.0, _tri_area(V0, V3, V4) / 2.0,
                 _tri_area(V1, V2, V4) / (2.0 * np.sqrt(2.0)), _tri_area(V3, V2, V4) / (2.0 * np.sqrt(2.0)))
    cj = max(js_base, js_tri) / min(Jv)
    expect = CFL / (COMPUTED_TRACE[PYR][N - 1] * cj)
    assert abs(_dt_of(m, N, R.PYR)[0] - expect) < 1e-12 * expect


@pytest.mark.parametrize("N", [1, 3])
def test_dt_single_tet(N):
    """Affine tetrahedron (0,0,0), (1,0,0), (0,2,0), (0,0,3): J = volume / (4/3)
    = 6/8, J^s = area / reference area (2 for the three right triangles,
    2 sqrt 3 for the slanted face); the largest is the face x = 0 (area 3)."""
    xyz = [[0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 3]]
    m = _mesh([TET], [[0, 1, 2, 3]], xyz)
    J = 1.0 * 2.0 * 3.0 / 6.0 / (4.0 / 3.0)
    areas = [1.0, 3.0, 1.5, 0.5 * np.sqrt(4 + 36 + 9)]
    js = max(areas[0] / 2, areas[1] / 2, areas[2] / 2, areas[3] / (2 * np.sqrt(3.0)))
    expect = CFL / (COMPUTED_TRACE[TET][N - 1] * js / J)
    assert abs(_dt_of(m, N, R.TET)[0] - expect) < 1e-12 * expect


def test_dt_material_factor_two_tets():
    """Two tetrahedra sharing a face with (kappa, rho) = (2, 1/2) and (1, 3):
    rho c = 1 and sqrt 3; the shared face has {rho c} = (1 + sqrt 3)/2,
    boundary faces the element's own rho c.  C_rhokappa^K =
    max(kappa_K max_f 1/{rho c}, max_f {rho c} / rho_K)."""
    xyz = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]]
    m = _mesh([TET, TET], [[0, 1, 2, 3], [1, 2, 3, 4]], xyz, kappa=[2.0, 1.0], rho=[0.5, 3.0])
    if np.linalg.det(np.stack([np.subtract(xyz[v], xyz[1]) for v in (2, 3, 4)], 1)) < 0:
        m.everts[1, :4] = [1, 3, 2, 4]
    d = Disc(m, 2)
    dte = d.dt_elements(CFL)[R.TET]
    rc = [1.0, np.sqrt(3.0)]
    avg = 0.5 * (rc[0] + rc[1])
    crk = [max(2.0 * max(1 / rc[0], 1 / avg), max(rc[0], avg) / 0.5),
           max(1.0 * max(1 / rc[1], 1 / avg), max(rc[1], avg) / 3.0)]
    for k in range(2):
        P = np.array([xyz[v] for v in m.everts[k, :4]], dtype=float)
        J = abs(np.linalg.det((P[1:] - P[0]).T)) / 6.0 / (4.0 / 3.0)
        faces = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
        ref = {(0, 1, 2): 2.0, (0, 1, 3): 2.0, (0, 2, 3): 2.0, (1, 2, 3): 2.0 * np.sqrt(3.0)}
        js = max(_tri_area(*P[list(f)]) / ref[f] for f in faces)
        expect = CFL / (crk[k] * COMPUTED_TRACE[TET][1] * js / J)
        assert abs(dte[k] - expect) < 1e-12 * expect, (k, dte[k], expect)


# --- energy (Section 3, the scaled mass matrix M) --------------------------
def _tet_volumes(P):
    return abs(np.linalg.det(np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], -1))) / 6.0


def _element_volume(t, P):
    """Volume of a flat-faced element by tetrahedral decomposition."""
    split = {HEX: [(0, 1, 3, 4), (1, 2, 3, 6), (1, 4, 5, 6), (3, 4, 6, 7), (1, 3, 4, 6)],
             WEDGE: [(0, 1, 2, 3), (1, 2, 3, 4), (2, 3, 4, 5)],
             PYR: [(0, 1, 2, 4), (0, 2, 3, 4)], TET: [(0, 1, 2, 3)]}[t]
    return sum(_tet_volumes(P[list(s)]) for s in split)


def test_energy_of_constant_state_is_half_volume_weighted():
    """p = p0, u = u0 constant on an unjittered four-slab mesh with random
    per-element kappa, rho: E = 1/2 sum_K |K| (p0^2 / kappa_K + rho_K |u0|^2),
    with |K| from a tetrahedral decomposition of each (flat-faced) element."""
    m = four_slab_mesh(4, seed=0, jitter=0.0)
    rng = np.random.default_rng(17)
    m.kappa = rng.uniform(0.5, 2.0, m.n_elem)
    m.rho = rng.uniform(0.5, 2.0, m.n_elem)
    p0, u0 = 1.7, np.array([0.3, -0.8, 0.5])
    d = Disc(m, 2)
    U = d.project(lambda x, y, z, t: (p0 + 0 * x, u0[0] + 0 * x, u0[1] + 0 * x, u0[2] + 0 * x))
    vol = np.array([_element_volume(int(m.etype[e]), m.xyz[m.everts[e, :{0: 8, 1: 6, 2: 5, 3: 4}[int(m.etype[e])]]])
                    for e in range(m.n_elem)])
    assert abs(vol.sum() - 1.0) < 1e-13
    expect = 0.5 * np.sum(vol * (p0 ** 2 / m.kappa + m.rho * (u0 @ u0)))
    assert abs(d.energy(U) - expect) < 1e-12 * expect


@pytest.mark.parametrize("N", [1, 2])
def test_energy_of_linear_state_on_the_unit_cube(N):
    """p = x + 2y - z, u = (y, 0, x), kappa = rho = 1 on the unit cube
    (unjittered mesh, so every space holds linear fields exactly):
    E = 1/2 int (p^2 + y^2 + x^2) with int p^2 = 1/3 + 4/3 + 1/3 + 2 (2/4 - 1/4 - 2/4)
    = 3/2 and int x^2 = int y^2 = 1/3."""
    m = four_slab_mesh(4, seed=0, jitter=0.0)
    d = Disc(m, N)
    U = d.project(lambda x, y, z, t: (x + 2 * y - z, y, 0 * x, x))
    ip2 = 1 / 3 + 4 / 3 + 1 / 3 + 2 * (2 * 0.25 - 0.25 - 2 * 0.25)
    expect = 0.5 * (ip2 + 1 / 3 + 1 / 3)
    assert abs(d.energy(U) - expect) < 1e-12


# --- spectrum vs. the real-part bound (Section 3.4, eq. bnd_re) -------------
def _dense_operator(d):
    """M^-1 A as a dense matrix, column by column from the right-hand side."""
    shapes = [(t, d.zeros()[t].shape) for t in d.types]
    sizes = [int(np.prod(s)) for _, s in shapes]
    n = sum(sizes)
    A = np.zeros((n, n))
    for j in range(n):
        x = np.zeros(n)
        x[j] = 1.0
        U, o = {}, 0
        for (t, s), k in zip(shapes, sizes):
            U[t] = x[o:o + k].reshape(s)
            o += k
        Rr = d.rhs(U)
        A[:, j] = np.concatenate([Rr[t].ravel() for t, _ in shapes])
    return A


@pytest.mark.parametrize("slabs,N", [(("hex", "wedge"), 1), (("pyrtet", "tet"), 1), (("pyrtet", "tet"), 2)])
def test_spectrum_within_trace_bound(slabs, N):
    """|Re lambda(M^-1 A)| <= max_K C_rhokappa C_T(N) C_J^K = C / min_K dtau_K
    (eq. bnd_re with the computed reference trace constants), the spectrum
    has no positive real part (energy stability), and the bound is within a
    small factor of rho(M^-1 A) (Table bounds: a factor below 2 in the paper)."""
    m = four_slab_mesh(2, seed=3, jitter=0.1, slabs=slabs)
    rng = np.random.default_rng(1)
    m.kappa = rng.uniform(0.7, 1.4, m.n_elem)
    m.rho = rng.uniform(0.7, 1.4, m.n_elem)
    d = Disc(m, N)
    lam = np.linalg.eigvals(_dense_operator(d))
    bound = CFL / d.dt_min(CFL)
    rho_spec = np.abs(lam).max()
    assert lam.real.max() < 1e-9 * rho_spec
    assert np.abs(lam.real).max() <= bound
    assert rho_spec <= bound < 4.0 * rho_spec, (rho_spec, bound)
