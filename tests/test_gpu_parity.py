"""Parity of the HIP library with the FP64 oracle (needs an MI355X).

Tolerances: the library computes in FP32 from FP64-built operators and
geometry.  A right-hand side entry is a sum of O(Np + faces*Nfq) FP32
products, so its rounding error is a few hundred ulp of the largest term at
worst; measured errors are ~4e-7 of max|rhs|.  The bar used here is 1e-5
relative (max-norm per element type), and rel L2 <= 1e-5 for whole runs,
the FP32 target of the method's single-precision path.
"""
import numpy as np
import pytest
import torch

from oracle import refel as R
from oracle.solver import BC_FREE_SURFACE, BC_RIGID_WALL, Disc, lserk4_step
from paper_1507_02557_amd import hdg
from paper_1507_02557_amd.inputs import four_slab_mesh, gaussian_pulse, pulse_centre, standing_mode_rigid

from .parity_util import lib_state_to_oracle, local_index, patch_mesh, random_state, set_lib_state, type_rel_err

pytestmark = pytest.mark.gpu

TOL_RHS = 1e-5
PATHS = [hdg.PATH_AUTO, hdg.PATH_GENERIC]


@pytest.fixture(scope="module")
def slab4_mesh():
    return four_slab_mesh(4, seed=0, jitter=0.1)


def _global_dt(disc, d_el):
    out = np.zeros(sum(disc.els[t].size for t in disc.types))
    for t in disc.types:
        out[disc.els[t]] = d_el[t]
    return out


def test_dt_matches_oracle(slab4_mesh):
    d = Disc(slab4_mesh, 3)
    s = hdg.Solver(slab4_mesh, 3)
    dte, mn = s.dt(0.5)
    ref = _global_dt(d, d.dt_elements(0.5))
    assert np.max(np.abs(dte - ref) / ref) < 1e-12
    assert abs(mn - d.dt_min(0.5)) < 1e-12 * mn


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_rhs_matches_oracle(slab4_mesh, N, path):
    d = Disc(slab4_mesh, N)
    s = hdg.Solver(slab4_mesh, N, path=path)
    assert s.get_path() == (path, 1 if path == hdg.PATH_AUTO else 0)
    U = random_state(d, seed=N)
    set_lib_state(s, U)
    Rl = {t: v.double().cpu().numpy() for t, v in s.rhs().items()}
    err = type_rel_err(Rl, d.rhs(U))
    print("N", N, "rel err per type", err)
    assert max(err.values()) < TOL_RHS, err


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_rhs_free_surface_and_materials(N, path):
    """Free-surface mirror states and random materials, at every order the
    matrix-core pyramid kernel serves (N = 3..5) and one it does not."""
    m = four_slab_mesh(4, seed=5, jitter=0.1)
    rng = np.random.default_rng(9)
    m.kappa = rng.uniform(0.5, 2.0, m.n_elem)
    m.rho = rng.uniform(0.5, 2.0, m.n_elem)
    d = Disc(m, N, bc=BC_FREE_SURFACE)
    s = hdg.Solver(m, N, bc=hdg.BC_FREE_SURFACE, path=path)
    U = random_state(d, seed=3)
    set_lib_state(s, U)
    Rl = {t: v.double().cpu().numpy() for t, v in s.rhs().items()}
    err = type_rel_err(Rl, d.rhs(U))
    assert max(err.values()) < TOL_RHS, err
    dte, _ = s.dt(0.5)
    ref = _global_dt(d, d.dt_elements(0.5))
    assert np.max(np.abs(dte - ref) / ref) < 1e-12


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N", [2, 4])
def test_rhs_per_face_boundary_conditions(N, path):
    """Free-surface and rigid-wall faces mixed at random on the boundary
    (per element and local face), random materials."""
    m = four_slab_mesh(4, seed=3, jitter=0.1)
    rng = np.random.default_rng(9)
    m.kappa = rng.uniform(0.5, 2.0, m.n_elem)
    m.rho = rng.uniform(0.5, 2.0, m.n_elem)
    m.bc_face = rng.integers(-1, 2, size=(m.n_elem, 6)).astype(np.int8)
    d = Disc(m, N, bc=BC_FREE_SURFACE)
    s = hdg.Solver(m, N, bc=hdg.BC_FREE_SURFACE, path=path)
    U = random_state(d, seed=30 + N)
    set_lib_state(s, U)
    Rl = {t: v.double().cpu().numpy() for t, v in s.rhs().items()}
    err = type_rel_err(Rl, d.rhs(U))
    assert max(err.values()) < TOL_RHS, err


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("slabs,n", [(("hex",), 1), (("tet",), 1), (("pyr6",), 2), (("wedge",), 2), (("pyrtet",), 2)])
def test_single_type_meshes(slabs, n, path):
    """Single-element and single-type meshes (all faces on the boundary for n=1)."""
    m = four_slab_mesh(n, seed=2, jitter=0.1, slabs=slabs)
    d = Disc(m, 3)
    s = hdg.Solver(m, 3, path=path)
    U = random_state(d, seed=7)
    set_lib_state(s, U)
    Rl = {t: v.double().cpu().numpy() for t, v in s.rhs().items()}
    err = type_rel_err(Rl, d.rhs(U))
    assert max(err.values()) < TOL_RHS, err


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N", [2, 4, 5])
def test_ragged_batches_match_oracle(slab4_mesh, N, path):
    """A patch of the n=4 mesh whose per-type element counts are not multiples
    of the kernels' batch and tile sizes (odd counts, partial 16-element tiles):
    right-hand side and three LSERK4 steps against the oracle."""
    rng = np.random.default_rng(11)
    centre = np.concatenate([rng.choice(np.nonzero(slab4_mesh.etype == t)[0], 3, replace=False) for t in range(4)])
    m, _, _ = patch_mesh(slab4_mesh, centre)
    counts = [int(np.sum(m.etype == t)) for t in range(4)]
    print("element counts per type", counts)
    assert any(k % 2 == 1 for k in counts) and any(k % 16 != 0 for k in counts)
    d = Disc(m, N)
    s = hdg.Solver(m, N, path=path)
    U = random_state(d, seed=3)
    set_lib_state(s, U)
    Rl = {t: v.double().cpu().numpy() for t, v in s.rhs().items()}
    err = type_rel_err(Rl, d.rhs(U))
    assert max(err.values()) < TOL_RHS, err
    dt = d.dt_min(0.5)
    Uo = U
    for _ in range(3):
        Uo = lserk4_step(d, Uo, dt)
    s.step(dt, 3)
    rel = d.rel_l2(lib_state_to_oracle(s), Uo)
    print("rel L2 after 3 steps", rel)
    assert rel < 1e-5


def test_projection_matches_oracle(slab4_mesh):
    d = Disc(slab4_mesh, 3)
    s = hdg.Solver(slab4_mesh, 3)
    s.project_function(standing_mode_rigid)
    err = type_rel_err(lib_state_to_oracle(s), d.project(standing_mode_rigid))
    assert max(err.values()) < 1e-6, err


@pytest.mark.parametrize("path", PATHS)
def test_slab4_standing_mode_100_steps(slab4_mesh, path):
    """The n=4 jittered four-slab mesh, N=3, rigid walls, standing
    mode, 100 LSERK4 steps at the derived stable step: rel L2 <= 1e-5."""
    d = Disc(slab4_mesh, 3)
    s = hdg.Solver(slab4_mesh, 3, path=path)
    dt = d.dt_min(0.5)
    Uo = d.project(standing_mode_rigid)
    s.project_function(standing_mode_rigid)
    E0 = s.energy()
    assert abs(E0 - d.energy(Uo)) < 1e-6 * E0
    for _ in range(100):
        Uo = lserk4_step(d, Uo, dt)
    s.step(dt, 100)
    Ul = lib_state_to_oracle(s)
    rel = d.rel_l2(Ul, Uo)
    print("n=4 mesh, rel L2 after 100 steps:", rel)
    assert rel < 1e-5
    E1 = s.energy()
    assert abs(E1 - d.energy(Uo)) < 1e-6 * E1
    assert E1 <= E0 * (1 + 1e-6)
    e_lib = d.l2_error(Ul, standing_mode_rigid, 100 * dt)
    e_or = d.l2_error(Uo, standing_mode_rigid, 100 * dt)
    assert abs(e_lib - e_or) < 1e-3 * e_or


def test_energy_nonincreasing(slab4_mesh):
    s = hdg.Solver(slab4_mesh, 3)
    s.project_function(standing_mode_rigid)
    _, dt = s.dt(0.5)
    E = [s.energy()]
    for _ in range(10):
        s.step(dt, 10)
        E.append(s.energy())
    assert all(b <= a * (1 + 1e-6) for a, b in zip(E, E[1:])), E


def test_bitwise_deterministic(slab4_mesh):
    out = []
    for _ in range(2):
        s = hdg.Solver(slab4_mesh, 4)
        s.project_function(standing_mode_rigid)
        _, dt = s.dt(0.5)
        s.step(dt, 7)
        out.append(lib_state_to_oracle(s))
    for t in out[0]:
        assert np.array_equal(out[0][t], out[1][t])


def test_inverted_element_rejected():
    m = four_slab_mesh(1, seed=0, jitter=0.0, slabs=("tet",))
    m.everts[0, [2, 3]] = m.everts[0, [3, 2]]
    with pytest.raises(hdg.HdgError, match=r"\(-2\).*Jacobian"):
        hdg.Solver(m, 2)


def test_full_size_sampled_rhs():
    """The benchmark's workload (n=48 four-slab mesh, N=4, 527,616 elements) in
    its launch configuration: a random state, one right-hand side,
    checked against the oracle on a patch around 160 sampled elements."""
    m = four_slab_mesh(48, seed=0, jitter=0.1)
    s = hdg.Solver(m, 4)
    gen = torch.Generator(device="cpu").manual_seed(1234)
    for t in s.types:
        K, Np, _ = s.info[t]
        s.set_state(t, [torch.randn(K, Np, generator=gen) for _ in range(4)])
    Rl = s.rhs()
    tglob, tidx = local_index(m)
    rng = np.random.default_rng(4)
    centre = np.concatenate([rng.choice(np.nonzero(m.etype == t)[0], 40, replace=False) for t in s.types])
    sub, ids, pos = patch_mesh(m, centre)
    d = Disc(sub, 4)
    U = {t: np.zeros(d.zeros()[t].shape) for t in d.types}
    full = {t: s.get_field(t).double().cpu().numpy() for t in s.types}
    for t in d.types:
        U[t] = full[t][tidx[ids[d.els[t]]]]
    Ro = d.rhs(U)
    loc_in_type = {}
    for t in d.types:
        loc_in_type.update({int(g): (t, k) for k, g in enumerate(d.els[t])})
    for t in s.types:
        rl, ro = [], []
        for p in pos:
            tt, k = loc_in_type[int(p)]
            if tt != t:
                continue
            rl.append(Rl[t][tidx[ids[p]]].double().cpu().numpy())
            ro.append(Ro[t][k])
        rl, ro = np.array(rl), np.array(ro)
        rel = np.abs(rl - ro).max() / np.abs(ro).max()
        print("type", t, "sampled rel err", rel)
        assert rel < TOL_RHS
    # one LSERK4 step of the Gaussian pulse stays finite and energy-stable
    s.project_function(lambda x, y, z, tt: gaussian_pulse(x, y, z, pulse_centre(0)))
    _, dt = s.dt(0.5)
    E0 = s.energy()
    s.step(dt, 2)
    E1 = s.energy()
    assert np.isfinite(E1) and E1 <= E0 * (1 + 1e-6)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("N,L", [(2, 3), (3, 2)])
def test_mrab_matches_oracle(slab4_mesh, N, L, path):
    """Multi-rate AB3 (levels, start-up and coarse steps) against the oracle."""
    from oracle.mrab import MRAB3
    d = Disc(slab4_mesh, N)
    mr = MRAB3(d, L)
    s = hdg.Solver(slab4_mesh, N, path=path)
    dtmin, cnt, lev = s.mrab_setup(L)
    g = np.zeros(slab4_mesh.n_elem, dtype=np.int64)
    for t in d.types:
        g[d.els[t]] = mr.level[t]
    assert np.array_equal(g, lev.astype(np.int64))
    assert abs(dtmin - mr.dtmin) < 1e-12 * dtmin
    U = mr.startup(d.project(standing_mode_rigid))
    s.project_function(standing_mode_rigid)
    tl = s.mrab_advance(0)
    assert abs(tl - mr.t) < 1e-12
    for _ in range(3):
        U = mr.coarse_step(U)
    s.mrab_advance(3)
    rel = d.rel_l2(lib_state_to_oracle(s), U)
    print("MRAB N", N, "L", L, "rel L2", rel)
    assert rel < 1e-5


@pytest.mark.parametrize("materials", ["uniform", "random kappa"])
@pytest.mark.parametrize("N", [3, 4])
def test_mrab_level_sorted_storage_matches_oracle(slab4_mesh, N, materials):
    """Elements of each type stored finest level first: the multi-rate kernels
    run without indirection (contiguous tiles, one-level tiles of the
    tetrahedron update as float4 vectors) and still match the oracle.
    Log-uniform kappa in [1/4, 4] spreads every type over the levels, so
    tiles mixing two levels occur too."""
    from oracle.mrab import MRAB3
    L = 3
    base = slab4_mesh
    if materials != "uniform":
        base = slab4_mesh.permuted(np.arange(slab4_mesh.n_elem))
        rng = np.random.default_rng(4)
        base.kappa = np.exp(rng.uniform(np.log(0.25), np.log(4.0), base.n_elem))
    s0 = hdg.Solver(base, N)
    _, _, lev = s0.mrab_setup(L)
    s0.close()
    mesh = base.permuted(base.level_order(lev))
    d = Disc(mesh, N)
    mr = MRAB3(d, L)
    s = hdg.Solver(mesh, N)
    _, _, lev2 = s.mrab_setup(L)
    assert np.array_equal(lev2, lev[base.level_order(lev)])
    U = mr.startup(d.project(standing_mode_rigid))
    s.project_function(standing_mode_rigid)
    s.mrab_advance(0)
    for _ in range(3):
        U = mr.coarse_step(U)
    s.mrab_advance(3)
    rel = d.rel_l2(lib_state_to_oracle(s), U)
    print("MRAB level-sorted N", N, "rel L2", rel)
    assert rel < 1e-5


def test_mrab_full_size_runs_and_stays_bounded():
    """Multi-rate run on the n=48 four-slab mesh, N=3, three
    levels: start-up and one coarse step stay finite with bounded energy."""
    m = four_slab_mesh(48, seed=0, jitter=0.1)
    s = hdg.Solver(m, 3)
    dtmin, cnt, _ = s.mrab_setup(3)
    assert cnt.sum() == m.n_elem
    s.project_function(lambda x, y, z, tt: gaussian_pulse(x, y, z, pulse_centre(0)))
    E0 = s.energy()
    s.mrab_advance(1)
    E1 = s.energy()
    assert np.isfinite(E1) and E1 <= E0 * (1 + 1e-3)


def test_paths_agree_after_steps(slab4_mesh):
    """Lattice traces with matrix-core tetrahedra and cubature traces with the
    vector kernels compute the same operator: 20 LSERK4 steps agree to FP32
    rounding."""
    out = []
    for path in PATHS:
        s = hdg.Solver(slab4_mesh, 4, path=path)
        s.project_function(standing_mode_rigid)
        _, dt = s.dt(0.5)
        s.step(dt, 20)
        out.append({t: s.get_field(t).double().cpu().numpy() for t in s.types})
    d = Disc(slab4_mesh, 4)
    assert d.rel_l2(out[0], out[1]) < 2e-6


def _wedge_tet_mesh():
    """A wedge and a tetrahedron sharing the wedge's triangular face s = -1,
    plus a pyramid on one quadrilateral face: lattice traces must be off."""
    from paper_1507_02557_amd.inputs import Mesh
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 0, 1],        # wedge s=-1 triangle (y = 0)
                    [0, 1, 0], [1, 1, 0], [0, 1, 1],        # wedge s=+1 triangle (y = 1)
                    [0.3, -0.8, 0.3],                       # tet apex below y = 0
                    [0.4, 0.5, -0.9]], dtype=np.float64)    # pyramid apex below z = 0
    ev = -np.ones((3, 8), dtype=np.int64)
    ev[0, :6] = [0, 1, 2, 3, 4, 5]
    ev[1, :4] = [0, 1, 2, 6]
    ev[2, :5] = [0, 3, 4, 1, 7]
    m = Mesh(xyz=xyz, etype=np.array([hdg.WEDGE, hdg.TET, hdg.PYR], dtype=np.int8), everts=ev,
             kappa=np.array([1.0, 1.5, 0.8]), rho=np.array([1.0, 0.7, 1.2]))
    return m


def test_wedge_tet_face_falls_back_to_cubature_traces():
    m = _wedge_tet_mesh()
    d = Disc(m, 3)
    s = hdg.Solver(m, 3)
    assert s.get_path() == (hdg.PATH_AUTO, 0)
    U = random_state(d, seed=11)
    set_lib_state(s, U)
    Rl = {t: v.double().cpu().numpy() for t, v in s.rhs().items()}
    err = type_rel_err(Rl, d.rhs(U))
    assert max(err.values()) < TOL_RHS, err


PRECS = [hdg.PREC_FP16X2, hdg.PREC_FP16X2_K16, hdg.PREC_BF16X2, hdg.PREC_BF16X3]
# Right-hand-side bar per operand precision: the split FP16 modes and the
# three-piece BF16 split carry 22-24 significant bits and meet the FP32 bar;
# the two-piece BF16 split carries about 16 (x = hi + lo with 8-bit pieces),
# so one product is good to about 2^-16 relative and the bar is 1e-4.
TOL_PREC = {hdg.PREC_FP16X2: TOL_RHS, hdg.PREC_FP16X2_K16: TOL_RHS, hdg.PREC_BF16X2: 1e-4, hdg.PREC_BF16X3: TOL_RHS}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_split_precision_rhs_matches_oracle(slab4_mesh, N, prec):
    """Split-FP16 matrix-core products: the right-hand side stays within the
    FP32 tolerance of the FP64 oracle."""
    d = Disc(slab4_mesh, N)
    s = hdg.Solver(slab4_mesh, N, precision=prec)
    U = random_state(d, seed=20 + N)
    set_lib_state(s, U)
    Rl = {t: v.double().cpu().numpy() for t, v in s.rhs().items()}
    err = type_rel_err(Rl, d.rhs(U))
    print("prec", prec, "N", N, "rel err per type", err)
    assert max(err.values()) < TOL_PREC[prec], err


@pytest.mark.parametrize("prec", PRECS)
def test_split_precision_slab4_100_steps(slab4_mesh, prec):
    """The n=4 mesh at N=3 with split-FP16 products: rel L2 <= 1e-5 after 100 steps."""
    d = Disc(slab4_mesh, 3)
    s = hdg.Solver(slab4_mesh, 3, precision=prec)
    dt = d.dt_min(0.5)
    Uo = d.project(standing_mode_rigid)
    s.project_function(standing_mode_rigid)
    for _ in range(100):
        Uo = lserk4_step(d, Uo, dt)
    s.step(dt, 100)
    rel = d.rel_l2(lib_state_to_oracle(s), Uo)
    print("prec", prec, "n=4 mesh, rel L2 after 100 steps:", rel)
    assert rel < 1e-5


@pytest.mark.parametrize("prec", [hdg.PREC_FP16X2, hdg.PREC_BF16X3])
def test_split_precision_mrab(slab4_mesh, prec):
    from oracle.mrab import MRAB3
    d = Disc(slab4_mesh, 3)
    mr = MRAB3(d, 3)
    s = hdg.Solver(slab4_mesh, 3, precision=prec)
    s.mrab_setup(3)
    U = mr.startup(d.project(standing_mode_rigid))
    s.project_function(standing_mode_rigid)
    s.mrab_advance(0)
    for _ in range(2):
        U = mr.coarse_step(U)
    s.mrab_advance(2)
    assert d.rel_l2(lib_state_to_oracle(s), U) < 1e-5

