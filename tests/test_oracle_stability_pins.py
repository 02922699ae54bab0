"""Pins of the oracle's per-element trace constants and spectral bounds
(Section 3.2; Section 3.4, eq. bnd_re, eq. dtK, Table bounds).

* On the reference element itself C_T(N, K) is the reference constant C_T(N)
  of Appendix B (Table computedTrace; the hexahedron's closed form
  3 (N + 1)(N + 2) / 2 exactly), and an element scaled by h has C_T / h
  (M_s scales with h^2, M with h^3).
* C_T(N, K) <= C_T(N) C_J^K on every element of jittered hybrid meshes,
  conforming and 1:4 non-conforming: M_K >= min J Mhat and
  M_s,K <= max J^s Mhat_s as quadratic forms (wedges: J^s / J).
* On small hybrid meshes with random kappa, rho, a dense eigen-solve of
  M^{-1} A and of its symmetric part in the energy inner product: the
  symmetric part is negative semi-definite (the upwind flux dissipates,
  Section 3.1), every Re lambda lies in its spectrum's range (a Rayleigh
  quotient), and the chain of Table bounds holds:
  |Re lambda| <= rho(M^-1 A) <= rho(M^-1 A^s) <= max_K C_rhokappa C_T(N, K)
  <= max_K C_rhokappa C_T(N) C_J^K = C / min dtau_K.
"""
import numpy as np
import pytest

from oracle import refel as R
from oracle import stability as ST
from oracle.solver import Disc
from oracle.tables import COMPUTED_TRACE
from paper_1507_02557_amd.inputs import Mesh, four_slab_mesh

from .test_oracle_dt_energy_pins import _dense_operator

TYPES = (R.HEX, R.WEDGE, R.PYR, R.TET)


def _single(t, N, scale=1.0, shift=(0.0, 0.0, 0.0)):
    E = R.make(t, N)
    ev = -np.ones((1, 8), dtype=np.int64)
    ev[0, : E.nv] = np.arange(E.nv)
    xyz = np.asarray(E.vref, dtype=np.float64) * scale + np.asarray(shift)
    m = Mesh(xyz=xyz, etype=np.array([t], dtype=np.int8), everts=ev, kappa=np.ones(1), rho=np.ones(1))
    return Disc(m, N)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("t", TYPES)
def test_reference_element_gives_the_reference_constant(t, N):
    ct = ST.trace_constants(_single(t, N))[t][0]
    assert abs(ct - COMPUTED_TRACE[t][N - 1]) <= 0.0051, (t, N, ct)
    if t == R.HEX:
        assert abs(ct - 1.5 * (N + 1) * (N + 2)) < 1e-10 * ct


@pytest.mark.parametrize("t", TYPES)
def test_scaled_element_constant_scales_with_one_over_h(t):
    N = 2
    c1 = ST.trace_constants(_single(t, N))[t][0]
    ch = ST.trace_constants(_single(t, N, scale=0.25, shift=(3.0, -1.0, 2.0)))[t][0]
    assert abs(ch - 4.0 * c1) < 1e-10 * ch


@pytest.mark.parametrize("refine", [1, 2])
@pytest.mark.parametrize("N", [1, 3])
def test_per_element_constant_is_below_the_reference_bound(N, refine):
    m = four_slab_mesh(4, seed=5, jitter=0.1, refine_last=refine)
    d = Disc(m, N)
    ct = ST.trace_constants(d)
    ref = {t: ST.trace_constants(_single(t, N))[t][0] for t in d.types}
    crk = d.c_rhokappa()
    dte = d.dt_elements(0.5)
    for t in d.types:
        cj = 0.5 / (dte[t] * crk[t] * COMPUTED_TRACE[t][N - 1])   # C_J^K from the oracle's own dt
        bound = ref[t] * cj
        assert np.all(ct[t] <= bound * (1 + 1e-10)), (t, np.max(ct[t] / bound))
        assert np.all(ct[t] > 0)
    dtc = ST.dt_elements_computed(d, 0.5)
    for t in d.types:
        # the computed constants give longer (or equal) local steps
        assert np.all(dtc[t] >= dte[t] * (1 - 1e-3)), t


@pytest.mark.parametrize("slabs,N", [(("hex", "wedge"), 1), (("pyrtet", "tet"), 1), (("pyrtet", "tet"), 2),
                                     (("hex", "wedge"), 2)])
def test_table_bounds_ordering(slabs, N):
    m = four_slab_mesh(2, seed=3, jitter=0.1, slabs=slabs)
    rng = np.random.default_rng(1)
    m.kappa = rng.uniform(0.7, 1.4, m.n_elem)
    m.rho = rng.uniform(0.7, 1.4, m.n_elem)
    d = Disc(m, N)
    L = _dense_operator(d)
    W = ST.energy_weights(d)
    mu = ST.symmetric_part_spectrum(L, W)
    lam = np.linalg.eigvals(L)
    rho_l = np.abs(lam).max()
    rho_s = np.abs(mu).max()
    assert mu.max() <= 1e-10 * rho_s                     # dissipative symmetric part
    assert lam.real.min() >= mu.min() * (1 + 1e-9)       # Re lambda in the symmetric part's range
    assert lam.real.max() <= 1e-9 * rho_l
    ct = ST.trace_constants(d)
    crk = d.c_rhokappa()
    b_k = max(float(np.max(crk[t] * ct[t])) for t in d.types)
    b_ref = 0.5 / d.dt_min(0.5)
    assert np.abs(lam.real).max() <= rho_l <= rho_s <= b_k <= b_ref, (rho_l, rho_s, b_k, b_ref)
