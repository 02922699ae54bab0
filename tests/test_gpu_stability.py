"""Per-element trace constants and the time steps built from them, library
against the FP64 oracle (needs an MI355X).

The library computes C_T(N, K), the largest eigenvalue of M_s,K v = lambda
M_K v (Section 3.4), on the device in FP64 from its stored FP32 geometric
factors; the oracle solves the same generalised eigenproblem densely from its
own FP64 geometry.  Bar: relative difference <= 2e-6 per element (FP32
factors).  With the per-element constants selected, the local steps, the
multi-rate levels and a multi-rate run must match the oracle's built from
its own constants.
"""
import numpy as np
import pytest

from oracle import stability as ST
from oracle.mrab import MRAB3, bin_levels
from oracle.solver import Disc
from paper_1507_02557_amd import hdg
from paper_1507_02557_amd.inputs import four_slab_mesh, standing_mode_rigid

from .parity_util import lib_state_to_oracle

pytestmark = pytest.mark.gpu

TOL = 2e-6


def _global(disc, per_type):
    out = np.zeros(sum(disc.els[t].size for t in disc.types))
    for t in disc.types:
        out[disc.els[t]] = per_type[t]
    return out


@pytest.mark.parametrize("refine", [1, 2])
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_trace_constants_match_oracle(N, refine):
    m = four_slab_mesh(4, seed=0, jitter=0.1, refine_last=refine)
    d = Disc(m, N)
    s = hdg.Solver(m, N)
    ct = s.trace_constants()
    ref = _global(d, ST.trace_constants(d))
    err = np.abs(ct - ref) / ref
    print("N", N, "refine", refine, "max rel err", err.max())
    assert err.max() < TOL, (int(np.argmax(err)), err.max())


def test_trace_constants_at_order_5_and_random_materials():
    m = four_slab_mesh(4, seed=4, jitter=0.1)
    rng = np.random.default_rng(2)
    m.kappa = rng.uniform(0.5, 2.0, m.n_elem)
    m.rho = rng.uniform(0.5, 2.0, m.n_elem)
    N = 5
    d = Disc(m, N)
    s = hdg.Solver(m, N)
    ct = s.trace_constants()
    ref = _global(d, ST.trace_constants(d))
    assert np.max(np.abs(ct - ref) / ref) < TOL
    s.set_dt_mode(hdg.DT_ELEMENT)
    dte, mn = s.dt(0.5)
    refdt = _global(d, ST.dt_elements_computed(d, 0.5))
    assert np.max(np.abs(dte - refdt) / refdt) < TOL
    assert abs(mn - refdt.min()) < TOL * mn


def test_element_constants_give_longer_steps_and_oracle_levels():
    m = four_slab_mesh(4, seed=0, jitter=0.1, refine_last=2)
    N, L = 3, 3
    d = Disc(m, N)
    s = hdg.Solver(m, N)
    dt_ref, mn_ref = s.dt(0.5)
    s.set_dt_mode(hdg.DT_ELEMENT)
    dt_el, mn_el = s.dt(0.5)
    assert np.all(dt_el >= dt_ref * (1 - 1e-6))
    assert mn_el > mn_ref
    dtmin, cnt, lev = s.mrab_setup(L)
    level, odtmin = bin_levels(d, L, 0.5, ST.dt_elements_computed(d, 0.5))
    assert np.array_equal(lev.astype(np.int64), _global(d, level).astype(np.int64))
    assert abs(dtmin - odtmin) < TOL * dtmin
    s.set_dt_mode(hdg.DT_REFERENCE)
    dtmin_ref, _, _ = s.mrab_setup(L)
    # levels are relative to dtau_min; what the tighter constants buy is a
    # longer coarse step (2^(L-1) dtau_min) for the same work per substep
    assert dtmin > dtmin_ref


def test_multirate_run_with_element_constants_matches_oracle():
    m = four_slab_mesh(4, seed=0, jitter=0.1)
    N, L = 3, 3
    d = Disc(m, N)
    mr = MRAB3(d, L, dte=ST.dt_elements_computed(d, 0.5))
    s = hdg.Solver(m, N)
    s.set_dt_mode(hdg.DT_ELEMENT)
    s.mrab_setup(L)
    U = mr.startup(d.project(standing_mode_rigid))
    s.project_function(standing_mode_rigid)
    s.mrab_advance(0)
    for _ in range(3):
        U = mr.coarse_step(U)
    s.mrab_advance(3)
    rel = d.rel_l2(lib_state_to_oracle(s), U)
    print("MRAB with element constants, rel L2", rel)
    assert rel < 1e-5
