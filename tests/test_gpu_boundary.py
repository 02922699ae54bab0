"""The time-interval, watchdog and checkpoint calls of the C ABI (needs an MI355X).

* hdg_advance runs to t_final with the step shortened so that it divides the
  interval (LSERK4: n = ceil(T / dtau_min) steps of T / n; MRAB3: the same
  on the coarse step), and matches the FP64 oracle run with that step.
* The watchdog turns a NaN in the state into HDG_ENONFINITE.
* A run continued from a checkpoint is bit-identical to the uninterrupted one,
  single-rate and multi-rate.
"""
import math

import numpy as np
import pytest
import torch

from oracle.solver import Disc, lserk4_step
from paper_1507_02557_amd import hdg
from paper_1507_02557_amd.inputs import four_slab_mesh, standing_mode_rigid

from .parity_util import lib_state_to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slab4_mesh():
    return four_slab_mesh(4, seed=0, jitter=0.1)


def _state(s):
    return {t: v.cpu().numpy().copy() for t, v in s.state().items()}


def test_advance_lserk4_divides_the_interval_and_matches_oracle(slab4_mesh):
    N = 3
    d = Disc(slab4_mesh, N)
    s = hdg.Solver(slab4_mesh, N)
    s.project_function(standing_mode_rigid)
    assert s.time == 0.0
    dtmin = d.dt_min(0.5)
    T = 7.3 * dtmin
    n = s.advance(T, hdg.STEPPER_LSERK4, 0.5, check_every=3)
    assert n == math.ceil(T / dtmin) == 8
    assert s.time == T
    U = d.project(standing_mode_rigid)
    for _ in range(n):
        U = lserk4_step(d, U, T / n)
    rel = d.rel_l2(lib_state_to_oracle(s), U)
    assert rel < 1e-5, rel
    # a second call to the same time takes no step
    assert s.advance(T, hdg.STEPPER_LSERK4, 0.5) == 0 and s.time == T


def test_advance_lserk4_equals_explicit_steps(slab4_mesh):
    s1 = hdg.Solver(slab4_mesh, 2)
    s2 = hdg.Solver(slab4_mesh, 2)
    for s in (s1, s2):
        s.project_function(standing_mode_rigid)
    _, dtmin = s1.dt(0.5)
    T = 5.5 * dtmin
    n = s1.advance(T, hdg.STEPPER_LSERK4, 0.5, check_every=2)
    s2.step(T / n, n)
    a, b = _state(s1), _state(s2)
    for t in a:
        assert np.array_equal(a[t], b[t])


def test_advance_mrab_matches_oracle(slab4_mesh):
    from oracle.mrab import MRAB3
    N, L = 2, 3
    d = Disc(slab4_mesh, N)
    mr = MRAB3(d, L)
    s = hdg.Solver(slab4_mesh, N)
    dtmin, _, _ = s.mrab_setup(L)
    s.project_function(standing_mode_rigid)
    coarse = 2 ** (L - 1) * dtmin
    T = 4.6 * coarse
    n = s.advance(T, hdg.STEPPER_MRAB3, 0.5, check_every=1)
    assert n == 5 and s.time == T
    # the oracle with the shortened step: start-up (two coarse steps), then three
    mr.dtmin = T / (n * 2 ** (L - 1))
    mr.dtl = {l: (2 ** (L - l)) * mr.dtmin for l in range(1, L + 1)}
    U = mr.startup(d.project(standing_mode_rigid))
    for _ in range(n - 2):
        U = mr.coarse_step(U)
    rel = d.rel_l2(lib_state_to_oracle(s), U)
    assert rel < 1e-5, rel


def test_advance_rejects_bad_arguments(slab4_mesh):
    s = hdg.Solver(slab4_mesh, 1)
    s.project_function(standing_mode_rigid)
    with pytest.raises(hdg.HdgError) as e:
        s.advance(1e-3, hdg.STEPPER_MRAB3)
    assert e.value.code == hdg.ESTATE
    s.time = 1.0
    with pytest.raises(hdg.HdgError) as e:
        s.advance(0.5)
    assert e.value.code == hdg.EINVAL
    with pytest.raises(hdg.HdgError) as e:
        s.advance(2.0, stepper=7)
    assert e.value.code == hdg.EINVAL
    with pytest.raises(hdg.HdgError) as e:
        s.advance(2.0, cfl=0.0)
    assert e.value.code == hdg.EINVAL


def test_watchdog_reports_a_nan(slab4_mesh):
    s = hdg.Solver(slab4_mesh, 2)
    s.project_function(standing_mode_rigid)
    s.check_finite()
    t = hdg.TET
    st = s.get_field(t)
    st[3, 1, 2] = float("nan")
    s.set_state(t, [st[:, c].contiguous() for c in range(4)])
    with pytest.raises(hdg.HdgError) as e:
        s.check_finite()
    assert e.value.code == hdg.ENONFINITE
    _, dtmin = s.dt(0.5)
    with pytest.raises(hdg.HdgError) as e:
        s.advance(10 * dtmin, hdg.STEPPER_LSERK4, 0.5, check_every=4)
    assert e.value.code == hdg.ENONFINITE
    assert s.steps_done == 4  # stopped at the first check


def test_checkpoint_resume_lserk4_is_bitwise(slab4_mesh):
    N = 3
    a = hdg.Solver(slab4_mesh, N)
    a.project_function(standing_mode_rigid)
    _, dtmin = a.dt(0.5)
    a.step(dtmin, 4)
    ck = a.checkpoint()
    a.step(dtmin, 5)
    b = hdg.Solver(slab4_mesh, N)
    b.restore(ck)
    assert b.time == 4 * dtmin
    b.step(dtmin, 5)
    sa, sb = _state(a), _state(b)
    for t in sa:
        assert np.array_equal(sa[t], sb[t]), t
    assert a.time == b.time


def test_checkpoint_resume_mrab_is_bitwise(slab4_mesh):
    N, L = 3, 3
    a = hdg.Solver(slab4_mesh, N)
    a.mrab_setup(L)
    a.project_function(standing_mode_rigid)
    a.mrab_advance(1)
    ck = a.checkpoint()
    a.mrab_advance(2)
    b = hdg.Solver(slab4_mesh, N)
    b.mrab_setup(L)
    b.restore(ck)
    b.mrab_advance(2)
    sa, sb = _state(a), _state(b)
    for t in sa:
        assert np.array_equal(sa[t], sb[t]), t
    assert a.time == b.time


def test_checkpoint_rejects_another_setup(slab4_mesh):
    a = hdg.Solver(slab4_mesh, 2)
    a.mrab_setup(3)
    a.project_function(standing_mode_rigid)
    a.mrab_advance(1)
    ck = a.checkpoint()
    b = hdg.Solver(slab4_mesh, 2)
    b.mrab_setup(2)
    with pytest.raises(hdg.HdgError) as e:
        b.restore(ck)
    assert e.value.code == hdg.EINVAL
    c = hdg.Solver(slab4_mesh, 3)
    with pytest.raises(hdg.HdgError) as e:
        c.restore(ck)
    assert e.value.code == hdg.EINVAL
    with pytest.raises(hdg.HdgError) as e:
        a.restore(ck[:100])
    assert e.value.code == hdg.EINVAL
