"""Batching form (needs an MI355X): many independent problems of one order in
one mesh (their disjoint union), so every stage is one launch per element
type for all of them, replayed from a captured HIP graph.

Per-element arithmetic does not depend on an element's neighbours in
storage (the matrix-core tiles accumulate each element column separately,
split-precision scales are per column), so every problem of a batch must
reproduce its standalone run bit for bit at the same step, and a graph
replay must reproduce the eager launches bit for bit, on every replay, with
the program's own eager work and synchronisations between replays.
"""
import numpy as np
import pytest
import torch

from paper_1507_02557_amd import hdg
from paper_1507_02557_amd.inputs import batch_meshes, four_slab_mesh, gaussian_pulse, standing_mode_rigid

pytestmark = pytest.mark.gpu


def _fields(s):
    return {t: s.get_field(t).clone() for t in s.types}


def _equal(a, b):
    return all(torch.equal(a[t], b[t]) for t in a)


@pytest.mark.parametrize("refine", [1, 2])
def test_graph_replay_is_bitwise_the_eager_steps(refine):
    m = four_slab_mesh(4, seed=0, jitter=0.1, refine_last=refine)
    N = 3
    s1 = hdg.Solver(m, N)
    s2 = hdg.Solver(m, N)
    for s in (s1, s2):
        s.project_function(standing_mode_rigid)
    _, dt = s1.dt(0.5)
    for k in (4, 3, 6, 2):
        s1.step(dt, k)
        s2.step_graph(dt, k)
        torch.cuda.synchronize()
        assert _equal(_fields(s1), _fields(s2)), k
        # eager work of the program between replays
        assert abs(s1.energy() - s2.energy()) == 0.0


@pytest.mark.parametrize("prec", [hdg.PREC_FP32, hdg.PREC_FP16X2_K16])
def test_batched_problems_reproduce_their_standalone_runs(prec):
    N = 3
    parts = [four_slab_mesh(4, seed=1, jitter=0.1), four_slab_mesh(4, seed=2, jitter=0.1, refine_last=2),
             four_slab_mesh(6, seed=3, jitter=0.1), four_slab_mesh(4, seed=4, jitter=0.05)]
    union, eoff, _ = batch_meshes(parts)
    alone = [hdg.Solver(p, N, precision=prec) for p in parts]
    centres = [np.array([0.3, 0.4, 0.5]), np.array([0.6, 0.5, 0.4]), np.array([0.5, 0.5, 0.5]),
               np.array([0.4, 0.6, 0.3])]
    for s, c in zip(alone, centres):
        s.project_function(lambda x, y, z, t, c=c: gaussian_pulse(x, y, z, c))
    dt = min(s.dt(0.5)[1] for s in alone)
    sb = hdg.Solver(union, N, precision=prec)
    # the batch's state: each type's elements of part b follow those of parts < b
    for t in sb.types:
        f = torch.cat([s.get_field(t) for s in alone if t in s.types], dim=0)
        sb.set_state(t, [f[:, c] for c in range(4)])
    for s in alone:
        s.step(dt, 5)
    sb.step_graph(dt, 5)
    torch.cuda.synchronize()
    for t in sb.types:
        got = sb.get_field(t)
        o = 0
        for s in alone:
            if t not in s.types:
                continue
            ref = s.get_field(t)
            assert torch.equal(got[o:o + ref.shape[0]], ref), t
            o += ref.shape[0]
        assert o == got.shape[0]


def _close(a, b, tol=1e-6):
    for t in a:
        scale = float(a[t].abs().max())
        if float((a[t] - b[t]).abs().max()) > tol * max(scale, 1e-30):
            return False
    return True


@pytest.mark.parametrize("N", [3, 4])
def test_autotune_keeps_results(N):
    """The launch-shape autotuner picks a batch size for the hexahedron and
    wedge block kernels; single-rate and multi-rate steps after tuning agree
    with untuned ones to FP32 rounding (a batch size can change the order of
    a kernel's sums)."""
    m = four_slab_mesh(6, seed=2, jitter=0.1)
    base, tuned = hdg.Solver(m, N), hdg.Solver(m, N)
    for s in (base, tuned):
        s.project_function(standing_mode_rigid)
    choice = tuned.autotune(3)
    print("elements per block chosen", choice)
    assert choice[0] in (2, 4, 8, 16) and choice[1] in (1, 2, 4, 8)
    assert choice[2] == 0 and choice[3] == 0
    tuned.project_function(standing_mode_rigid)  # (the tuner overwrote the rhs buffer only)
    _, dt = base.dt(0.5)
    base.step(dt, 3)
    tuned.step(dt, 3)
    assert _close(_fields(base), _fields(tuned))
    for s in (base, tuned):
        s.mrab_setup(2)
        s.mrab_advance(2)
    assert _close(_fields(base), _fields(tuned))
