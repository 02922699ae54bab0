"""hdg_project_noalloc against hdg_project (needs an MI355X).

The allocation-free projection takes its work buffer from the library's fixed
device array and projects wedges and pyramids in chunks through it; it must
give exactly the state hdg_project gives (same kernels, same arithmetic per
element).  Two calls in a row on one GPU: a large mesh whose wedges and
pyramids need several chunks, then a smaller one, so the second call reuses
the array the first left behind.
"""
import numpy as np
import pytest
import torch

from paper_1507_02557_amd import hdg
from paper_1507_02557_amd.inputs import four_slab_mesh, gaussian_pulse, pulse_centre

pytestmark = pytest.mark.gpu


def _fields(x, seed):
    c = pulse_centre(seed)
    p, ux, uy, uz = gaussian_pulse(x[..., 0], x[..., 1], x[..., 2], c)
    # non-zero velocity fields so every component is exercised
    return [p, ux + torch.sin(3 * x[..., 0]), uy + x[..., 1] * x[..., 2], uz - torch.cos(2 * x[..., 2])]


def _compare(mesh, N, seed):
    s = hdg.Solver(mesh, N)
    chunks = {}
    for t in s.types:
        x = s.points(t)
        f = [v.reshape(x.shape[0], -1).contiguous() for v in _fields(x, seed)]
        s.project(t, f)
        ref = s.get_field(t).clone()
        s.set_state(t, [torch.zeros_like(ref[:, 0]) for _ in range(4)])
        s.project_noalloc(t, f)
        got = s.get_field(t)
        assert torch.equal(got, ref), (t, (got - ref).abs().max().item())
        K, Np, ns = s.info[t]
        chunks[t] = -(-K // max(1, hdg.PROJECT_SCRATCH_BYTES // (32 * ns)))
    s.close()
    return chunks


def test_project_noalloc_matches_project_twice():
    big = _compare(four_slab_mesh(32, seed=1, jitter=0.1), 5, seed=1)
    assert big[hdg.WEDGE] > 1 and big[hdg.PYR] > 1, big  # several chunks through the array
    small = _compare(four_slab_mesh(4, seed=2, jitter=0.1), 3, seed=2)
    assert small[hdg.WEDGE] == 1
