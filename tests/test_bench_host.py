"""Host-side checks of bench.py: the per-element algorithmic byte counts behind
the roofline figures, the source hash that keys the committed traffic
counters, and the single-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _nodes(t, N):
    if t == 0:
        return (N + 1) ** 3
    if t == 1:
        return (N + 1) * (N + 1) * (N + 2) // 2
    if t == 2:
        return (N + 1) * (N + 2) * (2 * N + 3) // 6
    return (N + 1) * (N + 2) * (N + 3) // 6


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_alg_bytes_counts_state_traces_and_records(N):
    """Each type's figure is 64 B per node (U and res read and written) plus
    32 B per trace point plus geometry, material and face records; rebuilding
    the trace-point count from the face shapes must reproduce it."""
    nq, nl = (N + 1) ** 2, (N + 1) * (N + 2) // 2
    faces = {0: (6, 0), 1: (3, 2), 2: (1, 4), 3: (0, 4)}  # (quads, triangles)
    geometry = {0: 8 * 24, 1: 6 * 24, 2: 5 * 24, 3: 4 * 24}
    for lattice in (False, True):
        for t in range(4):
            quads, tris = faces[t]
            tri_pts = nl if (lattice and t in (2, 3)) else nq
            expect = (64 * _nodes(t, N) + 32 * (quads * nq + tris * tri_pts) + geometry[t] + 8
                      + 13 * (quads + tris))
            assert bench.alg_bytes(t, N, lattice) == expect, (t, N, lattice)


def test_alg_bytes_at_the_benchmark_order():
    # the figures quoted with the roofline (N = 4, lattice traces)
    assert [bench.alg_bytes(t, 4, True) for t in range(4)] == [13078, 9017, 6433, 4316]


@pytest.mark.parametrize("N", [3, 4, 5])
def test_multirate_bytes_split_the_stage_traffic(N):
    """The multi-rate right-hand-side kernel moves U once and one history slot
    (32 B/node) and reads the neighbours' traces (16 B/point); the update
    reads U and three slots and writes U (80 B/node) and writes synchronised
    and mid-step traces (32 B/point)."""
    faces = {0: (6, 0), 1: (3, 2), 2: (1, 4), 3: (0, 4)}
    geometry = {0: 8 * 24, 1: 6 * 24, 2: 5 * 24, 3: 4 * 24}
    nq, nl = (N + 1) ** 2, (N + 1) * (N + 2) // 2
    for t in range(4):
        quads, tris = faces[t]
        pts = quads * nq + tris * (nl if t in (2, 3) else nq)
        nf = quads + tris
        assert bench.mrab_alg_bytes(0, t, N, True) == 32 * _nodes(t, N) + 16 * pts + geometry[t] + 8 + 13 * nf
        assert bench.mrab_alg_bytes(1, t, N, True) == 80 * _nodes(t, N) + 32 * pts + nf
        assert bench.mrab_alg_bytes(1, t, N, True, mid=False) == 80 * _nodes(t, N) + 16 * pts + nf
    nfn = (N + 1) * (N + 2) // 2
    assert bench.mortar_alg_bytes(N, False) == 16 * nfn * 10 + 40


def test_coarse_step_bytes_weight_levels_and_mid_step_writers():
    """Level l is active 2^(l-1) times per coarse step; only the elements that
    write mid-step traces pay their 16 B per trace point."""
    import numpy as np

    info = np.zeros((4, 3, 2), dtype=np.int64)
    info[3] = [[5, 1], [7, 0], [11, 3]]          # tets per level, writers
    act = 5 + 2 * 7 + 4 * 11
    writers = 1 + 0 + 4 * 3
    tp = 4 * 15
    assert bench.mrab_step_bytes(0, 3, 4, True, info) == act * bench.mrab_alg_bytes(0, 3, 4, True)
    assert bench.mrab_step_bytes(1, 3, 4, True, info) == act * (80 * 35 + 16 * tp + 4) + writers * 16 * tp
    assert bench.mrab_step_bytes(1, 0, 4, True, info) == 0


def test_source_hash_is_stable_and_keys_the_traffic_file():
    h = bench.csrc_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    assert h == bench.csrc_hash()
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path) as fh:
        data = json.load(fh)
    assert len(data["source_hash"]) == 16
    assert data["fetch_scale"] > 0 and data["write_scale"] > 0
    if data["source_hash"] == h:
        for name in bench.MRAB_KERNELS.values():
            assert bench.measured_traffic(name, section="bytes_per_coarse_step") > 0, name
        for name in bench.STAGE_KERNELS.values():
            assert bench.measured_traffic(name, section="bytes_per_launch") > 0, name


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
