"""Writes the FP64 oracle results stored in this folder.

Calls only the oracle (``oracle/``) and the shared seeded input generators
(``paper_1507_02557_amd.inputs``); nothing here touches the HIP library.
Run from the repository root:

    python tests/golden/make_golden.py [small|patches|all]

small
    ``refined_n4_standing_N{3,4,5}.npz``: the four-slab mesh on 4^3 cubes
    (seed 0, jitter 0.1 h) with its last (tetrahedral) slab refined 2x (1:4
    non-conforming face), rigid walls, the rigid-wall standing mode, advanced
    by the multi-rate AB3 scheme on three levels (start-up of two coarse steps
    of LSERK4 at dtau_min, then ``COARSE`` coarse steps).  Per element type the
    FP64 state (K, 4, Np), plus N, the levels, dtau_min and the final time.

patches
    ``patches_{mesh}_N{N}.npz``: sampled elements of the full-size meshes
    (four-slab n = 48, and the same with the refined last slab) after one
    LSERK4 step of size DT (below dtau_min of both meshes at N <= 5) from the
    standing mode.  One step has five right-hand-side
    evaluations, so information moves at most five face layers: the oracle
    runs on the sub-mesh of all elements within six face layers of the
    sampled ones (closed under the four fine elements of a non-conforming
    coarse face), where the sampled elements' results are exact.  Stored:
    element ids (mesh order), their type, the state (n, 4, Np), dt.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import mesh as OM  # noqa: E402
from oracle import refel as R  # noqa: E402
from oracle.mrab import MRAB3  # noqa: E402
from oracle.solver import Disc, lserk4_step  # noqa: E402
from paper_1507_02557_amd.inputs import Mesh, four_slab_mesh, standing_mode_rigid  # noqa: E402

COARSE = 6          # coarse multi-rate steps after the start-up (small mesh)
LEVELS = 3
PATCH_LAYERS = 6    # face layers around a sampled element (one LSERK4 step: 5 stages)
DT = 1.0e-5         # step of the patch runs (dtau_min of the n = 48 meshes is 1.5e-5 or more)


def small(orders=(3, 4, 5)):
    mesh = four_slab_mesh(4, seed=0, jitter=0.1, refine_last=2)
    for N in orders:
        d = Disc(mesh, N)
        mr = MRAB3(d, LEVELS)
        U = mr.startup(d.project(standing_mode_rigid))
        for _ in range(COARSE):
            U = mr.coarse_step(U)
        lev = np.zeros(mesh.n_elem, dtype=np.int8)
        for t in d.types:
            lev[d.els[t]] = mr.level[t]
        out = {f"U{t}": U[t] for t in d.types}
        np.savez_compressed(os.path.join(HERE, f"refined_n4_standing_N{N}.npz"), N=N, levels=LEVELS,
                            coarse_steps=COARSE, t=mr.t, dtmin=mr.dtmin, level=lev, **out)
        print(f"small N={N}: t={mr.t:.6e}, dtmin={mr.dtmin:.6e}")


def _adjacency(mesh: Mesh):
    types = mesh.etype.astype(np.int64)
    refs = {t: R.make(t, 1) for t in np.unique(types)}
    slot_elem, slot_face, nbr = OM.match_faces(types, mesh.everts, refs)
    pairs = [(int(slot_elem[s]), int(slot_elem[nbr[s]])) for s in np.nonzero(nbr >= 0)[0]]
    groups = []
    if mesh.hanging.shape[0]:
        nc = OM.nonconforming_faces(types, mesh.everts, refs, slot_elem, slot_face, nbr, mesh.hanging)
        for s, subs in nc:
            g = [int(slot_elem[s])] + [int(slot_elem[fs]) for fs, _ in subs]
            groups.append(g)
            pairs += [(g[0], e) for e in g[1:]] + [(e, g[0]) for e in g[1:]]
    nb = [[] for _ in range(mesh.n_elem)]
    for a, b in pairs:
        nb[a].append(b)
    member = {}
    for i, g in enumerate(groups):
        for e in g:
            member.setdefault(e, []).append(i)
    return nb, groups, member


def _patch(mesh: Mesh, centre, nb, groups, member, layers):
    seen = {int(centre)}
    front = [int(centre)]
    for _ in range(layers):
        nxt = []
        for e in front:
            for f in nb[e]:
                if f not in seen:
                    seen.add(f)
                    nxt.append(f)
        front = nxt
    # every non-conforming face touched keeps all five of its elements
    for e in list(seen):
        for gi in member.get(e, []):
            seen.update(groups[gi])
    ids = np.array(sorted(seen), dtype=np.int64)
    ev = mesh.everts[ids]
    used = np.unique(ev[ev >= 0])
    # hanging vertices whose edge lies in the patch stay hanging
    hang = mesh.hanging
    if hang.shape[0]:
        keep = np.isin(hang[:, 0], used) & np.isin(hang[:, 1], used) & np.isin(hang[:, 2], used)
        hang = hang[keep]
    remap = -np.ones(mesh.xyz.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)   # increasing: canonical face frames are unchanged
    ev2 = np.where(ev >= 0, remap[np.maximum(ev, 0)], -1)
    sub = Mesh(xyz=mesh.xyz[used], etype=mesh.etype[ids], everts=ev2, kappa=mesh.kappa[ids], rho=mesh.rho[ids],
               hanging=remap[hang] if hang.shape[0] else np.zeros((0, 3), dtype=np.int64))
    return sub, ids


def sample_elements(mesh: Mesh, seed: int, per_type: int = 2):
    """Seeded sample: per type present, ``per_type`` random elements, plus (on a
    refined mesh) one coarse and one fine element of the non-conforming face."""
    rng = np.random.default_rng(seed)
    out = []
    for t in (R.HEX, R.WEDGE, R.PYR, R.TET):
        idx = np.nonzero(mesh.etype == t)[0]
        if idx.size:
            out += [int(i) for i in rng.choice(idx, size=min(per_type, idx.size), replace=False)]
    return out


def patches(meshes=("slab48", "refined48"), orders=(3, 4)):
    for name in meshes:
        mesh = four_slab_mesh(48, seed=0, jitter=0.1, refine_last=2 if name == "refined48" else 1)
        nb, groups, member = _adjacency(mesh)
        centres = sample_elements(mesh, seed=11)
        if groups:
            g = groups[len(groups) // 3]
            centres += [g[0], g[2]]
        for N in orders:
            dt = DT
            types, states = [], []
            for e in centres:
                sub, ids = _patch(mesh, e, nb, groups, member, PATCH_LAYERS)
                d = Disc(sub, N)
                U = d.project(standing_mode_rigid)
                U = lserk4_step(d, U, dt)
                pos = int(np.searchsorted(ids, e))
                t = int(sub.etype[pos])
                k = int(np.nonzero(d.els[t] == pos)[0][0])
                types.append(t)
                states.append(U[t][k])
                print(f"{name} N={N} element {e} (type {t}): patch of {sub.n_elem} elements")
            width = max(s.shape[1] for s in states)
            S = np.zeros((len(states), 4, width))
            for i, s in enumerate(states):
                S[i, :, : s.shape[1]] = s
            np.savez_compressed(os.path.join(HERE, f"patches_{name}_N{N}.npz"), N=N, dt=dt,
                                elems=np.array(centres), types=np.array(types), state=S)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("small", "all"):
        small()
    if what in ("patches", "all"):
        patches()
