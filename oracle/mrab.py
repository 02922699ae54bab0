"""Multi-rate Adams-Bashforth (MRAB3) stepping (oracle side, Section 2.4).

Levels: dtau_l = 2^(L-l) dtau_min, l = 1 (coarsest) .. L (finest).
Binning: element K takes the coarsest level whose step does not exceed its
stable step dtau_K (the printed inequality reads the other way round; this
is the reading that keeps every element stable).  A sweep then moves
elements to finer levels until face neighbours differ by at most one level,
repeated to a fixed point.  On a 1:4 non-conforming face the four fine
elements are moved to the finest level among them.

A coarse step (dtau_1) has 2^(L-1) substeps of dtau_min at t_k = t_0 + k dtau_min;
level l is active at substep k when k is a multiple of 2^(L-l).  At a substep:

1. every element provides its trace at t_k: its own state if active, else the
   AB3 dense output of its current step,
     u(t_s + theta dtau_l) = u_s + dtau_l sum_j beta_j(theta) r_{s-j},
   beta_0 = theta + 3 theta^2/4 + theta^3/6, beta_1 = -(theta^2 + theta^3/3),
   beta_2 = theta^2/4 + theta^3/6 (the integral of the quadratic through the
   last three right-hand sides);
2. active elements evaluate their right-hand side and push it on their level's
   history;
3. active elements take an AB3 step with their own dtau_l.

Start-up (the paper defers it to its references): single-rate LSERK4 at
dtau_min for two coarse steps, recording every level's right-hand side at the
step boundaries that are multiples of its dtau_l; the multi-rate stepping then
starts with a full history.
"""
from __future__ import annotations

import numpy as np

from .solver import LSERK_A, LSERK_B, Disc


def ab3_beta(theta: float) -> np.ndarray:
    """Dense-output AB3 weights beta_j(theta) for r_s, r_{s-1}, r_{s-2}."""
    t = float(theta)
    return np.array([t + 0.75 * t * t + t ** 3 / 6.0, -(t * t + t ** 3 / 3.0), 0.25 * t * t + t ** 3 / 6.0])


def bin_levels(disc: Disc, L: int, cfl: float = 0.5, dte=None):
    """Level per element (dict type -> int array) and dtau_min, from the local
    steps dte (dict type -> array; default: Disc.dt_elements)."""
    if dte is None:
        dte = disc.dt_elements(cfl)
    dtmin = min(float(np.min(v)) for v in dte.values())
    ne = sum(disc.els[t].size for t in disc.types)
    lev = np.zeros(ne, dtype=np.int64)
    for t in disc.types:
        ratio = dte[t] / dtmin
        j = np.floor(np.log2(ratio * (1.0 + 1e-12))).astype(np.int64)
        j = np.clip(j, 0, L - 1)
        lev[disc.els[t]] = L - j
    # neighbours differ by at most one level: move coarser elements finer;
    # the four elements on the sub-faces of one non-conforming coarse face
    # share a level (the finest among them), so the coarse element's view of
    # its face is of one level
    inner = disc.nbr >= 0
    a = disc.slot_elem[inner]
    b = disc.slot_elem[disc.nbr[inner]]
    groups = getattr(disc, "nc_groups", [])
    while True:
        need = np.maximum(lev[a], lev[b] - 1)
        new = lev.copy()
        np.maximum.at(new, a, need)
        for g in groups:
            new[g] = np.max(new[g])
        if np.array_equal(new, lev):
            break
        lev = new
    return {t: lev[disc.els[t]] for t in disc.types}, dtmin


class MRAB3:
    """Multi-rate AB3 integrator over a Disc."""

    def __init__(self, disc: Disc, L: int, cfl: float = 0.5, dte=None):
        self.d = disc
        self.L = L
        self.level, self.dtmin = bin_levels(disc, L, cfl, dte)
        self.dtl = {l: (2 ** (L - l)) * self.dtmin for l in range(1, L + 1)}
        self.hist = {t: np.zeros((3,) + disc.zeros()[t].shape) for t in disc.types}
        self.count = {l: 0 for l in range(1, L + 1)}  # right-hand sides pushed per level
        self.t = 0.0

    def _push(self, t, mask, R):
        """Push R (masked elements) on the history of their levels."""
        for l in range(1, self.L + 1):
            m = mask & (self.level[t] == l)
            if np.any(m):
                self.hist[t][self.count[l] % 3][m] = R[t][m]

    def _hist(self, t, l, j):
        return self.hist[t][(self.count[l] - 1 - j) % 3]

    def startup(self, U):
        """LSERK4 at dtau_min for two coarse steps, recording right-hand sides."""
        d = self.d
        nfine = 2 ** self.L
        res = {t: np.zeros_like(U[t]) for t in d.types}
        for j in range(nfine):
            R = d.rhs(U)
            for l in range(1, self.L + 1):
                if j % (2 ** (self.L - l)) == 0:
                    for t in d.types:
                        m = self.level[t] == l
                        if np.any(m):
                            self.hist[t][self.count[l] % 3][m] = R[t][m]
                    self.count[l] += 1
            for s in range(5):
                Rs = R if s == 0 else d.rhs(U)
                for t in d.types:
                    res[t] = LSERK_A[s] * res[t] + self.dtmin * Rs[t]
                    U[t] = U[t] + LSERK_B[s] * res[t]
        self.t += nfine * self.dtmin
        return U

    def coarse_step(self, U):
        """One coarse step.  U holds each element's state at the start of its
        current step (all elements are synchronised at coarse-step boundaries)."""
        d, L = self.d, self.L
        start = {t: U[t].copy() for t in d.types}
        for k in range(2 ** (L - 1)):
            active = {t: (k % (2 ** (L - self.level[t]))) == 0 for t in d.types}
            V = {}
            for t in d.types:
                start[t][active[t]] = U[t][active[t]]
                V[t] = U[t].copy()
                for l in range(1, L + 1):
                    m = (~active[t]) & (self.level[t] == l)
                    if not np.any(m):
                        continue
                    theta = (k % (2 ** (L - l))) / float(2 ** (L - l))
                    beta = ab3_beta(theta)
                    V[t][m] = start[t][m] + self.dtl[l] * sum(beta[j] * self._hist(t, l, j)[m] for j in range(3))
            R = d.rhs(V)
            act_levels = [l for l in range(1, L + 1) if k % (2 ** (L - l)) == 0]
            for t in d.types:
                self._push(t, active[t], R)
            for l in act_levels:
                self.count[l] += 1
            b1 = ab3_beta(1.0)
            for t in d.types:
                for l in act_levels:
                    m = self.level[t] == l
                    if np.any(m):
                        U[t][m] = start[t][m] + self.dtl[l] * sum(b1[j] * self._hist(t, l, j)[m] for j in range(3))
        self.t += (2 ** (L - 1)) * self.dtmin
        return U
