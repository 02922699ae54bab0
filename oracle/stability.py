"""Per-element trace-inequality constants and spectral bounds (oracle side,
test infrastructure: only the tests and the benchmark's CPU baseline use it).

Section 3.2 bounds the real part of the spectrum of M^{-1} A through trace
inequalities; Section 3.4 (eq. bnd_re, Table bounds) compares, on a hybrid
mesh, the spectral radius of M^{-1} A and of its symmetric part with the bound
built from trace constants computed over each mapped element K,

    C_T(N, K) = max { v^T M_s,K v / v^T M_K v },

the largest generalised eigenvalue of (M_s,K, M_K), and with the looser bound
C_T(N) C_J^K of the reference element (the local time step of eq. dtK).
Here M_K is the element's mass matrix of the method (hexahedra: GL collocation
diag(w J); tetrahedra: J Mhat; LSC wedges: I, the basis being phi / sqrt(J);
pyramids: diag(J(a_i, b_j))) and M_s,K = sum over faces of sum_q w_q J^s_q
phi_i(x_q) phi_j(x_q) with the same canonical face rules and orientation-
dependent face bases as the surface integrals (the wedge's integrand carries
1 / J at the face points; a coarse face of a 1:4 non-conforming interface is
the sum of its four sub-faces).  Parity unpinned parts: none; the pins are in
tests/test_oracle_stability_pins.py.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl

from . import refel as R


def element_masses(disc, t):
    """M_K (K_t, Np, Np) of every element of type t."""
    E = disc.refs[t]
    K = disc.els[t].size
    g = disc.geo[t]
    if t == R.HEX:
        return np.einsum("ki,ij->kij", g["mass"], np.eye(E.Np))
    if t == R.PYR:
        return np.einsum("ki,ij->kij", g["J"], np.eye(E.Np))
    if t == R.TET:
        return g["J"][:, None, None] * g["Mhat"][None, :, :]
    return np.broadcast_to(np.eye(E.Np), (K, E.Np, E.Np)).copy()


def surface_masses(disc, t):
    """M_s,K (K_t, Np, Np): sum over the element's faces of the face rule's
    sum_q w_q J^s_q phi_i(x_q) phi_j(x_q) (wedges: divided by J at x_q)."""
    E = disc.refs[t]
    K = disc.els[t].size
    Ms = np.zeros((K, E.Np, E.Np))
    for f in range(E.nfaces):
        slf = disc.slot[t][:, f]
        s = disc.wq[slf] * disc.Js[slf]
        if t == R.WEDGE:
            s = s / disc.fJ[slf]
        for idx, Phi in disc.groups[(t, f)]:
            Ms[idx] += np.einsum("qi,kq,qj->kij", Phi, s[idx], Phi)
    if t in disc.mortar:
        ms, ks, phis = disc.mortar[t]
        s = disc.wq[ms] * disc.Js[ms]
        if t == R.WEDGE:
            s = s / disc.fJ[ms]
        np.add.at(Ms, ks, np.einsum("mqi,mq,mqj->mij", phis, s, phis))
    return Ms


def trace_constants(disc):
    """C_T(N, K) per element: dict type -> (K_t,), the largest eigenvalue of
    M_s,K v = lambda M_K v (Section 3.4)."""
    out = {}
    for t in disc.types:
        M = element_masses(disc, t)
        Ms = surface_masses(disc, t)
        out[t] = np.array([sl.eigh(Ms[k], M[k], eigvals_only=True)[-1] for k in range(M.shape[0])])
    return out


def dt_elements_computed(disc, cfl: float = 0.5):
    """Local steps from the per-element constants: dtau_K = C / (C_rhokappa^K
    C_T(N, K)) (eq. dtK with the mapped element's own trace constant in place
    of C_T(N) C_J^K)."""
    ct = trace_constants(disc)
    crk = disc.c_rhokappa()
    return {t: cfl / (crk[t] * ct[t]) for t in disc.types}


def energy_weights(disc):
    """Blocks of the energy inner product for the flattened state (types in
    disc.types order, each (K_t, 4, Np) row-major): p with M_K / kappa_K,
    u with rho_K M_K.  Returns the dense matrix."""
    blocks = []
    for t in disc.types:
        M = element_masses(disc, t)
        e = disc.els[t]
        for k in range(M.shape[0]):
            blocks.append(M[k] / disc.kappa[e[k]])
            for _ in range(3):
                blocks.append(disc.rho[e[k]] * M[k])
    return sl.block_diag(*blocks)


def symmetric_part_spectrum(L, W):
    """Eigenvalues of the symmetric part of L = M^{-1} A in the energy inner
    product: (W L + L^T W) / 2 v = mu W v.  For every eigenvalue lambda of L,
    Re lambda lies in [min mu, max mu] (a Rayleigh quotient of v^* W L v)."""
    S = 0.5 * (W @ L + L.T @ W)
    return sl.eigh(S, W, eigvals_only=True)
