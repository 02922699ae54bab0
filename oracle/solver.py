"""Semi-discrete DG operator, energy, stable time step and steppers (oracle side).

The discretisation is that of Section 2 of the paper:

* hexahedra: GL nodal basis, strong form, collocated mass diag(w J)
  (Section 2.1.1, Algorithms 1-3);
* tetrahedra: nodal basis, strong form, mass J * Mhat (Section 2.1.2,
  Algorithm 4);
* wedges: modal LSC-DG basis phi/sqrt(J), skew-symmetric form, mass = I
  (Sections 2.1.3, 2.3.3, Algorithms 5-6);
* pyramids: semi-nodal basis, diagonal mass J(a_i, b_j); skew-symmetric form
  with the quadrature-free operators of Section 2.3.4 (Algorithm 7), the
  strong form as an option.

Flux (Section 2.2, eq. skewform and the strong form below it), with
[q] = q+ - q-, {u} = (u+ + u-)/2, tau_p = 1/{rho c}, tau_u = {rho c}:
  p:  strong  (tau_p [p] - n.[u]) / 2      skew  tau_p [p] / 2 - n.{u}
  u:  (tau_u n.[u] - [p]) n / 2
Boundary faces use a mirror state: rigid wall p+ = p-, u+ = u- - 2 (n.u-) n;
free surface p+ = -p-, u+ = u-; the boundary penalty uses the element's own
rho c.

All surface integrals use face cubature points placed in the canonical face
frame (``oracle.mesh``): (N+1)^2 Gauss-Legendre points on quadrilaterals and
the (N+1)^2 collapsed Gauss-Jacobi rule on triangles.

1:4 non-conforming triangular faces (a coarse face split into the four
triangles of its midpoint subdivision, each the face of a finer element; the
paper's meshes are conforming, so this follows the same flux pointwise): on
every sub-face the coarse element evaluates its trace at the fine face's
canonical points, the flux is formed there exactly as on a conforming face,
and the coarse element's integral over its face is the sum of the four
sub-face integrals.  The coarse element's side of each sub-face is held as
an extra ("mortar") slot paired with the fine element's slot; the coarse
face's own slot keeps its geometry (it enters the time step) but carries no
weight.

State layout: dict type -> array (K_t, 4, Np) with fields (p, ux, uy, uz).
"""
from __future__ import annotations

import numpy as np

from . import mesh as OM
from . import refel as R
from .tables import trace_constant

BC_FREE_SURFACE = 0
BC_RIGID_WALL = 1

# Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage Runge-Kutta
LSERK_A = np.array([0.0,
                    -567301805773.0 / 1357537059087.0,
                    -2404267990393.0 / 2016746695238.0,
                    -3550918686646.0 / 2091501179385.0,
                    -1275806237668.0 / 842570457699.0])
LSERK_B = np.array([1432997174477.0 / 9575080441755.0,
                    5161836677717.0 / 13612068292357.0,
                    1720146321549.0 / 2090206949498.0,
                    3134564353537.0 / 4481467310338.0,
                    2277821191437.0 / 14882151754819.0])


class Disc:
    """The DG discretisation of one mesh at order N."""

    def __init__(self, mesh, N: int, bc: int = BC_RIGID_WALL, pyr_form: str = "skew"):
        self.N = N
        self.bc = bc
        self.pyr_form = pyr_form
        types = mesh.etype.astype(np.int64)
        self.types = [t for t in (R.HEX, R.WEDGE, R.PYR, R.TET) if np.any(types == t)]
        self.refs = {t: R.make(t, N) for t in self.types}
        self.els = {t: np.nonzero(types == t)[0] for t in self.types}
        self.V = {}
        for t in self.types:
            nv = self.refs[t].nv
            self.V[t] = mesh.xyz[mesh.everts[self.els[t], :nv]]
        self.kappa = mesh.kappa
        self.rho = mesh.rho
        self.rhoc = np.sqrt(mesh.kappa * mesh.rho)

        slot_elem, slot_face, nbr = OM.match_faces(types, mesh.everts, self.refs)
        self.nslot = slot_elem.shape[0]
        self.slot_elem, self.slot_face, self.nbr = slot_elem, slot_face, nbr
        # boundary condition per face slot: the mesh's per-face choice where it
        # makes one (bc_face[element, local face] >= 0), else bc
        self.slot_bc = np.full(self.nslot, bc, dtype=np.int64)
        bcf = getattr(mesh, "bc_face", None)
        if bcf is not None:
            v = np.asarray(bcf, dtype=np.int64)[slot_elem, slot_face]
            self.slot_bc = np.where(v >= 0, v, bc)
        first = np.zeros(types.shape[0] + 1, dtype=np.int64)
        nfaces = np.array([self.refs[t].nfaces if t in self.refs else 0 for t in range(4)])
        first[1:] = np.cumsum(nfaces[types])
        self.slot = {t: first[self.els[t]][:, None] + np.arange(self.refs[t].nfaces)[None, :]
                     for t in self.types}

        n1 = N + 1
        self.Nfq = n1 * n1
        self.face_rule = {3: R.tri_rule(n1), 4: R.quad_rule(n1)}

        # ---- face geometry, trace matrices ------------------------------
        self.fx = np.zeros((self.nslot, self.Nfq, 3))
        self.Js = np.zeros((self.nslot, self.Nfq))
        self.Js_ref = np.zeros((self.nslot, self.Nfq))
        self.nrm = np.zeros((self.nslot, self.Nfq, 3))
        self.wq = np.zeros((self.nslot, self.Nfq))
        self.fJ = np.ones((self.nslot, self.Nfq))      # volume J at face points
        self.groups = {}  # (t, f) -> list of (element index array, trace matrix)
        for t in self.types:
            E = self.refs[t]
            V = self.V[t]
            gid = mesh.everts[self.els[t]]
            for f, fv in enumerate(E.faces):
                nfv = len(fv)
                eta, w = self.face_rule[nfv]
                S, dS = R.face_shape(nfv, eta)
                perms = np.array([OM.canonical_perm(gid[k, list(fv)]) for k in range(V.shape[0])])
                fvarr = np.array(fv)
                cv = fvarr[perms]                        # (K, nfv) canonical local vertex ids
                xc = np.take_along_axis(V, cv[:, :, None], axis=1)  # (K, nfv, 3)
                xq = np.einsum("qv,kvd->kqd", S, xc)
                t1 = np.einsum("qv,kvd->kqd", dS[0], xc)
                t2 = np.einsum("qv,kvd->kqd", dS[1], xc)
                cr = np.cross(t1, t2)
                js = np.linalg.norm(cr, axis=2)
                Xq = np.einsum("qv,kvd->kqd", S, E.vref[cv])   # reference coords per element
                xm, F, J, G = OM.vertex_map(E, Xq, V)
                if np.max(np.abs(xm - xq)) > 1e-11:
                    raise ValueError("face points of the vertex map and canonical frame differ")
                if np.any(J <= 0):
                    raise ValueError("non-positive Jacobian at a face point")
                outward = np.einsum("kqrd,r->kqd", G, E.face_nref[f])
                sgn = np.sign(np.einsum("kqd,kqd->kq", cr, outward))
                sl = self.slot[t][:, f]
                self.fx[sl] = xq
                self.Js[sl] = js
                self.Js_ref[sl] = js * ((2.0 if nfv == 3 else 4.0) / E.face_area[f])
                self.nrm[sl] = cr / js[:, :, None] * sgn[:, :, None]
                self.wq[sl] = w[None, :]
                self.fJ[sl] = J
                glist = []
                keys = {}
                for k in range(perms.shape[0]):
                    keys.setdefault(tuple(perms[k]), []).append(k)
                for key, idx in keys.items():
                    Xr = S @ E.vref[fvarr[list(key)]]
                    Phi, _ = E.basis(Xr)
                    glist.append((np.array(idx), Phi))
                self.groups[(t, f)] = glist

        # ---- 1:4 non-conforming faces: mortar slots ----------------------
        self._build_mortars(mesh, types, slot_face)

        # ---- volume geometry and operators -----------------------------
        self.geo = {}
        for t in self.types:
            E = self.refs[t]
            V = self.V[t]
            g = {}
            if t == R.HEX:
                _, _, J, G = OM.vertex_map(E, E.nodes, V)
                _, dPhi = E.basis(E.nodes)
                g.update(J=J, G=G, D=dPhi, mass=E.wnodes[None, :] * J)
            elif t == R.TET:
                _, _, J, G = OM.vertex_map(E, E.nodes, V)
                _, dPhi = E.basis(E.nodes)
                Xe, we = R.collapsed_volume_rule(R.TET, N + 2)
                Pe, _ = E.basis(Xe)
                Mhat = (Pe * we[:, None]).T @ Pe
                g.update(J=J[:, 0], G=G[:, 0], D=dPhi, Mhat=Mhat, Minv=np.linalg.inv(Mhat))
            elif t == R.WEDGE:
                Xc, wc = E.cubature()
                Phi, dPhi = E.basis(Xc)
                _, F, J, G = OM.vertex_map(E, Xc, V)
                # grad_rst J = J tr(G dF/dxi_m), dF from second derivatives of the shape functions
                d2 = E.shape2(Xc)
                dF = np.einsum("rmqv,kvd->kqdrm", d2, V)
                dJ = J[:, :, None] * np.einsum("kqrd,kqdrm->kqm", G, dF)
                gJ = np.einsum("kqmd,kqm->kqd", G, dJ)   # physical gradient of J
                g.update(J=J, G=G, gJ=gJ, Phi=Phi, dPhi=dPhi, w=wc)
            elif t == R.PYR:
                _, _, J, G = OM.vertex_map(E, E.geo_points, V)
                Xe, we = R.collapsed_volume_rule(R.PYR, N + 3)
                Pe, dPe = E.basis(Xe)
                Dw = np.stack([(Pe * we[:, None]).T @ dPe[r] for r in range(3)], 0)  # D^r_ij = int phi_i d_r phi_j
                g.update(J=J, G=G, Dw=Dw, mass=J)
            if np.any(g["J"] <= 0):
                raise ValueError("non-positive Jacobian")
            self.geo[t] = g

    def _build_mortars(self, mesh, types, slot_face):
        hang = getattr(mesh, "hanging", None)
        hang = np.zeros((0, 3), dtype=np.int64) if hang is None else hang
        nc = OM.nonconforming_faces(types, mesh.everts, self.refs, self.slot_elem, slot_face, self.nbr, hang)
        ns0 = self.nslot
        self.is_parent = np.zeros(ns0, dtype=bool)
        self.nc_groups = []          # elements on the four sub-faces of each coarse face
        self.mortar = {}             # type -> (mortar slots, element index within type, trace matrices)
        pairs = [(s, fs, bary) for s, subs in nc for fs, bary in subs]
        nm = len(pairs)
        if nm == 0:
            return
        ext = lambda a, fill=0.0: np.concatenate([a, np.full((nm,) + a.shape[1:], fill, dtype=a.dtype)])
        self.slot_elem = ext(self.slot_elem, 0)
        self.nbr = ext(self.nbr, -1)
        self.fx, self.Js, self.Js_ref = ext(self.fx), ext(self.Js), ext(self.Js_ref)
        self.nrm, self.wq, self.fJ = ext(self.nrm), ext(self.wq), ext(self.fJ, 1.0)
        self.is_parent = ext(self.is_parent, False)
        self.slot_bc = ext(self.slot_bc, self.bc)
        eta, _ = self.face_rule[3]
        S, _ = R.face_shape(3, eta)
        local = {}
        for t in self.types:
            for k, e in enumerate(self.els[t]):
                local[int(e)] = (t, k)
        per_type = {}
        for s, subs in nc:
            self.is_parent[s] = True
            self.wq[s] = 0.0
            self.nc_groups.append(np.array([self.slot_elem[fs] for fs, _ in subs]))
        for i, (s, fs, bary) in enumerate(pairs):
            m = ns0 + i
            e = int(self.slot_elem[s])
            t, k = local[e]
            E = self.refs[t]
            fv = list(E.faces[int(slot_face[s])])
            fe = int(self.slot_elem[fs])
            fE = self.refs[int(types[fe])]
            fg = mesh.everts[fe, list(fE.faces[int(slot_face[fs])])]
            cv = sorted(int(v) for v in fg)                 # the fine face's canonical vertex order
            B = np.array([bary[v] for v in cv])            # canonical sub-face vertices in coarse barycentrics
            Xq = S @ B @ E.vref[fv]                         # coarse reference coordinates of the fine points
            xm, _, J, _ = OM.vertex_map(E, Xq, self.V[t][k:k + 1])
            if np.max(np.abs(xm[0] - self.fx[fs])) > 1e-11:
                raise ValueError("sub-face points of the coarse element and the fine face differ")
            nrm = self.nrm[s][0]
            if np.max(np.abs(nrm[None, :] + self.nrm[fs])) > 1e-9:
                raise ValueError("coarse and fine normals of a sub-face are not opposite")
            Phi, _ = E.basis(Xq)
            self.slot_elem[m] = e
            self.nbr[m], self.nbr[fs] = fs, m
            self.fx[m] = self.fx[fs]
            self.Js[m] = self.Js[fs]
            self.wq[m] = self.wq[fs]
            self.nrm[m] = nrm[None, :]
            self.fJ[m] = J[0]
            per_type.setdefault(t, ([], [], []))
            per_type[t][0].append(m)
            per_type[t][1].append(k)
            per_type[t][2].append(Phi)
        self.nslot = ns0 + nm
        for t, (ms, ks, phis) in per_type.items():
            self.mortar[t] = (np.array(ms), np.array(ks), np.stack(phis))

    # ------------------------------------------------------------------
    def zeros(self):
        return {t: np.zeros((self.els[t].size, 4, self.refs[t].Np)) for t in self.types}

    def traces(self, U):
        """Traces (nslot, Nfq, 4) at the canonical face points."""
        TR = np.zeros((self.nslot, self.Nfq, 4))
        for t in self.types:
            for f in range(self.refs[t].nfaces):
                for idx, Phi in self.groups[(t, f)]:
                    TR[self.slot[t][idx, f]] = np.einsum("qj,kcj->kqc", Phi, U[t][idx])
            if t in self.mortar:
                ms, ks, phis = self.mortar[t]
                TR[ms] = np.einsum("mqj,mcj->mqc", phis, U[t][ks])
            if t == R.WEDGE:
                sl = self.slot[t].ravel()
                if t in self.mortar:
                    sl = np.concatenate([sl, self.mortar[t][0]])
                TR[sl] /= np.sqrt(self.fJ[sl])[:, :, None]
        return TR

    def fluxes(self, TR):
        """Per-slot flux (nslot, Nfq, 4): strong p-flux, skew p-flux in slot 4 of an extra array."""
        own = TR
        nb = np.empty_like(TR)
        inner = self.nbr >= 0
        nb[inner] = TR[self.nbr[inner]]
        n = self.nrm
        # boundary mirror states: rigid wall p+ = p-, u+ = u- - 2 (n.u-) n;
        # free surface p+ = -p-, u+ = u-
        rig = ~inner & (self.slot_bc == BC_RIGID_WALL)
        fre = ~inner & (self.slot_bc != BC_RIGID_WALL)
        pm, um = own[rig, :, 0], own[rig, :, 1:]
        un = np.einsum("kqd,kqd->kq", um, n[rig])
        nb[rig, :, 0] = pm
        nb[rig, :, 1:] = um - 2.0 * un[:, :, None] * n[rig]
        nb[fre, :, 0] = -own[fre, :, 0]
        nb[fre, :, 1:] = own[fre, :, 1:]
        rc_own = self.rhoc[self.slot_elem]
        rc_nb = rc_own.copy()
        rc_nb[inner] = self.rhoc[self.slot_elem[self.nbr[inner]]]
        avg = 0.5 * (rc_own + rc_nb)
        tau_p = (1.0 / avg)[:, None]
        tau_u = avg[:, None]
        jp = nb[:, :, 0] - own[:, :, 0]
        ju = nb[:, :, 1:] - own[:, :, 1:]
        au = 0.5 * (nb[:, :, 1:] + own[:, :, 1:])
        nju = np.einsum("kqd,kqd->kq", n, ju)
        nau = np.einsum("kqd,kqd->kq", n, au)
        fp_strong = 0.5 * (tau_p * jp - nju)
        fp_skew = 0.5 * tau_p * jp - nau
        fu = (0.5 * (tau_u * nju - jp))[:, :, None] * n
        return fp_strong, fp_skew, fu

    def surface(self, t, fp, fu):
        """Surface integrals S (K_t, 4, Np) = sum_faces sum_q w_q Js_q flux_q phi_i(x_q)."""
        E = self.refs[t]
        S = np.zeros((self.els[t].size, 4, E.Np))
        for f in range(E.nfaces):
            sl = self.slot[t][:, f]
            scale = self.wq[sl] * self.Js[sl]
            if t == R.WEDGE:
                scale = scale / np.sqrt(self.fJ[sl])
            flux = np.concatenate([fp[sl][:, :, None], fu[sl]], axis=2) * scale[:, :, None]
            for idx, Phi in self.groups[(t, f)]:
                S[idx] += np.einsum("qi,kqc->kci", Phi, flux[idx])
        if t in self.mortar:
            ms, ks, phis = self.mortar[t]
            scale = self.wq[ms] * self.Js[ms]
            if t == R.WEDGE:
                scale = scale / np.sqrt(self.fJ[ms])
            flux = np.concatenate([fp[ms][:, :, None], fu[ms]], axis=2) * scale[:, :, None]
            np.add.at(S, ks, np.einsum("mqi,mqc->mci", phis, flux))
        return S

    def rhs(self, U):
        """dU/dt = M^{-1} A U for every element type."""
        TR = self.traces(U)
        fp_strong, fp_skew, fu = self.fluxes(TR)
        out = {}
        for t in self.types:
            g = self.geo[t]
            kap = self.kappa[self.els[t]][:, None]
            irho = (1.0 / self.rho[self.els[t]])[:, None]
            u = U[t]
            p, ud = u[:, 0], u[:, 1:]
            skew = (t == R.WEDGE) or (t == R.PYR and self.pyr_form == "skew")
            S = self.surface(t, fp_skew if skew else fp_strong, fu)
            r = np.zeros_like(u)
            if t == R.HEX:
                D, G, mass = g["D"], g["G"], g["mass"]
                dp = np.einsum("rij,kj->kir", D, p)               # (K, Np, 3) reference derivatives
                du = np.einsum("rij,kdj->kidr", D, ud)            # (K, Np, 3d, 3r)
                div = np.einsum("kird,kidr->ki", G, du)
                grad = np.einsum("kird,kir->kid", G, dp)
                r[:, 0] = kap * (-div + S[:, 0] / mass)
                r[:, 1:] = irho[:, :, None] * (-np.transpose(grad, (0, 2, 1)) + S[:, 1:] / mass[:, None, :])
            elif t == R.TET:
                D, G, J, Minv = g["D"], g["G"], g["J"], g["Minv"]
                dp = np.einsum("rij,kj->kir", D, p)
                du = np.einsum("rij,kdj->kidr", D, ud)
                div = np.einsum("krd,kidr->ki", G, du)
                grad = np.einsum("krd,kir->kid", G, dp)
                lift = np.einsum("ij,kcj->kci", Minv, S) / J[:, None, None]
                r[:, 0] = kap * (-div + lift[:, 0])
                r[:, 1:] = irho[:, :, None] * (-np.transpose(grad, (0, 2, 1)) + lift[:, 1:])
            elif t == R.WEDGE:
                Phi, dPhi, w, G, J, gJ = g["Phi"], g["dPhi"], g["w"], g["G"], g["J"], g["gJ"]
                P = np.einsum("qj,kj->kq", Phi, p)
                dP = np.einsum("rqj,kj->kqr", dPhi, p)
                Uq = np.einsum("qj,kdj->kqd", Phi, ud)
                GU = np.einsum("kqrd,kqd->kqr", G, Uq)
                hJ = gJ / (2.0 * J[:, :, None])
                vol_p = (np.einsum("q,rqi,kqr->ki", w, dPhi, GU)
                         - np.einsum("q,qi,kqd,kqd->ki", w, Phi, hJ, Uq))
                gP = np.einsum("kqrd,kqr->kqd", G, dP) - P[:, :, None] * hJ
                vol_u = -np.einsum("q,qi,kqd->kdi", w, Phi, gP)
                r[:, 0] = kap * (vol_p + S[:, 0])
                r[:, 1:] = irho[:, :, None] * (vol_u + S[:, 1:])
            elif t == R.PYR:
                Dw, G, J = g["Dw"], g["G"], g["J"]
                Dp = np.einsum("rij,kj->kir", Dw, p)
                grad = np.einsum("kird,kir->kid", G, Dp)
                r[:, 1:] = irho[:, :, None] * (-np.transpose(grad, (0, 2, 1)) + S[:, 1:] / J[:, None, :])
                if self.pyr_form == "skew":
                    Ur = J[:, :, None] * np.einsum("kjrd,kdj->kjr", G, ud)
                    vol = np.einsum("rji,kjr->ki", Dw, Ur)
                    r[:, 0] = kap * (vol + S[:, 0]) / J
                else:
                    Du = np.einsum("rij,kdj->kidr", Dw, ud)
                    div = np.einsum("kird,kidr->ki", G, Du)
                    r[:, 0] = kap * (-div + S[:, 0] / J)
            out[t] = r
        return out

    # ------------------------------------------------------------------
    def mass_apply(self, t, v):
        """M v for one field array v (K_t, ..., Np) with the element mass matrices."""
        g = self.geo[t]
        if t == R.HEX:
            return v * g["mass"].reshape(g["mass"].shape[0], *([1] * (v.ndim - 2)), -1)
        if t == R.PYR:
            return v * g["J"].reshape(g["J"].shape[0], *([1] * (v.ndim - 2)), -1)
        if t == R.TET:
            return np.einsum("ij,k...j->k...i", g["Mhat"], v) * g["J"].reshape(-1, *([1] * (v.ndim - 1)))
        return v.copy()

    def inner(self, A, B):
        """sum_K sum_fields A^T M B (no material weights)."""
        return sum(float(np.sum(A[t] * self.mass_apply(t, B[t]))) for t in self.types)

    def energy(self, U):
        """E = 1/2 sum_K ( p^T M p / kappa + rho u^T M u )."""
        E = 0.0
        for t in self.types:
            Mu = self.mass_apply(t, U[t])
            k = self.kappa[self.els[t]]
            rh = self.rho[self.els[t]]
            E += 0.5 * float(np.sum(U[t][:, 0] * Mu[:, 0] / k[:, None]))
            E += 0.5 * float(np.sum(rh[:, None, None] * U[t][:, 1:] * Mu[:, 1:]))
        return E

    def rel_l2(self, A, B):
        """sqrt(sum (A-B)^T M (A-B)) / sqrt(sum B^T M B), all four fields."""
        D = {t: A[t] - B[t] for t in self.types}
        return np.sqrt(self.inner(D, D) / self.inner(B, B))

    # ------------------------------------------------------------------
    def sample_points(self, t):
        """Physical points where initial data is sampled: nodes (hex, tet),
        the wedge cubature, the pyramid projection rule."""
        E = self.refs[t]
        if t in (R.HEX, R.TET):
            X = E.nodes
        elif t == R.WEDGE:
            X, _ = E.cubature()
        else:
            X, _ = E.projection_rule()
        x, _, _, _ = OM.vertex_map(E, X, self.V[t])
        return x

    def project(self, func, time: float = 0.0):
        """Initial data: interpolation at nodes (hex, tet); L2 projection (wedge, pyramid)."""
        U = {}
        for t in self.types:
            E = self.refs[t]
            x = self.sample_points(t)
            vals = np.stack(func(x[..., 0], x[..., 1], x[..., 2], time), 1)  # (K, 4, npts)
            if t in (R.HEX, R.TET):
                U[t] = vals
            elif t == R.WEDGE:
                Xc, wc = E.cubature()
                Phi, _ = E.basis(Xc)
                J = self.geo[t]["J"]
                U[t] = np.einsum("q,qi,kq,kcq->kci", wc, Phi, np.sqrt(J), vals)
            else:
                Xp, wp = E.projection_rule()
                Phi, _ = E.basis(Xp)
                _, _, Jq, _ = OM.vertex_map(E, Xp, self.V[t])
                U[t] = np.einsum("q,qi,kq,kcq->kci", wp, Phi, Jq, vals) / self.geo[t]["J"][:, None, :]
        return U

    def l2_error(self, U, func, time: float):
        """sqrt( sum_K int_K |U_h - U_exact|^2 ) over all four fields."""
        err = 0.0
        for t in self.types:
            E = self.refs[t]
            X, w = R.collapsed_volume_rule(t, self.N + 3)
            Phi, _ = E.basis(X)
            x, _, J, _ = OM.vertex_map(E, X, self.V[t])
            uh = np.einsum("qj,kcj->kcq", Phi, U[t])
            if t == R.WEDGE:
                uh = uh / np.sqrt(J)[:, None, :]
            ex = np.stack(func(x[..., 0], x[..., 1], x[..., 2], time), 1)
            err += float(np.einsum("q,kq,kcq->", w, J, (uh - ex) ** 2))
        return np.sqrt(err)

    # ------------------------------------------------------------------
    def min_jacobian(self, t):
        """min J of each element of type t, the 1/||J^{-1}||_inf of C_J^K (Section 3.4).

        The paper approximates the sup norms by maxima over quadrature points;
        here the element's vertices are added to the volume points (hex GL
        nodes, pyramid semi-nodal points (a_i, b_j)), so that a corner where
        the trilinear Jacobian dips below its value at the GL nodes is seen.
        For the pyramid J is bilinear in (a, b) and independent of c, so the
        four base vertices give its exact minimum.  Tetrahedra: J is constant.
        """
        J = self.geo[t]["J"]
        if J.ndim == 1:
            return J
        E = self.refs[t]
        corners = E.vref if t == R.HEX else E.vref[:4]
        _, _, Jv, _ = OM.vertex_map(E, corners, self.V[t])
        return np.minimum(np.min(J, axis=1), np.min(Jv, axis=1))

    def c_rhokappa(self):
        """C_rhokappa^K = max(tau_p,K kappa_K, tau_u,K / rho_K) per element
        (Section 3.4), with tau_p,K, tau_u,K the maxima over the element's faces
        (sub-faces for a coarse non-conforming face, whose own slot is left out)."""
        rc_own = self.rhoc[self.slot_elem]
        rc_nb = rc_own.copy()
        inner = self.nbr >= 0
        rc_nb[inner] = self.rhoc[self.slot_elem[self.nbr[inner]]]
        avg = 0.5 * (rc_own + rc_nb)
        ne = self.kappa.shape[0]
        use = ~self.is_parent
        taup_e = np.zeros(ne)
        tauu_e = np.zeros(ne)
        np.maximum.at(taup_e, self.slot_elem[use], 1.0 / avg[use])
        np.maximum.at(tauu_e, self.slot_elem[use], avg[use])
        out = {}
        for t in self.types:
            e = self.els[t]
            out[t] = np.maximum(taup_e[e] * self.kappa[e], tauu_e[e] / self.rho[e])
        return out

    def dt_elements(self, cfl: float = 0.5):
        """Local stable steps dtau_K = C / (C_rhokappa C_T(N) C_J^K) (Section 3, eq. dtK)."""
        out = {}
        crk = self.c_rhokappa()
        for t in self.types:
            sl = self.slot[t]
            e = self.els[t]
            jsr = self.Js_ref[sl]                      # (K, nf, Nfq)
            if t == R.WEDGE:
                cj = np.max((jsr / self.fJ[sl]).reshape(e.size, -1), axis=1)
            else:
                cj = np.max(jsr.reshape(e.size, -1), axis=1) / self.min_jacobian(t)
            out[t] = cfl / (crk[t] * trace_constant(t, self.N) * cj)
        return out

    def dt_min(self, cfl: float = 0.5):
        d = self.dt_elements(cfl)
        return min(float(np.min(v)) for v in d.values())


def lserk4_step(disc: Disc, U, dt: float):
    """One step of the 5-stage 2N-storage RK: res = a_s res + dt rhs(U); U = U + b_s res."""
    res = {t: np.zeros_like(U[t]) for t in disc.types}
    U = {t: U[t].copy() for t in disc.types}
    for s in range(5):
        Rhs = disc.rhs(U)
        for t in disc.types:
            res[t] = LSERK_A[s] * res[t] + dt * Rhs[t]
            U[t] = U[t] + LSERK_B[s] * res[t]
    return U
