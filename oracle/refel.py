"""Reference elements of the hybrid-mesh DG method (oracle side).

Each class gives, for polynomial order N:

* the reference vertices and the vertex (order-1) shape functions of the
  vertex map and their reference derivatives (Section 2: vertex-mapped
  elements);
* the faces (local vertex lists, cyclic for quadrilaterals), their reference
  outward normals and true reference areas;
* the basis functions of the element's approximation space and their
  reference gradients at arbitrary reference points (Section 2.1);
* the points and rules the method uses (nodes, cubature).

Conventions shared with the GPU library (each side implements them on its
own) are stated in the docstrings: dof orderings, node sets and rule
orderings.

Reference coordinates are (r,s,t); the collapsed coordinates are (a,b,c).
"""
from __future__ import annotations

import numpy as np

from .quad import djacobi, dlagrange, gauss_jacobi, gauss_legendre, jacobi, lagrange

HEX, WEDGE, PYR, TET = 0, 1, 2, 3


# ---------------------------------------------------------------------------
# Rules on the canonical face and on reference volumes
# ---------------------------------------------------------------------------

def tri_rule(n: int):
    """Collapsed rule on the triangle (-1,-1),(1,-1),(-1,1): GL(n) in a x GJ^{(1,0)}(n) in b.

    eta1 = (1+a)(1-b)/2 - 1, eta2 = b; exact to degree 2n-1.  Point
    q = j*n + i for a-index i and b-index j.  Weights sum to 2.
    """
    xa, wa = gauss_legendre(n)
    xb, wb = gauss_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(xa, xb, indexing="xy")  # A[j,i] = xa[i]
    WA, WB = np.meshgrid(wa, wb, indexing="xy")
    e1 = (1.0 + A) * (1.0 - B) / 2.0 - 1.0
    e2 = B
    return np.stack([e1.ravel(), e2.ravel()], 1), (WA * WB / 2.0).ravel()


def quad_rule(n: int):
    """Tensor GL(n) x GL(n) on [-1,1]^2; point q = j*n + i."""
    x, w = gauss_legendre(n)
    X1, X2 = np.meshgrid(x, x, indexing="xy")
    W1, W2 = np.meshgrid(w, w, indexing="xy")
    return np.stack([X1.ravel(), X2.ravel()], 1), (W1 * W2).ravel()


def face_shape(nv: int, eta):
    """Shape functions of the canonical face frame and their eta-derivatives.

    Triangle (canonical vertices at (-1,-1),(1,-1),(-1,1)): barycentric.
    Quadrilateral (canonical vertices (-1,-1),(1,-1),(1,1),(-1,1)): bilinear.
    Returns S (npts, nv), dS (2, npts, nv).
    """
    e1, e2 = eta[:, 0], eta[:, 1]
    if nv == 3:
        S = np.stack([-(e1 + e2) / 2.0, (1.0 + e1) / 2.0, (1.0 + e2) / 2.0], 1)
        d1 = np.tile([-0.5, 0.5, 0.0], (eta.shape[0], 1))
        d2 = np.tile([-0.5, 0.0, 0.5], (eta.shape[0], 1))
    else:
        cs = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
        S = np.stack([(1 + e1 * c[0]) * (1 + e2 * c[1]) / 4.0 for c in cs], 1)
        d1 = np.stack([c[0] * (1 + e2 * c[1]) / 4.0 for c in cs], 1)
        d2 = np.stack([(1 + e1 * c[0]) * c[1] / 4.0 for c in cs], 1)
    return S, np.stack([d1, d2], 0)


def collapsed_volume_rule(etype: int, n: int):
    """Exact-by-construction collapsed rules on the reference volumes (n points per direction).

    hex: GL^3.  wedge: GL(a) x GL(b=s) x GJ^{(1,0)}(c), weight /2.
    pyramid: GL(a) x GL(b) x GJ^{(2,0)}(c), weight /4.
    tet: GL(a) x GJ^{(1,0)}(b) x GJ^{(2,0)}(c), weight /8.
    Points ordered with the first collapsed index fastest.
    """
    if etype == HEX:
        x, w = gauss_legendre(n)
        xa = xb = xc = x
        wa = wb = wc = w
        scale = 1.0
    elif etype == WEDGE:
        xa, wa = gauss_legendre(n)
        xb, wb = gauss_legendre(n)
        xc, wc = gauss_jacobi(n, 1.0, 0.0)
        scale = 0.5
    elif etype == PYR:
        xa, wa = gauss_legendre(n)
        xb, wb = gauss_legendre(n)
        xc, wc = gauss_jacobi(n, 2.0, 0.0)
        scale = 0.25
    else:
        xa, wa = gauss_legendre(n)
        xb, wb = gauss_jacobi(n, 1.0, 0.0)
        xc, wc = gauss_jacobi(n, 2.0, 0.0)
        scale = 0.125
    C, B, A = np.meshgrid(xc, xb, xa, indexing="ij")
    WC, WB, WA = np.meshgrid(wc, wb, wa, indexing="ij")
    a, b, c = A.ravel(), B.ravel(), C.ravel()
    if etype == HEX:
        r, s, t = a, b, c
    elif etype == WEDGE:
        r, s, t = (1 + a) * (1 - c) / 2 - 1, b, c
    elif etype == PYR:
        r, s, t = (1 + a) * (1 - c) / 2 - 1, (1 + b) * (1 - c) / 2 - 1, c
    else:
        r, s, t = (1 + a) * (1 - b) * (1 - c) / 4 - 1, (1 + b) * (1 - c) / 2 - 1, c
    return np.stack([r, s, t], 1), (WA * WB * WC).ravel() * scale


# ---------------------------------------------------------------------------
# Element classes
# ---------------------------------------------------------------------------

class RefElement:
    etype: int
    name: str
    vref: np.ndarray
    faces: list
    face_nref: np.ndarray
    face_area: np.ndarray

    def __init__(self, N: int):
        if N < 1:
            raise ValueError("N >= 1 required")
        self.N = N

    @property
    def nv(self):
        return self.vref.shape[0]

    @property
    def nfaces(self):
        return len(self.faces)

    # vertex map -------------------------------------------------------------
    def shape(self, X):
        """Vertex shape functions Nv (npts, nv) and derivatives dN (3, npts, nv)."""
        raise NotImplementedError

    def shape2(self, X):
        """Second derivatives d2N (3, 3, npts, nv) of the vertex shape functions."""
        raise NotImplementedError

    # basis ----------------------------------------------------------------
    def basis(self, X):
        """Basis values Phi (npts, Np) and reference gradients dPhi (3, npts, Np)."""
        raise NotImplementedError


class Hex(RefElement):
    """GL nodal hexahedron (Section 2.1.1).

    Nodes: tensor (N+1)-point Gauss-Legendre; node m = i + (N+1)(j + (N+1)k)
    at (x_i, x_j, x_k).  Basis l_i(r) l_j(s) l_k(t).
    """

    etype = HEX
    name = "hex"
    vref = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                     [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
    faces = [(0, 3, 7, 4), (1, 2, 6, 5), (0, 1, 5, 4), (3, 2, 6, 7), (0, 1, 2, 3), (4, 5, 6, 7)]
    face_nref = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], dtype=np.float64)
    face_area = np.array([4.0] * 6)

    def __init__(self, N):
        super().__init__(N)
        self.Np = (N + 1) ** 3
        self.x1d, self.w1d = gauss_legendre(N + 1)
        n1 = N + 1
        # m = i + n1*(j + n1*k): build with k outermost
        K, J, I = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
        self.ijk = np.stack([I.ravel(), J.ravel(), K.ravel()], 1)
        self.nodes = self.x1d[self.ijk]
        self.wnodes = np.prod(self.w1d[self.ijk], axis=1)

    def shape(self, X):
        S = np.ones((X.shape[0], 8))
        dS = np.ones((3, X.shape[0], 8))
        for v in range(8):
            f = [(1 + X[:, d] * self.vref[v, d]) / 2 for d in range(3)]
            df = [self.vref[v, d] / 2 * np.ones(X.shape[0]) for d in range(3)]
            S[:, v] = f[0] * f[1] * f[2]
            dS[0, :, v] = df[0] * f[1] * f[2]
            dS[1, :, v] = f[0] * df[1] * f[2]
            dS[2, :, v] = f[0] * f[1] * df[2]
        return S, dS

    def basis(self, X):
        L = [lagrange(self.x1d, X[:, d]) for d in range(3)]
        D = [dlagrange(self.x1d, X[:, d]) for d in range(3)]
        i, j, k = self.ijk[:, 0], self.ijk[:, 1], self.ijk[:, 2]
        Phi = L[0][:, i] * L[1][:, j] * L[2][:, k]
        dPhi = np.stack([D[0][:, i] * L[1][:, j] * L[2][:, k],
                         L[0][:, i] * D[1][:, j] * L[2][:, k],
                         L[0][:, i] * L[1][:, j] * D[2][:, k]], 0)
        return Phi, dPhi


class Tet(RefElement):
    """Nodal tetrahedron (Section 2.1.2).

    Nodes: equispaced lattice (-1 + 2i/N, -1 + 2j/N, -1 + 2k/N), i+j+k <= N,
    ordered k outermost, then j, then i fastest.  The Lagrange basis on these
    nodes is expressed through the spanning set P_a(r) P_b(s) P_c(t),
    a+b+c <= N (Legendre polynomials), which spans P_N.
    """

    etype = TET
    name = "tet"
    vref = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    faces = [(0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)]
    face_nref = np.array([[0, 0, -1], [0, -1, 0], [1, 1, 1], [-1, 0, 0]], dtype=np.float64)
    face_area = np.array([2.0, 2.0, 2.0 * np.sqrt(3.0), 2.0])

    def __init__(self, N):
        super().__init__(N)
        self.Np = (N + 1) * (N + 2) * (N + 3) // 6
        nodes = []
        for k in range(N + 1):
            for j in range(N + 1 - k):
                for i in range(N + 1 - k - j):
                    nodes.append((-1 + 2 * i / N, -1 + 2 * j / N, -1 + 2 * k / N))
        self.nodes = np.array(nodes, dtype=np.float64)
        self.pows = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]
        V, _ = self._span(self.nodes)
        self.Cinv = np.linalg.inv(V)

    def _span(self, X):
        cols, dcols = [], []
        for (a, b, c) in self.pows:
            pa, pb, pc = jacobi(a, 0, 0, X[:, 0]), jacobi(b, 0, 0, X[:, 1]), jacobi(c, 0, 0, X[:, 2])
            da, db, dc = djacobi(a, 0, 0, X[:, 0]), djacobi(b, 0, 0, X[:, 1]), djacobi(c, 0, 0, X[:, 2])
            cols.append(pa * pb * pc)
            dcols.append(np.stack([da * pb * pc, pa * db * pc, pa * pb * dc], 0))
        return np.stack(cols, 1), np.stack(dcols, 2)

    def shape(self, X):
        r, s, t = X[:, 0], X[:, 1], X[:, 2]
        S = np.stack([-(1 + r + s + t) / 2, (1 + r) / 2, (1 + s) / 2, (1 + t) / 2], 1)
        d = np.array([[-0.5, 0.5, 0.0, 0.0], [-0.5, 0.0, 0.5, 0.0], [-0.5, 0.0, 0.0, 0.5]])
        dS = np.repeat(d[:, None, :], X.shape[0], axis=1)
        return S, dS

    def basis(self, X):
        P, dP = self._span(X)
        return P @ self.Cinv, np.einsum("dqm,mj->dqj", dP, self.Cinv)


class Wedge(RefElement):
    """Modal LSC-DG wedge (Section 2.1.3).

    Basis phi_{i j k}(a,b,c) = P_i(a) P_j(b) ((1-c)/2)^i P_k^{(2i+1,0)}(c),
    0 <= i,j <= N, 0 <= k <= N-i, with r = (1+a)(1-c)/2 - 1, s = b, t = c,
    each scaled to unit L2 norm on the reference wedge.  Dof ordering
    m = j * Ntri + tri(i,k), where tri enumerates (i,k) with i outer, k inner.
    """

    etype = WEDGE
    name = "wedge"
    vref = np.array([[-1, -1, -1], [1, -1, -1], [-1, -1, 1], [-1, 1, -1], [1, 1, -1], [-1, 1, 1]], dtype=np.float64)
    faces = [(0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (0, 2, 5, 3), (1, 2, 5, 4)]
    face_nref = np.array([[0, -1, 0], [0, 1, 0], [0, 0, -1], [-1, 0, 0], [1, 0, 1]], dtype=np.float64)
    face_area = np.array([2.0, 2.0, 4.0, 4.0, 4.0 * np.sqrt(2.0)])

    def __init__(self, N):
        super().__init__(N)
        self.Ntri = (N + 1) * (N + 2) // 2
        self.Np = self.Ntri * (N + 1)
        tri = [(i, k) for i in range(N + 1) for k in range(N + 1 - i)]
        self.idx = [(i, j, k) for j in range(N + 1) for (i, k) in tri]
        # unit-norm scaling: ||phi||^2 = 2/(2i+1) * 2/(2j+1) * 2/(2i+2k+2)
        # evaluated here by quadrature of the unscaled function
        X, w = collapsed_volume_rule(WEDGE, N + 2)
        P, _ = self._raw(X)
        self.scale = 1.0 / np.sqrt(np.einsum("q,qm->m", w, P * P))

    def _raw(self, X):
        r, s, t = X[:, 0], X[:, 1], X[:, 2]
        c = t
        b = s
        one_m_c = 1.0 - c
        a = np.where(one_m_c > 1e-14, 2.0 * (1.0 + r) / np.where(one_m_c > 1e-14, one_m_c, 1.0) - 1.0, -1.0)
        h = one_m_c / 2.0
        vals, grads = [], []
        for (i, j, k) in self.idx:
            A, dA = jacobi(i, 0, 0, a), djacobi(i, 0, 0, a)
            B, dB = jacobi(j, 0, 0, b), djacobi(j, 0, 0, b)
            Pk, dPk = jacobi(k, 2 * i + 1, 0, c), djacobi(k, 2 * i + 1, 0, c)
            hi = h ** i
            him1 = h ** (i - 1) if i >= 1 else np.zeros_like(h)
            C = hi * Pk
            dC = (-(i / 2.0) * him1 * Pk if i >= 1 else 0.0) + hi * dPk
            v = A * B * C
            dr = dA * B * him1 * Pk
            ds = A * dB * C
            dt = dA * B * (1 + a) / 2.0 * him1 * Pk + A * B * dC
            vals.append(v)
            grads.append(np.stack([dr, ds, dt], 0))
        return np.stack(vals, 1), np.stack(grads, 2)

    def basis(self, X):
        P, dP = self._raw(X)
        return P * self.scale, dP * self.scale

    def shape(self, X):
        r, s, t = X[:, 0], X[:, 1], X[:, 2]
        L = [-(r + t) / 2, (1 + r) / 2, (1 + t) / 2]
        dL = [(-0.5, -0.5), (0.5, 0.0), (0.0, 0.5)]  # (d/dr, d/dt)
        sig = [(1 - s) / 2, (1 + s) / 2]
        dsig = [-0.5, 0.5]
        S = np.zeros((X.shape[0], 6))
        dS = np.zeros((3, X.shape[0], 6))
        for lvl in range(2):
            for i in range(3):
                v = 3 * lvl + i
                S[:, v] = L[i] * sig[lvl]
                dS[0, :, v] = dL[i][0] * sig[lvl]
                dS[1, :, v] = L[i] * dsig[lvl]
                dS[2, :, v] = dL[i][1] * sig[lvl]
        return S, dS

    def shape2(self, X):
        dL = [(-0.5, -0.5), (0.5, 0.0), (0.0, 0.5)]
        dsig = [-0.5, 0.5]
        d2 = np.zeros((3, 3, X.shape[0], 6))
        for lvl in range(2):
            for i in range(3):
                v = 3 * lvl + i
                d2[0, 1, :, v] = d2[1, 0, :, v] = dL[i][0] * dsig[lvl]
                d2[2, 1, :, v] = d2[1, 2, :, v] = dL[i][1] * dsig[lvl]
        return d2

    def cubature(self):
        """The method's volume cubature: GL(N+1) x GL(N+1) x GJ^{(1,0)}(N+1), collapsed."""
        return collapsed_volume_rule(WEDGE, self.N + 1)


class Pyramid(RefElement):
    """Semi-nodal pyramid (Section 2.1.4).

    Basis phi_{ijk}(a,b,c) = l_i^k(a) l_j^k(b) ((1-c)/2)^k P_{N-k}^{(2k+3,0)}(c),
    0 <= i,j <= k <= N, with l^k the Lagrange polynomials at the (k+1)-point
    GL nodes, r = (1+a)(1-c)/2 - 1, s = (1+b)(1-c)/2 - 1, t = c; each
    function is scaled to unit L2 norm on the reference pyramid.  Dof
    ordering m = off_k + j (k+1) + i.  The dof's geometry point is
    (r,s,t) = (a_i^k, b_j^k, -1).
    """

    etype = PYR
    name = "pyr"
    vref = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    faces = [(0, 1, 2, 3), (0, 3, 4), (0, 1, 4), (1, 2, 4), (3, 2, 4)]
    face_nref = np.array([[0, 0, -1], [-1, 0, 0], [0, -1, 0], [1, 0, 1], [0, 1, 1]], dtype=np.float64)
    face_area = np.array([4.0, 2.0, 2.0, 2.0 * np.sqrt(2.0), 2.0 * np.sqrt(2.0)])

    def __init__(self, N):
        super().__init__(N)
        self.Np = (N + 1) * (N + 2) * (2 * N + 3) // 6
        self.gl = [gauss_legendre(k + 1) for k in range(N + 1)]
        self.idx = [(i, j, k) for k in range(N + 1) for j in range(k + 1) for i in range(k + 1)]
        self.geo_points = np.array([[self.gl[k][0][i], self.gl[k][0][j], -1.0] for (i, j, k) in self.idx])
        X, w = collapsed_volume_rule(PYR, N + 3)
        P, _ = self._raw(X)
        self.scale = 1.0 / np.sqrt(np.einsum("q,qm->m", w, P * P))

    def _raw(self, X):
        r, s, t = X[:, 0], X[:, 1], X[:, 2]
        c = t
        one_m_c = 1.0 - c
        safe = np.where(one_m_c > 1e-14, one_m_c, 1.0)
        a = np.where(one_m_c > 1e-14, 2.0 * (1.0 + r) / safe - 1.0, -1.0)
        b = np.where(one_m_c > 1e-14, 2.0 * (1.0 + s) / safe - 1.0, -1.0)
        h = one_m_c / 2.0
        N = self.N
        La = [lagrange(self.gl[k][0], a) for k in range(N + 1)]
        Lb = [lagrange(self.gl[k][0], b) for k in range(N + 1)]
        dLa = [dlagrange(self.gl[k][0], a) for k in range(N + 1)]
        dLb = [dlagrange(self.gl[k][0], b) for k in range(N + 1)]
        vals, grads = [], []
        for (i, j, k) in self.idx:
            Pc, dPc = jacobi(N - k, 2 * k + 3, 0, c), djacobi(N - k, 2 * k + 3, 0, c)
            hk = h ** k
            hkm1 = h ** (k - 1) if k >= 1 else np.zeros_like(h)
            E = hk * Pc
            dE = (-(k / 2.0) * hkm1 * Pc if k >= 1 else 0.0) + hk * dPc
            la, lb, dla, dlb = La[k][:, i], Lb[k][:, j], dLa[k][:, i], dLb[k][:, j]
            v = la * lb * E
            dr = dla * lb * hkm1 * Pc
            ds = la * dlb * hkm1 * Pc
            dt = ((1 + a) / 2 * dla * lb + (1 + b) / 2 * la * dlb) * hkm1 * Pc + la * lb * dE
            vals.append(v)
            grads.append(np.stack([dr, ds, dt], 0))
        return np.stack(vals, 1), np.stack(grads, 2)

    def basis(self, X):
        P, dP = self._raw(X)
        return P * self.scale, dP * self.scale

    def shape(self, X):
        r, s, t = X[:, 0], X[:, 1], X[:, 2]
        c = t
        one_m_c = 1.0 - c
        safe = np.where(one_m_c > 1e-14, one_m_c, 1.0)
        a = 2.0 * (1.0 + r) / safe - 1.0
        b = 2.0 * (1.0 + s) / safe - 1.0
        npts = X.shape[0]
        S = np.zeros((npts, 5))
        dS = np.zeros((3, npts, 5))
        for v in range(4):
            av, bv = self.vref[v, 0], self.vref[v, 1]
            B = (1 + a * av) / 2 * (1 + b * bv) / 2
            Ba = av / 2 * (1 + b * bv) / 2
            Bb = (1 + a * av) / 2 * bv / 2
            S[:, v] = B * one_m_c / 2
            dS[0, :, v] = Ba
            dS[1, :, v] = Bb
            dS[2, :, v] = (1 + a) / 2 * Ba + (1 + b) / 2 * Bb - B / 2
        S[:, 4] = (1 + c) / 2
        dS[2, :, 4] = 0.5
        return S, dS

    def projection_rule(self):
        """Rule used to project initial data: GL(N+1)^2 x GJ^{(2,0)}(N+1), collapsed."""
        return collapsed_volume_rule(PYR, self.N + 1)


def make(etype: int, N: int) -> RefElement:
    return {HEX: Hex, WEDGE: Wedge, PYR: Pyramid, TET: Tet}[etype](N)
