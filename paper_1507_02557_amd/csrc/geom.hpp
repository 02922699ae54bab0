// FP64 geometry of vertex-mapped elements (Section 2: x = sum_v N_v x_v).
//
// Per element, evaluated once at set-up on the device (one thread per
// element): the Jacobian matrix F = dx/d(r,s,t), J = det F and
// G = F^{-1} = d(r,s,t)/dx at the points the stage kernels need, the outward
// unit normal and surface Jacobian at the canonical face cubature points, and
// for LSC-DG wedges the physical gradient of J.
#pragma once

#include <hip/hip_runtime.h>

#define HD __host__ __device__

namespace hdg {

struct GeoTables {
  // element descriptions, indexed by type
  double vref[4][8][3];
  int nv[4], nf[4];
  int fnv[4][6];
  int fv[4][6][4];
  double nref[4][6][3];
  double farea[4][6];
  // canonical face rules
  int Nfq;
  double tri_eta[64][2], tri_w[64];
  double quad_eta[64][2], quad_w[64];
  int tri_P[6][3];   // canonical vertex k -> local face vertex position
  int quad_P[8][4];
};

// Vertices of element e (nv of them, Vall = [K][nv][3]) into registers.  Every
// index is a compile-time constant so the array never lives in scratch
// memory; entries past nv are zero.
HD __forceinline__ void load_verts(const double* Vall, int64_t e, int nv, double V[8][3]) {
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int vv = v < nv ? v : 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double x = Vall[(e * nv + vv) * 3 + d];
      V[v][d] = v < nv ? x : 0.0;
    }
  }
}

// Vertex map of a type at reference point X: physical x and F[d][r] = dx_d/dxi_r.
HD __forceinline__ void vmap(int type, const double (*V)[3], const double* X, double* x, double F[3][3]) {
  const double r = X[0], s = X[1], t = X[2];
  for (int d = 0; d < 3; ++d) {
    x[d] = 0.0;
    F[d][0] = F[d][1] = F[d][2] = 0.0;
  }
  if (type == 0) {  // hex: trilinear
    const double sg[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                             {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
    for (int v = 0; v < 8; ++v) {
      const double a = 0.5 * (1 + sg[v][0] * r), b = 0.5 * (1 + sg[v][1] * s), c = 0.5 * (1 + sg[v][2] * t);
      const double n = a * b * c;
      const double dn[3] = {0.5 * sg[v][0] * b * c, a * 0.5 * sg[v][1] * c, a * b * 0.5 * sg[v][2]};
      for (int d = 0; d < 3; ++d) {
        x[d] += n * V[v][d];
        for (int k = 0; k < 3; ++k) F[d][k] += dn[k] * V[v][d];
      }
    }
  } else if (type == 1) {  // wedge: triangle (r,t) x linear in s
    const double L[3] = {-0.5 * (r + t), 0.5 * (1 + r), 0.5 * (1 + t)};
    const double Lr[3] = {-0.5, 0.5, 0.0}, Lt[3] = {-0.5, 0.0, 0.5};
    for (int lv = 0; lv < 2; ++lv) {
      const double sg = lv == 0 ? 0.5 * (1 - s) : 0.5 * (1 + s);
      const double ds = lv == 0 ? -0.5 : 0.5;
      for (int i = 0; i < 3; ++i) {
        const int v = 3 * lv + i;
        const double n = L[i] * sg;
        const double dn[3] = {Lr[i] * sg, L[i] * ds, Lt[i] * sg};
        for (int d = 0; d < 3; ++d) {
          x[d] += n * V[v][d];
          for (int k = 0; k < 3; ++k) F[d][k] += dn[k] * V[v][d];
        }
      }
    }
  } else if (type == 2) {  // pyramid: x = (1-c)/2 X(a,b) + (1+c)/2 x_apex
    const double omc = 1.0 - t;
    const double a = omc > 1e-14 ? 2.0 * (1.0 + r) / omc - 1.0 : -1.0;
    const double b = omc > 1e-14 ? 2.0 * (1.0 + s) / omc - 1.0 : -1.0;
    const double sg[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
    double X[3] = {0, 0, 0}, Xa[3] = {0, 0, 0}, Xb[3] = {0, 0, 0};
    for (int v = 0; v < 4; ++v) {
      const double fa = 0.5 * (1 + sg[v][0] * a), fb = 0.5 * (1 + sg[v][1] * b);
      for (int d = 0; d < 3; ++d) {
        X[d] += fa * fb * V[v][d];
        Xa[d] += 0.5 * sg[v][0] * fb * V[v][d];
        Xb[d] += fa * 0.5 * sg[v][1] * V[v][d];
      }
    }
    for (int d = 0; d < 3; ++d) {
      x[d] = 0.5 * omc * X[d] + 0.5 * (1.0 + t) * V[4][d];
      F[d][0] = Xa[d];
      F[d][1] = Xb[d];
      F[d][2] = 0.5 * (1 + a) * Xa[d] + 0.5 * (1 + b) * Xb[d] + 0.5 * (V[4][d] - X[d]);
    }
  } else {  // tet: affine
    const double L[4] = {-0.5 * (1 + r + s + t), 0.5 * (1 + r), 0.5 * (1 + s), 0.5 * (1 + t)};
    const double dL[4][3] = {{-0.5, -0.5, -0.5}, {0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5}};
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) {
        x[d] += L[v] * V[v][d];
        for (int k = 0; k < 3; ++k) F[d][k] += dL[v][k] * V[v][d];
      }
  }
}

HD __forceinline__ double det3(const double F[3][3]) {
  return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
         F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
}

// G = F^{-1}: G[r][d] = dxi_r / dx_d
HD __forceinline__ double inv3(const double F[3][3], double G[3][3]) {
  const double J = det3(F);
  const double iJ = 1.0 / J;
  G[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) * iJ;
  G[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * iJ;
  G[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * iJ;
  G[1][0] = (F[1][2] * F[2][0] - F[1][0] * F[2][2]) * iJ;
  G[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * iJ;
  G[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * iJ;
  G[2][0] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) * iJ;
  G[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * iJ;
  G[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * iJ;
  return J;
}

// Physical gradient of J for a wedge at X: grad_rst J = J tr(G dF/dxi_m),
// dF/dxi_m from the (constant) second derivatives of the wedge shape functions.
HD __forceinline__ void wedge_gradJ(const double (*V)[3], const double* X, double gJ[3]) {
  double x[3], F[3][3], G[3][3];
  vmap(1, V, X, x, F);
  const double J = inv3(F, G);
  // d2N/dr ds = dL/dr * dsig/ds, d2N/dt ds = dL/dt * dsig/ds; others vanish
  const double Lr[3] = {-0.5, 0.5, 0.0}, Lt[3] = {-0.5, 0.0, 0.5};
  double dF[3][3][3] = {};  // dF[m][d][r]
  for (int lv = 0; lv < 2; ++lv) {
    const double ds = lv == 0 ? -0.5 : 0.5;
    for (int i = 0; i < 3; ++i) {
      const int v = 3 * lv + i;
      for (int d = 0; d < 3; ++d) {
        // r-s and s-r pairs
        dF[1][d][0] += Lr[i] * ds * V[v][d];
        dF[0][d][1] += Lr[i] * ds * V[v][d];
        // t-s and s-t pairs
        dF[1][d][2] += Lt[i] * ds * V[v][d];
        dF[2][d][1] += Lt[i] * ds * V[v][d];
      }
    }
  }
  double dJ[3];
  for (int m = 0; m < 3; ++m) {
    double tr = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int d = 0; d < 3; ++d) tr += G[r][d] * dF[m][d][r];
    dJ[m] = J * tr;
  }
  for (int d = 0; d < 3; ++d) gJ[d] = G[0][d] * dJ[0] + G[1][d] * dJ[1] + G[2][d] * dJ[2];
}

// Canonical face point q of face f (orientation code o) of an element of the
// given type: reference coordinates Xr, physical point xq, tangent cross
// product cr (not normalised, canonical frame orientation).  Ve points to the
// element's vertices in global memory ([nv][3]); the face's vertices are read
// from there by runtime index.
HD __forceinline__ void face_point(const GeoTables& T, int type, const double* Ve, int f, int o, int q, double* Xr,
                          double* xq, double* cr) {
  const int nv = T.fnv[type][f];
  const int* P = nv == 3 ? T.tri_P[o] : T.quad_P[o];
  const double e1 = nv == 3 ? T.tri_eta[q][0] : T.quad_eta[q][0];
  const double e2 = nv == 3 ? T.tri_eta[q][1] : T.quad_eta[q][1];
  // shape functions of the canonical frame (triangle: barycentric, 4th = 0)
  double S[4], d1[4], d2[4];
  if (nv == 3) {
    S[0] = -0.5 * (e1 + e2); S[1] = 0.5 * (1 + e1); S[2] = 0.5 * (1 + e2); S[3] = 0.0;
    d1[0] = -0.5; d1[1] = 0.5; d1[2] = 0.0; d1[3] = 0.0;
    d2[0] = -0.5; d2[1] = 0.0; d2[2] = 0.5; d2[3] = 0.0;
  } else {
    const double cs[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      S[k] = 0.25 * (1 + e1 * cs[k][0]) * (1 + e2 * cs[k][1]);
      d1[k] = 0.25 * cs[k][0] * (1 + e2 * cs[k][1]);
      d2[k] = 0.25 * (1 + e1 * cs[k][0]) * cs[k][1];
    }
  }
  double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    Xr[d] = 0.0;
    xq[d] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k >= nv) continue;
    const int lv = T.fv[type][f][P[k]];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double xv = Ve[lv * 3 + d];
      Xr[d] += S[k] * T.vref[type][lv][d];
      xq[d] += S[k] * xv;
      t1[d] += d1[k] * xv;
      t2[d] += d2[k] * xv;
    }
  }
  cr[0] = t1[1] * t2[2] - t1[2] * t2[1];
  cr[1] = t1[2] * t2[0] - t1[0] * t2[2];
  cr[2] = t1[0] * t2[1] - t1[1] * t2[0];
}

}  // namespace hdg
