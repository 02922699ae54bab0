// Fused stage kernel body for semi-nodal pyramids (Section 2.3.4,
// Algorithm 7: skew-symmetric form with the quadrature-free operators).
//
// Volume:  rhs_u_d = -(1/rho) sum_r G_rd (D^r p),
//          rhs_p   = (kappa / J_i) sum_r sum_j D^r_ji U^r_j,
//          U^r_j   = J_j sum_d G_rd,j u_d,j   (premultiplied dofs),
//          with G, J at (a_i^k, b_j^k) (constant in c) and mass diag(J).
// Surface: base (quadrilateral) face through the basis values at its local GL
//          points; triangular faces through the face's equispaced lattice
//          (the pyramid's trace on a triangle is a degree-N polynomial), as
//          for tetrahedra.  With lattice traces (a.lat) the triangular faces
//          exchange lattice values; the flux (a degree-N polynomial on the
//          planar face) is taken at the lattice nodes and weighted by the
//          face-lattice mass matrix, which gives the cubature rule's face
//          integrals exactly.
#pragma once

#include "stage_common.hpp"

namespace hdg {

template <int N, int EPB, int NTH = 256>
struct PyrStage {
  static constexpr int Np = (N + 1) * (N + 2) * (2 * N + 3) / 6;
  static constexpr int Nfn = (N + 1) * (N + 2) / 2;
  static constexpr int Nfq = (N + 1) * (N + 1);
  static constexpr int TS = trace_stride(N), LW = lattice_width(N);
  static constexpr int NT = NTH;
  static constexpr int kEPB = EPB;
  static constexpr int nphase = 7;
  static constexpr int kTraceBegin = 5;  // first phase that writes traces
  static constexpr bool kDInLds = (3 * Np * Np * 4) <= 48 * 1024;
  static constexpr int kOpsFloats = 3 * Np * Np + Nfq * Np + 4 * Nfn * Np + Nfq * Nfn + Nfn * Nfn;
  static constexpr int kOpsInts = 8 * Nfq + 6 * Nfn;
  static constexpr int kDl = kDInLds ? Np : 1;

  // operator tables (shared by all batches of a block) and one batch's data
  struct Ops {
    float D[3][kDl][kDl];
    float Fq[Nfq][Np];
    float Ft[4][Nfn][Np];
    float Ican[Nfq][Nfn];
    float Mw[Nfn][Nfn];  // face-lattice mass matrix / w_0 (w_0: weight of cubature point 0)
    int qperm[8][Nfq];
    int tperm[6][Nfn];
  };
  struct Batch {
    float u[4][EPB][Np];
    float un[4][EPB][Np];
    float ur[3][EPB][Np];
    float J[EPB][Np];
    float g[EPB][5][Nfq][4];
    float c[EPB][4][Nfn][4];
    float s[EPB][Np][4];
    float mat[EPB][2];
    // face records: neighbour slot (or boundary code), orientation,
    // penalties, 1 if the neighbour's value comes from the mid-step traces
    int nb[EPB][5];
    int ori[EPB][5];
    float2 tau[EPB][5];
    int half[EPB][5];
  };
  struct Smem {
    Ops o;
    Batch b;
  };
  // a wavefront's view: the block's tables and the wavefront's own batch
  struct WaveRef {
    const Ops& o;
    Batch& b;
  };
  HD static Batch& batch(Smem& sm) { return sm.b; }
  HD static Batch& batch(WaveRef& r) { return r.b; }

  HD static bool active(int ph, int mode) {
    if (mode == kModeTrace) return ph == 0 || ph >= 5;
    if (mode == kModeRhs || mode == kModeRhsHist) return ph <= 4;
    return true;
  }

  HD static float Dop(const Ops& o, const StageArgs& a, int r, int i, int j) {
    if (kDInLds) return o.D[r][i % kDl][j % kDl];
    return a.ops[(r * Np + i) * Np + j];
  }

  // tables into LDS by nthr threads
  HD static void load_ops(int tid, int nthr, Ops& o, const StageArgs& a) {
    if (kDInLds)
      for (int i = tid; i < 3 * Np * Np; i += nthr) (&o.D[0][0][0])[i] = a.ops[i];
    const int o1 = 3 * Np * Np, o2 = o1 + Nfq * Np, o3 = o2 + 4 * Nfn * Np;
    for (int i = tid; i < Nfq * Np; i += nthr) (&o.Fq[0][0])[i] = a.ops[o1 + i];
    for (int i = tid; i < 4 * Nfn * Np; i += nthr) (&o.Ft[0][0][0])[i] = a.ops[o2 + i];
    for (int i = tid; i < Nfq * Nfn; i += nthr) (&o.Ican[0][0])[i] = a.ops[o3 + i];
    for (int i = tid; i < Nfn * Nfn; i += nthr) (&o.Mw[0][0])[i] = a.ops[o3 + Nfq * Nfn + i];
    for (int i = tid; i < 8 * Nfq; i += nthr) (&o.qperm[0][0])[i] = a.iops[i];
    for (int i = tid; i < 6 * Nfn; i += nthr) (&o.tperm[0][0])[i] = a.iops[8 * Nfq + i];
  }
  HD static void load_ops(int tid, Smem& sm, const StageArgs& a) { load_ops(tid, NT, sm.o, a); }

  HD static void phase(int ph, int tid, Smem& sm, const StageArgs& a, int64_t e0) { phase(ph, tid, sm.o, sm.b, a, e0); }
  HD static void phase(int ph, int tid, WaveRef& r, const StageArgs& a, int64_t e0) { phase(ph, tid, r.o, r.b, a, e0); }

  HD static void phase(int ph, int tid, const Ops& o, Batch& sm, const StageArgs& a, int64_t e0) {
    const int64_t K = a.K;
    if (ph == 0) {
      // state, J, material and face records, all loads issued together
      constexpr int NU = (4 * EPB * Np + NT - 1) / NT, NJ = (EPB * Np + NT - 1) / NT;
      static_assert(5 * EPB <= NT, "one face record per thread");
      float vu[NU], vj[NJ];
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        const int it = tid + r * NT;
        vu[r] = 0.f;
        if (it >= 4 * EPB * Np) continue;
        const int f = it / (EPB * Np), rr = it % (EPB * Np);
        const int el = rr / Np, i = rr % Np;
        const int64_t e = item(a, e0 + el);
        if (e >= 0) vu[r] = a.U[(int64_t)f * K * Np + e * Np + i];
      }
#pragma unroll
      for (int r = 0; r < NJ; ++r) {
        const int it = tid + r * NT;
        vj[r] = 1.f;
        if (it >= EPB * Np) continue;
        const int el = it / Np, i = it % Np;
        const int64_t e = item(a, e0 + el);
        if (e >= 0) vj[r] = a.geo[(e * 10 + 9) * Np + i];
      }
      const bool rec = tid < 5 * EPB;
      const int rel = tid / 5, rf = tid % 5;
      int nb = -1, ori = 0, half = 0;
      float2 tau = make_float2(0.f, 0.f), mt = tau;
      if (rec) {
        const int64_t e = item(a, e0 + rel);
        if (e >= 0) {
          const int64_t slot = a.slot0 + e * 5 + rf;
          nb = a.nbr[slot];
          ori = a.ori[slot];
          tau = a.tau[slot];
          if (rf == 0) mt = a.mat[e];
          if (nb >= 0) half = neighbour_mid(a, slot, nb);
        }
      }
#pragma unroll
      for (int r = 0; r < NU; ++r) {
        const int it = tid + r * NT;
        if (it < 4 * EPB * Np) (&sm.u[0][0][0])[it] = vu[r];
      }
#pragma unroll
      for (int r = 0; r < NJ; ++r) {
        const int it = tid + r * NT;
        if (it < EPB * Np) (&sm.J[0][0])[it] = vj[r];
      }
      if (rec) {
        sm.nb[rel][rf] = nb;
        sm.ori[rel][rf] = ori;
        sm.tau[rel][rf] = tau;
        sm.half[rel][rf] = half;
        if (rf == 0) {
          sm.mat[rel][0] = mt.x;
          sm.mat[rel][1] = mt.y;
        }
      }
    } else if (ph == 1) {
      // premultiplied contravariant velocities U^r = J sum_d G_rd u_d; the
      // flux at the base face's cubature points (all faces' without lattice
      // traces) and, with lattice traces, at the triangular faces' lattice
      // nodes (canonical order, weighted by w_0 J^s, constant on the planar
      // face).  Loads first, all issued together.
      constexpr int NR = (EPB * Np + NT - 1) / NT, NC = (EPB * 5 * Nfq + NT - 1) / NT;
      constexpr int NL = (EPB * 4 * Nfn + NT - 1) / NT;
      const int nfc = a.lat ? 1 : 5;
      const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
      float gr[NR][10];
      float4 cg[NC], co[NC], cp[NC], lg[NL], lo[NL], lp[NL];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int it = tid + r * NT;
        const int el = it / Np, i = it % Np;
        const int64_t e = it < EPB * Np ? item(a, e0 + el) : -1;
#pragma unroll
        for (int k = 0; k < 10; ++k) gr[r][k] = e >= 0 ? a.geo[(e * 10 + k) * Np + i] : 0.f;
      }
#pragma unroll
      for (int r = 0; r < NC; ++r) {
        const int it = tid + r * NT;
        cg[r] = co[r] = cp[r] = z;
        if (it >= EPB * nfc * Nfq) continue;
        const int el = it / (nfc * Nfq), rr = it % (nfc * Nfq);
        const int f = rr / Nfq, q = rr % Nfq;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t slot = a.slot0 + e * 5 + f;
        const int nb = sm.nb[el][f];
        cg[r] = a.fgeo[(e * 5 + f) * Nfq + q];
        co[r] = a.tr_in[slot * TS + q];
        if (nb >= 0) cp[r] = (sm.half[el][f] ? a.tr_half : a.tr_in)[(int64_t)nb * TS + q];
      }
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        const int it = tid + r * NT;
        lg[r] = lo[r] = lp[r] = z;
        if (!a.lat || it >= EPB * 4 * Nfn) continue;
        const int el = it / (4 * Nfn), rr = it % (4 * Nfn);
        const int tf = rr / Nfn, m = rr % Nfn;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t slot = a.slot0 + e * 5 + 1 + tf;
        const int nb = sm.nb[el][1 + tf];
        lg[r] = a.fgeo[(e * 5 + 1 + tf) * Nfq];
        lo[r] = a.tr_in[slot * TS + m];
        if (nb >= 0) lp[r] = (sm.half[el][1 + tf] ? a.tr_half : a.tr_in)[(int64_t)nb * TS + m];
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const int it = tid + r * NT;
        if (it >= EPB * Np) continue;
        const int el = it / Np, i = it % Np;
#pragma unroll
        for (int d = 0; d < 3; ++d)
          sm.ur[d][el][i] = gr[r][9] * (gr[r][3 * d] * sm.u[1][el][i] + gr[r][3 * d + 1] * sm.u[2][el][i] +
                                        gr[r][3 * d + 2] * sm.u[3][el][i]);
      }
#pragma unroll
      for (int r = 0; r < NC; ++r) {
        const int it = tid + r * NT;
        if (it >= EPB * nfc * Nfq) continue;
        const int el = it / (nfc * Nfq), rr = it % (nfc * Nfq);
        const int f = rr / Nfq, q = rr % Nfq;
        if (item(a, e0 + el) < 0) continue;
        const int nb = sm.nb[el][f];
        const float4 g = cg[r];
        const float4 p = nb >= 0 ? cp[r] : mirror_state(co[r], -nb - 1, g.x, g.y, g.z);
        float out[4];
        upwind_flux(co[r], p, g, sm.tau[el][f], true, out);
        const int l = (f == 0) ? o.qperm[sm.ori[el][0]][q] : q;
        for (int c = 0; c < 4; ++c) sm.g[el][f][l][c] = out[c];
      }
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        const int it = tid + r * NT;
        if (!a.lat || it >= EPB * 4 * Nfn) continue;
        const int el = it / (4 * Nfn), rr = it % (4 * Nfn);
        const int tf = rr / Nfn, m = rr % Nfn;
        if (item(a, e0 + el) < 0) continue;
        const int nb = sm.nb[el][1 + tf];
        const float4 g = lg[r];
        const float4 p = nb >= 0 ? lp[r] : mirror_state(lo[r], -nb - 1, g.x, g.y, g.z);
        float out[4];
        upwind_flux(lo[r], p, g, sm.tau[el][1 + tf], true, out);
        for (int c = 0; c < 4; ++c) sm.g[el][1 + tf][m][c] = out[c];
      }
    } else if (ph == 2) {
      for (int it = tid; it < EPB * 4 * Nfn; it += NT) {
        const int el = it / (4 * Nfn), rr = it % (4 * Nfn);
        const int tf = rr / Nfn, m = rr % Nfn;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int ori = sm.ori[el][1 + tf];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        if (a.lat) {
          // c = M_f f / w_0 from the lattice flux
          for (int j = 0; j < Nfn; ++j) {
            const float w = o.Mw[m][j];
            for (int c = 0; c < 4; ++c) acc[c] += w * sm.g[el][1 + tf][j][c];
          }
        } else {
          // c = Ican^T (w J^s f) from the cubature flux
          for (int q = 0; q < Nfq; ++q) {
            const float w = o.Ican[q][m];
            for (int c = 0; c < 4; ++c) acc[c] += w * sm.g[el][1 + tf][q][c];
          }
        }
        const int l = o.tperm[ori][m];
        for (int c = 0; c < 4; ++c) sm.c[el][tf][l][c] = acc[c];
      }
    } else if (ph == 3) {
      for (int it = tid; it < EPB * Np; it += NT) {
        const int el = it / Np, i = it % Np;
        if (item(a, e0 + el) < 0) continue;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int l = 0; l < Nfq; ++l) {
          const float w = o.Fq[l][i];
          for (int c = 0; c < 4; ++c) acc[c] += w * sm.g[el][0][l][c];
        }
        for (int tf = 0; tf < 4; ++tf)
          for (int l = 0; l < Nfn; ++l) {
            const float w = o.Ft[tf][l][i];
            for (int c = 0; c < 4; ++c) acc[c] += w * sm.c[el][tf][l][c];
          }
        for (int c = 0; c < 4; ++c) sm.s[el][i][c] = acc[c];
      }
    } else if (ph == 4) {
      for (int it = tid; it < EPB * Np; it += NT) {
        const int el = it / Np, i = it % Np;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t base = e * Np + i;
        float r0[4];
        load_residual(a, base, Np, r0);
        const float* gp = a.geo + e * 10 * Np + i;
        float G[3][3];
        for (int r = 0; r < 3; ++r)
          for (int d = 0; d < 3; ++d) G[r][d] = gp[(3 * r + d) * Np];
        float Dp[3] = {0.f, 0.f, 0.f}, volp = 0.f;
        for (int j = 0; j < Np; ++j) {
          const float pj = sm.u[0][el][j];
          for (int r = 0; r < 3; ++r) {
            Dp[r] += Dop(o, a, r, i, j) * pj;
            volp += Dop(o, a, r, j, i) * sm.ur[r][el][j];
          }
        }
        const float iJ = 1.0f / sm.J[el][i];
        const float kap = sm.mat[el][0], irho = sm.mat[el][1];
        float rhs[4];
        rhs[0] = kap * iJ * (volp + sm.s[el][i][0]);
        for (int d = 0; d < 3; ++d)
          rhs[1 + d] = irho * (-(G[0][d] * Dp[0] + G[1][d] * Dp[1] + G[2][d] * Dp[2]) + iJ * sm.s[el][i][1 + d]);
        node_update(a, e, Np, base, rhs, r0, &sm.u[0][el][i], &sm.un[0][el][i], EPB * Np);
      }
    } else if (ph == 5) {
      // base-face traces at canonical points; triangle-face lattice values
      const float(*src)[EPB][Np] = (a.mode == kModeTrace) ? sm.u : sm.un;
      for (int it = tid; it < EPB * Nfq; it += NT) {
        const int el = it / Nfq, q = it % Nfq;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t slot = a.slot0 + e * 5;
        const int l = o.qperm[sm.ori[el][0]][q];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int j = 0; j < Np; ++j) {
          const float w = o.Fq[l][j];
          for (int c = 0; c < 4; ++c) acc[c] += w * src[c][el][j];
        }
        a.tr_out[slot * TS + q] = make_float4(acc[0], acc[1], acc[2], acc[3]);
      }
      pad_traces(a, a.tr_out, tid, NT, e0, EPB, 5, 0, 1, Nfq, TS);
      for (int it = tid; it < EPB * 4 * Nfn; it += NT) {
        const int el = it / (4 * Nfn), rr = it % (4 * Nfn);
        const int tf = rr / Nfn, l = rr % Nfn;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int j = 0; j < Np; ++j) {
          const float w = o.Ft[tf][l][j];
          for (int c = 0; c < 4; ++c) acc[c] += w * src[c][el][j];
        }
        for (int c = 0; c < 4; ++c) sm.c[el][tf][l][c] = acc[c];
      }
    } else if (ph == 6 && a.lat) {
      // lattice traces: the face-lattice values in the canonical order,
      // padded with zeros to whole lines
      for (int it = tid; it < EPB * 4 * LW; it += NT) {
        const int el = it / (4 * LW), rr = it % (4 * LW);
        const int tf = rr / LW, m = rr % LW;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t slot = a.slot0 + e * 5 + 1 + tf;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (m < Nfn) {
          const int l = o.tperm[sm.ori[el][1 + tf]][m];
          v = make_float4(sm.c[el][tf][l][0], sm.c[el][tf][l][1], sm.c[el][tf][l][2], sm.c[el][tf][l][3]);
        }
        a.tr_out[slot * TS + m] = v;
      }
    } else if (ph == 6) {
      for (int it = tid; it < EPB * 4 * Nfq; it += NT) {
        const int el = it / (4 * Nfq), rr = it % (4 * Nfq);
        const int tf = rr / Nfq, q = rr % Nfq;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t slot = a.slot0 + e * 5 + 1 + tf;
        const int ori = sm.ori[el][1 + tf];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int m = 0; m < Nfn; ++m) {
          const float w = o.Ican[q][m];
          const int l = o.tperm[ori][m];
          for (int c = 0; c < 4; ++c) acc[c] += w * sm.c[el][tf][l][c];
        }
        a.tr_out[slot * TS + q] = make_float4(acc[0], acc[1], acc[2], acc[3]);
      }
      pad_traces(a, a.tr_out, tid, NT, e0, EPB, 5, 1, 4, Nfq, TS);
    }
  }
};

}  // namespace hdg
