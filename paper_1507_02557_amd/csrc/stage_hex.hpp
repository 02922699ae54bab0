// Fused stage kernel body for GL nodal hexahedra (Section 2.3.1,
// Algorithms 1-3; strong form, collocated mass diag(w J)).
//
// Volume:  reference derivatives by 1D contractions with D_ij = l_j'(x_i)
//          along each tensor line, chain rule with G = d(r,s,t)/dx per node.
// Surface: node (i,j,k) receives l_i(-1) w J^s flux on face r = -1 at local
//          face point (j,k), and likewise for the other five faces; the
//          inverse mass 1/(w_ijk J_ijk) is applied per node.
// Traces:  u(+-1, s_j, t_k) = sum_m l_m(+-1) u_mjk (Algorithm 2) at the local
//          face point that the canonical point maps to under the face's
//          orientation (a permutation of the GL tensor grid).  The element's
//          own trace is recomputed from the state rather than read back, so
//          only the neighbour's trace is read.
#pragma once

#include "stage_common.hpp"

namespace hdg {

template <int N, int EPB>
struct HexStage {
  static constexpr int n1 = N + 1;
  static constexpr int Np = n1 * n1 * n1;
  static constexpr int Nfq = n1 * n1;
  static constexpr int TS = trace_stride(N);
  static constexpr int NT = 256;
  static constexpr int kEPB = EPB;
  static constexpr int nphase = 4;
  static constexpr int kTraceBegin = 3;  // first phase that writes traces
  static constexpr int kOpsFloats = n1 * n1 + 2 * n1;
  static constexpr int kOpsInts = 8 * Nfq;

  struct Smem {
    float D1[n1][n1];
    float Lf[2][n1];  // l_m(-1), l_m(+1)
    int qperm[8][Nfq];
    float u[4][EPB][Np];
    float un[4][EPB][Np];
    float g[EPB][6][Nfq][4];
    float mat[EPB][2];
  };

  HD static bool active(int ph, int mode) {
    if (mode == kModeTrace) return ph == 0 || ph == 3;
    if (mode == kModeRhs || mode == kModeRhsHist) return ph <= 2;
    return true;
  }

  HD static Smem& batch(Smem& sm) { return sm; }

  HD static void load_ops(int tid, Smem& sm, const StageArgs& a) {
    for (int i = tid; i < n1 * n1; i += NT) (&sm.D1[0][0])[i] = a.ops[i];
    for (int i = tid; i < 2 * n1; i += NT) (&sm.Lf[0][0])[i] = a.ops[n1 * n1 + i];
    for (int i = tid; i < 8 * Nfq; i += NT) (&sm.qperm[0][0])[i] = a.iops[i];
  }

  // element node index of the m-th node on the line normal to face f through
  // local face point (l1, l2)
  HD static int line_node(int f, int m, int l1, int l2) {
    if (f < 2) return m + n1 * (l1 + n1 * l2);
    if (f < 4) return l1 + n1 * (m + n1 * l2);
    return l1 + n1 * (l2 + n1 * m);
  }

  HD static void phase(int ph, int tid, Smem& sm, const StageArgs& a, int64_t e0) {
    const int64_t K = a.K;
    // Global loads of a phase are issued together, from indices clamped to
    // an element of the batch (item e0 always exists), and used after.
    const int64_t e_any = item(a, e0);
    if (ph == 0) {
      constexpr int NL = 4 * EPB * Np, RL = (NL + NT - 1) / NT;
      float v[RL];
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int it = tid + r * NT;
        const int itc = it < NL ? it : 0;
        const int f = itc / (EPB * Np), rr = itc % (EPB * Np);
        const int el = rr / Np, i = rr % Np;
        const int64_t e = item(a, e0 + el);
        v[r] = a.U[(int64_t)f * K * Np + (e >= 0 ? e : e_any) * Np + i];
        if (e < 0) v[r] = 0.f;
      }
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int it = tid + r * NT;
        if (it < NL) (&sm.u[0][0][0])[it] = v[r];
      }
      for (int it = tid; it < EPB; it += NT) {
        const int64_t e = item(a, e0 + it);
        sm.mat[it][0] = e >= 0 ? a.mat[e].x : 0.f;
        sm.mat[it][1] = e >= 0 ? a.mat[e].y : 0.f;
      }
    } else if (ph == 1) {
      constexpr int NF = EPB * 6 * Nfq, RF = (NF + NT - 1) / NT;
      float4 fg[RF], fp[RF];
      float2 ftau[RF];
      int fo[RF], fnb[RF];
#pragma unroll
      for (int r = 0; r < RF; ++r) {
        const int it = tid + r * NT;
        const int itc = it < NF ? it : 0;
        const int el = itc / (6 * Nfq), rr = itc % (6 * Nfq);
        const int f = rr / Nfq, q = rr % Nfq;
        const int64_t e0v = item(a, e0 + el);
        const int64_t e = e0v >= 0 ? e0v : e_any;
        const int64_t slot = a.slot0 + e * 6 + f;
        fg[r] = a.fgeo[(e * 6 + f) * Nfq + q];
        fo[r] = a.ori[slot];
        fnb[r] = a.nbr[slot];
        ftau[r] = a.tau[slot];
      }
#pragma unroll
      for (int r = 0; r < RF; ++r) {
        const int it = tid + r * NT;
        const int itc = it < NF ? it : 0;
        const int el = itc / (6 * Nfq), rr = itc % (6 * Nfq);
        const int f = rr / Nfq, q = rr % Nfq;
        const int64_t e0v = item(a, e0 + el);
        const int64_t e = e0v >= 0 ? e0v : e_any;
        const int64_t slot = a.slot0 + e * 6 + f;
        if (fnb[r] >= 0) fp[r] = neighbour_src(a, slot, fnb[r])[(int64_t)fnb[r] * TS + q];
      }
#pragma unroll
      for (int r = 0; r < RF; ++r) {
        const int it = tid + r * NT;
        if (it >= NF) continue;
        const int el = it / (6 * Nfq), rr = it % (6 * Nfq);
        const int f = rr / Nfq, q = rr % Nfq;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const float4 g = fg[r];
        const int l = sm.qperm[fo[r]][q];
        // own trace recomputed from the state (Algorithm 2), not read back
        const int l1 = l % n1, l2 = l / n1;
        const float* L = sm.Lf[f & 1];
        float mv[4] = {0.f, 0.f, 0.f, 0.f};
        for (int k = 0; k < n1; ++k) {
          const int nd = line_node(f, k, l1, l2);
          for (int c = 0; c < 4; ++c) mv[c] += L[k] * sm.u[c][el][nd];
        }
        const float4 m = make_float4(mv[0], mv[1], mv[2], mv[3]);
        const int nb = fnb[r];
        const float4 p = nb >= 0 ? fp[r] : mirror_state(m, -nb - 1, g.x, g.y, g.z);
        float out[4];
        upwind_flux(m, p, g, ftau[r], false, out);
        for (int c = 0; c < 4; ++c) sm.g[el][f][l][c] = out[c];
      }
    } else if (ph == 2) {
      constexpr int NN = EPB * Np, RN = (NN + NT - 1) / NT;
      float rq[RN][4], gq[RN][10];
#pragma unroll
      for (int r = 0; r < RN; ++r) {
        const int it = tid + r * NT;
        const int itc = it < NN ? it : 0;
        const int64_t e = item(a, e0 + itc / Np);
        const int64_t es = e >= 0 ? e : e_any;
        load_residual(a, es * Np + itc % Np, Np, rq[r]);
        const float* gp = a.geo + es * 10 * Np + itc % Np;
#pragma unroll
        for (int k = 0; k < 10; ++k) gq[r][k] = gp[k * Np];
      }
#pragma unroll
      for (int r = 0; r < RN; ++r) {
        const int it = tid + r * NT;
        if (it >= NN) continue;
        const int el = it / Np, node = it % Np;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t base = e * Np + node;
        const int i = node % n1, j = (node / n1) % n1, k = node / (n1 * n1);
        float du[4][3];
        for (int c = 0; c < 4; ++c) {
          float dr = 0.f, ds = 0.f, dt = 0.f;
          for (int m = 0; m < n1; ++m) {
            dr += sm.D1[i][m] * sm.u[c][el][m + n1 * (j + n1 * k)];
            ds += sm.D1[j][m] * sm.u[c][el][i + n1 * (m + n1 * k)];
            dt += sm.D1[k][m] * sm.u[c][el][i + n1 * (j + n1 * m)];
          }
          du[c][0] = dr;
          du[c][1] = ds;
          du[c][2] = dt;
        }
        float G[3][3];
        for (int x = 0; x < 3; ++x)
          for (int d = 0; d < 3; ++d) G[x][d] = gq[r][3 * x + d];
        const float iwJ = gq[r][9];
        float div = 0.f;
        for (int x = 0; x < 3; ++x)
          for (int d = 0; d < 3; ++d) div += G[x][d] * du[1 + d][x];
        float surf[4];
        for (int c = 0; c < 4; ++c)
          surf[c] = sm.Lf[0][i] * sm.g[el][0][k * n1 + j][c] + sm.Lf[1][i] * sm.g[el][1][k * n1 + j][c] +
                    sm.Lf[0][j] * sm.g[el][2][k * n1 + i][c] + sm.Lf[1][j] * sm.g[el][3][k * n1 + i][c] +
                    sm.Lf[0][k] * sm.g[el][4][j * n1 + i][c] + sm.Lf[1][k] * sm.g[el][5][j * n1 + i][c];
        const float kap = sm.mat[el][0], irho = sm.mat[el][1];
        float rhs[4];
        rhs[0] = kap * (-div + iwJ * surf[0]);
        for (int d = 0; d < 3; ++d)
          rhs[1 + d] = irho * (-(G[0][d] * du[0][0] + G[1][d] * du[0][1] + G[2][d] * du[0][2]) + iwJ * surf[1 + d]);
        node_update(a, e, Np, base, rhs, rq[r], &sm.u[0][el][node], &sm.un[0][el][node], EPB * Np);
      }
    } else if (ph == 3) {
      const float(*src)[EPB][Np] = (a.mode == kModeTrace) ? sm.u : sm.un;
      constexpr int NF = EPB * 6 * Nfq, RF = (NF + NT - 1) / NT;
      int fo[RF];
#pragma unroll
      for (int r = 0; r < RF; ++r) {
        const int it = tid + r * NT;
        const int itc = it < NF ? it : 0;
        const int64_t e = item(a, e0 + itc / (6 * Nfq));
        fo[r] = a.ori[a.slot0 + (e >= 0 ? e : e_any) * 6 + (itc % (6 * Nfq)) / Nfq];
      }
#pragma unroll
      for (int r = 0; r < RF; ++r) {
        const int it = tid + r * NT;
        if (it >= NF) continue;
        const int el = it / (6 * Nfq), rr = it % (6 * Nfq);
        const int f = rr / Nfq, q = rr % Nfq;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t slot = a.slot0 + e * 6 + f;
        const int l = sm.qperm[fo[r]][q];
        const int l1 = l % n1, l2 = l / n1;
        const float* L = sm.Lf[f & 1];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int m = 0; m < n1; ++m) {
          const int nd = line_node(f, m, l1, l2);
          for (int c = 0; c < 4; ++c) acc[c] += L[m] * src[c][el][nd];
        }
        a.tr_out[slot * TS + q] = make_float4(acc[0], acc[1], acc[2], acc[3]);
      }
      pad_traces(a, a.tr_out, tid, NT, e0, EPB, 6, 0, 6, Nfq, TS);
    }
  }
};

}  // namespace hdg
