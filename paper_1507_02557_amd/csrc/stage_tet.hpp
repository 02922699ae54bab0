// Fused stage kernel body for nodal tetrahedra (Section 2.3.2, Algorithm 4;
// strong form with constant geometric factors per element).
//
// Volume:  rhs_p = -kappa sum_r D^r (G_r . u),  rhs_u = -(1/rho) G^T (D^r p)
// Surface: canonical-point fluxes are projected onto the face's equispaced
//          lattice nodes (Ican^T), permuted from the canonical to the local
//          face frame, gathered onto element nodes and multiplied by
//          Mhat^{-1} / J.  This equals V_f^T W J^s applied to the flux because
//          the trace of a degree-N polynomial on a face depends only on its
//          face-node values and the lattice is invariant under the face's
//          vertex permutations.
// Traces:  the same lattice -> cubature interpolation Ican applied to the
//          face-node values of the updated state.
#pragma once

#include "stage_common.hpp"

namespace hdg {

template <int N, int EPB>
struct TetStage {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfn = (N + 1) * (N + 2) / 2;
  static constexpr int Nfq = (N + 1) * (N + 1);
  static constexpr int TS = trace_stride(N);
  static constexpr int NT = 256;
  static constexpr int kEPB = EPB;
  static constexpr int nphase = 6;
  static constexpr int kTraceBegin = 5;  // first phase that writes traces
  // packed table sizes
  static constexpr int kOpsFloats = 4 * Np * Np + Nfq * Nfn + Nfq;
  static constexpr int kOpsInts = 4 * Nfn + 6 * Nfn + 4 * Np;

  struct Smem {
    float D[3][Np][Np];
    float Minv[Np][Np];
    float Ican[Nfq][Nfn];
    float w[Nfq];
    int fnode[4][Nfn];
    int tperm[6][Nfn];
    int nodeface[4][Np];
    float u[4][EPB][Np];
    float un[4][EPB][Np];
    float ut[3][EPB][Np];
    float g[EPB][4][Nfq][4];
    float c[EPB][4][Nfn][4];
    float s[EPB][Np][4];
    float geo[EPB][12];
  };

  HD static bool active(int ph, int mode) {
    if (mode == kModeTrace) return ph == 0 || ph == 5;
    if (mode == kModeRhs || mode == kModeRhsHist) return ph <= 4;
    return true;
  }

  HD static Smem& batch(Smem& sm) { return sm; }

  HD static void load_ops(int tid, Smem& sm, const StageArgs& a) {
    float* D = &sm.D[0][0][0];
    for (int i = tid; i < 3 * Np * Np; i += NT) D[i] = a.ops[i];
    float* Mi = &sm.Minv[0][0];
    for (int i = tid; i < Np * Np; i += NT) Mi[i] = a.ops[3 * Np * Np + i];
    float* Ic = &sm.Ican[0][0];
    for (int i = tid; i < Nfq * Nfn; i += NT) Ic[i] = a.ops[4 * Np * Np + i];
    for (int i = tid; i < Nfq; i += NT) sm.w[i] = a.ops[4 * Np * Np + Nfq * Nfn + i];
    int* fn = &sm.fnode[0][0];
    for (int i = tid; i < 4 * Nfn; i += NT) fn[i] = a.iops[i];
    int* tp = &sm.tperm[0][0];
    for (int i = tid; i < 6 * Nfn; i += NT) tp[i] = a.iops[4 * Nfn + i];
    int* nf = &sm.nodeface[0][0];
    for (int i = tid; i < 4 * Np; i += NT) nf[i] = a.iops[10 * Nfn + i];
  }

  HD static void phase(int ph, int tid, Smem& sm, const StageArgs& a, int64_t e0) {
    const int64_t K = a.K;
    if (ph == 0) {
      for (int it = tid; it < 4 * EPB * Np; it += NT) {
        const int f = it / (EPB * Np), r = it % (EPB * Np);
        const int el = r / Np, i = r % Np;
        const int64_t e = item(a, e0 + el);
        (&sm.u[0][0][0])[it] = (e >= 0) ? a.U[(int64_t)f * K * Np + e * Np + i] : 0.0f;
      }
      for (int it = tid; it < EPB * 12; it += NT) {
        const int el = it / 12, c = it % 12;
        const int64_t e = item(a, e0 + el);
        float v = 0.0f;
        if (e >= 0) v = (c < 10) ? a.geo[e * 12 + c] : (c == 10 ? a.mat[e].x : a.mat[e].y);
        sm.geo[el][c] = v;
      }
    } else if (ph == 1) {
      for (int it = tid; it < EPB * Np; it += NT) {
        const int el = it / Np, i = it % Np;
        for (int r = 0; r < 3; ++r)
          sm.ut[r][el][i] = sm.geo[el][3 * r] * sm.u[1][el][i] + sm.geo[el][3 * r + 1] * sm.u[2][el][i] +
                            sm.geo[el][3 * r + 2] * sm.u[3][el][i];
      }
      for (int it = tid; it < EPB * 4 * Nfq; it += NT) {
        const int el = it / (4 * Nfq), rr = it % (4 * Nfq);
        const int f = rr / Nfq, q = rr % Nfq;
        const int64_t e = item(a, e0 + el);
        float out[4] = {0.f, 0.f, 0.f, 0.f};
        if (e >= 0) {
          const int64_t slot = a.slot0 + e * 4 + f;
          float4 g = a.fgeo[e * 4 + f];
          g.w *= sm.w[q];
          float4 m, p;
          face_states(a, slot, TS, q, g, m, p);
          upwind_flux(m, p, g, a.tau[slot], false, out);
        }
        for (int c = 0; c < 4; ++c) sm.g[el][f][q][c] = out[c];
      }
    } else if (ph == 2) {
      for (int it = tid; it < EPB * 4 * Nfn; it += NT) {
        const int el = it / (4 * Nfn), rr = it % (4 * Nfn);
        const int f = rr / Nfn, m = rr % Nfn;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int o = a.ori[a.slot0 + e * 4 + f];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int q = 0; q < Nfq; ++q) {
          const float w = sm.Ican[q][m];
          for (int c = 0; c < 4; ++c) acc[c] += w * sm.g[el][f][q][c];
        }
        const int l = sm.tperm[o][m];
        for (int c = 0; c < 4; ++c) sm.c[el][f][l][c] = acc[c];
      }
    } else if (ph == 3) {
      for (int it = tid; it < EPB * Np; it += NT) {
        const int el = it / Np, i = it % Np;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int f = 0; f < 4; ++f) {
          const int l = sm.nodeface[f][i];
          if (l >= 0)
            for (int c = 0; c < 4; ++c) acc[c] += sm.c[el][f][l][c];
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
        float dp[3] = {0.f, 0.f, 0.f}, div = 0.f, lift[4] = {0.f, 0.f, 0.f, 0.f};
        for (int j = 0; j < Np; ++j) {
          const float pj = sm.u[0][el][j];
          for (int r = 0; r < 3; ++r) {
            const float d = sm.D[r][i][j];
            dp[r] += d * pj;
            div += d * sm.ut[r][el][j];
          }
          const float mi = sm.Minv[i][j];
          for (int c = 0; c < 4; ++c) lift[c] += mi * sm.s[el][j][c];
        }
        const float* G = sm.geo[el];
        const float iJ = G[9], kap = G[10], irho = G[11];
        float rhs[4];
        rhs[0] = kap * (-div + iJ * lift[0]);
        for (int d = 0; d < 3; ++d)
          rhs[1 + d] = irho * (-(G[d] * dp[0] + G[3 + d] * dp[1] + G[6 + d] * dp[2]) + iJ * lift[1 + d]);
        node_update(a, e, Np, base, rhs, r0, &sm.u[0][el][i], &sm.un[0][el][i], EPB * Np);
      }
    } else if (ph == 5) {
      const float(*src)[EPB][Np] = (a.mode == kModeTrace) ? sm.u : sm.un;
      for (int it = tid; it < EPB * 4 * Nfq; it += NT) {
        const int el = it / (4 * Nfq), rr = it % (4 * Nfq);
        const int f = rr / Nfq, q = rr % Nfq;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t slot = a.slot0 + e * 4 + f;
        const int o = a.ori[slot];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int m = 0; m < Nfn; ++m) {
          const float w = sm.Ican[q][m];
          const int node = sm.fnode[f][sm.tperm[o][m]];
          for (int c = 0; c < 4; ++c) acc[c] += w * src[c][el][node];
        }
        a.tr_out[slot * TS + q] = make_float4(acc[0], acc[1], acc[2], acc[3]);
      }
      pad_traces(a, a.tr_out, tid, NT, e0, EPB, 4, 0, 4, Nfq, TS);
    }
  }
};

}  // namespace hdg
