// Fused stage kernel body for LSC-DG wedges (Sections 2.1.3 and 2.3.3,
// Algorithms 5-6: skew-symmetric form, basis phi/sqrt(J), mass = I).
//
// The basis is a tensor product phi_{js,jt} = phi^tri_jt(r,t) phi^1D_js(s),
// and so is the cubature (triangle rule x GL in s), so every evaluation and
// every test integral is done by sum factorisation: contract the 1D index
// first, then the triangle index.  The trial integrand at cubature point q is
//   B_r = w_q (G U)_r,  B_h = w_q (grad J / 2J) . U,
//   C_d = w_q (sum_r G_rd d_r P - P (grad J / 2J)_d),
// with P, U the polynomial parts sum_j u_j phi_j, and the test integrals are
//   rhs_p,i   = kappa (sum_q grad_rst phi_i . B - phi_i B_h + surface),
//   rhs_u_d,i = (1/rho) (-sum_q phi_i C_d + surface).
// The intermediate values stay in LDS (the paper writes them to global
// memory between two kernels).
#pragma once

#include "stage_common.hpp"

namespace hdg {

template <int N, int EPB, int NTH = 256>
struct WedgeStage {
  static constexpr int n1 = N + 1;
  static constexpr int Ntri = (N + 1) * (N + 2) / 2;
  static constexpr int Np = n1 * Ntri;
  static constexpr int Nct = n1 * n1;
  static constexpr int Nq = n1 * Nct;
  static constexpr int Nfq = n1 * n1;
  static constexpr int TS = trace_stride(N);
  static constexpr int Nfn = Ntri;
  static constexpr int NT = NTH;
  static constexpr int kEPB = EPB;
  static constexpr int nphase = 6;
  static constexpr int kTraceBegin = 3;  // first phase that writes traces
  // ops: (Pt, Ptr, Ptt, 0) [Nct][Ntri][4]; tri_w [Nct]; P1, dP1 [n1][n1]; w1 [n1];
  //      P1f [2][n1]; Ftri [Nfn][Ntri]; Fedge [3][n1][Ntri]; Ican [Nfq][Nfn]
  static constexpr int oP3 = 0, oTw = oP3 + 4 * Nct * Ntri;
  static constexpr int oP1 = oTw + Nct, odP1 = oP1 + n1 * n1, ow1 = odP1 + n1 * n1, oP1f = ow1 + n1;
  static constexpr int oFt = oP1f + 2 * n1, oFe = oFt + Nfn * Ntri, oIc = oFe + 3 * n1 * Ntri;
  static constexpr int kOpsFloats = oIc + Nfq * Nfn;
  static constexpr int kOpsInts = 8 * Nfq + 6 * Nfn;

  // operator tables (shared by all batches of a block) and one batch's data
  struct Ops {
    float ops[kOpsFloats];
    int qperm[8][Nfq];
    int tperm[6][Nfn];
  };
  struct Batch {
    float u[4][EPB][Np];
    // buffers whose lifetimes do not overlap share storage (phase parts in
    // brackets write / read them: 0 loads and face fluxes, 1a s-contraction,
    // 1b volume values, 2a test contractions, 2b node update, 3-5 traces):
    union {
      float A[5][EPB][n1][Ntri];  // s-contracted state [1a] / [1b]
      float T[5][EPB][n1][Ntri];  // test contractions with the quad faces folded in [2a] / [2b]
    };
    union {
      alignas(16) float B[EPB][Nq][8];  // trial integrands at the volume points (7 used) [1b] / [2a]
      float W[EPB][3][n1][n1][4];       // quad-face trace operands [3] / [4]
    };
    union {
      float g[EPB][5][Nfq][4];  // weighted face fluxes [0] / [1b, 2a]
      float un[4][EPB][Np];     // updated state [2b] / [3, 4, 5]
    };
    float c[EPB][2][Nfn][4];
    float z[EPB][2][Ntri][4];   // triangle-face operands [2a, 3] / [2b, 4]
    float mat[EPB][2];
    float isj[EPB][5][Nfq];  // 1/sqrt(J) at the face points [0] / [0, 4, 5]
    int fori[EPB][5];        // face orientation codes [0] / [0, 4, 5]
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
  // barrier between the two parts of a phase: the block's, or the
  // wavefront's when one wavefront runs the batch
  HD static void batch_sync() {
    if constexpr (NT == 64) wave_sync();
    else __syncthreads();
  }

  HD static bool active(int ph, int mode) {
    if (mode == kModeTrace) return ph == 0 || ph >= kTraceBegin;
    if (mode == kModeRhs || mode == kModeRhsHist) return ph < kTraceBegin;
    return true;
  }

  // tables into LDS by nthr threads
  HD static void load_ops(int tid, int nthr, Ops& o, const StageArgs& a) {
    for (int i = tid; i < kOpsFloats; i += nthr) o.ops[i] = a.ops[i];
    for (int i = tid; i < 8 * Nfq; i += nthr) (&o.qperm[0][0])[i] = a.iops[i];
    for (int i = tid; i < 6 * Nfn; i += nthr) (&o.tperm[0][0])[i] = a.iops[8 * Nfq + i];
  }
  HD static void load_ops(int tid, Smem& sm, const StageArgs& a) { load_ops(tid, NT, sm.o, a); }

  HD static void phase(int ph, int tid, Smem& sm, const StageArgs& a, int64_t e0) { phase(ph, tid, sm.o, sm.b, a, e0); }
  HD static void phase(int ph, int tid, WaveRef& r, const StageArgs& a, int64_t e0) { phase(ph, tid, r.o, r.b, a, e0); }

  HD static void phase(int ph, int tid, const Ops& op, Batch& sm, const StageArgs& a, int64_t e0) {
    const int64_t K = a.K;
    const float* O = op.ops;
    // triangle basis and its r, t derivatives at the triangle points, read as one vector
    const float4* P3 = reinterpret_cast<const float4*>(O + oP3);
    const float* Tw = O + oTw;
    const float* P1 = O + oP1;
    const float* dP1 = O + odP1;
    const float* w1 = O + ow1;
    const float* P1f = O + oP1f;
    const float* Ft = O + oFt;
    const float* Fe = O + oFe;
    const float* Ic = O + oIc;
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
      // faces: the own trace comes from the trace buffer, so the flux needs no
      // state and its loads are in flight together with the state loads
      const bool flux = a.mode != kModeTrace;
      constexpr int NF = EPB * 5 * Nfq, RF = (NF + NT - 1) / NT;
      float4 fg[RF], fm[RF], fp[RF];
      float fisj[RF];
      float2 ftau[RF];
      int fo[RF], fdst[RF];
#pragma unroll
      for (int r = 0; r < RF; ++r) {
        const int it = tid + r * NT;
        const int itc = it < NF ? it : 0;
        const int el = itc / (5 * Nfq), rr = itc % (5 * Nfq);
        const int f = rr / Nfq, q = rr % Nfq;
        const int64_t e0v = item(a, e0 + el);
        const int64_t e = e0v >= 0 ? e0v : e_any;
        const int64_t slot = a.slot0 + e * 5 + f;
        fisj[r] = a.isqJ[(e * 5 + f) * Nfq + q];
        fo[r] = a.ori[slot];
        fdst[r] = (it < NF && e0v >= 0) ? el * 5 + f : -1;
        if (!flux) continue;
        fg[r] = a.fgeo[(e * 5 + f) * Nfq + q];
        face_states(a, slot, TS, q, fg[r], fm[r], fp[r]);
        ftau[r] = a.tau[slot];
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
#pragma unroll
      for (int r = 0; r < RF; ++r) {
        if (fdst[r] < 0) continue;
        const int el = fdst[r] / 5, f = fdst[r] % 5, q = (tid + r * NT) % Nfq;
        sm.isj[el][f][q] = fisj[r];
        if (q == 0) sm.fori[el][f] = fo[r];
        if (!flux) continue;
        float out[4];
        upwind_flux(fm[r], fp[r], fg[r], ftau[r], true, out);
        const int l = (f < 2) ? q : op.qperm[fo[r]][q];
        float* gd = sm.g[el][f][l];
        for (int c = 0; c < 4; ++c) gd[c] = out[c] * fisj[r];
      }
    } else if (ph == 1) {
      // geometric factors in flight during the s-contraction
      constexpr int NB = EPB * Nq, RB = (NB + NT - 1) / NT;
      float gq[RB][12];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int it = tid + r * NT;
        const int itc = it < NB ? it : 0;
        const int64_t e = item(a, e0 + itc / Nq);
        const float* gp = a.geo + (e >= 0 ? e : e_any) * 12 * Nq + itc % Nq;
#pragma unroll
        for (int k = 0; k < 12; ++k) gq[r][k] = gp[k * Nq];
      }
      for (int it = tid; it < EPB * 5 * n1 * Ntri; it += NT) {
        const int el = it / (5 * n1 * Ntri), rr = it % (5 * n1 * Ntri);
        const int c = rr / (n1 * Ntri), r2 = rr % (n1 * Ntri);
        const int qs = r2 / Ntri, jt = r2 % Ntri;
        const float* op = (c < 4) ? P1 : dP1;
        const int src = (c < 4) ? c : 0;
        float acc = 0.f;
        for (int js = 0; js < n1; ++js) acc += op[qs * n1 + js] * sm.u[src][el][js * Ntri + jt];
        sm.A[c][el][qs][jt] = acc;
      }
      // the rest of the phase reads what the first part wrote: one barrier
      // (every thread of the block runs every phase)
      batch_sync();
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int it = tid + r * NT;
        if (it >= NB) continue;
        const int el = it / Nq, q = it % Nq;
        const int qs = q / Nct, qt = q % Nct;
        const int64_t e = item(a, e0 + el);
        float4* bd = reinterpret_cast<float4*>(sm.B[el][q]);
        if (e < 0) {
          bd[0] = bd[1] = make_float4(0.f, 0.f, 0.f, 0.f);
          continue;
        }
        float P = 0.f, dPr = 0.f, dPt = 0.f, dPs = 0.f, U[3] = {0.f, 0.f, 0.f};
        for (int jt = 0; jt < Ntri; ++jt) {
          const float4 pv = P3[qt * Ntri + jt];
          const float pt = pv.x;
          const float a0 = sm.A[0][el][qs][jt];
          P += pt * a0;
          dPr += pv.y * a0;
          dPt += pv.z * a0;
          dPs += pt * sm.A[4][el][qs][jt];
          for (int d = 0; d < 3; ++d) U[d] += pt * sm.A[1 + d][el][qs][jt];
        }
        float G[3][3], hJ[3];
        for (int i = 0; i < 3; ++i)
          for (int d = 0; d < 3; ++d) G[i][d] = gq[r][3 * i + d];
        for (int d = 0; d < 3; ++d) hJ[d] = gq[r][9 + d];
        const float w = Tw[qt] * w1[qs];
        const float dP[3] = {dPr, dPs, dPt};
        float Bv[7];
        for (int i = 0; i < 3; ++i) Bv[i] = w * (G[i][0] * U[0] + G[i][1] * U[1] + G[i][2] * U[2]);
        Bv[3] = w * (hJ[0] * U[0] + hJ[1] * U[1] + hJ[2] * U[2]);
        for (int d = 0; d < 3; ++d) Bv[4 + d] = w * (G[0][d] * dP[0] + G[1][d] * dP[1] + G[2][d] * dP[2] - P * hJ[d]);
        bd[0] = make_float4(Bv[0], Bv[1], Bv[2], Bv[3]);
        bd[1] = make_float4(Bv[4], Bv[5], Bv[6], 0.f);
      }
      for (int it = tid; it < EPB * 2 * Nfn; it += NT) {
        const int el = it / (2 * Nfn), rr = it % (2 * Nfn);
        const int tf = rr / Nfn, m = rr % Nfn;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int o = sm.fori[el][tf];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int q = 0; q < Nfq; ++q) {
          const float w = Ic[q * Nfn + m];
          for (int c = 0; c < 4; ++c) acc[c] += w * sm.g[el][tf][q][c];
        }
        const int l = op.tperm[o][m];
        for (int c = 0; c < 4; ++c) sm.c[el][tf][l][c] = acc[c];
      }
    } else if (ph == 2) {
      // residual in flight during the test contractions
      constexpr int NN = EPB * Np, RN = (NN + NT - 1) / NT;
      float rq[RN][4];
#pragma unroll
      for (int r = 0; r < RN; ++r) {
        const int it = tid + r * NT;
        const int itc = it < NN ? it : 0;
        const int64_t e = item(a, e0 + itc / Np);
        load_residual(a, (e >= 0 ? e : e_any) * Np + itc % Np, Np, rq[r]);
      }
      for (int it = tid; it < EPB * n1 * Ntri; it += NT) {
        const int el = it / (n1 * Ntri), rr = it % (n1 * Ntri);
        const int qs = rr / Ntri, jt = rr % Ntri;
        float t0 = 0.f, t1 = 0.f, t2 = 0.f, t3 = 0.f, t4 = 0.f;
#pragma unroll 5
        for (int qt = 0; qt < Nct; ++qt) {
          const int q = qs * Nct + qt;
          const float4 pv = P3[qt * Ntri + jt];
          const float4* bs = reinterpret_cast<const float4*>(sm.B[el][q]);
          const float4 b0 = bs[0], b1 = bs[1];
          t0 += pv.y * b0.x + pv.z * b0.z - pv.x * b0.w;
          t1 += pv.x * b0.y;
          t2 += pv.x * b1.x;
          t3 += pv.x * b1.y;
          t4 += pv.x * b1.z;
        }
        // quad faces: their s points are the volume points qs, so their test
        // integrals share the final s-contraction with the volume terms
        for (int ef = 0; ef < 3; ++ef)
          for (int l1 = 0; l1 < n1; ++l1) {
            const float w = Fe[(ef * n1 + l1) * Ntri + jt];
            const float* gq = sm.g[el][2 + ef][qs * n1 + l1];
            t0 += w * gq[0];
            t2 -= w * gq[1];
            t3 -= w * gq[2];
            t4 -= w * gq[3];
          }
        sm.T[0][el][qs][jt] = t0;
        sm.T[1][el][qs][jt] = t1;
        sm.T[2][el][qs][jt] = t2;
        sm.T[3][el][qs][jt] = t3;
        sm.T[4][el][qs][jt] = t4;
      }
      // triangle faces: z[tf][jt] = sum_l Ft[l][jt] c[tf][l]
      for (int it = tid; it < EPB * 2 * Ntri; it += NT) {
        const int el = it / (2 * Ntri), rr = it % (2 * Ntri);
        const int tf = rr / Ntri, jt = rr % Ntri;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int l = 0; l < Nfn; ++l) {
          const float w = Ft[l * Ntri + jt];
          for (int c = 0; c < 4; ++c) acc[c] += w * sm.c[el][tf][l][c];
        }
        for (int c = 0; c < 4; ++c) sm.z[el][tf][jt][c] = acc[c];
      }
      // the rest of the phase reads what the first part wrote: one barrier
      // (every thread of the block runs every phase)
      batch_sync();
#pragma unroll
      for (int r = 0; r < RN; ++r) {
        const int it = tid + r * NT;
        if (it >= NN) continue;
        const int el = it / Np, m = it % Np;
        const int js = m / Ntri, jt = m % Ntri;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t base = e * Np + m;
        float vp = 0.f, vu[3] = {0.f, 0.f, 0.f};
        for (int qs = 0; qs < n1; ++qs) {
          const float p1 = P1[qs * n1 + js];
          vp += p1 * sm.T[0][el][qs][jt] + dP1[qs * n1 + js] * sm.T[1][el][qs][jt];
          for (int d = 0; d < 3; ++d) vu[d] -= p1 * sm.T[2 + d][el][qs][jt];
        }
        // triangle faces: sum_tf P1f[tf][js] z[tf][jt]
        float sf[4] = {0.f, 0.f, 0.f, 0.f};
        for (int tf = 0; tf < 2; ++tf) {
          const float w = P1f[tf * n1 + js];
          for (int c = 0; c < 4; ++c) sf[c] += w * sm.z[el][tf][jt][c];
        }
        const float kap = sm.mat[el][0], irho = sm.mat[el][1];
        float rhs[4];
        rhs[0] = kap * (vp + sf[0]);
        for (int d = 0; d < 3; ++d) rhs[1 + d] = irho * (vu[d] + sf[1 + d]);
        node_update(a, e, Np, base, rhs, rq[r], &sm.u[0][el][m], &sm.un[0][el][m], EPB * Np);
      }
    } else if (ph == 3) {
      // s-contractions of the traces: triangle faces z[tf][jt] = sum_js P1f[tf][js] u[js][jt],
      // quad faces W[ef][l1][js] = sum_jt Fe[ef][l1][jt] u[js][jt]
      const float(*src)[EPB][Np] = (a.mode == kModeTrace) ? sm.u : sm.un;
      for (int it = tid; it < EPB * 2 * Ntri; it += NT) {
        const int el = it / (2 * Ntri), rr = it % (2 * Ntri);
        const int tf = rr / Ntri, jt = rr % Ntri;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int js = 0; js < n1; ++js) {
          const float w = P1f[tf * n1 + js];
          for (int c = 0; c < 4; ++c) acc[c] += w * src[c][el][js * Ntri + jt];
        }
        for (int c = 0; c < 4; ++c) sm.z[el][tf][jt][c] = acc[c];
      }
      for (int it = tid; it < EPB * 3 * n1 * n1; it += NT) {
        const int el = it / (3 * n1 * n1), rr = it % (3 * n1 * n1);
        const int ef = rr / (n1 * n1), r2 = rr % (n1 * n1);
        const int l1 = r2 / n1, js = r2 % n1;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int jt = 0; jt < Ntri; ++jt) {
          const float w = Fe[(ef * n1 + l1) * Ntri + jt];
          for (int c = 0; c < 4; ++c) acc[c] += w * src[c][el][js * Ntri + jt];
        }
        for (int c = 0; c < 4; ++c) sm.W[el][ef][l1][js][c] = acc[c];
      }
    } else if (ph == 4) {
      // triangle lattice values c = Ft z; quad traces sum_js P1[l2][js] W[ef][l1][js] / sqrt(J)
      for (int it = tid; it < EPB * 2 * Nfn; it += NT) {
        const int el = it / (2 * Nfn), rr = it % (2 * Nfn);
        const int tf = rr / Nfn, l = rr % Nfn;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int jt = 0; jt < Ntri; ++jt) {
          const float w = Ft[l * Ntri + jt];
          for (int c = 0; c < 4; ++c) acc[c] += w * sm.z[el][tf][jt][c];
        }
        for (int c = 0; c < 4; ++c) sm.c[el][tf][l][c] = acc[c];
      }
      for (int it = tid; it < EPB * 3 * Nfq; it += NT) {
        const int el = it / (3 * Nfq), rr = it % (3 * Nfq);
        const int ef = rr / Nfq, q = rr % Nfq;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int f = 2 + ef;
        const int64_t slot = a.slot0 + e * 5 + f;
        const int l = op.qperm[sm.fori[el][f]][q];
        const int l1 = l % n1, l2 = l / n1;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int js = 0; js < n1; ++js) {
          const float w = P1[l2 * n1 + js];
          for (int c = 0; c < 4; ++c) acc[c] += w * sm.W[el][ef][l1][js][c];
        }
        const float isj = sm.isj[el][f][q];
        a.tr_out[slot * TS + q] = make_float4(acc[0] * isj, acc[1] * isj, acc[2] * isj, acc[3] * isj);
      }
      pad_traces(a, a.tr_out, tid, NT, e0, EPB, 5, 2, 3, Nfq, TS);
    } else if (ph == 5) {
      for (int it = tid; it < EPB * 2 * Nfq; it += NT) {
        const int el = it / (2 * Nfq), rr = it % (2 * Nfq);
        const int tf = rr / Nfq, q = rr % Nfq;
        const int64_t e = item(a, e0 + el);
        if (e < 0) continue;
        const int64_t slot = a.slot0 + e * 5 + tf;
        const int o = sm.fori[el][tf];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int m = 0; m < Nfn; ++m) {
          const float w = Ic[q * Nfn + m];
          const int l = op.tperm[o][m];
          for (int c = 0; c < 4; ++c) acc[c] += w * sm.c[el][tf][l][c];
        }
        const float isj = sm.isj[el][tf][q];
        a.tr_out[slot * TS + q] = make_float4(acc[0] * isj, acc[1] * isj, acc[2] * isj, acc[3] * isj);
      }
      pad_traces(a, a.tr_out, tid, NT, e0, EPB, 5, 0, 2, Nfq, TS);
    }
  }
};

}  // namespace hdg
