// Shared pieces of the fused per-type stage kernels.
//
// One launch per element type and Runge-Kutta stage computes, for every
// element of the type: the upwind-penalty flux at the canonical face cubature
// points (own trace and the neighbour's trace read from the trace buffer
// written in the previous stage), the surface lift, the volume term, the
// inverse mass, the low-storage RK update of the state, and the traces of the
// updated state at the face cubature points (written to the other trace
// buffer).  This fuses the paper's volume, surface and update kernels
// (Section 2.3) into one pass over the state.
//
// Each kernel body is written as a sequence of phases separated by block
// barriers; a phase is a loop "for (item = tid; item < n; item += NT)" over
// independent work items and communicates with later phases only through
// LDS.  Elements are processed in batches of EPB per block; blocks stride
// over batches so the operator tables are loaded into LDS once per block.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HD __host__ __device__

namespace hdg {

// Multi-rate (MRAB3) parameters of one launch, indexed by level 1..L.
struct MrabParams {
  int L;                 // number of levels (0: single rate)
  int ksub;              // substep index within the coarse step
  int dense;             // 1: read a coarser neighbour's mid-step trace when it is mid-step
  int hs[9][3];          // history slot of r_s, r_{s-1}, r_{s-2} per level (rhs mode: [l][0] = new slot)
  float b1[9][3];        // AB3 weights beta_j(1) per level (order-limited at start)
  float bh[9][3];        // dense-output weights beta_j(1/2) per level
  float dtl[9];          // dtau_l
};

struct StageArgs {
  int64_t K;             // field stride in elements (the type's count rounded up to 4)
  int64_t n_items;       // elements processed by this launch
  const int* elist;      // element of each item (NULL: item i is element i)
  const int8_t* elevel;  // level per element (multi-rate)
  const int8_t* ehalf;   // 1: a face neighbour is finer, so the element's mid-step traces are read
  const int8_t* slevel;  // level of each slot's element [nslot] (multi-rate)
  float* H;              // right-hand-side history [3][4][K][Np] (multi-rate)
  float4* tr_half;       // mid-step traces [nslot][Nfq] (multi-rate)
  MrabParams mr;
  float* U;              // state [4][K][Np], fields p, ux, uy, uz
  float* R;              // LSERK residual (or rhs) [4][K][Np]
  const float* geo;      // per-type volume geometry
  const double* V;       // element vertices [K][nv][3] (geometry recomputed in FP64)
  const float2* mat;     // [K] (kappa, 1/rho)
  const int* nbr;        // [nslot] neighbour slot, or -(1 + bc) on the boundary
  const int8_t* ori;     // [nslot] orientation code of the canonical face frame
  const float2* tau;     // [nslot] (tau_p, tau_u)
  const float4* fgeo;    // [K*nf][fstride] (nx, ny, nz, w*J^s) of this type
  const float* isqJ;     // wedges: [K*nf][Nfq] 1/sqrt(J) at face points
  const float4* tr_in;   // traces read this stage [nslot][Nfq]
  float4* tr_out;        // traces written this stage [nslot][Nfq]
  int64_t slot0;         // first slot of this type
  const float* ops;      // packed FP32 operator tables
  const int* iops;       // packed integer tables
  float a, b, dt;        // res = a res + dt rhs; U = U + b res
  int mode;              // kModeStage, kModeTrace, kModeRhs, kModeRhsHist or kModeMrab
  int lat;               // 1: triangular faces between tetrahedra and pyramids carry
                         // lattice traces (face-lattice values, canonical order)
};

// kModeMrab: multi-rate update (state, traces, mid-step traces) of the items.
enum { kModeStage = 0, kModeTrace = 1, kModeRhs = 2, kModeRhsHist = 3, kModeMrab = 4 };

// Neighbour code of the coarse face of a 1:4 non-conforming interface:
// nbr = -(kNcBase + s) says that trace slot s holds the face's flux (already
// weighted by J^s, face-lattice values in canonical order) instead of a
// neighbour trace.  Boundary codes -(1 + bc) stay above -kNcBase.
constexpr int kNcBase = 16;

// Float4 entries per trace slot: the face's cubature points rounded up to
// whole 128-byte lines, so every slot starts on a line boundary.  A lattice
// trace (triangular face between tetrahedra or pyramids) is written as
// lattice_width values, its lattice padded with zeros to whole lines: full
// lines go to memory as plain writes, where a partly written line costs a
// read-modify-write.  At N = 1 (four points, 64 bytes) a slot is not padded:
// doubling every trace costs more there than the partial lines.
HD constexpr int trace_stride(int N) { return N == 1 ? 4 : ((N + 1) * (N + 1) + 7) / 8 * 8; }
HD constexpr int lattice_width(int N) {
  return ((N + 1) * (N + 2) / 2 + 7) / 8 * 8 < trace_stride(N) ? ((N + 1) * (N + 2) / 2 + 7) / 8 * 8
                                                                 : trace_stride(N);
}

// LDS writes of this wavefront become visible to its later LDS reads (LDS
// operations of one wavefront complete in order; this stops the compiler
// from moving memory operations across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Element processed by item i, or -1 past the end of the launch.
HD inline int64_t item(const StageArgs& a, int64_t i) {
  if (i >= a.n_items) return -1;
  return a.elist ? (int64_t)a.elist[i] : i;
}

// Zero padding of the trace slots written at cubature points: entries
// [nfq, ts) of faces f0 .. f0 + nfaces - 1 of the batch's elements (nf faces
// per element), so each slot goes to memory in whole lines.
HD inline void pad_traces(const StageArgs& a, float4* tr, int tid, int nt, int64_t e0, int epb, int nf, int f0,
                          int nfaces, int nfq, int ts) {
  const int w = ts - nfq;
  for (int it = tid; it < epb * nfaces * w; it += nt) {
    const int el = it / (nfaces * w), r = it % (nfaces * w);
    const int64_t e = item(a, e0 + el);
    if (e < 0) continue;
    tr[(a.slot0 + e * nf + f0 + r / w) * ts + nfq + r % w] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// Where a right-hand side goes: the rhs buffer, or the history slot of the
// element's level.
HD inline float* rhs_dst(const StageArgs& a, int64_t e, int Np) {
  if (a.mode == kModeRhsHist) return a.H + (int64_t)a.mr.hs[a.elevel[e]][0] * 4 * a.K * Np;
  return a.R;
}

// Neighbour state on a boundary face (mirror principle):
// rigid wall p+ = p-, u+ = u- - 2 (n.u-) n; free surface p+ = -p-, u+ = u-.
// Residual of the four fields at one node, read at the start of the node's
// work so the four loads overlap it and one another (stores to R and U that
// come later could alias them as far as the compiler can tell).
HD inline void load_residual(const StageArgs& a, int64_t base, int Np, float (&r)[4]) {
  const bool upd = a.mode != kModeRhs && a.mode != kModeRhsHist;
  for (int c = 0; c < 4; ++c) r[c] = upd ? a.R[(int64_t)c * a.K * Np + base] : 0.f;
}

// Output of the four fields at one node: the rhs itself, or the low-storage
// Runge-Kutta update of residual and state (u and un point at field 0 of the
// node in the block's state arrays, fields fstride apart).
HD inline void node_update(const StageArgs& a, int64_t e, int Np, int64_t base, const float (&rhs)[4],
                           const float (&r)[4], const float* u, float* un, int fstride) {
  for (int c = 0; c < 4; ++c) {
    const int64_t gi = (int64_t)c * a.K * Np + base;
    if (a.mode == kModeRhs || a.mode == kModeRhsHist) {
      rhs_dst(a, e, Np)[gi] = rhs[c];
    } else {
      const float res = a.a * r[c] + a.dt * rhs[c];
      const float v = u[c * fstride] + a.b * res;
      a.R[gi] = res;
      a.U[gi] = v;
      un[c * fstride] = v;
    }
  }
}

HD inline float4 mirror_state(float4 m, int bc, float nx, float ny, float nz) {
  if (bc == 1) {
    const float un = m.y * nx + m.z * ny + m.w * nz;
    return make_float4(m.x, m.y - 2.0f * un * nx, m.z - 2.0f * un * ny, m.w - 2.0f * un * nz);
  }
  return make_float4(-m.x, m.y, m.z, m.w);
}

// Upwind-penalty flux (Section 2.2) scaled by w J^s; m own trace, p the
// neighbour's.  p-flux: strong (tau_p [p] - n.[u])/2, skew tau_p [p]/2 - n.{u};
// u-flux (tau_u n.[u] - [p]) n / 2.
HD inline void upwind_flux(float4 m, float4 p, float4 g, float2 tau, bool skew, float out[4]) {
  const float nx = g.x, ny = g.y, nz = g.z;
  const float jp = p.x - m.x;
  const float nju = nx * (p.y - m.y) + ny * (p.z - m.z) + nz * (p.w - m.w);
  float fp;
  if (skew) {
    const float nau = 0.5f * (nx * (p.y + m.y) + ny * (p.z + m.z) + nz * (p.w + m.w));
    fp = 0.5f * tau.x * jp - nau;
  } else {
    fp = 0.5f * (tau.x * jp - nju);
  }
  const float fu = 0.5f * (tau.y * nju - jp) * g.w;
  out[0] = fp * g.w;
  out[1] = fu * nx;
  out[2] = fu * ny;
  out[3] = fu * nz;
}

// Whether the neighbour slot nb supplies its dense-output (mid-step) trace:
// a coarser neighbour between its step boundaries.  Kernels that keep this
// as a flag take it from here, never by comparing the buffer pointer that
// neighbour_src returns (a pointer chosen in divergent control flow and then
// compared has been compiled wrongly for gfx950: the tr_in branch's value
// was lost).
HD inline bool neighbour_mid(const StageArgs& a, int64_t slot, int nb) {
  if (!a.mr.dense) return false;
  const int ln = a.slevel[nb];
  return ln < a.slevel[slot] && (a.mr.ksub & ((1 << (a.mr.L - ln)) - 1)) != 0;
}

// Trace buffer holding the neighbour slot nb's current trace.
HD inline const float4* neighbour_src(const StageArgs& a, int64_t slot, int nb) {
  return neighbour_mid(a, slot, nb) ? a.tr_half : a.tr_in;
}

// Own and neighbour traces at canonical point q of a slot (ts: trace stride).
HD inline void face_states(const StageArgs& a, int64_t slot, int ts, int q, float4 g, float4& m, float4& p) {
  m = a.tr_in[slot * ts + q];
  const int nb = a.nbr[slot];
  if (nb >= 0) {
    p = neighbour_src(a, slot, nb)[(int64_t)nb * ts + q];
  } else {
    p = mirror_state(m, -nb - 1, g.x, g.y, g.z);
  }
}

// Multi-rate update of one batch, as a sequence of barrier-separated steps:
// load the state; u_new = u + dtau_l sum_j beta_j(1) r_{s-j} (written to U);
// traces of u_new into tr_out; u_half = u + dtau_l sum_j beta_j(1/2) r_{s-j};
// traces of u_half into tr_half (the dense output at the middle of the step).
template <class S>
struct MrabUpdate {
  static constexpr int T = S::nphase - S::kTraceBegin;
  static constexpr int nstep = 3 + 2 * T;

  template <class SM>
  HD static void combine(int tid, SM& smem, const StageArgs& a, int64_t e0, bool half) {
    constexpr int EPB = S::kEPB, Np = S::Np;
    auto& sm = S::batch(smem);
    const int64_t K = a.K;
    const int64_t hstr = 4 * K * Np;
    for (int it = tid; it < 4 * EPB * Np; it += S::NT) {
      const int c = it / (EPB * Np), r = it % (EPB * Np);
      const int el = r / Np, i = r % Np;
      const int64_t e = item(a, e0 + el);
      if (e < 0) continue;
      const int lv = a.elevel[e];
      const float* w = half ? a.mr.bh[lv] : a.mr.b1[lv];
      const int64_t gi = (int64_t)c * K * Np + e * Np + i;
      const float acc = w[0] * a.H[a.mr.hs[lv][0] * hstr + gi] + w[1] * a.H[a.mr.hs[lv][1] * hstr + gi] +
                        w[2] * a.H[a.mr.hs[lv][2] * hstr + gi];
      const float un = sm.u[c][el][i] + a.mr.dtl[lv] * acc;
      sm.un[c][el][i] = un;
      if (!half) a.U[gi] = un;
    }
  }

  // mid-step traces are written only for batches holding an element whose
  // finer neighbour reads them
  HD static bool any_half(const StageArgs& a, int64_t e0) {
    for (int el = 0; el < S::kEPB; ++el) {
      const int64_t e = item(a, e0 + el);
      if (e >= 0 && a.ehalf[e]) return true;
    }
    return false;
  }

  template <class SM>
  HD static void step(int st, int tid, SM& sm, const StageArgs& a, int64_t e0) {
    if (st >= 2 + T && !any_half(a, e0)) return;
    StageArgs b = a;
    b.mode = kModeStage;
    if (st == 0) {
      // phase 0 in trace mode only loads the batch's state
      StageArgs l = a;
      l.mode = kModeTrace;
      S::phase(0, tid, sm, l, e0);
    } else if (st == 1) {
      combine(tid, sm, a, e0, false);
    } else if (st < 2 + T) {
      S::phase(S::kTraceBegin + st - 2, tid, sm, b, e0);
    } else if (st == 2 + T) {
      combine(tid, sm, a, e0, true);
    } else {
      b.tr_out = a.tr_half;
      S::phase(S::kTraceBegin + st - 3 - T, tid, sm, b, e0);
    }
  }
};

}  // namespace hdg
