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

struct StageArgs {
  int64_t K;             // elements of this type
  float* U;              // state [4][K][Np], fields p, ux, uy, uz
  float* R;              // LSERK residual (or rhs) [4][K][Np]
  const float* geo;      // per-type volume geometry
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
  int mode;              // 0: full stage, 1: traces of U only, 2: rhs into R only
};

enum { kModeStage = 0, kModeTrace = 1, kModeRhs = 2 };

// Neighbour state on a boundary face (mirror principle):
// rigid wall p+ = p-, u+ = u- - 2 (n.u-) n; free surface p+ = -p-, u+ = u-.
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

// Own and neighbour traces at canonical point q of a slot.
HD inline void face_states(const StageArgs& a, int64_t slot, int nfq, int q, float4 g, float4& m, float4& p) {
  m = a.tr_in[slot * nfq + q];
  const int nb = a.nbr[slot];
  if (nb >= 0) p = a.tr_in[(int64_t)nb * nfq + q];
  else p = mirror_state(m, -nb - 1, g.x, g.y, g.z);
}

}  // namespace hdg
