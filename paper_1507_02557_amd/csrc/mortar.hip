// 1:4 non-conforming triangular faces between tetrahedra.
//
// A coarse face is the union of the four triangles of its midpoint
// subdivision, each the face of one finer tetrahedron.  The paper's meshes
// are conforming (Section 4.2); the coupling here applies its flux (Section
// 2.2) pointwise on every sub-face:
//
//  * the fine element sees, as its neighbour's trace, the coarse element's
//    trace evaluated at the sub-face's lattice nodes (a "virtual" slot in the
//    fine face's canonical frame), so its own face term is the conforming one;
//  * the coarse element's face integral is the sum over the four sub-faces of
//    the flux against its test functions.  Both traces are degree-N
//    polynomials on a planar sub-face, so the sub-face flux is one too and its
//    lattice values with the lattice mass matrix M give that integral exactly:
//      int_sub f phi_i = J^s_sub (I_s phi_i)^T M f_s,
//    I_s the interpolation from the coarse lattice to the sub-face lattice.
//    The coarse kernel lifts J^s_c M g with g = sum_s M^-1 I_s^T M f_s
//    J^s_sub / J^s_c, the L2 projection onto P_N(coarse face) of the
//    piecewise flux; this kernel writes J^s_c g (with J^s_sub = J^s_c / 4,
//    the sub-triangles having a quarter of the area) into the coarse face's
//    flux slot.
//
// The kernel runs before every right-hand-side evaluation, on the traces that
// evaluation reads.  Under multi-rate stepping a coarse element that is
// mid-step supplies its mid-step trace to the virtual slots of the mid-step
// buffer, and a fine side one level coarser than the coarse element is read
// from the mid-step buffer at substeps between its step boundaries (the rule
// of the stage kernels' neighbour reads).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace hdg {

namespace {

constexpr int kFacesPerBlock = 8;  // 32 lanes per face (Nfn <= 21)
constexpr int kLanes = 32;

__device__ inline float4 fma4(float w, float4 x, float4 acc) {
  acc.x += w * x.x;
  acc.y += w * x.y;
  acc.z += w * x.z;
  acc.w += w * x.w;
  return acc;
}

__global__ __launch_bounds__(kFacesPerBlock* kLanes) void mortar_kernel(MortarArgs a) {
  __shared__ float4 C[kFacesPerBlock][kLanes];      // coarse trace, canonical coarse lattice
  __shared__ float4 Ch[kFacesPerBlock][kLanes];     // coarse mid-step trace
  __shared__ float4 Fl[kFacesPerBlock][4][kLanes];  // sub-face fluxes (J^s_sub weighted)
  __shared__ int R[kFacesPerBlock][kNcRec];          // the face's record
  const int lf = threadIdx.x / kLanes, m = threadIdx.x % kLanes;
  const int64_t i = (int64_t)blockIdx.x * kFacesPerBlock + lf;
  const bool face = i < a.n;
  const bool act = face && m < a.nfn;
  // written slots are padded with zeros to whole lines (within the slot)
  const int lw = (a.nfn + 7) / 8 * 8 < a.ts ? (a.nfn + 7) / 8 * 8 : a.ts;
  const bool pad = face && m >= a.nfn && m < lw;
  const int nfn = a.nfn;
  const int64_t ts = a.ts;
  if (face && m < kNcRec) R[lf][m] = a.rec[i * kNcRec + m];
  __syncthreads();
  const int parent = face ? R[lf][0] : 0, flux = face ? R[lf][1] : 0;
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  if (act) {
    C[lf][m] = a.tr[(int64_t)parent * ts + m];
    float4 h = z;
    if (a.tr_half) h = a.tr_half[(int64_t)parent * ts + m];
    Ch[lf][m] = h;
  }
  __syncthreads();
  if (act) {
    const float4 g = a.cgeo[parent - a.cslot0];
    const float4 gs = make_float4(g.x, g.y, g.z, 0.25f * g.w);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t vs = a.vslot0 + 4 * i + s;
      const int fine = R[lf][2 + s], var = R[lf][6 + s];
      const float* Is = a.I + ((int64_t)var * nfn + m) * nfn;
      float4 x = z, xh = z;
      for (int j = 0; j < nfn; ++j) {
        const float w = Is[j];
        x = fma4(w, C[lf][j], x);
        xh = fma4(w, Ch[lf][j], xh);
      }
      a.tr[vs * ts + m] = x;
      if (a.tr_half) a.tr_half[vs * ts + m] = xh;
      // the fine side: its mid-step trace when it is one level coarser and
      // between its step boundaries
      const float4* src = a.tr;
      if (a.dense) {
        const int ln = a.slevel[fine];
        if (ln < a.slevel[parent] && (a.ksub & ((1 << (a.L - ln)) - 1)) != 0) src = a.tr_half;
      }
      const float4 p = src[(int64_t)fine * ts + m];
      float out[4];
      upwind_flux(x, p, gs, a.tau[vs], false, out);
      Fl[lf][s][m] = make_float4(out[0], out[1], out[2], out[3]);
    }
  }
  __syncthreads();
  if (act) {
    float4 gsum = z;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float* Ps = a.P + ((int64_t)R[lf][6 + s] * nfn + m) * nfn;
      for (int j = 0; j < nfn; ++j) gsum = fma4(Ps[j], Fl[lf][s][j], gsum);
    }
    a.tr[(int64_t)flux * ts + m] = gsum;
  }
  if (pad) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t vs = a.vslot0 + 4 * i + s;
      a.tr[vs * ts + m] = z;
      if (a.tr_half) a.tr_half[vs * ts + m] = z;
    }
    a.tr[(int64_t)R[lf][1] * ts + m] = z;
  }
}

}  // namespace

void launch_mortar(const MortarArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  const int64_t nblk = (a.n + kFacesPerBlock - 1) / kFacesPerBlock;
  hipLaunchKernelGGL(mortar_kernel, dim3((unsigned)nblk), dim3(kFacesPerBlock * kLanes), 0, s, a);
}

}  // namespace hdg
