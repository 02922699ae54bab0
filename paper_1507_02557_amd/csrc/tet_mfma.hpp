// Tetrahedra on the matrix cores (Section 2.3.2, Algorithm 4: strong form,
// dense reference derivative matrices, constant geometric factors).
//
// Each wavefront owns a tile of 16 consecutive elements; the element index is
// the column index of every matrix product, so one 16x16x4 FP32 MFMA applies
// a 16-row slice of an operator to 16 elements at once:
//
//   grad:   G_r = D^r p                  (3 products per k-step)
//   div:    P   = sum_r D^r (-u^r)       u^r = sum_d dxi_r/dx_d u_d
//   lift:   P  += sum_f L_f (J^s F_p / J),  U_d = sum_f L_f (J^s F_d / J)
//
// with L_f = M^-1 E_f M_f, M_f the face mass matrix of the equispaced face
// lattice (E_f scatters face lattice nodes onto element nodes).  On a planar
// face between elements whose traces are degree-N polynomials (tetrahedra,
// pyramids) the upwind flux is a degree-N polynomial with constant
// coefficients, so evaluating it at the lattice nodes and weighting by M_f
// gives the same face integral as the canonical cubature rule.  The lattice
// is invariant under the face's vertex permutations, so M_f is the same in
// every local frame, and the trace of an element on such a face is just its
// face-node values: the kernel writes them (permuted to the canonical frame)
// to the trace buffer and reads the neighbour's in the same form.
//
// Operators live in LDS in MFMA fragment order (entry [lane] of a fragment
// is the value lane 'lane' passes to the instruction), so every fragment
// load is one conflict-free 32-bit LDS read.  The element tile lives in LDS
// row-major per element with an odd row stride, which makes the B-fragment
// reads (16 elements x 4 consecutive nodes) conflict-free as well.
#pragma once

#include "mfma_common.hpp"

namespace hdg {

// ST = false: a kernel for the right-hand-side modes only (no residual
// registers, no stage update).
template <int N, int NW, int P, bool ST = true>
struct TetMfma {
  typedef Prec<P> PR;
  typedef typename PR::V V;
  static constexpr int KI = PR::KI, KK = PR::KK, NPC = PR::NPC;
  static constexpr int VF = (int)(sizeof(V) / sizeof(float));  // floats per fragment entry
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfn = (N + 1) * (N + 2) / 2;
  static constexpr int Nfq = (N + 1) * (N + 1);
  static constexpr int TS = trace_stride(N), LW = lattice_width(N);
  static constexpr int Mt = (Np + 15) / 16;  // 16-row tiles of the element operators
  static constexpr int Ks = (Np + 3) / 4;    // k-steps over element nodes
  static constexpr int Kf = (Nfn + 3) / 4;   // k-steps over one face's lattice
  // Odd row strides.  An odd Np is its own stride: the tile is then one flat
  // array, so the tile stores read aligned 16-byte LDS vectors, and a
  // B-fragment read past the end of a row meets finite values of the next
  // row (the operator columns there are zero).  Otherwise the rows are padded
  // and the padding stays zero.
  static constexpr int SX = (Np & 1) ? Np : ((4 * Ks) | 1);
  static constexpr int SF = (4 * Kf) | 1;
  static constexpr int NT = 64 * NW;
  static constexpr int KsP = (Np + KK - 1) / KK;   // k-steps over nodes at this precision
  static constexpr int KfP = (Nfn + KK - 1) / KK;  // k-steps over a face lattice
  static constexpr int kDFloats = 3 * Mt * KsP * NPC * 64 * VF;
  static constexpr int kLFloats = 4 * Mt * KfP * NPC * 64 * VF;
  static constexpr int kOpsFloats = kDFloats + kLFloats + 2;  // + inverse operator scales
  static constexpr int kOpsInts = 4 * Nfn + 6 * Nfn;

  struct alignas(16) Wave {
    float X[4][16][SX];  // state tile (p, ux, uy, uz)
    float F[4][16][SF];  // one face's scaled flux; staging of one output field
  };
  static_assert(4 * 16 * SF >= 16 * SX, "output staging does not fit the flux buffer");

  struct Smem {
    V D[3][Mt][KsP][NPC][64];
    V L[4][Mt][KfP][NPC][64];
    float inv_sD, inv_sL;
    int fnode[4][Nfn];  // element node of local face lattice node
    int tperm[6][Nfn];  // canonical lattice node -> local lattice node
    Wave w[NW];
  };

  static constexpr int Q4 = 4 * Np;          // float4 per field of a full tile (16 Np floats)
  static constexpr int JQ = (Q4 + 63) / 64;  // of them per lane
  static constexpr int JF = (Nfn + 3) / 4;   // lattice nodes m = g + 4 j per lane and face

  // rows [0, Np) of 16 elements of one field, global [K][Np] <-> LDS [16][S]
  template <int S>
  __device__ static void load_rows(float (*dst)[S], const float* src, const StageArgs& a, int64_t e0, int lane) {
    for (int it = lane; it < 16 * Np; it += 64) {
      const int n = it / Np, k = it - n * Np;
      const int64_t e = item(a, e0 + n);
      dst[n][k] = e >= 0 ? src[e * Np + k] : 0.0f;
    }
  }
  template <int S>
  __device__ static void store_rows(float* dst, const float (*src)[S], const StageArgs& a, int64_t e0, int lane) {
    for (int it = lane; it < 16 * Np; it += 64) {
      const int n = it / Np, k = it - n * Np;
      const int64_t e = item(a, e0 + n);
      if (e >= 0) dst[e * Np + k] = src[n][k];
    }
  }
  // four consecutive entries q0 .. q0+3 of a tile in flat [16][Np] order
  template <int S>
  __device__ static void put4(float (*dst)[S], int q0, float4 v) {
    const float x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = q0 + i, n = q / Np;
      dst[n][q - n * Np] = x[i];
    }
  }
  template <int S>
  __device__ static float4 get4(const float (*src)[S], int q0) {
    float x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = q0 + i, n = q / Np;
      x[i] = src[n][q - n * Np];
    }
    return make_float4(x[0], x[1], x[2], x[3]);
  }
  // A full tile of consecutive elements whose fields start 16-byte aligned
  // moves as flat float4 vectors, all loads of a field group issued at once.
  __device__ static bool contiguous(const StageArgs& a, int64_t e0) {
    return a.elist == nullptr && e0 + 16 <= a.n_items && ((a.K * Np) & 3) == 0;
  }
  __device__ static void load_field(float4 (&v)[JQ], const float* base, int64_t e0, int lane) {
    const float4* src = reinterpret_cast<const float4*>(base + e0 * Np);
#pragma unroll
    for (int j = 0; j < JQ; ++j)
      if (lane + 64 * j < Q4) v[j] = src[lane + 64 * j];
  }
  template <int S>
  __device__ static void put_field(float (*dst)[S], const float4 (&v)[JQ], int lane) {
#pragma unroll
    for (int j = 0; j < JQ; ++j) {
      if (lane + 64 * j >= Q4) continue;
      put4<S>(dst, 4 * (lane + 64 * j), v[j]);
    }
  }
  template <int S>
  __device__ static void store_tile(float* dst, const float (*src)[S], const StageArgs& a, int64_t e0, int lane,
                                    bool contig) {
    if (contig) {
      float4* d4 = reinterpret_cast<float4*>(dst + e0 * Np);
#pragma unroll
      for (int j = 0; j < JQ; ++j) {
        if (lane + 64 * j >= Q4) continue;
        if constexpr (S == Np)
          d4[lane + 64 * j] = reinterpret_cast<const float4*>(&src[0][0])[lane + 64 * j];
        else
          d4[lane + 64 * j] = get4<S>(src, 4 * (lane + 64 * j));
      }
    } else {
      store_rows<S>(dst, src, a, e0, lane);
    }
  }

  // Per-lane face record: element (lane & 15) of the tile, face (lane >> 4).
  struct FaceRec {
    int nb, ori, half;  // neighbour slot (or -(1 + bc)), orientation, read the mid-step trace
    float4 g;           // normal, J^s
    float2 tau;
  };
  __device__ static FaceRec load_rec(const StageArgs& a, int64_t e, int f) {
    FaceRec r{-1, 0, 0, make_float4(0.f, 0.f, 0.f, 0.f), make_float2(0.f, 0.f)};
    if (e < 0) return r;
    const int64_t slot = a.slot0 + e * 4 + f;
    r.nb = a.nbr[slot];
    r.ori = a.ori[slot];
    r.g = a.fgeo[e * 4 + f];
    r.tau = a.tau[slot];
    if (r.nb >= 0) r.half = neighbour_mid(a, slot, r.nb);
    return r;
  }
  __device__ static FaceRec shfl_rec(const FaceRec& r, int src) {
    FaceRec o;
    o.nb = __shfl(r.nb, src);
    o.ori = __shfl(r.ori, src);
    o.half = __shfl(r.half, src);
    o.g = make_float4(__shfl(r.g.x, src), __shfl(r.g.y, src), __shfl(r.g.z, src), __shfl(r.g.w, src));
    o.tau = make_float2(__shfl(r.tau.x, src), __shfl(r.tau.y, src));
    return o;
  }

  // the neighbour's lattice trace values of face f at the lane's nodes
  // m = g + 4 j (element n of the tile); on the coarse face of a
  // non-conforming interface, the face's flux from its flux slot
  __device__ static void fetch_nbr(const StageArgs& a, const FaceRec& rec, int64_t e, int n, int g, int f,
                                   float4 (&pv)[JF]) {
    const int src = n + 16 * f;
    const int nb = __shfl(rec.nb, src);
    const float4* nsrc = __shfl(rec.half, src) ? a.tr_half : a.tr_in;
    const int64_t base = nb >= 0 ? (int64_t)nb * TS : (int64_t)(-nb - kNcBase) * TS;
    const bool fetch = nb >= 0 || nb <= -kNcBase;
#pragma unroll
    for (int j = 0; j < JF; ++j) {
      const int m = g + 4 * j;
      if (e >= 0 && m < Nfn && fetch) pv[j] = nsrc[base + m];
    }
  }

  // face-node values of the tile's state, canonical lattice order, padded
  // with zeros to whole lines: lane (q, m) = (lane >> 4, lane & 15) writes
  // entry m of element 4 k + q, so one store instruction covers the whole
  // face traces of four elements (LEAN: one face at a time, for callers with
  // many registers in use)
  static constexpr int MJ = (LW + 15) / 16;  // entries m = (lane & 15) + 16 j per lane
  template <bool LEAN = false, class SM>
  __device__ static void write_traces(const SM& sm, const float (&X)[4][16][SX], const StageArgs& a, int64_t e0,
                                      int lane, const FaceRec& rec, float4* tr, bool col_active = true) {
    if constexpr (LEAN) {
#pragma unroll 1
      for (int f = 0; f < 4; ++f) trace_face(sm, X, a, e0, lane, f, rec, tr, col_active);
    } else {
#pragma unroll
      for (int f = 0; f < 4; ++f) trace_face(sm, X, a, e0, lane, f, rec, tr, col_active);
    }
  }
  template <class SM>
  __device__ static void trace_face(const SM& sm, const float (&X)[4][16][SX], const StageArgs& a, int64_t e0,
                                    int lane, int f, const FaceRec& rec, float4* tr, bool col_active) {
    const int q = lane >> 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int n = 4 * k + q;
      // orientation of face f of element n, and whether element n writes
      const int o = __shfl(rec.ori, n + 16 * f);
      const int act = __shfl((int)col_active, n);
      const int64_t e = item(a, e0 + n);
      if (e < 0 || !act) continue;
      const int64_t base = (a.slot0 + e * 4 + f) * TS;
#pragma unroll
      for (int j = 0; j < MJ; ++j) {
        const int m = (lane & 15) + 16 * j;
        if (m >= LW) continue;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (m < Nfn) {
          const int node = sm.fnode[f][sm.tperm[o][m]];
          v = make_float4(X[0][n][node], X[1][n][node], X[2][n][node], X[3][n][node]);
        }
        tr[base + m] = v;
      }
    }
  }

  // ---- multi-rate AB3 update: a kernel of its own (no operator tables, a
  // state tile per wavefront, its own register budget)
  //   u_half = u + dtau_l sum_j beta_j(1/2) r_{s-j}   (dense output at mid-step)
  //   u_new  = u + dtau_l sum_j beta_j(1)   r_{s-j}
  // One LDS tile per wavefront (12 wavefronts per compute unit at N <= 4,
  // set by the registers): it holds u_half while the mid-step traces are
  // written (tiles with an element whose finer neighbour reads them), then
  // u_new, which is stored with its traces; in the one-level tiles u_new waits
  // in registers and the history is read once.
  static constexpr int NWU = 4;  // wavefronts per block of the update kernel
  // wavefronts per SIMD the update kernel's register allocation must allow
  static constexpr int kUpdateWaves = N <= 4 ? 3 : 2;
  static constexpr int JN = (16 * Np + 63) / 64;  // flat tile entries per lane
  struct alignas(16) UWave {
    float X[4][16][SX];  // state tile
  };
  struct USmem {
    MrabParams mr;  // per-level weights and history slots (indexed by the element's level)
    int fnode[4][Nfn];
    int tperm[6][Nfn];
    UWave w[NWU];
  };

  __device__ static void update_tile(const USmem& sm, UWave& W, const StageArgs& a, int64_t e0, int lane) {
    const int64_t K = a.K;
    const int64_t hstr = 4 * K * Np;
    const int64_t fs = K * Np;
    const int n = lane & 15, g = lane >> 4;
    const int64_t e = item(a, e0 + n);
    const bool contig = contiguous(a, e0);
    wave_sync();
    // only the orientation codes of the face records are needed here
    FaceRec rec{-1, 0, 0, make_float4(0.f, 0.f, 0.f, 0.f), make_float2(0.f, 0.f)};
    if (e >= 0) rec.ori = a.ori[a.slot0 + e * 4 + g];
    const bool half = e >= 0 && a.ehalf[e];
    const bool any_half = __any(half);
    const MrabParams& mr = sm.mr;
    // a tile of consecutive elements of one level (the common case with the
    // elements stored finest level first) moves as flat float4 vectors;
    // without an item list the storage is in that order, so equal levels at
    // both ends of the tile mean one level throughout
    const int lv0 = contig ? a.elevel[e0] : 0;
    if (contig && a.elevel[e0 + 15] == lv0) {
      const float dl = mr.dtl[lv0];
      const float w1[3] = {dl * mr.b1[lv0][0], dl * mr.b1[lv0][1], dl * mr.b1[lv0][2]};
      const float wh[3] = {dl * mr.bh[lv0][0], dl * mr.bh[lv0][1], dl * mr.bh[lv0][2]};
      const float* h0 = a.H + mr.hs[lv0][0] * hstr;
      const float* h1 = a.H + mr.hs[lv0][1] * hstr;
      const float* h2 = a.H + mr.hs[lv0][2] * hstr;
      float4 un[4][JQ];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float4 u[JQ], x0[JQ], x1[JQ], x2[JQ];
        load_field(u, a.U + c * fs, e0, lane);
        load_field(x0, h0 + c * fs, e0, lane);
        load_field(x1, h1 + c * fs, e0, lane);
        load_field(x2, h2 + c * fs, e0, lane);
        float4* U4 = reinterpret_cast<float4*>(a.U + c * fs + e0 * Np);
#pragma unroll
        for (int j = 0; j < JQ; ++j) {
          if (lane + 64 * j >= Q4) continue;
          un[c][j] = u[j] + w1[0] * x0[j] + w1[1] * x1[j] + w1[2] * x2[j];
          const float4 uh = u[j] + wh[0] * x0[j] + wh[1] * x1[j] + wh[2] * x2[j];
          U4[lane + 64 * j] = un[c][j];
          put4<SX>(W.X[c], 4 * (lane + 64 * j), any_half ? uh : un[c][j]);
        }
        // the next field's loads are issued after this field's stores (all
        // four fields' loads in flight at once would not fit the registers)
        __builtin_amdgcn_sched_barrier(0);
      }
      wave_sync();
      if (any_half) {
        // mid-step traces of the elements whose finer neighbours read them
        write_traces<true>(sm, W.X, a, e0, lane, rec, a.tr_half, half);
        wave_sync();
#pragma unroll
        for (int c = 0; c < 4; ++c) put_field<SX>(W.X[c], un[c], lane);
        wave_sync();
      }
      write_traces(sm, W.X, a, e0, lane, rec, a.tr_out);
      return;
    }
    if (contig) {
#pragma unroll 1
      for (int c = 0; c < 4; ++c) {
        float4 v[JQ];
        load_field(v, a.U + c * fs, e0, lane);
        put_field<SX>(W.X[c], v, lane);
      }
    } else {
      for (int c = 0; c < 4; ++c) load_rows<SX>(W.X[c], a.U + (int64_t)c * K * Np, a, e0, lane);
    }
    wave_sync();
    // general tiles (an item list, or two levels in one tile): per-entry
    // history reads, one field at a time; with mid-step traces to write the
    // history is read twice (u_half, then u_new - u_half)
    if (any_half) {
      hist_pass(sm, W, a, e0, lane, 0);
      wave_sync();
      write_traces<true>(sm, W.X, a, e0, lane, rec, a.tr_half, half);
      wave_sync();
      hist_pass(sm, W, a, e0, lane, 1);
    } else {
      hist_pass(sm, W, a, e0, lane, 2);
    }
    wave_sync();
#pragma unroll 1
    for (int c = 0; c < 4; ++c) store_tile<SX>(a.U + (int64_t)c * K * Np, W.X[c], a, e0, lane, contig);
    write_traces<true>(sm, W.X, a, e0, lane, rec, a.tr_out);
  }

  // X += dtau_l sum_j w_j r_{s-j} over the tile, per entry at the entry's
  // element level: w = beta(1/2) (which 0), beta(1) - beta(1/2) (1), beta(1) (2)
  __device__ static void hist_pass(const USmem& sm, UWave& W, const StageArgs& a, int64_t e0, int lane, int which) {
    const int64_t K = a.K;
    const int64_t hstr = 4 * K * Np;
    const MrabParams& mr = sm.mr;
#pragma unroll 1
    for (int c = 0; c < 4; ++c)
#pragma unroll 1
      for (int j = 0; j < JN; ++j) {
        const int it = lane + 64 * j;
        if (it >= 16 * Np) continue;
        const int nn = it / Np, k = it - nn * Np;
        const int64_t ee = item(a, e0 + nn);
        if (ee < 0) continue;
        const int lv = a.elevel[ee];
        const int64_t gi = (int64_t)c * K * Np + ee * Np + k;
        const float x0 = a.H[mr.hs[lv][0] * hstr + gi], x1 = a.H[mr.hs[lv][1] * hstr + gi],
                    x2 = a.H[mr.hs[lv][2] * hstr + gi];
        float w[3];
#pragma unroll
        for (int q = 0; q < 3; ++q)
          w[q] = which == 0 ? mr.bh[lv][q] : (which == 1 ? mr.b1[lv][q] - mr.bh[lv][q] : mr.b1[lv][q]);
        W.X[c][nn][k] += mr.dtl[lv] * (w[0] * x0 + w[1] * x1 + w[2] * x2);
      }
  }

  __device__ static void run_update(USmem& sm, const StageArgs& a) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) sm.mr = a.mr;
    for (int i = tid; i < 4 * Nfn; i += 64 * NWU) (&sm.fnode[0][0])[i] = a.iops[i];
    for (int i = tid; i < 6 * Nfn; i += 64 * NWU) (&sm.tperm[0][0])[i] = a.iops[4 * Nfn + i];
    // padded rows of the tiles must hold finite values
    float* wz = &sm.w[0].X[0][0][0];
    for (int i = tid; i < (int)(NWU * sizeof(UWave) / sizeof(float)); i += 64 * NWU) wz[i] = 0.f;
    __syncthreads();
    UWave& W = sm.w[wv];
    const int64_t ntile = (a.n_items + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * NWU + wv; t < ntile; t += (int64_t)gridDim.x * NWU)
      update_tile(sm, W, a, t * 16, lane);
  }

  // acc += L_f F (one field) with split operands and a column scale.
  __device__ static void lift_split(const Smem& sm, const Wave& W, int f, int n, int g, int lane,
                                    const float (*Fc)[SF], f32x4 (&acc)[Mt]) {
    float mf = 0.f;
#pragma unroll
    for (int j = 0; j < JF; ++j) {
      const int l = g + 4 * j;
      if (l < Nfn) mf = fmaxf(mf, fabsf(Fc[n][l]));
    }
    const float sf = col_scale(col_max(mf));
    f32x4 tmp[Mt];
#pragma unroll
    for (int t = 0; t < Mt; ++t) tmp[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KfP; ++s) {
      float v[KI];
#pragma unroll
      for (int i = 0; i < KI; ++i) {
        const int k = KK * s + KI * g + i;
        v[i] = k < Nfn ? Fc[n][k < Nfn ? k : 0] : 0.f;
      }
      V b[NPC];
      split_pieces<PR>(v, sf, b);
#pragma unroll
      for (int t = 0; t < Mt; ++t) {
        V a[NPC];
#pragma unroll
        for (int q = 0; q < NPC; ++q) a[q] = sm.L[f][t][s][q][lane];
        tmp[t] = mma_split<PR>(a, b, tmp[t]);
      }
    }
    const float gs = sm.inv_sL / sf;
#pragma unroll
    for (int t = 0; t < Mt; ++t) acc[t] += tmp[t] * gs;
  }

  // One face: the strong-form flux at the face's lattice nodes (own value
  // from the tile, neighbour's from pv), scaled by J^s / J, then the lift
  // products acc += L_f F.
  __device__ static void face(const Smem& sm, Wave& W, const StageArgs& a, const FaceRec& rec, int64_t e, int f,
                              int n, int g, int lane, float iJ, const float4 (&pv)[JF], f32x4 (&accP)[Mt],
                              f32x4 (&accL)[3][Mt]) {
    const FaceRec fr = shfl_rec(rec, n + 16 * f);
#pragma unroll
    for (int j = 0; j < JF; ++j) {
      const int m = g + 4 * j;
      if (m >= Nfn) continue;
      float out[4] = {0.f, 0.f, 0.f, 0.f};
      int l = m;
      if (e >= 0) {
        l = sm.tperm[fr.ori][m];
        const int node = sm.fnode[f][l];
        if (fr.nb <= -kNcBase) {
          // coarse face of a non-conforming interface: the flux itself
          out[0] = pv[j].x;
          out[1] = pv[j].y;
          out[2] = pv[j].z;
          out[3] = pv[j].w;
        } else {
          const float4 own = make_float4(W.X[0][n][node], W.X[1][n][node], W.X[2][n][node], W.X[3][n][node]);
          const float4 nb = fr.nb >= 0 ? pv[j] : mirror_state(own, -fr.nb - 1, fr.g.x, fr.g.y, fr.g.z);
          upwind_flux(own, nb, fr.g, fr.tau, false, out);
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) W.F[c][n][l] = out[c] * iJ;
    }
    wave_sync();
    if constexpr (P == 0) {
#pragma unroll
      for (int s = 0; s < Kf; ++s) {
        const int k = 4 * s + g;
        const float b0 = W.F[0][n][k], b1 = W.F[1][n][k], b2 = W.F[2][n][k], b3 = W.F[3][n][k];
#pragma unroll
        for (int t = 0; t < Mt; ++t) {
          const float lf = sm.L[f][t][s][0][lane];
          accP[t] = mma_f32(lf, b0, accP[t]);
          accL[0][t] = mma_f32(lf, b1, accL[0][t]);
          accL[1][t] = mma_f32(lf, b2, accL[1][t]);
          accL[2][t] = mma_f32(lf, b3, accL[2][t]);
        }
      }
    } else {
      lift_split(sm, W, f, n, g, lane, W.F[0], accP);
      lift_split(sm, W, f, n, g, lane, W.F[1], accL[0]);
      lift_split(sm, W, f, n, g, lane, W.F[2], accL[1]);
      lift_split(sm, W, f, n, g, lane, W.F[3], accL[2]);
    }
    wave_sync();
  }

  // Output of field C: rhs = sc * acc at rows 16 t + 4 g + i of column n,
  // then the stage update (res = a res + dt rhs, u += b res) or the rhs store.
  // hist: the history slot of a tile of consecutive elements of one level
  // (multi-rate right-hand side), else null
  template <int C>
  __device__ static void emit(Wave& W, const StageArgs& a, int64_t e0, int lane, bool contig, const float4 (&rv)[JQ],
                              const f32x4 (&acc)[Mt], float sc, float* hist) {
    const int64_t K = a.K;
    const int n = lane & 15, g = lane >> 4;
    const bool stage = ST && a.mode == kModeStage;
    float(*RB)[SX] = reinterpret_cast<float(*)[SX]>(&W.F[0][0][0]);
    if (stage) {
      if (contig) {
        put_field<SX>(RB, rv, lane);
      } else {
        load_rows<SX>(RB, a.R + (int64_t)C * K * Np, a, e0, lane);
      }
      wave_sync();
    }
#pragma unroll
    for (int t = 0; t < Mt; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * t + 4 * g + i;
        if (row >= Np) continue;
        const float rhs = sc * acc[t][i];
        if (stage) {
          const float res = a.a * RB[n][row] + a.dt * rhs;
          RB[n][row] = res;
          W.X[C][n][row] += a.b * res;
        } else {
          RB[n][row] = rhs;
        }
      }
    wave_sync();
    if (hist) {
      store_tile<SX>(hist + (int64_t)C * K * Np, RB, a, e0, lane, true);
    } else if (a.mode == kModeRhsHist) {
      for (int it = lane; it < 16 * Np; it += 64) {
        const int nn = it / Np, k = it - nn * Np;
        const int64_t ee = item(a, e0 + nn);
        if (ee >= 0) rhs_dst(a, ee, Np)[(int64_t)C * K * Np + ee * Np + k] = RB[nn][k];
      }
    } else {
      store_tile<SX>(a.R + (int64_t)C * K * Np, RB, a, e0, lane, contig);
    }
    if (stage) store_tile<SX>(a.U + (int64_t)C * K * Np, W.X[C], a, e0, lane, contig);
    wave_sync();
  }

  __device__ static void tile(const Smem& sm, Wave& W, const StageArgs& a, int64_t e0, int lane) {
    const int64_t K = a.K;
    const int n = lane & 15, g = lane >> 4;
    const int64_t e = item(a, e0 + n);  // element of this lane's column
    const bool contig = contiguous(a, e0);
    // lanes of the previous tile may still read other columns of the tile
    wave_sync();
    const FaceRec rec = load_rec(a, e, g);
    // geometric factors and material of this lane's element (column n)
    float G[10], kap = 0.f, irho = 0.f;
#pragma unroll
    for (int i = 0; i < 10; ++i) G[i] = e >= 0 ? a.geo[e * 12 + i] : 0.f;
    if (e >= 0) {
      kap = a.mat[e].x;
      irho = a.mat[e].y;
    }
    if (contig) {
      const int64_t fs = K * Np;
      float4 v0[JQ], v1[JQ], v2[JQ], v3[JQ];
      load_field(v0, a.U, e0, lane);
      load_field(v1, a.U + fs, e0, lane);
      load_field(v2, a.U + 2 * fs, e0, lane);
      load_field(v3, a.U + 3 * fs, e0, lane);
      put_field<SX>(W.X[0], v0, lane);
      put_field<SX>(W.X[1], v1, lane);
      put_field<SX>(W.X[2], v2, lane);
      put_field<SX>(W.X[3], v3, lane);
    } else {
      for (int c = 0; c < 4; ++c) load_rows<SX>(W.X[c], a.U + (int64_t)c * K * Np, a, e0, lane);
    }
    wave_sync();
    if (a.mode == kModeTrace) {
      write_traces(sm, W.X, a, e0, lane, rec, a.tr_out);
      return;
    }
    const float iJ = G[9];
    // neighbour traces: with FP32 operands faces 0 and 1 are in flight
    // during the volume products and faces 2 and 3 during the first two
    // faces' lift products; the split-precision kernels (more registers in
    // use) fetch each face's at its start
    float4 pv[4][JF];
    if constexpr (P == 0) {
      fetch_nbr(a, rec, e, n, g, 0, pv[0]);
      fetch_nbr(a, rec, e, n, g, 1, pv[1]);
    }
    f32x4 accP[Mt], accG[3][Mt];
#pragma unroll
    for (int t = 0; t < Mt; ++t) {
      accP[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      for (int r = 0; r < 3; ++r) accG[r][t] = accP[t];
    }
    // volume
    if constexpr (P == 0) {
#pragma unroll 2
      for (int s = 0; s < Ks; ++s) {
        const int k = 4 * s + g;
        const float p = W.X[0][n][k], u1 = W.X[1][n][k], u2 = W.X[2][n][k], u3 = W.X[3][n][k];
        float ut[3];
        for (int r = 0; r < 3; ++r) ut[r] = -(G[3 * r] * u1 + G[3 * r + 1] * u2 + G[3 * r + 2] * u3);
#pragma unroll
        for (int t = 0; t < Mt; ++t)
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const float d = sm.D[r][t][s][0][lane];
            accG[r][t] = mma_f32(d, p, accG[r][t]);
            accP[t] = mma_f32(d, ut[r], accP[t]);
          }
      }
    } else {
      // column scales of p and of the contravariant velocities
      float mp = 0.f, mu = 0.f;
      for (int k = g; k < Np; k += 4) {
        const float u1 = W.X[1][n][k], u2 = W.X[2][n][k], u3 = W.X[3][n][k];
        mp = fmaxf(mp, fabsf(W.X[0][n][k]));
#pragma unroll
        for (int r = 0; r < 3; ++r) mu = fmaxf(mu, fabsf(G[3 * r] * u1 + G[3 * r + 1] * u2 + G[3 * r + 2] * u3));
      }
      const float sp = col_scale(col_max(mp)), su = col_scale(col_max(mu));
#pragma unroll 1
      for (int s = 0; s < KsP; ++s) {
        float pv[KI], uv[3][KI];
#pragma unroll
        for (int i = 0; i < KI; ++i) {
          const int k = KK * s + KI * g + i;
          const bool in = k < Np;
          const int kk = in ? k : 0;
          const float u1 = W.X[1][n][kk], u2 = W.X[2][n][kk], u3 = W.X[3][n][kk];
          pv[i] = in ? W.X[0][n][kk] : 0.f;
#pragma unroll
          for (int r = 0; r < 3; ++r) uv[r][i] = in ? -(G[3 * r] * u1 + G[3 * r + 1] * u2 + G[3 * r + 2] * u3) : 0.f;
        }
        V pb[NPC], ub[3][NPC];
        split_pieces<PR>(pv, sp, pb);
#pragma unroll
        for (int r = 0; r < 3; ++r) split_pieces<PR>(uv[r], su, ub[r]);
#pragma unroll
        for (int t = 0; t < Mt; ++t)
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            V a[NPC];
#pragma unroll
            for (int q = 0; q < NPC; ++q) a[q] = sm.D[r][t][s][q][lane];
            accG[r][t] = mma_split<PR>(a, pb, accG[r][t]);
            accP[t] = mma_split<PR>(a, ub[r], accP[t]);
          }
      }
      const float gp = sm.inv_sD / sp, gu = sm.inv_sD / su;
#pragma unroll
      for (int t = 0; t < Mt; ++t) {
        accP[t] *= gu;
#pragma unroll
        for (int r = 0; r < 3; ++r) accG[r][t] *= gp;
      }
    }
    // velocity rhs accumulators start from the physical pressure gradient
    f32x4 accL[3][Mt];
#pragma unroll
    for (int t = 0; t < Mt; ++t)
#pragma unroll
      for (int d = 0; d < 3; ++d) accL[d][t] = -(G[d] * accG[0][t] + G[3 + d] * accG[1][t] + G[6 + d] * accG[2][t]);
    const bool stage = ST && a.mode == kModeStage;
    float4 rv0[JQ], rv1[JQ], rv2[JQ], rv3[JQ];
    // faces: flux at the lattice nodes, then the lift products
    if constexpr (P == 0) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if (f == 0) {
          fetch_nbr(a, rec, e, n, g, 2, pv[2]);
          fetch_nbr(a, rec, e, n, g, 3, pv[3]);
        }
        if (f == 2 && stage && contig) {
          // the residual of the stage, fetched while the last faces are processed
          const int64_t fs = K * Np;
          load_field(rv0, a.R, e0, lane);
          load_field(rv1, a.R + fs, e0, lane);
          load_field(rv2, a.R + 2 * fs, e0, lane);
          load_field(rv3, a.R + 3 * fs, e0, lane);
        }
        face(sm, W, a, rec, e, f, n, g, lane, iJ, pv[f], accP, accL);
      }
    } else {
      if (stage && contig) {
        const int64_t fs = K * Np;
        load_field(rv0, a.R, e0, lane);
        load_field(rv1, a.R + fs, e0, lane);
        load_field(rv2, a.R + 2 * fs, e0, lane);
        load_field(rv3, a.R + 3 * fs, e0, lane);
      }
#pragma unroll 1
      for (int f = 0; f < 4; ++f) {
        float4 pf[JF];
        fetch_nbr(a, rec, e, n, g, f, pf);
        face(sm, W, a, rec, e, f, n, g, lane, iJ, pf, accP, accL);
      }
    }
    // rhs at rows 16 t + 4 g + i of column n; stage update or rhs output
    // (a multi-rate launch without an item list has its elements stored
    // finest level first, so equal levels at both ends mean one level)
    float* hist = nullptr;
    if (a.mode == kModeRhsHist && contig) {
      const int lv = a.elevel[e0];
      if (a.elevel[e0 + 15] == lv) hist = a.H + (int64_t)a.mr.hs[lv][0] * 4 * K * Np;
    }
    emit<0>(W, a, e0, lane, contig, rv0, accP, kap, hist);
    emit<1>(W, a, e0, lane, contig, rv1, accL[0], irho, hist);
    emit<2>(W, a, e0, lane, contig, rv2, accL[1], irho, hist);
    emit<3>(W, a, e0, lane, contig, rv3, accL[2], irho, hist);
    if (stage) write_traces(sm, W.X, a, e0, lane, rec, a.tr_out);
  }

  __device__ static void run(Smem& sm, const StageArgs& a) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    float* dD = reinterpret_cast<float*>(&sm.D[0][0][0][0][0]);
    float* dL = reinterpret_cast<float*>(&sm.L[0][0][0][0][0]);
    for (int i = tid; i < kDFloats; i += NT) dD[i] = a.ops[i];
    for (int i = tid; i < kLFloats; i += NT) dL[i] = a.ops[kDFloats + i];
    if (tid == 0) {
      sm.inv_sD = a.ops[kDFloats + kLFloats];
      sm.inv_sL = a.ops[kDFloats + kLFloats + 1];
    }
    for (int i = tid; i < 4 * Nfn; i += NT) (&sm.fnode[0][0])[i] = a.iops[i];
    for (int i = tid; i < 6 * Nfn; i += NT) (&sm.tperm[0][0])[i] = a.iops[4 * Nfn + i];
    // padded rows and columns of the tiles must hold finite values
    float* wz = &sm.w[0].X[0][0][0];
    for (int i = tid; i < (int)(NW * sizeof(Wave) / sizeof(float)); i += NT) wz[i] = 0.f;
    __syncthreads();
    Wave& W = sm.w[wv];
    const int64_t ntile = (a.n_items + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * NW + wv; t < ntile; t += (int64_t)gridDim.x * NW) tile(sm, W, a, t * 16, lane);
  }
};

}  // namespace hdg
