// Pyramids on the matrix cores (Section 2.3.4, Algorithm 7: semi-nodal
// basis, skew-symmetric form, quadrature-free operators), with lattice
// traces on the four triangular faces.
//
// Each wavefront owns a tile of 16 consecutive pyramids (the column index of
// every product).  With D^r_ij the quadrature-free derivative matrices, the
// right-hand side at node i of an element is
//
//   rhs_p   = kappa / J_i (sum_r [(D^r)^T U^r]_i + S_p,i),
//   rhs_u_d = (1/rho) (-sum_r G_rd,i [D^r p]_i + S_d,i / J_i),
//   U^r_j   = sum_d adj(F)_rd,j u_d,j          (adj(F) = J G),
//
// with G = dxi/dx and J evaluated at the node's (a, b) (they do not depend on
// the collapsed coordinate c) and S the surface term
//
//   S = Fq^T (w J^s flux at the base face's local points)
//     + sum_f Ft_f^T M_f (J^s flux at face f's local lattice nodes),
//
// Fq, Ft_f the basis at the base face's GL points and at the triangle's
// lattice nodes, M_f the lattice mass matrix.  The flux on a triangle is
// linear in planar-face traces that are degree-N polynomials, so its
// lattice values and M_f give the cubature rule's integral exactly.
//
// The geometric factors are recomputed per node in FP64 from the five
// vertices (no stored per-node geometry).  The element's own traces at the
// stage start are those it wrote at the end of the previous stage, so they
// are read from the trace buffer rather than recomputed; the traces of the
// updated state are the products Fq u and Ft_f u.
//
// Operator tables: in the LDS (G = false), or, where they do not fit there
// (N = 5: D alone is 97 KiB), in global memory in fragment order (G = true):
// each (matrix, row tile, k-step) is 64 consecutive floats, one per lane, so
// a wavefront reads a fragment as one coalesced 256-byte load, and the
// fragments of one k-step lie together (one base address per step, the
// rest immediate offsets); a tile of 16 elements reads each fragment once,
// from the L2 after the first tiles.
#pragma once

#include "mfma_common.hpp"

namespace hdg {

// Jacobian matrix F[d][r] = dx_d/dxi_r of the pyramid map on the plane
// c = -1 at collapsed coordinates (a, b); V = 5 vertices (base 0..3, apex 4).
__device__ __forceinline__ void pyr_jacobian(const double (&V)[5][3], double a, double b, double F[3][3]) {
  const double sa[4] = {-1.0, 1.0, 1.0, -1.0}, sb[4] = {-1.0, -1.0, 1.0, 1.0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double X = 0.0, Xa = 0.0, Xb = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double fa = 0.5 * (1.0 + sa[v] * a), fb = 0.5 * (1.0 + sb[v] * b);
      X += fa * fb * V[v][d];
      Xa += 0.5 * sa[v] * fb * V[v][d];
      Xb += fa * 0.5 * sb[v] * V[v][d];
    }
    F[d][0] = Xa;
    F[d][1] = Xb;
    F[d][2] = 0.5 * (1.0 + a) * Xa + 0.5 * (1.0 + b) * Xb + 0.5 * (V[4][d] - X);
  }
}

// adj(F)[r][d] = J dxi_r/dx_d; returns J = det F.
__device__ __forceinline__ double adjugate(const double F[3][3], double A[3][3]) {
  A[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  A[0][1] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
  A[0][2] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
  A[1][0] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  A[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
  A[1][2] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
  A[2][0] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  A[2][1] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
  A[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  return F[0][0] * A[0][0] + F[0][1] * A[1][0] + F[0][2] * A[2][0];
}

template <int N, int NW, bool G = false>
struct PyrMfma {
  static constexpr int Np = (N + 1) * (N + 2) * (2 * N + 3) / 6;
  static constexpr int Nfn = (N + 1) * (N + 2) / 2;
  static constexpr int Nfq = (N + 1) * (N + 1);
  static constexpr int TS = trace_stride(N), LW = lattice_width(N);
  static constexpr int Mt = (Np + 15) / 16;   // row tiles over element nodes
  static constexpr int Ks = (Np + 3) / 4;     // k-steps over element nodes
  static constexpr int Mq = (Nfq + 15) / 16;  // row tiles over base-face points
  static constexpr int Kq = (Nfq + 3) / 4;    // k-steps over base-face points
  static constexpr int Kf = (Nfn + 3) / 4;    // k-steps over a triangle's lattice
  static constexpr int Mf = (Nfn + 15) / 16;  // row tiles over a triangle's lattice
  static constexpr int SD = Np | 1;           // odd strides: conflict-free fragment reads
  static constexpr int SX = Np | 1;
  static constexpr int SF = Nfq | 1;
  static constexpr int NT = 64 * NW;
  static constexpr int kLFloats = 4 * Mt * Kf * 64;
  // G = false: D [3][Np][SD], Fq [Nfq][SD], Ft [4][Nfn][SD] (row-major, copied
  // to the LDS as they are);
  // G = true: fragments [64] of D and D^T [Ks][2][3][Mt], the trace
  // operator [Ks][Mq + 4 Mf] (Fq's row tiles, then Ft_f's), Fq^T [Kq][Mt]
  // (k-step before row tile);
  // then in both: the Lt fragments ([4][Mt][Kf], with G [4][Kf][Mt]), w0, and
  // the geometry points (a, b) as doubles at an even float offset
  static constexpr int kOpsOpf = G ? 0 : (3 * Np + Nfq + 4 * Nfn) * SD;
  static constexpr int kDD = 0, kFW = kDD + 6 * Mt * Ks * 64;
  static constexpr int kFqT = kFW + (Mq + 4 * Mf) * Ks * 64, kFragEnd = kFqT + Kq * Mt * 64;
  static constexpr int kLtOff = G ? kFragEnd : kOpsOpf;
  static constexpr int kGabOff = (kLtOff + kLFloats + 2) & ~1;
  static constexpr int kOpsFloats = kGabOff + 4 * Np;
  static constexpr int kOpsInts = 2 * 8 * Nfq + 2 * 6 * Nfn;
  static constexpr int Q4 = 4 * Np;
  static constexpr int JQ = (Q4 + 63) / 64;
  static constexpr int JB = (Nfq + 3) / 4;  // base points q = g + 4 j per lane
  static constexpr int JF = (Nfn + 3) / 4;  // lattice nodes m = g + 4 j per lane

  struct Wave {
    float X[4][16][SX];  // state tile
    float F[4][16][SF];  // one face's weighted flux; staging of one output field
  };
  static_assert(4 * 16 * SF >= 16 * SX, "output staging does not fit the flux buffer");

  // LDS operator extents (a single float each when the tables stay in
  // global memory)
  static constexpr int LN = G ? 1 : Np, LS = G ? 1 : SD, LQ = G ? 1 : Nfq, LF = G ? 1 : Nfn;
  struct Smem {
    float D[3][LN][LS];
    float Fq[LQ][LS];
    float Ft[4][LF][LS];
    float Lt[G ? 1 : 4][G ? 1 : Mt][G ? 1 : Kf][G ? 1 : 64];
    double gab[Np][2];
    int qperm[8][Nfq], iqperm[8][Nfq];  // canonical <-> local base point
    int tperm[6][Nfn], itperm[6][Nfn];  // canonical <-> local lattice node
    float w0;                           // canonical triangle weight of point 0
    Wave w[NW];
  };

  // operator entry with zero outside [0, R) x [0, C)
  template <int R, int C, int S>
  __device__ __forceinline__ static float at(const float (*A)[S], int i, int j) {
    const bool in = i < R && j < C;
    return in ? A[in ? i : 0][in ? j : 0] : 0.f;
  }
  // With the tables in global memory, the fragments of a step are all issued
  // before its products: left to itself the scheduler (at the register
  // limit) puts each load next to its product, with one or two loads in
  // flight, and every product then waits a full L2 round trip.
  __device__ __forceinline__ static void loads_issued() {
    if constexpr (G) __builtin_amdgcn_sched_barrier(0);
  }
  // A loop over S k-steps whose body takes the M operator entries of its
  // step.  With the tables in global memory the entries of step s + 1 are
  // loaded while step s computes: the wait for a step's entries comes before
  // the next step's loads are issued (a wait placed after them would wait for
  // both).  With the tables in the LDS each step reads its own, unrolled U
  // times.
  template <int M, int U, class Load, class Body>
  __device__ __forceinline__ static void ksteps(int S, const Load& load, const Body& body) {
    if constexpr (G) {
      float cur[M];
#pragma unroll
      for (int m = 0; m < M; ++m) cur[m] = load(m, 0);
#pragma unroll 1
      for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int m = 0; m < M; ++m) __asm__ volatile("" : "+v"(cur[m]));
        loads_issued();
        const int sn = s + 1 < S ? s + 1 : s;
        float nxt[M];
#pragma unroll
        for (int m = 0; m < M; ++m) nxt[m] = load(m, sn);
        loads_issued();
        body(s, cur);
#pragma unroll
        for (int m = 0; m < M; ++m) cur[m] = nxt[m];
      }
    } else {
#pragma unroll U
      for (int s = 0; s < S; ++s) {
        float cur[M];
#pragma unroll
        for (int m = 0; m < M; ++m) cur[m] = load(m, s);
        body(s, cur);
      }
    }
  }
  // lane's A-operand entries of the operator fragments
  __device__ __forceinline__ static float frag(const StageArgs& a, int off, int lane) { return a.ops[off + lane]; }
  __device__ __forceinline__ static float opD(const Smem& sm, const StageArgs& a, int r, int t, int s, int lane) {
    if constexpr (G) return frag(a, kDD + ((2 * s * 3 + r) * Mt + t) * 64, lane);
    else return at<Np, Np, SD>(sm.D[r], 16 * t + (lane & 15), 4 * s + (lane >> 4));
  }
  __device__ __forceinline__ static float opDT(const Smem& sm, const StageArgs& a, int r, int t, int s, int lane) {
    if constexpr (G) return frag(a, kDD + (((2 * s + 1) * 3 + r) * Mt + t) * 64, lane);
    else return at<Np, Np, SD>(sm.D[r], 4 * s + (lane >> 4), 16 * t + (lane & 15));
  }
  __device__ __forceinline__ static float opFq(const Smem& sm, const StageArgs& a, int t, int s, int lane) {
    return at<Nfq, Np, SD>(sm.Fq, 16 * t + (lane & 15), 4 * s + (lane >> 4));
  }
  __device__ __forceinline__ static float opFqT(const Smem& sm, const StageArgs& a, int s, int t, int lane) {
    if constexpr (G) return frag(a, kFqT + (s * Mt + t) * 64, lane);
    else return at<Nfq, Np, SD>(sm.Fq, 4 * s + (lane >> 4), 16 * t + (lane & 15));
  }
  __device__ __forceinline__ static float opFt(const Smem& sm, const StageArgs& a, int tf, int t, int s, int lane) {
    return at<Nfn, Np, SD>(sm.Ft[tf], 16 * t + (lane & 15), 4 * s + (lane >> 4));
  }
  __device__ __forceinline__ static float opLt(const Smem& sm, const StageArgs& a, int tf, int t, int s, int lane) {
    if constexpr (G) return frag(a, kLtOff + ((tf * Kf + s) * Mt + t) * 64, lane);
    else return sm.Lt[tf][t][s][lane];
  }

  // ---- tile I/O (global [K][Np] per field <-> LDS [16][SX])
  __device__ __forceinline__ static bool contiguous(const StageArgs& a, int64_t e0) {
    return a.elist == nullptr && e0 + 16 <= a.n_items && ((a.K * Np) & 3) == 0;
  }
  __device__ __forceinline__ static void load_rows(float (*dst)[SX], const float* src, const StageArgs& a, int64_t e0, int lane) {
    for (int it = lane; it < 16 * Np; it += 64) {
      const int n = it / Np, k = it - n * Np;
      const int64_t e = item(a, e0 + n);
      dst[n][k] = e >= 0 ? src[e * Np + k] : 0.0f;
    }
  }
  __device__ __forceinline__ static void store_rows(float* dst, const float (*src)[SX], const StageArgs& a, int64_t e0, int lane) {
    for (int it = lane; it < 16 * Np; it += 64) {
      const int n = it / Np, k = it - n * Np;
      const int64_t e = item(a, e0 + n);
      if (e >= 0) dst[e * Np + k] = src[n][k];
    }
  }
  __device__ __forceinline__ static void put4(float (*dst)[SX], int q0, float4 v) {
    const float x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = q0 + i, n = q / Np;
      dst[n][q - n * Np] = x[i];
    }
  }
  __device__ __forceinline__ static float4 get4(const float (*src)[SX], int q0) {
    float x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = q0 + i, n = q / Np;
      x[i] = src[n][q - n * Np];
    }
    return make_float4(x[0], x[1], x[2], x[3]);
  }
  __device__ __forceinline__ static void load_field(float4 (&v)[JQ], const float* base, int64_t e0, int lane) {
    const float4* src = reinterpret_cast<const float4*>(base + e0 * Np);
#pragma unroll
    for (int j = 0; j < JQ; ++j)
      if (lane + 64 * j < Q4) v[j] = src[lane + 64 * j];
  }
  __device__ __forceinline__ static void put_field(float (*dst)[SX], const float4 (&v)[JQ], int lane) {
#pragma unroll
    for (int j = 0; j < JQ; ++j)
      if (lane + 64 * j < Q4) put4(dst, 4 * (lane + 64 * j), v[j]);
  }
  __device__ __forceinline__ static void store_tile(float* dst, const float (*src)[SX], const StageArgs& a, int64_t e0, int lane,
                                    bool contig) {
    if (contig) {
      float4* d4 = reinterpret_cast<float4*>(dst + e0 * Np);
#pragma unroll
      for (int j = 0; j < JQ; ++j)
        if (lane + 64 * j < Q4) d4[lane + 64 * j] = get4(src, 4 * (lane + 64 * j));
    } else {
      store_rows(dst, src, a, e0, lane);
    }
  }
  __device__ __forceinline__ static void load_state(Wave& W, const StageArgs& a, int64_t e0, int lane, bool contig) {
    const int64_t fs = a.K * Np;
    if (contig) {
      float4 v0[JQ], v1[JQ], v2[JQ], v3[JQ];
      load_field(v0, a.U, e0, lane);
      load_field(v1, a.U + fs, e0, lane);
      load_field(v2, a.U + 2 * fs, e0, lane);
      load_field(v3, a.U + 3 * fs, e0, lane);
      put_field(W.X[0], v0, lane);
      put_field(W.X[1], v1, lane);
      put_field(W.X[2], v2, lane);
      put_field(W.X[3], v3, lane);
    } else {
      for (int c = 0; c < 4; ++c) load_rows(W.X[c], a.U + (int64_t)c * fs, a, e0, lane);
    }
  }

  // ---- traces of the tile's state: base face at canonical GL points,
  // triangles at canonical lattice nodes.  One k-loop for all five faces:
  // row tiles u < Mq are the base face's (Fq), the others Mf per triangle
  // (Ft_f), so each state entry is read from the LDS once per step and a step
  // has 4 (Mq + 4 Mf) independent products.
  static constexpr int MW = Mq + 4 * Mf;
  __device__ __forceinline__ static float opW(const Smem& sm, const StageArgs& a, int u, int s, int lane) {
    if constexpr (G) return frag(a, kFW + (s * MW + u) * 64, lane);
    else if (u < Mq) return opFq(sm, a, u, s, lane);
    else return opFt(sm, a, (u - Mq) / Mf, (u - Mq) % Mf, s, lane);
  }
  __device__ __forceinline__ static void write_traces(const Smem& sm, const Wave& W, const StageArgs& a, int64_t e0,
                                                      int lane, float4* tr) {
    const int n = lane & 15, g = lane >> 4;
    const int64_t e = item(a, e0 + n);
    const int64_t slot = a.slot0 + (e >= 0 ? e : 0) * 5;
    f32x4 acc[MW][4];
#pragma unroll
    for (int u = 0; u < MW; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[u][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    ksteps<MW, 2>(
        Ks, [&](int u, int s) { return opW(sm, a, u, s, lane); },
        [&](int s, const float(&af)[MW]) {
          const int k = 4 * s + g;
          const bool in = k < Np;
          const int kk = in ? k : 0;
          float b[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) b[c] = in ? W.X[c][n][kk] : 0.f;
#pragma unroll
          for (int u = 0; u < MW; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[u][c] = mma_f32(af[u], b[c], acc[u][c]);
        });
    if (e < 0) return;
    int ori[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) ori[f] = a.ori[slot + f];
#pragma unroll
    for (int u = 0; u < MW; ++u) {
      const int f = u < Mq ? 0 : 1 + (u - Mq) / Mf;
      const int t = u < Mq ? u : (u - Mq) % Mf;
      float4* dst = tr + (slot + f) * TS;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int l = 16 * t + 4 * g + i;
        const float4 v = make_float4(acc[u][0][i], acc[u][1][i], acc[u][2][i], acc[u][3][i]);
        if (f == 0) {
          if (l < Nfq) dst[sm.iqperm[ori[0]][l]] = v;
          else if (l < TS) dst[l] = make_float4(0.f, 0.f, 0.f, 0.f);  // padding to whole lines
        } else {
          if (l < Nfn) dst[sm.itperm[ori[f]][l]] = v;
          else if (l < LW) dst[l] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
    }
  }

  // a triangle's own and neighbour lattice traces and its face factors
  struct TriIn {
    float4 own[JF], pv[JF], gf;
  };
  __device__ __forceinline__ static void load_tri(const StageArgs& a, int64_t e, int64_t slot0, int tf, int nb,
                                                  bool mid, int g, TriIn& x) {
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t slot = slot0 + 1 + tf;
    const float4* nsrc = mid ? a.tr_half : a.tr_in;
    float4 gf = z4;
    if (e >= 0) gf = a.fgeo[(slot - a.slot0) * Nfq];
#pragma unroll
    for (int j = 0; j < JF; ++j) {
      const int m = g + 4 * j;
      float4 own = z4, pv = z4;
      if (e >= 0 && m < Nfn) {
        own = a.tr_in[slot * TS + m];
        if (nb >= 0) pv = nsrc[(int64_t)nb * TS + m];
      }
      x.own[j] = own;
      x.pv[j] = pv;
    }
    x.gf = gf;
  }

  // vertices of element e (a reference pyramid for e < 0, keeping the
  // geometry of unused columns finite)
  __device__ __forceinline__ static void load_verts5(const StageArgs& a, int64_t e, double (&V)[5][3]) {
    const double ref[5][3] = {{-1, -1, 0}, {1, -1, 0}, {1, 1, 0}, {-1, 1, 0}, {0, 0, 1}};
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) V[v][d] = e >= 0 ? a.V[(e * 5 + v) * 3 + d] : ref[v][d];
  }

  template <int C>
  __device__ __forceinline__ static void emit(Wave& W, const StageArgs& a, int64_t e0, int lane, bool contig, const float4 (&rv)[JQ],
                              const f32x4 (&rhs)[Mt], float* hist) {
    const int64_t K = a.K;
    const int n = lane & 15, g = lane >> 4;
    const bool stage = a.mode == kModeStage;
    float(*RB)[SX] = reinterpret_cast<float(*)[SX]>(&W.F[0][0][0]);
    if (stage) {
      if (contig && !G) {
        put_field(RB, rv, lane);
      } else if (contig) {
        float4 v[JQ];
        load_field(v, a.R + (int64_t)C * K * Np, e0, lane);
        put_field(RB, v, lane);
      } else {
        load_rows(RB, a.R + (int64_t)C * K * Np, a, e0, lane);
      }
      wave_sync();
    }
#pragma unroll
    for (int t = 0; t < Mt; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * t + 4 * g + i;
        if (row >= Np) continue;
        if (stage) {
          const float res = a.a * RB[n][row] + a.dt * rhs[t][i];
          RB[n][row] = res;
          W.X[C][n][row] += a.b * res;
        } else {
          RB[n][row] = rhs[t][i];
        }
      }
    wave_sync();
    if (a.mode == kModeRhsHist && hist) {
      store_tile(hist + (int64_t)C * K * Np, RB, a, e0, lane, true);
    } else if (a.mode == kModeRhsHist) {
      for (int it = lane; it < 16 * Np; it += 64) {
        const int nn = it / Np, k = it - nn * Np;
        const int64_t ee = item(a, e0 + nn);
        if (ee >= 0) rhs_dst(a, ee, Np)[(int64_t)C * K * Np + ee * Np + k] = RB[nn][k];
      }
    } else {
      store_tile(a.R + (int64_t)C * K * Np, RB, a, e0, lane, contig);
    }
    if (stage) store_tile(a.U + (int64_t)C * K * Np, W.X[C], a, e0, lane, contig);
    wave_sync();
  }

  // Multi-rate AB3 update of a tile: u_new = u + dtau_l sum_j beta_j(1) r_j
  // (state and traces) and, when an element of the tile has a finer
  // neighbour, the mid-step state u + dtau_l sum_j beta_j(1/2) r_j (traces
  // only).  A contiguous tile of one level reads u and the history once, as
  // vectors; otherwise each value is combined on its own, the mid-step state
  // first (u is still the old state then).
  __device__ __forceinline__ static void mrab(const Smem& sm, Wave& W, const StageArgs& a, int64_t e0, int lane,
                                              bool contig) {
    const int64_t K = a.K, fs = K * Np, hstr = 4 * fs;
    bool hf = false;
    {
      const int64_t e = item(a, e0 + (lane & 15));
      hf = e >= 0 && a.ehalf[e] != 0;
    }
    const bool half = __ballot(hf) != 0;
    if (contig && a.elevel[e0] == a.elevel[e0 + 15]) {
      const int lv = a.elevel[e0];
      const float dtl = a.mr.dtl[lv];
      float b1[3], bh[3];
      const float* hj[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        b1[j] = a.mr.b1[lv][j];
        bh[j] = a.mr.bh[lv][j];
        hj[j] = a.H + a.mr.hs[lv][j] * hstr;
      }
      float4 mid[4][JQ];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float4 u[JQ], h0[JQ], h1[JQ], h2[JQ];
        load_field(u, a.U + c * fs, e0, lane);
        load_field(h0, hj[0] + c * fs, e0, lane);
        load_field(h1, hj[1] + c * fs, e0, lane);
        load_field(h2, hj[2] + c * fs, e0, lane);
        float4 un[JQ];
#pragma unroll
        for (int j = 0; j < JQ; ++j) {
          if (lane + 64 * j >= Q4) continue;
          const float4 x = u[j], p = h0[j], q = h1[j], r = h2[j];
          un[j] = make_float4(x.x + dtl * (b1[0] * p.x + b1[1] * q.x + b1[2] * r.x),
                              x.y + dtl * (b1[0] * p.y + b1[1] * q.y + b1[2] * r.y),
                              x.z + dtl * (b1[0] * p.z + b1[1] * q.z + b1[2] * r.z),
                              x.w + dtl * (b1[0] * p.w + b1[1] * q.w + b1[2] * r.w));
          mid[c][j] = make_float4(x.x + dtl * (bh[0] * p.x + bh[1] * q.x + bh[2] * r.x),
                                  x.y + dtl * (bh[0] * p.y + bh[1] * q.y + bh[2] * r.y),
                                  x.z + dtl * (bh[0] * p.z + bh[1] * q.z + bh[2] * r.z),
                                  x.w + dtl * (bh[0] * p.w + bh[1] * q.w + bh[2] * r.w));
          reinterpret_cast<float4*>(a.U + c * fs + e0 * Np)[lane + 64 * j] = un[j];
        }
        put_field(W.X[c], un, lane);
      }
      wave_sync();
      write_traces(sm, W, a, e0, lane, a.tr_out);
      if (!half) return;
      wave_sync();  // the traces have read the tile
#pragma unroll
      for (int c = 0; c < 4; ++c) put_field(W.X[c], mid[c], lane);
      wave_sync();
      write_traces(sm, W, a, e0, lane, a.tr_half);
      return;
    }
    for (int pass = half ? 0 : 1; pass < 2; ++pass) {
      const bool m = pass == 0;  // mid-step state first, then the new state
#pragma unroll 1
      for (int it = lane; it < 4 * 16 * Np; it += 64) {
        const int c = it / (16 * Np), r = it - c * 16 * Np;
        const int nn = r / Np, k = r - nn * Np;
        const int64_t ee = item(a, e0 + nn);
        float v = 0.f;
        if (ee >= 0) {
          const int lv = a.elevel[ee];
          const float* w = m ? a.mr.bh[lv] : a.mr.b1[lv];
          const int64_t gi = c * fs + ee * Np + k;
          const float acc = w[0] * a.H[a.mr.hs[lv][0] * hstr + gi] + w[1] * a.H[a.mr.hs[lv][1] * hstr + gi] +
                            w[2] * a.H[a.mr.hs[lv][2] * hstr + gi];
          v = a.U[gi] + a.mr.dtl[lv] * acc;
          if (!m) a.U[gi] = v;
        }
        W.X[c][nn][k] = v;
      }
      wave_sync();
      write_traces(sm, W, a, e0, lane, m ? a.tr_half : a.tr_out);
      wave_sync();
    }
  }

  // One tile: the multi-rate update (MR), or the stage, right-hand-side and
  // trace modes.
  template <bool MR>
  __device__ __forceinline__ static void tile(const Smem& sm, Wave& W, const StageArgs& a, int64_t e0, int lane) {
    const bool contig = contiguous(a, e0);
    // lanes of the previous tile may still read other columns of the tile
    wave_sync();
    if constexpr (MR) {
      mrab(sm, W, a, e0, lane, contig);
      return;
    }
    load_state(W, a, e0, lane, contig);
    wave_sync();
    if (a.mode != kModeTrace) rhs(sm, W, a, e0, lane, contig);
    // traces of the (updated) state, from one call site: the code of a tile
    // has to stay small enough for the instruction cache
    if (a.mode == kModeTrace || a.mode == kModeStage) write_traces(sm, W, a, e0, lane, a.tr_out);
  }

  __device__ __forceinline__ static void rhs(const Smem& sm, Wave& W, const StageArgs& a, int64_t e0, int lane,
                                             bool contig) {
    const int64_t K = a.K;
    const int n = lane & 15, g = lane >> 4;
    const int64_t e = item(a, e0 + n);
    double V[5][3];
    load_verts5(a, e, V);
    float kap = 0.f, irho = 0.f;
    if (e >= 0) {
      kap = a.mat[e].x;
      irho = a.mat[e].y;
    }
    // face records (neighbour or boundary code, orientation, penalties, and
    // whether the neighbour's traces are the mid-step ones), read now so that
    // their latency passes during the volume products
    const int64_t slot0 = a.slot0 + (e >= 0 ? e : 0) * 5;
    int rnb[5], rori[5];
    bool rmid[5];
    float2 rtau[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      rnb[f] = -1;
      rori[f] = 0;
      rmid[f] = false;
      rtau[f] = make_float2(0.f, 0.f);
      if (e >= 0) {
        rnb[f] = a.nbr[slot0 + f];
        rori[f] = a.ori[slot0 + f];
        rtau[f] = a.tau[slot0 + f];
        if (rnb[f] >= 0) rmid[f] = neighbour_mid(a, slot0 + f, rnb[f]);
      }
    }
    // volume: grad = D^r p, div = sum_r (D^r)^T U^r
    f32x4 accG[3][Mt], accV[Mt];
#pragma unroll
    for (int t = 0; t < Mt; ++t) {
      accV[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 3; ++r) accG[r][t] = accV[t];
    }
    // operator entries one step ahead (with the tables in global memory their
    // latency then overlaps a whole step of products)
    float fd[3][Mt], fdt[3][Mt];
#pragma unroll
    for (int t = 0; t < Mt; ++t)
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        fd[r][t] = opD(sm, a, r, t, 0, lane);
        fdt[r][t] = opDT(sm, a, r, t, 0, lane);
      }
#pragma unroll 2
    for (int s = 0; s < Ks; ++s) {
      const int k = 4 * s + g;
      const bool in = k < Np;
      const int kk = in ? k : 0;
      float nd[3][Mt], ndt[3][Mt];
      const int sn = s + 1 < Ks ? s + 1 : s;  // (the last step reads its own entries again)
      if constexpr (G) {
        // this step's entries are waited for here, before the next step's
        // loads are issued (a wait placed after them would wait for both)
#pragma unroll
        for (int t = 0; t < Mt; ++t)
#pragma unroll
          for (int r = 0; r < 3; ++r) __asm__ volatile("" : "+v"(fd[r][t]), "+v"(fdt[r][t]));
        loads_issued();
      }
#pragma unroll
      for (int t = 0; t < Mt; ++t)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          nd[r][t] = opD(sm, a, r, t, sn, lane);
          ndt[r][t] = opDT(sm, a, r, t, sn, lane);
        }
      loads_issued();
      double F[3][3], A[3][3];
      pyr_jacobian(V, sm.gab[kk][0], sm.gab[kk][1], F);
      adjugate(F, A);
      const float p = in ? W.X[0][n][kk] : 0.f;
      const float u1 = W.X[1][n][kk], u2 = W.X[2][n][kk], u3 = W.X[3][n][kk];
      float ur[3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
        ur[r] = in ? (float)A[r][0] * u1 + (float)A[r][1] * u2 + (float)A[r][2] * u3 : 0.f;
#pragma unroll
      for (int t = 0; t < Mt; ++t)
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          accG[r][t] = mma_f32(fd[r][t], p, accG[r][t]);
          accV[t] = mma_f32(fdt[r][t], ur[r], accV[t]);
          fd[r][t] = nd[r][t];
          fdt[r][t] = ndt[r][t];
        }
    }
    // surface-term accumulators start from the volume terms, scaled so that
    // rhs_p = kappa/J (S_p) and rhs_u = (1/rho)/J (S_u):
    //   S_p = sum_r (D^r)^T U^r,  S_u_d = -sum_r adj(F)_rd [D^r p]
    f32x4 accS[4][Mt];
#pragma unroll
    for (int t = 0; t < Mt; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * t + 4 * g + i;
        double F[3][3], A[3][3];
        const int rr = row < Np ? row : 0;
        pyr_jacobian(V, sm.gab[rr][0], sm.gab[rr][1], F);
        adjugate(F, A);
        accS[0][t][i] = accV[t][i];
#pragma unroll
        for (int d = 0; d < 3; ++d)
          accS[1 + d][t][i] = -((float)A[0][d] * accG[0][t][i] + (float)A[1][d] * accG[1][t][i] +
                                (float)A[2][d] * accG[2][t][i]);
        // one row's FP64 geometry at a time (interleaved, the rows' temporaries
        // would exceed the registers)
        __builtin_amdgcn_sched_barrier(0);
      }
    // the residual of the stage, fetched while the faces are processed
    const bool stage = a.mode == kModeStage;
    // (not with the tables in global memory: there the registers hold the
    // larger tiles, and each field's residual is read when it is emitted)
    float4 rv0[JQ], rv1[JQ], rv2[JQ], rv3[JQ];
    if (!G && stage && contig) {
      const int64_t fs = K * Np;
      load_field(rv0, a.R, e0, lane);
      load_field(rv1, a.R + fs, e0, lane);
      load_field(rv2, a.R + 2 * fs, e0, lane);
      load_field(rv3, a.R + 3 * fs, e0, lane);
    }
    // surface term S.  The trace loads of the base face and of the first
    // triangle are issued together; each triangle's are issued before the
    // previous triangle is processed.
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 bown[JB], bpv[JB], bg[JB];
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      const int q = g + 4 * j;
      bown[j] = bpv[j] = bg[j] = z4;
      if (e >= 0 && q < Nfq) {
        bown[j] = a.tr_in[slot0 * TS + q];
        bg[j] = a.fgeo[(slot0 - a.slot0) * Nfq + q];
        if (rnb[0] >= 0) bpv[j] = (rmid[0] ? a.tr_half : a.tr_in)[(int64_t)rnb[0] * TS + q];
      }
    }
    TriIn tri[2];  // (indexed by the unrolled face counter: registers, not memory)
    load_tri(a, e, slot0, 0, rnb[1], rmid[1], g, tri[0]);
    // base face: weighted flux at local GL points, then Fq^T
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      const int q = g + 4 * j;
      if (q >= Nfq) continue;
      float out[4] = {0.f, 0.f, 0.f, 0.f};
      int l = q;
      if (e >= 0) {
        l = sm.qperm[rori[0]][q];
        const float4 p = rnb[0] >= 0 ? bpv[j] : mirror_state(bown[j], -rnb[0] - 1, bg[j].x, bg[j].y, bg[j].z);
        upwind_flux(bown[j], p, bg[j], rtau[0], true, out);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) W.F[c][n][l] = out[c];
    }
    wave_sync();
    ksteps<Mt, 1>(
        Kq, [&](int t, int s) { return opFqT(sm, a, s, t, lane); },
        [&](int s, const float(&af)[Mt]) {
          const int k = 4 * s + g;
          const bool in = k < Nfq;
          const int kk = in ? k : 0;
          float b[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) b[c] = in ? W.F[c][n][kk] : 0.f;
#pragma unroll
          for (int t = 0; t < Mt; ++t)
#pragma unroll
            for (int c = 0; c < 4; ++c) accS[c][t] = mma_f32(af[t], b[c], accS[c][t]);
        });
    wave_sync();
    // triangular faces: J^s-weighted flux at local lattice nodes, then Ft^T M_f
#pragma unroll
    for (int tf = 0; tf < 4; ++tf) {
      if (tf < 3) load_tri(a, e, slot0, tf + 1, rnb[tf + 2], rmid[tf + 2], g, tri[(tf + 1) & 1]);
      const TriIn& cur = tri[tf & 1];
      const int nb = rnb[1 + tf];
      float4 gf = cur.gf;
      gf.w /= sm.w0;  // J^s (the stored value carries the weight of point 0)
#pragma unroll
      for (int j = 0; j < JF; ++j) {
        const int m = g + 4 * j;
        if (m >= Nfn) continue;
        float out[4] = {0.f, 0.f, 0.f, 0.f};
        int l = m;
        if (e >= 0) {
          const float4 p = nb >= 0 ? cur.pv[j] : mirror_state(cur.own[j], -nb - 1, gf.x, gf.y, gf.z);
          l = sm.tperm[rori[1 + tf]][m];
          upwind_flux(cur.own[j], p, gf, rtau[1 + tf], true, out);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) W.F[c][n][l] = out[c];
      }
      wave_sync();
      ksteps<Mt, Kf>(
          Kf, [&](int t, int s) { return opLt(sm, a, tf, t, s, lane); },
          [&](int s, const float(&lf)[Mt]) {
            const int k = 4 * s + g;
            const bool in = k < Nfn;
            const int kk = in ? k : 0;
            float b[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = in ? W.F[c][n][kk] : 0.f;
#pragma unroll
            for (int t = 0; t < Mt; ++t)
#pragma unroll
              for (int c = 0; c < 4; ++c) accS[c][t] = mma_f32(lf[t], b[c], accS[c][t]);
          });
      wave_sync();
    }
    // right-hand side at rows 16 t + 4 g + i (overwrites accS); 1/J from the
    // vertices again (cheaper than keeping it live across the faces: the
    // opaque copies keep the compiler from reusing the first evaluation)
    load_verts5(a, e, V);
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) __asm__ volatile("" : "+v"(V[v][d]));
#pragma unroll
    for (int t = 0; t < Mt; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * t + 4 * g + i;
        const int rr = row < Np ? row : 0;
        double F[3][3], A[3][3];
        pyr_jacobian(V, sm.gab[rr][0], sm.gab[rr][1], F);
        const float iJ = (float)(1.0 / adjugate(F, A));
        const float sp = kap * iJ, su = irho * iJ;
        accS[0][t][i] *= sp;
#pragma unroll
        for (int d = 0; d < 3; ++d) accS[1 + d][t][i] *= su;
        __builtin_amdgcn_sched_barrier(0);
      }
    // a multi-rate launch without an item list has its elements stored finest
    // level first, so equal levels at both ends of a contiguous tile mean one
    // level: its history slot takes the tile as float4 vectors
    float* hist = nullptr;
    if (a.mode == kModeRhsHist && contig) {
      const int lv = a.elevel[e0];
      if (a.elevel[e0 + 15] == lv) hist = a.H + (int64_t)a.mr.hs[lv][0] * 4 * K * Np;
    }
    emit<0>(W, a, e0, lane, contig, rv0, accS[0], hist);
    emit<1>(W, a, e0, lane, contig, rv1, accS[1], hist);
    emit<2>(W, a, e0, lane, contig, rv2, accS[2], hist);
    emit<3>(W, a, e0, lane, contig, rv3, accS[3], hist);
  }

  template <bool MR>
  __device__ __forceinline__ static void run(Smem& sm, const StageArgs& a) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if constexpr (!G) {
      float* dst = &sm.D[0][0][0];
      for (int i = tid; i < kOpsOpf; i += NT) dst[i] = a.ops[i];  // D, Fq, Ft are contiguous in Smem
      float* lt = &sm.Lt[0][0][0][0];
      for (int i = tid; i < kLFloats; i += NT) lt[i] = a.ops[kOpsOpf + i];
    }
    if (tid == 0) sm.w0 = a.ops[kLtOff + kLFloats];
    const double* gab = reinterpret_cast<const double*>(a.ops + kGabOff);
    for (int i = tid; i < 2 * Np; i += NT) (&sm.gab[0][0])[i] = gab[i];
    int* ip = &sm.qperm[0][0];
    for (int i = tid; i < kOpsInts; i += NT) ip[i] = a.iops[i];  // qperm, iqperm, tperm, itperm contiguous
    float* wz = &sm.w[0].X[0][0][0];
    for (int i = tid; i < (int)(NW * sizeof(Wave) / sizeof(float)); i += NT) wz[i] = 0.f;
    __syncthreads();
    Wave& W = sm.w[wv];
    const int64_t ntile = (a.n_items + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * NW + wv; t < ntile; t += (int64_t)gridDim.x * NW) {
      // an opaque copy of the lane index keeps the lane-dependent indices
      // inside the loop (hoisted out of it, they would stay live in
      // registers across the whole tile)
      int ln = lane;
      if constexpr (G) __asm__ volatile("" : "+v"(ln));
      tile<MR>(sm, W, a, t * 16, ln);
    }
  }
};

}  // namespace hdg
