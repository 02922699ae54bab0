// C ABI of the hybrid-mesh DG solver (declared in include/hdg.h).
//
// hdg_create does all set-up: FP64 reference operators on the host, face
// matching and canonical orientations, upload, FP64 geometry on the device,
// FP32 operator tables.  The hot path is hdg_step: per Runge-Kutta stage one
// fused kernel per element type, traces double-buffered between stages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/hdg.h"
#include "kernels.hpp"
#include "refel.hpp"

using namespace hdg;

namespace {

thread_local std::string g_create_error;

// Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage RK.
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

struct TypeData {
  int present = 0;
  int64_t K = 0;
  // Field stride in elements: K rounded up to a multiple of 4, so that each
  // of the four fields of U, R and H starts 16-byte aligned and element tiles
  // move as float4 vectors whatever K is (the pad elements stay zero).
  int64_t Ks = 0;
  int Np = 0, nf = 0, nv = 0, nsample = 0, nvp = 0;
  std::vector<int64_t> elems;  // global element ids in mesh order
  int64_t slot0 = 0;
  float* U = nullptr;
  float* R = nullptr;
  float* geo = nullptr;
  float2* mat = nullptr;
  float4* fgeo = nullptr;
  float* isqJ = nullptr;
  double* V = nullptr;         // [K][nv][3]
  float* ops = nullptr;
  int* iops = nullptr;
  float* mops = nullptr;       // matrix-core kernel tables (tetrahedra, pyramids)
  int* miops = nullptr;
  double* spts = nullptr;      // sample reference points [nsample][3]
  double* sw = nullptr;        // sample weights (wedge, pyramid)
  double* Phi = nullptr;       // basis at sample points (wedge, pyramid)
  double* gpts = nullptr;      // pyramid geometry points [Np][3]
  double* Mhat = nullptr;      // tet reference mass
  std::vector<double> cJ, minJ, crk;
  std::vector<double> ctk;      // computed trace constant C_T(N, K) per element (empty until computed)
  // multi-rate
  int* elist = nullptr;        // elements sorted by level, finest first
  bool elist_identity = false; // the sorted order is the storage order (no indirection needed)
  int8_t* elevel = nullptr;    // level per element
  int8_t* ehalf = nullptr;     // 1: a face neighbour is on a finer level (reads the mid-step traces)
  float* H = nullptr;          // right-hand-side history [3][4][Ks][Np]
  int64_t n_from[10] = {};     // number of elements with level >= l
};

}  // namespace

struct hdg_ctx {
  int N = 0;
  hipStream_t stream = nullptr;
  std::string err;
  FaceTables ft;
  HexRef hex;
  TetRef tet;
  WedgeRef wedge;
  PyrRef pyr;
  TypeData td[4];
  int64_t n_elem = 0;
  int64_t nslot = 0;
  int* nbr = nullptr;
  int8_t* ori = nullptr;
  float2* tau = nullptr;
  float4* trace[2] = {nullptr, nullptr};
  int cur = 0;
  bool traces_valid = false;
  bool lattice_ok = false;     // no triangular face joins a wedge to a tet or pyramid
  int path = HDG_PATH_AUTO;
  int prec = HDG_PREC_FP32;    // operand precision of the matrix-core products
  int max_blocks = 256;        // cap of persistent matrix-core grids (one block per compute unit)
  int epb[4] = {0, 0, 0, 0};   // elements per block of the block kernels (0: default; hdg_autotune)
  GeoTables* gtab = nullptr;
  double* partial = nullptr;
  int* flag = nullptr;
  std::vector<void*> allocs;
  bool prof = false;
  // host copies of the connectivity (multi-rate binning)
  std::vector<int64_t> slot_elem_h;
  std::vector<int> nbr_h;
  std::vector<int> etype_h, eidx_h;
  // multi-rate state
  int L = 0;
  double mr_dtmin = 0.0;
  int8_t* slevel = nullptr;
  int64_t hcount[10] = {};
  bool mr_ready = false;
  std::vector<std::array<hipEvent_t, 2>> ev_pool;
  std::vector<int> ev_type;
  size_t ev_used = 0;
  double time = 0.0;           // simulated time of the state
  double mr_dtmin0 = 0.0;      // dtau_min of hdg_mrab_setup (hdg_advance may scale it down)
  std::vector<int8_t> level_h; // multi-rate level per element (mesh order)
  std::vector<int8_t> half_h;  // 1: the element writes mid-step traces (mesh order)
  int dt_mode = HDG_DT_REFERENCE;  // local steps from the reference or the per-element trace constants
  // captured graph of two LSERK4 steps (ten stages, so the trace buffers
  // come back to the captured parity) for hdg_step_graph
  hipGraphExec_t graph = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream the graph is captured on
  double graph_dt = 0.0;
  int graph_cur = -1, graph_path = -1;
  double* pscratch = nullptr;  // fixed work buffer of hdg_project_noalloc on this context's GPU
  // 1:4 non-conforming faces: slots [nslot0, nslot0 + 4 n_nc) are the
  // virtual slots (the coarse trace at a sub-face, read by the fine
  // element), then n_nc flux slots (the coarse face's flux)
  int64_t n_nc = 0;
  int64_t nslot0 = 0;
  int* ncrec = nullptr;        // [n_nc][kNcRec]
  float* ncI = nullptr;        // [nvar][Nfn][Nfn]
  float* ncP = nullptr;        // [nvar][Nfn][Nfn]
  std::vector<std::array<int64_t, 4>> nc_fine_elems;  // elements on the sub-faces of each coarse face
};

namespace {

int fail(hdg_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_error = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(ctx, HDG_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

template <class T>
int dalloc(hdg_ctx* c, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return fail(c, HDG_ENOMEM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  c->allocs.push_back((void*)*p);
  return HDG_OK;
}

template <class T>
int upload(hdg_ctx* c, T** p, const std::vector<T>& h) {
  int rc = dalloc(c, p, h.size());
  if (rc) return rc;
  if (!h.empty()) {
    HIPCHK(c, hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));  // h is pageable and may be released by the caller
  }
  return HDG_OK;
}

std::vector<float> to_f(const Vec& v) { return std::vector<float>(v.begin(), v.end()); }

void append(std::vector<float>& dst, const Vec& v) {
  for (double x : v) dst.push_back((float)x);
}

int build_tables(hdg_ctx* c, int t, std::vector<float>& ops, std::vector<int>& iops) {
  const int N = c->N;
  const FaceTables& ft = c->ft;
  ops.clear();
  iops.clear();
  if (t == kHex) {
    append(ops, c->hex.D1);
    append(ops, c->hex.Lm);
    append(ops, c->hex.Lp);
    iops.insert(iops.end(), ft.quad_perm.begin(), ft.quad_perm.end());
  } else if (t == kTet) {
    const TetRef& T = c->tet;
    append(ops, T.Dr);
    append(ops, T.Ds);
    append(ops, T.Dt);
    append(ops, T.Minv);
    append(ops, ft.Ican);
    append(ops, ft.tri_w);
    iops.insert(iops.end(), T.fnode.begin(), T.fnode.end());
    iops.insert(iops.end(), ft.tri_perm.begin(), ft.tri_perm.end());
    std::vector<int> nodeface(4 * T.Np, -1);
    for (int f = 0; f < 4; ++f)
      for (int m = 0; m < ft.Nfn; ++m) nodeface[f * T.Np + T.fnode[f * ft.Nfn + m]] = m;
    iops.insert(iops.end(), nodeface.begin(), nodeface.end());
  } else if (t == kPyr) {
    const PyrRef& P = c->pyr;
    append(ops, P.Dr);
    append(ops, P.Ds);
    append(ops, P.Dt);
    append(ops, P.Fquad);
    append(ops, P.Ftri);
    append(ops, ft.Ican);
    // face-lattice mass matrix M_f = Ican^T W Ican over the weight of
    // cubature point 0 (the kernels' face factor carries w_0 J^s)
    for (int x = 0; x < ft.Nfn; ++x)
      for (int y = 0; y < ft.Nfn; ++y) {
        double v = 0.0;
        for (int q = 0; q < ft.Nfq; ++q) v += ft.Ican[q * ft.Nfn + x] * ft.tri_w[q] * ft.Ican[q * ft.Nfn + y];
        ops.push_back((float)(v / ft.tri_w[0]));
      }
    iops.insert(iops.end(), ft.quad_perm.begin(), ft.quad_perm.end());
    iops.insert(iops.end(), ft.tri_perm.begin(), ft.tri_perm.end());
  } else {
    const WedgeRef& W = c->wedge;
    for (size_t i = 0; i < W.Pt.size(); ++i) {
      ops.push_back((float)W.Pt[i]);
      ops.push_back((float)W.Ptr[i]);
      ops.push_back((float)W.Ptt[i]);
      ops.push_back(0.f);
    }
    append(ops, W.tri_w);
    append(ops, W.P1);
    append(ops, W.dP1);
    Vec x1, w1;
    gauss_jacobi(N + 1, 0.0, 0.0, x1, w1);
    append(ops, w1);
    append(ops, W.P1m);
    append(ops, W.P1p);
    append(ops, W.Ftri);
    append(ops, W.Fedge);
    append(ops, ft.Ican);
    iops.insert(iops.end(), ft.quad_perm.begin(), ft.quad_perm.end());
    iops.insert(iops.end(), ft.tri_perm.begin(), ft.tri_perm.end());
  }
  int nf = 0, ni = 0;
  stage_table_sizes(t, N, &nf, &ni);
  if ((int)ops.size() != nf || (int)iops.size() != ni)
    return fail(c, HDG_EINVAL, "internal: operator table size mismatch for type " + std::to_string(t));
  return HDG_OK;
}

// BF16 rounding (nearest, ties to even) of a finite float, as its bits.
uint16_t bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
double bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

// MFMA A-fragments of a row-major R x C matrix, appended to out: for each
// 16-row tile t and k-step s (K = kk per instruction), piece pc and lane l,
// the ki entries A[16t + l%16][kk s + ki (l/16) + i] (0 outside the matrix).
// Precision 0 stores FP32 values; otherwise x = sc A is stored as npc pieces,
// each the FP16 (P = 1, 2) or BF16 (P = 3, 4) rounding of what the previous
// pieces leave: hi = r(x), lo = r(x - hi) (and, three pieces, mid, lo).
void pack_frags(const double* A, int R, int C, int P, double sc, std::vector<float>& out) {
  int kk, ki, npc;
  tet_mfma_frag_shape(P, &kk, &ki, &npc);
  const int Mt = (R + 15) / 16, Ks = (C + kk - 1) / kk;
  auto at = [&](int t, int s, int l, int i) {
    const int row = 16 * t + l % 16, col = kk * s + ki * (l / 16) + i;
    return row < R && col < C ? A[(size_t)row * C + col] : 0.0;
  };
  if (P == 0) {
    for (int t = 0; t < Mt; ++t)
      for (int s = 0; s < Ks; ++s)
        for (int l = 0; l < 64; ++l) out.push_back((float)at(t, s, l, 0));
    return;
  }
  std::vector<uint16_t> h;
  for (int t = 0; t < Mt; ++t)
    for (int s = 0; s < Ks; ++s)
      for (int pc = 0; pc < npc; ++pc)
        for (int l = 0; l < 64; ++l)
          for (int i = 0; i < ki; ++i) {
            double x = at(t, s, l, i) * sc;
            uint16_t bits = 0;
            for (int q = 0; q <= pc; ++q) {
              if (P == 3 || P == 4) {
                bits = bf16_bits((float)x);
                x -= bf16_value(bits);
              } else {
                const _Float16 v = (_Float16)x;
                std::memcpy(&bits, &v, 2);
                x -= (double)v;
              }
            }
            h.push_back(bits);
          }
  const size_t o = out.size();
  out.resize(o + h.size() / 2);
  std::memcpy(out.data() + o, h.data(), h.size() * 2);
}

// Packs nmat consecutive R x C matrices with one scale for the group (a power
// of two bringing the group maximum into [2^13, 2^14)); returns 1/scale.
double pack_group(const std::vector<double>& all, int nmat, int R, int C, int P, std::vector<float>& out) {
  double sc = 1.0;
  if (P != 0) {
    double m = 0.0;
    for (double v : all) m = std::max(m, std::fabs(v));
    int e = 0;
    std::frexp(m > 0.0 ? m : 1.0, &e);
    sc = std::ldexp(1.0, 14 - e);
  }
  for (int k = 0; k < nmat; ++k) pack_frags(all.data() + (size_t)k * R * C, R, C, P, sc, out);
  return 1.0 / sc;
}

// Tables of the matrix-core tetrahedron kernel: D^{r,s,t} and the lattice
// lift matrices L_f = M^-1 E_f M_f as MFMA fragments of precision P, where
// M_f = Ican^T W Ican is the mass matrix of the face lattice (exact: the
// canonical rule integrates degree 2N on the triangle).
int build_tet_mfma_tables(hdg_ctx* c, int P, std::vector<float>& ops, std::vector<int>& iops) {
  const TetRef& T = c->tet;
  const FaceTables& ft = c->ft;
  const int Np = T.Np, Nfn = ft.Nfn, Nfq = ft.Nfq;
  std::vector<double> Mf((size_t)Nfn * Nfn, 0.0);
  for (int q = 0; q < Nfq; ++q)
    for (int x = 0; x < Nfn; ++x)
      for (int y = 0; y < Nfn; ++y) Mf[x * Nfn + y] += ft.Ican[q * Nfn + x] * ft.tri_w[q] * ft.Ican[q * Nfn + y];
  double mx = 0.0;
  for (double v : Mf) mx = std::max(mx, std::fabs(v));
  // the lattice is symmetric: M_f must not depend on the face frame
  for (int o = 0; o < 6; ++o) {
    const int* Pm = &ft.tri_perm[o * Nfn];
    for (int x = 0; x < Nfn; ++x)
      for (int y = 0; y < Nfn; ++y)
        if (std::fabs(Mf[Pm[x] * Nfn + Pm[y]] - Mf[x * Nfn + y]) > 1e-10 * mx)
          return fail(c, HDG_EINVAL, "internal: face lattice mass matrix is not permutation invariant");
  }
  std::vector<double> L((size_t)4 * Np * Nfn, 0.0);
  for (int f = 0; f < 4; ++f)
    for (int i = 0; i < Np; ++i)
      for (int l = 0; l < Nfn; ++l) {
        double acc = 0.0;
        for (int j = 0; j < Nfn; ++j) acc += T.Minv[(size_t)i * Np + T.fnode[f * Nfn + j]] * Mf[j * Nfn + l];
        L[((size_t)f * Np + i) * Nfn + l] = acc;
      }
  std::vector<double> Dall;
  for (const Vec* D : {&T.Dr, &T.Ds, &T.Dt}) Dall.insert(Dall.end(), D->begin(), D->end());
  ops.clear();
  iops.clear();
  const double iD = pack_group(Dall, 3, Np, Np, P, ops);
  const double iL = pack_group(L, 4, Np, Nfn, P, ops);
  ops.push_back((float)iD);
  ops.push_back((float)iL);
  iops.insert(iops.end(), T.fnode.begin(), T.fnode.end());
  iops.insert(iops.end(), ft.tri_perm.begin(), ft.tri_perm.end());
  int nf = 0, ni = 0;
  tet_mfma_table_sizes(c->N, P, &nf, &ni);
  if ((int)ops.size() != nf || (int)iops.size() != ni)
    return fail(c, HDG_EINVAL, "internal: matrix-core table size mismatch");
  return HDG_OK;
}

// Tables of the matrix-core pyramid kernel: D^{r,s,t}, the base-face basis
// Fq and the triangle-face bases Ft_f as rows with an odd stride (zero
// padded), the lattice lift fragments Ft_f^T M_f, the canonical triangle
// weight of point 0, the geometry points (a, b) as doubles; the base and
// lattice orientation permutations and their inverses.
int build_pyr_mfma_tables(hdg_ctx* c, std::vector<float>& ops, std::vector<int>& iops) {
  const PyrRef& P = c->pyr;
  const FaceTables& ft = c->ft;
  const int Np = P.Np, Nfn = ft.Nfn, Nfq = ft.Nfq;
  const int SD = Np | 1, Mt = (Np + 15) / 16, Kf = (Nfn + 3) / 4;
  const int Ks = (Np + 3) / 4, Mq = (Nfq + 15) / 16, Kq = (Nfq + 3) / 4, Mtf = (Nfn + 15) / 16;
  int nf = 0, ni = 0;
  if (pyr_mfma_table_sizes(c->N, &nf, &ni)) return fail(c, HDG_EINVAL, "internal: no pyramid matrix-core kernel");
  ops.clear();
  iops.clear();
  if (pyr_mfma_global(c->N)) {
    // fragment order: lane l of (row tile t, k-step s) holds A[16t + l%16][4s + l/16]
    // (transposed: A[4s + l/16][16t + l%16]), zero outside the R x C matrix
    // (k-step outer, row tile inner)
    auto frag = [&](const double* A, int R, int C, int t, int st, bool tr) {
      for (int l = 0; l < 64; ++l) {
        const int i = tr ? 4 * st + l / 16 : 16 * t + l % 16, j = tr ? 16 * t + l % 16 : 4 * st + l / 16;
        ops.push_back(i < R && j < C ? (float)A[(size_t)i * C + j] : 0.0f);
      }
    };
    const Vec* D[3] = {&P.Dr, &P.Ds, &P.Dt};
    for (int st = 0; st < Ks; ++st)
      for (int tr = 0; tr < 2; ++tr)
        for (int r = 0; r < 3; ++r)
          for (int t = 0; t < Mt; ++t) frag(D[r]->data(), Np, Np, t, st, tr == 1);
    // trace operator: per k-step the base face's row tiles, then each triangle's
    for (int st = 0; st < Ks; ++st) {
      for (int t = 0; t < Mq; ++t) frag(P.Fquad.data(), Nfq, Np, t, st, false);
      for (int tf = 0; tf < 4; ++tf)
        for (int t = 0; t < Mtf; ++t) frag(P.Ftri.data() + (size_t)tf * Nfn * Np, Nfn, Np, t, st, false);
    }
    for (int st = 0; st < Kq; ++st)
      for (int t = 0; t < Mt; ++t) frag(P.Fquad.data(), Nfq, Np, t, st, true);
  } else {
    auto rows = [&](const Vec& A, int R) {
      for (int i = 0; i < R; ++i)
        for (int j = 0; j < SD; ++j) ops.push_back(j < Np ? (float)A[(size_t)i * Np + j] : 0.0f);
    };
    rows(P.Dr, Np);
    rows(P.Ds, Np);
    rows(P.Dt, Np);
    rows(P.Fquad, Nfq);
    rows(P.Ftri, 4 * Nfn);
  }
  std::vector<double> Mf((size_t)Nfn * Nfn, 0.0);
  for (int q = 0; q < Nfq; ++q)
    for (int x = 0; x < Nfn; ++x)
      for (int y = 0; y < Nfn; ++y) Mf[x * Nfn + y] += ft.Ican[q * Nfn + x] * ft.tri_w[q] * ft.Ican[q * Nfn + y];
  // Lt fragments [4][Mt][Kf] (LDS tables) or [4][Kf][Mt] (global fragment order)
  const bool g_order = pyr_mfma_global(c->N) != 0;
  for (int tf = 0; tf < 4; ++tf)
    for (int u = 0; u < (g_order ? Kf : Mt); ++u)
      for (int v = 0; v < (g_order ? Mt : Kf); ++v)
        for (int l = 0; l < 64; ++l) {
          const int t = g_order ? v : u, s = g_order ? u : v;
          const int i = 16 * t + l % 16, col = 4 * s + l / 16;
          double acc = 0.0;
          if (i < Np && col < Nfn)
            for (int m = 0; m < Nfn; ++m) acc += P.Ftri[((size_t)tf * Nfn + m) * Np + i] * Mf[m * Nfn + col];
          ops.push_back((float)acc);
        }
  ops.push_back((float)ft.tri_w[0]);
  while (ops.size() % 2) ops.push_back(0.0f);
  std::vector<double> gab;
  for (int i = 0; i < Np; ++i) {
    gab.push_back(P.geo_pts[3 * i]);
    gab.push_back(P.geo_pts[3 * i + 1]);
  }
  const size_t o = ops.size();
  ops.resize(o + 2 * gab.size());
  std::memcpy(ops.data() + o, gab.data(), gab.size() * sizeof(double));
  std::vector<int> iq(8 * Nfq), it(6 * Nfn);
  for (int k = 0; k < 8; ++k)
    for (int q = 0; q < Nfq; ++q) iq[k * Nfq + ft.quad_perm[k * Nfq + q]] = q;
  for (int k = 0; k < 6; ++k)
    for (int m = 0; m < Nfn; ++m) it[k * Nfn + ft.tri_perm[k * Nfn + m]] = m;
  iops.insert(iops.end(), ft.quad_perm.begin(), ft.quad_perm.end());
  iops.insert(iops.end(), iq.begin(), iq.end());
  iops.insert(iops.end(), ft.tri_perm.begin(), ft.tri_perm.end());
  iops.insert(iops.end(), it.begin(), it.end());
  if ((int)ops.size() != nf || (int)iops.size() != ni)
    return fail(c, HDG_EINVAL, "internal: pyramid matrix-core table size mismatch");
  return HDG_OK;
}

bool use_lattice(const hdg_ctx* c) { return c->path == HDG_PATH_AUTO && c->lattice_ok; }

// One launch of the kernel serving type t: tetrahedra go to the matrix-core
// kernel when lattice traces are in use; mrab selects the multi-rate update.
int launch_type(hdg_ctx* c, int t, StageArgs a, bool mrab) {
  a.lat = use_lattice(c) ? 1 : 0;
  a.V = c->td[t].V;
  // The matrix-core pyramid kernel serves every mode at N = 3..5; N <= 2
  // uses the wavefront-batched vector kernels.
  const bool pyr_mfma = t == kPyr && a.lat && c->td[t].mops && c->N >= 3;
  if (pyr_mfma) {
    a.ops = c->td[t].mops;
    a.iops = c->td[t].miops;
    if (mrab) a.mode = kModeMrab;
    if (launch_pyr_mfma(c->N, a, c->stream, c->max_blocks)) return fail(c, HDG_EINVAL, "no kernel for this order");
    return HDG_OK;
  }
  if (t == kTet && a.lat) {
    a.ops = c->td[t].mops;
    a.iops = c->td[t].miops;
    if (mrab) a.mode = kModeMrab;
    if (launch_tet_mfma(c->N, c->prec, a, c->stream, c->max_blocks)) return fail(c, HDG_EINVAL, "no kernel for this order");
    return HDG_OK;
  }
  const int r = mrab ? launch_mrab_update(t, c->N, a, c->stream, c->epb[t]) : launch_stage(t, c->N, a, c->stream, c->epb[t]);
  if (r) return fail(c, HDG_EINVAL, "no stage kernel for this order");
  return HDG_OK;
}

int check_type(const hdg_ctx* c, int t) {
  if (t < 0 || t > 3) return HDG_EINVAL;
  return c->td[t].present ? HDG_OK : HDG_EINVAL;
}

int ensure_traces(hdg_ctx* c) {
  if (c->traces_valid) return HDG_OK;
  for (int t = 0; t < 4; ++t) {
    TypeData& d = c->td[t];
    if (!d.present) continue;
    StageArgs a{};
    a.K = d.Ks;
    a.n_items = d.K;
    a.U = d.U;
    a.R = d.R;
    a.geo = d.geo;
    a.mat = d.mat;
    a.nbr = c->nbr;
    a.ori = c->ori;
    a.tau = c->tau;
    a.fgeo = d.fgeo;
    a.isqJ = d.isqJ;
    a.tr_in = c->trace[c->cur];
    a.tr_out = c->trace[c->cur];
    a.slot0 = d.slot0;
    a.ops = d.ops;
    a.iops = d.iops;
    a.mode = kModeTrace;
    int rc = launch_type(c, t, a, false);
    if (rc) return rc;
  }
  HIPCHK(c, hipGetLastError());
  c->traces_valid = true;
  return HDG_OK;
}

// Profile categories: kind * 4 + type, kind 0 = stage / right-hand-side
// kernels, 1 = multi-rate update kernels, 2 = non-conforming interface
// (mortar) kernel, filed under the tetrahedra.
constexpr int kProfRhs = 0, kProfUpdate = 1, kProfMortar = 2;

int prof_begin(hdg_ctx* c, int t, hipEvent_t* stop) {
  *stop = nullptr;
  if (!c->prof) return HDG_OK;
  if (c->ev_used == c->ev_pool.size()) {
    std::array<hipEvent_t, 2> p;
    HIPCHK(c, hipEventCreate(&p[0]));
    HIPCHK(c, hipEventCreate(&p[1]));
    c->ev_pool.push_back(p);
    c->ev_type.push_back(t);
  }
  c->ev_type[c->ev_used] = t;
  HIPCHK(c, hipEventRecord(c->ev_pool[c->ev_used][0], c->stream));
  *stop = c->ev_pool[c->ev_used][1];
  c->ev_used++;
  return HDG_OK;
}

// Virtual-slot traces and coarse-face fluxes of the non-conforming faces for
// a right-hand-side evaluation that reads trace buffer tr (multi-rate: with
// the mid-step buffer and the substep's level rule).
int run_mortar(hdg_ctx* c, float4* tr, float4* tr_half, int ksub, int dense) {
  if (c->n_nc == 0) return HDG_OK;
  MortarArgs m{};
  m.n = c->n_nc;
  m.rec = c->ncrec;
  m.vslot0 = c->nslot0;
  m.nfn = c->ft.Nfn;
  m.ts = trace_stride(c->N);
  m.I = c->ncI;
  m.P = c->ncP;
  m.cgeo = c->td[kTet].fgeo;
  m.cslot0 = c->td[kTet].slot0;
  m.tau = c->tau;
  m.tr = tr;
  m.tr_half = tr_half;
  m.slevel = c->slevel;
  m.L = c->L;
  m.ksub = ksub;
  m.dense = dense;
  hipEvent_t stop;
  int rc = prof_begin(c, kProfMortar * 4 + kTet, &stop);
  if (rc) return rc;
  launch_mortar(m, c->stream);
  if (stop) HIPCHK(c, hipEventRecord(stop, c->stream));
  HIPCHK(c, hipGetLastError());
  return HDG_OK;
}

// Arguments of one type's stage kernel (mode, LSERK4 coefficients, step).
StageArgs stage_args(hdg_ctx* c, const TypeData& d, int mode, float ra, float rb, float dt) {
  StageArgs a{};
  a.K = d.Ks;
  a.n_items = d.K;
  a.U = d.U;
  a.R = d.R;
  a.geo = d.geo;
  a.mat = d.mat;
  a.nbr = c->nbr;
  a.ori = c->ori;
  a.tau = c->tau;
  a.fgeo = d.fgeo;
  a.isqJ = d.isqJ;
  a.tr_in = c->trace[c->cur];
  a.tr_out = c->trace[1 - c->cur];
  a.slot0 = d.slot0;
  a.ops = d.ops;
  a.iops = d.iops;
  a.a = ra;
  a.b = rb;
  a.dt = dt;
  a.mode = mode;
  return a;
}

int run_stage(hdg_ctx* c, int mode, float ra, float rb, float dt) {
  int rc0 = run_mortar(c, c->trace[c->cur], nullptr, 0, 0);
  if (rc0) return rc0;
  for (int t = 0; t < 4; ++t) {
    TypeData& d = c->td[t];
    if (!d.present) continue;
    const StageArgs a = stage_args(c, d, mode, ra, rb, dt);
    hipEvent_t stop;
    int rc = prof_begin(c, t, &stop);
    if (rc) return rc;
    if ((rc = launch_type(c, t, a, false))) return rc;
    if (stop) HIPCHK(c, hipEventRecord(stop, c->stream));
  }
  HIPCHK(c, hipGetLastError());
  if (mode == kModeStage) c->cur = 1 - c->cur;
  return HDG_OK;
}

// 1:4 non-conforming triangular faces (hdg.h, hdg_mesh): finds the coarse
// faces among the unmatched triangles, appends four virtual slots and one
// flux slot per coarse face to the slot arrays, pairs each fine face with its
// virtual slot, and builds the mortar records and the interpolation /
// projection tables of every distinct sub-face placement.
int match_nonconforming(hdg_ctx* c, const hdg_mesh* m, std::vector<int>& nbr, std::vector<int8_t>& ori,
                        std::vector<int64_t>& slot_elem, std::vector<int>& rec, std::vector<float>& Itab,
                        std::vector<float>& Ptab) {
  if (m->n_hanging <= 0) return HDG_OK;
  if (!m->hanging) return fail(c, HDG_EINVAL, "hanging vertex list is NULL");
  const int64_t ns0 = (int64_t)nbr.size();
  std::map<std::pair<int64_t, int64_t>, int64_t> mid;
  std::map<int64_t, std::pair<int64_t, int64_t>> parents;
  for (int64_t r = 0; r < m->n_hanging; ++r) {
    const int64_t v = m->hanging[3 * r], a = m->hanging[3 * r + 1], b = m->hanging[3 * r + 2];
    if (v < 0 || a < 0 || b < 0 || v >= m->n_vert || a >= m->n_vert || b >= m->n_vert || a == b || v == a || v == b)
      return fail(c, HDG_EINVAL, "hanging vertex row " + std::to_string(r) + " has a bad vertex id");
    double scale = 1.0, dev = 0.0;
    for (int d = 0; d < 3; ++d) {
      scale = std::max({scale, std::fabs(m->xyz[3 * a + d]), std::fabs(m->xyz[3 * b + d])});
      dev = std::max(dev, std::fabs(m->xyz[3 * v + d] - 0.5 * (m->xyz[3 * a + d] + m->xyz[3 * b + d])));
    }
    if (dev > 1e-12 * scale)
      return fail(c, HDG_EMESH, "hanging vertex " + std::to_string(v) + " is not the midpoint of its edge");
    mid[{std::min(a, b), std::max(a, b)}] = v;
    parents[v] = {a, b};
  }
  // unmatched triangular faces by sorted vertex ids
  struct Tri {
    int64_t slot, elem;
    int type;
    int64_t g[3];
  };
  std::vector<Tri> tris;
  std::map<std::array<int64_t, 3>, size_t> free_tri;
  for (int t = 0; t < 4; ++t) {
    const TypeData& d = c->td[t];
    const ElemDesc& E = elem_desc(t);
    for (int64_t k = 0; k < d.K; ++k)
      for (int f = 0; f < E.nf; ++f) {
        const int64_t sl = d.slot0 + k * E.nf + f;
        if (nbr[sl] >= 0 || E.fnv[f] != 3) continue;
        Tri T{sl, d.elems[k], t, {0, 0, 0}};
        for (int v = 0; v < 3; ++v) T.g[v] = m->verts[8 * d.elems[k] + E.fv[f][v]];
        std::array<int64_t, 3> key{T.g[0], T.g[1], T.g[2]};
        std::sort(key.begin(), key.end());
        free_tri[key] = tris.size();
        tris.push_back(T);
      }
  }
  auto find_mid = [&](int64_t a, int64_t b) -> int64_t {
    auto it = mid.find({std::min(a, b), std::max(a, b)});
    return it == mid.end() ? -1 : it->second;
  };
  struct Nc {
    size_t parent;
    size_t fine[4];
  };
  std::vector<Nc> list;
  std::vector<char> used(tris.size(), 0);
  for (size_t i = 0; i < tris.size(); ++i) {
    const Tri& T = tris[i];
    const int64_t m01 = find_mid(T.g[0], T.g[1]), m12 = find_mid(T.g[1], T.g[2]), m20 = find_mid(T.g[2], T.g[0]);
    if (m01 < 0 || m12 < 0 || m20 < 0) continue;
    const int64_t sub[4][3] = {{T.g[0], m01, m20}, {T.g[1], m12, m01}, {T.g[2], m20, m12}, {m01, m12, m20}};
    Nc nc{i, {0, 0, 0, 0}};
    for (int q = 0; q < 4; ++q) {
      std::array<int64_t, 3> key{sub[q][0], sub[q][1], sub[q][2]};
      std::sort(key.begin(), key.end());
      auto it = free_tri.find(key);
      if (it == free_tri.end() || used[it->second])
        return fail(c, HDG_EMESH, "a sub-face of a refined triangular face has no element");
      used[it->second] = 1;
      nc.fine[q] = it->second;
    }
    if (T.type != kTet) return fail(c, HDG_EMESH, "non-conforming faces are supported between tetrahedra only");
    for (int q = 0; q < 4; ++q)
      if (tris[nc.fine[q]].type != kTet)
        return fail(c, HDG_EMESH, "non-conforming faces are supported between tetrahedra only");
    list.push_back(nc);
  }
  if (list.empty()) return HDG_OK;
  if (!c->lattice_ok) return fail(c, HDG_EMESH, "non-conforming faces need a mesh with lattice traces");
  const int64_t nnc = (int64_t)list.size();
  const int64_t ntot = ns0 + 5 * nnc;
  if (ntot >= ((int64_t)1 << 31) - kNcBase) return fail(c, HDG_EINVAL, "mesh too large (face slots exceed int32)");
  nbr.resize(ntot, -1 - m->bc);
  ori.resize(ntot, 0);
  slot_elem.resize(ntot, 0);
  // sub-face placements: coarse barycentrics (x2) of the sub-face's canonical vertices
  std::map<std::array<int, 9>, int> variants;
  std::vector<std::array<int, 9>> vlist;
  rec.assign((size_t)nnc * kNcRec, 0);
  c->nc_fine_elems.clear();
  for (int64_t i = 0; i < nnc; ++i) {
    const Tri& P = tris[list[i].parent];
    int64_t cc[3] = {P.g[0], P.g[1], P.g[2]};
    std::sort(cc, cc + 3);
    const int64_t flux = ns0 + 4 * nnc + i;
    nbr[P.slot] = -(int)(kNcBase + flux);
    slot_elem[flux] = P.elem;
    int* r = &rec[(size_t)i * kNcRec];
    r[0] = (int)P.slot;
    r[1] = (int)flux;
    std::array<int64_t, 4> fe{};
    for (int q = 0; q < 4; ++q) {
      const Tri& F = tris[list[i].fine[q]];
      const int64_t vs = ns0 + 4 * i + q;
      nbr[vs] = (int)F.slot;
      nbr[F.slot] = (int)vs;
      slot_elem[vs] = P.elem;
      fe[q] = F.elem;
      int64_t ff[3] = {F.g[0], F.g[1], F.g[2]};
      std::sort(ff, ff + 3);
      std::array<int, 9> B{};
      for (int k = 0; k < 3; ++k) {
        int64_t pa = ff[k], pb = ff[k];
        auto it = parents.find(ff[k]);
        if (it != parents.end()) {
          pa = it->second.first;
          pb = it->second.second;
        }
        for (int j = 0; j < 3; ++j) B[3 * k + j] = (pa == cc[j]) + (pb == cc[j]);
        if (B[3 * k] + B[3 * k + 1] + B[3 * k + 2] != 2)
          return fail(c, HDG_EMESH, "a sub-face vertex is neither a vertex nor an edge midpoint of its coarse face");
      }
      auto vit = variants.find(B);
      int var;
      if (vit == variants.end()) {
        var = (int)vlist.size();
        variants[B] = var;
        vlist.push_back(B);
      } else {
        var = vit->second;
      }
      r[2 + q] = (int)F.slot;
      r[6 + q] = var;
    }
    c->nc_fine_elems.push_back(fe);
  }
  // tables: I_v evaluates the coarse lattice basis at the sub-face lattice
  // nodes; P_v = M^-1 I_v^T M maps sub-face lattice fluxes to the equivalent
  // coarse lattice flux (M the lattice mass matrix)
  const FaceTables& ft = c->ft;
  const int Nfn = ft.Nfn, N = c->N;
  const Vec M = tri_lattice_mass(ft);
  Vec Mi;
  if (!invert(Nfn, M, Mi)) return fail(c, HDG_EINVAL, "internal: singular face lattice mass matrix");
  Itab.clear();
  Ptab.clear();
  for (const auto& B : vlist) {
    Vec pts(2 * Nfn);
    for (int q = 0; q < Nfn; ++q) {
      const double lam[3] = {ft.lattice_ij[q][2] / (double)N, ft.lattice_ij[q][0] / (double)N,
                             ft.lattice_ij[q][1] / (double)N};
      double mu[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) mu[j] += 0.5 * lam[k] * B[3 * k + j];
      pts[2 * q] = -1.0 + 2.0 * mu[1];
      pts[2 * q + 1] = -1.0 + 2.0 * mu[2];
    }
    Vec I;
    tri_lattice_basis(ft, pts, I);
    Vec T((size_t)Nfn * Nfn, 0.0);  // I^T M
    for (int a = 0; a < Nfn; ++a)
      for (int b = 0; b < Nfn; ++b) {
        double acc = 0.0;
        for (int q = 0; q < Nfn; ++q) acc += I[q * Nfn + a] * M[q * Nfn + b];
        T[a * Nfn + b] = acc;
      }
    for (double v : I) Itab.push_back((float)v);
    for (int a = 0; a < Nfn; ++a)
      for (int b = 0; b < Nfn; ++b) {
        double acc = 0.0;
        for (int q = 0; q < Nfn; ++q) acc += Mi[a * Nfn + q] * T[q * Nfn + b];
        Ptab.push_back((float)acc);
      }
  }
  c->n_nc = nnc;
  c->nslot0 = ns0;
  return HDG_OK;
}

int create_impl(hdg_ctx* c, const hdg_mesh* m, int N) {
  c->N = N;
  build_face_tables(N, c->ft);
  const FaceTables& ft = c->ft;
  const int64_t ne = m->n_elem;
  c->n_elem = ne;
  // ---- element lists per type, vertex checks
  for (int64_t e = 0; e < ne; ++e) {
    const int t = m->type[e];
    if (t < 0 || t > 3) return fail(c, HDG_EINVAL, "element " + std::to_string(e) + " has bad type");
    const int nv = elem_desc(t).nv;
    for (int v = 0; v < nv; ++v) {
      const int64_t id = m->verts[8 * e + v];
      if (id < 0 || id >= m->n_vert) return fail(c, HDG_EINVAL, "element " + std::to_string(e) + " has a bad vertex id");
    }
    if (!(m->kappa[e] > 0.0) || !(m->rho[e] > 0.0))
      return fail(c, HDG_EINVAL, "element " + std::to_string(e) + " has non-positive kappa or rho");
    c->td[t].elems.push_back(e);
  }
  std::vector<int> etype_local(ne), eidx(ne);
  int64_t slot = 0;
  for (int t = 0; t < 4; ++t) {
    TypeData& d = c->td[t];
    d.K = (int64_t)d.elems.size();
    d.present = d.K > 0;
    const ElemDesc& E = elem_desc(t);
    d.nv = E.nv;
    d.nf = E.nf;
    d.Np = np_of(t, N);
    d.slot0 = slot;
    slot += d.K * d.nf;
    for (int64_t k = 0; k < d.K; ++k) {
      etype_local[d.elems[k]] = t;
      eidx[d.elems[k]] = (int)k;
    }
  }
  c->nslot = slot;
  if (c->nslot >= (int64_t)1 << 31) return fail(c, HDG_EINVAL, "mesh too large (face slots exceed int32)");
  if (c->td[kHex].present) build_hex(N, c->hex);
  if (c->td[kTet].present) build_tet(N, ft, c->tet);
  if (c->td[kWedge].present) build_wedge(N, ft, c->wedge);
  if (c->td[kPyr].present) build_pyr(N, ft, c->pyr);

  // ---- face matching by sorted vertex ids, canonical orientation codes
  const int64_t ns = c->nslot;
  std::vector<std::array<int64_t, 4>> keys(ns);
  std::vector<int8_t> ori(ns);
  std::vector<int64_t> slot_elem(ns);
  for (int t = 0; t < 4; ++t) {
    TypeData& d = c->td[t];
    const ElemDesc& E = elem_desc(t);
    for (int64_t k = 0; k < d.K; ++k) {
      const int64_t e = d.elems[k];
      for (int f = 0; f < E.nf; ++f) {
        const int64_t s = d.slot0 + k * E.nf + f;
        int64_t g[4];
        for (int v = 0; v < E.fnv[f]; ++v) g[v] = m->verts[8 * e + E.fv[f][v]];
        ori[s] = (int8_t)face_orientation(E.fnv[f], g, nullptr);
        std::array<int64_t, 4> key{-1, -1, -1, -1};
        std::sort(g, g + E.fnv[f]);
        for (int v = 0; v < E.fnv[f]; ++v) key[4 - E.fnv[f] + v] = g[v];
        keys[s] = key;
        slot_elem[s] = e;
      }
    }
  }
  std::vector<int64_t> order(ns);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return keys[x] < keys[y]; });
  // boundary faces: -(1 + bc), bc per face where the mesh gives one
  std::vector<int> nbr(ns, -1 - m->bc);
  if (m->bc_face) {
    for (int t = 0; t < 4; ++t) {
      const TypeData& d = c->td[t];
      const int nf = elem_desc(t).nf;
      for (int64_t k = 0; k < d.K; ++k)
        for (int f = 0; f < nf; ++f) {
          const int b = m->bc_face[6 * d.elems[k] + f];
          if (b != -1 && b != HDG_BC_FREE_SURFACE && b != HDG_BC_RIGID_WALL)
            return fail(c, HDG_EINVAL, "element " + std::to_string(d.elems[k]) + " has a bad face boundary condition");
          if (b >= 0) nbr[d.slot0 + k * nf + f] = -1 - b;
        }
    }
  }
  for (int64_t i = 0; i < ns;) {
    int64_t j = i + 1;
    while (j < ns && keys[order[j]] == keys[order[i]]) ++j;
    if (j - i == 2) {
      nbr[order[i]] = (int)order[i + 1];
      nbr[order[i + 1]] = (int)order[i];
    } else if (j - i > 2) {
      return fail(c, HDG_EMESH, "a face is shared by more than two elements");
    }
    i = j;
  }
  // lattice traces need every triangular face touching a tetrahedron or a
  // pyramid to have no wedge on either side (wedge traces are not polynomial)
  {
    std::vector<int8_t> slot_type(ns), slot_nv(ns);
    for (int t = 0; t < 4; ++t) {
      const TypeData& d = c->td[t];
      const ElemDesc& E = elem_desc(t);
      for (int64_t k = 0; k < d.K; ++k)
        for (int f = 0; f < E.nf; ++f) {
          slot_type[d.slot0 + k * E.nf + f] = (int8_t)t;
          slot_nv[d.slot0 + k * E.nf + f] = (int8_t)E.fnv[f];
        }
    }
    c->lattice_ok = true;
    for (int64_t s = 0; s < ns && c->lattice_ok; ++s) {
      if (nbr[s] < 0 || slot_nv[s] != 3) continue;
      const int ta = slot_type[s], tb = slot_type[nbr[s]];
      if ((ta == kWedge) != (tb == kWedge)) c->lattice_ok = false;
    }
  }
  // 1:4 non-conforming faces: virtual and flux slots appended
  std::vector<int> ncrec;
  std::vector<float> ncI, ncP;
  int rc = match_nonconforming(c, m, nbr, ori, slot_elem, ncrec, ncI, ncP);
  if (rc) return rc;
  c->nslot = (int64_t)nbr.size();
  const int64_t nsall = c->nslot;
  // penalties: tau_p = 1 / {rho c}, tau_u = {rho c}; boundary uses own rho c.
  // An element's maxima run over its faces, and over the sub-faces (virtual
  // slots) instead of a coarse non-conforming face (whose own slot and flux
  // slot carry no penalty).
  std::vector<float2> tau(nsall);
  std::vector<double> taup_max(ne, 0.0), tauu_max(ne, 0.0);
  for (int64_t s = 0; s < nsall; ++s) {
    const int64_t e = slot_elem[s];
    const double rc = std::sqrt(m->kappa[e] * m->rho[e]);
    const double rn = nbr[s] >= 0 ? std::sqrt(m->kappa[slot_elem[nbr[s]]] * m->rho[slot_elem[nbr[s]]]) : rc;
    const double avg = 0.5 * (rc + rn);
    tau[s] = make_float2((float)(1.0 / avg), (float)avg);
    const bool aux = nbr[s] <= -kNcBase || (c->n_nc > 0 && s >= c->nslot0 + 4 * c->n_nc);
    if (aux) continue;
    taup_max[e] = std::max(taup_max[e], 1.0 / avg);
    tauu_max[e] = std::max(tauu_max[e], avg);
  }
  c->slot_elem_h = slot_elem;
  c->nbr_h = nbr;
  c->etype_h = etype_local;
  c->eidx_h = eidx;
  {
    int dev = 0, ncu = 0;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (ncu > 0) c->max_blocks = ncu;
  }
  if (project_scratch(&c->pscratch)) return fail(c, HDG_EHIP, "address of the projection work buffer not found");
  if ((rc = upload(c, &c->nbr, nbr))) return rc;
  if ((rc = upload(c, &c->ori, ori))) return rc;
  if ((rc = upload(c, &c->tau, tau))) return rc;
  if (c->n_nc > 0) {
    if ((rc = upload(c, &c->ncrec, ncrec))) return rc;
    if ((rc = upload(c, &c->ncI, ncI))) return rc;
    if ((rc = upload(c, &c->ncP, ncP))) return rc;
  }

  // ---- geometry tables
  GeoTables G{};
  for (int t = 0; t < 4; ++t) {
    const ElemDesc& E = elem_desc(t);
    G.nv[t] = E.nv;
    G.nf[t] = E.nf;
    for (int v = 0; v < E.nv; ++v)
      for (int d = 0; d < 3; ++d) G.vref[t][v][d] = E.vref[v][d];
    for (int f = 0; f < E.nf; ++f) {
      G.fnv[t][f] = E.fnv[f];
      G.farea[t][f] = E.farea[f];
      for (int v = 0; v < 4; ++v) G.fv[t][f][v] = E.fv[f][v];
      for (int d = 0; d < 3; ++d) G.nref[t][f][d] = E.nref[f][d];
    }
  }
  G.Nfq = ft.Nfq;
  if (ft.Nfq > 64) return fail(c, HDG_EINVAL, "order too high for the face tables");
  for (int q = 0; q < ft.Nfq; ++q) {
    G.tri_eta[q][0] = ft.tri_eta[2 * q];
    G.tri_eta[q][1] = ft.tri_eta[2 * q + 1];
    G.tri_w[q] = ft.tri_w[q];
    G.quad_eta[q][0] = ft.quad_eta[2 * q];
    G.quad_eta[q][1] = ft.quad_eta[2 * q + 1];
    G.quad_w[q] = ft.quad_w[q];
  }
  for (int o = 0; o < 6; ++o) orientation_perm(3, o, G.tri_P[o]);
  for (int o = 0; o < 8; ++o) orientation_perm(4, o, G.quad_P[o]);
  if ((rc = dalloc(c, &c->gtab, 1))) return rc;
  HIPCHK(c, hipMemcpyAsync(c->gtab, &G, sizeof(G), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));

  // ---- per-type data
  for (int t = 0; t < 4; ++t) {
    TypeData& d = c->td[t];
    if (!d.present) continue;
    const int64_t K = d.K;
    std::vector<double> V(K * d.nv * 3);
    std::vector<float2> mat(K);
    for (int64_t k = 0; k < K; ++k) {
      const int64_t e = d.elems[k];
      for (int v = 0; v < d.nv; ++v)
        for (int dd = 0; dd < 3; ++dd) V[(k * d.nv + v) * 3 + dd] = m->xyz[3 * m->verts[8 * e + v] + dd];
      mat[k] = make_float2((float)m->kappa[e], (float)(1.0 / m->rho[e]));
    }
    if ((rc = upload(c, &d.V, V))) return rc;
    if ((rc = upload(c, &d.mat, mat))) return rc;
    std::vector<double> vpts, vw, spts, sw, Phi, gpts;
    const int n1 = N + 1;
    if (t == kHex) {
      for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            vpts.insert(vpts.end(), {c->hex.x1[i], c->hex.x1[j], c->hex.x1[k]});
            vw.push_back(c->hex.w1[i] * c->hex.w1[j] * c->hex.w1[k]);
          }
      spts = vpts;
    } else if (t == kTet) {
      vpts = {-0.5, -0.5, -0.5};
      spts = c->tet.nodes;
    } else if (t == kWedge) {
      vpts = c->wedge.vol_pts;
      spts = c->wedge.vol_pts;
      sw = c->wedge.vol_w;
      Phi = c->wedge.Phi;
    } else {
      vpts = c->pyr.geo_pts;
      spts = c->pyr.proj_pts;
      sw = c->pyr.proj_w;
      Phi = c->pyr.Phi;
      gpts = c->pyr.geo_pts;
    }
    d.nvp = (int)(vpts.size() / 3);
    d.nsample = (int)(spts.size() / 3);
    double* d_vpts = nullptr;
    double* d_vw = nullptr;
    if ((rc = upload(c, &d_vpts, vpts))) return rc;
    if ((rc = upload(c, &d_vw, vw))) return rc;
    if ((rc = upload(c, &d.spts, spts))) return rc;
    if ((rc = upload(c, &d.sw, sw))) return rc;
    if ((rc = upload(c, &d.Phi, Phi))) return rc;
    if ((rc = upload(c, &d.gpts, gpts))) return rc;
    if (t == kTet && (rc = upload(c, &d.Mhat, c->tet.Mhat))) return rc;
    const int ngeo = (t == kTet) ? 12 : (t == kWedge ? 12 * d.nvp : 10 * d.nvp);
    if ((rc = dalloc(c, &d.geo, (size_t)K * ngeo))) return rc;
    const int fstride = (t == kTet) ? 1 : ft.Nfq;
    if ((rc = dalloc(c, &d.fgeo, (size_t)K * d.nf * fstride))) return rc;
    if (t == kWedge && (rc = dalloc(c, &d.isqJ, (size_t)K * d.nf * ft.Nfq))) return rc;
    double *cJ = nullptr, *minJ = nullptr;
    if ((rc = dalloc(c, &cJ, K))) return rc;
    if ((rc = dalloc(c, &minJ, K))) return rc;
    GeoArgs ga{};
    ga.type = t;
    ga.K = K;
    ga.V = d.V;
    ga.ori = c->ori + d.slot0;
    ga.T = c->gtab;
    ga.vpts = d_vpts;
    ga.nvp = d.nvp;
    ga.vw = d_vw;
    ga.geo = d.geo;
    ga.fgeo = d.fgeo;
    ga.fstride = fstride;
    ga.isqJ = d.isqJ;
    ga.cJ = cJ;
    ga.minJ = minJ;
    launch_geometry(ga, c->stream);
    HIPCHK(c, hipGetLastError());
    d.cJ.resize(K);
    d.minJ.resize(K);
    HIPCHK(c, hipMemcpyAsync(d.cJ.data(), cJ, K * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(d.minJ.data(), minJ, K * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    d.crk.resize(K);
    for (int64_t k = 0; k < K; ++k) {
      const int64_t e = d.elems[k];
      d.crk[k] = std::max(taup_max[e] * m->kappa[e], tauu_max[e] / m->rho[e]);
    }
    std::vector<float> ops;
    std::vector<int> iops;
    if ((rc = build_tables(c, t, ops, iops))) return rc;
    if ((rc = upload(c, &d.ops, ops))) return rc;
    if ((rc = upload(c, &d.iops, iops))) return rc;
    if (t == kTet) {
      if ((rc = build_tet_mfma_tables(c, c->prec, ops, iops))) return rc;
      if ((rc = upload(c, &d.mops, ops))) return rc;
      if ((rc = upload(c, &d.miops, iops))) return rc;
    }
    int pnf = 0, pni = 0;
    if (t == kPyr && pyr_mfma_table_sizes(N, &pnf, &pni) == 0) {
      if ((rc = build_pyr_mfma_tables(c, ops, iops))) return rc;
      if ((rc = upload(c, &d.mops, ops))) return rc;
      if ((rc = upload(c, &d.miops, iops))) return rc;
    }
    d.Ks = (K + 3) / 4 * 4;
    const size_t nstate = (size_t)4 * d.Ks * d.Np;
    if ((rc = dalloc(c, &d.U, nstate))) return rc;
    if ((rc = dalloc(c, &d.R, nstate))) return rc;
    HIPCHK(c, hipMemsetAsync(d.U, 0, nstate * sizeof(float), c->stream));
    HIPCHK(c, hipMemsetAsync(d.R, 0, nstate * sizeof(float), c->stream));
  }
  if ((rc = dalloc(c, &c->trace[0], (size_t)nsall * trace_stride(c->N)))) return rc;
  if ((rc = dalloc(c, &c->trace[1], (size_t)nsall * trace_stride(c->N)))) return rc;
  if ((rc = dalloc(c, &c->partial, (size_t)(ne / 256 + 8)))) return rc;
  if ((rc = dalloc(c, &c->flag, 1))) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int t = 0; t < 4; ++t) {
    const TypeData& d = c->td[t];
    for (int64_t k = 0; k < d.K; ++k)
      if (!(d.minJ[k] > 0.0))
        return fail(c, HDG_EMESH, "element " + std::to_string(d.elems[k]) + " has a non-positive Jacobian");
  }
  return HDG_OK;
}

}  // namespace

extern "C" {

int hdg_create(hdg_ctx** out, const hdg_mesh* m, int N, int precision, void* hip_stream) {
  if (!out) return fail(nullptr, HDG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!m || !m->xyz || !m->type || !m->verts || !m->kappa || !m->rho)
    return fail(nullptr, HDG_EINVAL, "mesh or one of its arrays is NULL");
  if (N < 1 || N > kMaxN) return fail(nullptr, HDG_EINVAL, "order N must be in [1, 5]");
  if (precision != HDG_PREC_FP32 && precision != HDG_PREC_FP16X2 && precision != HDG_PREC_FP16X2_K16 &&
      precision != HDG_PREC_BF16X2 && precision != HDG_PREC_BF16X3)
    return fail(nullptr, HDG_EINVAL, "unsupported precision mode");
  if (m->n_elem < 1 || m->n_vert < 1) return fail(nullptr, HDG_EINVAL, "empty mesh");
  if (m->bc != HDG_BC_FREE_SURFACE && m->bc != HDG_BC_RIGID_WALL)
    return fail(nullptr, HDG_EINVAL, "unknown boundary condition");
  hdg_ctx* c = new hdg_ctx();
  c->stream = (hipStream_t)hip_stream;
  c->prec = precision;
  int rc;
  try {
    rc = create_impl(c, m, N);
  } catch (const std::exception& ex) {
    rc = fail(c, HDG_EINVAL, std::string("set-up failed: ") + ex.what());
  }
  if (rc != HDG_OK) {
    g_create_error = c->err;
    hdg_destroy(c);
    return rc;
  }
  *out = c;
  return HDG_OK;
}

void hdg_destroy(hdg_ctx* c) {
  if (!c) return;
  // teardown: errors cannot be reported any more, every resource is released anyway
  if (!c->allocs.empty()) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
  }
  for (auto& p : c->ev_pool) {
    (void)hipEventDestroy(p[0]);
    (void)hipEventDestroy(p[1]);
  }
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (void* p : c->allocs) (void)hipFree(p);
  delete c;
}

const char* hdg_last_error(const hdg_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int hdg_type_info(const hdg_ctx* c, int t, int64_t* n_elem, int32_t* np, int32_t* n_sample) {
  if (!c || t < 0 || t > 3) return HDG_EINVAL;
  const TypeData& d = c->td[t];
  if (n_elem) *n_elem = d.K;
  if (np) *np = np_of(t, c->N);
  if (n_sample) *n_sample = d.present ? d.nsample : 0;
  return HDG_OK;
}

namespace {

// Element basis of type t at the canonical cubature points of every face and
// orientation: V [nf][8][Nfq][Np] (FP64), built from the same reference
// tables and local-point conventions as the stage kernels' trace
// evaluation (hexahedra: 1D extrapolation along the lines through the face
// points; wedges: triangle basis at the edge points times the 1D basis in s,
// or at the lattice times the 1D basis at s = -1, +1; pyramids: the base
// basis at its GL points, the triangle faces through the lattice;
// tetrahedra: the face nodes through the lattice).
void build_face_bases(const hdg_ctx* c, int t, std::vector<double>& V) {
  const FaceTables& ft = c->ft;
  const int Nfq = ft.Nfq, Nfn = ft.Nfn, n1 = ft.n1;
  const int Np = np_of(t, c->N);
  const ElemDesc& E = elem_desc(t);
  V.assign((size_t)E.nf * 8 * Nfq * Np, 0.0);
  for (int f = 0; f < E.nf; ++f) {
    const bool tri = E.fnv[f] == 3;
    for (int o = 0; o < (tri ? 6 : 8); ++o)
      for (int q = 0; q < Nfq; ++q) {
        double* row = V.data() + ((size_t)(f * 8 + o) * Nfq + q) * Np;
        if (!tri) {
          const int l = ft.quad_perm[o * Nfq + q], l1 = l % n1, l2 = l / n1;
          if (t == kHex) {
            const Vec& L = (f & 1) ? c->hex.Lp : c->hex.Lm;
            for (int m = 0; m < n1; ++m) {
              const int node = f < 2 ? m + n1 * (l1 + n1 * l2) : (f < 4 ? l1 + n1 * (m + n1 * l2) : l1 + n1 * (l2 + n1 * m));
              row[node] = L[m];
            }
          } else if (t == kWedge) {
            const WedgeRef& W = c->wedge;
            const int ef = f - 2;
            for (int js = 0; js < n1; ++js)
              for (int jt = 0; jt < W.Ntri; ++jt)
                row[js * W.Ntri + jt] = W.P1[l2 * n1 + js] * W.Fedge[((size_t)ef * n1 + l1) * W.Ntri + jt];
          } else {  // pyramid base
            for (int j = 0; j < Np; ++j) row[j] = c->pyr.Fquad[(size_t)l * Np + j];
          }
        } else {
          for (int m = 0; m < Nfn; ++m) {
            const double w = ft.Ican[q * Nfn + m];
            const int lm = ft.tri_perm[o * Nfn + m];
            if (t == kWedge) {
              const WedgeRef& W = c->wedge;
              const Vec& P1s = f == 0 ? W.P1m : W.P1p;
              for (int js = 0; js < n1; ++js)
                for (int jt = 0; jt < W.Ntri; ++jt)
                  row[js * W.Ntri + jt] += w * W.Ftri[(size_t)lm * W.Ntri + jt] * P1s[js];
            } else if (t == kPyr) {
              for (int j = 0; j < Np; ++j) row[j] += w * c->pyr.Ftri[((size_t)(f - 1) * Nfn + lm) * Np + j];
            } else {  // tetrahedron
              row[c->tet.fnode[f * Nfn + lm]] += w;
            }
          }
        }
      }
  }
}

// C_T(N, K) of every element on the device (once per context).
int compute_trace_constants(hdg_ctx* c) {
  bool done = true;
  for (int t = 0; t < 4; ++t)
    if (c->td[t].present && c->td[t].ctk.size() != (size_t)c->td[t].K) done = false;
  if (done) return HDG_OK;
  int rc = HDG_OK;
  for (int t = 0; t < 4 && rc == HDG_OK; ++t) {
    TypeData& d = c->td[t];
    if (!d.present) continue;
    std::vector<double> V;
    build_face_bases(c, t, V);
    std::vector<double> Linv;
    if (t == kTet) {
      // Mhat = L L^T; the kernel applies L^-1 and L^-T
      const int n = d.Np;
      const Vec& M = c->tet.Mhat;
      std::vector<double> L((size_t)n * n, 0.0);
      for (int j = 0; j < n; ++j) {
        double dg = M[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) dg -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(dg > 0.0)) return fail(c, HDG_EINVAL, "internal: tetrahedron mass matrix is not positive definite");
        L[(size_t)j * n + j] = std::sqrt(dg);
        for (int i = j + 1; i < n; ++i) {
          double v = M[(size_t)i * n + j];
          for (int k = 0; k < j; ++k) v -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
          L[(size_t)i * n + j] = v / L[(size_t)j * n + j];
        }
      }
      Linv.assign((size_t)n * n, 0.0);
      for (int j = 0; j < n; ++j) {  // forward substitution, column j of L^-1
        for (int i = j; i < n; ++i) {
          double v = i == j ? 1.0 : 0.0;
          for (int k = j; k < i; ++k) v -= L[(size_t)i * n + k] * Linv[(size_t)k * n + j];
          Linv[(size_t)i * n + j] = v / L[(size_t)i * n + i];
        }
      }
    }
    double *dV = nullptr, *dW = nullptr, *dL = nullptr, *dout = nullptr;
    auto put = [&](double** p, const std::vector<double>& h) -> int {
      if (h.empty()) return HDG_OK;
      if (hipMalloc((void**)p, h.size() * sizeof(double)) != hipSuccess) return fail(c, HDG_ENOMEM, "trace constant tables");
      if (hipMemcpyAsync(*p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return fail(c, HDG_EHIP, "trace constant tables");
      return HDG_OK;
    };
    rc = put(&dV, V);
    if (rc == HDG_OK) rc = put(&dW, c->ft.tri_w);
    if (rc == HDG_OK) rc = put(&dL, Linv);
    if (rc == HDG_OK && hipMalloc((void**)&dout, (size_t)d.K * sizeof(double)) != hipSuccess)
      rc = fail(c, HDG_ENOMEM, "trace constant output");
    if (rc == HDG_OK) {
      TraceConstArgs a{};
      a.type = t;
      a.K = d.K;
      a.Np = d.Np;
      a.nf = d.nf;
      a.Nfq = c->ft.Nfq;
      a.iters = 96;
      a.V = dV;
      a.tri_w = dW;
      a.Linv = dL;
      a.geo = d.geo;
      a.fgeo = d.fgeo;
      a.isqJ = d.isqJ;
      a.ori = c->ori;
      a.slot0 = d.slot0;
      a.out = dout;
      launch_trace_constants(a, c->stream);
      d.ctk.resize(d.K);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess)
        e = hipMemcpyAsync(d.ctk.data(), dout, (size_t)d.K * sizeof(double), hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) {
        d.ctk.clear();
        rc = fail(c, HDG_EHIP, std::string("trace constants: ") + hipGetErrorString(e));
      }
    }
    for (double* p : {dV, dW, dL, dout})
      if (p) (void)hipFree(p);
  }
  return rc;
}

}  // namespace

int hdg_trace_constants(hdg_ctx* c, double* out) {
  if (!c || !out) return HDG_EINVAL;
  int rc = compute_trace_constants(c);
  if (rc) return rc;
  for (int t = 0; t < 4; ++t) {
    const TypeData& d = c->td[t];
    for (int64_t k = 0; k < d.K; ++k) out[d.elems[k]] = d.ctk[k];
  }
  return HDG_OK;
}

int hdg_set_dt_mode(hdg_ctx* c, int mode) {
  if (!c) return HDG_EINVAL;
  if (mode != HDG_DT_REFERENCE && mode != HDG_DT_ELEMENT) return fail(c, HDG_EINVAL, "unknown time step mode");
  if (mode == HDG_DT_ELEMENT) {
    const int rc = compute_trace_constants(c);
    if (rc) return rc;
  }
  c->dt_mode = mode;
  return HDG_OK;
}

int hdg_dt(hdg_ctx* c, double cfl, double* dt_out, double* dt_min_out) {
  if (!c) return HDG_EINVAL;
  if (!(cfl > 0.0)) return fail(c, HDG_EINVAL, "CFL constant must be positive");
  double mn = 1e300;
  for (int t = 0; t < 4; ++t) {
    const TypeData& d = c->td[t];
    const double ct = trace_constant(t, c->N);
    const bool elem = c->dt_mode == HDG_DT_ELEMENT;
    for (int64_t k = 0; k < d.K; ++k) {
      const double dt = elem ? cfl / (d.crk[k] * d.ctk[k]) : cfl / (d.crk[k] * ct * d.cJ[k]);
      if (dt_out) dt_out[d.elems[k]] = dt;
      mn = std::min(mn, dt);
    }
  }
  if (dt_min_out) *dt_min_out = mn;
  return HDG_OK;
}

int hdg_get_points(hdg_ctx* c, int t, double* xyz) {
  if (!c) return HDG_EINVAL;
  if (check_type(c, t) || !xyz) return fail(c, HDG_EINVAL, "bad type or NULL output");
  const TypeData& d = c->td[t];
  launch_points(t, d.K, d.nv, d.V, d.spts, d.nsample, xyz, c->stream);
  HIPCHK(c, hipGetLastError());
  return HDG_OK;
}

int hdg_project(hdg_ctx* c, int t, const double* p, const double* ux, const double* uy, const double* uz) {
  if (!c) return HDG_EINVAL;
  if (check_type(c, t) || !p || !ux || !uy || !uz) return fail(c, HDG_EINVAL, "bad type or NULL input");
  TypeData& d = c->td[t];
  double* tmp = nullptr;
  if (t == kWedge || t == kPyr) {
    if (hipMalloc((void**)&tmp, (size_t)4 * d.K * d.nsample * sizeof(double)) != hipSuccess)
      return fail(c, HDG_ENOMEM, "projection scratch allocation failed");
  }
  launch_project(t, d.K, d.nv, d.V, d.spts, d.sw, d.nsample, d.Np, d.Phi, d.gpts, p, ux, uy, uz, tmp, d.K, d.Ks,
                 d.U, c->stream);
  hipError_t e = hipGetLastError();
  if (tmp) {
    const hipError_t es = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);  // freed on every path; a failure here is reported by the next call
    if (e == hipSuccess) e = es;
  }
  if (e != hipSuccess) return fail(c, HDG_EHIP, std::string("projection: ") + hipGetErrorString(e));
  c->traces_valid = false;
  c->mr_ready = false;
  return HDG_OK;
}

int hdg_project_noalloc(hdg_ctx* c, int t, const double* p, const double* ux, const double* uy,
                        const double* uz) {
  if (!c) return HDG_EINVAL;
  if (check_type(c, t) || !p || !ux || !uy || !uz) return fail(c, HDG_EINVAL, "bad type or NULL input");
  TypeData& d = c->td[t];
  int64_t chunk = d.K;
  if (t == kWedge || t == kPyr) {
    const int64_t per_elem = (int64_t)4 * d.nsample * (int64_t)sizeof(double);
    if (per_elem > kProjectScratchBytes)
      return fail(c, HDG_EINVAL, "one element's samples exceed the fixed projection work buffer");
    if (!c->pscratch) return fail(c, HDG_EHIP, "projection work buffer unavailable");
    chunk = kProjectScratchBytes / per_elem;
  }
  launch_project(t, d.K, d.nv, d.V, d.spts, d.sw, d.nsample, d.Np, d.Phi, d.gpts, p, ux, uy, uz, c->pscratch,
                 chunk, d.Ks, d.U, c->stream);
  HIPCHK(c, hipGetLastError());
  c->traces_valid = false;
  c->mr_ready = false;
  return HDG_OK;
}

int hdg_set_state(hdg_ctx* c, int t, const float* p, const float* ux, const float* uy, const float* uz) {
  if (!c) return HDG_EINVAL;
  if (check_type(c, t) || !p || !ux || !uy || !uz) return fail(c, HDG_EINVAL, "bad type or NULL input");
  TypeData& d = c->td[t];
  const size_t n = (size_t)d.K * d.Np, fs = (size_t)d.Ks * d.Np;
  const float* src[4] = {p, ux, uy, uz};
  for (int f = 0; f < 4; ++f)
    HIPCHK(c, hipMemcpyAsync(d.U + f * fs, src[f], n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  c->traces_valid = false;
  c->mr_ready = false;
  return HDG_OK;
}

int hdg_get_field(hdg_ctx* c, int which, int t, float* p, float* ux, float* uy, float* uz) {
  if (!c) return HDG_EINVAL;
  if (check_type(c, t) || !p || !ux || !uy || !uz || (which != 0 && which != 1))
    return fail(c, HDG_EINVAL, "bad type, selector or NULL output");
  TypeData& d = c->td[t];
  const size_t n = (size_t)d.K * d.Np, fs = (size_t)d.Ks * d.Np;
  const float* base = which == 0 ? d.U : d.R;
  float* dst[4] = {p, ux, uy, uz};
  for (int f = 0; f < 4; ++f)
    HIPCHK(c, hipMemcpyAsync(dst[f], base + f * fs, n * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  return HDG_OK;
}

int hdg_rhs(hdg_ctx* c) {
  if (!c) return HDG_EINVAL;
  int rc = ensure_traces(c);
  if (rc) return rc;
  return run_stage(c, kModeRhs, 0.f, 0.f, 1.f);
}

int hdg_autotune(hdg_ctx* c, int reps, int32_t* epb_out) {
  if (!c) return HDG_EINVAL;
  if (reps < 1 || reps > 1000) return fail(c, HDG_EINVAL, "reps must be in [1, 1000]");
  if (c->prof) return fail(c, HDG_ESTATE, "profiling is on: turn it off first");
  int rc = ensure_traces(c);
  if (rc) return rc;
  struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  HIPCHK(c, hipEventCreate(&ev.e[0]));
  HIPCHK(c, hipEventCreate(&ev.e[1]));
  for (int t = 0; t < 4; ++t) {
    if (epb_out) epb_out[t] = 0;
    const TypeData& d = c->td[t];
    int opts[4];
    // (hexahedra and wedges; the other types' kernels keep their shapes)
    const int n = d.present ? stage_epb_options(t, c->N, opts) : 0;
    if (n == 0) continue;
    const StageArgs a = stage_args(c, d, kModeRhs, 0.f, 0.f, 1.f);
    int best = 0;
    float best_ms = 0.f;
    for (int i = 0; i < n; ++i) {
      c->epb[t] = opts[i];
      if ((rc = launch_type(c, t, a, false))) return rc;  // first launch untimed
      HIPCHK(c, hipEventRecord(ev.e[0], c->stream));
      for (int r = 0; r < reps; ++r)
        if ((rc = launch_type(c, t, a, false))) return rc;
      HIPCHK(c, hipEventRecord(ev.e[1], c->stream));
      HIPCHK(c, hipEventSynchronize(ev.e[1]));
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
      if (best == 0 || ms < best_ms) {
        best = opts[i];
        best_ms = ms;
      }
    }
    c->epb[t] = best;
    if (epb_out) epb_out[t] = best;
  }
  // a captured graph holds the previous launch shapes
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  return HDG_OK;
}

int hdg_step(hdg_ctx* c, double dt, int64_t n_steps) {
  if (!c) return HDG_EINVAL;
  if (!(dt > 0.0) || n_steps < 0) return fail(c, HDG_EINVAL, "dt must be positive and n_steps >= 0");
  int rc = ensure_traces(c);
  if (rc) return rc;
  c->mr_ready = false;
  for (int64_t n = 0; n < n_steps; ++n) {
    for (int s = 0; s < 5; ++s)
      if ((rc = run_stage(c, kModeStage, (float)kRkA[s], (float)kRkB[s], (float)dt))) return rc;
    c->time += dt;
  }
  return HDG_OK;
}

int hdg_step_graph(hdg_ctx* c, double dt, int64_t n_steps) {
  if (!c) return HDG_EINVAL;
  if (!(dt > 0.0) || n_steps < 0) return fail(c, HDG_EINVAL, "dt must be positive and n_steps >= 0");
  if (c->prof) return fail(c, HDG_ESTATE, "profiling is on: use hdg_step");
  int rc = ensure_traces(c);
  if (rc) return rc;
  c->mr_ready = false;
  const int64_t pairs = n_steps / 2;
  if (pairs > 0) {
    if (!c->graph || c->graph_dt != dt || c->graph_cur != c->cur || c->graph_path != c->path) {
      if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
      }
      const int cur0 = c->cur;
      // the context's stream may be the default stream, which cannot be
      // captured: capture on a private stream (the graph is launched on the
      // context's stream, after the work already enqueued there)
      if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      hipStream_t user = c->stream;
      c->stream = c->cap_stream;
      const hipError_t eb = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
      if (eb != hipSuccess) {
        c->stream = user;
        return fail(c, HDG_EHIP, std::string("graph capture: ") + hipGetErrorString(eb));
      }
      for (int n = 0; n < 2 && rc == HDG_OK; ++n)
        for (int st = 0; st < 5 && rc == HDG_OK; ++st)
          rc = run_stage(c, kModeStage, (float)kRkA[st], (float)kRkB[st], (float)dt);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(c->stream, &g);
      c->stream = user;
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        c->cur = cur0;
        return rc;
      }
      if (ec != hipSuccess) return fail(c, HDG_EHIP, std::string("graph capture: ") + hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        c->graph = nullptr;
        return fail(c, HDG_EHIP, std::string("graph instantiation: ") + hipGetErrorString(ei));
      }
      c->graph_dt = dt;
      c->graph_cur = cur0;
      c->graph_path = c->path;
      // ten stages leave the buffer parity where it was
    }
    for (int64_t k = 0; k < pairs; ++k) HIPCHK(c, hipGraphLaunch(c->graph, c->stream));
    c->time += 2.0 * dt * (double)pairs;
  }
  if (n_steps % 2) return hdg_step(c, dt, 1);
  return HDG_OK;
}

// ---- multi-rate AB3 (Section 2.4) -----------------------------------------
namespace {

// AB3 dense-output weights beta_j(theta) for r_s, r_{s-1}, r_{s-2}: the
// integral over [0, theta] of the quadratic through the last three
// right-hand sides (unit step).
void ab3_beta(double th, double b[3]) {
  b[0] = th + 0.75 * th * th + th * th * th / 6.0;
  b[1] = -(th * th + th * th * th / 3.0);
  b[2] = 0.25 * th * th + th * th * th / 6.0;
}

// Lowest active level at substep k of a coarse step: level l is active when
// k is a multiple of 2^(L-l).
int lmin_of(int L, int k) {
  for (int l = 1; l <= L; ++l)
    if (k % (1 << (L - l)) == 0) return l;
  return L;
}

StageArgs mr_args(hdg_ctx* c, TypeData& d, int lmin, int k, int dense) {
  StageArgs a{};
  a.K = d.Ks;
  a.n_items = d.n_from[lmin];
  // when the elements are already stored finest level first, the active set
  // is a prefix of the storage order and tiles move as contiguous blocks
  a.elist = d.elist_identity ? nullptr : d.elist;
  a.elevel = d.elevel;
  a.ehalf = d.ehalf;
  a.slevel = c->slevel;
  a.H = d.H;
  a.tr_half = c->trace[1 - c->cur];
  a.U = d.U;
  a.R = d.R;
  a.geo = d.geo;
  a.mat = d.mat;
  a.nbr = c->nbr;
  a.ori = c->ori;
  a.tau = c->tau;
  a.fgeo = d.fgeo;
  a.isqJ = d.isqJ;
  a.tr_in = c->trace[c->cur];
  a.tr_out = c->trace[c->cur];
  a.slot0 = d.slot0;
  a.ops = d.ops;
  a.iops = d.iops;
  a.mr.L = c->L;
  a.mr.ksub = k;
  a.mr.dense = dense;
  double b1[3], bh[3];
  ab3_beta(1.0, b1);
  ab3_beta(0.5, bh);
  for (int l = 1; l <= c->L; ++l) {
    for (int j = 0; j < 3; ++j) {
      a.mr.b1[l][j] = (float)b1[j];
      a.mr.bh[l][j] = (float)bh[j];
    }
    a.mr.dtl[l] = (float)(std::ldexp(c->mr_dtmin, c->L - l));
  }
  return a;
}

// Right-hand sides of the active elements into their levels' history.
int mr_rhs(hdg_ctx* c, int k, int dense) {
  const int lmin = lmin_of(c->L, k);
  int rc0 = run_mortar(c, c->trace[c->cur], dense ? c->trace[1 - c->cur] : nullptr, k, dense);
  if (rc0) return rc0;
  for (int t = 0; t < 4; ++t) {
    TypeData& d = c->td[t];
    if (!d.present || d.n_from[lmin] == 0) continue;
    StageArgs a = mr_args(c, d, lmin, k, dense);
    a.mode = kModeRhsHist;
    for (int l = lmin; l <= c->L; ++l) a.mr.hs[l][0] = (int)(c->hcount[l] % 3);
    hipEvent_t stop;
    int rc = prof_begin(c, t, &stop);
    if (rc) return rc;
    if ((rc = launch_type(c, t, a, false))) return rc;
    if (stop) HIPCHK(c, hipEventRecord(stop, c->stream));
  }
  for (int l = lmin; l <= c->L; ++l) c->hcount[l]++;
  HIPCHK(c, hipGetLastError());
  return HDG_OK;
}

// AB3 update of the active elements, their traces and mid-step traces.
int mr_update(hdg_ctx* c, int k) {
  const int lmin = lmin_of(c->L, k);
  for (int t = 0; t < 4; ++t) {
    TypeData& d = c->td[t];
    if (!d.present || d.n_from[lmin] == 0) continue;
    StageArgs a = mr_args(c, d, lmin, k, 0);
    for (int l = lmin; l <= c->L; ++l)
      for (int j = 0; j < 3; ++j) a.mr.hs[l][j] = (int)((c->hcount[l] - 1 - j + 3 * 1000) % 3);
    hipEvent_t stop;
    int rc = prof_begin(c, kProfUpdate * 4 + t, &stop);
    if (rc) return rc;
    if ((rc = launch_type(c, t, a, true))) return rc;
    if (stop) HIPCHK(c, hipEventRecord(stop, c->stream));
  }
  HIPCHK(c, hipGetLastError());
  return HDG_OK;
}

}  // namespace

int hdg_mrab_setup(hdg_ctx* c, int n_levels, double cfl, double* dt_min_out, int64_t* level_counts_out,
                   int8_t* level_out) {
  if (!c) return HDG_EINVAL;
  if (n_levels < 1 || n_levels > 8) return fail(c, HDG_EINVAL, "n_levels must be in [1, 8]");
  std::vector<double> dte(c->n_elem);
  double dtmin = 0.0;
  int rc = hdg_dt(c, cfl, dte.data(), &dtmin);
  if (rc) return rc;
  const int L = n_levels;
  std::vector<int> lev(c->n_elem);
  for (int64_t e = 0; e < c->n_elem; ++e) {
    int j = (int)std::floor(std::log2(dte[e] / dtmin * (1.0 + 1e-12)));
    j = std::max(0, std::min(L - 1, j));
    lev[e] = L - j;
  }
  // neighbours differ by at most one level: move coarser elements finer; the
  // four elements on the sub-faces of a non-conforming coarse face share the
  // finest level among them (the coarse element then sees one level there)
  for (;;) {
    std::vector<int> nw(lev);
    for (size_t s = 0; s < c->nbr_h.size(); ++s) {
      if (c->nbr_h[s] < 0) continue;
      const int64_t a = c->slot_elem_h[s], b = c->slot_elem_h[c->nbr_h[s]];
      nw[a] = std::max(nw[a], lev[b] - 1);
    }
    for (const auto& g : c->nc_fine_elems) {
      const int mx = std::max({nw[g[0]], nw[g[1]], nw[g[2]], nw[g[3]]});
      for (int q = 0; q < 4; ++q) nw[g[q]] = mx;
    }
    if (nw == lev) break;
    lev.swap(nw);
  }
  c->L = L;
  c->mr_dtmin = dtmin;
  c->mr_dtmin0 = dtmin;
  c->level_h.assign(lev.begin(), lev.end());
  std::vector<int8_t> slev(c->nslot);
  for (int64_t s = 0; s < c->nslot; ++s) slev[s] = (int8_t)lev[c->slot_elem_h[s]];
  if (!c->slevel && (rc = dalloc(c, &c->slevel, c->nslot))) return rc;
  HIPCHK(c, hipMemcpyAsync(c->slevel, slev.data(), c->nslot, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // elements with a finer face neighbour (through a sub-face too) write
  // mid-step traces
  std::vector<int8_t> half(c->n_elem, 0);
  for (size_t s = 0; s < c->nbr_h.size(); ++s) {
    if (c->nbr_h[s] < 0) continue;
    const int64_t a = c->slot_elem_h[s], b = c->slot_elem_h[c->nbr_h[s]];
    if (lev[b] > lev[a]) half[a] = 1;
  }
  c->half_h = half;
  std::vector<int64_t> cnt(L + 1, 0);
  for (int t = 0; t < 4; ++t) {
    TypeData& d = c->td[t];
    if (!d.present) continue;
    std::vector<int> order(d.K);
    std::vector<int8_t> el(d.K), hf(d.K);
    for (int64_t k = 0; k < d.K; ++k) hf[k] = half[d.elems[k]];
    for (int64_t k = 0; k < d.K; ++k) {
      order[k] = (int)k;
      el[k] = (int8_t)lev[d.elems[k]];
      cnt[el[k]]++;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return el[x] > el[y]; });
    for (int l = 0; l <= 9; ++l) d.n_from[l] = 0;
    for (int64_t k = 0; k < d.K; ++k)
      for (int l = 1; l <= el[k]; ++l) d.n_from[l]++;
    if (!d.elist && (rc = dalloc(c, &d.elist, d.K))) return rc;
    if (!d.elevel && (rc = dalloc(c, &d.elevel, d.K))) return rc;
    if (!d.ehalf && (rc = dalloc(c, &d.ehalf, d.K))) return rc;
    HIPCHK(c, hipMemcpyAsync(d.ehalf, hf.data(), d.K, hipMemcpyHostToDevice, c->stream));
    if (!d.H && (rc = dalloc(c, &d.H, (size_t)3 * 4 * d.Ks * d.Np))) return rc;
    HIPCHK(c, hipMemcpyAsync(d.elist, order.data(), d.K * sizeof(int), hipMemcpyHostToDevice, c->stream));
    d.elist_identity = true;
    for (int64_t k = 0; k < d.K && d.elist_identity; ++k) d.elist_identity = order[k] == (int)k;
    HIPCHK(c, hipMemcpyAsync(d.elevel, el.data(), d.K, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(d.H, 0, (size_t)3 * 4 * d.Ks * d.Np * sizeof(float), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  if (dt_min_out) *dt_min_out = dtmin;
  if (level_counts_out)
    for (int l = 1; l <= L; ++l) level_counts_out[l - 1] = cnt[l];
  if (level_out)
    for (int64_t e = 0; e < c->n_elem; ++e) level_out[e] = (int8_t)lev[e];
  c->mr_ready = false;
  return HDG_OK;
}

int hdg_mrab_level_info(const hdg_ctx* c, int64_t* out) {
  if (!c || !out) return HDG_EINVAL;
  if (c->level_h.empty() || c->half_h.size() != c->level_h.size()) return HDG_ESTATE;
  const int L = c->L;
  for (int i = 0; i < 4 * L * 2; ++i) out[i] = 0;
  for (int t = 0; t < 4; ++t) {
    const TypeData& d = c->td[t];
    if (!d.present) continue;
    for (int64_t k = 0; k < d.K; ++k) {
      const int64_t e = d.elems[k];
      const int l = c->level_h[e];
      out[(t * L + l - 1) * 2] += 1;
      out[(t * L + l - 1) * 2 + 1] += c->half_h[e];
    }
  }
  return HDG_OK;
}

namespace {

// n_coarse multi-rate coarse steps after the start-up (which runs first, for
// two coarse steps, when no history is in flight); adds the simulated time.
int mrab_run(hdg_ctx* c, int64_t n_coarse, double* t_advanced) {
  int rc = ensure_traces(c);
  if (rc) return rc;
  const int L = c->L;
  const int nsub = 1 << (L - 1);
  double tadv = 0.0;
  if (!c->mr_ready) {
    // start-up: LSERK4 at dtau_min for two coarse steps, recording each
    // level's right-hand side at the boundaries that are multiples of dtau_l
    for (int l = 0; l <= 9; ++l) c->hcount[l] = 0;
    for (int j = 0; j < 2 * nsub; ++j) {
      if ((rc = mr_rhs(c, j % nsub, 0))) return rc;
      for (int s = 0; s < 5; ++s)
        if ((rc = run_stage(c, kModeStage, (float)kRkA[s], (float)kRkB[s], (float)c->mr_dtmin))) return rc;
    }
    tadv += 2.0 * nsub * c->mr_dtmin;
    c->mr_ready = true;
  }
  for (int64_t n = 0; n < n_coarse; ++n) {
    for (int k = 0; k < nsub; ++k) {
      if ((rc = mr_rhs(c, k, 1))) return rc;
      if ((rc = mr_update(c, k))) return rc;
    }
    tadv += nsub * c->mr_dtmin;
  }
  c->time += tadv;
  if (t_advanced) *t_advanced = tadv;
  return HDG_OK;
}

// flag[0] = 1 if any state value is NaN or Inf (flag cleared by a fill
// kernel, so the sequence may sit in a captured graph)
int check_finite_impl(hdg_ctx* c, bool* finite) {
  launch_fill_int(c->flag, 1, 0, c->stream);
  for (int t = 0; t < 4; ++t) {
    const TypeData& d = c->td[t];
    if (d.present) launch_finite((int64_t)4 * d.Ks * d.Np, d.U, c->flag, c->stream);
  }
  HIPCHK(c, hipGetLastError());
  int h = 0;
  HIPCHK(c, hipMemcpyAsync(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *finite = h == 0;
  return HDG_OK;
}

}  // namespace

int hdg_mrab_advance(hdg_ctx* c, int64_t n_coarse, double* t_advanced) {
  if (!c) return HDG_EINVAL;
  if (c->L < 1) return fail(c, HDG_ESTATE, "hdg_mrab_setup has not been called");
  if (n_coarse < 0) return fail(c, HDG_EINVAL, "n_coarse must be >= 0");
  return mrab_run(c, n_coarse, t_advanced);
}

int hdg_get_time(const hdg_ctx* c, double* t) {
  if (!c || !t) return HDG_EINVAL;
  *t = c->time;
  return HDG_OK;
}

int hdg_set_time(hdg_ctx* c, double t) {
  if (!c) return HDG_EINVAL;
  if (!std::isfinite(t)) return fail(c, HDG_EINVAL, "time must be finite");
  c->time = t;
  return HDG_OK;
}

int hdg_check_finite(hdg_ctx* c) {
  if (!c) return HDG_EINVAL;
  bool fin = true;
  int rc = check_finite_impl(c, &fin);
  if (rc) return rc;
  return fin ? HDG_OK : fail(c, HDG_ENONFINITE, "the state holds a NaN or Inf");
}

int hdg_advance(hdg_ctx* c, double t_final, int stepper, double cfl, int64_t check_every, int64_t* steps_done) {
  if (!c) return HDG_EINVAL;
  if (steps_done) *steps_done = 0;
  if (stepper != HDG_STEPPER_LSERK4 && stepper != HDG_STEPPER_MRAB3) return fail(c, HDG_EINVAL, "unknown stepper");
  if (!std::isfinite(t_final) || t_final < c->time) return fail(c, HDG_EINVAL, "t_final must be finite and >= t");
  if (check_every < 0) return fail(c, HDG_EINVAL, "check_every must be >= 0");
  const double span = t_final - c->time;
  int64_t n = 0, done = 0;
  int rc;
  if (stepper == HDG_STEPPER_LSERK4) {
    if (!(cfl > 0.0)) return fail(c, HDG_EINVAL, "CFL constant must be positive");
    double dtmin = 0.0;
    if ((rc = hdg_dt(c, cfl, nullptr, &dtmin))) return rc;
    if (span > 0.0) n = std::max<int64_t>(1, (int64_t)std::ceil(span / dtmin * (1.0 - 1e-12)));
    const double dt = n > 0 ? span / (double)n : 0.0;
    const double t0 = c->time;
    while (done < n) {
      const int64_t m = check_every > 0 ? std::min(check_every, n - done) : n - done;
      if ((rc = hdg_step(c, dt, m))) return rc;
      done += m;
      if (steps_done) *steps_done = done;
      bool fin = true;
      if ((rc = check_finite_impl(c, &fin))) return rc;
      if (!fin)
        return fail(c, HDG_ENONFINITE, "non-finite state after LSERK4 step " + std::to_string(done));
    }
    c->time = n > 0 ? t_final : t0;
    return HDG_OK;
  }
  if (c->L < 1) return fail(c, HDG_ESTATE, "hdg_mrab_setup has not been called");
  const int nsub = 1 << (c->L - 1);
  if (span > 0.0) {
    n = std::max<int64_t>(1, (int64_t)std::ceil(span / (nsub * c->mr_dtmin0) * (1.0 - 1e-12)));
    double dtmin = span / ((double)n * nsub);
    if (!c->mr_ready || std::fabs(dtmin - c->mr_dtmin) > 1e-13 * c->mr_dtmin) {
      // the history in flight belongs to another step: restart it
      if (n < 2) {
        n = 2;
        dtmin = span / ((double)n * nsub);
      }
      c->mr_dtmin = dtmin;
      c->mr_ready = false;
    }
  }
  const double t0 = c->time;
  while (done < n) {
    int64_t m = check_every > 0 ? std::min(check_every, n - done) : n - done;
    int64_t run = m;
    if (!c->mr_ready) {
      m = std::max<int64_t>(m, 2);  // the start-up takes two coarse steps
      run = m - 2;
    }
    if ((rc = mrab_run(c, run, nullptr))) return rc;
    done += m;
    if (steps_done) *steps_done = done;
    bool fin = true;
    if ((rc = check_finite_impl(c, &fin))) return rc;
    if (!fin) return fail(c, HDG_ENONFINITE, "non-finite state after coarse step " + std::to_string(done));
  }
  c->time = n > 0 ? t_final : t0;
  return HDG_OK;
}

// ---- checkpoint / resume ---------------------------------------------------
namespace {

struct CkptHeader {
  char magic[8];
  int32_t N, L, mr_ready, pad;
  int64_t K[4];
  int32_t Np[4];
  int32_t hmod[10];
  double time, mr_dtmin, mr_dtmin0;
  int64_t level_count[10];
  uint64_t level_hash;
};

uint64_t level_hash(const std::vector<int8_t>& lev) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a
  for (int8_t v : lev) {
    h ^= (uint8_t)v;
    h *= 1099511628211ull;
  }
  return h;
}

int64_t ckpt_bytes(const hdg_ctx* c, bool with_hist) {
  int64_t b = sizeof(CkptHeader);
  for (int t = 0; t < 4; ++t) {
    const TypeData& d = c->td[t];
    if (!d.present) continue;
    b += (int64_t)4 * d.K * d.Np * (int64_t)sizeof(float);
    if (with_hist) b += (int64_t)12 * d.K * d.Np * (int64_t)sizeof(float);
  }
  return b;
}

}  // namespace

int hdg_checkpoint_size(const hdg_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return HDG_EINVAL;
  *bytes = ckpt_bytes(c, c->L >= 1 && c->mr_ready);
  return HDG_OK;
}

int hdg_checkpoint_save(hdg_ctx* c, void* buf, int64_t bytes) {
  if (!c) return HDG_EINVAL;
  if (!buf) return fail(c, HDG_EINVAL, "checkpoint buffer is NULL");
  const bool hist = c->L >= 1 && c->mr_ready;
  if (bytes < ckpt_bytes(c, hist)) return fail(c, HDG_EINVAL, "checkpoint buffer too small");
  CkptHeader h{};
  std::memcpy(h.magic, "HDGCKPT1", 8);
  h.N = c->N;
  h.L = c->L;
  h.mr_ready = hist ? 1 : 0;
  for (int t = 0; t < 4; ++t) {
    h.K[t] = c->td[t].K;
    h.Np[t] = c->td[t].present ? c->td[t].Np : 0;
  }
  for (int l = 0; l < 10; ++l) h.hmod[l] = (int32_t)(c->hcount[l] % 3);
  h.time = c->time;
  h.mr_dtmin = c->mr_dtmin;
  h.mr_dtmin0 = c->mr_dtmin0;
  for (int8_t v : c->level_h) h.level_count[v]++;
  h.level_hash = level_hash(c->level_h);
  char* p = static_cast<char*>(buf);
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  for (int t = 0; t < 4; ++t) {
    const TypeData& d = c->td[t];
    if (!d.present) continue;
    // fields unpadded in the checkpoint: K Np values each
    const size_t n = (size_t)d.K * d.Np * sizeof(float), fs = (size_t)d.Ks * d.Np;
    for (int f = 0; f < 4; ++f, p += n) HIPCHK(c, hipMemcpyAsync(p, d.U + f * fs, n, hipMemcpyDeviceToHost, c->stream));
    if (hist)
      for (int f = 0; f < 12; ++f, p += n)
        HIPCHK(c, hipMemcpyAsync(p, d.H + f * fs, n, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HDG_OK;
}

int hdg_checkpoint_load(hdg_ctx* c, const void* buf, int64_t bytes) {
  if (!c) return HDG_EINVAL;
  if (!buf || bytes < (int64_t)sizeof(CkptHeader)) return fail(c, HDG_EINVAL, "checkpoint buffer too small");
  CkptHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, "HDGCKPT1", 8) != 0) return fail(c, HDG_EINVAL, "not a checkpoint of this library");
  if (h.N != c->N) return fail(c, HDG_EINVAL, "checkpoint of another order");
  for (int t = 0; t < 4; ++t)
    if (h.K[t] != c->td[t].K) return fail(c, HDG_EINVAL, "checkpoint of another mesh");
  const bool hist = h.mr_ready != 0;
  if (hist) {
    if (h.L != c->L) return fail(c, HDG_EINVAL, "checkpoint of another multi-rate set-up (levels)");
    int64_t cnt[10] = {};
    for (int8_t v : c->level_h) cnt[v]++;
    for (int l = 0; l < 10; ++l)
      if (cnt[l] != h.level_count[l]) return fail(c, HDG_EINVAL, "checkpoint of another multi-rate set-up");
    if (h.level_hash != level_hash(c->level_h))
      return fail(c, HDG_EINVAL, "checkpoint of another multi-rate set-up (levels differ)");
  }
  if (bytes < ckpt_bytes(c, hist)) return fail(c, HDG_EINVAL, "checkpoint buffer too small");
  const char* p = static_cast<const char*>(buf) + sizeof(h);
  for (int t = 0; t < 4; ++t) {
    TypeData& d = c->td[t];
    if (!d.present) continue;
    const size_t n = (size_t)d.K * d.Np * sizeof(float), fs = (size_t)d.Ks * d.Np;
    for (int f = 0; f < 4; ++f, p += n) HIPCHK(c, hipMemcpyAsync(d.U + f * fs, p, n, hipMemcpyHostToDevice, c->stream));
    if (hist)
      for (int f = 0; f < 12; ++f, p += n)
        HIPCHK(c, hipMemcpyAsync(d.H + f * fs, p, n, hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->time = h.time;
  c->traces_valid = false;
  c->mr_ready = hist;
  if (hist) {
    for (int l = 0; l < 10; ++l) c->hcount[l] = h.hmod[l];
    c->mr_dtmin = h.mr_dtmin;
    c->mr_dtmin0 = h.mr_dtmin0;
  }
  return HDG_OK;
}

int hdg_energy(hdg_ctx* c, double* E) {
  if (!c || !E) return HDG_EINVAL;
  double total = 0.0;
  std::vector<double> part;
  for (int t = 0; t < 4; ++t) {
    TypeData& d = c->td[t];
    if (!d.present) continue;
    EnergyArgs a{};
    a.type = t;
    a.K = d.K;
    a.Ks = d.Ks;
    a.Np = d.Np;
    a.U = d.U;
    a.geo = d.geo;
    a.mat = d.mat;
    a.Mhat = d.Mhat;
    a.partial = c->partial;
    const int nb = launch_energy(a, c->stream);
    if (nb < 0) return fail(c, HDG_EINVAL, "internal: no energy kernel for this order");
    HIPCHK(c, hipGetLastError());
    part.resize(nb);
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (double v : part) total += v;
  }
  *E = total;
  return std::isfinite(total) ? HDG_OK : fail(c, HDG_ENONFINITE, "energy is not finite");
}

int hdg_set_path(hdg_ctx* c, int path) {
  if (!c) return HDG_EINVAL;
  if (path != HDG_PATH_AUTO && path != HDG_PATH_GENERIC) return fail(c, HDG_EINVAL, "unknown path");
  if (c->mr_ready) return fail(c, HDG_ESTATE, "the path cannot change after hdg_mrab_setup");
  if (path == HDG_PATH_GENERIC && c->n_nc > 0)
    return fail(c, HDG_EINVAL, "non-conforming faces need the lattice-trace path");
  if (path != c->path) {
    c->path = path;
    c->traces_valid = false;
  }
  return HDG_OK;
}

int hdg_get_path(const hdg_ctx* c, int* path_out, int* lattice_out) {
  if (!c) return HDG_EINVAL;
  if (path_out) *path_out = c->path;
  if (lattice_out) *lattice_out = use_lattice(c) ? 1 : 0;
  return HDG_OK;
}

int hdg_profile(hdg_ctx* c, int on) {
  if (!c) return HDG_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->prof = on != 0;
  c->ev_used = 0;
  return HDG_OK;
}

int hdg_profile_read(hdg_ctx* c, double* ms_out, int64_t* count_out) {
  if (!c) return HDG_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double ms[12] = {};
  int64_t cnt[12] = {};
  for (size_t i = 0; i < c->ev_used; ++i) {
    float v = 0.f;
    HIPCHK(c, hipEventElapsedTime(&v, c->ev_pool[i][0], c->ev_pool[i][1]));
    ms[c->ev_type[i]] += v;
    cnt[c->ev_type[i]] += 1;
  }
  for (int k = 0; k < 12; ++k) {
    if (ms_out) ms_out[k] = ms[k];
    if (count_out) count_out[k] = cnt[k];
  }
  c->ev_used = 0;
  return HDG_OK;
}

}  // extern "C"
