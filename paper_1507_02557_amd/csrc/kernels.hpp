// Host-visible launch interface of the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geom.hpp"
#include "stage_common.hpp"

namespace hdg {

struct GeoArgs {
  int type;
  int64_t K;
  const double* V;        // [K][nv][3]
  const int8_t* ori;      // [K*nf] orientation codes of this type's slots
  const GeoTables* T;     // device copy
  const double* vpts;     // volume reference points [nvp][3]
  int nvp;
  const double* vw;       // hex node weights [nvp]
  float* geo;             // volume factors (layout per type)
  float4* fgeo;           // face factors
  int fstride;            // 1 (planar tet faces) or Nfq
  float* isqJ;            // wedge only
  double* cJ;             // [K] C_J^K
  double* minJ;           // [K] minimum J over the element's points
};

struct EnergyArgs {
  int type;
  int64_t K;
  int64_t Ks;             // field stride of U in elements
  int Np;
  const float* U;
  const float* geo;
  const float2* mat;
  const double* Mhat;     // tet reference mass [Np][Np]
  double* partial;        // one per block
};

// 1:4 non-conforming triangular faces between tetrahedra with lattice traces.
// Record i: coarse (parent) slot, flux slot, the four fine slots, the four
// sub-face interpolation variants; the virtual slot that the fine element of
// sub-face s reads as its neighbour is vslot0 + 4 i + s.
constexpr int kNcRec = 10;
struct MortarArgs {
  int64_t n;              // non-conforming coarse faces
  const int* rec;         // [n][kNcRec]
  int64_t vslot0;
  int nfn, ts;            // face lattice nodes; trace stride (float4 per slot)
  const float* I;         // [nvar][nfn][nfn] coarse lattice -> sub-face lattice (canonical frames)
  const float* P;         // [nvar][nfn][nfn] sub-face lattice flux -> equivalent coarse lattice flux
  const float4* cgeo;     // coarse type's face factors [K][4] (n, J^s)
  int64_t cslot0;         // first slot of the coarse type
  const float2* tau;      // [nslot]
  float4* tr;             // traces of the current state (read; virtual and flux slots written)
  float4* tr_half;        // multi-rate mid-step traces (virtual slots written), or NULL
  const int8_t* slevel;   // multi-rate level per slot, or NULL
  int L, ksub, dense;     // multi-rate substep (dense: a coarser fine side may be mid-step)
};
void launch_mortar(const MortarArgs& a, hipStream_t s);

// Per-element trace constants C_T(N, K) of one element type (FP64).
struct TraceConstArgs {
  int type;
  int64_t K;
  int Np, nf, Nfq, iters;
  const double* V;        // [nf][8][Nfq][Np] element basis at canonical face points per orientation
  const double* tri_w;    // [Nfq] canonical triangle weights (tetrahedra)
  const double* Linv;     // tetrahedra: inverse of the Cholesky factor of Mhat [Np][Np] (lower)
  const float* geo;       // stored geometric factors of the type
  const float4* fgeo;     // face factors (n, w J^s) or, for tetrahedra, (n, J^s) per face
  const float* isqJ;      // wedges: 1 / sqrt(J) at face points
  const int8_t* ori;      // orientation codes per slot
  int64_t slot0;
  double* out;            // [K]
};
void launch_trace_constants(const TraceConstArgs& a, hipStream_t s);

void launch_geometry(const GeoArgs& g, hipStream_t s);
void launch_points(int type, int64_t K, int nv, const double* V, const double* pts, int npts, double* out,
                   hipStream_t s);
// Projection of sampled initial data into U (fields Ks Np floats apart;
// wedge, pyramid: in chunks of at most `chunk` elements through the work
// buffer tmp of 4 chunk npts doubles; chunk < 1: all K at once).
void launch_project(int type, int64_t K, int nv, const double* V, const double* pts, const double* w, int npts,
                    int Np, const double* Phi, const double* geo_pts, const double* f0, const double* f1,
                    const double* f2, const double* f3, double* tmp, int64_t chunk, int64_t Ks, float* U, hipStream_t s);
// Fixed device work buffer of the allocation-free projection (bytes per GPU).
constexpr int64_t kProjectScratchBytes = 16 * 1024 * 1024;
constexpr int kMaxDevices = 64;
// Device address of that buffer on the current device (looked up once per
// device with hipGetSymbolAddress); 0 on success, -1 on a HIP error.
int project_scratch(double** ptr);
void launch_fill_int(int* p, int n, int v, hipStream_t s);
int launch_energy(const EnergyArgs& a, hipStream_t s);
void launch_finite(int64_t n, const float* x, int* flag, hipStream_t s);

// Fused stage kernel for one element type; returns 0 or -1 if (type, N) has
// no instantiation.  eb: elements per block of the hexahedron or wedge block
// kernel, one of stage_epb_options (0: the default of stage_config.hpp).
int launch_stage(int type, int N, const StageArgs& a, hipStream_t s, int eb = 0);
// Multi-rate AB3 update of the items of a (state, traces, mid-step traces).
int launch_mrab_update(int type, int N, const StageArgs& a, hipStream_t s, int eb = 0);
// Batch sizes the block kernel of (type, N) is instantiated with (hexahedra,
// wedges; 0 for other types); out holds at least 4.
int stage_epb_options(int type, int N, int* out);
// Packed operator table sizes of the stage kernel for (type, N).
void stage_table_sizes(int type, int N, int* n_floats, int* n_ints);
int stage_batch(int type, int N);
// Tetrahedra on the matrix cores with lattice traces (all modes, including
// kModeMrab); P is the operand precision (0 FP32, 1 split FP16 16x16x32,
// 2 split FP16 16x16x16); max_blocks caps the persistent grid.
int launch_tet_mfma(int N, int P, const StageArgs& a, hipStream_t s, int max_blocks);
// Packed table sizes (in floats): D fragments [3][Mt][Ks][pieces][64][KI],
// lift fragments [4][Mt][Kf][pieces][64][KI], then 1/s_D and 1/s_L;
// integers fnode [4][Nfn], tperm [6][Nfn].
void tet_mfma_table_sizes(int N, int P, int* n_floats, int* n_ints);
// Pyramids on the matrix cores with lattice traces on their triangular faces
// (orders 1..4, all modes); returns -1 for other orders.
int launch_pyr_mfma(int N, const StageArgs& a, hipStream_t s, int max_blocks);
// Table sizes in floats / ints (D, Fq, Ft rows with odd stride, lattice lift
// fragments, w0, geometry points; base and lattice permutations and their
// inverses); -1 for orders without the kernel.
int pyr_mfma_table_sizes(int N, int* n_floats, int* n_ints);
// 1 if the order's pyramid tables are read from global memory in fragment
// order (they exceed the LDS), 0 if they are copied to the LDS row-major.
int pyr_mfma_global(int N);
// Fragment geometry of precision P: K per instruction, entries per lane, pieces.
void tet_mfma_frag_shape(int P, int* kk, int* ki, int* npc);

}  // namespace hdg
