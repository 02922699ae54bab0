// Host-side FP64 reference elements of the hybrid-mesh DG method.
//
// Everything here is set-up arithmetic: 1D Gauss rules (Newton iteration on
// Jacobi polynomials), the four reference elements of Section 2.1, the face
// rules of Section 2.3 (placed in a canonical face frame), and the tables that
// turn a face orientation into an index permutation.
#pragma once

#include <array>
#include <cstdint>
#include <vector>

namespace hdg {

constexpr int kHex = 0, kWedge = 1, kPyr = 2, kTet = 3;
constexpr int kMaxN = 5;

using Vec = std::vector<double>;

// ---- 1D ------------------------------------------------------------------
double jacobi_p(int n, double a, double b, double x);
double jacobi_dp(int n, double a, double b, double x);
void gauss_jacobi(int n, double a, double b, Vec& x, Vec& w);
double lagrange_1d(const Vec& nodes, int j, double y);
double dlagrange_1d(const Vec& nodes, int j, double y);

// Dense row-major inverse by LU with partial pivoting; returns false if singular.
bool invert(int n, const Vec& A, Vec& Ainv);

// ---- element geometry descriptions ---------------------------------------
struct ElemDesc {
  int nv;                 // vertices
  int nf;                 // faces
  double vref[8][3];      // reference vertex coordinates
  int fnv[6];             // vertices per face (3 or 4)
  int fv[6][4];           // local face vertex lists (cyclic for quadrilaterals)
  double nref[6][3];      // reference outward normals (direction only)
  double farea[6];        // true reference face areas
};
const ElemDesc& elem_desc(int type);

// ---- face rules and orientation tables (shared by all element types) -----
struct FaceTables {
  int N, n1, Nfq, Nfn;
  Vec tri_eta, tri_w;      // canonical triangle cubature [Nfq][2], weights (sum 2)
  Vec quad_eta, quad_w;    // canonical quadrilateral GL tensor rule [Nfq][2]
  Vec lattice;             // equispaced triangle lattice [Nfn][2] (face frame)
  std::vector<std::array<int, 3>> lattice_ij;  // (i, j) lattice indices
  Vec Ican;                // [Nfq][Nfn] lattice -> canonical triangle cubature
  std::vector<int> quad_perm;  // [8][Nfq] canonical point -> local point
  std::vector<int> tri_perm;   // [6][Nfn] canonical lattice node -> local node
};
void build_face_tables(int N, FaceTables& ft);
// Lagrange basis of the equispaced face lattice at face-frame points
// pts [np][2] (reference triangle (-1,-1), (1,-1), (-1,1)): out [np][Nfn].
void tri_lattice_basis(const FaceTables& ft, const Vec& pts, Vec& out);
// Mass matrix of the lattice Lagrange basis on the reference triangle,
// Ican^T W Ican (exact: the canonical rule integrates degree 2N): [Nfn][Nfn].
Vec tri_lattice_mass(const FaceTables& ft);

// Orientation code of an element face from the global ids of its local
// vertices (in the face's local order): triangles 0..5, quadrilaterals 0..7.
// perm_out receives the local positions of canonical vertices c0..c_{nv-1}.
int face_orientation(int nv, const int64_t* gids, int* perm_out);
// Local positions of canonical vertices for an orientation code.
void orientation_perm(int nv, int code, int* perm_out);

// ---- per-type reference operators -----------------------------------------
struct HexRef {
  int N, n1, Np;
  Vec x1, w1;       // GL nodes / weights
  Vec D1;           // [n1][n1]  D1[i][j] = l_j'(x_i)
  Vec Lm, Lp;       // l_j(-1), l_j(+1)
};
struct TetRef {
  int N, Np, Nfn;
  Vec nodes;              // [Np][3]
  Vec Dr, Ds, Dt;         // [Np][Np]
  Vec Mhat, Minv;         // [Np][Np]
  std::vector<int> fnode; // [4][Nfn] element node of local face lattice node
};
struct WedgeRef {
  int N, n1, Ntri, Np, Nct;
  Vec tri_pts, tri_w;          // [Nct][2] (r,t), weights (sum 2)
  Vec Pt, Ptr, Ptt;            // [Nct][Ntri] triangle basis and r,t derivatives
  Vec P1, dP1;                 // [n1][n1] 1D basis at GL points: P1[q][j]
  Vec P1m, P1p;                // 1D basis at s = -1, +1: [n1]
  Vec Ftri;                    // [Nfn][Ntri] triangle basis at face lattice nodes (r,t)
  Vec Fedge;                   // [3][n1][Ntri] triangle basis at quad-face edge points
  Vec vol_pts, vol_w;          // [n1*Nct][3], weights; q = qs*Nct + qt
  Vec Phi;                     // [n1*Nct][Np] full basis at volume points (projection)
};
struct PyrRef {
  int N, Np, Nfn, Nfq;
  std::vector<std::array<int, 3>> idx;  // (i, j, k) per dof
  Vec geo_pts;                // [Np][3] (a_i^k, b_j^k, -1)
  Vec Dr, Ds, Dt;             // [Np][Np]  D^r_{ij} = int phi_i d_r phi_j
  Vec Ftri;                   // [4][Nfn][Np] basis at tri-face lattice nodes
  Vec Fquad;                  // [Nfq][Np] basis at base GL points
  Vec proj_pts, proj_w;       // projection rule [Nq][3]
  Vec Phi;                    // [Nq][Np]
  double basis(int m, double r, double s, double t) const;
  Vec gl_x[kMaxN + 1], gl_w[kMaxN + 1];
  Vec gamma;                  // c-normalisation per level k
};

void build_hex(int N, HexRef& h);
void build_tet(int N, const FaceTables& ft, TetRef& t);
void build_wedge(int N, const FaceTables& ft, WedgeRef& w);
void build_pyr(int N, const FaceTables& ft, PyrRef& p);

// Computed trace constants C_T(N), Appendix B (GL formulation), 1 <= N <= 9.
double trace_constant(int type, int N);

int np_of(int type, int N);

}  // namespace hdg
