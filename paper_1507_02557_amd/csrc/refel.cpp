// Host-side FP64 reference elements (Section 2.1 bases, Section 2.3 operators).
#include "refel.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace hdg {

// ---------------------------------------------------------------------------
// 1D: Jacobi polynomials by the three-term recurrence, Gauss-Jacobi rules by
// Newton iteration with deflation, Lagrange polynomials by the product form.
// ---------------------------------------------------------------------------
double jacobi_p(int n, double a, double b, double x) {
  if (n < 0) return 0.0;
  double p0 = 1.0;
  if (n == 0) return p0;
  double p1 = 0.5 * (a - b + (a + b + 2.0) * x);
  for (int k = 2; k <= n; ++k) {
    const double s = 2.0 * k + a + b;
    const double c1 = 2.0 * k * (k + a + b) * (s - 2.0);
    const double c2 = (s - 1.0) * (a * a - b * b);
    const double c3 = (s - 2.0) * (s - 1.0) * s;
    const double c4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * s;
    const double p2 = ((c2 + c3 * x) * p1 - c4 * p0) / c1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

double jacobi_dp(int n, double a, double b, double x) {
  if (n <= 0) return 0.0;
  return 0.5 * (n + a + b + 1.0) * jacobi_p(n - 1, a + 1.0, b + 1.0, x);
}

void gauss_jacobi(int n, double a, double b, Vec& x, Vec& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < n; ++k) {
    double z = -std::cos((2.0 * k + 1.0) * pi / (2.0 * n));
    for (int it = 0; it < 200; ++it) {
      const double p = jacobi_p(n, a, b, z);
      const double dp = jacobi_dp(n, a, b, z);
      double s = 0.0;
      for (int j = 0; j < k; ++j) s += 1.0 / (z - x[j]);
      const double delta = p / (dp - p * s);
      z -= delta;
      if (std::fabs(delta) < 1e-16) break;
    }
    x[k] = z;
  }
  std::sort(x.begin(), x.end());
  const double lc = std::lgamma(n + a + 1.0) + std::lgamma(n + b + 1.0) -
                    std::lgamma(n + a + b + 1.0) - std::lgamma(n + 1.0);
  const double c = std::exp(lc) * std::pow(2.0, a + b + 1.0);
  for (int k = 0; k < n; ++k) {
    const double dp = jacobi_dp(n, a, b, x[k]);
    w[k] = c / ((1.0 - x[k] * x[k]) * dp * dp);
  }
}

double lagrange_1d(const Vec& nodes, int j, double y) {
  double v = 1.0;
  for (size_t m = 0; m < nodes.size(); ++m)
    if ((int)m != j) v *= (y - nodes[m]) / (nodes[j] - nodes[m]);
  return v;
}

double dlagrange_1d(const Vec& nodes, int j, double y) {
  double d = 0.0;
  for (size_t k = 0; k < nodes.size(); ++k) {
    if ((int)k == j) continue;
    double term = 1.0 / (nodes[j] - nodes[k]);
    for (size_t m = 0; m < nodes.size(); ++m)
      if ((int)m != j && m != k) term *= (y - nodes[m]) / (nodes[j] - nodes[m]);
    d += term;
  }
  return d;
}

bool invert(int n, const Vec& A, Vec& Ainv) {
  Vec M(A);
  std::vector<int> piv(n);
  for (int i = 0; i < n; ++i) piv[i] = i;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(M[k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(M[i * n + k]) > best) { best = std::fabs(M[i * n + k]); p = i; }
    if (best < 1e-300) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(M[k * n + j], M[p * n + j]);
      std::swap(piv[k], piv[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = M[i * n + k] / M[k * n + k];
      M[i * n + k] = f;
      for (int j = k + 1; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
    }
  }
  Ainv.assign((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    Vec y(n, 0.0);
    for (int i = 0; i < n; ++i) {
      double s = (piv[i] == c) ? 1.0 : 0.0;
      for (int j = 0; j < i; ++j) s -= M[i * n + j] * y[j];
      y[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int j = i + 1; j < n; ++j) s -= M[i * n + j] * y[j];
      y[i] = s / M[i * n + i];
    }
    for (int i = 0; i < n; ++i) Ainv[i * n + c] = y[i];
  }
  return true;
}

// ---------------------------------------------------------------------------
// Element descriptions
// ---------------------------------------------------------------------------
static ElemDesc make_hex() {
  ElemDesc d{};
  d.nv = 8;
  d.nf = 6;
  const double v[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                          {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};
  const int f[6][4] = {{0, 3, 7, 4}, {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 2, 6, 7}, {0, 1, 2, 3}, {4, 5, 6, 7}};
  const double n[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
  for (int i = 0; i < 8; ++i)
    for (int c = 0; c < 3; ++c) d.vref[i][c] = v[i][c];
  for (int i = 0; i < 6; ++i) {
    d.fnv[i] = 4;
    d.farea[i] = 4.0;
    for (int c = 0; c < 4; ++c) d.fv[i][c] = f[i][c];
    for (int c = 0; c < 3; ++c) d.nref[i][c] = n[i][c];
  }
  return d;
}

static ElemDesc make_wedge() {
  ElemDesc d{};
  d.nv = 6;
  d.nf = 5;
  const double v[6][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {1, 1, -1}, {-1, 1, 1}};
  const int f[5][4] = {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {0, 2, 5, 3}, {1, 2, 5, 4}};
  const int nv[5] = {3, 3, 4, 4, 4};
  const double n[5][3] = {{0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {-1, 0, 0}, {1, 0, 1}};
  const double ar[5] = {2.0, 2.0, 4.0, 4.0, 4.0 * std::sqrt(2.0)};
  for (int i = 0; i < 6; ++i)
    for (int c = 0; c < 3; ++c) d.vref[i][c] = v[i][c];
  for (int i = 0; i < 5; ++i) {
    d.fnv[i] = nv[i];
    d.farea[i] = ar[i];
    for (int c = 0; c < 4; ++c) d.fv[i][c] = f[i][c];
    for (int c = 0; c < 3; ++c) d.nref[i][c] = n[i][c];
  }
  return d;
}

static ElemDesc make_pyr() {
  ElemDesc d{};
  d.nv = 5;
  d.nf = 5;
  const double v[5][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1}, {-1, -1, 1}};
  const int f[5][4] = {{0, 1, 2, 3}, {0, 3, 4, -1}, {0, 1, 4, -1}, {1, 2, 4, -1}, {3, 2, 4, -1}};
  const int nv[5] = {4, 3, 3, 3, 3};
  const double n[5][3] = {{0, 0, -1}, {-1, 0, 0}, {0, -1, 0}, {1, 0, 1}, {0, 1, 1}};
  const double ar[5] = {4.0, 2.0, 2.0, 2.0 * std::sqrt(2.0), 2.0 * std::sqrt(2.0)};
  for (int i = 0; i < 5; ++i)
    for (int c = 0; c < 3; ++c) d.vref[i][c] = v[i][c];
  for (int i = 0; i < 5; ++i) {
    d.fnv[i] = nv[i];
    d.farea[i] = ar[i];
    for (int c = 0; c < 4; ++c) d.fv[i][c] = f[i][c];
    for (int c = 0; c < 3; ++c) d.nref[i][c] = n[i][c];
  }
  return d;
}

static ElemDesc make_tet() {
  ElemDesc d{};
  d.nv = 4;
  d.nf = 4;
  const double v[4][3] = {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
  const int f[4][4] = {{0, 1, 2, -1}, {0, 1, 3, -1}, {1, 2, 3, -1}, {0, 2, 3, -1}};
  const double n[4][3] = {{0, 0, -1}, {0, -1, 0}, {1, 1, 1}, {-1, 0, 0}};
  const double ar[4] = {2.0, 2.0, 2.0 * std::sqrt(3.0), 2.0};
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < 3; ++c) d.vref[i][c] = v[i][c];
  for (int i = 0; i < 4; ++i) {
    d.fnv[i] = 3;
    d.farea[i] = ar[i];
    for (int c = 0; c < 4; ++c) d.fv[i][c] = f[i][c];
    for (int c = 0; c < 3; ++c) d.nref[i][c] = n[i][c];
  }
  return d;
}

const ElemDesc& elem_desc(int type) {
  static const ElemDesc H = make_hex(), W = make_wedge(), P = make_pyr(), T = make_tet();
  switch (type) {
    case kHex: return H;
    case kWedge: return W;
    case kPyr: return P;
    default: return T;
  }
}

int np_of(int type, int N) {
  switch (type) {
    case kHex: return (N + 1) * (N + 1) * (N + 1);
    case kWedge: return (N + 1) * (N + 1) * (N + 2) / 2;
    case kPyr: return (N + 1) * (N + 2) * (2 * N + 3) / 6;
    default: return (N + 1) * (N + 2) * (N + 3) / 6;
  }
}

// ---------------------------------------------------------------------------
// Face rules and orientation permutations
// ---------------------------------------------------------------------------
static const int kTriPerms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static const double kCorner[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};

void orientation_perm(int nv, int code, int* P) {
  if (nv == 3) {
    for (int k = 0; k < 3; ++k) P[k] = kTriPerms[code][k];
  } else {
    const int p = code / 2;
    const int d = (code % 2 == 0) ? 1 : 3;
    P[0] = p;
    P[1] = (p + d) % 4;
    P[2] = (p + 2) % 4;
    P[3] = (p + 4 - d) % 4;
  }
}

int face_orientation(int nv, const int64_t* g, int* P) {
  if (nv == 3) {
    int o[3] = {0, 1, 2};
    std::sort(o, o + 3, [&](int x, int y) { return g[x] < g[y]; });
    for (int c = 0; c < 6; ++c)
      if (kTriPerms[c][0] == o[0] && kTriPerms[c][1] == o[1] && kTriPerms[c][2] == o[2]) {
        if (P) orientation_perm(3, c, P);
        return c;
      }
    return -1;
  }
  int p = 0;
  for (int i = 1; i < 4; ++i)
    if (g[i] < g[p]) p = i;
  const int nxt = (p + 1) % 4, prv = (p + 3) % 4;
  const int code = 2 * p + (g[nxt] < g[prv] ? 0 : 1);
  if (P) orientation_perm(4, code, P);
  return code;
}

static double mono2(int a, int b, double x, double y) { return std::pow(x, a) * std::pow(y, b); }

void build_face_tables(int N, FaceTables& ft) {
  ft.N = N;
  ft.n1 = N + 1;
  const int n1 = N + 1;
  ft.Nfq = n1 * n1;
  ft.Nfn = (N + 1) * (N + 2) / 2;
  Vec xa, wa, xb, wb;
  gauss_jacobi(n1, 0.0, 0.0, xa, wa);
  gauss_jacobi(n1, 1.0, 0.0, xb, wb);
  ft.tri_eta.assign(2 * ft.Nfq, 0.0);
  ft.tri_w.assign(ft.Nfq, 0.0);
  ft.quad_eta.assign(2 * ft.Nfq, 0.0);
  ft.quad_w.assign(ft.Nfq, 0.0);
  for (int j = 0; j < n1; ++j)
    for (int i = 0; i < n1; ++i) {
      const int q = j * n1 + i;
      ft.tri_eta[2 * q] = (1.0 + xa[i]) * (1.0 - xb[j]) / 2.0 - 1.0;
      ft.tri_eta[2 * q + 1] = xb[j];
      ft.tri_w[q] = wa[i] * wb[j] / 2.0;
      ft.quad_eta[2 * q] = xa[i];
      ft.quad_eta[2 * q + 1] = xa[j];
      ft.quad_w[q] = wa[i] * wa[j];
    }
  ft.lattice.clear();
  ft.lattice_ij.clear();
  for (int j = 0; j <= N; ++j)
    for (int i = 0; i <= N - j; ++i) {
      ft.lattice.push_back(-1.0 + 2.0 * i / N);
      ft.lattice.push_back(-1.0 + 2.0 * j / N);
      ft.lattice_ij.push_back({i, j, N - i - j});
    }
  // Lagrange interpolation from the lattice: monomials x^a y^b, a+b <= N
  const int Nfn = ft.Nfn;
  std::vector<std::array<int, 2>> pw;
  for (int a = 0; a <= N; ++a)
    for (int b = 0; b + a <= N; ++b) pw.push_back({a, b});
  Vec V((size_t)Nfn * Nfn), Vi;
  for (int m = 0; m < Nfn; ++m)
    for (int k = 0; k < Nfn; ++k) V[m * Nfn + k] = mono2(pw[k][0], pw[k][1], ft.lattice[2 * m], ft.lattice[2 * m + 1]);
  if (!invert(Nfn, V, Vi)) throw std::runtime_error("singular triangle lattice Vandermonde");
  ft.Ican.assign((size_t)ft.Nfq * Nfn, 0.0);
  for (int q = 0; q < ft.Nfq; ++q)
    for (int m = 0; m < Nfn; ++m) {
      double s = 0.0;
      for (int k = 0; k < Nfn; ++k) s += mono2(pw[k][0], pw[k][1], ft.tri_eta[2 * q], ft.tri_eta[2 * q + 1]) * Vi[k * Nfn + m];
      ft.Ican[q * Nfn + m] = s;
    }
  // quadrilateral: canonical GL point -> local GL point, per orientation code
  ft.quad_perm.assign(8 * ft.Nfq, -1);
  for (int code = 0; code < 8; ++code) {
    int P[4];
    orientation_perm(4, code, P);
    for (int q = 0; q < ft.Nfq; ++q) {
      const double e1 = ft.quad_eta[2 * q], e2 = ft.quad_eta[2 * q + 1];
      double xi[2];
      for (int c = 0; c < 2; ++c)
        xi[c] = kCorner[P[0]][c] + 0.5 * (e1 + 1.0) * (kCorner[P[1]][c] - kCorner[P[0]][c]) +
                0.5 * (e2 + 1.0) * (kCorner[P[3]][c] - kCorner[P[0]][c]);
      int l1 = -1, l2 = -1;
      for (int i = 0; i < n1; ++i) {
        if (std::fabs(xa[i] - xi[0]) < 1e-12) l1 = i;
        if (std::fabs(xa[i] - xi[1]) < 1e-12) l2 = i;
      }
      if (l1 < 0 || l2 < 0) throw std::runtime_error("quad orientation map off the GL grid");
      ft.quad_perm[code * ft.Nfq + q] = l2 * n1 + l1;
    }
  }
  // triangle: canonical lattice node -> local lattice node
  ft.tri_perm.assign(6 * Nfn, -1);
  for (int code = 0; code < 6; ++code) {
    int P[3];
    orientation_perm(3, code, P);
    for (int m = 0; m < Nfn; ++m) {
      // canonical barycentric integers for canonical vertices c0, c1, c2
      const int beta[3] = {ft.lattice_ij[m][2], ft.lattice_ij[m][0], ft.lattice_ij[m][1]};
      int loc[3];
      for (int k = 0; k < 3; ++k) loc[P[k]] = beta[k];
      for (int l = 0; l < Nfn; ++l)
        if (ft.lattice_ij[l][0] == loc[1] && ft.lattice_ij[l][1] == loc[2]) ft.tri_perm[code * Nfn + m] = l;
      if (ft.tri_perm[code * Nfn + m] < 0) throw std::runtime_error("triangle orientation map failed");
    }
  }
}

void tri_lattice_basis(const FaceTables& ft, const Vec& pts, Vec& out) {
  const int N = ft.N, Nfn = ft.Nfn;
  std::vector<std::array<int, 2>> pw;
  for (int a = 0; a <= N; ++a)
    for (int b = 0; b + a <= N; ++b) pw.push_back({a, b});
  Vec V((size_t)Nfn * Nfn), Vi;
  for (int m = 0; m < Nfn; ++m)
    for (int k = 0; k < Nfn; ++k) V[m * Nfn + k] = mono2(pw[k][0], pw[k][1], ft.lattice[2 * m], ft.lattice[2 * m + 1]);
  if (!invert(Nfn, V, Vi)) throw std::runtime_error("singular triangle lattice Vandermonde");
  const size_t np = pts.size() / 2;
  out.assign(np * Nfn, 0.0);
  for (size_t q = 0; q < np; ++q)
    for (int m = 0; m < Nfn; ++m) {
      double s = 0.0;
      for (int k = 0; k < Nfn; ++k) s += mono2(pw[k][0], pw[k][1], pts[2 * q], pts[2 * q + 1]) * Vi[k * Nfn + m];
      out[q * Nfn + m] = s;
    }
}

Vec tri_lattice_mass(const FaceTables& ft) {
  const int Nfn = ft.Nfn, Nfq = ft.Nfq;
  Vec Mf((size_t)Nfn * Nfn, 0.0);
  for (int q = 0; q < Nfq; ++q)
    for (int x = 0; x < Nfn; ++x)
      for (int y = 0; y < Nfn; ++y) Mf[x * Nfn + y] += ft.Ican[q * Nfn + x] * ft.tri_w[q] * ft.Ican[q * Nfn + y];
  return Mf;
}

// ---------------------------------------------------------------------------
// Hexahedron: GL nodal (Section 2.1.1, Algorithms 1-3)
// ---------------------------------------------------------------------------
void build_hex(int N, HexRef& h) {
  h.N = N;
  h.n1 = N + 1;
  h.Np = h.n1 * h.n1 * h.n1;
  gauss_jacobi(h.n1, 0.0, 0.0, h.x1, h.w1);
  h.D1.assign(h.n1 * h.n1, 0.0);
  h.Lm.assign(h.n1, 0.0);
  h.Lp.assign(h.n1, 0.0);
  for (int i = 0; i < h.n1; ++i)
    for (int j = 0; j < h.n1; ++j) h.D1[i * h.n1 + j] = dlagrange_1d(h.x1, j, h.x1[i]);
  for (int j = 0; j < h.n1; ++j) {
    h.Lm[j] = lagrange_1d(h.x1, j, -1.0);
    h.Lp[j] = lagrange_1d(h.x1, j, 1.0);
  }
}

// ---------------------------------------------------------------------------
// Tetrahedron: nodal, equispaced nodes (Section 2.1.2, Algorithm 4)
// ---------------------------------------------------------------------------
static void tet_rule(int n, Vec& pts, Vec& w) {
  Vec xa, wa, xb, wb, xc, wc;
  gauss_jacobi(n, 0.0, 0.0, xa, wa);
  gauss_jacobi(n, 1.0, 0.0, xb, wb);
  gauss_jacobi(n, 2.0, 0.0, xc, wc);
  pts.clear();
  w.clear();
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const double a = xa[i], b = xb[j], c = xc[k];
        pts.push_back((1 + a) * (1 - b) * (1 - c) / 4.0 - 1.0);
        pts.push_back((1 + b) * (1 - c) / 2.0 - 1.0);
        pts.push_back(c);
        w.push_back(wa[i] * wb[j] * wc[k] / 8.0);
      }
}

void build_tet(int N, const FaceTables& ft, TetRef& T) {
  T.N = N;
  T.Np = np_of(kTet, N);
  T.Nfn = ft.Nfn;
  const int Np = T.Np;
  T.nodes.clear();
  for (int k = 0; k <= N; ++k)
    for (int j = 0; j <= N - k; ++j)
      for (int i = 0; i <= N - k - j; ++i) {
        T.nodes.push_back(-1.0 + 2.0 * i / N);
        T.nodes.push_back(-1.0 + 2.0 * j / N);
        T.nodes.push_back(-1.0 + 2.0 * k / N);
      }
  std::vector<std::array<int, 3>> pw;
  for (int a = 0; a <= N; ++a)
    for (int b = 0; a + b <= N; ++b)
      for (int c = 0; a + b + c <= N; ++c) pw.push_back({a, b, c});
  auto mono = [&](int k, const double* x, int d) {
    // d = -1 value, 0/1/2 derivative
    double v = 1.0;
    for (int c = 0; c < 3; ++c) {
      const int e = pw[k][c];
      if (c == d) v *= (e == 0) ? 0.0 : e * std::pow(x[c], e - 1);
      else v *= std::pow(x[c], e);
    }
    return v;
  };
  Vec V((size_t)Np * Np), Vi;
  for (int i = 0; i < Np; ++i)
    for (int k = 0; k < Np; ++k) V[i * Np + k] = mono(k, &T.nodes[3 * i], -1);
  if (!invert(Np, V, Vi)) throw std::runtime_error("singular tet Vandermonde");
  Vec* D[3] = {&T.Dr, &T.Ds, &T.Dt};
  for (int d = 0; d < 3; ++d) {
    D[d]->assign((size_t)Np * Np, 0.0);
    for (int i = 0; i < Np; ++i)
      for (int j = 0; j < Np; ++j) {
        double s = 0.0;
        for (int k = 0; k < Np; ++k) s += mono(k, &T.nodes[3 * i], d) * Vi[k * Np + j];
        (*D[d])[i * Np + j] = s;
      }
  }
  Vec pts, w;
  tet_rule(N + 2, pts, w);
  const int nq = (int)w.size();
  Vec L((size_t)nq * Np, 0.0);
  for (int q = 0; q < nq; ++q)
    for (int j = 0; j < Np; ++j) {
      double s = 0.0;
      for (int k = 0; k < Np; ++k) s += mono(k, &pts[3 * q], -1) * Vi[k * Np + j];
      L[q * Np + j] = s;
    }
  T.Mhat.assign((size_t)Np * Np, 0.0);
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) {
      double s = 0.0;
      for (int q = 0; q < nq; ++q) s += w[q] * L[q * Np + i] * L[q * Np + j];
      T.Mhat[i * Np + j] = s;
    }
  if (!invert(Np, T.Mhat, T.Minv)) throw std::runtime_error("singular tet mass");
  // face lattice nodes -> element nodes
  const ElemDesc& E = elem_desc(kTet);
  T.fnode.assign(4 * ft.Nfn, -1);
  for (int f = 0; f < 4; ++f)
    for (int m = 0; m < ft.Nfn; ++m) {
      const double l1 = ft.lattice_ij[m][0] / (double)N, l2 = ft.lattice_ij[m][1] / (double)N;
      const double l0 = 1.0 - l1 - l2;
      double X[3];
      for (int c = 0; c < 3; ++c)
        X[c] = l0 * E.vref[E.fv[f][0]][c] + l1 * E.vref[E.fv[f][1]][c] + l2 * E.vref[E.fv[f][2]][c];
      for (int i = 0; i < Np; ++i)
        if (std::fabs(T.nodes[3 * i] - X[0]) < 1e-12 && std::fabs(T.nodes[3 * i + 1] - X[1]) < 1e-12 &&
            std::fabs(T.nodes[3 * i + 2] - X[2]) < 1e-12)
          T.fnode[f * ft.Nfn + m] = i;
      if (T.fnode[f * ft.Nfn + m] < 0) throw std::runtime_error("tet face node not found");
    }
}

// ---------------------------------------------------------------------------
// Wedge: modal LSC-DG (Section 2.1.3, Algorithms 5-6), tensor of an
// orthonormal triangle basis in (r,t) and normalised Legendre in s.
// ---------------------------------------------------------------------------
static void tri_basis(int N, double r, double t, Vec& v, Vec& dr, Vec& dt) {
  const int Ntri = (N + 1) * (N + 2) / 2;
  v.assign(Ntri, 0.0);
  dr.assign(Ntri, 0.0);
  dt.assign(Ntri, 0.0);
  const double omc = 1.0 - t;
  const double a = (omc > 1e-14) ? 2.0 * (1.0 + r) / omc - 1.0 : -1.0;
  const double c = t;
  const double h = omc / 2.0;
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int k = 0; k <= N - i; ++k, ++m) {
      const double nrm = std::sqrt((2.0 * i + 1.0) * (2.0 * i + 2.0 * k + 2.0) / 4.0);
      const double A = jacobi_p(i, 0, 0, a), dA = jacobi_dp(i, 0, 0, a);
      const double Pk = jacobi_p(k, 2.0 * i + 1.0, 0, c), dPk = jacobi_dp(k, 2.0 * i + 1.0, 0, c);
      const double hi = std::pow(h, i);
      const double him1 = (i >= 1) ? std::pow(h, i - 1) : 0.0;
      const double dC = ((i >= 1) ? -(i / 2.0) * him1 * Pk : 0.0) + hi * dPk;
      v[m] = nrm * A * hi * Pk;
      dr[m] = nrm * dA * him1 * Pk;
      dt[m] = nrm * (dA * (1.0 + a) / 2.0 * him1 * Pk + A * dC);
    }
}

void build_wedge(int N, const FaceTables& ft, WedgeRef& W) {
  W.N = N;
  W.n1 = N + 1;
  W.Ntri = (N + 1) * (N + 2) / 2;
  W.Np = W.Ntri * W.n1;
  const int n1 = W.n1, Ntri = W.Ntri;
  Vec xa, wa, xc, wc, x1, w1;
  gauss_jacobi(n1, 0.0, 0.0, xa, wa);
  gauss_jacobi(n1, 1.0, 0.0, xc, wc);
  x1 = xa;
  w1 = wa;
  W.Nct = n1 * n1;
  W.tri_pts.clear();
  W.tri_w.clear();
  for (int ic = 0; ic < n1; ++ic)
    for (int ia = 0; ia < n1; ++ia) {
      W.tri_pts.push_back((1.0 + xa[ia]) * (1.0 - xc[ic]) / 2.0 - 1.0);
      W.tri_pts.push_back(xc[ic]);
      W.tri_w.push_back(wa[ia] * wc[ic] / 2.0);
    }
  W.Pt.assign((size_t)W.Nct * Ntri, 0.0);
  W.Ptr.assign((size_t)W.Nct * Ntri, 0.0);
  W.Ptt.assign((size_t)W.Nct * Ntri, 0.0);
  Vec v, dr, dt;
  for (int q = 0; q < W.Nct; ++q) {
    tri_basis(N, W.tri_pts[2 * q], W.tri_pts[2 * q + 1], v, dr, dt);
    for (int m = 0; m < Ntri; ++m) {
      W.Pt[q * Ntri + m] = v[m];
      W.Ptr[q * Ntri + m] = dr[m];
      W.Ptt[q * Ntri + m] = dt[m];
    }
  }
  W.P1.assign(n1 * n1, 0.0);
  W.dP1.assign(n1 * n1, 0.0);
  W.P1m.assign(n1, 0.0);
  W.P1p.assign(n1, 0.0);
  for (int j = 0; j < n1; ++j) {
    const double nrm = std::sqrt((2.0 * j + 1.0) / 2.0);
    for (int q = 0; q < n1; ++q) {
      W.P1[q * n1 + j] = nrm * jacobi_p(j, 0, 0, x1[q]);
      W.dP1[q * n1 + j] = nrm * jacobi_dp(j, 0, 0, x1[q]);
    }
    W.P1m[j] = nrm * jacobi_p(j, 0, 0, -1.0);
    W.P1p[j] = nrm * jacobi_p(j, 0, 0, 1.0);
  }
  W.Ftri.assign((size_t)ft.Nfn * Ntri, 0.0);
  for (int m = 0; m < ft.Nfn; ++m) {
    tri_basis(N, ft.lattice[2 * m], ft.lattice[2 * m + 1], v, dr, dt);
    for (int k = 0; k < Ntri; ++k) W.Ftri[m * Ntri + k] = v[k];
  }
  W.Fedge.assign((size_t)3 * n1 * Ntri, 0.0);
  for (int e = 0; e < 3; ++e)
    for (int i = 0; i < n1; ++i) {
      double r, t;
      if (e == 0) { r = x1[i]; t = -1.0; }        // face t = -1: xi1 = r
      else if (e == 1) { r = -1.0; t = x1[i]; }   // face r = -1: xi1 = t
      else { r = -x1[i]; t = x1[i]; }             // face r + t = 0: xi1 from (1,-1) to (-1,1)
      tri_basis(N, r, t, v, dr, dt);
      for (int k = 0; k < Ntri; ++k) W.Fedge[(e * n1 + i) * Ntri + k] = v[k];
    }
  const int Nq = n1 * W.Nct;
  W.vol_pts.assign(3 * Nq, 0.0);
  W.vol_w.assign(Nq, 0.0);
  W.Phi.assign((size_t)Nq * W.Np, 0.0);
  for (int qs = 0; qs < n1; ++qs)
    for (int qt = 0; qt < W.Nct; ++qt) {
      const int q = qs * W.Nct + qt;
      W.vol_pts[3 * q] = W.tri_pts[2 * qt];
      W.vol_pts[3 * q + 1] = x1[qs];
      W.vol_pts[3 * q + 2] = W.tri_pts[2 * qt + 1];
      W.vol_w[q] = W.tri_w[qt] * w1[qs];
      for (int js = 0; js < n1; ++js)
        for (int jt = 0; jt < Ntri; ++jt) W.Phi[(size_t)q * W.Np + js * Ntri + jt] = W.Pt[qt * Ntri + jt] * W.P1[qs * n1 + js];
    }
}

// ---------------------------------------------------------------------------
// Pyramid: semi-nodal basis and quadrature-free operators (Section 2.1.4,
// Section 2.3.4).  D^r, D^s, D^c are assembled from the factorised formulas;
// D^t = ((1+a)/2) D^r + ((1+b)/2) D^s + D^c with the (1+a)/2, (1+b)/2
// factors taken at the test node (a_l^n, b_m^n), where the GL collocation in
// (a, b) that produces the formula evaluates them.
// ---------------------------------------------------------------------------
double PyrRef::basis(int m, double r, double s, double t) const {
  const int i = idx[m][0], j = idx[m][1], k = idx[m][2];
  const double omc = 1.0 - t;
  const double a = (omc > 1e-14) ? 2.0 * (1.0 + r) / omc - 1.0 : -1.0;
  const double b = (omc > 1e-14) ? 2.0 * (1.0 + s) / omc - 1.0 : -1.0;
  const double h = omc / 2.0;
  const double la = lagrange_1d(gl_x[k], i, a), lb = lagrange_1d(gl_x[k], j, b);
  const double pc = jacobi_p(N - k, 2.0 * k + 3.0, 0.0, t);
  return la * lb * std::pow(h, k) * pc / std::sqrt(gl_w[k][i] * gl_w[k][j] * gamma[k]);
}

void build_pyr(int N, const FaceTables& ft, PyrRef& P) {
  P.N = N;
  P.Np = np_of(kPyr, N);
  P.Nfn = ft.Nfn;
  P.Nfq = ft.Nfq;
  const int Np = P.Np;
  for (int k = 0; k <= N; ++k) gauss_jacobi(k + 1, 0.0, 0.0, P.gl_x[k], P.gl_w[k]);
  P.idx.clear();
  for (int k = 0; k <= N; ++k)
    for (int j = 0; j <= k; ++j)
      for (int i = 0; i <= k; ++i) P.idx.push_back({i, j, k});
  Vec xc, wc;
  gauss_jacobi(2 * N + 6, 0.0, 0.0, xc, wc);
  const int nc = (int)xc.size();
  P.gamma.assign(N + 1, 0.0);
  for (int k = 0; k <= N; ++k) {
    double s = 0.0;
    for (int q = 0; q < nc; ++q) {
      const double h = (1.0 - xc[q]) / 2.0, pk = jacobi_p(N - k, 2.0 * k + 3.0, 0.0, xc[q]);
      s += wc[q] * std::pow(h, 2 * k + 2) * pk * pk;
    }
    P.gamma[k] = s;
  }
  // c-integrals Mc[n][k] and Mcc[n][k]
  Vec Mc((N + 1) * (N + 1), 0.0), Mcc((N + 1) * (N + 1), 0.0);
  for (int n = 0; n <= N; ++n)
    for (int k = 0; k <= N; ++k) {
      double s1 = 0.0, s2 = 0.0;
      for (int q = 0; q < nc; ++q) {
        const double c = xc[q], h = (1.0 - c) / 2.0;
        const double pk = jacobi_p(N - k, 2.0 * k + 3.0, 0.0, c), dpk = jacobi_dp(N - k, 2.0 * k + 3.0, 0.0, c);
        const double pn = jacobi_p(N - n, 2.0 * n + 3.0, 0.0, c);
        const double dE = dpk * std::pow(h, k) - ((k >= 1) ? (k / 2.0) * pk * std::pow(h, k - 1) : 0.0);
        s1 += wc[q] * std::pow(h, 1 + k + n) * pk * pn;
        s2 += wc[q] * dE * pn * std::pow(h, 2 + n);
      }
      const double nrm = std::sqrt(P.gamma[n] * P.gamma[k]);
      Mc[n * (N + 1) + k] = s1 / nrm;
      Mcc[n * (N + 1) + k] = s2 / nrm;
    }
  P.Dr.assign((size_t)Np * Np, 0.0);
  P.Ds.assign((size_t)Np * Np, 0.0);
  P.Dt.assign((size_t)Np * Np, 0.0);
  for (int row = 0; row < Np; ++row) {
    const int l = P.idx[row][0], m = P.idx[row][1], n = P.idx[row][2];
    const double al = P.gl_x[n][l], bm = P.gl_x[n][m];
    const double wl = P.gl_w[n][l], wm = P.gl_w[n][m];
    for (int col = 0; col < Np; ++col) {
      const int i = P.idx[col][0], j = P.idx[col][1], k = P.idx[col][2];
      const double sc = std::sqrt(wl * wm / (P.gl_w[k][i] * P.gl_w[k][j]));
      const double la = lagrange_1d(P.gl_x[k], i, al), lb = lagrange_1d(P.gl_x[k], j, bm);
      const double dla = dlagrange_1d(P.gl_x[k], i, al), dlb = dlagrange_1d(P.gl_x[k], j, bm);
      const double mc = Mc[n * (N + 1) + k], mcc = Mcc[n * (N + 1) + k];
      const double dr = sc * dla * lb * mc, ds = sc * la * dlb * mc, dc = sc * la * lb * mcc;
      P.Dr[row * Np + col] = dr;
      P.Ds[row * Np + col] = ds;
      P.Dt[row * Np + col] = 0.5 * (1.0 + al) * dr + 0.5 * (1.0 + bm) * ds + dc;
    }
  }
  P.geo_pts.assign(3 * Np, 0.0);
  for (int m = 0; m < Np; ++m) {
    P.geo_pts[3 * m] = P.gl_x[P.idx[m][2]][P.idx[m][0]];
    P.geo_pts[3 * m + 1] = P.gl_x[P.idx[m][2]][P.idx[m][1]];
    P.geo_pts[3 * m + 2] = -1.0;
  }
  const ElemDesc& E = elem_desc(kPyr);
  P.Ftri.assign((size_t)4 * ft.Nfn * Np, 0.0);
  for (int f = 1; f < 5; ++f)
    for (int mm = 0; mm < ft.Nfn; ++mm) {
      const double l1 = ft.lattice_ij[mm][0] / (double)N, l2 = ft.lattice_ij[mm][1] / (double)N, l0 = 1.0 - l1 - l2;
      double X[3];
      for (int c = 0; c < 3; ++c)
        X[c] = l0 * E.vref[E.fv[f][0]][c] + l1 * E.vref[E.fv[f][1]][c] + l2 * E.vref[E.fv[f][2]][c];
      for (int m = 0; m < Np; ++m) P.Ftri[((size_t)(f - 1) * ft.Nfn + mm) * Np + m] = P.basis(m, X[0], X[1], X[2]);
    }
  Vec x1, w1;
  gauss_jacobi(N + 1, 0.0, 0.0, x1, w1);
  P.Fquad.assign((size_t)ft.Nfq * Np, 0.0);
  for (int l2 = 0; l2 <= N; ++l2)
    for (int l1 = 0; l1 <= N; ++l1)
      for (int m = 0; m < Np; ++m) P.Fquad[(size_t)(l2 * (N + 1) + l1) * Np + m] = P.basis(m, x1[l1], x1[l2], -1.0);
  // projection rule GL(N+1)^2 x GJ^{(2,0)}(N+1), collapsed
  Vec xj, wj;
  gauss_jacobi(N + 1, 2.0, 0.0, xj, wj);
  P.proj_pts.clear();
  P.proj_w.clear();
  for (int ic = 0; ic <= N; ++ic)
    for (int ib = 0; ib <= N; ++ib)
      for (int ia = 0; ia <= N; ++ia) {
        const double a = x1[ia], b = x1[ib], c = xj[ic];
        P.proj_pts.push_back((1 + a) * (1 - c) / 2 - 1);
        P.proj_pts.push_back((1 + b) * (1 - c) / 2 - 1);
        P.proj_pts.push_back(c);
        P.proj_w.push_back(w1[ia] * w1[ib] * wj[ic] / 4.0);
      }
  const int nq = (int)P.proj_w.size();
  P.Phi.assign((size_t)nq * Np, 0.0);
  for (int q = 0; q < nq; ++q)
    for (int m = 0; m < Np; ++m)
      P.Phi[(size_t)q * Np + m] = P.basis(m, P.proj_pts[3 * q], P.proj_pts[3 * q + 1], P.proj_pts[3 * q + 2]);
}

// Appendix B, Table computedTrace (GL formulation), N = 1..9.
double trace_constant(int type, int N) {
  static const double T[4][9] = {
      {9, 18, 30, 45, 63, 84, 108, 135, 165},
      {9.93, 18.56, 29.03, 42.99, 58.80, 78.01, 99.27, 123.76, 150.48},
      {11.68, 20.89, 32.84, 47.59, 65.17, 85.60, 108.90, 135.07, 164.11},
      {12.22, 20.46, 29.18, 41.65, 54.45, 71.10, 88.32, 109.04, 130.67}};
  if (N < 1 || N > 9 || type < 0 || type > 3) return -1.0;
  return T[type][N - 1];
}

}  // namespace hdg
