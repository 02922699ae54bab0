// FP64 set-up and diagnostic kernels: geometric factors, face normals and
// surface Jacobians, sample points and projection of initial data, energy.
#include <hip/hip_runtime.h>

#include <mutex>

#include "geom.hpp"
#include "kernels.hpp"

namespace hdg {

// One thread per element: volume factors at the type's points, face factors at
// the canonical face points, and the inputs of the stable time step.
__global__ __launch_bounds__(64) void geometry_kernel(GeoArgs g) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.K) return;
  const GeoTables& T = *g.T;
  const int type = g.type;
  const int nv = T.nv[type], nf = T.nf[type];
  double V[8][3];
  load_verts(g.V, e, nv, V);
  double minJ = 1e300;   // over volume points: enters C_J^K (Section 3.4)
  double minJall;        // over volume and face points: validity check
  // ---- volume points
  for (int i = 0; i < g.nvp; ++i) {
    double x[3], F[3][3], G[3][3];
    vmap(type, V, g.vpts + 3 * i, x, F);
    const double J = inv3(F, G);
    minJ = J < minJ ? J : minJ;
    if (type == 3) {
      for (int r = 0; r < 3; ++r)
        for (int d = 0; d < 3; ++d) g.geo[e * 12 + 3 * r + d] = (float)G[r][d];
      g.geo[e * 12 + 9] = (float)(1.0 / J);
      g.geo[e * 12 + 10] = 0.f;
      g.geo[e * 12 + 11] = 0.f;
    } else if (type == 1) {
      double gJ[3];
      wedge_gradJ(V, g.vpts + 3 * i, gJ);
      const int64_t base = e * 12 * g.nvp + i;
      for (int r = 0; r < 3; ++r)
        for (int d = 0; d < 3; ++d) g.geo[base + (3 * r + d) * g.nvp] = (float)G[r][d];
      for (int d = 0; d < 3; ++d) g.geo[base + (9 + d) * g.nvp] = (float)(gJ[d] / (2.0 * J));
    } else {
      const int64_t base = e * 10 * g.nvp + i;
      for (int r = 0; r < 3; ++r)
        for (int d = 0; d < 3; ++d) g.geo[base + (3 * r + d) * g.nvp] = (float)G[r][d];
      g.geo[base + 9 * g.nvp] = (type == 0) ? (float)(1.0 / (g.vw[i] * J)) : (float)J;
    }
  }
  // ---- vertices: ||J^-1||_inf of C_J^K is taken over the volume points and
  // the corners (hex: all eight; pyramid: the four base vertices, where its
  // J, bilinear in (a, b) and independent of c, takes its extremes)
  if (type == 0 || type == 2) {
    const int ncorner = type == 0 ? 8 : 4;
    for (int v = 0; v < ncorner; ++v) {
      double x[3], F[3][3];
      const double X[3] = {T.vref[type][v][0], T.vref[type][v][1], T.vref[type][v][2]};
      vmap(type, V, X, x, F);
      const double J = det3(F);
      minJ = J < minJ ? J : minJ;
    }
  }
  // ---- faces
  minJall = minJ;
  double cj = 0.0;
  const int Nfq = T.Nfq;
  for (int f = 0; f < nf; ++f) {
    const int o = g.ori[e * nf + f];
    const int fnv = T.fnv[type][f];
    const double sref = (fnv == 3 ? 2.0 : 4.0) / T.farea[type][f];
    for (int q = 0; q < Nfq; ++q) {
      double Xr[3], xq[3], cr[3], x[3], F[3][3], G[3][3];
      face_point(T, type, g.V + e * nv * 3, f, o, q, Xr, xq, cr);
      vmap(type, V, Xr, x, F);
      const double J = inv3(F, G);
      minJall = J < minJall ? J : minJall;
      const double js = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      double out[3];
      for (int d = 0; d < 3; ++d)
        out[d] = G[0][d] * T.nref[type][f][0] + G[1][d] * T.nref[type][f][1] + G[2][d] * T.nref[type][f][2];
      const double sg = (cr[0] * out[0] + cr[1] * out[1] + cr[2] * out[2]) >= 0.0 ? 1.0 : -1.0;
      const double w = (fnv == 3) ? T.tri_w[q] : T.quad_w[q];
      const double jsr = js * sref;
      if (type == 1) {
        cj = jsr / J > cj ? jsr / J : cj;
        g.isqJ[(e * nf + f) * Nfq + q] = (float)(1.0 / sqrt(J));
      } else {
        cj = jsr > cj ? jsr : cj;
      }
      if (g.fstride == 1) {
        if (q == 0)
          g.fgeo[e * nf + f] = make_float4((float)(sg * cr[0] / js), (float)(sg * cr[1] / js),
                                           (float)(sg * cr[2] / js), (float)js);
      } else {
        g.fgeo[(e * nf + f) * Nfq + q] = make_float4((float)(sg * cr[0] / js), (float)(sg * cr[1] / js),
                                                     (float)(sg * cr[2] / js), (float)(w * js));
      }
    }
  }
  g.minJ[e] = minJall;
  g.cJ[e] = (type == 1) ? cj : cj / minJ;
}

// Physical coordinates of the sample points: out[(e*npts + i)*3 + d].
__global__ void points_kernel(int type, int64_t K, int nv, const double* Vall, const double* pts, int npts,
                              double* out) {
  const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= K * npts) return;
  const int64_t e = it / npts;
  const int i = (int)(it % npts);
  double V[8][3];
  load_verts(Vall, e, nv, V);
  double x[3], F[3][3];
  vmap(type, V, pts + 3 * i, x, F);
  for (int d = 0; d < 3; ++d) out[it * 3 + d] = x[d];
}

// Projection step 1, elements e0 .. e0+Kc-1:
// tmp[c][e-e0][q] = w_q * jw(J_q) * f_c(e, q), with jw = sqrt(J) (LSC wedge)
// or J (pyramid).
__global__ void project_weight_kernel(int type, int64_t e0, int64_t Kc, int nv, const double* Vall,
                                      const double* pts, const double* w, int npts, const double* f0,
                                      const double* f1, const double* f2, const double* f3, double* tmp) {
  const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= Kc * npts) return;
  const int64_t e = e0 + it / npts;
  const int q = (int)(it % npts);
  double V[8][3];
  load_verts(Vall, e, nv, V);
  double x[3], F[3][3];
  vmap(type, V, pts + 3 * q, x, F);
  const double J = det3(F);
  const double s = w[q] * (type == 1 ? sqrt(J) : J);
  const int64_t n = Kc * npts, gi = e0 * npts + it;
  tmp[it] = s * f0[gi];
  tmp[n + it] = s * f1[gi];
  tmp[2 * n + it] = s * f2[gi];
  tmp[3 * n + it] = s * f3[gi];
}

// Projection step 2, elements e0 .. e0+Kc-1 (fields Ks Np floats apart):
// U[c][e][i] = sum_q Phi[q][i] tmp[c][e-e0][q] / m_i, with m_i = J(a_i, b_j)
// for the pyramid and 1 for the wedge.
__global__ void project_apply_kernel(int type, int64_t e0, int64_t Kc, int64_t Ks, int nv, const double* Vall,
                                     const double* Phi, int npts, int Np, const double* geo_pts,
                                     const double* tmp, float* U) {
  const int64_t lt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (lt >= Kc * Np) return;
  const int64_t el = lt / Np, e = e0 + el, it = e * Np + lt % Np;
  const int i = (int)(lt % Np);
  double m = 1.0;
  if (type == 2) {
    double V[8][3];
    load_verts(Vall, e, nv, V);
    double x[3], F[3][3];
    vmap(type, V, geo_pts + 3 * i, x, F);
    m = det3(F);
  }
  const int64_t n = Kc * npts;
  for (int c = 0; c < 4; ++c) {
    double s = 0.0;
    for (int q = 0; q < npts; ++q) s += Phi[(int64_t)q * Np + i] * tmp[c * n + el * npts + q];
    U[(int64_t)c * Ks * Np + it] = (float)(s / m);
  }
}

__global__ void copy_samples_kernel(int64_t n, int64_t fs, const double* f0, const double* f1, const double* f2,
                                    const double* f3, float* U) {
  const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= n) return;
  U[it] = (float)f0[it];
  U[fs + it] = (float)f1[it];
  U[2 * fs + it] = (float)f2[it];
  U[3 * fs + it] = (float)f3[it];
}

// Energy 1/2 sum (p^T M p / kappa + rho u^T M u) in FP64: one wavefront per
// element (lanes over the element's nodes, so the loads of a field are
// contiguous), four wavefronts per block striding over the elements, one
// partial sum per block.  Tetrahedra: the element's values go to the LDS and
// lane i forms (M p)_i with the reference mass (symmetric, read by column so
// that consecutive lanes read consecutive entries); other types have a
// diagonal mass.
constexpr int kEnergyWaves = 4, kEnergyNpMax = 216, kTetNpMax = 56;
__global__ __launch_bounds__(64 * kEnergyWaves) void energy_kernel(EnergyArgs a) {
  __shared__ double red[kEnergyWaves];
  __shared__ float uv[kEnergyWaves][4][kTetNpMax];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int Np = a.Np;
  const int64_t n = a.Ks * Np;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kEnergyWaves + w; e < a.K; e += (int64_t)gridDim.x * kEnergyWaves) {
    const double kap = a.mat[e].x, rho = 1.0 / a.mat[e].y;
    const float* U = a.U + e * Np;
    if (a.type == 3) {
      for (int i = lane; i < Np; i += 64)
        for (int c = 0; c < 4; ++c) uv[w][c][i] = U[c * n + i];
      wave_sync();
      const double J = 1.0 / a.geo[e * 12 + 9];
      for (int i = lane; i < Np; i += 64) {
        double mu[4] = {0.0, 0.0, 0.0, 0.0};
        for (int j = 0; j < Np; ++j) {
          const double m = a.Mhat[j * Np + i];
          for (int c = 0; c < 4; ++c) mu[c] += m * uv[w][c][j];
        }
        acc += J * (uv[w][0][i] * mu[0] / kap + rho * (uv[w][1][i] * mu[1] + uv[w][2][i] * mu[2] +
                                                      uv[w][3][i] * mu[3]));
      }
      // the next element's values overwrite these only after every lane has read them
      wave_sync();
    } else {
      for (int i = lane; i < Np; i += 64) {
        double m = 1.0;
        if (a.type == 0) m = 1.0 / a.geo[(e * 10 + 9) * Np + i];
        else if (a.type == 2) m = a.geo[(e * 10 + 9) * Np + i];
        const double p = U[i], u1 = U[n + i], u2 = U[2 * n + i], u3 = U[3 * n + i];
        acc += m * (p * p / kap + rho * (u1 * u1 + u2 * u2 + u3 * u3));
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (lane == 0) red[w] = 0.5 * acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kEnergyWaves; ++k) t += red[k];
    a.partial[blockIdx.x] = t;
  }
}

__global__ void fill_int_kernel(int* p, int n, int v) {
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it < n) p[it] = v;
}

// Finite check of a float array: flag[0] = 1 if any entry is NaN or Inf.
__global__ void finite_kernel(int64_t n, const float* x, int* flag) {
  const int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= n) return;
  const float v = x[it];
  if (!(v == v) || v > 3.0e38f || v < -3.0e38f) flag[0] = 1;
}

// ---- host launchers --------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_geometry(const GeoArgs& g, hipStream_t s) {
  if (g.K == 0) return;
  hipLaunchKernelGGL(geometry_kernel, dim3(nblk(g.K, 64)), dim3(64), 0, s, g);
}

void launch_points(int type, int64_t K, int nv, const double* V, const double* pts, int npts, double* out,
                   hipStream_t s) {
  if (K == 0) return;
  hipLaunchKernelGGL(points_kernel, dim3(nblk(K * npts, 256)), dim3(256), 0, s, type, K, nv, V, pts, npts, out);
}

void launch_project(int type, int64_t K, int nv, const double* V, const double* pts, const double* w, int npts,
                    int Np, const double* Phi, const double* geo_pts, const double* f0, const double* f1,
                    const double* f2, const double* f3, double* tmp, int64_t chunk, int64_t Ks, float* U, hipStream_t s) {
  if (K == 0) return;
  if (type == 0 || type == 3) {
    hipLaunchKernelGGL(copy_samples_kernel, dim3(nblk(K * Np, 256)), dim3(256), 0, s, K * Np, Ks * Np, f0, f1, f2,
                       f3, U);
    return;
  }
  if (chunk < 1) chunk = K;
  // chunks run in stream order: each reuses tmp after the previous one has read it
  for (int64_t e0 = 0; e0 < K; e0 += chunk) {
    const int64_t Kc = K - e0 < chunk ? K - e0 : chunk;
    hipLaunchKernelGGL(project_weight_kernel, dim3(nblk(Kc * npts, 256)), dim3(256), 0, s, type, e0, Kc, nv, V,
                       pts, w, npts, f0, f1, f2, f3, tmp);
    hipLaunchKernelGGL(project_apply_kernel, dim3(nblk(Kc * Np, 256)), dim3(256), 0, s, type, e0, Kc, Ks, nv, V,
                       Phi, npts, Np, geo_pts, tmp, U);
  }
}

// Work buffer of hdg_project_noalloc: a fixed device array, one copy per GPU.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): project_scratch() returns the device
// address that hipGetSymbolAddress reports for the current device.
static __device__ __align__(256) double scratch[kProjectScratchBytes / sizeof(double)];

int project_scratch(double** ptr) {
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  *ptr = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  return 0;
}

void launch_fill_int(int* p, int n, int v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_int_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, v);
}

int launch_energy(const EnergyArgs& a, hipStream_t s) {
  if (a.K == 0) return 0;
  if (a.Np > kEnergyNpMax || (a.type == 3 && a.Np > kTetNpMax)) return -1;
  // at most K / 256 + 8 partial sums (the size of the caller's buffer)
  const int64_t want = (a.K + kEnergyWaves - 1) / kEnergyWaves, cap = a.K / 256 + 8;
  const unsigned nb = (unsigned)(want < cap ? want : cap);
  hipLaunchKernelGGL(energy_kernel, dim3(nb), dim3(64 * kEnergyWaves), 0, s, a);
  return (int)nb;
}

void launch_finite(int64_t n, const float* x, int* flag, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(finite_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, n, x, flag);
}

}  // namespace hdg
