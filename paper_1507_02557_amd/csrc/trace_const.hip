// Per-element trace-inequality constants C_T(N, K) (Section 3.4: the largest
// eigenvalue of M_s,K v = lambda M_K v, which bounds the real part of the
// spectrum through eq. bnd_re and gives the local steps of eq. dtK with the
// mapped element's own constant).
//
// M_K is the element's mass matrix of the method (hexahedra diag(w J), wedges
// I, pyramids diag(J), tetrahedra J Mhat) and M_s,K = sum_f V_f^T S_f V_f,
// with V_f the element basis at face f's canonical cubature points for the
// face's orientation and S_f the weights w_q J^s_q (wedges: times 1/J at the
// point, the LSC basis being phi / sqrt(J)).  One wavefront per element runs
// Lanczos in FP64 on the symmetric C = M^-1/2 M_s M^-1/2 (matrix-free: a face
// evaluation and its transpose per step) and finds the largest eigenvalue of
// the Lanczos tridiagonal matrix by 64-way multisection of its Sturm count.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace hdg {
namespace {

constexpr int kHex = 0, kWedge = 1, kPyr = 2, kTet = 3;  // element types
constexpr int kWaves = 4;           // wavefronts (elements) per block
constexpr int kNpMax = 216;         // hexahedron, N = 5
constexpr int kNfqMax = 36;
constexpr int kItersMax = 96;

struct WaveMem {
  double v0[kNpMax], v1[kNpMax], u[kNpMax], z[kNpMax], d[kNpMax];
  double s[6][kNfqMax];
  double fv[kNfqMax];
  double alpha[kItersMax], beta[kItersMax];
};

__device__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// number of eigenvalues of the m x m tridiagonal (alpha, beta) below x
__device__ int sturm_count(const double* al, const double* be, int m, double x) {
  int c = 0;
  double q = al[0] - x;
  if (q < 0.0) ++c;
  for (int i = 1; i < m; ++i) {
    const double qq = q != 0.0 ? q : 1e-300;
    q = al[i] - x - be[i - 1] * be[i - 1] / qq;
    if (q < 0.0) ++c;
  }
  return c;
}

__global__ __launch_bounds__(64 * kWaves) void trace_constant_kernel(TraceConstArgs a) {
  __shared__ WaveMem mem[kWaves];
  const int lane = threadIdx.x & 63;
  WaveMem& w = mem[threadIdx.x >> 6];
  const int Np = a.Np, Nfq = a.Nfq, nf = a.nf;
  const int iters = a.iters < Np ? a.iters : Np;
  for (int64_t e = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); e < a.K; e += (int64_t)gridDim.x * kWaves) {
    // face weights and the mass scaling M^-1/2
    for (int it = lane; it < nf * Nfq; it += 64) {
      const int f = it / Nfq, q = it % Nfq;
      double s;
      if (a.type == kTet) s = a.tri_w[q] * (double)a.fgeo[e * nf + f].w;
      else s = (double)a.fgeo[(e * nf + f) * Nfq + q].w;
      if (a.type == kWedge) {
        const double r = (double)a.isqJ[(e * nf + f) * Nfq + q];
        s *= r * r;
      }
      w.s[f][q] = s;
    }
    double sJ = 1.0;  // tetrahedra: 1 / sqrt(J)
    if (a.type == kTet) sJ = sqrt((double)a.geo[e * 12 + 9]);
    for (int i = lane; i < Np; i += 64) {
      double d = 1.0;
      if (a.type == kHex) d = sqrt((double)a.geo[(e * 10 + 9) * Np + i]);          // 1 / sqrt(w J)
      else if (a.type == kPyr) d = 1.0 / sqrt((double)a.geo[(e * 10 + 9) * Np + i]);  // 1 / sqrt(J)
      w.d[i] = d;
      w.v0[i] = 0.0;
      w.v1[i] = 1.0 + 0.125 * sin(1.0 + 0.37 * i);  // fixed start vector
    }
    wave_sync();
    {
      double nn = 0.0;
      for (int i = lane; i < Np; i += 64) nn += w.v1[i] * w.v1[i];
      nn = sqrt(wave_sum(nn));
      for (int i = lane; i < Np; i += 64) w.v1[i] /= nn;
    }
    wave_sync();
    int m = iters;
    double bprev = 0.0;
    for (int k = 0; k < iters; ++k) {
      // u = M^-1/2 v1
      for (int i = lane; i < Np; i += 64) {
        double x;
        if (a.type == kTet) {
          x = 0.0;
          for (int j = i; j < Np; ++j) x += a.Linv[j * Np + i] * w.v1[j];  // L^-T v1
          x *= sJ;
        } else {
          x = w.d[i] * w.v1[i];
        }
        w.u[i] = x;
        w.z[i] = 0.0;
      }
      wave_sync();
      // z = sum_f V_f^T S_f V_f u
      for (int f = 0; f < nf; ++f) {
        const int o = a.ori[a.slot0 + e * nf + f];
        const double* V = a.V + ((int64_t)(f * 8 + o) * Nfq) * Np;
        if (lane < Nfq) {
          double t = 0.0;
          for (int j = 0; j < Np; ++j) t += V[lane * Np + j] * w.u[j];
          w.fv[lane] = w.s[f][lane] * t;
        }
        wave_sync();
        for (int j = lane; j < Np; j += 64) {
          double t = 0.0;
          for (int q = 0; q < Nfq; ++q) t += V[q * Np + j] * w.fv[q];
          w.z[j] += t;
        }
        wave_sync();
      }
      // y = M^-1/2 z, alpha = y . v1, y -= alpha v1 + beta v0
      double al = 0.0;
      for (int i = lane; i < Np; i += 64) {
        double y;
        if (a.type == kTet) {
          y = 0.0;
          for (int j = 0; j <= i; ++j) y += a.Linv[i * Np + j] * w.z[j];  // L^-1 z
          y *= sJ;
        } else {
          y = w.d[i] * w.z[i];
        }
        w.u[i] = y;
        al += y * w.v1[i];
      }
      al = wave_sum(al);
      double bb = 0.0;
      for (int i = lane; i < Np; i += 64) {
        const double y = w.u[i] - al * w.v1[i] - bprev * w.v0[i];
        w.u[i] = y;
        bb += y * y;
      }
      bb = sqrt(wave_sum(bb));
      if (lane == 0) {
        w.alpha[k] = al;
        w.beta[k] = bb;
      }
      if (!(bb > 1e-13 * fabs(al)) || k == iters - 1) {
        m = k + 1;
        break;
      }
      for (int i = lane; i < Np; i += 64) {
        w.v0[i] = w.v1[i];
        w.v1[i] = w.u[i] / bb;
      }
      bprev = bb;
      wave_sync();
    }
    wave_sync();
    // largest eigenvalue of the tridiagonal matrix: Gershgorin interval, then
    // 64-way multisection of the Sturm count
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
      const double r = (i > 0 ? fabs(w.beta[i - 1]) : 0.0) + (i + 1 < m ? fabs(w.beta[i]) : 0.0);
      lo = fmin(lo, w.alpha[i] - r);
      hi = fmax(hi, w.alpha[i] + r);
    }
    for (int round = 0; round < 12; ++round) {
      const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
      const bool all_below = sturm_count(w.alpha, w.beta, m, x) >= m;  // every eigenvalue < x
      const uint64_t mask = __ballot(all_below);
      // first multisection point above every eigenvalue
      const int first = mask ? __ffsll((unsigned long long)mask) - 1 : 64;
      const double nhi = first < 64 ? lo + (hi - lo) * (double)(first + 1) / 65.0 : hi;
      const double nlo = lo + (hi - lo) * (double)first / 65.0;
      lo = nlo;
      hi = nhi;
    }
    if (lane == 0) a.out[e] = 0.5 * (lo + hi);
    wave_sync();
  }
}

}  // namespace

void launch_trace_constants(const TraceConstArgs& a, hipStream_t s) {
  if (a.K <= 0) return;
  const int64_t nblk = (a.K + kWaves - 1) / kWaves;
  const unsigned grid = (unsigned)(nblk < 4096 ? nblk : 4096);
  hipLaunchKernelGGL(trace_constant_kernel, dim3(grid), dim3(64 * kWaves), 0, s, a);
}

}  // namespace hdg
