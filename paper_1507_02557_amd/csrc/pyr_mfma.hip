// Instantiation and dispatch of the matrix-core pyramid kernel (orders
// N = 1..5; at N = 5 the operator tables exceed the LDS and are read from
// global memory in fragment order).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "pyr_mfma.hpp"

namespace hdg {

template <class S>
__global__ __launch_bounds__(S::NT) void pyr_mfma_kernel(StageArgs a) {
  __shared__ typename S::Smem sm;
  S::template run<false>(sm, a);
}

// multi-rate AB3 update of the pyramids (kModeMrab)
template <class S>
__global__ __launch_bounds__(S::NT) void pyr_mrab_update_kernel(StageArgs a) {
  __shared__ typename S::Smem sm;
  S::template run<true>(sm, a);
}

// operator tables in global memory when they do not fit the LDS beside one
// wavefront's tile
template <int N>
constexpr bool pyr_global() {
  return sizeof(typename PyrMfma<N, 1, false>::Smem) > 160 * 1024;
}
template <int N, int NW>
constexpr bool pyr_fits() {
  return sizeof(typename PyrMfma<N, NW, pyr_global<N>()>::Smem) <= 160 * 1024;
}
// (above N = 2 the kernel needs more than the 256 registers a lane gets at 8
// wavefronts per block)
template <int N>
constexpr int pyr_waves() {
  return (pyr_fits<N, 8>() && N <= 2) ? 8 : (pyr_fits<N, 4>() ? 4 : 2);
}
template <int N>
using PyrM = PyrMfma<N, pyr_waves<N>(), pyr_global<N>()>;

template <class S>
static int go(const StageArgs& a, hipStream_t s, int max_blocks) {
  static_assert(sizeof(typename S::Smem) <= 160 * 1024, "LDS budget exceeded");
  if (a.n_items == 0) return 0;
  const int64_t ntile = (a.n_items + 15) / 16;
  const int64_t nblk = (ntile + S::NT / 64 - 1) / (S::NT / 64);
  const unsigned grid = (unsigned)(nblk < max_blocks ? nblk : max_blocks);
  if (a.mode == kModeMrab) hipLaunchKernelGGL(pyr_mrab_update_kernel<S>, dim3(grid), dim3(S::NT), 0, s, a);
  else hipLaunchKernelGGL(pyr_mfma_kernel<S>, dim3(grid), dim3(S::NT), 0, s, a);
  return 0;
}

int launch_pyr_mfma(int N, const StageArgs& a, hipStream_t s, int max_blocks) {
  if (max_blocks < 1) max_blocks = 1;
  switch (N) {
    case 1: return go<PyrM<1>>(a, s, max_blocks);
    case 2: return go<PyrM<2>>(a, s, max_blocks);
    case 3: return go<PyrM<3>>(a, s, max_blocks);
    case 4: return go<PyrM<4>>(a, s, max_blocks);
    case 5: return go<PyrM<5>>(a, s, max_blocks);
  }
  return -1;
}

int pyr_mfma_global(int N) {
  switch (N) {
    case 1: return pyr_global<1>();
    case 2: return pyr_global<2>();
    case 3: return pyr_global<3>();
    case 4: return pyr_global<4>();
    case 5: return pyr_global<5>();
  }
  return 0;
}

int pyr_mfma_table_sizes(int N, int* nf, int* ni) {
  switch (N) {
    case 1: *nf = PyrM<1>::kOpsFloats; *ni = PyrM<1>::kOpsInts; return 0;
    case 2: *nf = PyrM<2>::kOpsFloats; *ni = PyrM<2>::kOpsInts; return 0;
    case 3: *nf = PyrM<3>::kOpsFloats; *ni = PyrM<3>::kOpsInts; return 0;
    case 4: *nf = PyrM<4>::kOpsFloats; *ni = PyrM<4>::kOpsInts; return 0;
    case 5: *nf = PyrM<5>::kOpsFloats; *ni = PyrM<5>::kOpsInts; return 0;
  }
  return -1;
}

}  // namespace hdg
