// Instantiation and dispatch of the matrix-core tetrahedron kernel (orders
// N = 1..5).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "tet_mfma.hpp"

namespace hdg {

// ---- tetrahedra on the matrix cores (lattice traces)

template <class S>
__global__ __launch_bounds__(S::NT) void tet_mfma_kernel(StageArgs a) {
  __shared__ typename S::Smem sm;
  S::run(sm, a);
}

// wavefronts per block: LDS holds the operator fragments once per block
constexpr int tet_waves(int N) { return N <= 4 ? 8 : 4; }
template <int N>
using TetM = TetMfma<N, tet_waves(N)>;

template <class S>
static int go_mfma(const StageArgs& a, hipStream_t s, int max_blocks) {
  static_assert(sizeof(typename S::Smem) <= 160 * 1024, "LDS budget exceeded");
  if (a.n_items == 0) return 0;
  const int64_t ntile = (a.n_items + 15) / 16;
  const int64_t nblk = (ntile + S::NT / 64 - 1) / (S::NT / 64);
  const unsigned grid = (unsigned)(nblk < max_blocks ? nblk : max_blocks);
  hipLaunchKernelGGL(tet_mfma_kernel<S>, dim3(grid), dim3(S::NT), 0, s, a);
  return 0;
}

int launch_tet_mfma(int N, const StageArgs& a, hipStream_t s, int max_blocks) {
  if (max_blocks < 1) max_blocks = 1;
  switch (N) {
    case 1: return go_mfma<TetM<1>>(a, s, max_blocks);
    case 2: return go_mfma<TetM<2>>(a, s, max_blocks);
    case 3: return go_mfma<TetM<3>>(a, s, max_blocks);
    case 4: return go_mfma<TetM<4>>(a, s, max_blocks);
    case 5: return go_mfma<TetM<5>>(a, s, max_blocks);
  }
  return -1;
}

void tet_mfma_table_sizes(int N, int* nf, int* ni) {
  switch (N) {
    case 1: *nf = TetM<1>::kOpsFloats; *ni = TetM<1>::kOpsInts; break;
    case 2: *nf = TetM<2>::kOpsFloats; *ni = TetM<2>::kOpsInts; break;
    case 3: *nf = TetM<3>::kOpsFloats; *ni = TetM<3>::kOpsInts; break;
    case 4: *nf = TetM<4>::kOpsFloats; *ni = TetM<4>::kOpsInts; break;
    default: *nf = TetM<5>::kOpsFloats; *ni = TetM<5>::kOpsInts; break;
  }
}

}  // namespace hdg
