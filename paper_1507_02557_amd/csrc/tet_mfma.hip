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

// multi-rate AB3 update of the tetrahedra (kModeMrab)
template <class S>
__global__ __launch_bounds__(64 * S::NWU, S::kUpdateWaves) void tet_mrab_update_kernel(StageArgs a) {
  __shared__ typename S::USmem sm;
  S::run_update(sm, a);
}

// wavefronts per block: as many as fit the LDS (operator fragments are held
// once per block)
template <int N, int P, int NW, bool ST>
constexpr bool tet_fits() {
  return sizeof(typename TetMfma<N, NW, P, ST>::Smem) <= 160 * 1024;
}
// (split-precision stage kernels above N = 2 need more than the 256
// registers a lane gets at 8 wavefronts per block)
template <int N, int P, bool ST>
constexpr int tet_waves() {
  return (tet_fits<N, P, 8, ST>() && (P == 0 || N <= 2 || !ST))
             ? 8
             : (tet_fits<N, P, 4, ST>() ? 4 : (tet_fits<N, P, 2, ST>() ? 2 : 1));
}
template <int N, int P, bool ST = true>
using TetM = TetMfma<N, tet_waves<N, P, ST>(), P, ST>;

template <class S>
static int go_mfma(const StageArgs& a, hipStream_t s, int max_blocks) {
  static_assert(sizeof(typename S::Smem) <= 160 * 1024, "LDS budget exceeded");
  static_assert(sizeof(typename S::USmem) <= 160 * 1024, "LDS budget of the update kernel exceeded");
  if (a.n_items == 0) return 0;
  const int64_t ntile = (a.n_items + 15) / 16;
  if (a.mode == kModeMrab) {
    // persistent grid of the blocks the device holds at once
    static const int64_t per_cu = [] {
      int b = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &b, reinterpret_cast<const void*>(&tet_mrab_update_kernel<S>), 64 * S::NWU, 0) != hipSuccess || b < 1)
        b = 1;
      return (int64_t)b;
    }();
    const int64_t nblk = (ntile + S::NWU - 1) / S::NWU;
    const int64_t cap = per_cu * max_blocks;
    const unsigned grid = (unsigned)(nblk < cap ? nblk : cap);
    hipLaunchKernelGGL(tet_mrab_update_kernel<S>, dim3(grid), dim3(64 * S::NWU), 0, s, a);
    return 0;
  }
  const int64_t nblk = (ntile + S::NT / 64 - 1) / (S::NT / 64);
  const unsigned grid = (unsigned)(nblk < max_blocks ? nblk : max_blocks);
  hipLaunchKernelGGL(tet_mfma_kernel<S>, dim3(grid), dim3(S::NT), 0, s, a);
  return 0;
}

template <int N, int P>
static int go_n(const StageArgs& a, hipStream_t s, int max_blocks) {
  if (a.mode == kModeRhs || a.mode == kModeRhsHist) return go_mfma<TetM<N, P, false>>(a, s, max_blocks);
  return go_mfma<TetM<N, P>>(a, s, max_blocks);
}

template <int P>
static int launch_p(int N, const StageArgs& a, hipStream_t s, int max_blocks) {
  switch (N) {
    case 1: return go_n<1, P>(a, s, max_blocks);
    case 2: return go_n<2, P>(a, s, max_blocks);
    case 3: return go_n<3, P>(a, s, max_blocks);
    case 4: return go_n<4, P>(a, s, max_blocks);
    case 5: return go_n<5, P>(a, s, max_blocks);
  }
  return -1;
}

int launch_tet_mfma(int N, int P, const StageArgs& a, hipStream_t s, int max_blocks) {
  if (max_blocks < 1) max_blocks = 1;
  switch (P) {
    case 0: return launch_p<0>(N, a, s, max_blocks);
    case 1: return launch_p<1>(N, a, s, max_blocks);
    case 2: return launch_p<2>(N, a, s, max_blocks);
    case 3: return launch_p<3>(N, a, s, max_blocks);
    case 4: return launch_p<4>(N, a, s, max_blocks);
  }
  return -1;
}

template <int P>
static void sizes_p(int N, int* nf, int* ni) {
  switch (N) {
    case 1: *nf = TetM<1, P>::kOpsFloats; *ni = TetM<1, P>::kOpsInts; break;
    case 2: *nf = TetM<2, P>::kOpsFloats; *ni = TetM<2, P>::kOpsInts; break;
    case 3: *nf = TetM<3, P>::kOpsFloats; *ni = TetM<3, P>::kOpsInts; break;
    case 4: *nf = TetM<4, P>::kOpsFloats; *ni = TetM<4, P>::kOpsInts; break;
    default: *nf = TetM<5, P>::kOpsFloats; *ni = TetM<5, P>::kOpsInts; break;
  }
}

template <int P>
static void shape_p(int* kk, int* ki, int* npc) {
  *kk = Prec<P>::KK;
  *ki = Prec<P>::KI;
  *npc = Prec<P>::NPC;
}

void tet_mfma_frag_shape(int P, int* kk, int* ki, int* npc) {
  switch (P) {
    case 1: shape_p<1>(kk, ki, npc); break;
    case 2: shape_p<2>(kk, ki, npc); break;
    case 3: shape_p<3>(kk, ki, npc); break;
    case 4: shape_p<4>(kk, ki, npc); break;
    default: shape_p<0>(kk, ki, npc); break;
  }
}

void tet_mfma_table_sizes(int N, int P, int* nf, int* ni) {
  switch (P) {
    case 1: sizes_p<1>(N, nf, ni); break;
    case 2: sizes_p<2>(N, nf, ni); break;
    case 3: sizes_p<3>(N, nf, ni); break;
    case 4: sizes_p<4>(N, nf, ni); break;
    default: sizes_p<0>(N, nf, ni); break;
  }
}

}  // namespace hdg
