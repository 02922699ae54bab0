// Instantiation and dispatch of the fused stage kernels (one per element type
// and order N = 1..5).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "stage_config.hpp"
#include "stage_hex.hpp"
#include "stage_pyr.hpp"
#include "stage_tet.hpp"
#include "stage_wedge.hpp"

namespace hdg {

// Minimum wavefronts per SIMD the register allocation must allow.
template <class S>
struct Occupancy {
  static constexpr int value = 1;
};
template <int N, int E, int T>
struct Occupancy<WedgeStage<N, E, T>> {
  static constexpr int value = N == 4 ? 5 : (N < 4 ? 3 : 1);
};

template <class S>
__global__ __launch_bounds__(S::NT, Occupancy<S>::value) void stage_kernel(StageArgs a) {
  __shared__ typename S::Smem sm;
  S::load_ops(threadIdx.x, sm, a);
  __syncthreads();
  constexpr int EPB = S::kEPB;
  const int64_t nb = (a.n_items + EPB - 1) / EPB;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    for (int ph = 0; ph < S::nphase; ++ph) {
      if (!S::active(ph, a.mode)) continue;
      // an opaque copy of the thread index keeps each phase's index
      // arithmetic inside the loop (hoisted out of it, the values of all
      // phases would stay live in registers across the whole batch loop)
      int t = threadIdx.x;
      __asm__ volatile("" : "+v"(t));
      S::phase(ph, t, sm, a, b * EPB);
      __syncthreads();
    }
  }
}

template <class S>
__global__ __launch_bounds__(S::NT) void mrab_update_kernel(StageArgs a) {
  __shared__ typename S::Smem sm;
  S::load_ops(threadIdx.x, sm, a);
  __syncthreads();
  constexpr int EPB = S::kEPB;
  const int64_t nb = (a.n_items + EPB - 1) / EPB;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    for (int st = 0; st < MrabUpdate<S>::nstep; ++st) {
      int t = threadIdx.x;
      __asm__ volatile("" : "+v"(t));
      MrabUpdate<S>::step(st, t, sm, a, b * EPB);
      __syncthreads();
    }
  }
}

// Wavefront-batched form (vector pyramids at N <= 4, the wedges' multi-rate
// update at N = 4): the block holds the
// operator tables once; each of its W wavefronts runs the same phases on a
// batch of its own (one element), separated by wavefront syncs instead of
// block barriers, so the wavefronts of a compute unit proceed independently
// and hide one another's memory latency.
template <class S, int W>
__global__ __launch_bounds__(64 * W) void wave_stage_kernel(StageArgs a) {
  __shared__ typename S::Ops o;
  __shared__ typename S::Batch bt[W];
  S::load_ops(threadIdx.x, 64 * W, o, a);
  __syncthreads();
  typename S::WaveRef r{o, bt[threadIdx.x >> 6]};
  constexpr int EPB = S::kEPB;
  const int64_t nb = (a.n_items + EPB - 1) / EPB;
  for (int64_t b = (int64_t)blockIdx.x * W + (threadIdx.x >> 6); b < nb; b += (int64_t)gridDim.x * W) {
    for (int ph = 0; ph < S::nphase; ++ph) {
      if (!S::active(ph, a.mode)) continue;
      int t = threadIdx.x & 63;
      __asm__ volatile("" : "+v"(t));
      S::phase(ph, t, r, a, b * EPB);
      wave_sync();
    }
  }
}

template <class S, int W>
__global__ __launch_bounds__(64 * W) void wave_mrab_update_kernel(StageArgs a) {
  __shared__ typename S::Ops o;
  __shared__ typename S::Batch bt[W];
  S::load_ops(threadIdx.x, 64 * W, o, a);
  __syncthreads();
  typename S::WaveRef r{o, bt[threadIdx.x >> 6]};
  constexpr int EPB = S::kEPB;
  const int64_t nb = (a.n_items + EPB - 1) / EPB;
  for (int64_t b = (int64_t)blockIdx.x * W + (threadIdx.x >> 6); b < nb; b += (int64_t)gridDim.x * W) {
    for (int st = 0; st < MrabUpdate<S>::nstep; ++st) {
      int t = threadIdx.x & 63;
      __asm__ volatile("" : "+v"(t));
      MrabUpdate<S>::step(st, t, r, a, b * EPB);
      wave_sync();
    }
  }
}

// Blocks of a kernel that the whole device holds at once.  The persistent
// grid is never larger: blocks beyond that number would start only when the
// first ones finish, and the last of them would run alone.
static int64_t resident_blocks(const void* kernel, int nt) {
  int per_cu = 0, dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) != hipSuccess || per_cu < 1 || ncu < 1)
    return 2048;
  return (int64_t)per_cu * ncu;
}

template <class S>
static int go(const StageArgs& a, hipStream_t s, bool mrab) {
  static_assert(sizeof(typename S::Smem) <= 160 * 1024, "LDS budget exceeded");
  if (a.n_items == 0) return 0;
  const int64_t nb = (a.n_items + S::kEPB - 1) / S::kEPB;
  int64_t cap;
  if (mrab) {
    static const int64_t c = resident_blocks(reinterpret_cast<const void*>(&mrab_update_kernel<S>), S::NT);
    cap = c;
  } else {
    static const int64_t c = resident_blocks(reinterpret_cast<const void*>(&stage_kernel<S>), S::NT);
    cap = c;
  }
  const unsigned grid = (unsigned)(nb < cap ? nb : cap);
  if (mrab) hipLaunchKernelGGL(mrab_update_kernel<S>, dim3(grid), dim3(S::NT), 0, s, a);
  else hipLaunchKernelGGL(stage_kernel<S>, dim3(grid), dim3(S::NT), 0, s, a);
  return 0;
}

template <class S, int W>
static int go_wave(const StageArgs& a, hipStream_t s, bool mrab) {
  static_assert(S::NT == 64, "one wavefront per batch");
  static_assert(sizeof(typename S::Ops) + W * sizeof(typename S::Batch) <= 160 * 1024, "LDS budget exceeded");
  if (a.n_items == 0) return 0;
  const int64_t nb = (a.n_items + S::kEPB - 1) / S::kEPB;
  const int64_t nblk = (nb + W - 1) / W;
  int64_t cap;
  if (mrab) {
    static const int64_t c = resident_blocks(reinterpret_cast<const void*>(&wave_mrab_update_kernel<S, W>), 64 * W);
    cap = c;
  } else {
    static const int64_t c = resident_blocks(reinterpret_cast<const void*>(&wave_stage_kernel<S, W>), 64 * W);
    cap = c;
  }
  const unsigned grid = (unsigned)(nblk < cap ? nblk : cap);
  if (mrab) hipLaunchKernelGGL((wave_mrab_update_kernel<S, W>), dim3(grid), dim3(64 * W), 0, s, a);
  else hipLaunchKernelGGL((wave_stage_kernel<S, W>), dim3(grid), dim3(64 * W), 0, s, a);
  return 0;
}

template <class S>
static void sizes(int* nf, int* ni) {
  *nf = S::kOpsFloats;
  *ni = S::kOpsInts;
}

// Elements per block the autotuner may choose for the hexahedron and wedge
// block kernels: the batch sizes whose LDS fits a compute unit and, for
// hexahedra, whose per-thread arrays fit the registers (at most 1000 nodes a
// batch: larger ones spill).
constexpr int kHexEpb[] = {2, 4, 8, 16}, kWedgeEpb[] = {1, 2, 4, 8};
template <class S>
constexpr bool fits() {
  return sizeof(typename S::Smem) <= 160 * 1024;
}
template <int N, int E>
constexpr bool hex_fits() {
  return fits<HexStage<N, E>>() && E * HexStage<N, E>::Np <= 1000;
}
template <class S>
static int go_fit(const StageArgs& a, hipStream_t s, bool mrab) {
  if constexpr (fits<S>()) return go<S>(a, s, mrab);
  else return -1;
}
template <int N, int I>
static int hex_epb(const StageArgs& a, hipStream_t s, bool mrab, int eb) {
  if constexpr (I < 4) {
    if constexpr (hex_fits<N, kHexEpb[I]>()) {
      if (eb == kHexEpb[I]) return go<HexStage<N, kHexEpb[I]>>(a, s, mrab);
    }
    return hex_epb<N, I + 1>(a, s, mrab, eb);
  } else {
    return -1;
  }
}
template <int N, int I>
static int wedge_epb(const StageArgs& a, hipStream_t s, bool mrab, int eb) {
  if constexpr (I < 4) {
    if (eb == kWedgeEpb[I]) return go_fit<WedgeStage<N, kWedgeEpb[I]>>(a, s, mrab);
    return wedge_epb<N, I + 1>(a, s, mrab, eb);
  } else {
    return -1;
  }
}
template <int N>
static int epb_options_n(int type, int* out) {
  int n = 0;
  if (type == 0) {
    if (hex_fits<N, 2>()) out[n++] = 2;
    if (hex_fits<N, 4>()) out[n++] = 4;
    if (hex_fits<N, 8>()) out[n++] = 8;
    if (hex_fits<N, 16>()) out[n++] = 16;
  } else if (type == 1) {
    if (fits<WedgeStage<N, 1>>()) out[n++] = 1;
    if (fits<WedgeStage<N, 2>>()) out[n++] = 2;
    if (fits<WedgeStage<N, 4>>()) out[n++] = 4;
    if (fits<WedgeStage<N, 8>>()) out[n++] = 8;
  }
  return n;
}

// eb: elements per block of the hexahedron or wedge block kernel (0: the
// default of stage_config.hpp).
template <int N>
static int launch_n(int type, const StageArgs& a, hipStream_t s, bool mrab, int eb) {
  switch (type) {
    case 0:
      if (eb > 0) return hex_epb<N, 0>(a, s, mrab, eb);
      return go<HexStage<N, epb(0, N)>>(a, s, mrab);
    case 1:
      // the multi-rate update runs faster wavefront-batched, the stage and
      // right-hand side in blocks of EPB elements (measured at N = 4)
      if constexpr (N == 4) {
        if (mrab) return go_wave<WedgeStage<N, 1, 64>, wedge_waves(N)>(a, s, mrab);
      }
      if (eb > 0) return wedge_epb<N, 0>(a, s, mrab, eb);
      return go<WedgeStage<N, epb(1, N)>>(a, s, mrab);
    case 2:
      if constexpr (N <= 4) return go_wave<PyrStage<N, 1, 64>, pyr_waves(N)>(a, s, mrab);
      else return go<PyrStage<N, epb(2, N)>>(a, s, mrab);
    case 3: return go<TetStage<N, epb(3, N)>>(a, s, mrab);
  }
  return -1;
}

template <int N>
static void sizes_n(int type, int* nf, int* ni) {
  switch (type) {
    case 0: sizes<HexStage<N, epb(0, N)>>(nf, ni); break;
    case 1: sizes<WedgeStage<N, epb(1, N)>>(nf, ni); break;
    case 2: sizes<PyrStage<N, epb(2, N)>>(nf, ni); break;
    default: sizes<TetStage<N, epb(3, N)>>(nf, ni); break;
  }
}

static int launch_any(int type, int N, const StageArgs& a, hipStream_t s, bool mrab, int eb) {
  switch (N) {
    case 1: return launch_n<1>(type, a, s, mrab, eb);
    case 2: return launch_n<2>(type, a, s, mrab, eb);
    case 3: return launch_n<3>(type, a, s, mrab, eb);
    case 4: return launch_n<4>(type, a, s, mrab, eb);
    case 5: return launch_n<5>(type, a, s, mrab, eb);
  }
  return -1;
}

int launch_stage(int type, int N, const StageArgs& a, hipStream_t s, int eb) {
  return launch_any(type, N, a, s, false, eb);
}

int launch_mrab_update(int type, int N, const StageArgs& a, hipStream_t s, int eb) {
  return launch_any(type, N, a, s, true, eb);
}

int stage_epb_options(int type, int N, int* out) {
  switch (N) {
    case 1: return epb_options_n<1>(type, out);
    case 2: return epb_options_n<2>(type, out);
    case 3: return epb_options_n<3>(type, out);
    case 4: return epb_options_n<4>(type, out);
    case 5: return epb_options_n<5>(type, out);
  }
  return 0;
}

void stage_table_sizes(int type, int N, int* nf, int* ni) {
  switch (N) {
    case 1: sizes_n<1>(type, nf, ni); break;
    case 2: sizes_n<2>(type, nf, ni); break;
    case 3: sizes_n<3>(type, nf, ni); break;
    case 4: sizes_n<4>(type, nf, ni); break;
    default: sizes_n<5>(type, nf, ni); break;
  }
}

int stage_batch(int type, int N) { return epb(type, N); }

}  // namespace hdg
