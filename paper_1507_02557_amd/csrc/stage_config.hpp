// Launch configuration of the fused stage kernels.
#pragma once

namespace hdg {

// Elements per block: operator tables plus per-element LDS stay well inside
// the 160 KB of LDS of a CDNA4 compute unit, and small batches let several
// blocks share a compute unit (at N = 4 the wedge runs fastest with 2, the
// hexahedron with 4, measured on the n = 48 four-slab mesh).
constexpr int epb(int type, int N) {
  if (type == 0) return N <= 2 ? 16 : (N <= 3 ? 8 : 4);
  if (type == 1) return N <= 3 ? 8 : 2;
  if (type == 2) return 2;  // N = 5 (N <= 4: the wavefront-batched kernels)
  return N == 1 ? 32 : (N == 2 ? 16 : (N == 3 ? 12 : (N == 4 ? 8 : 4)));
}

// Wavefronts per block of the wavefront-batched pyramid kernels (N <= 4): the
// tables plus one element's data per wavefront fit the LDS, and each
// wavefront's registers fit without spilling (N = 3 needs more than 168).
constexpr int pyr_waves(int N) { return N == 4 ? 12 : (N == 3 ? 8 : 16); }

// Wavefronts per block of the wavefront-batched wedge kernel (the multi-rate
// update at N = 4): fourteen batches of one element beside the tables fill
// the LDS.
constexpr int wedge_waves(int N) { return N == 5 ? 8 : (N == 4 ? 14 : 16); }

}  // namespace hdg
