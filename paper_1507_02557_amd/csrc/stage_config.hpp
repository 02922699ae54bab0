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
  if (type == 2) return N <= 2 ? 8 : (N <= 4 ? 16 : 2);
  return N == 1 ? 32 : (N == 2 ? 16 : (N == 3 ? 12 : (N == 4 ? 8 : 4)));
}

// Threads per block of the vector pyramid kernel: one block per compute unit
// holds the operator tables once, so the batch and the block grow together
// (16 elements: 16 wavefronts per compute unit at N = 4; 8 at N = 3, whose
// stage kernel needs more than the 128 registers a lane gets at 16).
constexpr int pyr_threads(int N) { return N == 4 ? 1024 : (N == 3 ? 512 : 256); }

}  // namespace hdg
