// Contracting-grid and multi-detector kernels for the axial LRF kind
// (one translation unit per kind so the instantiations compile in parallel).
#include "grid_impl.h"

namespace ants {

hipError_t launch_grid_axial(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t s,
                        int max_blocks) {
  return launch_grid_k<ANTS_LRF_AXIAL>(L, G, io, s, max_blocks);
}

hipError_t launch_multi_axial(const MultiP& P, int stat, int max_nn, int max_na, bool nonneg,
                         int blocks, hipStream_t s) {
  return launch_multi_k<ANTS_LRF_AXIAL>(P, stat, max_nn, max_na, nonneg, blocks, s);
}

}  // namespace ants
