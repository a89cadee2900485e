// Contracting-grid kernels for the sliced LRF kind (one translation unit per
// kind so the instantiations compile in parallel; no multi-detector launch).
#include "grid_impl.h"

namespace ants {

hipError_t launch_grid_sliced(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t s,
                           int max_blocks) {
  return launch_grid_k<ANTS_LRF_SLICED>(L, G, io, s, max_blocks);
}

}  // namespace ants
