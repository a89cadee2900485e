// Dispatch of the contracting-grid launches by LRF kind (kernels in
// grid_impl.h, instantiated in grid_axial.hip, grid_xy.hip, grid_rz.hip,
// grid_composite.hip, grid_sliced.hip).
#include "ants_internal.h"

namespace ants {

hipError_t launch_grid_axial(const DevLrf&, const GridP&, const IoP&, hipStream_t, int);
hipError_t launch_grid_xy(const DevLrf&, const GridP&, const IoP&, hipStream_t, int);
hipError_t launch_grid_rz(const DevLrf&, const GridP&, const IoP&, hipStream_t, int);
hipError_t launch_grid_composite(const DevLrf&, const GridP&, const IoP&, hipStream_t, int);
hipError_t launch_grid_sliced(const DevLrf&, const GridP&, const IoP&, hipStream_t, int);
hipError_t launch_multi_axial(const MultiP&, int, int, int, bool, int, hipStream_t);
hipError_t launch_multi_xy(const MultiP&, int, int, int, bool, int, hipStream_t);
hipError_t launch_multi_rz(const MultiP&, int, int, int, bool, int, hipStream_t);

hipError_t launch_grid(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t stream,
                       int max_blocks) {
  if (L.kind == ANTS_LRF_AXIAL) return launch_grid_axial(L, G, io, stream, max_blocks);
  if (L.kind == ANTS_LRF_XY) return launch_grid_xy(L, G, io, stream, max_blocks);
  if (L.kind == ANTS_LRF_COMPOSITE) return launch_grid_composite(L, G, io, stream, max_blocks);
  if (L.kind == ANTS_LRF_SLICED) return launch_grid_sliced(L, G, io, stream, max_blocks);
  return launch_grid_rz(L, G, io, stream, max_blocks);
}

hipError_t launch_multi(const MultiP& P, int kind, int stat, int max_nn, int max_na, bool nonneg,
                        int blocks, hipStream_t s) {
  if (kind == ANTS_LRF_AXIAL) return launch_multi_axial(P, stat, max_nn, max_na, nonneg, blocks, s);
  if (kind == ANTS_LRF_XY) return launch_multi_xy(P, stat, max_nn, max_na, nonneg, blocks, s);
  return launch_multi_rz(P, stat, max_nn, max_na, nonneg, blocks, s);
}

}  // namespace ants
