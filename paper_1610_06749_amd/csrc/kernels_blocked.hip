// Temporally blocked stepping kernel (several steps per HBM pass).
#include "reduce.h"

namespace it {

int blocked_supported(int T, int tile_y) {
  (void)T;
  (void)tile_y;
  return 0;
}

void blocked_tiling(int nx, int ny, int nz, int T, int tile_y, int* grid, int* per_xcd, int* tiles_x,
                    int* tiles_y, int* ntiles) {
  (void)nx; (void)ny; (void)nz; (void)T; (void)tile_y;
  *grid = *per_xcd = *tiles_x = *tiles_y = *ntiles = 0;
}

hipError_t launch_step_blocked(const StepParams& p, int T, int tile_y, hipStream_t s) {
  (void)p; (void)T; (void)tile_y; (void)s;
  return hipErrorNotSupported;
}

}  // namespace it
