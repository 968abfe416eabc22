// Temporally blocked stepping kernel for one chamber: T explicit time steps
// per HBM pass (the tile pass itself is blocked_tile_pass in
// stencil_blocked.h), its launch shapes and its launcher.
//
// As in the one-step kernel, a launch has one block more than tiles when the
// previous pass is still unrecorded: that block sums the previous pass's
// partials in a fixed order and records its steps while the others step.
#include <algorithm>

#include "stencil_blocked.h"

namespace it {

namespace {

constexpr int kMinT = 2, kMaxBlockedT = 4;  // T = 5 would need 170 KB of LDS for its edge rows

// Records the previous pass (its partials, block count and step count come
// with the launch): the extra block of a launch.
__device__ void record_previous_pass(const StepParams& p) {
  if (p.state->done) return;
  __shared__ double totals[kAcc * kMaxT];
  reduce_partials<kBNT>(p.prev_partials, p.prev_nblocks, kAcc * p.prev_T, kAcc * p.prev_T, totals);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    finalize_steps(p.state, p.trace, totals, p.prev_T, p.prev_step, p.cp, p.cn, p.dV, p.stop_tol,
                   p.min_stop_step);
}

// SC: with the space-charge term (two more tallies per level); AB: absorbing
// lateral boundaries (the escaped tallies).
template <int T, int R, bool SC, bool AB>
__global__ __launch_bounds__(kBNT) __attribute__((amdgpu_waves_per_eu(2, 2))) void step_blocked_kernel(StepParams p) {
  if (p.prev_partials && blockIdx.x == gridDim.x - 1) {
    record_previous_pass(p);
    return;
  }
  // The extra block of this launch may set the stop flag while the others
  // start: one thread reads it for the whole block, so that every wave takes
  // the same branch (the waves meet at barriers below).
  __shared__ int stopped;
  if (threadIdx.x == 0 && threadIdx.y == 0) stopped = p.state->done;
  __syncthreads();
  if (stopped) return;
  const int L = blocked_tile_index(blockIdx.x, p.per_xcd);
  TileCoord tc = tile_of(L < p.ntiles ? L : 0, p.tiles_x, p.tiles_y);
  tc.valid = L < p.ntiles;
  blocked_tile_pass<T, R, SC, false, AB>(p, tc, p.partials + (size_t)blockIdx.x * kAcc * T);
}

// Rows per thread for T fused steps when the caller does not choose: the
// largest that keeps two waves per SIMD (the registers of two planes per
// level per row, the level's tallies and the loads in flight).
int default_rows(int T) { return T == 2 ? 6 : T == 3 ? 4 : 3; }

constexpr int kMinR = 3, kMaxR = 6;

// Planes per chunk: the fewest chunks (each recomputes T planes of halo at
// both ends) whose blocks still fill the machine in as few rounds of one
// block per CU as possible.
int zchunk_for(long cols, int nint, int T) {
  constexpr long kCUs = 256;
  int best_zc = nint;
  double best = 1e30;
  for (int ch = 1; ch <= nint; ++ch) {
    const int zc = (nint + ch - 1) / ch;
    if (ch > 1 && zc < 4 * T) break;
    const long blocks = cols * ((nint + zc - 1) / zc);
    const double rounds = (double)((blocks + kCUs - 1) / kCUs);
    const double cost = rounds * (zc + 2.0 * T);
    if (cost < best - 1e-9) {
      best = cost;
      best_zc = zc;
    }
  }
  return best_zc;
}

template <int T, int R>
void launch_rows(const StepParams& p, dim3 g, hipStream_t s) {
  const dim3 block(kWave, kBW);
  const bool sc = p.gsp != 0.0 || p.gsn != 0.0;
  switch ((sc ? 2 : 0) + (p.absorbing ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((step_blocked_kernel<T, R, false, false>), g, block, 0, s, p); break;
    case 1: hipLaunchKernelGGL((step_blocked_kernel<T, R, false, true>), g, block, 0, s, p); break;
    case 2: hipLaunchKernelGGL((step_blocked_kernel<T, R, true, false>), g, block, 0, s, p); break;
    default: hipLaunchKernelGGL((step_blocked_kernel<T, R, true, true>), g, block, 0, s, p); break;
  }
}

}  // namespace

// Rows per thread of a run's passes: tile_y / 8 (tile_y = rows of the
// extended tile, a multiple of 8), or the default for its T.  Passes cut
// short by a deposit keep the run's rows.
int blocked_rows(int T, int tile_y) { return tile_y > 0 ? tile_y / kBW : default_rows(T); }

int blocked_supported(int T, int tile_y) {
  if (T < kMinT || T > kMaxBlockedT) return 0;
  if (tile_y < 0 || tile_y % kBW) return 0;
  const int R = blocked_rows(T, tile_y);
  return R >= kMinR && R <= kMaxR ? 1 : 0;
}

void blocked_tiling(int nx, int ny, int nz, int T, int R, int* grid, int* per_xcd, int* tiles_x,
                    int* tiles_y, int* ntiles, int* zc_out, int* zchunks_out) {
  const int OX = kBX - 2 * T, OY = kBW * R - 2 * T;
  *tiles_x = (nx + OX - 1) / OX;
  *tiles_y = (ny + OY - 1) / OY;
  const long cols = (long)*tiles_x * *tiles_y;
  const int nint = nz - 1;
  const int zc = zchunk_for(cols, nint, T);
  const int zchunks = (nint + zc - 1) / zc;
  *ntiles = (int)(cols * zchunks);
  *per_xcd = (*ntiles + 7) / 8;
  *grid = 8 * *per_xcd;
  if (zc_out) *zc_out = zc;
  if (zchunks_out) *zchunks_out = zchunks;
}

// Tiling of a chamber of a batch: chunks of zc planes as given.
void blocked_tiling_zc(int nx, int ny, int nz, int T, int R, int zc, int* tiles_x, int* tiles_y, int* ntiles,
                       int* zc_out, int* zchunks_out) {
  const int OX = kBX - 2 * T, OY = kBW * R - 2 * T;
  *tiles_x = (nx + OX - 1) / OX;
  *tiles_y = (ny + OY - 1) / OY;
  const int nint = nz - 1;
  const int z = std::max(1, std::min(zc, nint));
  const int zchunks = (nint + z - 1) / z;
  *ntiles = *tiles_x * *tiles_y * zchunks;
  *zc_out = z;
  *zchunks_out = zchunks;
}

hipError_t launch_step_blocked(const StepParams& p0, int T, int R, hipStream_t s, hipEvent_t ev_begin,
                               hipEvent_t ev_end, int* nblocks) {
  StepParams p = p0;
  int grid, per, tx, ty, nt, zc, zch;
  blocked_tiling(p.nx, p.ny, p.nz, T, R, &grid, &per, &tx, &ty, &nt, &zc, &zch);
  p.tiles_x = tx;
  p.tiles_y = ty;
  p.zchunks = zch;
  p.zc = zc;
  p.ntiles = nt;
  p.per_xcd = per;
  *nblocks = grid;
  if (T < kMinT || T > kMaxBlockedT || R < kMinR || R > kMaxR) return hipErrorInvalidValue;
  if (ev_begin && hipEventRecord(ev_begin, s) != hipSuccess) return hipErrorInvalidValue;
  const dim3 g(grid + (p.prev_partials ? 1 : 0));
  switch (T * 16 + R) {
    case 2 * 16 + 3: launch_rows<2, 3>(p, g, s); break;
    case 2 * 16 + 4: launch_rows<2, 4>(p, g, s); break;
    case 2 * 16 + 5: launch_rows<2, 5>(p, g, s); break;
    case 2 * 16 + 6: launch_rows<2, 6>(p, g, s); break;
    case 3 * 16 + 3: launch_rows<3, 3>(p, g, s); break;
    case 3 * 16 + 4: launch_rows<3, 4>(p, g, s); break;
    case 3 * 16 + 5: launch_rows<3, 5>(p, g, s); break;
    case 3 * 16 + 6: launch_rows<3, 6>(p, g, s); break;
    case 4 * 16 + 3: launch_rows<4, 3>(p, g, s); break;
    case 4 * 16 + 4: launch_rows<4, 4>(p, g, s); break;
    case 4 * 16 + 5: launch_rows<4, 5>(p, g, s); break;
    case 4 * 16 + 6: launch_rows<4, 6>(p, g, s); break;
    default: return hipErrorInvalidValue;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_end && hipEventRecord(ev_end, s) != hipSuccess) return hipErrorInvalidValue;
  return hipSuccess;
}

}  // namespace it
