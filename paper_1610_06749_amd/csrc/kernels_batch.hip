// Batched stepping: one launch advances every still-running chamber of a
// sweep by one time step.  The tiles of all instances form one list (each
// instance keeps its own grid, tiling, coefficients, fields and run state in
// a device table); a block finds its instance by binary search, skips it
// once the instance has stopped, and otherwise runs the same tile step as
// the single-chamber kernel.  The same launch has one more block per
// instance: it reduces that instance's partial tallies of the previous pass
// (the partials alternate between two buffers) and records its step and stop
// decision while the tile blocks compute the next step.  Blocks that read the
// stop flag while it is being set only decide whether to compute one step
// past the stop, which no result reads.  Kernel boundaries order the passes;
// the host captures a chain of passes in a HIP graph and replays it until
// every instance has stopped.
#include "stencil_blocked.h"

namespace it {

namespace {

__device__ inline int find_instance(const BatchInstance* inst, int ninst, int L) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {  // last instance with tile_begin <= L
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].tile_begin <= L) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Records the previous pass's T steps of instance q (its partials are in
// the buffer of the other parity), up to the instance's step limit: a pass
// may run past it, and those steps are not recorded.
template <int NT>
__device__ void record_previous(const BatchInstance& bi, int parity, int T) {
  const StepParams& p = bi.sp[parity ^ 1];
  if (p.state->done) return;
  __shared__ double totals[kAcc * kMaxT];
  reduce_partials<NT>(p.partials, bi.ntiles, kAcc * T, kAcc * T, totals);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    const int64_t step = p.state->steps;
    const int Te = (int)min((int64_t)T, bi.max_steps - step);
    finalize_steps(p.state, p.trace, totals, Te, step, p.cp, p.cn, p.dV, p.stop_tol, p.min_stop_step);
    if (!p.state->done && p.state->steps >= bi.max_steps) {
      p.state->done = 1;
      p.state->by_limit = 1;
    }
  }
}

template <int SY, bool SC, bool AB, int TX>
__global__ __launch_bounds__(kTX * SY) __attribute__((amdgpu_waves_per_eu(4, 8)))
void batch_step_kernel(const BatchInstance* __restrict__ inst, int ninst, int total_tiles, int per_xcd,
                       int parity) {
  const int b = blockIdx.x;
  if (b >= 8 * per_xcd) {  // the recording blocks, one per instance
    record_previous<kTX * SY>(inst[b - 8 * per_xcd], parity, 1);
    return;
  }
  const int L = (b & 7) * per_xcd + (b >> 3);  // XCD-aware order over the whole list
  if (L >= total_tiles) return;
  const int q = find_instance(inst, ninst, L);
  const StepParams& p = inst[q].sp[parity];
  if (p.state->done) return;
  const int l = L - inst[q].tile_begin;
  TileCoord t = tile_of(l, p.tiles_x, p.tiles_y);
  t.valid = true;
  plain_tile_step<SY, SC, AB, TX>(p, t, p.partials + (size_t)l * kAcc);
}

// T steps per launch: the temporally blocked tile pass of stencil_blocked.h
// on each running instance's tiles (64 x 8R extended tiles, chunks of
// planes), one recording block per instance as above.
template <int T, int R, bool SC>
__global__ __launch_bounds__(kBNT) __attribute__((amdgpu_waves_per_eu(2, 2)))
void batch_blocked_kernel(const BatchInstance* __restrict__ inst, int ninst, int total_tiles, int per_xcd,
                          int parity) {
  const int b = blockIdx.x;
  if (b >= 8 * per_xcd) {
    record_previous<kBNT>(inst[b - 8 * per_xcd], parity, T);
    return;
  }
  const int L = (b & 7) * per_xcd + (b >> 3);  // XCD-aware order over the whole list
  if (L >= total_tiles) return;
  const int q = find_instance(inst, ninst, L);
  const StepParams& p = inst[q].sp[parity];
  // the recording block of this launch may set the flag: one read for the block
  __shared__ int stopped;
  if (threadIdx.x == 0 && threadIdx.y == 0) stopped = p.state->done;
  __syncthreads();
  if (stopped) return;
  const int l = L - inst[q].tile_begin;
  TileCoord t = tile_of(l, p.tiles_x, p.tiles_y);
  t.valid = true;
  blocked_tile_pass<T, R, SC>(p, t, p.partials + (size_t)l * kAcc * T);
}

}  // namespace

namespace {

template <int SY, bool SC, bool AB, int TX>
void launch_batch_instance(const BatchInstance* inst, int nrecord, int ninst, int total_tiles, int per_xcd,
                           int parity, hipStream_t s) {
  hipLaunchKernelGGL((batch_step_kernel<SY, SC, AB, TX>), dim3(8 * per_xcd + nrecord), dim3(kTX, SY), 0, s, inst,
                     ninst, total_tiles, per_xcd, parity);
}

template <int SY, int TX>
void launch_batch_terms(const BatchInstance* inst, int nrecord, int ninst, int total_tiles, int per_xcd,
                        int parity, bool sc, bool ab, hipStream_t s) {
  switch ((sc ? 2 : 0) + (ab ? 1 : 0)) {
    case 0: launch_batch_instance<SY, false, false, TX>(inst, nrecord, ninst, total_tiles, per_xcd, parity, s); break;
    case 1: launch_batch_instance<SY, false, true, TX>(inst, nrecord, ninst, total_tiles, per_xcd, parity, s); break;
    case 2: launch_batch_instance<SY, true, false, TX>(inst, nrecord, ninst, total_tiles, per_xcd, parity, s); break;
    default: launch_batch_instance<SY, true, true, TX>(inst, nrecord, ninst, total_tiles, per_xcd, parity, s); break;
  }
}

}  // namespace

namespace {

// The kernel instance of a pass and its block shape.
template <int SY, int TX>
const void* batch_kernel_terms(bool sc, bool ab) {
  switch ((sc ? 2 : 0) + (ab ? 1 : 0)) {
    case 0: return reinterpret_cast<const void*>(&batch_step_kernel<SY, false, false, TX>);
    case 1: return reinterpret_cast<const void*>(&batch_step_kernel<SY, false, true, TX>);
    case 2: return reinterpret_cast<const void*>(&batch_step_kernel<SY, true, false, TX>);
    default: return reinterpret_cast<const void*>(&batch_step_kernel<SY, true, true, TX>);
  }
}

template <int T, int R>
const void* batch_blocked_ptr(bool sc) {
  return sc ? reinterpret_cast<const void*>(&batch_blocked_kernel<T, R, true>)
            : reinterpret_cast<const void*>(&batch_blocked_kernel<T, R, false>);
}

// The blocked batch kernel for T steps and R rows per thread (null if not
// offered): the depths and row counts the single-chamber kernel offers.
const void* batch_blocked(int T, int R, bool sc) {
  switch (T * 16 + R) {
    case 2 * 16 + 3: return batch_blocked_ptr<2, 3>(sc);
    case 2 * 16 + 4: return batch_blocked_ptr<2, 4>(sc);
    case 2 * 16 + 5: return batch_blocked_ptr<2, 5>(sc);
    case 2 * 16 + 6: return batch_blocked_ptr<2, 6>(sc);
    case 3 * 16 + 3: return batch_blocked_ptr<3, 3>(sc);
    case 3 * 16 + 4: return batch_blocked_ptr<3, 4>(sc);
    case 3 * 16 + 5: return batch_blocked_ptr<3, 5>(sc);
    case 3 * 16 + 6: return batch_blocked_ptr<3, 6>(sc);
    case 4 * 16 + 3: return batch_blocked_ptr<4, 3>(sc);
    case 4 * 16 + 4: return batch_blocked_ptr<4, 4>(sc);
    case 4 * 16 + 5: return batch_blocked_ptr<4, 5>(sc);
    case 4 * 16 + 6: return batch_blocked_ptr<4, 6>(sc);
    default: return nullptr;
  }
}

const void* batch_kernel(int tile_y, int tile_x, bool sc, bool ab, int* sy) {
  if (plain_tile_cols(tile_x) == 32) {
    *sy = 8;
    return batch_kernel_terms<8, 32>(sc, ab);
  }
  if (plain_tile_rows(tile_y, tile_x) == 16) {
    *sy = 16;
    return batch_kernel_terms<16, 64>(sc, ab);
  }
  *sy = 8;
  return batch_kernel_terms<8, 64>(sc, ab);
}

}  // namespace

hipError_t add_batch_pass_node(hipGraph_t graph, hipGraphNode_t dep, hipGraphNode_t* node, const void* table,
                               int ninst, int total_tiles, int tile_y, int tile_x, bool sc, bool ab, int parity,
                               int T, int R) {
  const BatchInstance* inst = (const BatchInstance*)table;
  int per_xcd = (total_tiles + 7) / 8;
  int sy = 8;
  const void* fn = T > 1 ? batch_blocked(T, R, sc) : batch_kernel(tile_y, tile_x, sc, ab, &sy);
  if (!fn) return hipErrorInvalidValue;
  if (T > 1) sy = kBW;  // blocks of 8 waves
  // the node copies the argument values when it is added
  void* args[] = {(void*)&inst, (void*)&ninst, (void*)&total_tiles, (void*)&per_xcd, (void*)&parity};
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(fn);
  kp.gridDim = dim3(8 * per_xcd + ninst);  // tile blocks, then one recording block per instance
  kp.blockDim = dim3(kTX, sy);
  kp.sharedMemBytes = 0;
  kp.kernelParams = args;
  kp.extra = nullptr;
  return hipGraphAddKernelNode(node, graph, dep ? &dep : nullptr, dep ? 1 : 0, &kp);
}

hipError_t launch_batch_pass(const void* table, int ninst, int total_tiles, int tile_y, int tile_x, bool sc,
                             bool ab, int parity, bool record_prev, int T, int R, hipStream_t s) {
  const BatchInstance* inst = (const BatchInstance*)table;
  const int per_xcd = (total_tiles + 7) / 8;
  const int nr = record_prev ? ninst : 0;
  if (T > 1) {
    const void* fn = batch_blocked(T, R, sc);
    if (!fn || ab) return hipErrorInvalidValue;  // the blocked pass is periodic only
    void* args[] = {(void*)&inst, (void*)&ninst, (void*)&total_tiles, (void*)const_cast<int*>(&per_xcd),
                    (void*)&parity};
    return hipLaunchKernel(fn, dim3(8 * per_xcd + nr), dim3(kWave, kBW), args, 0, s);
  }
  if (plain_tile_cols(tile_x) == 32)
    launch_batch_terms<8, 32>(inst, nr, ninst, total_tiles, per_xcd, parity, sc, ab, s);
  else if (plain_tile_rows(tile_y, tile_x) == 16)
    launch_batch_terms<16, 64>(inst, nr, ninst, total_tiles, per_xcd, parity, sc, ab, s);
  else
    launch_batch_terms<8, 64>(inst, nr, ninst, total_tiles, per_xcd, parity, sc, ab, s);
  return hipGetLastError();
}

}  // namespace it
