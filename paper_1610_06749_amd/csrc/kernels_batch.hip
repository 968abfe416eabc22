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
//
// Pulse trains (a period of at least T steps, so at most one pulse in a
// pass): a pass computes steps c0 .. c0 + T - 1, and the pass in which a
// pulse falls due adds it to the outputs of the level that computes the
// step before it (pulse_add = j for a pulse at step c0 + j, j = 1..T; one
// at c0 + T is thus added by the pass before the one it precedes).  The
// recording block of a pass, which records the previous pass's steps
// r0 .. r0 + T - 1, books the release of a pulse deposited before one of
// them with that step (the first pulse's release, from the deposit, is
// kept when step 0 is recorded), then sets the flag of the next pass, which
// computes steps r0 + 2T .. r0 + 3T - 1.  The flags alternate by pass
// parity, so the tile blocks of a pass read a flag the previous pass wrote.
template <int NT>
__device__ void record_previous(const BatchInstance& bi, int parity, int T) {
  const StepParams& p = bi.sp[parity ^ 1];
  if (p.state->done) return;
  // the previous pass's tile count, which its own recording block stored
  // (the host may have re-tiled the running instances since)
  __shared__ int nprev;
  if (threadIdx.x == 0 && threadIdx.y == 0) nprev = p.state->rec_ntiles;
  __syncthreads();
  __shared__ double totals[kAcc * kMaxT];
  reduce_partials<NT>(p.partials, nprev, kAcc * T, kAcc * T, totals);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    RunState* st = p.state;
    const int64_t step = st->steps;
    const int Te = (int)min((int64_t)T, bi.max_steps - step);
    const bool train = bi.npulses >= 2;
    int inject = -1;
    if (train) {
      if (step == 0) {
        st->pulse_q[0] = st->released;
        st->pulse_q[1] = st->released_neg;
      }
      const int k = st->pulses_counted;
      const int64_t s_k = (int64_t)k * bi.period_steps;
      if (k < bi.npulses && s_k >= step && s_k < step + Te) {
        inject = (int)(s_k - step);
        st->pulses_counted = k + 1;
      }
    }
    finalize_steps(st, p.trace, totals, Te, step, p.cp, p.cn, p.dV, p.stop_tol, p.min_stop_step, inject,
                   train ? st->pulse_q[0] : 0.0, train ? st->pulse_q[1] : 0.0);
    if (!st->done && st->steps >= bi.max_steps) {
      st->done = 1;
      st->by_limit = 1;
    }
    st->rec_ntiles = bi.ntiles;  // this pass's tiles, for the next recording block
    if (train) {
      // the next pass computes steps c1 .. c1 + T - 1; a pulse at or past
      // the run's last step is never deposited
      const int64_t c1 = step + 2 * T;
      const int kf = st->pulses_flagged;
      const int64_t s_due = (int64_t)kf * bi.period_steps;
      const bool due = kf < bi.npulses && s_due > c1 && s_due <= c1 + T && s_due < bi.max_steps;
      st->pulse_add[parity ^ 1] = due ? (int)(s_due - c1) : 0;
      if (due) st->pulses_flagged = kf + 1;
    }
  }
}

// PU: some instance of the batch has a pulse train (its tile blocks add
// the pulse when their instance's flag for this pass is set).
template <int SY, bool SC, bool AB, int TX, bool PU>
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
  if (PU) {
    const BatchInstance& bi = inst[q];
    // written by the previous pass's recording block; one value for the block
    const int add = bi.npulses >= 2 ? __builtin_amdgcn_readfirstlane(p.state->pulse_add[parity]) : 0;
    plain_tile_step<SY, SC, AB, TX, true>(p, t, p.partials + (size_t)l * kAcc, add ? bi.pulse_pos : nullptr,
                                          add ? bi.pulse_neg : nullptr);
  } else {
    plain_tile_step<SY, SC, AB, TX>(p, t, p.partials + (size_t)l * kAcc);
  }
}

// T steps per launch: the temporally blocked tile pass of stencil_blocked.h
// on each running instance's tiles (64 x 8R extended tiles, chunks of
// planes), one recording block per instance as above.  PU: some instance
// has a pulse train (its tile blocks add the pulse to the level its flag
// for this pass names); AB: some instance has absorbing lateral boundaries.
template <int T, int R, bool SC, bool PU, bool AB>
__global__ __launch_bounds__(kBNT) __attribute__((amdgpu_waves_per_eu(2, 2)))
void batch_blocked_kernel(const BatchInstance* __restrict__ inst, int ninst, int total_tiles, int per_xcd,
                          int parity) {
  const int b = blockIdx.x;
  if (b >= 8 * per_xcd) {
    record_previous<kBNT>(inst[b - 8 * per_xcd], parity, T);
    return;
  }
  const int L = blocked_tile_index(b, per_xcd);  // XCD-aware order over the whole list
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
  if (PU) {
    const BatchInstance& bi = inst[q];
    // written by the previous pass's recording block; one value for the block
    const int j = bi.npulses >= 2 ? __builtin_amdgcn_readfirstlane(p.state->pulse_add[parity]) : 0;
    blocked_tile_pass<T, R, SC, true, AB>(p, t, p.partials + (size_t)l * kAcc * T, j, bi.pulse_pos, bi.pulse_neg);
  } else {
    blocked_tile_pass<T, R, SC, false, AB>(p, t, p.partials + (size_t)l * kAcc * T);
  }
}

}  // namespace

namespace {

// The kernel instance of a one-step pass.
template <int SY, int TX, bool PU>
const void* batch_kernel_pu(bool sc, bool ab) {
  switch ((sc ? 2 : 0) + (ab ? 1 : 0)) {
    case 0: return reinterpret_cast<const void*>(&batch_step_kernel<SY, false, false, TX, PU>);
    case 1: return reinterpret_cast<const void*>(&batch_step_kernel<SY, false, true, TX, PU>);
    case 2: return reinterpret_cast<const void*>(&batch_step_kernel<SY, true, false, TX, PU>);
    default: return reinterpret_cast<const void*>(&batch_step_kernel<SY, true, true, TX, PU>);
  }
}

template <int SY, int TX>
const void* batch_kernel_terms(bool sc, bool ab, bool pu) {
  return pu ? batch_kernel_pu<SY, TX, true>(sc, ab) : batch_kernel_pu<SY, TX, false>(sc, ab);
}

template <int T, int R, bool AB>
const void* batch_blocked_terms(bool sc, bool pu) {
  switch ((sc ? 2 : 0) + (pu ? 1 : 0)) {
    case 0: return reinterpret_cast<const void*>(&batch_blocked_kernel<T, R, false, false, AB>);
    case 1: return reinterpret_cast<const void*>(&batch_blocked_kernel<T, R, false, true, AB>);
    case 2: return reinterpret_cast<const void*>(&batch_blocked_kernel<T, R, true, false, AB>);
    default: return reinterpret_cast<const void*>(&batch_blocked_kernel<T, R, true, true, AB>);
  }
}

template <int T, int R>
const void* batch_blocked_ptr(bool sc, bool pu, bool ab) {
  return ab ? batch_blocked_terms<T, R, true>(sc, pu) : batch_blocked_terms<T, R, false>(sc, pu);
}

// The blocked batch kernel for T steps and R rows per thread (null if not
// offered): the depths and row counts the single-chamber kernel offers.
const void* batch_blocked(int T, int R, bool sc, bool pu, bool ab) {
  switch (T * 16 + R) {
    case 2 * 16 + 3: return batch_blocked_ptr<2, 3>(sc, pu, ab);
    case 2 * 16 + 4: return batch_blocked_ptr<2, 4>(sc, pu, ab);
    case 2 * 16 + 5: return batch_blocked_ptr<2, 5>(sc, pu, ab);
    case 2 * 16 + 6: return batch_blocked_ptr<2, 6>(sc, pu, ab);
    case 3 * 16 + 3: return batch_blocked_ptr<3, 3>(sc, pu, ab);
    case 3 * 16 + 4: return batch_blocked_ptr<3, 4>(sc, pu, ab);
    case 3 * 16 + 5: return batch_blocked_ptr<3, 5>(sc, pu, ab);
    case 3 * 16 + 6: return batch_blocked_ptr<3, 6>(sc, pu, ab);
    case 4 * 16 + 3: return batch_blocked_ptr<4, 3>(sc, pu, ab);
    case 4 * 16 + 4: return batch_blocked_ptr<4, 4>(sc, pu, ab);
    case 4 * 16 + 5: return batch_blocked_ptr<4, 5>(sc, pu, ab);
    case 4 * 16 + 6: return batch_blocked_ptr<4, 6>(sc, pu, ab);
    default: return nullptr;
  }
}

// The one-step kernel of a pass and its waves per block.
const void* batch_kernel(int tile_y, int tile_x, bool sc, bool ab, bool pu, int* sy) {
  if (plain_tile_cols(tile_x) == 32) {
    *sy = 8;
    return batch_kernel_terms<8, 32>(sc, ab, pu);
  }
  if (plain_tile_rows(tile_y, tile_x) == 16) {
    *sy = 16;
    return batch_kernel_terms<16, 64>(sc, ab, pu);
  }
  *sy = 8;
  return batch_kernel_terms<8, 64>(sc, ab, pu);
}

}  // namespace

hipError_t add_batch_pass_node(hipGraph_t graph, hipGraphNode_t dep, hipGraphNode_t* node, const void* table,
                               int ninst, int total_tiles, int tile_y, int tile_x, bool sc, bool ab, bool pu,
                               int parity, int T, int R) {
  const BatchInstance* inst = (const BatchInstance*)table;
  int per_xcd = (total_tiles + 7) / 8;
  int sy = 8;
  const void* fn = T > 1 ? batch_blocked(T, R, sc, pu, ab) : batch_kernel(tile_y, tile_x, sc, ab, pu, &sy);
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
                             bool ab, bool pu, int parity, bool record_prev, int T, int R, hipStream_t s) {
  const BatchInstance* inst = (const BatchInstance*)table;
  int per_xcd = (total_tiles + 7) / 8;
  const int nr = record_prev ? ninst : 0;
  int sy = 8;
  const void* fn = T > 1 ? batch_blocked(T, R, sc, pu, ab) : batch_kernel(tile_y, tile_x, sc, ab, pu, &sy);
  if (!fn) return hipErrorInvalidValue;
  if (T > 1) sy = kBW;
  void* args[] = {(void*)&inst, (void*)&ninst, (void*)&total_tiles, (void*)&per_xcd, (void*)&parity};
  return hipLaunchKernel(fn, dim3(8 * per_xcd + nr), dim3(kTX, sy), args, 0, s);
}

}  // namespace it
