// Deterministic block reductions and the end-of-launch tally finalisation
// shared by the stepping kernels.  Every sum is taken in a fixed order
// (wave butterfly, then waves in index order, then blocks in index order),
// so a run is bitwise reproducible.
#pragma once

#include "internal.h"

namespace it {

constexpr int kWave = 64;

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global load and store of the wave, which would drain
// the prefetches the stepping loops keep in flight across their barriers.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Sums N values per thread over a block of NT threads; thread 0 writes the N
// block totals to out[0..N).  lds must hold (NT/64) * N doubles.  Slots set
// in ZERO (bit q for slot q) are known to be zero in every thread: they are
// stored as zero without the wave reduction.
template <int N, int NT, uint32_t ZERO = 0u>
__device__ inline void block_sum_store(double (&acc)[N], double* out, double* lds) {
  constexpr int W = NT / kWave;
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int wave = tid / kWave, lane = tid % kWave;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const double v = (ZERO >> q) & 1u ? 0.0 : wave_sum(acc[q]);
    if (lane == 0) lds[wave * N + q] = v;
  }
  __syncthreads();
  if (tid < N) {
    double s = lds[tid];
#pragma unroll
    for (int w = 1; w < W; ++w) s += lds[w * N + tid];
    out[tid] = s;
  }
}

// Called by all threads of every block after the block wrote its partials.
// Returns true in exactly one block: the last to arrive.  That block then
// sees every other block's partials.  (Used only by the rare deposit launch:
// the device-scope fence of every block costs an L2 write-back, so the
// stepping kernels leave their partials to the next launch, whose kernel
// boundary makes them visible.)
template <int NT>
__device__ inline bool arrive_last(unsigned* counter) {
  __shared__ int last;
  __syncthreads();
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  if (tid == 0) {
    __threadfence();
    const unsigned ticket = atomicAdd(counter, 1u);
    last = ticket == gridDim.x * gridDim.y * gridDim.z - 1;
  }
  __syncthreads();
  if (last) __threadfence();
  return last != 0;
}

// In the last block: totals[q] = sum over blocks b of partials[b * stride + q]
// for q < n.  Component q is reduced by wave q % W; its lanes take the blocks
// in a fixed stride (8 independent loads in flight each) and the wave sums
// them by a fixed butterfly, so all components finish in a few round trips.
template <int NT>
__device__ inline void reduce_partials(const double* partials, int nblocks, int stride, int n,
                                       double* totals) {
  constexpr int W = NT / kWave;
  constexpr int kBatch = 8;
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int wave = tid / kWave, lane = tid % kWave;
  for (int q = wave; q < n; q += W) {
    double s = 0.0;
    for (int b0 = lane; b0 < nblocks; b0 += kWave * kBatch) {
      double v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int b = b0 + u * kWave;
        v[u] = b < nblocks ? partials[(size_t)b * stride + q] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) s += v[u];
    }
    s = wave_sum(s);
    if (lane == 0) totals[q] = s;
  }
  __syncthreads();
}

// Thread 0 of the last block: turns the reduced sums of T consecutive steps
// (tot[s * kAcc + q]) into trace records and updates the run state and the
// stop decision (trace may be NULL: no per-step records kept).  Works on
// register copies of the fields it updates (a whole-struct copy would pass
// the untouched fields through private memory).  inject_at >= 0: a pulse of
// a batched pulse train released inj_pos and inj_neg ions before the step
// step0 + inject_at, which are booked with that step.
__device__ inline void finalize_steps(RunState* gst, double* trace, const double* tot, int T,
                                      int64_t step0, const Coef& cp, const Coef& cn, double dV,
                                      double stop_tol, int64_t min_stop_step, int inject_at = -1,
                                      double inj_pos = 0.0, double inj_neg = 0.0) {
  double released = gst->released, released_neg = gst->released_neg;
  double pending = gst->released_pending, pending_neg = gst->released_pending_neg;
  double sums[5], last[4], screened[2], escaped[2];
#pragma unroll
  for (int q = 0; q < 5; ++q) sums[q] = gst->sums[q];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    screened[q] = gst->screened[q];
    escaped[q] = gst->escaped[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) last[q] = gst->last[q];
  int64_t steps = gst->steps;
  int done = gst->done, flags = gst->flags;
  const int64_t period_step = gst->period_step;
  bool injected = false;
  for (int s = 0; s < T && !done; ++s) {
    const int64_t l = step0 + s;
    const double* a = tot + s * kAcc;
    if (s == inject_at) {
      released += inj_pos;
      released_neg += inj_neg;
      pending += inj_pos;
      pending_neg += inj_neg;
      injected = true;
    }
    double rec[IT_TRACE_COLS];
    rec[0] = a[0] * dV;
    rec[1] = cp.azp * a[1] * dV;
    rec[2] = cp.azm * a[2] * dV;
    rec[3] = cn.azp * a[3] * dV;
    rec[4] = cn.azm * a[4] * dV;
    rec[5] = a[5] * dV;
    rec[6] = a[6] * dV;
    rec[7] = a[7] * dV;
    rec[8] = a[8] * dV;
    rec[9] = pending;
    rec[10] = a[9] * dV;
    rec[11] = a[10] * dV;
    rec[12] = pending_neg;
    rec[13] = a[11] * dV;
    rec[14] = a[12] * dV;
    pending = 0.0;
    pending_neg = 0.0;
    if (l == period_step) {  // the last period of a pulse train begins with this step
#pragma unroll
      for (int q = 0; q < 5; ++q) gst->period_sums[q] = sums[q];
      gst->period_rel[0] = rec[9];
      gst->period_rel[1] = rec[12];
      gst->period_started = 1;
    }
    bool finite = true;
#pragma unroll
    for (int q = 0; q < IT_TRACE_COLS; ++q) {
      if (trace) trace[l * IT_TRACE_COLS + q] = rec[q];
      finite = finite && isfinite(rec[q]);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) sums[q] += rec[q];
#pragma unroll
    for (int q = 0; q < 4; ++q) last[q] = rec[5 + q];
    screened[0] += rec[10];
    screened[1] += rec[11];
    escaped[0] += rec[13];
    escaped[1] += rec[14];
    steps = l + 1;
    if (!finite) {
      flags |= IT_FLAG_NONFINITE;
      done = 1;
    } else if (l >= min_stop_step && rec[7] <= stop_tol * released && rec[8] <= stop_tol * released_neg) {
      done = 1;
    }
  }
  gst->released_pending = pending;
  gst->released_pending_neg = pending_neg;
  if (injected) {
    gst->released = released;
    gst->released_neg = released_neg;
    gst->released_q += inj_neg;  // negative charge: the ions (no free electrons in a train)
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) gst->sums[q] = sums[q];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    gst->screened[q] = screened[q];
    gst->escaped[q] = escaped[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) gst->last[q] = last[q];
  gst->steps = steps;
  gst->done = done;
  gst->flags = flags;
  gst->passes += 1;
}

// Tile coordinates: column tile (tx, ty) and z chunk.
struct TileCoord {
  int tx, ty, zc;
  bool valid;
};

// Tile l of a tiling with tiles_x x tiles_y columns and zchunks chunks, in
// the order (chunk, row, column): consecutive tiles are lateral neighbours
// at the same depth, so a run of them on one XCD shares the rim rows and
// columns through that XCD's L2 while they march up z together.
__device__ inline TileCoord tile_of(int l, int tiles_x, int tiles_y) {
  TileCoord t;
  t.tx = l % tiles_x;
  const int rest = l / tiles_x;
  t.ty = rest % tiles_y;
  t.zc = rest / tiles_y;
  return t;
}

// Block -> tile, XCD-aware: the dispatcher deals blocks to the 8 XCDs in
// turn, so block b runs on XCD b % 8; XCD x gets the contiguous tile run
// [x * per_xcd, (x + 1) * per_xcd).
__device__ inline TileCoord decode_tile(int tiles_x, int tiles_y, int ntiles, int per_xcd) {
  const int b = blockIdx.x;
  const int L = (b & 7) * per_xcd + (b >> 3);
  const bool valid = L < ntiles;
  TileCoord t = tile_of(valid ? L : 0, tiles_x, tiles_y);
  t.valid = valid;
  return t;
}

}  // namespace it
