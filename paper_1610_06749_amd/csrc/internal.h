// Internal declarations of the HIP recombination solver (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "iontracks.h"

namespace it {

// Per-step tally slots accumulated by the stepping kernels (per block, then
// reduced in a fixed order):
//   0 sum beta n+ n-            (recombined, before the dV factor)
//   1 sum n+ on plane k = 1      2 sum n+ on plane k = nz-1
//   3 sum n- on plane k = 1      4 sum n- on plane k = nz-1
//   5 sum n+' (new)              6 sum n-'
//   7 sum |n+'|                  8 sum |n-'|
//   9 sum of the space-charge change of n+   10 the same of n-
//  11 sum over nodes next to an absorbing lateral boundary of what the
//     missing neighbours would receive from n+ (ax or ay times n+ per
//     missing neighbour)                      12 the same of n-
constexpr int kAcc = 13;

// elementary charge [C] and vacuum permittivity [F/cm] (CODATA 2018)
constexpr double kElementaryCharge = 1.602176634e-19;
constexpr double kEpsilon0 = 8.8541878128e-14;
constexpr int kMaxT = 8;  // largest number of fused steps per pass

// Coefficients of the explicit update of one species at an interior node:
//   n' = a0 n + ax (n_{i+1} + n_{i-1}) + ay (n_{j+1} + n_{j-1})
//        + azp n_{k+1} + azm n_{k-1} - beta n+ n-
// azp is the weight of the neighbour towards the cathode (k+1); it is also
// the fraction of n_{k=1} that reaches the anode plane in one step, and azm
// the fraction of n_{k=nz-1} that reaches the cathode plane.
struct Coef {
  double a0, ax, ay, azp, azm;
};

// Device-resident run state, updated only by the last block of each launch.
struct RunState {
  double released;          // positive ions released so far
  double released_pending;  // positive ions released since the last recorded step
  double released_neg;      // the same for the negative ions (equal unless the
  double released_pending_neg;  // tracks give them their own radius)
  double sums[5];           // running recombined, pos anode/cathode, neg anode/cathode
  double last[4];           // in-flight pos/neg and |n| sums after the last step
  double max_beta_n;        // max over deposits of beta * max(n)
  double screened[2];       // running space-charge change of n+ and n-
  double escaped[2];        // running loss of n+ and n- through absorbing lateral boundaries
  // free-electron component
  double released_q;        // negative charge released (ions + electrons)
  double released_e;        // free electrons released
  double e_sums[3];         // electrons collected at anode, cathode; recombined
  double e_left;            // electrons in flight after the last electron step
  int64_t e_steps;          // electron-phase steps recorded
  int32_t e_done;           // 1 once the electrons are collected
  int32_t e_pad;
  int64_t steps;            // steps recorded so far
  int32_t done;             // 1 once the stop criterion (or a non-finite tally) is met
  int32_t flags;            // IT_FLAG_NONFINITE
  int32_t passes;           // stepping launches that ran (not skipped)
  int32_t by_limit;         // 1 if a batched run stopped the instance at max_steps
  // pulse train: the last period begins at step period_step (INT64_MAX:
  // no train); when its step is recorded, the running sums and the ions its
  // pulse released are kept
  int64_t period_step;
  double period_sums[5];
  double period_rel[2];
  int32_t period_started;
  // batched pulse trains: a pass of parity p adds the pulse to its outputs
  // when pulse_add[p] is set (a pulse is due at the next step); the release
  // of each later pulse (pulse_q, the first pulse's) is recorded with its step
  int32_t pulse_add[2];
  int32_t pulses_counted;   // pulses whose release is recorded
  int32_t pulses_flagged;   // pulses whose pulse_add flag has been set
  // batches: the tiles whose partials the next recording block reduces (the
  // previous pass's tiling, which a rebuilt table may have changed since)
  int32_t rec_ntiles;
  double pulse_q[2];
};

// A run state before any deposit (no pulse train).
inline RunState initial_run_state() {
  RunState s;
  __builtin_memset(&s, 0, sizeof(s));
  s.period_step = INT64_MAX;
  return s;
}

// Track prepared on the host for the deposit kernel.
struct DepTrack {
  double x0, y0;            // axis position at mid-gap
  double ux, uy, uz;        // axis direction
  double peak;              // N0 / (pi b^2)
  double inv_b2;            // 1 / b^2
  double cut2;              // (8 b)^2
  double peak_n, inv_b2_n, cut2_n;  // the same with the negative ions' radius
};

struct StepParams {
  const double* pin;
  const double* nin;
  double* pout;
  double* nout;
  int nx, ny, nz;
  int tiles_x, tiles_y, zchunks, zc;  // tiling of the interior
  int ntiles;                         // tiles_x * tiles_y * zchunks
  int per_xcd;                        // tiles per XCD slot (grid = 8 * per_xcd)
  Coef cp, cn;
  double beta, dV, stop_tol;
  // space-charge screening, signed as it enters the update:
  //   n+' += gsp n+ (n+ - n-),  n-' += gsn n- (n+ - n-)
  // gsp = -mu+ dt q/eps0, gsn = +mu- dt q/eps0 (both 0 when off)
  double gsp, gsn;
  int absorbing;            // 1: absorbing lateral boundaries (zero beyond the cell), 0: periodic
  int64_t step0;            // index of the step this launch computes
  int64_t min_stop_step;    // the stop criterion is tested only from this step on
  double* partials;         // [gridDim][kAcc * T]
  unsigned* counter;
  RunState* state;
  double* trace;            // [max_steps][IT_TRACE_COLS]
  // when set, one extra block of the launch reduces the partials of the
  // previous launch (prev_nblocks blocks, prev_T steps) and records its steps
  // from prev_step on, overlapping the reduction with this launch's stencil
  const double* prev_partials;
  int prev_nblocks;
  int prev_T;
  int64_t prev_step;
};

struct DepositParams {
  double* pos;
  double* neg;
  int nx, ny, nz;
  int tiles_x, tiles_y, zchunks, zc, ntiles, per_xcd;
  double dx, dy, dz, half_gap, Lx, Ly;
  int absorbing;            // 1: transverse offsets as they are; 0: nearest periodic image
  double uniform;           // uniform density added at this deposit (0 if none)
  const DepTrack* par;      // tracks parallel to the field
  int npar;
  const DepTrack* tilt;     // tilted tracks
  int ntilt;
  double dV, beta;
  int same_radii;           // 1: every track gives both species the same radius
  // free electrons: the negative charge splits into negative ions
  // (1 - e^{-a z}) and electrons (fraction pfree) written to `ele`
  int free_e;
  double attach, pfree;
  double* ele;
  double* partials;         // [gridDim][5]
  unsigned* counter;
  RunState* state;
};

// One chamber of a batched sweep (device table entry).
struct BatchInstance {
  StepParams sp[2];  // [parity]: field pair 0 -> pair 1, and pair 1 -> pair 0
  int tile_begin;    // first entry of this instance in the batch's tile list
  int ntiles;
  int64_t max_steps;
  // pulse train (npulses >= 2; 0 otherwise): pulse k is due at step
  // k * period_steps; pulse_pos/pulse_neg hold the first pulse's densities
  int npulses;
  int64_t period_steps;
  const double* pulse_pos;
  const double* pulse_neg;
};

// One electron-phase step of the three carriers (free-electron component).
constexpr int kAcc3 = 14;  // per-block tally slots of the electron phase
struct Step3Params {
  const double* in[3];      // n+, n-, n_e
  double* out[3];
  int nx, ny, nz;
  int tiles_x, tiles_y, zchunks, zc, ntiles, per_xcd;
  Coef co[3];
  double beta, dV, stop_tol;
  double* partials;         // [gridDim][kAcc3]
  RunState* state;
};
hipError_t launch_step3(const Step3Params& p, hipStream_t s);

// Launch errors are read with hipGetLastError(), which also returns an error
// left by any earlier HIP call of the thread (the caller's included).  Entry
// points that launch kernels clear that state first, so a stale error is not
// reported as theirs.
inline void clear_stale_error() { (void)hipGetLastError(); }

// Launchers (stream-ordered, no synchronisation).
// Tile shape of the one-step kernels: tile_x 32 gives 32 x 16 tiles (8 waves,
// two rows each); tile_x 128 tiles of 128 columns (each lane a pair of
// columns) by tile_y = 16 or 8 rows; otherwise 64 columns by tile_y = 16 or
// 8 rows (one wave per row).
inline int plain_tile_cols(int tile_x) { return tile_x == 32 || tile_x == 128 ? tile_x : 64; }
int plain_tile_rows(int tile_y, int tile_x);
// ev_begin / ev_end (may be null) are recorded around the stepping kernel
// alone, before the tally reduction is launched.
// fused: leave this step's partials to the next launch's extra block (or a
// closing launch_reduce_steps) instead of launching the reduction now.
hipError_t launch_step_plain(const StepParams& p, int tile_y, int tile_x, hipStream_t s,
                             hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr, bool fused = false);
hipError_t launch_deposit(const DepositParams& p, hipStream_t s);
hipError_t launch_reduce_steps(const StepParams& p, int nblocks, int T, hipStream_t s);
// sc: some instance has the space-charge term on; ab: some instance has
// absorbing lateral boundaries; pu: some instance has a pulse train (one
// step per pass); record_prev: the launch also records the previous pass's
// step of every instance (false only for the first pass)
// T > 1: T steps per launch with the blocked tile pass, R rows per thread
// (tile_y and tile_x are then unused)
hipError_t launch_batch_pass(const void* table, int ninst, int total_tiles, int tile_y, int tile_x, bool sc,
                             bool ab, bool pu, int parity, bool record_prev, int T, int R, hipStream_t s);
// The same pass (recording the previous one) as a kernel node of `graph`
// that depends on `dep` (null: none).
hipError_t add_batch_pass_node(hipGraph_t graph, hipGraphNode_t dep, hipGraphNode_t* node, const void* table,
                               int ninst, int total_tiles, int tile_y, int tile_x, bool sc, bool ab, bool pu,
                               int parity, int T, int R);

}  // namespace it
