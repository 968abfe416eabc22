// Plain one-step stencil kernel and the track deposition kernel (gfx950).
//
// Step kernel: one explicit time step of both ion species (eq. theEquation
// with the Appendix's difference scheme, written as per-node coefficients),
// plus the per-step tallies.  Each block (8 or 16 waves) owns a 64 x 8,
// 64 x 16 or 32 x 16 column tile (plain_tile_step), or a 128 x 8 or
// 128 x 16 tile of column pairs (pair_tile_step), and a chunk of planes and
// marches up it; with one step per launch an extra block records the
// previous step from its partials.  Every thread
// keeps n_{k-1}, n_k, n_{k+1} of its column in registers, the block stages
// plane k of the tile in LDS for the lateral neighbours, and neighbours
// outside the tile (its one-node rim, or a periodic wrap) are read from
// global memory, where they are L2 hits of the neighbouring tiles.  Results
// go out with non-temporal stores: the new densities are not read again in
// this launch, and keeping them out of L2 leaves it to the reused inputs.
// No MFMA: the update is a 7-point stencil, not a contraction, and the
// kernel is bound by HBM bandwidth (32 bytes per node and step).
#include "stencil_plain.h"

namespace it {

constexpr int kTY = 4, kNT = kTX * kTY;  // deposition tile

// With p.prev_partials set, the launch has one block more than tiles: that
// block sums the previous step's partials in a fixed order and records the
// step (finalize_steps), while the others compute this step.  The kernel
// boundary before this launch makes the previous partials visible; the
// state it writes is read by the next launch.  Stepping blocks that read
// `done` while it is being set only decide whether to compute a step past
// the stop, whose output goes to the field pair not holding the stop step.
// Tiles of column pairs aim at 8 waves per CU, so they may use more
// registers (at least 2 waves per SIMD instead of 4).
template <int SY, bool SC, bool AB, int TX>
__global__ __launch_bounds__(kTX * SY) __attribute__((amdgpu_waves_per_eu(TX == 2 * kTX ? 2 : 4, 8))) void step_plain_kernel(StepParams p) {
  if (p.prev_partials && blockIdx.x == gridDim.x - 1) {
    if (p.state->done) return;
    __shared__ double totals[kAcc * kMaxT];
    reduce_partials<kTX * SY>(p.prev_partials, p.prev_nblocks, kAcc * p.prev_T, kAcc * p.prev_T, totals);
    if (threadIdx.x == 0 && threadIdx.y == 0)
      finalize_steps(p.state, p.trace, totals, p.prev_T, p.prev_step, p.cp, p.cn, p.dV, p.stop_tol,
                     p.min_stop_step);
    return;
  }
  if (p.state->done) return;  // set by an earlier launch: every block skips
  const TileCoord t = decode_tile(p.tiles_x, p.tiles_y, p.ntiles, p.per_xcd);
  if constexpr (TX == 2 * kTX)
    pair_tile_step<SY, SC, AB>(p, t, p.partials + (size_t)blockIdx.x * kAcc);
  else
    plain_tile_step<SY, SC, AB, TX>(p, t, p.partials + (size_t)blockIdx.x * kAcc);
}

// One block: sums the per-block partial tallies of a stepping launch in a
// fixed order and turns them into T trace records (see finalize_steps).
// Running as its own launch, it sees every partial without device-wide
// fences in the stepping kernel.
__global__ __launch_bounds__(1024) void reduce_steps_kernel(StepParams p, int nblocks, int T) {
  if (p.state->done) return;
  __shared__ double totals[kAcc * kMaxT];
  reduce_partials<1024>(p.partials, nblocks, kAcc * T, kAcc * T, totals);
  if (threadIdx.x == 0)
    finalize_steps(p.state, p.trace, totals, T, p.step0, p.cp, p.cn, p.dV, p.stop_tol,
                   p.min_stop_step);
}

hipError_t launch_reduce_steps(const StepParams& p, int nblocks, int T, hipStream_t s) {
  hipLaunchKernelGGL(reduce_steps_kernel, dim3(1), dim3(1024), 0, s, p, nblocks, T);
  return hipGetLastError();
}

int plain_tile_rows(int tile_y, int tile_x) { return tile_x == 32 || tile_y == 16 ? 16 : 8; }

namespace {

template <int SY, bool SC, bool AB, int TX>
void launch_plain_instance(const StepParams& p, dim3 g, hipStream_t s) {
  hipLaunchKernelGGL((step_plain_kernel<SY, SC, AB, TX>), g, dim3(kTX, SY), 0, s, p);
}

template <int SY, int TX>
void launch_plain_terms(const StepParams& p, dim3 g, hipStream_t s) {
  const bool sc = p.gsp != 0.0 || p.gsn != 0.0;
  const bool ab = p.absorbing != 0;
  switch ((sc ? 2 : 0) + (ab ? 1 : 0)) {
    case 0: launch_plain_instance<SY, false, false, TX>(p, g, s); break;
    case 1: launch_plain_instance<SY, false, true, TX>(p, g, s); break;
    case 2: launch_plain_instance<SY, true, false, TX>(p, g, s); break;
    default: launch_plain_instance<SY, true, true, TX>(p, g, s); break;
  }
}

// the kernel instance for the tile shape, the space-charge term and the
// lateral boundary option of the run
void launch_plain_variant(const StepParams& p, int tile_y, int tile_x, dim3 g, hipStream_t s) {
  if (plain_tile_cols(tile_x) == 128) {
    if (plain_tile_rows(tile_y, tile_x) == 16) launch_plain_terms<16, 128>(p, g, s);
    else launch_plain_terms<8, 128>(p, g, s);
  } else if (plain_tile_cols(tile_x) == 32) launch_plain_terms<8, 32>(p, g, s);
  else if (plain_tile_rows(tile_y, tile_x) == 16) launch_plain_terms<16, 64>(p, g, s);
  else launch_plain_terms<8, 64>(p, g, s);
}

}  // namespace

hipError_t launch_step_plain(const StepParams& p, int tile_y, int tile_x, hipStream_t s, hipEvent_t ev_begin,
                             hipEvent_t ev_end, bool fused) {
  const int grid = 8 * p.per_xcd;
  if (ev_begin && hipEventRecord(ev_begin, s) != hipSuccess) return hipErrorInvalidValue;
  const dim3 g(grid + (p.prev_partials ? 1 : 0));
  launch_plain_variant(p, tile_y, tile_x, g, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_end && hipEventRecord(ev_end, s) != hipSuccess) return hipErrorInvalidValue;
  if (fused) return hipSuccess;  // the next launch (or a closing reduction) records this step
  return launch_reduce_steps(p, grid, 1, s);
}

// ---------------------------------------------------------------------------
// Deposition (eq. Gaussian around each track axis, eq. linear_density for N0).
// Each thread owns one transverse column of a tile and a chunk of planes.
// Tracks parallel to the field give the same density on every plane, so
// their sum is formed once per column; tilted tracks are evaluated per node.
// The perpendicular distance is |w x u| with w the node's offset from the
// axis point (x0, y0, d/2), its transverse part wrapped to the nearest
// periodic image (taken as it is with absorbing lateral boundaries); the
// profile is cut at r^2 > (8 b)^2.
// ---------------------------------------------------------------------------

__device__ inline double wrap_near(double d, double L) { return d - L * floor(d / L + 0.5); }

__device__ inline double lateral_offset(const DepositParams& p, double d, double L) {
  return p.absorbing ? d : wrap_near(d, L);
}

__device__ inline double axis_r2(const DepTrack& tr, double wx, double wy, double wz) {
  const double cx = wy * tr.uz - wz * tr.uy;
  const double cy = wz * tr.ux - wx * tr.uz;
  const double cz = wx * tr.uy - wy * tr.ux;
  return cx * cx + cy * cy + cz * cz;
}

// Densities of the positive and (with its own radius) negative ions.
__device__ inline void track_values(const DepTrack& tr, double wx, double wy, double wz, bool same,
                                    double& dp, double& dn) {
  const double r2 = axis_r2(tr, wx, wy, wz);
  dp = r2 > tr.cut2 ? 0.0 : tr.peak * exp(-r2 * tr.inv_b2);
  dn = same ? dp : (r2 > tr.cut2_n ? 0.0 : tr.peak_n * exp(-r2 * tr.inv_b2_n));
}

__global__ __launch_bounds__(kNT) void deposit_kernel(DepositParams p) {
  constexpr int NP = 5;  // partials: released n+, n- ions, electrons, negative charge; max density
  __shared__ double lds[(kNT / kWave) * NP];
  double acc[NP] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const bool same = p.same_radii != 0;
  const TileCoord t = decode_tile(p.tiles_x, p.tiles_y, p.ntiles, p.per_xcd);
  const int i = t.tx * kTX + threadIdx.x;
  const int j = t.ty * kTY + threadIdx.y;
  if (t.valid && i < p.nx && j < p.ny) {
    const int k0 = 1 + t.zc * p.zc;
    const int k1 = min(k0 + p.zc, p.nz);
    const double x = i * p.dx, y = j * p.dy;
    double g0p = p.uniform, g0n = p.uniform;
    for (int q = 0; q < p.npar; ++q) {
      const DepTrack tr = p.par[q];
      double dp, dn;
      track_values(tr, lateral_offset(p, x - tr.x0, p.Lx), lateral_offset(p, y - tr.y0, p.Ly), 0.0, same, dp,
                   dn);
      g0p += dp;
      g0n += dn;
    }
    const size_t plane = (size_t)p.nx * p.ny;
    size_t c = (size_t)k0 * plane + (size_t)j * p.nx + i;
    for (int k = k0; k < k1; ++k, c += plane) {
      double d_p = g0p, d_n = g0n;
      if (p.ntilt) {
        const double wz = k * p.dz - p.half_gap;
        for (int q = 0; q < p.ntilt; ++q) {
          const DepTrack tr = p.tilt[q];
          double dp, dn;
          track_values(tr, lateral_offset(p, x - tr.x0, p.Lx), lateral_offset(p, y - tr.y0, p.Ly), wz, same,
                       dp, dn);
          d_p += dp;
          d_n += dn;
        }
      }
      const double a = p.pos[c] + d_p;
      p.pos[c] = a;
      acc[0] += d_p;
      acc[3] += d_n;
      if (p.free_e) {  // eq. ion_elec_distribution: ions (1 - e^{-a z}), electrons p
        const double di = d_n * -expm1(-p.attach * (k * p.dz)), de = d_n * p.pfree;
        const double b = p.neg[c] + di, e = p.ele[c] + de;
        p.neg[c] = b;
        p.ele[c] = e;
        acc[1] += di;
        acc[2] += de;
        acc[4] = fmax(acc[4], fmax(a, b + e));
      } else {
        const double b = p.neg[c] + d_n;
        p.neg[c] = b;
        acc[1] += d_n;
        acc[4] = fmax(acc[4], fmax(a, b));
      }
    }
  }
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  {
    double v[NP];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = wave_sum(acc[q]);
    v[4] = wave_max(acc[4]);
    if (tid % kWave == 0)
      for (int q = 0; q < NP; ++q) lds[(tid / kWave) * NP + q] = v[q];
    __syncthreads();
    if (tid == 0) {
      double r[NP];
      for (int q = 0; q < NP; ++q) r[q] = lds[q];
      for (int w = 1; w < kNT / kWave; ++w) {
        for (int q = 0; q < 4; ++q) r[q] += lds[w * NP + q];
        r[4] = fmax(r[4], lds[w * NP + 4]);
      }
      for (int q = 0; q < NP; ++q) p.partials[(size_t)blockIdx.x * NP + q] = r[q];
    }
  }
  if (!arrive_last<kNT>(p.counter)) return;
  {
    double v[NP] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = tid; b < (int)gridDim.x; b += kNT) {
      for (int q = 0; q < 4; ++q) v[q] += p.partials[(size_t)b * NP + q];
      v[4] = fmax(v[4], p.partials[(size_t)b * NP + 4]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = wave_sum(v[q]);
    v[4] = wave_max(v[4]);
    __syncthreads();
    if (tid % kWave == 0)
      for (int q = 0; q < NP; ++q) lds[(tid / kWave) * NP + q] = v[q];
    __syncthreads();
    if (tid == 0) {
      double r[NP];
      for (int q = 0; q < NP; ++q) r[q] = lds[q];
      for (int w = 1; w < kNT / kWave; ++w) {
        for (int q = 0; q < 4; ++q) r[q] += lds[w * NP + q];
        r[4] = fmax(r[4], lds[w * NP + 4]);
      }
      RunState* st = p.state;
      st->released += r[0] * p.dV;
      st->released_pending += r[0] * p.dV;
      st->released_neg += r[1] * p.dV;
      st->released_pending_neg += r[1] * p.dV;
      st->released_e += r[2] * p.dV;
      st->released_q += r[3] * p.dV;
      st->max_beta_n = fmax(st->max_beta_n, p.beta * r[4]);
      *p.counter = 0u;
    }
  }
}

hipError_t launch_deposit(const DepositParams& p, hipStream_t s) {
  const int grid = 8 * p.per_xcd;
  hipLaunchKernelGGL(deposit_kernel, dim3(grid), dim3(kTX, kTY), 0, s, p);
  return hipGetLastError();
}

}  // namespace it
