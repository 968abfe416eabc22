// Temporally blocked stepping kernel: T explicit time steps per HBM pass.
//
// A block of 8 waves owns an extended tile of 64 columns by 8 R rows: lane l
// holds column l, and wave w the R consecutive rows w R .. w R + R - 1, in
// registers.  Every lane loads its periodically wrapped column, so lane and
// row neighbours are always the periodic x and y neighbours.  Each of the T
// steps (levels) is exact on one node less on every side, so after T steps
// the centre (64 - 2T) x (8 R - 2T) columns are exact: the block's owned
// columns.  The block marches up a chunk of planes with a software pipeline
// over the levels: at iteration K it loads level 0 on plane K and computes
// level t on plane K - t for t = 1..T from level t-1 on planes K-t-1, K-t and
// K-t+1, which the thread keeps in registers (two planes per level plus the
// one just computed).
//
// Lateral neighbours of level t-1 on plane K-t: x from the adjacent lanes
// (whole-wave DPP shifts), y from the thread's own rows; only the first and
// the last row of a wave's strip need the row of the wave above or below,
// which the waves exchange through LDS: at the end of an iteration every
// wave writes the edge rows of each level's newest plane into one of two
// buffers, and a single barrier at the top of the next iteration makes them
// visible (the other buffer is being read meanwhile).  Only level T goes
// back to HBM (non-temporal stores), so a pass reads and writes each owned
// node once for T steps; the price is the redundant work on the tile's rim
// and on the T planes of z halo at each end of a chunk.
//
// The per-step tallies (the same quantities as the one-step kernel, one
// record per level) are taken on owned columns and on the block's own chunk
// of planes only, so every node and electrode face is counted once.  As in
// the one-step kernel, a launch has one block more than tiles when the
// previous pass is still unrecorded: that block sums the previous pass's
// partials in a fixed order and records its steps while the others step.
#include <algorithm>

#include "reduce.h"

namespace it {

namespace {

constexpr int kBW = 8;                // waves per block
constexpr int kBX = 64;               // columns of the extended tile
constexpr int kBNT = kBW * kWave;     // threads per block
constexpr int kMinT = 2, kMaxBlockedT = 4;  // T = 5 would need 170 KB of LDS for its edge rows

// Values of the neighbouring lanes (whole-wave DPP shifts by one lane); the
// lane at the wave's edge, which has no such neighbour, gets 0.
__device__ inline double lane_from_left(double v) {  // value of lane - 1
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ inline double lane_from_right(double v) {  // value of lane + 1
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Global-memory byte pointer and a wave-uniform plane pointer in scalar
// registers (threads add their 32-bit in-plane byte offsets: a plane holds
// at most 2^28 nodes, checked on the host).
typedef __attribute__((address_space(1))) char gchar;
typedef __attribute__((address_space(1))) double gdouble;

__device__ inline gchar* uniform_ptr(const void* ptr) {
  const uint64_t v = (uint64_t)ptr;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gchar*)(((uint64_t)hi << 32) | lo);
}

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

// SC: with the space-charge term (two more tallies per level).
template <int T, int R, bool SC>
__global__ __launch_bounds__(kBNT) __attribute__((amdgpu_waves_per_eu(2, 2))) void step_blocked_kernel(StepParams p) {
  if (p.prev_partials && blockIdx.x == gridDim.x - 1) {
    record_previous_pass(p);
    return;
  }
  constexpr int EY = kBW * R;             // rows of the extended tile
  constexpr int OX = kBX - 2 * T, OY = EY - 2 * T;
  constexpr int NA = SC ? 7 : 5;          // tallies kept per level
  // The extra block of this launch may set the stop flag while the others
  // start: one thread reads it for the whole block, so that every wave takes
  // the same branch (the waves meet at barriers below).
  __shared__ int stopped;
  if (threadIdx.x == 0 && threadIdx.y == 0) stopped = p.state->done;
  __syncthreads();
  if (stopped) return;
  // edge rows of each level's newest plane: [buffer][level][wave][first/last][species][lane]
  __shared__ double edge_rows[2][T][kBW][2][2][kWave];
  __shared__ double edge_sum[T][kBW][4];  // per-wave sums of n on the planes next to the electrodes
  __shared__ double lds[(kBNT / kWave) * kAcc * T];

  const int lane = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);  // the wave (uniform)
  const TileCoord tc = decode_tile(p.tiles_x, p.tiles_y, p.ntiles, p.per_xcd);
  const int x0 = tc.tx * OX, y0 = tc.ty * OY;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  // wrapped position of this lane's column and of the thread's rows
  int xs = (x0 - T + lane) % nx;
  if (xs < 0) xs += nx;
  const bool own_x = lane >= T && lane < kBX - T && x0 + (lane - T) < nx;
  unsigned off[R];  // in-plane byte offsets of the thread's nodes
  bool own_y[R];    // the row is owned (wave-uniform)
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int g = w * R + r;  // row in the extended tile
    int ys = (y0 - T + g) % ny;
    if (ys < 0) ys += ny;
    off[r] = (unsigned)(ys * nx + xs) * 8u;
    own_y[r] = tc.valid && g >= T && g < EY - T && y0 + (g - T) < ny;
  }
  const int za = 1 + tc.zc * p.zc;
  const int zb = tc.valid ? min(za + p.zc, nz) : za;
  const size_t plane = (size_t)nx * ny;
  const Coef cp = p.cp, cn = p.cn;
  const double beta = p.beta, gsp = p.gsp, gsn = p.gsn;

  if (lane < 4)
#pragma unroll
    for (int t = 0; t < T; ++t) edge_sum[t][w][lane] = 0.0;

  // level t (0..T-1): mp/mn its plane K-t-2, cpv/cnv its plane K-t-1 at the
  // start of iteration K
  double mp[T][R], mn[T][R], cpv[T][R], cnv[T][R];
  double acc[T][NA];  // tallies of the owned rows, all columns (masked at the end)
#pragma unroll
  for (int t = 0; t < T; ++t) {
#pragma unroll
    for (int r = 0; r < R; ++r) mp[t][r] = mn[t][r] = cpv[t][r] = cnv[t][r] = 0.0;
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[t][q] = 0.0;
  }

  const int Klo = za - T, Khi = zb + T - 1;
  // Level 0 of plane K.  Planes before the anode and beyond the cathode read
  // the electrode plane itself, which always holds zero: the loads need no
  // branch or select, so they stay in flight across the iteration (a
  // branch around them made the compiler wait for them at once).
  double np0[R], nn0[R];
  auto load0 = [&](int K) {
    const int Kc = min(max(K, 0), nz);
    const gchar* bp = uniform_ptr(p.pin + (size_t)Kc * plane);
    const gchar* bn = uniform_ptr(p.nin + (size_t)Kc * plane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      np0[r] = *(const gdouble*)(bp + off[r]);
      nn0[r] = *(const gdouble*)(bn + off[r]);
    }
  };
  // the zero planes' edge rows held at the start
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      edge_rows[Klo & 1][t][w][0][s][lane] = 0.0;
      edge_rows[Klo & 1][t][w][1][s][lane] = 0.0;
    }
  const int wu = w > 0 ? w - 1 : 0, wd = w < kBW - 1 ? w + 1 : kBW - 1;

  // One iteration: planes K - t of levels t = 1..T, then the edge rows of
  // every level's newest plane for the next iteration.  (One copy of this
  // body: the register allocator keeps the pipeline's state in registers
  // only when the loop body is not duplicated.)
  auto iterate = [&](int K) {
    const int buf = K & 1;
    lds_barrier();  // the edge rows written at the end of the previous iteration
    double vp[R], vn[R];  // the newest level's values, plane K - t
#pragma unroll
    for (int r = 0; r < R; ++r) {
      vp[r] = np0[r];
      vn[r] = nn0[r];
    }
    if (K + 1 <= Khi) load0(K + 1);
#pragma unroll
    for (int t = 1; t <= T; ++t) {
      const int q = K - t;  // plane of level t in this iteration (block-uniform)
      const bool interior = q >= 1 && q <= nz - 1;
      const bool counted = q >= za && q < zb;
      if (counted && (q == 1 || q == nz - 1)) {  // the old values of step t next to an electrode
        double sp_ = 0.0, sn_ = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (own_y[r]) {
            sp_ += cpv[t - 1][r];
            sn_ += cnv[t - 1][r];
          }
        sp_ = wave_sum(own_x ? sp_ : 0.0);
        sn_ = wave_sum(own_x ? sn_ : 0.0);
        if (lane == 0) {
          if (q == 1) {
            edge_sum[t - 1][w][0] += sp_;
            edge_sum[t - 1][w][2] += sn_;
          }
          if (q == nz - 1) {
            edge_sum[t - 1][w][1] += sp_;
            edge_sum[t - 1][w][3] += sn_;
          }
        }
      }
      // neighbours above the strip's first row and below its last, level t-1
      // on plane q (the other waves' edge rows)
      const double up_p = edge_rows[buf][t - 1][wu][1][0][lane], up_n = edge_rows[buf][t - 1][wu][1][1][lane];
      const double dn_p = edge_rows[buf][t - 1][wd][0][0][lane], dn_n = edge_rows[buf][t - 1][wd][0][1][lane];
      double np[R], nn[R];
#pragma unroll
      for (int r = 0; r < R; ++r) np[r] = nn[r] = 0.0;  // electrode planes and beyond hold zero
      if (interior)  // block-uniform
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double pc = cpv[t - 1][r], nc = cnv[t - 1][r];
        const double pxl = lane_from_left(pc), pxr = lane_from_right(pc);
        const double nxl = lane_from_left(nc), nxr = lane_from_right(nc);
        const double pyl = r > 0 ? cpv[t - 1][r - 1] : up_p, pyr = r < R - 1 ? cpv[t - 1][r + 1] : dn_p;
        const double nyl = r > 0 ? cnv[t - 1][r - 1] : up_n, nyr = r < R - 1 ? cnv[t - 1][r + 1] : dn_n;
        const double sink = beta * pc * nc;
        const double net = pc - nc;
        const double scp = SC ? gsp * pc * net : 0.0, scn = SC ? gsn * nc * net : 0.0;
        const double a = cp.a0 * pc + cp.ax * (pxr + pxl) + cp.ay * (pyr + pyl) + cp.azp * vp[r] +
                         cp.azm * mp[t - 1][r] - sink + scp;
        const double b = cn.a0 * nc + cn.ax * (nxr + nxl) + cn.ay * (nyr + nyl) + cn.azp * vn[r] +
                         cn.azm * mn[t - 1][r] - sink + scn;
        np[r] = a;
        nn[r] = b;
        if (counted && own_y[r]) {  // wave-uniform; the columns are masked at the end
          acc[t - 1][0] += sink;
          acc[t - 1][1] += a;
          acc[t - 1][2] += b;
          acc[t - 1][3] += fabs(a);
          acc[t - 1][4] += fabs(b);
          if constexpr (SC) {
            acc[t - 1][5] += scp;
            acc[t - 1][6] += scn;
          }
        }
      }
      // level t-1 moves on: plane K-t becomes its older plane, K-t+1 its current one
#pragma unroll
      for (int r = 0; r < R; ++r) {
        mp[t - 1][r] = cpv[t - 1][r];
        mn[t - 1][r] = cnv[t - 1][r];
        cpv[t - 1][r] = vp[r];
        cnv[t - 1][r] = vn[r];
        vp[r] = np[r];
        vn[r] = nn[r];
      }
    }
    // level T on plane K - T: the pass's output
    const int q = K - T;
    if (q >= za && q < zb) {
      gchar* op = uniform_ptr(p.pout + (size_t)q * plane);
      gchar* on = uniform_ptr(p.nout + (size_t)q * plane);
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (own_y[r] && own_x) {
          __builtin_nontemporal_store(vp[r], (gdouble*)(op + off[r]));
          __builtin_nontemporal_store(vn[r], (gdouble*)(on + off[r]));
        }
    }
    // edge rows of every level's current plane, for the next iteration
#pragma unroll
    for (int t = 0; t < T; ++t) {
      edge_rows[buf ^ 1][t][w][0][0][lane] = cpv[t][0];
      edge_rows[buf ^ 1][t][w][0][1][lane] = cnv[t][0];
      edge_rows[buf ^ 1][t][w][1][0][lane] = cpv[t][R - 1];
      edge_rows[buf ^ 1][t][w][1][1][lane] = cnv[t][R - 1];
    }
  };

  if (tc.valid) {
    load0(Klo);
    for (int K = Klo; K <= Khi; ++K) iterate(K);
  }

  __syncthreads();  // edge sums of the last planes
  // block reduction of T records of kAcc slots (layout [level][slot]); the
  // tallies of columns outside the owned ones are selected away here
  double a[kAcc * T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    a[t * kAcc + 0] = own_x ? acc[t][0] : 0.0;
    a[t * kAcc + 1] = lane == 0 ? edge_sum[t][w][0] : 0.0;
    a[t * kAcc + 2] = lane == 0 ? edge_sum[t][w][1] : 0.0;
    a[t * kAcc + 3] = lane == 0 ? edge_sum[t][w][2] : 0.0;
    a[t * kAcc + 4] = lane == 0 ? edge_sum[t][w][3] : 0.0;
    a[t * kAcc + 5] = own_x ? acc[t][1] : 0.0;
    a[t * kAcc + 6] = own_x ? acc[t][2] : 0.0;
    a[t * kAcc + 7] = own_x ? acc[t][3] : 0.0;
    a[t * kAcc + 8] = own_x ? acc[t][4] : 0.0;
    if constexpr (SC) {
      a[t * kAcc + 9] = own_x ? acc[t][5] : 0.0;
      a[t * kAcc + 10] = own_x ? acc[t][6] : 0.0;
    } else {
      a[t * kAcc + 9] = 0.0;
      a[t * kAcc + 10] = 0.0;
    }
    a[t * kAcc + 11] = 0.0;  // escaped: the blocked kernel is periodic only
    a[t * kAcc + 12] = 0.0;
  }
  block_sum_store<kAcc * T, kBNT>(a, p.partials + (size_t)blockIdx.x * kAcc * T, lds);
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
  if (sc)
    hipLaunchKernelGGL((step_blocked_kernel<T, R, true>), g, block, 0, s, p);
  else
    hipLaunchKernelGGL((step_blocked_kernel<T, R, false>), g, block, 0, s, p);
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
