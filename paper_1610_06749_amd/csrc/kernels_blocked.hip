// Temporally blocked stepping kernel: T explicit time steps per HBM pass.
//
// Each block (16 waves) owns an extended tile of 64 x 16 columns, one wave
// per row and one lane per column; every lane loads its periodically wrapped
// column, so lane neighbours are always the periodic x-neighbours.  After T
// steps only the centre (64 - 2T) x (16 - 2T) columns are still exact; those
// are the block's owned columns.  The block marches up a chunk of planes
// with a software pipeline over the T levels (time steps): at iteration K
// it loads level 0 on plane K and computes level t on plane K - t for
// t = 1..T, each from level t-1 on planes K-t-1, K-t, K-t+1.  The thread's
// own column of every level lives in registers; x-neighbours come from the
// adjacent lanes (DPP wave shifts), y-neighbours from one LDS plane per
// level written at the end of the previous iteration.  Only level T goes
// back to HBM (non-temporal stores), so a pass reads and writes each node
// once for T steps; the price is redundant work on the tile rim.
//
// The per-step tallies (the same quantities as the one-step kernel, one
// record per level) are taken on owned columns and on the block's own chunk
// of planes only, so every node and electrode face is counted once.
#include <algorithm>

#include "reduce.h"

namespace it {

namespace {

constexpr int kEX = 64, kEY = 16, kBNT = kEX * kEY;

__device__ inline double lane_from_left(double v) {  // value of lane - 1
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ inline double lane_from_right(double v) {  // value of lane + 1
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// SC: with the space-charge term (two more tallies per level).
template <int T, bool SC>
__global__ __launch_bounds__(kBNT) void step_blocked_kernel(StepParams p) {
  constexpr int NA = SC ? 7 : 5;  // tallies kept per level
  constexpr int OX = kEX - 2 * T, OY = kEY - 2 * T;
  if (p.state->done) return;
  __shared__ double lp[T][kEY][kEX], ln[T][kEY][kEX];
  __shared__ double edge[T][kEY][4];
  __shared__ double lds[(kBNT / kWave) * kAcc * T];

  const int lane = threadIdx.x, ty = threadIdx.y;
  const TileCoord tc = decode_tile(p.tiles_x, p.tiles_y, p.ntiles, p.per_xcd);
  const int x0 = tc.tx * OX, y0 = tc.ty * OY;
  // wrapped position of this column
  int xs = x0 - T + lane, ys = y0 - T + ty;
  xs = ((xs % p.nx) + p.nx) % p.nx;
  ys = ((ys % p.ny) + p.ny) % p.ny;
  const bool owned = tc.valid && lane >= T && lane < kEX - T && ty >= T && ty < kEY - T &&
                     x0 + (lane - T) < p.nx && y0 + (ty - T) < p.ny;
  const int za = 1 + tc.zc * p.zc;
  const int zb = tc.valid ? min(za + p.zc, p.nz) : za;
  const size_t plane = (size_t)p.nx * p.ny;
  const size_t col = (size_t)ys * p.nx + xs;
  const int tyl = ty > 0 ? ty - 1 : 0, tyr = ty + 1 < kEY ? ty + 1 : kEY - 1;
  const Coef cp = p.cp, cn = p.cn;
  const double beta = p.beta, gsp = p.gsp, gsn = p.gsn;
  const double* __restrict__ pin = p.pin;
  const double* __restrict__ nin = p.nin;
  double* __restrict__ pout = p.pout;
  double* __restrict__ nout = p.nout;

  for (int t = 0; t < T; ++t)
    if (lane < 4) edge[t][ty][lane] = 0.0;

  double mp[T], cpv[T], mn[T], cnv[T];  // levels 0..T-1: planes K-t-1 and K-t
  double acc[T][NA];  // per level: sink, n+', n-', |n+'|, |n-'| (, space-charge change of n+, n-)
#pragma unroll
  for (int t = 0; t < T; ++t) {
    mp[t] = cpv[t] = mn[t] = cnv[t] = 0.0;
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[t][q] = 0.0;
  }

  const int Klo = za - T, Khi = zb + T - 1;
  // level 0 of plane K is loaded one iteration ahead (planes outside
  // 0..nz read as zero; their address is clamped to plane 0)
  auto load0 = [&](int K, double& a, double& b) {
    const bool in = K >= 0 && K <= p.nz;
    const size_t off = (size_t)(in ? K : 0) * plane + col;
    a = pin[off];
    b = nin[off];
    if (!in) a = b = 0.0;
  };
  double np0, nn0;
  load0(Klo, np0, nn0);
  for (int K = tc.valid ? Klo : Khi + 1; K <= Khi; ++K) {
    double vp[T + 1], vn[T + 1];
    vp[0] = np0;
    vn[0] = nn0;
    load0(K + 1, np0, nn0);
#pragma unroll
    for (int t = 1; t <= T; ++t) {
      const int q = K - t;  // plane of level t in this iteration (uniform)
      const double pc = cpv[t - 1], nc = cnv[t - 1];
      // lateral neighbours of level t-1 on plane q (every lane takes part)
      const double pxl = lane_from_left(pc), pxr = lane_from_right(pc);
      const double nxl = lane_from_left(nc), nxr = lane_from_right(nc);
      if (q >= 1 && q <= p.nz - 1) {
        const double pyl = lp[t - 1][tyl][lane], pyr = lp[t - 1][tyr][lane];
        const double nyl = ln[t - 1][tyl][lane], nyr = ln[t - 1][tyr][lane];
        const double sink = beta * pc * nc;
        const double net = pc - nc;
        const double scp = SC ? gsp * pc * net : 0.0, scn = SC ? gsn * nc * net : 0.0;
        vp[t] = cp.a0 * pc + cp.ax * (pxr + pxl) + cp.ay * (pyr + pyl) + cp.azp * vp[t - 1] +
                cp.azm * mp[t - 1] - sink + scp;
        vn[t] = cn.a0 * nc + cn.ax * (nxr + nxl) + cn.ay * (nyr + nyl) + cn.azp * vn[t - 1] +
                cn.azm * mn[t - 1] - sink + scn;
        const bool mine = owned && q >= za && q < zb;
        if (mine) {
          acc[t - 1][0] += sink;
          acc[t - 1][1] += vp[t];
          acc[t - 1][2] += vn[t];
          acc[t - 1][3] += fabs(vp[t]);
          acc[t - 1][4] += fabs(vn[t]);
          if constexpr (SC) {
            acc[t - 1][5] += scp;
            acc[t - 1][6] += scn;
          }
        }
        if ((q == 1 || q == p.nz - 1) && q >= za && q < zb) {  // uniform over the block
          const double ep = wave_sum(owned ? pc : 0.0), en = wave_sum(owned ? nc : 0.0);
          if (lane == 0) {
            if (q == 1) {
              edge[t - 1][ty][0] += ep;
              edge[t - 1][ty][2] += en;
            }
            if (q == p.nz - 1) {
              edge[t - 1][ty][1] += ep;
              edge[t - 1][ty][3] += en;
            }
          }
        }
      } else {
        vp[t] = vn[t] = 0.0;  // electrode planes (and beyond) hold zero
      }
    }
    {
      const int q = K - T;
      if (owned && q >= za && q < zb) {
        const size_t c = (size_t)q * plane + col;
        __builtin_nontemporal_store(vp[T], &pout[c]);
        __builtin_nontemporal_store(vn[T], &nout[c]);
      }
    }
    lds_barrier();  // every level read its LDS plane of the previous iteration
#pragma unroll
    for (int t = 0; t < T; ++t) {
      lp[t][ty][lane] = vp[t];
      ln[t][ty][lane] = vn[t];
      mp[t] = cpv[t];
      cpv[t] = vp[t];
      mn[t] = cnv[t];
      cnv[t] = vn[t];
    }
    lds_barrier();
  }

  // block reduction of T records of kAcc slots (layout [level][slot])
  double a[kAcc * T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    a[t * kAcc + 0] = acc[t][0];
    a[t * kAcc + 1] = lane == 0 ? edge[t][ty][0] : 0.0;
    a[t * kAcc + 2] = lane == 0 ? edge[t][ty][1] : 0.0;
    a[t * kAcc + 3] = lane == 0 ? edge[t][ty][2] : 0.0;
    a[t * kAcc + 4] = lane == 0 ? edge[t][ty][3] : 0.0;
    a[t * kAcc + 5] = acc[t][1];
    a[t * kAcc + 6] = acc[t][2];
    a[t * kAcc + 7] = acc[t][3];
    a[t * kAcc + 8] = acc[t][4];
    if constexpr (SC) {
      a[t * kAcc + 9] = acc[t][5];
      a[t * kAcc + 10] = acc[t][6];
    } else {
      a[t * kAcc + 9] = 0.0;
      a[t * kAcc + 10] = 0.0;
    }
    a[t * kAcc + 11] = 0.0;  // escaped: the blocked kernel is periodic only
    a[t * kAcc + 12] = 0.0;
  }
  block_sum_store<kAcc * T, kBNT>(a, p.partials + (size_t)blockIdx.x * kAcc * T, lds);
}

constexpr int kMinT = 2, kMaxBlockedT = 5;

int zchunk_for(long cols, int nint, int T) {
  // longest chunk (least z redundancy, 2T extra planes per chunk) that still
  // gives about a thousand blocks
  int zc = 64;
  while (zc > 2 * T && cols * ((nint + zc - 1) / zc) < 1024) zc /= 2;
  return std::max(1, std::min(zc, nint));
}

}  // namespace

int blocked_supported(int T, int tile_y) {
  (void)tile_y;
  return T >= kMinT && T <= kMaxBlockedT;
}

void blocked_tiling(int nx, int ny, int nz, int T, int tile_y, int* grid, int* per_xcd, int* tiles_x,
                    int* tiles_y, int* ntiles, int* zc_out, int* zchunks_out) {
  (void)tile_y;
  const int OX = kEX - 2 * T, OY = kEY - 2 * T;
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

hipError_t launch_step_blocked(const StepParams& p0, int T, int tile_y, hipStream_t s, hipEvent_t ev_begin,
                               hipEvent_t ev_end) {
  StepParams p = p0;
  int grid, per, tx, ty, nt, zc, zch;
  blocked_tiling(p.nx, p.ny, p.nz, T, tile_y, &grid, &per, &tx, &ty, &nt, &zc, &zch);
  p.tiles_x = tx;
  p.tiles_y = ty;
  p.zchunks = zch;
  p.zc = zc;
  p.ntiles = nt;
  p.per_xcd = per;
  const dim3 block(kEX, kEY);
  if (T < 2 || T > 5) return hipErrorInvalidValue;
  if (ev_begin && hipEventRecord(ev_begin, s) != hipSuccess) return hipErrorInvalidValue;
  const bool sc = p.gsp != 0.0 || p.gsn != 0.0;
  const dim3 g(grid);
  switch (T * 2 + (sc ? 1 : 0)) {
    case 4: hipLaunchKernelGGL((step_blocked_kernel<2, false>), g, block, 0, s, p); break;
    case 5: hipLaunchKernelGGL((step_blocked_kernel<2, true>), g, block, 0, s, p); break;
    case 6: hipLaunchKernelGGL((step_blocked_kernel<3, false>), g, block, 0, s, p); break;
    case 7: hipLaunchKernelGGL((step_blocked_kernel<3, true>), g, block, 0, s, p); break;
    case 8: hipLaunchKernelGGL((step_blocked_kernel<4, false>), g, block, 0, s, p); break;
    case 9: hipLaunchKernelGGL((step_blocked_kernel<4, true>), g, block, 0, s, p); break;
    case 10: hipLaunchKernelGGL((step_blocked_kernel<5, false>), g, block, 0, s, p); break;
    case 11: hipLaunchKernelGGL((step_blocked_kernel<5, true>), g, block, 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_end && hipEventRecord(ev_end, s) != hipSuccess) return hipErrorInvalidValue;
  return launch_reduce_steps(p, grid, T, s);
}

}  // namespace it
