// One explicit time step of both species on one 64 x SY column tile and a
// chunk of planes, with the per-block partial tallies (shared by the
// single-chamber and the batched stepping kernels).
#pragma once

#include "reduce.h"

namespace it {

constexpr int kTX = 64;

// Stepping tile: 64 x SY columns (SY = 8 or 16 rows, one wave per row).
// LDS holds plane k of the tile with a one-node rim: interior (r, x) sits at
// [r + 1][x + 1]; the rim column/row that follows the last valid column/row
// (w, h of the tile, smaller than 64/SY on the ragged edge of the grid)
// holds the periodic neighbour, so every active node reads its four lateral
// neighbours from LDS at fixed offsets.  Waves 0-3 load the rim from global
// memory (wave-uniform branches), all other loads are unconditional.
template <int SY>
__device__ inline void plain_tile_step(const StepParams& p, const TileCoord t, double* partial_out) {
  constexpr int kSNT = kTX * SY;
  __shared__ double sp[SY + 2][kTX + 2], sn[SY + 2][kTX + 2];
  __shared__ double lds[(kSNT / kWave) * kAcc];
  // per-wave sums of n on the planes next to the electrodes (slots 1-4)
  __shared__ double edge[SY][4];

  // running sums of slots 0 and 5-8 (slots 1-4 go through `edge`)
  double acc[kAcc];
#pragma unroll
  for (int q = 0; q < kAcc; ++q) acc[q] = 0.0;

  const int lane = threadIdx.x, ty = threadIdx.y;
  if (lane < 4) edge[ty][lane] = 0.0;
  const int x0 = t.tx * kTX, y0 = t.ty * SY;
  const int w = min(kTX, p.nx - x0), h = min(SY, p.ny - y0);  // valid extent of the tile
  const int i = x0 + lane, j = y0 + ty;
  const bool active = t.valid && lane < w && ty < h;
  const int k0 = 1 + t.zc * p.zc;
  const int k1 = t.valid ? min(k0 + p.zc, p.nz) : k0;
  const size_t plane = (size_t)p.nx * p.ny;
  const int ic = min(i, p.nx - 1), jc = min(j, p.ny - 1);
  // rim sources (periodic wraps)
  const int i_left = x0 == 0 ? p.nx - 1 : x0 - 1;
  const int i_right = x0 + w == p.nx ? 0 : x0 + w;
  const int j_top = y0 == 0 ? p.ny - 1 : y0 - 1;
  const int j_bot = y0 + h == p.ny ? 0 : y0 + h;
  const double* __restrict__ pin = p.pin;
  const double* __restrict__ nin = p.nin;
  double* __restrict__ pout = p.pout;
  double* __restrict__ nout = p.nout;
  const Coef cp = p.cp, cn = p.cn;
  const double beta = p.beta;
  const size_t own = (size_t)jc * p.nx + ic;
  // rim element this thread loads (if any): waves 0/1 rows, waves 2/3 columns
  size_t rim_off = 0;
  int rim_r = -1, rim_c = -1;
  if (ty == 0 && lane < w) { rim_off = (size_t)j_top * p.nx + i; rim_r = 0; rim_c = lane + 1; }
  if (ty == 1 && lane < w) { rim_off = (size_t)j_bot * p.nx + i; rim_r = h + 1; rim_c = lane + 1; }
  if (ty == 2 && lane < h) { rim_off = (size_t)(y0 + lane) * p.nx + i_left; rim_r = lane + 1; rim_c = 0; }
  if (ty == 3 && lane < h) { rim_off = (size_t)(y0 + lane) * p.nx + i_right; rim_r = lane + 1; rim_c = w + 1; }
  const bool rim = t.valid && rim_r >= 0;

  // Loads and arithmetic run unpredicated on clamped addresses (inactive
  // lanes compute values nobody uses); only LDS interior writes, stores and
  // tallies depend on `active`.  This keeps the loop free of divergent
  // branches around loads, so the compiler can overlap them.
  const double am = active ? 1.0 : 0.0;
  const size_t own_k0 = (size_t)k0 * plane + own;
  double pm = pin[own_k0 - plane], pc = pin[own_k0];
  double nm = nin[own_k0 - plane], nc = nin[own_k0];
  for (int k = k0; k < k1; ++k) {
    const size_t base = (size_t)k * plane;
    const size_t c = base + own;
    const double pp = pin[c + plane], np = nin[c + plane];  // plane k+1 <= nz
    if (rim) {
      sp[rim_r][rim_c] = pin[base + rim_off];
      sn[rim_r][rim_c] = nin[base + rim_off];
    }
    if (active) {  // inactive threads must not touch the rim slots past the valid extent
      sp[ty + 1][lane + 1] = pc;
      sn[ty + 1][lane + 1] = nc;
    }
    __syncthreads();
    const double pxl = sp[ty + 1][lane], pxr = sp[ty + 1][lane + 2];
    const double pyl = sp[ty][lane + 1], pyr = sp[ty + 2][lane + 1];
    const double nxl = sn[ty + 1][lane], nxr = sn[ty + 1][lane + 2];
    const double nyl = sn[ty][lane + 1], nyr = sn[ty + 2][lane + 1];
    const double sink = beta * pc * nc;
    const double vp = cp.a0 * pc + cp.ax * (pxr + pxl) + cp.ay * (pyr + pyl) + cp.azp * pp +
                      cp.azm * pm - sink;
    const double vn = cn.a0 * nc + cn.ax * (nxr + nxl) + cn.ay * (nyr + nyl) + cn.azp * np +
                      cn.azm * nm - sink;
    if (active) {
      __builtin_nontemporal_store(vp, &pout[c]);
      __builtin_nontemporal_store(vn, &nout[c]);
    }
    acc[0] += am * sink;
    acc[5] += am * vp;
    acc[6] += am * vn;
    acc[7] += am * fabs(vp);
    acc[8] += am * fabs(vn);
    if (k == 1 || k == p.nz - 1) {  // uniform over the block
      const double sp_ = wave_sum(am * pc), sn_ = wave_sum(am * nc);
      if (lane == 0) {
        if (k == 1) {  // anode side
          edge[ty][0] += sp_;
          edge[ty][2] += sn_;
        }
        if (k == p.nz - 1) {  // cathode side (the same plane when nz = 2)
          edge[ty][1] += sp_;
          edge[ty][3] += sn_;
        }
      }
    }
    __syncthreads();
    pm = pc;
    pc = pp;
    nm = nc;
    nc = np;
  }

  if (lane == 0) {  // the electrode-plane sums enter the block reduction per wave
    acc[1] = edge[ty][0];
    acc[2] = edge[ty][1];
    acc[3] = edge[ty][2];
    acc[4] = edge[ty][3];
  }
  block_sum_store<kAcc, kSNT>(acc, partial_out, lds);
}

}  // namespace it
