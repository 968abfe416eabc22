// One explicit time step of both species on one 64 x SY column tile and a
// chunk of planes, with the per-block partial tallies (shared by the
// single-chamber and the batched stepping kernels).
#pragma once

#include "reduce.h"

namespace it {

constexpr int kTX = 64;

// Global-memory byte pointer.
typedef __attribute__((address_space(1))) char gchar;

// A wave-uniform global pointer held in scalar registers.
__device__ inline gchar* uniform_ptr(const void* ptr) {
  const uint64_t v = (uint64_t)ptr;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gchar*)(((uint64_t)hi << 32) | lo);
}

// Per-plane work of the tile step: the own column's values at k-1, k, k+1
// are in registers, plane k of the tile with its one-node rim in LDS.
struct PlaneRegs {
  double p, n;
};

// Stepping tile: TX x (SY * 64 / TX) columns with SY waves: TX = 64 gives one
// row per wave (64 x 8 or 64 x 16), TX = 32 two rows of 32 per wave (32 x 16
// with 8 waves: less rim per node, and fewer idle lanes on narrow grids).
// LDS holds plane k of the tile with a one-node rim: interior (r, x) sits at
// [r + 1][x + 1]; the rim column/row that follows the last valid column/row
// (w, h of the tile, smaller than 64/SY on the ragged edge of the grid)
// holds the periodic neighbour (or zero beyond an absorbing lateral
// boundary), so every active node reads its four lateral neighbours from LDS
// at fixed offsets.  Waves 0-3 load the rim from global
// memory (wave-uniform branches), all other loads are unconditional.
//
// Pipelining: plane k+2 of the own column and the rim of plane k+1 are
// requested while plane k is computed, so two planes of loads are in flight
// per thread (70 VGPRs without the optional terms: seven waves per SIMD, more
// than the 16 waves per CU the default tiling places).  The LDS plane is double-buffered, so one barrier per plane
// suffices: buffer k&1 is rewritten at plane k+2, after every thread has
// passed the barrier of plane k+1 and hence finished reading plane k.  The
// barrier orders LDS only; it does not wait for the global loads in flight.
// SC: with the space-charge term (its two extra tallies cost registers, so
// runs without it use the instance without them).  AB: honours
// p.absorbing (absorbing lateral boundaries and the escaped tally, slots
// 11-12); the instance without it is periodic only.
template <int SY, bool SC, bool AB, int TX = kTX>
__device__ inline void plain_tile_step(const StepParams& p, const TileCoord t, double* partial_out) {
  static_assert(TX == 64 || TX == 32, "tile width");
  constexpr int kSNT = kTX * SY;
  constexpr int SR = SY * (kTX / TX);  // rows of the tile
  __shared__ double sp[2][SR + 2][TX + 2], sn[2][SR + 2][TX + 2];
  __shared__ double lds[(kSNT / kWave) * kAcc];
  // per-wave sums of n on the planes next to the electrodes (slots 1-4)
  __shared__ double edge[SY][4];

  // running sums of slots 0 and 5-12 (slots 1-4 go through `edge`)
  double acc[kAcc];
#pragma unroll
  for (int q = 0; q < kAcc; ++q) acc[q] = 0.0;

  const int lane = threadIdx.x, ty = threadIdx.y;  // ty: the wave
  if (lane < 4) edge[ty][lane] = 0.0;
  const int xl = lane % TX, rl = ty * (kTX / TX) + lane / TX;  // column and row of this thread in the tile
  const int x0 = t.tx * TX, y0 = t.ty * SR;
  const int w = min(TX, p.nx - x0), h = min(SR, p.ny - y0);  // valid extent of the tile
  const int i = x0 + xl, j = y0 + rl;
  const bool active = t.valid && xl < w && rl < h;
  const int nz = p.nz;
  const int k0 = 1 + t.zc * p.zc;
  const int k1 = t.valid ? min(k0 + p.zc, nz) : k0;
  const size_t plane = (size_t)p.nx * p.ny;
  const int ic = min(i, p.nx - 1), jc = min(j, p.ny - 1);
  // rim sources (periodic wraps)
  const int i_left = x0 == 0 ? p.nx - 1 : x0 - 1;
  const int i_right = x0 + w == p.nx ? 0 : x0 + w;
  const int j_top = y0 == 0 ? p.ny - 1 : y0 - 1;
  const int j_bot = y0 + h == p.ny ? 0 : y0 + h;
  const Coef cp = p.cp, cn = p.cn;
  const double beta = p.beta, gsp = p.gsp, gsn = p.gsn;
  // in-plane byte offsets (a plane holds at most 2^28 nodes, checked on the
  // host, so they fit 32 bits and the loads take a scalar base address)
  const unsigned own = (unsigned)(jc * p.nx + ic) * 8u;
  // rim element this thread loads (if any): waves 0/1 rows, waves 2/3 columns
  unsigned rim_off = 0;
  int rim_r = -1, rim_c = -1;
  if (ty == 0 && lane < w) { rim_off = (unsigned)(j_top * p.nx + i) * 8u; rim_r = 0; rim_c = lane + 1; }
  if (ty == 1 && lane < w) { rim_off = (unsigned)(j_bot * p.nx + i) * 8u; rim_r = h + 1; rim_c = lane + 1; }
  if (ty == 2 && lane < h) { rim_off = (unsigned)((y0 + lane) * p.nx + i_left) * 8u; rim_r = lane + 1; rim_c = 0; }
  if (ty == 3 && lane < h) { rim_off = (unsigned)((y0 + lane) * p.nx + i_right) * 8u; rim_r = lane + 1; rim_c = w + 1; }
  const bool rim = t.valid && rim_r >= 0;
  // absorbing lateral boundaries: a rim node beyond the cell is zero (never
  // loaded; its registers stay 0), and each node next to the boundary loses
  // ax (or ay) times its density per missing neighbour
  const bool absorbing = AB && p.absorbing;
  bool rim_outside = false;
  double esc_p = 0.0, esc_n = 0.0;  // weights of the escaped tally
  if (absorbing) {
    rim_outside = (ty == 0 && y0 == 0) || (ty == 1 && y0 + h == p.ny) || (ty == 2 && x0 == 0) ||
                  (ty == 3 && x0 + w == p.nx);
    const double mx = (double)((i == 0) + (i == p.nx - 1)), my = (double)((j == 0) + (j == p.ny - 1));
    esc_p = p.cp.ax * mx + p.cp.ay * my;
    esc_n = p.cn.ax * mx + p.cn.ay * my;
  }

  // plane pointers are block-uniform (scalar registers); threads add their
  // 32-bit in-plane byte offset
  auto in_p = [&](int k) { return uniform_ptr(p.pin + (size_t)k * plane); };
  auto in_n = [&](int k) { return uniform_ptr(p.nin + (size_t)k * plane); };
  auto ld = [](const gchar* base, unsigned off) {
    return *(const __attribute__((address_space(1))) double*)(base + off);
  };

  // One plane.  (m, c, q1): own column at k-1, k, k+1; q2 receives k+2.
  // rc: rim values of plane k; rn receives the rim of plane k+1.
  auto plane_step = [&](int k, int buf, const PlaneRegs& m, const PlaneRegs& c, const PlaneRegs& q1,
                        PlaneRegs& q2, const PlaneRegs& rc, PlaneRegs& rn) {
    const int k2 = min(k + 2, nz);  // plane nz exists (the cathode, zero)
    q2.p = ld(in_p(k2), own);
    q2.n = ld(in_n(k2), own);
    if (rim) {  // one branch: the periodic instance keeps its loads and LDS stores together
      if (!rim_outside) {
        rn.p = ld(in_p(k + 1), rim_off);
        rn.n = ld(in_n(k + 1), rim_off);
      }
      sp[buf][rim_r][rim_c] = rc.p;
      sn[buf][rim_r][rim_c] = rc.n;
    }
    if (active) {  // inactive threads must not touch the rim slots past the valid extent
      sp[buf][rl + 1][xl + 1] = c.p;
      sn[buf][rl + 1][xl + 1] = c.n;
    }
    lds_barrier();
    const double pxl = sp[buf][rl + 1][xl], pxr = sp[buf][rl + 1][xl + 2];
    const double pyl = sp[buf][rl][xl + 1], pyr = sp[buf][rl + 2][xl + 1];
    const double nxl = sn[buf][rl + 1][xl], nxr = sn[buf][rl + 1][xl + 2];
    const double nyl = sn[buf][rl][xl + 1], nyr = sn[buf][rl + 2][xl + 1];
    const double sink = beta * c.p * c.n;
    const double net = c.p - c.n;  // div E in units of q/eps0 (space charge)
    const double scp = SC ? gsp * c.p * net : 0.0, scn = SC ? gsn * c.n * net : 0.0;
    const double vp = cp.a0 * c.p + cp.ax * (pxr + pxl) + cp.ay * (pyr + pyl) + cp.azp * q1.p +
                      cp.azm * m.p - sink + scp;
    const double vn = cn.a0 * c.n + cn.ax * (nxr + nxl) + cn.ay * (nyr + nyl) + cn.azp * q1.n +
                      cn.azm * m.n - sink + scn;
    if (active) {
      const size_t o = (size_t)k * plane;
      __builtin_nontemporal_store(vp, (__attribute__((address_space(1))) double*)(uniform_ptr(p.pout + o) + own));
      __builtin_nontemporal_store(vn, (__attribute__((address_space(1))) double*)(uniform_ptr(p.nout + o) + own));
    }
    // Threads outside the tile's valid extent read LDS slots that this
    // block never wrote (whatever an earlier workgroup left, possibly NaN),
    // so their values are selected away, never multiplied by zero.
    const double vpa = active ? vp : 0.0, vna = active ? vn : 0.0;
    acc[0] += active ? sink : 0.0;
    acc[5] += vpa;
    acc[6] += vna;
    acc[7] += fabs(vpa);
    acc[8] += fabs(vna);
    if (SC) {
      acc[9] += active ? scp : 0.0;
      acc[10] += active ? scn : 0.0;
    }
    if (AB) {
      acc[11] += active ? esc_p * c.p : 0.0;
      acc[12] += active ? esc_n * c.n : 0.0;
    }
    if (k == 1 || k == nz - 1) {  // uniform over the block
      const double sp_ = wave_sum(active ? c.p : 0.0), sn_ = wave_sum(active ? c.n : 0.0);
      if (lane == 0) {
        if (k == 1) {  // anode side
          edge[ty][0] += sp_;
          edge[ty][2] += sn_;
        }
        if (k == nz - 1) {  // cathode side (the same plane when nz = 2)
          edge[ty][1] += sp_;
          edge[ty][3] += sn_;
        }
      }
    }
  };

  // Registers rotate with period 4 (own column) and 2 (rim); the loop is
  // unrolled by 4 so that no value is moved between registers while its
  // load may still be in flight.
  PlaneRegs r0, r1, r2, r3, ra, rb;
  ra.p = ra.n = rb.p = rb.n = 0.0;
  if (rim && !rim_outside) {
    ra.p = ld(in_p(k0), rim_off);
    ra.n = ld(in_n(k0), rim_off);
  }
  r0.p = ld(in_p(k0 - 1), own);
  r0.n = ld(in_n(k0 - 1), own);
  r1.p = ld(in_p(k0), own);
  r1.n = ld(in_n(k0), own);
  r2.p = ld(in_p(k0 + 1), own);  // k0 + 1 <= nz
  r2.n = ld(in_n(k0 + 1), own);
  for (int k = k0; k < k1; k += 4) {
    plane_step(k, 0, r0, r1, r2, r3, ra, rb);
    if (k + 1 >= k1) break;
    plane_step(k + 1, 1, r1, r2, r3, r0, rb, ra);
    if (k + 2 >= k1) break;
    plane_step(k + 2, 0, r2, r3, r0, r1, ra, rb);
    if (k + 3 >= k1) break;
    plane_step(k + 3, 1, r3, r0, r1, r2, rb, ra);
  }

  __syncthreads();  // edge sums of the last plane
  if (lane == 0) {  // the electrode-plane sums enter the block reduction per wave
    acc[1] = edge[ty][0];
    acc[2] = edge[ty][1];
    acc[3] = edge[ty][2];
    acc[4] = edge[ty][3];
  }
  // slots 9-10 (space charge) and 11-12 (escaped) are zero in instances
  // without those terms
  constexpr uint32_t kZero = (SC ? 0u : 3u << 9) | (AB ? 0u : 3u << 11);
  block_sum_store<kAcc, kSNT, kZero>(acc, partial_out, lds);
}

}  // namespace it
