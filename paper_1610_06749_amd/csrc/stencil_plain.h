// One explicit time step of both species on one column tile and a chunk of
// planes, with the per-block partial tallies: plain_tile_step (64 x SY or
// 32 x 16 tiles, one column per lane; the single-chamber and the batched
// stepping kernels) and pair_tile_step (128 x SY tiles, two columns per
// lane; single chambers).
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
// 11-12); the instance without it is periodic only.  PU: when add_p and
// add_n are given (block-uniform), a pulse of a pulse train is due at the
// next step: those densities are added to the stored outputs after the
// tallies of this step are taken, and beta times the largest density the
// outputs then hold enters the run's max_beta_n, as a deposit does.
template <int SY, bool SC, bool AB, int TX = kTX, bool PU = false>
__device__ inline void plain_tile_step(const StepParams& p, const TileCoord t, double* partial_out,
                                       const double* add_p = nullptr, const double* add_n = nullptr) {
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
  const bool add = PU && add_p != nullptr;
  double add_max = 0.0;  // largest output density after the pulse is added
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
      double sp_ = vp, sn_ = vn;
      if (add) {  // the pulse due at the next step joins the outputs
        sp_ += ld(uniform_ptr(add_p + o), own);
        sn_ += ld(uniform_ptr(add_n + o), own);
        add_max = fmax(add_max, fmax(sp_, sn_));
      }
      __builtin_nontemporal_store(sp_, (__attribute__((address_space(1))) double*)(uniform_ptr(p.pout + o) + own));
      __builtin_nontemporal_store(sn_, (__attribute__((address_space(1))) double*)(uniform_ptr(p.nout + o) + own));
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
  if (add) {  // block-uniform
    __shared__ double wave_maxima[SY];
    const double m = wave_max(add_max);
    if (lane == 0) wave_maxima[ty] = m;
    __syncthreads();
    if (lane == 0 && ty == 0) {
      double b = wave_maxima[0];
      for (int w = 1; w < SY; ++w) b = fmax(b, wave_maxima[w]);
      const double v = beta * b;
      // non-negative doubles order like their bit patterns
      atomicMax((unsigned long long*)&p.state->max_beta_n,
                (unsigned long long)__double_as_longlong(v > 0.0 ? v : 0.0));
    }
  }
}

// Paired tile: 128 x SY columns with SY waves; lane l of wave r owns the
// two adjacent columns 2l and 2l+1 of row r, so every own-column load, LDS
// access and store moves 16 bytes (a streaming kernel with 16-byte accesses
// runs about 4 % faster on MI355X than with 8-byte ones).  Needs an even nx
// and 16-byte aligned fields (checked on the host): a pair never straddles
// the grid's edge, and a tile's valid width is even.  LDS row layout: column
// c of the tile at index c + 2, the left rim at 1, the right rim at w + 2;
// rows are 132 doubles, so every pair sits on a 16-byte boundary.  The rest
// (pipelining, rim loads by waves 0-3, double-buffered LDS plane, tallies)
// is as in plain_tile_step, and the update of each column is written in the
// same order, so both give the same fields bit for bit.  112 VGPRs without
// the optional terms: four waves per SIMD, twice the 8 waves per CU that the
// default tiling of column pairs places.
typedef double double2_t __attribute__((ext_vector_type(2)));

struct PairRegs {
  double2_t p, n;
};

template <int SY, bool SC, bool AB>
__device__ inline void pair_tile_step(const StepParams& p, const TileCoord t, double* partial_out) {
  constexpr int kSNT = kTX * SY;
  constexpr int TXP = 2 * kTX;        // columns of the tile
  constexpr int kLW = (TXP + 4) / 2;  // LDS row in pairs
  __shared__ double2_t sp[2][SY + 2][kLW], sn[2][SY + 2][kLW];
  __shared__ double lds[(kSNT / kWave) * kAcc];
  __shared__ double edge[SY][4];

  double acc[kAcc];
#pragma unroll
  for (int q = 0; q < kAcc; ++q) acc[q] = 0.0;

  const int lane = threadIdx.x, ty = threadIdx.y;  // ty: the wave and the row
  if (lane < 4) edge[ty][lane] = 0.0;
  const int x0 = t.tx * TXP, y0 = t.ty * SY;
  const int w = min(TXP, p.nx - x0), h = min(SY, p.ny - y0);  // valid extent (w even)
  const int i = x0 + 2 * lane, j = y0 + ty;                    // first column of the pair, row
  const bool active = t.valid && 2 * lane < w && ty < h;
  const int nz = p.nz;
  const int k0 = 1 + t.zc * p.zc;
  const int k1 = t.valid ? min(k0 + p.zc, nz) : k0;
  const size_t plane = (size_t)p.nx * p.ny;
  const int ic = min(i, p.nx - 2), jc = min(j, p.ny - 1);
  const int i_left = x0 == 0 ? p.nx - 1 : x0 - 1;
  const int i_right = x0 + w == p.nx ? 0 : x0 + w;
  const int j_top = y0 == 0 ? p.ny - 1 : y0 - 1;
  const int j_bot = y0 + h == p.ny ? 0 : y0 + h;
  const Coef cp = p.cp, cn = p.cn;
  const double beta = p.beta, gsp = p.gsp, gsn = p.gsn;
  const unsigned own = (unsigned)(jc * p.nx + ic) * 8u;
  // rim element(s) this thread loads: waves 0/1 a pair of the row above /
  // below, waves 2/3 one node of the column left / right
  unsigned rim_off = 0;
  int rim_r = -1, rim_c = -1;  // LDS row and (double) index
  if (ty == 0 && 2 * lane < w) { rim_off = (unsigned)(j_top * p.nx + i) * 8u; rim_r = 0; rim_c = 2 * lane + 2; }
  if (ty == 1 && 2 * lane < w) { rim_off = (unsigned)(j_bot * p.nx + i) * 8u; rim_r = h + 1; rim_c = 2 * lane + 2; }
  if (ty == 2 && lane < h) { rim_off = (unsigned)((y0 + lane) * p.nx + i_left) * 8u; rim_r = lane + 1; rim_c = 1; }
  if (ty == 3 && lane < h) { rim_off = (unsigned)((y0 + lane) * p.nx + i_right) * 8u; rim_r = lane + 1; rim_c = w + 2; }
  const bool rim = t.valid && rim_r >= 0;
  const bool rim_pair = ty < 2;  // wave-uniform
  const bool absorbing = AB && p.absorbing;
  bool rim_outside = false;
  double esc_p0 = 0.0, esc_n0 = 0.0, esc_p1 = 0.0, esc_n1 = 0.0;
  if (absorbing) {
    rim_outside = (ty == 0 && y0 == 0) || (ty == 1 && y0 + h == p.ny) || (ty == 2 && x0 == 0) ||
                  (ty == 3 && x0 + w == p.nx);
    const double my = (double)((j == 0) + (j == p.ny - 1));
    const double mx0 = (double)((i == 0) + (i == p.nx - 1)), mx1 = (double)((i + 1 == p.nx - 1));
    esc_p0 = p.cp.ax * mx0 + p.cp.ay * my;
    esc_n0 = p.cn.ax * mx0 + p.cn.ay * my;
    esc_p1 = p.cp.ax * mx1 + p.cp.ay * my;
    esc_n1 = p.cn.ax * mx1 + p.cn.ay * my;
  }

  auto in_p = [&](int k) { return uniform_ptr(p.pin + (size_t)k * plane); };
  auto in_n = [&](int k) { return uniform_ptr(p.nin + (size_t)k * plane); };
  auto ld = [](const gchar* base, unsigned off) {
    return *(const __attribute__((address_space(1))) double*)(base + off);
  };
  auto ld2 = [](const gchar* base, unsigned off) {
    return *(const __attribute__((address_space(1))) double2_t*)(base + off);
  };
  auto lds_at = [](double2_t (*a)[kLW], int r, int c) -> double& { return ((double*)&a[r][0])[c]; };

  auto plane_step = [&](int k, int buf, const PairRegs& m, const PairRegs& c, const PairRegs& q1, PairRegs& q2,
                        const PairRegs& rc, PairRegs& rn) {
    const int k2 = min(k + 2, nz);
    q2.p = ld2(in_p(k2), own);
    q2.n = ld2(in_n(k2), own);
    if (rim) {
      if (!rim_outside) {
        if (rim_pair) {
          rn.p = ld2(in_p(k + 1), rim_off);
          rn.n = ld2(in_n(k + 1), rim_off);
        } else {
          rn.p.x = ld(in_p(k + 1), rim_off);
          rn.n.x = ld(in_n(k + 1), rim_off);
        }
      }
      if (rim_pair) {
        sp[buf][rim_r][rim_c / 2] = rc.p;
        sn[buf][rim_r][rim_c / 2] = rc.n;
      } else {
        lds_at(sp[buf], rim_r, rim_c) = rc.p.x;
        lds_at(sn[buf], rim_r, rim_c) = rc.n.x;
      }
    }
    if (active) {
      sp[buf][ty + 1][lane + 1] = c.p;
      sn[buf][ty + 1][lane + 1] = c.n;
    }
    lds_barrier();
    // pairs to the left and right (their odd and even member are the x
    // neighbours), above and below
    const double2_t pl = sp[buf][ty + 1][lane], pr = sp[buf][ty + 1][lane + 2];
    const double2_t pu = sp[buf][ty][lane + 1], pd = sp[buf][ty + 2][lane + 1];
    const double2_t nl = sn[buf][ty + 1][lane], nr = sn[buf][ty + 1][lane + 2];
    const double2_t nu = sn[buf][ty][lane + 1], nd = sn[buf][ty + 2][lane + 1];
    const double sink0 = beta * c.p.x * c.n.x, sink1 = beta * c.p.y * c.n.y;
    const double net0 = c.p.x - c.n.x, net1 = c.p.y - c.n.y;
    const double scp0 = SC ? gsp * c.p.x * net0 : 0.0, scn0 = SC ? gsn * c.n.x * net0 : 0.0;
    const double scp1 = SC ? gsp * c.p.y * net1 : 0.0, scn1 = SC ? gsn * c.n.y * net1 : 0.0;
    const double vp0 = cp.a0 * c.p.x + cp.ax * (c.p.y + pl.y) + cp.ay * (pd.x + pu.x) + cp.azp * q1.p.x +
                       cp.azm * m.p.x - sink0 + scp0;
    const double vp1 = cp.a0 * c.p.y + cp.ax * (pr.x + c.p.x) + cp.ay * (pd.y + pu.y) + cp.azp * q1.p.y +
                       cp.azm * m.p.y - sink1 + scp1;
    const double vn0 = cn.a0 * c.n.x + cn.ax * (c.n.y + nl.y) + cn.ay * (nd.x + nu.x) + cn.azp * q1.n.x +
                       cn.azm * m.n.x - sink0 + scn0;
    const double vn1 = cn.a0 * c.n.y + cn.ax * (nr.x + c.n.x) + cn.ay * (nd.y + nu.y) + cn.azp * q1.n.y +
                       cn.azm * m.n.y - sink1 + scn1;
    if (active) {
      const size_t o = (size_t)k * plane;
      const double2_t vp = {vp0, vp1}, vn = {vn0, vn1};
      __builtin_nontemporal_store(vp, (__attribute__((address_space(1))) double2_t*)(uniform_ptr(p.pout + o) + own));
      __builtin_nontemporal_store(vn, (__attribute__((address_space(1))) double2_t*)(uniform_ptr(p.nout + o) + own));
    }
    // inactive threads' values come from LDS slots this block did not
    // write: selected away, never multiplied by zero
    acc[0] += active ? sink0 + sink1 : 0.0;
    acc[5] += active ? vp0 + vp1 : 0.0;
    acc[6] += active ? vn0 + vn1 : 0.0;
    acc[7] += active ? fabs(vp0) + fabs(vp1) : 0.0;
    acc[8] += active ? fabs(vn0) + fabs(vn1) : 0.0;
    if (SC) {
      acc[9] += active ? scp0 + scp1 : 0.0;
      acc[10] += active ? scn0 + scn1 : 0.0;
    }
    if (AB) {
      acc[11] += active ? esc_p0 * c.p.x + esc_p1 * c.p.y : 0.0;
      acc[12] += active ? esc_n0 * c.n.x + esc_n1 * c.n.y : 0.0;
    }
    if (k == 1 || k == nz - 1) {  // uniform over the block
      const double sp_ = wave_sum(active ? c.p.x + c.p.y : 0.0), sn_ = wave_sum(active ? c.n.x + c.n.y : 0.0);
      if (lane == 0) {
        if (k == 1) {
          edge[ty][0] += sp_;
          edge[ty][2] += sn_;
        }
        if (k == nz - 1) {
          edge[ty][1] += sp_;
          edge[ty][3] += sn_;
        }
      }
    }
  };

  PairRegs r0, r1, r2, r3, ra, rb;
  ra.p = ra.n = rb.p = rb.n = double2_t{0.0, 0.0};
  if (rim && !rim_outside) {
    if (rim_pair) {
      ra.p = ld2(in_p(k0), rim_off);
      ra.n = ld2(in_n(k0), rim_off);
    } else {
      ra.p.x = ld(in_p(k0), rim_off);
      ra.n.x = ld(in_n(k0), rim_off);
    }
  }
  r0.p = ld2(in_p(k0 - 1), own);
  r0.n = ld2(in_n(k0 - 1), own);
  r1.p = ld2(in_p(k0), own);
  r1.n = ld2(in_n(k0), own);
  r2.p = ld2(in_p(k0 + 1), own);
  r2.n = ld2(in_n(k0 + 1), own);
  for (int k = k0; k < k1; k += 4) {
    plane_step(k, 0, r0, r1, r2, r3, ra, rb);
    if (k + 1 >= k1) break;
    plane_step(k + 1, 1, r1, r2, r3, r0, rb, ra);
    if (k + 2 >= k1) break;
    plane_step(k + 2, 0, r2, r3, r0, r1, ra, rb);
    if (k + 3 >= k1) break;
    plane_step(k + 3, 1, r3, r0, r1, r2, rb, ra);
  }

  __syncthreads();
  if (lane == 0) {
    acc[1] = edge[ty][0];
    acc[2] = edge[ty][1];
    acc[3] = edge[ty][2];
    acc[4] = edge[ty][3];
  }
  constexpr uint32_t kZero = (SC ? 0u : 3u << 9) | (AB ? 0u : 3u << 11);
  block_sum_store<kAcc, kSNT, kZero>(acc, partial_out, lds);
}

}  // namespace it
