// One temporally blocked pass (T explicit time steps) of one block over one
// extended tile: the device code shared by the single-chamber blocked
// kernel and the batched one.
//
// A block of 8 waves owns an extended tile of 64 columns by 8 R rows: lane l
// holds column l, and wave w the R consecutive rows w R .. w R + R - 1, in
// registers.  Every lane loads its periodically wrapped column, so lane and
// row neighbours are always the periodic x and y neighbours.  Each of the T
// steps (levels) is exact on one node less on every side, so after T steps
// the centre (64 - 2T) x (8 R - 2T) columns are exact: the block's owned
// columns.  The block marches up a chunk of planes with a software pipeline
// over the levels: at iteration K it has level 0 on plane K (loaded one or
// two iterations ahead) and computes level t on plane K - t for t = 1..T
// from level t-1 on planes K-t-1, K-t and K-t+1, which the thread keeps in
// registers (per level the current plane and a_{z-} times the one below it,
// plus the plane just computed).
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
// of planes only, so every node and electrode face is counted once.
#pragma once

#include "stencil_plain.h"

namespace it {

constexpr int kBW = 8;                // waves per block
constexpr int kBX = 64;               // columns of the extended tile
constexpr int kBNT = kBW * kWave;     // threads per block

typedef __attribute__((address_space(1))) double gdouble;

// Block b of a blocked launch of 8 per_xcd blocks -> its entry in the tile
// list.  A blocked block fills a CU, so a launch runs in rounds of 256
// blocks, 32 per XCD (the dispatcher deals blocks to the 8 XCDs in turn).
// Round r takes the 256 consecutive tiles from 256 r, XCD x the x-th run of
// them: each XCD works on a compact patch of lateral neighbours (their rims
// meet in its L2), and the patches of a round are neighbours too, so the
// rims between them are read by two XCDs at about the same time.  (Giving
// each XCD one contiguous run of the whole list instead put the XCDs on
// unrelated patches and took 2.7 % longer on the 512 x 512 x 256 grid.)
__device__ inline int blocked_tile_index(int b, int per_xcd) {
  constexpr int kXcds = 8, kCusPerXcd = 32;
  const int x = b % kXcds, j = b / kXcds;
  const int r = j / kCusPerXcd, within = j % kCusPerXcd;
  const int run = min(kCusPerXcd, per_xcd - kCusPerXcd * r);  // tiles per XCD in this round
  return kXcds * kCusPerXcd * r + run * x + within;
}

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

// One pass of the block over tile tc (tc.valid false: an idle block, which
// still stores zero partials); the block's T records of kAcc partial
// tallies go to partial_out.  The caller has checked the run's stop flag.
// PU: with add_j in 1..T (block-uniform), a pulse of a pulse train falls due
// after the step of level add_j: the densities add_p and add_n join that
// level's outputs once its tallies are taken (on every node the tile
// computes but those beyond an absorbing boundary, so the later levels step
// from them), and beta times the largest owned output enters the run's
// max_beta_n, as a deposit does.
// AB: honours p.absorbing (absorbing lateral boundaries; a batch mixes both
// kinds): the tile's nodes beyond the cell hold zero at every level
// instead of the periodic image, and each owned node next to the boundary
// adds a_x (a_y) times its old density per missing neighbour to the escaped
// tally of its species, as in the one-step kernel.
template <int T, int R, bool SC, bool PU = false, bool AB = false>
__device__ __forceinline__ void blocked_tile_pass(const StepParams& p, const TileCoord tc, double* partial_out,
                                                  int add_j = 0, const double* add_p = nullptr,
                                                  const double* add_n = nullptr) {
  constexpr int EY = kBW * R;             // rows of the extended tile
  constexpr int OX = kBX - 2 * T, OY = EY - 2 * T;
  constexpr int NE = SC ? 7 : 5;          // index of the escaped tallies (AB)
  constexpr int NA = NE + (AB ? 2 : 0);   // tallies kept per level
  // edge rows of each level's newest plane: [buffer][level][wave][first/last][species][lane]
  __shared__ double edge_rows[2][T][kBW][2][2][kWave];
  __shared__ double edge_sum[T][kBW][4];  // per-wave sums of n on the planes next to the electrodes
  __shared__ double lds[(kBNT / kWave) * kAcc * T];

  const int lane = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);  // the wave (uniform)
  const int x0 = tc.tx * OX, y0 = tc.ty * OY;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  // wrapped position of this lane's column and of the thread's rows
  int xs = (x0 - T + lane) % nx;
  if (xs < 0) xs += nx;
  const bool own_x = lane >= T && lane < kBX - T && x0 + (lane - T) < nx;
  unsigned off[R];  // in-plane byte offsets of the thread's nodes
  bool own_y[R];    // the row is owned (wave-uniform)
  // absorbing: the node lies in the cell (else it holds zero), and the
  // missing neighbours of the lane's column and of each row
  const bool absorbing = AB && p.absorbing;
  const int gx = x0 - T + lane;
  const bool in_x = !absorbing || (gx >= 0 && gx < nx);
  const double miss_x = absorbing ? (double)((gx == 0) + (gx == nx - 1)) : 0.0;
  bool in_y[R];
  double miss_y[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int g = w * R + r;  // row in the extended tile
    int ys = (y0 - T + g) % ny;
    if (ys < 0) ys += ny;
    off[r] = (unsigned)(ys * nx + xs) * 8u;
    own_y[r] = tc.valid && g >= T && g < EY - T && y0 + (g - T) < ny;
    const int gy = y0 - T + g;
    in_y[r] = !absorbing || (gy >= 0 && gy < ny);
    miss_y[r] = absorbing ? (double)((gy == 0) + (gy == ny - 1)) : 0.0;
  }
  const int za = 1 + tc.zc * p.zc;
  const int zb = tc.valid ? min(za + p.zc, nz) : za;
  const size_t plane = (size_t)nx * ny;
  const Coef cp = p.cp, cn = p.cn;
  const double beta = p.beta, gsp = p.gsp, gsn = p.gsn;
  double add_max = 0.0;  // largest owned output density after a pulse is added

  if (lane < 4)
#pragma unroll
    for (int t = 0; t < T; ++t) edge_sum[t][w][lane] = 0.0;

  // level t (0..T-1) at the start of iteration K: cpv/cnv its plane K-t-1,
  // mp/mn the lower z-neighbour term of the next step's update on that plane,
  // a_{z-} times its plane K-t-2 (kept instead of the plane itself, so the
  // march shifts one register pair less per node, level and species)
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
  // Level 0 of plane K into (lp, ln).  Planes before the anode and beyond the
  // cathode read the electrode plane itself, which always holds zero: the
  // loads need no branch or select, so they stay in flight across the
  // iteration (a branch around them made the compiler wait for them at once).
  // Where the registers allow (T R <= 12 and R <= 4: the default rows at
  // T = 3 and 4, and T = 2 passes cut short in such runs), two buffers
  // alternate and each plane is loaded two iterations ahead, the march taking
  // two iterations per loop trip (1 % faster on the 512 x 512 x 256 grid, 2 %
  // on the 96-chamber sweep); otherwise one buffer, one plane ahead.
  constexpr bool kTwoBuffers = T * R <= 12 && R <= 4 && !AB;
  constexpr int kAhead = kTwoBuffers ? 2 : 1;
  double pa[R], na[R], pb[R], nb[R];
  auto load0 = [&](int K, double (&lp)[R], double (&ln)[R]) {
    const int Kc = min(max(K, 0), nz);
    const gchar* bp = uniform_ptr(p.pin + (size_t)Kc * plane);
    const gchar* bn = uniform_ptr(p.nin + (size_t)Kc * plane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      lp[r] = *(const gdouble*)(bp + off[r]);
      ln[r] = *(const gdouble*)(bn + off[r]);
      if (AB && !(in_x && in_y[r])) lp[r] = ln[r] = 0.0;  // beyond an absorbing boundary
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
  // every level's newest plane for the next iteration; level 0 of plane K
  // comes from (lp, ln), which then take the plane kAhead further (with two
  // buffers, past the chunk's last plane a clamped plane, unused).
  auto iterate = [&](int K, double (&lp)[R], double (&ln)[R]) {
    const int buf = K & 1;
    lds_barrier();  // the edge rows written at the end of the previous iteration
    double vp[R], vn[R];  // the newest level's values, plane K - t
#pragma unroll
    for (int r = 0; r < R; ++r) {
      vp[r] = lp[r];
      vn[r] = ln[r];
    }
    if (kTwoBuffers || K + 1 <= Khi) load0(K + kAhead, lp, ln);
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
      for (int i = 0; i < R; ++i) {
        const int r = (i + 1) % R;  // the strip's first row last: its upper neighbour comes from LDS
        const double pc = cpv[t - 1][r], nc = cnv[t - 1][r];
        const double pxl = lane_from_left(pc), pxr = lane_from_right(pc);
        const double nxl = lane_from_left(nc), nxr = lane_from_right(nc);
        const double pyl = r > 0 ? cpv[t - 1][r - 1] : up_p, pyr = r < R - 1 ? cpv[t - 1][r + 1] : dn_p;
        const double nyl = r > 0 ? cnv[t - 1][r - 1] : up_n, nyr = r < R - 1 ? cnv[t - 1][r + 1] : dn_n;
        const double sink = beta * pc * nc;
        const double net = pc - nc;
        const double scp = SC ? gsp * pc * net : 0.0, scn = SC ? gsn * nc * net : 0.0;
        double a = mp[t - 1][r] + cp.a0 * pc + cp.ax * (pxr + pxl) + cp.ay * (pyr + pyl) + cp.azp * vp[r] - sink;
        double b = mn[t - 1][r] + cn.a0 * nc + cn.ax * (nxr + nxl) + cn.ay * (nyr + nyl) + cn.azp * vn[r] - sink;
        if constexpr (SC) {  // (not "+ 0.0" without it: x + 0 is not folded away, as -0 + 0 = +0)
          a += scp;
          b += scn;
        }
        if (AB && !(in_x && in_y[r])) a = b = 0.0;  // beyond an absorbing boundary
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
          if constexpr (AB) {
            acc[t - 1][NE] += (cp.ax * miss_x + cp.ay * miss_y[r]) * pc;
            acc[t - 1][NE + 1] += (cn.ax * miss_x + cn.ay * miss_y[r]) * nc;
          }
        }
      }
      if (PU && t == add_j && interior) {  // block-uniform: the pulse due after this level's step
        const gchar* pp = uniform_ptr(add_p + (size_t)q * plane);
        const gchar* pn = uniform_ptr(add_n + (size_t)q * plane);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (AB && !(in_x && in_y[r])) continue;  // beyond an absorbing boundary: stays zero
          np[r] += *(const gdouble*)(pp + off[r]);
          nn[r] += *(const gdouble*)(pn + off[r]);
          if (counted && own_y[r] && own_x) add_max = fmax(add_max, fmax(np[r], nn[r]));
        }
      }
      // level t-1 moves on: plane K-t gives the lower-neighbour term, K-t+1
      // becomes its current plane
#pragma unroll
      for (int r = 0; r < R; ++r) {
        mp[t - 1][r] = cp.azm * cpv[t - 1][r];
        mn[t - 1][r] = cn.azm * cnv[t - 1][r];
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
    load0(Klo, pa, na);
    if constexpr (kTwoBuffers) {
      load0(Klo + 1, pb, nb);
      int K = Klo;
      for (; K + 1 <= Khi; K += 2) {
        iterate(K, pa, na);
        iterate(K + 1, pb, nb);
      }
      if (K <= Khi) iterate(K, pa, na);
    } else {
      for (int K = Klo; K <= Khi; ++K) iterate(K, pa, na);
    }
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
    if constexpr (AB) {  // escaped (absorbing boundaries)
      a[t * kAcc + 11] = own_x ? acc[t][NE] : 0.0;
      a[t * kAcc + 12] = own_x ? acc[t][NE + 1] : 0.0;
    } else {
      a[t * kAcc + 11] = 0.0;
      a[t * kAcc + 12] = 0.0;
    }
  }
  block_sum_store<kAcc * T, kBNT>(a, partial_out, lds);
  if (PU && add_j > 0) {  // block-uniform
    __shared__ double wave_maxima[kBW];
    const double m = wave_max(add_max);
    if (lane == 0) wave_maxima[w] = m;
    __syncthreads();
    if (lane == 0 && w == 0) {
      double b = wave_maxima[0];
      for (int i = 1; i < kBW; ++i) b = fmax(b, wave_maxima[i]);
      const double v = beta * b;
      // non-negative doubles order like their bit patterns
      atomicMax((unsigned long long*)&p.state->max_beta_n,
                (unsigned long long)__double_as_longlong(v > 0.0 ? v : 0.0));
    }
  }
}


}  // namespace it
