// Plain one-step stencil kernel and the track deposition kernel (gfx950).
//
// Step kernel: one explicit time step of both ion species (eq. theEquation
// with the Appendix's difference scheme, written as per-node coefficients),
// plus the per-step tallies.  Each block owns a 64 x 4 column tile of the
// transverse plane and a chunk of z planes; each thread owns one column and
// marches up the chunk keeping n_{k-1}, n_k, n_{k+1} of both species in
// registers, so every interior value is read once as a column centre (64
// lanes = 512 contiguous bytes per wave) and its lateral neighbours come
// from L1/L2.  No MFMA: the update is a 7-point stencil, not a contraction,
// and the kernel is bound by HBM bandwidth (32 bytes per node and step).
#include "reduce.h"

namespace it {

constexpr int kTX = 64, kTY = 4, kNT = kTX * kTY;

__global__ __launch_bounds__(kNT) void step_plain_kernel(StepParams p) {
  if (p.state->done) return;  // set by an earlier launch: every block skips
  __shared__ double lds[(kNT / kWave) * kAcc];
  __shared__ double totals[kAcc];

  double acc[kAcc];
#pragma unroll
  for (int q = 0; q < kAcc; ++q) acc[q] = 0.0;

  const TileCoord t = decode_tile(p.tiles_x, p.zchunks, p.ntiles, p.per_xcd);
  const int i = t.tx * kTX + threadIdx.x;
  const int j = t.ty * kTY + threadIdx.y;
  if (t.valid && i < p.nx && j < p.ny) {
    const int k0 = 1 + t.zc * p.zc;
    const int k1 = min(k0 + p.zc, p.nz);
    const size_t plane = (size_t)p.nx * p.ny;
    const long dxp = (i + 1 == p.nx) ? -(long)i : 1;
    const long dxm = (i == 0) ? (long)(p.nx - 1) : -1;
    const long dyp = ((j + 1 == p.ny) ? -(long)j : 1) * (long)p.nx;
    const long dym = ((j == 0) ? (long)(p.ny - 1) : -1) * (long)p.nx;
    const double* __restrict__ pin = p.pin;
    const double* __restrict__ nin = p.nin;
    double* __restrict__ pout = p.pout;
    double* __restrict__ nout = p.nout;
    size_t c = (size_t)k0 * plane + (size_t)j * p.nx + i;
    double pm = pin[c - plane], pc = pin[c];
    double nm = nin[c - plane], nc = nin[c];
    const Coef cp = p.cp, cn = p.cn;
    const double beta = p.beta;
    for (int k = k0; k < k1; ++k) {
      const double pp = pin[c + plane], np = nin[c + plane];
      const double pl = pin[c + dxp] + pin[c + dxm];
      const double pt = pin[c + dyp] + pin[c + dym];
      const double nl = nin[c + dxp] + nin[c + dxm];
      const double nt = nin[c + dyp] + nin[c + dym];
      const double sink = beta * pc * nc;
      const double vp = cp.a0 * pc + cp.ax * pl + cp.ay * pt + cp.azp * pp + cp.azm * pm - sink;
      const double vn = cn.a0 * nc + cn.ax * nl + cn.ay * nt + cn.azp * np + cn.azm * nm - sink;
      pout[c] = vp;
      nout[c] = vn;
      acc[0] += sink;
      if (k == 1) {
        acc[1] += pc;
        acc[3] += nc;
      }
      if (k == p.nz - 1) {
        acc[2] += pc;
        acc[4] += nc;
      }
      acc[5] += vp;
      acc[6] += vn;
      acc[7] += fabs(vp);
      acc[8] += fabs(vn);
      pm = pc;
      pc = pp;
      nm = nc;
      nc = np;
      c += plane;
    }
  }

  block_sum_store<kAcc, kNT>(acc, p.partials + (size_t)blockIdx.x * kAcc, lds);
  if (!arrive_last<kNT>(p.counter)) return;
  reduce_partials<kNT>(p.partials, gridDim.x, kAcc, kAcc, totals, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    finalize_steps(p.state, p.trace, totals, 1, p.step0, p.cp, p.cn, p.dV, p.stop_tol,
                   p.min_stop_step);
    *p.counter = 0u;
  }
}

hipError_t launch_step_plain(const StepParams& p, hipStream_t s) {
  const int grid = 8 * p.per_xcd;
  hipLaunchKernelGGL(step_plain_kernel, dim3(grid), dim3(kTX, kTY), 0, s, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deposition (eq. Gaussian around each track axis, eq. linear_density for N0).
// Each thread owns one transverse column of a tile and a chunk of planes.
// Tracks parallel to the field give the same density on every plane, so
// their sum is formed once per column; tilted tracks are evaluated per node.
// The perpendicular distance is |w x u| with w the node's offset from the
// axis point (x0, y0, d/2), its transverse part wrapped to the nearest
// periodic image; the profile is cut at r^2 > (8 b)^2.
// ---------------------------------------------------------------------------

__device__ inline double wrap_near(double d, double L) { return d - L * floor(d / L + 0.5); }

__device__ inline double track_value(const DepTrack& tr, double wx, double wy, double wz) {
  const double cx = wy * tr.uz - wz * tr.uy;
  const double cy = wz * tr.ux - wx * tr.uz;
  const double cz = wx * tr.uy - wy * tr.ux;
  const double r2 = cx * cx + cy * cy + cz * cz;
  return r2 > tr.cut2 ? 0.0 : tr.peak * exp(-r2 * tr.inv_b2);
}

__global__ __launch_bounds__(kNT) void deposit_kernel(DepositParams p) {
  __shared__ double lds[(kNT / kWave) * 2];
  __shared__ double totals[2];
  double sum = 0.0, mx = 0.0;
  const TileCoord t = decode_tile(p.tiles_x, p.zchunks, p.ntiles, p.per_xcd);
  const int i = t.tx * kTX + threadIdx.x;
  const int j = t.ty * kTY + threadIdx.y;
  if (t.valid && i < p.nx && j < p.ny) {
    const int k0 = 1 + t.zc * p.zc;
    const int k1 = min(k0 + p.zc, p.nz);
    const double x = i * p.dx, y = j * p.dy;
    double g0 = p.uniform;
    for (int q = 0; q < p.npar; ++q) {
      const DepTrack tr = p.par[q];
      g0 += track_value(tr, wrap_near(x - tr.x0, p.Lx), wrap_near(y - tr.y0, p.Ly), 0.0);
    }
    const size_t plane = (size_t)p.nx * p.ny;
    size_t c = (size_t)k0 * plane + (size_t)j * p.nx + i;
    for (int k = k0; k < k1; ++k, c += plane) {
      double d = g0;
      if (p.ntilt) {
        const double wz = k * p.dz - p.half_gap;
        for (int q = 0; q < p.ntilt; ++q) {
          const DepTrack tr = p.tilt[q];
          d += track_value(tr, wrap_near(x - tr.x0, p.Lx), wrap_near(y - tr.y0, p.Ly), wz);
        }
      }
      const double a = p.pos[c] + d, b = p.neg[c] + d;
      p.pos[c] = a;
      p.neg[c] = b;
      sum += d;
      mx = fmax(mx, fmax(a, b));
    }
  }
  // block partials: [sum, max]
  {
    double s = wave_sum(sum), m = wave_max(mx);
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    if (tid % kWave == 0) {
      lds[(tid / kWave) * 2] = s;
      lds[(tid / kWave) * 2 + 1] = m;
    }
    __syncthreads();
    if (tid == 0) {
      double ss = lds[0], mm = lds[1];
      for (int w = 1; w < kNT / kWave; ++w) {
        ss += lds[w * 2];
        mm = fmax(mm, lds[w * 2 + 1]);
      }
      p.partials[(size_t)blockIdx.x * 2] = ss;
      p.partials[(size_t)blockIdx.x * 2 + 1] = mm;
    }
  }
  if (!arrive_last<kNT>(p.counter)) return;
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  {
    double s = 0.0, m = 0.0;
    for (int b = tid; b < (int)gridDim.x; b += kNT) {
      s += p.partials[(size_t)b * 2];
      m = fmax(m, p.partials[(size_t)b * 2 + 1]);
    }
    s = wave_sum(s);
    m = wave_max(m);
    __syncthreads();
    if (tid % kWave == 0) {
      lds[(tid / kWave) * 2] = s;
      lds[(tid / kWave) * 2 + 1] = m;
    }
    __syncthreads();
    if (tid == 0) {
      double ss = lds[0], mm = lds[1];
      for (int w = 1; w < kNT / kWave; ++w) {
        ss += lds[w * 2];
        mm = fmax(mm, lds[w * 2 + 1]);
      }
      totals[0] = ss;
      totals[1] = mm;
      RunState* st = p.state;
      const double rel = ss * p.dV;
      st->released += rel;
      st->released_pending += rel;
      st->max_beta_n = fmax(st->max_beta_n, p.beta * mm);
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
