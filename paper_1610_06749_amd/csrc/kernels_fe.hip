// Electron phase of the free-electron component (sections "The
// free-electron component" and "Implementation of the free-electron
// models"): one explicit step of the three carriers n+, n-, n_e at the
// electrons' step, each with its own drift and diffusion coefficients (the
// Appendix's scheme), the positive ions recombining with both negative
// carriers (Jacobi: the old densities), plus the per-step tallies.  The
// kernel follows the one-step ion kernel's pipeline: 64 x 8 column tiles
// marching up a chunk of planes, the plane k of the tile (three carriers)
// in a double-buffered LDS plane with one LDS-only barrier per plane, plane
// k+2 of the own column and the rim of plane k+1 requested while plane k is
// computed, registers rotating with period 4 (own column) and 2 (rim).
#include "stencil_plain.h"

namespace it {

namespace {

constexpr int kTX3 = 64, kTY3 = 8, kNT3 = kTX3 * kTY3;

struct Regs3 {
  double v[3];
};

// tally slots: 0 recombined n+ n-, 1 recombined n+ n_e, 2..7 sums of
// n+, n-, n_e on plane 1 and plane nz-1 (anode, cathode per carrier),
// 8..10 in-flight sums, 11..13 sums of |n|
__global__ __launch_bounds__(kNT3) __attribute__((amdgpu_waves_per_eu(4, 8))) void step3_kernel(Step3Params p) {
  if (p.state->e_done) return;
  __shared__ double sl[2][3][kTY3 + 2][kTX3 + 2];
  __shared__ double lds[(kNT3 / kWave) * kAcc3];
  double acc[kAcc3];
#pragma unroll
  for (int q = 0; q < kAcc3; ++q) acc[q] = 0.0;
  const TileCoord t = decode_tile(p.tiles_x, p.tiles_y, p.ntiles, p.per_xcd);
  const int lane = threadIdx.x, ty = threadIdx.y;
  const int x0 = t.tx * kTX3, y0 = t.ty * kTY3;
  const int w = min(kTX3, p.nx - x0), h = min(kTY3, p.ny - y0);
  const bool active = t.valid && lane < w && ty < h;
  const int nz = p.nz;
  const int k0 = 1 + t.zc * p.zc;
  const int k1 = t.valid ? min(k0 + p.zc, nz) : k0;
  const size_t plane = (size_t)p.nx * p.ny;
  const int ic = min(x0 + lane, p.nx - 1), jc = min(y0 + ty, p.ny - 1);
  // in-plane byte offsets (planes hold at most 2^28 nodes, checked on the host)
  const unsigned own = (unsigned)(jc * p.nx + ic) * 8u;
  // rim: waves 0/1 the rows above/below, waves 2/3 the columns left/right
  const int i_left = x0 == 0 ? p.nx - 1 : x0 - 1, i_right = x0 + w == p.nx ? 0 : x0 + w;
  const int j_top = y0 == 0 ? p.ny - 1 : y0 - 1, j_bot = y0 + h == p.ny ? 0 : y0 + h;
  unsigned rim_off = 0;
  int rr = -1, rc = -1;
  if (ty == 0 && lane < w) { rim_off = (unsigned)(j_top * p.nx + x0 + lane) * 8u; rr = 0; rc = lane + 1; }
  if (ty == 1 && lane < w) { rim_off = (unsigned)(j_bot * p.nx + x0 + lane) * 8u; rr = h + 1; rc = lane + 1; }
  if (ty == 2 && lane < h) { rim_off = (unsigned)((y0 + lane) * p.nx + i_left) * 8u; rr = lane + 1; rc = 0; }
  if (ty == 3 && lane < h) { rim_off = (unsigned)((y0 + lane) * p.nx + i_right) * 8u; rr = lane + 1; rc = w + 1; }
  const bool rim = t.valid && rr >= 0;
  const Coef co0 = p.co[0], co1 = p.co[1], co2 = p.co[2];
  const double beta = p.beta;

  auto ld = [&](int s, int k, unsigned off) {
    return *(const __attribute__((address_space(1))) double*)(uniform_ptr(p.in[s] + (size_t)k * plane) + off);
  };
  // One plane.  (m, c, q1): own column at k-1, k, k+1; q2 receives k+2.
  // ra: rim of plane k; rb receives the rim of plane k+1.
  auto plane_step = [&](int k, int buf, const Regs3& m, const Regs3& c, const Regs3& q1, Regs3& q2,
                        const Regs3& ra, Regs3& rb) {
    const int k2 = min(k + 2, nz);  // plane nz exists (the cathode, zero)
#pragma unroll
    for (int s = 0; s < 3; ++s) q2.v[s] = ld(s, k2, own);
    if (rim) {
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        rb.v[s] = ld(s, k + 1, rim_off);
        sl[buf][s][rr][rc] = ra.v[s];
      }
    }
    if (active) {  // inactive threads must not touch the rim slots past the valid extent
#pragma unroll
      for (int s = 0; s < 3; ++s) sl[buf][s][ty + 1][lane + 1] = c.v[s];
    }
    lds_barrier();
    const double sink_n = beta * c.v[0] * c.v[1], sink_e = beta * c.v[0] * c.v[2];
    const double sinks[3] = {sink_n + sink_e, sink_n, sink_e};
    const Coef* cos[3] = {&co0, &co1, &co2};
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const Coef& co = *cos[s];
      const double v = co.a0 * c.v[s] + co.ax * (sl[buf][s][ty + 1][lane] + sl[buf][s][ty + 1][lane + 2]) +
                       co.ay * (sl[buf][s][ty][lane + 1] + sl[buf][s][ty + 2][lane + 1]) + co.azp * q1.v[s] +
                       co.azm * m.v[s] - sinks[s];
      if (active)
        __builtin_nontemporal_store(
            v, (__attribute__((address_space(1))) double*)(uniform_ptr(p.out[s] + (size_t)k * plane) + own));
      // outside the valid extent v comes from unwritten LDS slots (possibly
      // NaN): select it away rather than multiply by zero
      const double va = active ? v : 0.0;
      acc[8 + s] += va;
      acc[11 + s] += fabs(va);
    }
    acc[0] += active ? sink_n : 0.0;
    acc[1] += active ? sink_e : 0.0;
    if (k == 1) {
#pragma unroll
      for (int s = 0; s < 3; ++s) acc[2 + 2 * s] += active ? c.v[s] : 0.0;
    }
    if (k == nz - 1) {
#pragma unroll
      for (int s = 0; s < 3; ++s) acc[3 + 2 * s] += active ? c.v[s] : 0.0;
    }
  };

  Regs3 r0, r1, r2, r3, ra, rb;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    ra.v[s] = rim ? ld(s, k0, rim_off) : 0.0;
    rb.v[s] = 0.0;
    r0.v[s] = ld(s, k0 - 1, own);
    r1.v[s] = ld(s, k0, own);
    r2.v[s] = ld(s, k0 + 1, own);  // k0 + 1 <= nz
  }
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
  block_sum_store<kAcc3, kNT3>(acc, p.partials + (size_t)blockIdx.x * kAcc3, lds);
}

// One block: the step's totals in fixed order, then the run state.  The
// electron phase records no per-step trace; its ion tallies join the run's
// totals, and the deposit's released counts are consumed here (the ion phase
// that follows records no release).
__global__ __launch_bounds__(1024) void reduce3_kernel(Step3Params p, int nblocks) {
  if (p.state->e_done) return;
  __shared__ double tot[kAcc3];
  reduce_partials<1024>(p.partials, nblocks, kAcc3, kAcc3, tot);
  if (threadIdx.x != 0) return;
  RunState st = *p.state;
  const double dV = p.dV;
  const double col[6] = {p.co[0].azp * tot[2] * dV, p.co[0].azm * tot[3] * dV, p.co[1].azp * tot[4] * dV,
                         p.co[1].azm * tot[5] * dV, p.co[2].azp * tot[6] * dV, p.co[2].azm * tot[7] * dV};
  st.sums[0] += tot[0] * dV;
  for (int q = 0; q < 4; ++q) st.sums[1 + q] += col[q];
  st.e_sums[0] += col[4];
  st.e_sums[1] += col[5];
  st.e_sums[2] += tot[1] * dV;
  st.e_left = tot[10] * dV;
  st.released_pending = 0.0;
  st.released_pending_neg = 0.0;
  st.e_steps += 1;
  bool finite = true;
  for (int q = 0; q < kAcc3; ++q) finite = finite && isfinite(tot[q]);
  if (!finite) {
    st.flags |= IT_FLAG_NONFINITE;
    st.e_done = 1;
    st.done = 1;
  } else if (tot[13] * dV <= p.stop_tol * st.released_e) {
    st.e_done = 1;
  }
  *p.state = st;
}

}  // namespace

hipError_t launch_step3(const Step3Params& p, hipStream_t s) {
  const int grid = 8 * p.per_xcd;
  hipLaunchKernelGGL(step3_kernel, dim3(grid), dim3(kTX3, kTY3), 0, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce3_kernel, dim3(1), dim3(1024), 0, s, p, grid);
  return hipGetLastError();
}

}  // namespace it
