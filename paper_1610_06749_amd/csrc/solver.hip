// Host side of the C ABI: validation, time step, coefficients, workspace
// layout, the deposit schedule and the stepping loop with its stop checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace it {

// Temporally blocked kernel (kernels_blocked.hip): T steps per pass on
// tiles of 64 columns by 8 R rows (R rows per thread).
hipError_t launch_step_blocked(const StepParams& p, int T, int R, hipStream_t s, hipEvent_t ev_begin,
                               hipEvent_t ev_end, int* nblocks);
int blocked_supported(int T, int tile_y);
int blocked_rows(int T, int tile_y);
void blocked_tiling(int nx, int ny, int nz, int T, int R, int* grid, int* per_xcd,
                    int* tiles_x, int* tiles_y, int* ntiles, int* zc, int* zchunks);
void blocked_tiling_zc(int nx, int ny, int nz, int T, int R, int zc, int* tiles_x, int* tiles_y, int* ntiles,
                       int* zc_out, int* zchunks_out);

namespace {

constexpr size_t kAlign = 256;
constexpr int kBlockedT = 3;                // steps per pass of the blocked kernel when none is given
constexpr double kBlockedMinNodes = 4.0e6;  // interior nodes from which the library chooses it

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

constexpr int32_t kMaxPulses = 1 << 20;  // pulses of a pulse train

int check_chamber(const it_chamber* ch) {
  if (!ch) return IT_EINVAL;
  if (ch->nx < 1 || ch->ny < 1 || ch->nz < 2) return IT_EINVAL;
  if (ch->space_charge != 0 && ch->space_charge != 1) return IT_EINVAL;
  if (ch->lateral_bc != 0 && ch->lateral_bc != 1) return IT_EINVAL;
  const double cells = (double)ch->nx * ch->ny * (double)(ch->nz + 1);
  if (cells > 4.0e9) return IT_EINVAL;  // 32-bit tile indices and 64-bit offsets suffice below
  if ((double)ch->nx * ch->ny > (double)(1 << 28)) return IT_EINVAL;  // in-plane byte offsets fit 32 bits
  if (!(std::isfinite(ch->dx) && ch->dx > 0 && std::isfinite(ch->dy) && ch->dy > 0)) return IT_EINVAL;
  if (!(std::isfinite(ch->gap) && ch->gap > 0)) return IT_EINVAL;
  if (!std::isfinite(ch->voltage)) return IT_EINVAL;
  if (!finite_nonneg(ch->mu_pos) || !finite_nonneg(ch->mu_neg)) return IT_EINVAL;
  if (!finite_nonneg(ch->D_pos) || !finite_nonneg(ch->D_neg)) return IT_EINVAL;
  if (!finite_nonneg(ch->alpha)) return IT_EINVAL;
  if (!(std::isfinite(ch->W_eV) && ch->W_eV > 0)) return IT_EINVAL;
  if (!(std::isfinite(ch->dt_safety) && ch->dt_safety > 0 && ch->dt_safety <= 1.0)) return IT_EINVAL;
  if (!finite_nonneg(ch->stop_tol) || !finite_nonneg(ch->uniform_n0)) return IT_EINVAL;
  if (!finite_nonneg(ch->reaction_limit)) return IT_EINVAL;
  if (!finite_nonneg(ch->attach_coeff) || !finite_nonneg(ch->mu_e) || !finite_nonneg(ch->D_e)) return IT_EINVAL;
  if (ch->max_steps < 1) return IT_EINVAL;
  if (ch->n_pulses < 0 || ch->n_pulses > kMaxPulses) return IT_EINVAL;
  if (ch->n_pulses >= 2 && !(std::isfinite(ch->pulse_period_s) && ch->pulse_period_s > 0)) return IT_EINVAL;
  return IT_OK;
}

// Largest dt with 2(sx+sy+sz) + c^2 <= 1 for each species (eq. vNeum with
// the field along z; the product condition then holds for any dt).
double transport_dt(const it_chamber* ch) {
  const double dz = ch->gap / ch->nz;
  const double E = ch->voltage / ch->gap;
  const double h = 1.0 / (ch->dx * ch->dx) + 1.0 / (ch->dy * ch->dy) + 1.0 / (dz * dz);
  double best = INFINITY;
  const double mu[2] = {ch->mu_pos, ch->mu_neg}, D[2] = {ch->D_pos, ch->D_neg};
  for (int s = 0; s < 2; ++s) {
    const double a = 2.0 * D[s] * h;          // diffusion part, per unit dt
    const double vz = mu[s] * E / dz;
    const double b = vz * vz;                 // drift part, per unit dt^2
    double root;
    if (b > 0.0)
      root = 2.0 / (a + std::sqrt(a * a + 4.0 * b));
    else if (a > 0.0)
      root = 1.0 / a;
    else
      continue;
    best = std::min(best, root);
  }
  return best;
}

double wrap_near_host(double d, double L) { return d - L * std::floor(d / L + 0.5); }

// Reference density of the recombination bound: uniform_n0 plus the largest
// sum, over the tracks arriving together, of their Gaussian profiles at one
// of their axis points (x0, y0, d/2).
double reference_density(const it_chamber* ch, const it_track* tr, int64_t n) {
  const double Lx = ch->nx * ch->dx, Ly = ch->ny * ch->dy;
  double best = 0.0;
  for (int64_t a = 0; a < n; ++a) {
    double s[2] = {0.0, 0.0};
    for (int64_t q = 0; q < n; ++q) {
      const it_track& t = tr[q];
      if (t.t_s != tr[a].t_s) continue;
      const double ux = std::sin(t.theta) * std::cos(t.phi);
      const double uy = std::sin(t.theta) * std::sin(t.phi);
      const double uz = std::cos(t.theta);
      const double dx = tr[a].x_cm - t.x_cm, dy = tr[a].y_cm - t.y_cm;
      const double wx = ch->lateral_bc ? dx : wrap_near_host(dx, Lx);
      const double wy = ch->lateral_bc ? dy : wrap_near_host(dy, Ly);
      const double wz = 0.0;
      const double cx = wy * uz - wz * uy, cy = wz * ux - wx * uz, cz = wx * uy - wy * ux;
      const double r2 = cx * cx + cy * cy + cz * cz;
      for (int sp = 0; sp < 2; ++sp) {  // both species' radii
        const double b = sp == 1 && t.b_neg_cm > 0.0 ? t.b_neg_cm : t.b_cm;
        const double b2 = b * b;
        if (r2 > 64.0 * b2) continue;
        s[sp] += t.let_keV_um * 1.0e7 / ch->W_eV / (M_PI * b2) * std::exp(-r2 / b2);
      }
    }
    best = std::max(best, std::max(s[0], s[1]));
  }
  return ch->uniform_n0 + best;
}

// Rate constant of the explicit pointwise terms: recombination, plus the
// space-charge screening mu q/eps0 (the dielectric relaxation rate per unit
// density) when that term is on.
double pointwise_rate(const it_chamber* ch) {
  double k = ch->alpha;
  if (ch->space_charge) k += std::max(ch->mu_pos, ch->mu_neg) * kElementaryCharge / kEpsilon0;
  return k;
}

// Space-charge coefficients of species s as they enter the update.
double screening_coef(const it_chamber* ch, double dt, int s) {
  if (!ch->space_charge) return 0.0;
  const double g = dt * kElementaryCharge / kEpsilon0;
  return s == 0 ? -ch->mu_pos * g : ch->mu_neg * g;
}

// The run's time step; with a pulse train, also the steps per period
// (period_steps, may be null; 0 without a train): the single-pulse step is
// shortened so that a period is a whole number of steps.
int compute_dt(const it_chamber* ch, const it_track* tr, int64_t n, double* dt, int64_t* period_steps = nullptr) {
  double best = transport_dt(ch);
  const double rate = pointwise_rate(ch);
  if (ch->reaction_limit > 0.0 && rate > 0.0) {
    const double nref = reference_density(ch, tr, n);
    if (nref > 0.0) best = std::min(best, ch->reaction_limit / (rate * nref));
  }
  if (!(best < INFINITY)) return IT_ENODT;
  *dt = ch->dt_safety * best;
  if (period_steps) *period_steps = 0;
  if (ch->n_pulses >= 2) {
    const double per = std::ceil(ch->pulse_period_s / *dt);
    if (!(per <= 1.0e15 / (double)ch->n_pulses)) return IT_EINVAL;  // steps of the train out of range
    *dt = ch->pulse_period_s / per;
    if (period_steps) *period_steps = (int64_t)per;
  }
  return IT_OK;
}

// A pulse train repeats one instantaneous pulse: every track due at t = 0,
// and no free electrons.
int check_train(const it_chamber* ch, const it_track* tr, int64_t n) {
  if (ch->n_pulses < 2) return IT_OK;
  if (ch->mu_e > 0.0) return IT_ENOTSUP;
  for (int64_t q = 0; q < n; ++q)
    if (tr[q].t_s != 0.0) return IT_ENOTSUP;
  return IT_OK;
}

// Per-species update coefficients (see Coef).  c is signed with the drift
// velocity: +mu+ E for positive ions (towards the cathode at z = d), -mu- E
// for negative ions.  With a signed c the Appendix's blended drift
// derivative gives the Lax-Wendroff weights below.
// Coefficients of a carrier with signed mobility mu_s (+ for positive
// carriers, which drift towards the cathode) and diffusion constant D.
Coef carrier_coef(const it_chamber* ch, double dt, double mu_s, double D) {
  const double dz = ch->gap / ch->nz;
  const double E = ch->voltage / ch->gap;
  const double c = mu_s * E * dt / dz;
  const double sx = D * dt / (ch->dx * ch->dx);
  const double sy = D * dt / (ch->dy * ch->dy);
  const double sz = D * dt / (dz * dz);
  Coef k;
  k.ax = sx;
  k.ay = sy;
  k.azp = sz + 0.5 * c * c - 0.5 * c;
  k.azm = sz + 0.5 * c * c + 0.5 * c;
  k.a0 = 1.0 - 2.0 * (sx + sy + sz) - c * c;
  return k;
}

Coef species_coef(const it_chamber* ch, double dt, int s) {
  return s == 0 ? carrier_coef(ch, dt, ch->mu_pos, ch->D_pos) : carrier_coef(ch, dt, -ch->mu_neg, ch->D_neg);
}

// Largest dt of eq. vNeum for the free electrons (field along z).
double electron_dt(const it_chamber* ch) {
  const double dz = ch->gap / ch->nz;
  const double E = ch->voltage / ch->gap;
  const double A = 2.0 * ch->D_e * (1.0 / (ch->dx * ch->dx) + 1.0 / (ch->dy * ch->dy) + 1.0 / (dz * dz));
  const double v = ch->mu_e * E / dz;
  const double B = v * v;
  if (B > 0.0) return 2.0 / (A + std::sqrt(A * A + 4.0 * B));
  if (A > 0.0) return 1.0 / A;
  return INFINITY;
}

// p of eq. free_elec
double free_fraction(double a, double d) {
  const double x = a * d;
  return x == 0.0 ? 1.0 : -std::expm1(-x) / x;
}

struct Tiling {
  int tiles_x, tiles_y, zchunks, zc, ntiles, per_xcd, grid;
};

// Tiling of the interior: tile_x x tile_y columns by chunks of z planes.
// The stepping kernel marches 32 planes per block (down to 4 on small grids,
// to keep several hundred blocks); the deposit kernel aims at ~2048 blocks.
Tiling make_tiling(int nx, int ny, int nz, int tile_y, int zc, int tile_x = 64) {
  Tiling t;
  const int nint = nz - 1;
  t.tiles_x = (nx + tile_x - 1) / tile_x;
  t.tiles_y = (ny + tile_y - 1) / tile_y;
  const long cols = (long)t.tiles_x * t.tiles_y;
  t.zc = std::max(1, std::min(zc, nint));
  t.zchunks = (nint + t.zc - 1) / t.zc;
  t.ntiles = (int)(cols * t.zchunks);
  t.per_xcd = (t.ntiles + 7) / 8;
  t.grid = 8 * t.per_xcd;
  return t;
}

// z_chunk > 0: planes per tile as requested.  0: split every column into
// equal chunks so that the grid holds about 16 waves per CU (4096 waves on
// 256 CUs), all resident at once: the launch then takes as long as one
// chunk, so chunks of equal length and as few chunk starts (each re-reads
// two planes) as the occupancy allows are what count.
// Tiles of column pairs (tile_x 128) have one wave per row with twice the
// bytes in flight per wave, so they aim at half as many waves.
Tiling step_tiling(int nx, int ny, int nz, int rows, int z_chunk, int tile_x = 64) {
  if (z_chunk > 0) return make_tiling(nx, ny, nz, rows, z_chunk, tile_x);
  const int nint = nz - 1;
  const long cols = (long)((nx + tile_x - 1) / tile_x) * ((ny + rows - 1) / rows);
  const long target = tile_x == 128 ? 2048 / rows : 4096 / (rows * tile_x / 64);  // tiles
  long chunks = std::max<long>(1, (target + cols / 2) / cols);
  chunks = std::min<long>(chunks, std::max(1, nint / 4));  // at least 4 planes per chunk
  const int zc = (int)((nint + chunks - 1) / chunks);
  return make_tiling(nx, ny, nz, rows, zc, tile_x);
}

// Rows of the one-step kernel's tiles: 8 or 16 as requested, else 8 (on
// MI355X the 8-row tiles stream about 2 % faster at equal occupancy).
int resolve_rows(int tile_y, int ny) {
  (void)ny;
  return tile_y == 16 ? 16 : 8;
}

constexpr int kMinZChunk = 4, kMaxZChunk = 512;

int exec_z_chunk(const it_exec* ex) { return ex ? ex->z_chunk : 0; }

// Tile width of the one-step kernels for chambers ch[0..n): as asked, else
// (tile_x and tile_y both 0) 32 x 16 tiles where they cover the planes with
// at least a quarter fewer padded nodes than 64 x 8 tiles (narrow grids, where
// most lanes of a 64-wide tile would idle); else, for a single chamber
// (pairs: the caller runs the one-step kernel on one chamber) with an even
// nx, 128 x 8 tiles of column pairs where they pad no more than 64 x 8 tiles
// do; else 64.  On MI355X 32 x 16 tiles take 1.5 % longer per node on a
// 256-wide grid and 12 % longer on the 64..256-wide batched sweep, and 20 %
// less on 24-wide chambers; 128 x 8 tiles take 4.7 % less on the 256-wide
// grid.
int exec_tile_x(const it_exec* ex, const it_chamber* ch, int n, bool pairs) {
  if (ex && ex->tile_x != 0) return plain_tile_cols(ex->tile_x);
  if (ex && ex->tile_y != 0) return 64;
  double pad64 = 0.0, pad32 = 0.0;
  for (int q = 0; q < n; ++q) {
    const double planes = ch[q].nz - 1;
    pad64 += planes * (double)((ch[q].nx + 63) / 64 * 64) * (double)((ch[q].ny + 7) / 8 * 8);
    pad32 += planes * (double)((ch[q].nx + 31) / 32 * 32) * (double)((ch[q].ny + 15) / 16 * 16);
  }
  if (pad32 <= 0.75 * pad64) return 32;
  if (pairs && n == 1 && ch->nx % 2 == 0 && (ch->nx + 127) / 128 * 128 <= (ch->nx + 63) / 64 * 64) return 128;
  return 64;
}

// Tile shape fields: tile_x 0, 32, 64 or 128; 32-wide tiles have 16 rows.
bool tile_shape_ok(const it_exec* ex) {
  if (!ex) return true;
  if (ex->tile_x != 0 && ex->tile_x != 32 && ex->tile_x != 64 && ex->tile_x != 128) return false;
  return ex->tile_x != 32 || ex->tile_y == 0 || ex->tile_y == 16;
}

// Tiles of column pairs need an even nx (a pair never straddles the edge of
// the grid) and 16-byte aligned fields.
bool pair_tiles_ok(const it_chamber* ch, const void* a, const void* b) {
  return ch->nx % 2 == 0 && (uintptr_t)a % 16 == 0 && (uintptr_t)b % 16 == 0;
}

bool z_chunk_ok(const it_exec* ex) {
  const int z = exec_z_chunk(ex);
  return z == 0 || (z >= kMinZChunk && z <= kMaxZChunk);
}

// Steps per launch the caller asked for: 1 (the one-step kernel), T > 1 (the
// blocked kernel), or 0 (the library's choice).
int requested_steps(const it_exec* ex) {
  if (ex && ex->kernel == IT_KERNEL_PLAIN) return 1;
  if (ex && ex->steps_per_pass > 0) return ex->steps_per_pass;
  if (ex && ex->kernel == IT_KERNEL_BLOCKED) return kBlockedT;
  return 0;
}

// The library's choice: passes of kBlockedT steps of the blocked kernel on a
// grid large enough to fill the machine (on MI355X 1.8x faster per
// step than one step per launch at 13 M and 67 M interior nodes), else one
// step per launch.  Not when the caller sets a one-step tile option, and not
// when the final fields are asked for: a blocked pass that contains the step
// meeting the collection criterion still computes the pass's later steps,
// so its fields would be up to kBlockedT - 1 steps past the result's.
int auto_steps(const it_chamber* ch, const it_exec* ex, bool exact_fields) {
  if (exact_fields) return 1;
  if (ex && (ex->tile_x || ex->tile_y || ex->z_chunk)) return 1;
  const double nodes = (double)ch->nx * ch->ny * (double)(ch->nz - 1);
  if (nodes < kBlockedMinNodes || ch->nx < 64 || ch->ny < 32) return 1;
  return kBlockedT;
}

// Steps per launch of a run.
int exec_steps(const it_chamber* ch, const it_exec* ex, bool exact_fields) {
  const int T = requested_steps(ex);
  return T > 0 ? T : auto_steps(ch, ex, exact_fields);
}

// Host check of an execution choice (T steps per launch) for a chamber,
// made before any device work.
int check_exec(const it_chamber* ch, const it_exec* ex, int T) {
  if (T < 1 || T > kMaxT) return IT_EINVAL;
  if (T > 1 && !blocked_supported(T, ex ? ex->tile_y : 0)) return ex && ex->tile_y ? IT_EINVAL : IT_ENOTSUP;
  if (!z_chunk_ok(ex)) return IT_EINVAL;
  if (!tile_shape_ok(ex) || (ex && (ex->tile_x == 32 || ex->tile_x == 128) && T > 1)) return IT_EINVAL;
  if (ex && ex->tile_x == 128 && ch->nx % 2) return IT_EINVAL;
  return IT_OK;
}

// The same check plus what depends on the workspace: an explicit request for
// tiles of column pairs needs 16-byte aligned fields, and every field sits
// at a 256-byte offset from the workspace's start.
int check_exec_ws(const it_chamber* ch, const it_exec* ex, int T, const void* ws) {
  const int rc = check_exec(ch, ex, T);
  if (rc) return rc;
  if (ex && ex->tile_x == 128 && (uintptr_t)ws % 16 != 0) return IT_EINVAL;
  return IT_OK;
}

Tiling deposit_tiling(int nx, int ny, int nz) {
  const long cols = (long)((nx + 63) / 64) * ((ny + 3) / 4);
  const int nint = nz - 1;
  long want = std::max<long>(1, (2048 + cols - 1) / cols);
  want = std::min<long>(want, nint);
  int zc = (int)((nint + want - 1) / want);
  zc = std::max(zc, std::min(4, nint));
  return make_tiling(nx, ny, nz, 4, zc);
}

struct Layout {
  size_t field_elems;
  size_t off_field[4];
  size_t off_ele[2];        // electron densities (free-electron runs only)
  size_t off_partials, partial_doubles;
  size_t off_counter;
  size_t off_state;
  size_t off_tracks;
  size_t off_trace;
  size_t total;
};

size_t max_grid(const it_chamber* ch) {
  // the smallest z chunk gives the most stepping blocks of any launch shape
  size_t g = std::max((size_t)step_tiling(ch->nx, ch->ny, ch->nz, 8, kMinZChunk).grid,
                      (size_t)deposit_tiling(ch->nx, ch->ny, ch->nz).grid);
  g = std::max(g, (size_t)step_tiling(ch->nx, ch->ny, ch->nz, 16, kMinZChunk, 32).grid);
  for (int T = 2; T <= kMaxT; ++T)
    for (int R = 1; R <= 8; ++R) {  // every rows-per-thread choice the caller can make
      if (!blocked_supported(T, 8 * R)) continue;
      int grid, per, tx, ty, nt, zc, zch;
      blocked_tiling(ch->nx, ch->ny, ch->nz, T, R, &grid, &per, &tx, &ty, &nt, &zc, &zch);
      g = std::max(g, (size_t)grid * T);
    }
  return g;
}

Layout make_layout(const it_chamber* ch, int64_t ntracks) {
  Layout L;
  L.field_elems = (size_t)(ch->nz + 1) * ch->ny * ch->nx;
  size_t off = 0;
  for (int f = 0; f < 4; ++f) {
    L.off_field[f] = off;
    off = align_up(off + L.field_elems * sizeof(double));
  }
  // per-block partial tallies: kAcc slots per fused step (max_grid counts
  // blocks times fused steps)
  for (int f = 0; f < 2; ++f) {
    L.off_ele[f] = off;
    if (ch->mu_e > 0.0) off = align_up(off + L.field_elems * sizeof(double));
  }
  // two halves: the one-step kernel alternates between them (a step's
  // partials are reduced during the next step)
  L.partial_doubles = 2 * max_grid(ch) * (size_t)std::max(kAcc, kAcc3);
  L.off_partials = off;
  off = align_up(off + L.partial_doubles * sizeof(double));
  L.off_counter = off;
  off = align_up(off + 64 * sizeof(unsigned));
  L.off_state = off;
  off = align_up(off + sizeof(RunState));
  L.off_tracks = off;
  off = align_up(off + (size_t)std::max<int64_t>(ntracks, 1) * sizeof(DepTrack));
  L.off_trace = off;
  off = align_up(off + (size_t)ch->max_steps * IT_TRACE_COLS * sizeof(double));
  L.total = off;
  return L;
}

int check_tracks(const it_track* tr, int64_t n) {
  if (n < 0) return IT_EINVAL;
  if (n > 0 && !tr) return IT_EINVAL;
  if (n > (int64_t)1 << 31) return IT_EINVAL;
  for (int64_t q = 0; q < n; ++q) {
    const it_track& t = tr[q];
    if (!finite_nonneg(t.let_keV_um) || !(std::isfinite(t.b_cm) && t.b_cm > 0)) return IT_EINVAL;
    if (!std::isfinite(t.x_cm) || !std::isfinite(t.y_cm)) return IT_EINVAL;
    if (!std::isfinite(t.theta) || !std::isfinite(t.phi)) return IT_EINVAL;
    if (!finite_nonneg(t.t_s)) return IT_EINVAL;
    if (!finite_nonneg(t.b_neg_cm)) return IT_EINVAL;
  }
  return IT_OK;
}

int64_t deposit_step(double t, double dt) {
  const double s = std::floor(t / dt);
  if (s > 4.0e18) return INT64_MAX;
  return (int64_t)s;
}

// Host memory the run states are read back into: the caller's page-locked
// buffer when it is given and large enough (the device keeps stepping while
// a copy is in flight), else ordinary memory held here for the call (the
// copies then complete before the host goes on, so every read-back is
// synchronous).
constexpr size_t kHostSlots = 4;  // read-back slots of a single run

size_t host_slots_needed(int ninst) { return std::max<size_t>(kHostSlots, 2 * (size_t)ninst); }

struct HostSlots {
  RunState* p = nullptr;
  bool pinned = false;
  std::vector<RunState> own;
};

void host_slots(const it_exec* ex, int ninst, HostSlots& h) {
  const size_t n = host_slots_needed(ninst);
  if (ex && ex->host_buffer && ex->host_buffer_bytes >= n * sizeof(RunState) &&
      (uintptr_t)ex->host_buffer % alignof(RunState) == 0) {
    h.p = (RunState*)ex->host_buffer;
    h.pinned = true;
  } else {
    h.own.assign(n, RunState{});
    h.p = h.own.data();
    h.pinned = false;
  }
}

#define HIP_TRY(expr)                               \
  do {                                              \
    if ((expr) != hipSuccess) return IT_EHIP;       \
  } while (0)

// 1 when every track gives both species the same radius.
int same_radii(const it_track* tr, int64_t n) {
  for (int64_t q = 0; q < n; ++q)
    if (tr[q].b_neg_cm > 0.0 && tr[q].b_neg_cm != tr[q].b_cm) return 0;
  return 1;
}

// Per-track constants of the deposit kernel: axis direction, peak density
// N0/(pi b^2) with N0 = LET/W (keV/um -> eV/cm), 1/b^2 and the (8b)^2 cut.
DepTrack prepare_track(const it_chamber* ch, const it_track& t) {
  DepTrack d;
  d.x0 = t.x_cm;
  d.y0 = t.y_cm;
  d.ux = std::sin(t.theta) * std::cos(t.phi);
  d.uy = std::sin(t.theta) * std::sin(t.phi);
  d.uz = std::cos(t.theta);
  const double N0 = t.let_keV_um * 1.0e7 / ch->W_eV;
  d.peak = N0 / (M_PI * t.b_cm * t.b_cm);
  d.inv_b2 = 1.0 / (t.b_cm * t.b_cm);
  d.cut2 = 64.0 * t.b_cm * t.b_cm;
  const double bn = t.b_neg_cm > 0.0 ? t.b_neg_cm : t.b_cm;
  d.peak_n = N0 / (M_PI * bn * bn);
  d.inv_b2_n = 1.0 / (bn * bn);
  d.cut2_n = 64.0 * bn * bn;
  return d;
}

// Deposit parameters common to every deposit of a chamber (fields, tracks,
// partials and state pointers are filled in by the caller).
DepositParams base_deposit(const it_chamber* ch, double dt, const Tiling& td) {
  DepositParams dp;
  std::memset(&dp, 0, sizeof(dp));
  const double dz = ch->gap / ch->nz;
  dp.nx = ch->nx;
  dp.ny = ch->ny;
  dp.nz = ch->nz;
  dp.tiles_x = td.tiles_x;
  dp.tiles_y = td.tiles_y;
  dp.zchunks = td.zchunks;
  dp.zc = td.zc;
  dp.ntiles = td.ntiles;
  dp.per_xcd = td.per_xcd;
  dp.dx = ch->dx;
  dp.dy = ch->dy;
  dp.dz = dz;
  dp.half_gap = 0.5 * ch->gap;
  dp.Lx = ch->nx * ch->dx;
  dp.Ly = ch->ny * ch->dy;
  dp.absorbing = ch->lateral_bc;
  dp.dV = ch->dx * ch->dy * dz;
  dp.beta = ch->alpha * dt;
  return dp;
}

struct Event {
  int64_t step;
  int64_t par_begin, par_count, tilt_begin, tilt_count;
  bool uniform;
};

// The stepping loop shared by it_solve and it_advance.  Enqueues passes of
// up to T steps, cut at deposit steps, and reads the run state back every
// `check_every` steps (two checks in flight) to stop once the device has
// flagged completion.
int run_loop(const it_chamber* ch, double dt, const it_exec* ex, char* ws, const Layout& L,
             const std::vector<Event>& events, const std::vector<DepTrack>& dev_tracks, int same_r,
             int64_t nsteps, int64_t min_stop_step, double stop_tol, int T, hipStream_t stream, HostSlots& hs,
             RunState* final_state, int* passes_issued) {
  const int exec_rc = check_exec(ch, ex, T);
  if (exec_rc) return exec_rc;
  const int tile_y = ex ? ex->tile_y : 0;
  int64_t check_every = ex && ex->check_every > 0 ? ex->check_every : 64;
  const bool span = ex && ex->timing_events && ex->timing_span && ex->n_timing_events >= 2;
  const int n_timing = ex && ex->timing_events && !span ? std::max(ex->n_timing_events, 0) / 2 : 0;

  double* field[4];
  for (int f = 0; f < 4; ++f) field[f] = (double*)(ws + L.off_field[f]);
  double* partials = (double*)(ws + L.off_partials);
  unsigned* counter = (unsigned*)(ws + L.off_counter);
  RunState* state = (RunState*)(ws + L.off_state);
  DepTrack* tracks = (DepTrack*)(ws + L.off_tracks);
  double* trace = (double*)(ws + L.off_trace);
  (void)dev_tracks;

  const Coef cp = species_coef(ch, dt, 0), cn = species_coef(ch, dt, 1);
  const double dz = ch->gap / ch->nz;
  const double dV = ch->dx * ch->dy * dz;
  int tx = T == 1 ? exec_tile_x(ex, ch, 1, true) : 64;
  if (tx == 128 && !pair_tiles_ok(ch, field[0], field[1])) {
    if (ex && ex->tile_x == 128) return IT_EINVAL;
    tx = 64;  // the automatic choice falls back on unaligned fields
  }
  const int rows = tx == 32 ? 16 : resolve_rows(tile_y, ch->ny);
  const Tiling tp = step_tiling(ch->nx, ch->ny, ch->nz, rows, exec_z_chunk(ex), tx);
  const Tiling td = deposit_tiling(ch->nx, ch->ny, ch->nz);

  RunState* slots = hs.p;
  // read-backs in flight: two with the caller's page-locked buffer, else one
  // (an ordinary host buffer is filled before the copy call returns)
  const int depth = hs.pinned ? 2 : 1;

  StepParams sp;
  sp.nx = ch->nx;
  sp.ny = ch->ny;
  sp.nz = ch->nz;
  sp.cp = cp;
  sp.cn = cn;
  sp.beta = ch->alpha * dt;
  sp.gsp = screening_coef(ch, dt, 0);
  sp.gsn = screening_coef(ch, dt, 1);
  sp.absorbing = ch->lateral_bc;
  sp.dV = dV;
  sp.stop_tol = stop_tol;
  sp.min_stop_step = min_stop_step;
  sp.partials = partials;
  sp.counter = counter;
  sp.state = state;
  sp.trace = trace;
  sp.prev_partials = nullptr;
  sp.prev_nblocks = 0;
  sp.prev_T = 1;
  sp.prev_step = 0;

  DepositParams dp = base_deposit(ch, dt, td);
  dp.same_radii = same_r;
  dp.partials = partials;
  dp.counter = counter;
  dp.state = state;

  int cur = 0;  // field pair index: 0 -> (field0, field1), 1 -> (field2, field3)
  int64_t l = 0;
  size_t ev = 0;
  int issued = 0;
  int64_t since_check = 0;
  int pending = 0, slot_head = 0;
  // Span timing: one event pair per run of consecutive stepping launches
  // (runs are separated by deposits), as long as the caller gave events for
  // it; seg_open: the current run's first event is recorded.
  const int n_spans = span ? ex->n_timing_events / 2 : 0;
  int seg = 0;
  bool seg_open = false;
  // caller's timing events of the launch about to be issued (null when none)
  auto ev_pair = [&](int which) -> hipEvent_t {
    if (span) {
      if (which != 0 || seg_open || seg >= n_spans) return nullptr;
      seg_open = true;
      return (hipEvent_t)ex->timing_events[2 * seg];
    }
    return issued < n_timing ? (hipEvent_t)ex->timing_events[2 * issued + which] : nullptr;
  };
  auto close_span = [&]() -> hipError_t {
    if (!seg_open) return hipSuccess;
    seg_open = false;
    return hipEventRecord((hipEvent_t)ex->timing_events[2 * seg++ + 1], stream);
  };
  hipEvent_t evs[4];
  for (int q = 0; q < 4; ++q)
    if (hipEventCreateWithFlags(&evs[q], hipEventDisableTiming) != hipSuccess) {
      for (int r = 0; r < q; ++r) (void)hipEventDestroy(evs[r]);
      return IT_EHIP;
    }
  int rc = IT_OK;
  bool stopped = false;
  auto fail = [&](int code) {
    rc = code;
    return code;
  };
  // Launch i records the steps of launch i-1 (an extra block reduces its
  // partials while the others compute the next step or pass); the partials
  // alternate between two buffers by launch.  Steps still unrecorded are
  // closed by a reduction launch before a deposit (so that their records do
  // not count the deposit) and at the end.
  const int grid_plain = 8 * tp.per_xcd;
  const int R = T > 1 ? blocked_rows(T, tile_y) : 0;  // rows per thread of the blocked passes
  double* part_buf[2] = {partials, partials + L.partial_doubles / 2};
  bool unrecorded = false;
  int64_t unrecorded_step = 0;
  int unrecorded_T = 1, unrecorded_blocks = 0, unrecorded_buf = 0;
  auto close_step = [&]() -> hipError_t {
    if (!unrecorded) return hipSuccess;
    unrecorded = false;
    StepParams q = sp;
    q.partials = part_buf[unrecorded_buf];
    q.step0 = unrecorded_step;
    q.prev_partials = nullptr;
    return launch_reduce_steps(q, unrecorded_blocks, unrecorded_T, stream);
  };
  while (l < nsteps && !stopped) {
    if (ev < events.size() && events[ev].step == l) {
      const Event& e = events[ev];
      if (close_span() != hipSuccess || close_step() != hipSuccess) { fail(IT_EHIP); break; }
      dp.pos = field[2 * cur];
      dp.neg = field[2 * cur + 1];
      dp.uniform = e.uniform ? ch->uniform_n0 : 0.0;
      dp.par = tracks + e.par_begin;
      dp.npar = (int)e.par_count;
      dp.tilt = tracks + e.tilt_begin;
      dp.ntilt = (int)e.tilt_count;
      if (launch_deposit(dp, stream) != hipSuccess) { fail(IT_EHIP); break; }
      ++ev;
    }
    const int64_t next_dep = ev < events.size() ? events[ev].step : nsteps;
    const int64_t todo = std::min<int64_t>(std::min<int64_t>(T, next_dep - l), nsteps - l);
    sp.pin = field[2 * cur];
    sp.nin = field[2 * cur + 1];
    sp.pout = field[2 * (1 - cur)];
    sp.nout = field[2 * (1 - cur) + 1];
    sp.step0 = l;
    // this launch's partials, and the previous launch's for its extra block
    const int buf = issued & 1;
    sp.partials = part_buf[buf];
    sp.prev_partials = unrecorded ? part_buf[unrecorded_buf] : nullptr;
    sp.prev_nblocks = unrecorded_blocks;
    sp.prev_T = unrecorded_T;
    sp.prev_step = unrecorded_step;
    hipError_t e;
    int nblocks = grid_plain;
    if (todo == 1) {
      sp.tiles_x = tp.tiles_x;
      sp.tiles_y = tp.tiles_y;
      sp.zchunks = tp.zchunks;
      sp.zc = tp.zc;
      sp.ntiles = tp.ntiles;
      sp.per_xcd = tp.per_xcd;
      e = launch_step_plain(sp, rows, tx, stream, ev_pair(0), ev_pair(1), true);
    } else {
      e = launch_step_blocked(sp, (int)todo, R, stream, ev_pair(0), ev_pair(1), &nblocks);
    }
    unrecorded = true;
    unrecorded_step = l;
    unrecorded_T = (int)todo;
    unrecorded_blocks = nblocks;
    unrecorded_buf = buf;
    if (e != hipSuccess) { fail(IT_EHIP); break; }
    ++issued;
    cur = 1 - cur;
    l += todo;
    since_check += todo;
    if (since_check >= check_every || l >= nsteps) {
      since_check = 0;
      RunState* slot = &slots[slot_head];
      if (hipMemcpyAsync(slot, state, sizeof(RunState), hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipEventRecord(evs[slot_head], stream) != hipSuccess) { fail(IT_EHIP); break; }
      slot_head = (slot_head + 1) & 3;
      ++pending;
      if (pending >= depth) {
        const int oldest = (slot_head + 4 - pending) & 3;
        if (hipEventSynchronize(evs[oldest]) != hipSuccess) { fail(IT_EHIP); break; }
        --pending;
        if (slots[oldest].done) stopped = true;
      }
    }
  }
  if (rc == IT_OK && close_span() != hipSuccess) fail(IT_EHIP);
  if (rc == IT_OK && close_step() != hipSuccess) fail(IT_EHIP);
  if (rc == IT_OK) {
    if (hipMemcpyAsync(&slots[slot_head], state, sizeof(RunState), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      rc = IT_EHIP;
    else
      *final_state = slots[slot_head];
  } else {
    (void)hipStreamSynchronize(stream);
  }
  for (int q = 0; q < 4; ++q) (void)hipEventDestroy(evs[q]);
  *passes_issued = issued;
  return rc;
}


// ---------------------------------------------------------------------------
// Batched sweeps
// ---------------------------------------------------------------------------

struct InstLayout {
  size_t off_field[4], field_elems;
  size_t off_partials, off_counter, off_tracks;
  size_t off_pulse[2];  // the first pulse's densities (pulse trains only)
  int slots;        // partial slots per pass: the most stepping tiles the run can use
};

struct BatchLayout {
  std::vector<InstLayout> inst;
  size_t off_states;  // RunState[ninst], contiguous for one read-back
  size_t off_table;   // BatchInstance[ninst]
  size_t total;
};

// Planes per tile in a batch: as requested, else 16.  The single-chamber
// default sizes the chunks so that one chamber fills the machine; in a
// batch many chambers share it and, as they finish, the last ones run
// alone, so shorter chunks that keep the tail busy win (measured on the
// 96-chamber sweep: 16 planes 13.1 s, 32: 13.4 s, 64: 14.3 s, the
// single-chamber rule 16.6 s).
int batch_z_chunk(const it_exec* exec) {
  const int z = exec_z_chunk(exec);
  return z > 0 ? z : 16;
}

// One tile shape serves every instance of a batch.
int batch_rows(const it_chamber* ch, int ninst, const it_exec* exec) {
  if (exec_tile_x(exec, ch, ninst, false) == 32) return 16;
  int min_ny = ch[0].ny;
  for (int q = 1; q < ninst; ++q) min_ny = std::min(min_ny, ch[q].ny);
  return resolve_rows(exec ? exec->tile_y : 0, min_ny);
}

// Steps per pass of a batch: as asked, else passes of kBlockedT steps of the
// blocked tile pass unless a one-step tile option is set (then one step per
// launch).
int batch_steps(const it_chamber*, int, const it_exec* ex) {
  const int T = requested_steps(ex);
  if (T > 0) return T;
  if (ex && (ex->tile_x || ex->tile_y || ex->z_chunk)) return 1;
  return kBlockedT;
}

// Checks of a batch's steps per pass: the blocked pass needs a supported
// depth and rows, and takes no one-step tile width.
int check_batch_steps(const it_chamber*, int, const it_exec* ex, int T) {
  if (T < 1 || T > kMaxT) return IT_EINVAL;
  if (T == 1) return IT_OK;
  if (!blocked_supported(T, ex ? ex->tile_y : 0)) return ex && ex->tile_y ? IT_EINVAL : IT_ENOTSUP;
  if (ex && ex->tile_x) return IT_EINVAL;
  return IT_OK;
}

// Most planes per chunk of the blocked batch tiles: as requested, else 512
// (no cap in practice): batch_blocked_retile_z picks the chunk for the
// running instances below it.  Each chunk recomputes T planes of halo at
// both ends, so with many chambers running the longer chunks the search
// takes pay (the 96-chamber sweep: 6.55 s with a 24-plane cap, 6.34 s with
// 32, 6.00 s with 48, 5.98 s with 64 or more, where the search takes 49
// planes while all chambers run).
int batch_blocked_z_chunk(const it_exec* exec) {
  const int z = exec_z_chunk(exec);
  return z > 0 ? z : 512;
}

// Blocked tiles of one chamber of a batch in chunks of zc planes (T steps,
// R rows per thread).
Tiling batch_blocked_tiling(const it_chamber& c, int T, int R, int zc) {
  Tiling t;
  blocked_tiling_zc(c.nx, c.ny, c.nz, T, R, zc, &t.tiles_x, &t.tiles_y, &t.ntiles, &t.zc, &t.zchunks);
  t.per_xcd = (t.ntiles + 7) / 8;
  t.grid = 8 * t.per_xcd;
  return t;
}

// Stepping tiles of one chamber of a batch (T > 1: blocked tiles, R rows per
// thread, in chunks of zc planes, or of the caller's or default chunk when
// zc is 0).
Tiling batch_tiling(const it_chamber& c, int T, int R, int rows, const it_exec* exec, int tile_x, int zc = 0) {
  if (T == 1) return step_tiling(c.nx, c.ny, c.nz, rows, batch_z_chunk(exec), tile_x);
  return batch_blocked_tiling(c, T, R, zc > 0 ? zc : batch_blocked_z_chunk(exec));
}

// Shortest chunk the blocked batch tiles are re-chunked to: T planes (a
// chunk then computes three times its planes, which pays only when it puts
// blocks on otherwise idle CUs; the search below weighs exactly that).
int batch_blocked_min_z(int z0, int T) { return std::min(z0, T); }

// Chunk length of the blocked batch tiles for the running instances `set`:
// the caller's (or default) chunk z0 while the batch fills the machine, a
// shorter one once it leaves CUs idle.  One blocked block occupies a CU, so
// a launch takes about ceil(blocks / CUs) rounds of one block's march
// (its chunk plus T planes of halo at each end); the chunk minimises that,
// between batch_blocked_min_z(z0, T) planes and z0.  On MI355X's 256 CUs the
// 96-chamber sweep's tail, where a few chambers run, otherwise idles most of
// the machine.
int batch_blocked_retile_z(const it_chamber* ch, const int* set, int n, int T, int R, int z0) {
  constexpr long kCUs = 256;
  int most = 1;  // longer chunks than the deepest instance's planes change nothing
  for (int i = 0; i < n; ++i) most = std::max(most, ch[set[i]].nz - 1);
  z0 = std::min(z0, most);
  const int zmin = batch_blocked_min_z(z0, T);
  // tile columns and interior planes of each instance (the chunk count is
  // ceil(planes / min(z, planes)), as blocked_tiling_zc takes it)
  std::vector<long> cols(n);
  std::vector<int> planes(n);
  for (int i = 0; i < n; ++i) {
    const Tiling t = batch_blocked_tiling(ch[set[i]], T, R, 1);
    cols[i] = (long)t.tiles_x * t.tiles_y;
    planes[i] = ch[set[i]].nz - 1;
  }
  int best_z = z0;
  double best = 1e300;
  for (int z = z0; z >= zmin; --z) {
    long blocks = 0;
    for (int i = 0; i < n; ++i) {
      const int zz = std::min(z, planes[i]);
      blocks += cols[i] * ((planes[i] + zz - 1) / zz);
    }
    const double cost = (double)((blocks + kCUs - 1) / kCUs) * (z + 2.0 * T);
    if (cost < best - 1e-9) {
      best = cost;
      best_z = z;
    }
  }
  return best_z;
}

BatchLayout make_batch_layout(const it_chamber* ch, const int64_t* toff, int ninst, int rows, const it_exec* exec,
                              int tile_x, int T, int R) {
  BatchLayout B;
  size_t off = 0;
  B.inst.resize(ninst);
  for (int q = 0; q < ninst; ++q) {
    InstLayout& L = B.inst[q];
    const it_chamber& c = ch[q];
    L.field_elems = (size_t)(c.nz + 1) * c.ny * c.nx;
    for (int f = 0; f < 4; ++f) {
      L.off_field[f] = off;
      off = align_up(off + L.field_elems * sizeof(double));
    }
    // partial slots for the most tiles any chunk length of the run can give
    // (blocked tiles are re-chunked as instances stop)
    const int zmin = T > 1 ? batch_blocked_min_z(batch_blocked_z_chunk(exec), T) : 0;
    const Tiling ts = batch_tiling(c, T, R, rows, exec, tile_x, zmin);
    const Tiling td = deposit_tiling(c.nx, c.ny, c.nz);
    L.slots = ts.ntiles;
    L.off_partials = off;  // two halves of step partials (alternate passes); the deposit uses the start
    off = align_up(off + std::max((size_t)2 * ts.ntiles * kAcc * T, (size_t)td.grid * 5) * sizeof(double));
    L.off_counter = off;
    off = align_up(off + 64 * sizeof(unsigned));
    L.off_tracks = off;
    off = align_up(off + (size_t)std::max<int64_t>(toff[q + 1] - toff[q], 1) * sizeof(DepTrack));
    L.off_pulse[0] = L.off_pulse[1] = 0;
    if (c.n_pulses >= 2)
      for (int f = 0; f < 2; ++f) {
        L.off_pulse[f] = off;
        off = align_up(off + L.field_elems * sizeof(double));
      }
  }
  B.off_states = off;
  off = align_up(off + (size_t)ninst * sizeof(RunState));
  B.off_table = off;
  off = align_up(off + (size_t)ninst * sizeof(BatchInstance));
  B.total = off;
  return B;
}

int check_batch(const it_chamber* ch, const int64_t* toff, const it_track* tracks, int ninst) {
  if (!ch || !toff || ninst < 1 || ninst > 65536) return IT_EINVAL;
  if (toff[0] != 0) return IT_EINVAL;
  for (int q = 0; q < ninst; ++q) {
    if (toff[q + 1] < toff[q]) return IT_EINVAL;
    const int64_t n = toff[q + 1] - toff[q];
    int rc = check_chamber(&ch[q]);
    if (rc) return rc;
    rc = check_tracks(n ? tracks + toff[q] : nullptr, n);
    if (rc) return rc;
    if (ch[q].mu_e > 0.0) return IT_ENOTSUP;  // free electrons: single runs only
    rc = check_train(&ch[q], n ? tracks + toff[q] : nullptr, n);
    if (rc) return rc;
  }
  return IT_OK;
}

void fill_result(const RunState& fin, double dt, int64_t max_steps, int issued, it_result* out) {
  std::memset(out, 0, sizeof(*out));
  const double collected = fin.sums[1] + fin.sums[2] + fin.sums[3] + fin.sums[4];
  int flags = fin.flags;
  // stopped by the step limit (the criterion may also fire on the last step)
  if (fin.steps >= max_steps && (!fin.done || fin.by_limit)) flags |= IT_FLAG_MAX_STEPS;
  if (fin.max_beta_n > 1.0) flags |= IT_FLAG_REACTION;
  // charge released of both signs: positive ions + negative charge (negative
  // ions, plus free electrons when present)
  const double released = fin.released + fin.released_q;
  if (released > 0.0) {
    out->f = (collected + fin.e_sums[0] + fin.e_sums[1]) / released;
    out->f_R = 1.0 - 2.0 * (fin.sums[0] + fin.e_sums[2]) / released;
  } else {
    out->f = 1.0;
    out->f_R = 1.0;
    flags |= IT_FLAG_EMPTY;
  }
  out->ks = 1.0 / out->f;
  out->n_released = fin.released;
  out->n_released_neg = fin.released_neg;
  out->e_released = fin.released_e;
  out->e_collected_anode = fin.e_sums[0];
  out->e_collected_cathode = fin.e_sums[1];
  out->e_recombined = fin.e_sums[2];
  out->e_left = fin.e_left;
  out->released_neg_charge = fin.released_q;
  out->e_steps = fin.e_steps;
  out->n_recombined = fin.sums[0];
  out->n_inflight_pos = fin.last[0];
  out->n_inflight_neg = fin.last[1];
  out->col_pos_anode = fin.sums[1];
  out->col_pos_cathode = fin.sums[2];
  out->col_neg_anode = fin.sums[3];
  out->col_neg_cathode = fin.sums[4];
  out->dt = dt;
  out->max_beta_n = fin.max_beta_n;
  out->n_space_charge_pos = fin.screened[0];
  out->n_space_charge_neg = fin.screened[1];
  out->n_escaped_pos = fin.escaped[0];
  out->n_escaped_neg = fin.escaped[1];
  out->steps = fin.steps;
  out->flags = flags;
  out->passes = issued;
}

// The pulse-train part of a result (period_steps m > 0): pulses deposited,
// and f, ks, f_R and the period counts from the last period once it began.
void train_result(const RunState& fin, const it_chamber* ch, int64_t m, it_result* out) {
  if (ch->n_pulses < 2 || m <= 0) return;
  const int64_t delivered = (fin.steps + m - 1) / m;  // pulses at steps 0, m, 2m, ... below fin.steps
  out->pulses = (int32_t)std::min<int64_t>(delivered, ch->n_pulses);
  if (!fin.period_started) return;
  double collected = 0.0;
  for (int q = 1; q < 5; ++q) collected += fin.sums[q] - fin.period_sums[q];
  const double released = fin.period_rel[0] + fin.period_rel[1];
  const double recombined = fin.sums[0] - fin.period_sums[0];
  out->period_released = released;
  out->period_collected = collected;
  out->period_recombined = recombined;
  if (released > 0.0) {
    out->f = collected / released;
    out->ks = 1.0 / out->f;
    out->f_R = 1.0 - 2.0 * recombined / released;
  }
}

}  // namespace
}  // namespace it

using namespace it;

extern "C" {

const char* it_strerror(int code) {
  switch (code) {
    case IT_OK: return "ok";
    case IT_EINVAL: return "invalid argument (size, constant or track out of range)";
    case IT_ENODT: return "no stable time step: neither drift nor diffusion bounds dt";
    case IT_EWORKSPACE: return "workspace missing or smaller than it_workspace_size()";
    case IT_EHIP: return "HIP runtime error";
    case IT_ENOTSUP: return "option or combination of options not supported";
    default: return "unknown status code";
  }
}

int it_host_buffer_size(int32_t ninst, size_t* bytes) {
  if (!bytes || ninst < 1) return IT_EINVAL;
  *bytes = host_slots_needed(ninst) * sizeof(RunState);
  return IT_OK;
}

int it_dt(const it_chamber* ch, const it_track* tracks, int64_t ntracks, double* dt) {
  if (!dt) return IT_EINVAL;
  int rc = check_chamber(ch);
  if (rc) return rc;
  rc = check_tracks(tracks, ntracks);
  if (rc) return rc;
  return compute_dt(ch, tracks, ntracks, dt);
}

int it_validate(const it_chamber* ch, const it_track* tracks, int64_t ntracks) {
  double dt;
  return it_dt(ch, tracks, ntracks, &dt);
}

int it_workspace_size(const it_chamber* ch, int64_t ntracks, size_t* bytes) {
  if (!bytes || ntracks < 0) return IT_EINVAL;
  int rc = check_chamber(ch);
  if (rc) return rc;
  *bytes = make_layout(ch, ntracks).total;
  return IT_OK;
}

// Electron phase of a free-electron run: steps the three carriers from field
// pair 0 (and electron array 0) at the electrons' step until the device
// flags the electrons collected, then leaves the ions in field pair 0.
// Returns the phase's step count in *e_steps.
int electron_phase(const it_chamber* ch, double dt_ion, char* ws, const Layout& L, hipStream_t stream,
                   RunState* slot, int64_t* e_steps) {
  const double dt1 = std::min(dt_ion, ch->dt_safety * electron_dt(ch));
  Step3Params p;
  std::memset(&p, 0, sizeof(p));
  const Tiling tp = step_tiling(ch->nx, ch->ny, ch->nz, 8, 0);
  p.nx = ch->nx;
  p.ny = ch->ny;
  p.nz = ch->nz;
  p.tiles_x = tp.tiles_x;
  p.tiles_y = tp.tiles_y;
  p.zchunks = tp.zchunks;
  p.zc = tp.zc;
  p.ntiles = tp.ntiles;
  p.per_xcd = tp.per_xcd;
  p.co[0] = carrier_coef(ch, dt1, ch->mu_pos, ch->D_pos);
  p.co[1] = carrier_coef(ch, dt1, -ch->mu_neg, ch->D_neg);
  p.co[2] = carrier_coef(ch, dt1, -ch->mu_e, ch->D_e);
  p.beta = ch->alpha * dt1;
  p.dV = ch->dx * ch->dy * (ch->gap / ch->nz);
  p.stop_tol = ch->stop_tol;
  p.partials = (double*)(ws + L.off_partials);
  p.state = (RunState*)(ws + L.off_state);
  double* pair[2][3] = {{(double*)(ws + L.off_field[0]), (double*)(ws + L.off_field[1]), (double*)(ws + L.off_ele[0])},
                        {(double*)(ws + L.off_field[2]), (double*)(ws + L.off_field[3]), (double*)(ws + L.off_ele[1])}};
  // released electrons (set by the deposit): none means no electron phase
  HIP_TRY(hipMemcpyAsync(slot, p.state, sizeof(RunState), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  *e_steps = 0;
  if (!(slot->released_e > 0.0)) {
    // mark the phase done so later launches of its kernels (none) skip
    return IT_OK;
  }
  const int64_t check_every = 64;
  for (int64_t l = 0; l < ch->max_steps; ++l) {
    for (int s3 = 0; s3 < 3; ++s3) {
      p.in[s3] = pair[l & 1][s3];
      p.out[s3] = pair[(l + 1) & 1][s3];
    }
    HIP_TRY(launch_step3(p, stream));
    if ((l + 1) % check_every == 0 || l + 1 == ch->max_steps) {
      HIP_TRY(hipMemcpyAsync(slot, p.state, sizeof(RunState), hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      if (slot->e_done) break;
    }
  }
  HIP_TRY(hipMemcpyAsync(slot, p.state, sizeof(RunState), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  *e_steps = slot->e_steps;
  if (*e_steps & 1) {  // the ions ended in pair 1: move them to pair 0
    const size_t bytes = L.field_elems * sizeof(double);
    HIP_TRY(hipMemcpyAsync(ws + L.off_field[0], ws + L.off_field[2], bytes, hipMemcpyDeviceToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ws + L.off_field[1], ws + L.off_field[3], bytes, hipMemcpyDeviceToDevice, stream));
  }
  return IT_OK;
}

int it_solve(const it_chamber* ch, const it_track* tracks, int64_t ntracks, const it_exec* exec,
             void* d_workspace, size_t ws_bytes, void* stream_, double* h_trace, double* d_pos_out,
             double* d_neg_out, it_result* out) {
  clear_stale_error();
  if (!out) return IT_EINVAL;
  int rc = it_validate(ch, tracks, ntracks);
  if (rc) return rc;
  const bool fe = ch->mu_e > 0.0;
  if (fe) {  // free electrons: one instantaneous pulse, no space charge, periodic cell
    if (ch->space_charge || ch->lateral_bc) return IT_ENOTSUP;
    for (int64_t q = 0; q < ntracks; ++q)
      if (tracks[q].t_s != 0.0) return IT_ENOTSUP;
  }
  rc = check_train(ch, tracks, ntracks);
  if (rc) return rc;
  const bool train = ch->n_pulses >= 2;
  const int T = exec_steps(ch, exec, d_pos_out || d_neg_out);
  rc = check_exec_ws(ch, exec, T, d_workspace);
  if (rc) return rc;
  const Layout L = make_layout(ch, ntracks);
  if (!d_workspace || ws_bytes < L.total) return IT_EWORKSPACE;
  double dt;
  int64_t period_steps = 0;
  rc = compute_dt(ch, tracks, ntracks, &dt, &period_steps);
  if (rc) return rc;
  HostSlots hs;
  host_slots(exec, 1, hs);
  hipStream_t stream = (hipStream_t)stream_;
  char* ws = (char*)d_workspace;

  // Deposit schedule: tracks grouped by step floor(t/dt), parallel ones first.
  struct Item {
    int64_t step;
    int tilted;
    int64_t index;
  };
  std::vector<Item> items;
  items.reserve(ntracks);
  for (int64_t q = 0; q < ntracks; ++q) {
    const int64_t s = deposit_step(tracks[q].t_s, dt);
    if (s >= ch->max_steps) continue;
    const double st = std::sin(tracks[q].theta);
    const bool par = st == 0.0;
    items.push_back({s, par ? 0 : 1, q});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
    return a.step != b.step ? a.step < b.step : a.tilted < b.tilted;
  });
  std::vector<DepTrack> dev(items.size());
  for (size_t q = 0; q < items.size(); ++q) dev[q] = prepare_track(ch, tracks[items[q].index]);
  std::vector<Event> events;
  int64_t last_dep = -1;
  for (size_t q = 0; q < items.size();) {
    Event e;
    e.step = items[q].step;
    e.uniform = false;
    e.par_begin = (int64_t)q;
    size_t r = q;
    while (r < items.size() && items[r].step == e.step && items[r].tilted == 0) ++r;
    e.par_count = (int64_t)(r - q);
    e.tilt_begin = (int64_t)r;
    while (r < items.size() && items[r].step == e.step) ++r;
    e.tilt_count = (int64_t)r - e.tilt_begin;
    events.push_back(e);
    last_dep = e.step;
    q = r;
  }
  if (ch->uniform_n0 > 0.0) {
    if (events.empty() || events[0].step != 0) {
      Event e{0, 0, 0, 0, 0, true};
      events.insert(events.begin(), e);
    } else {
      events[0].uniform = true;
    }
    last_dep = std::max<int64_t>(last_dep, 0);
  }
  // a pulse train: pulse k repeats the deposit of step 0 (every track is due
  // then) at step k m
  if (train && !events.empty()) {
    const Event first = events[0];
    for (int64_t k = 1; k < ch->n_pulses && k * period_steps < ch->max_steps; ++k) {
      Event e = first;
      e.step = k * period_steps;
      events.push_back(e);
    }
  }

  for (int f = 0; f < 4; ++f)
    HIP_TRY(hipMemsetAsync(ws + L.off_field[f], 0, L.field_elems * sizeof(double), stream));
  HIP_TRY(hipMemsetAsync(ws + L.off_counter, 0, 64 * sizeof(unsigned), stream));
  RunState init = initial_run_state();
  if (train) init.period_step = (ch->n_pulses - 1) * period_steps;
  HIP_TRY(hipMemcpyAsync(ws + L.off_state, &init, sizeof(init), hipMemcpyHostToDevice, stream));
  if (!dev.empty())
    HIP_TRY(hipMemcpyAsync(ws + L.off_tracks, dev.data(), dev.size() * sizeof(DepTrack),
                           hipMemcpyHostToDevice, stream));

  int64_t e_steps = 0;
  if (fe) {
    // the pulse, split into ions and electrons, then the electron phase;
    // the ion phase below starts from its end with no further deposits
    for (int f = 0; f < 2; ++f)
      HIP_TRY(hipMemsetAsync(ws + L.off_ele[f], 0, L.field_elems * sizeof(double), stream));
    DepositParams dp = base_deposit(ch, dt, deposit_tiling(ch->nx, ch->ny, ch->nz));
    dp.pos = (double*)(ws + L.off_field[0]);
    dp.neg = (double*)(ws + L.off_field[1]);
    dp.ele = (double*)(ws + L.off_ele[0]);
    dp.free_e = 1;
    dp.attach = ch->attach_coeff;
    dp.pfree = free_fraction(ch->attach_coeff, ch->gap);
    dp.uniform = ch->uniform_n0;
    const DepTrack* tr_dev = (const DepTrack*)(ws + L.off_tracks);
    if (!events.empty()) {
      dp.par = tr_dev + events[0].par_begin;
      dp.npar = (int)events[0].par_count;
      dp.tilt = tr_dev + events[0].tilt_begin;
      dp.ntilt = (int)events[0].tilt_count;
    }
    dp.same_radii = same_radii(tracks, ntracks);
    dp.partials = (double*)(ws + L.off_partials);
    dp.counter = (unsigned*)(ws + L.off_counter);
    dp.state = (RunState*)(ws + L.off_state);
    if (!events.empty()) HIP_TRY(launch_deposit(dp, stream));
    rc = electron_phase(ch, dt, ws, L, stream, hs.p, &e_steps);
    if (rc) return rc;
    events.clear();
    last_dep = 0;
  }

  RunState fin;
  int issued = 0;
  const int64_t limit = ch->max_steps - e_steps;
  // a pulse train ends with its last period, with no collection test
  const int64_t ion_steps = train ? std::min<int64_t>(ch->n_pulses * period_steps, limit) : limit;
  const int64_t min_stop = train ? INT64_MAX : std::max<int64_t>(last_dep, 0);
  if (ion_steps > 0) {
    rc = run_loop(ch, dt, exec, ws, L, events, dev, same_radii(tracks, ntracks), ion_steps, min_stop,
                  ch->stop_tol, T, stream, hs, &fin, &issued);
    if (rc) return rc;
  } else {
    HIP_TRY(hipMemcpyAsync(hs.p, ws + L.off_state, sizeof(fin), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    fin = *hs.p;
  }

  fill_result(fin, dt, limit, issued, out);
  train_result(fin, ch, period_steps, out);
  if (fe) out->e_dt = std::min(dt, ch->dt_safety * electron_dt(ch));

  if (h_trace && fin.steps > 0) {
    HIP_TRY(hipMemcpyAsync(h_trace, ws + L.off_trace, (size_t)fin.steps * IT_TRACE_COLS * sizeof(double),
                           hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
  }
  const int last = fin.passes & 1;  // field pair holding the latest densities
  if (d_pos_out)
    HIP_TRY(hipMemcpyAsync(d_pos_out, ws + L.off_field[2 * last], L.field_elems * sizeof(double),
                           hipMemcpyDeviceToDevice, stream));
  if (d_neg_out)
    HIP_TRY(hipMemcpyAsync(d_neg_out, ws + L.off_field[2 * last + 1], L.field_elems * sizeof(double),
                           hipMemcpyDeviceToDevice, stream));
  if (d_pos_out || d_neg_out) HIP_TRY(hipStreamSynchronize(stream));
  return IT_OK;
}

int it_workspace_size_batch(const it_chamber* ch, const int64_t* track_offsets, int32_t ninst,
                            const it_exec* exec, size_t* bytes) {
  if (!bytes || !ch || !track_offsets || ninst < 1 || ninst > 65536) return IT_EINVAL;
  for (int q = 0; q < ninst; ++q) {
    const int rc = check_chamber(&ch[q]);
    if (rc) return rc;
    if (track_offsets[q + 1] < track_offsets[q]) return IT_EINVAL;
  }
  if (!z_chunk_ok(exec) || !tile_shape_ok(exec)) return IT_EINVAL;
  if (exec && exec->tile_x == 128) return IT_ENOTSUP;  // the batched kernel has no tiles of column pairs
  const int T = batch_steps(ch, ninst, exec);
  const int rc = check_batch_steps(ch, ninst, exec, T);
  if (rc) return rc;
  const int rows = batch_rows(ch, ninst, exec);
  const int R = T > 1 ? blocked_rows(T, exec ? exec->tile_y : 0) : 0;
  const int tile_x = exec_tile_x(exec, ch, ninst, false);
  *bytes = make_batch_layout(ch, track_offsets, ninst, rows, exec, tile_x, T, R).total;
  // with a pulse train the library's choice falls back to one step per pass
  // when a period is shorter than T steps (known only once the time steps
  // are): room for both
  bool train = false;
  for (int q = 0; q < ninst; ++q) train = train || ch[q].n_pulses >= 2;
  if (train && T > 1 && requested_steps(exec) == 0)
    *bytes = std::max(*bytes, make_batch_layout(ch, track_offsets, ninst, rows, exec, tile_x, 1, 0).total);
  return IT_OK;
}

int it_solve_batch(const it_chamber* ch, const int64_t* track_offsets, const it_track* tracks,
                   int32_t ninst, const it_exec* exec, void* d_workspace, size_t ws_bytes, void* stream_,
                   it_result* out) {
  clear_stale_error();
  if (!out) return IT_EINVAL;
  int rc = check_batch(ch, track_offsets, tracks, ninst);
  if (rc) return rc;
  const int rows = batch_rows(ch, ninst, exec);
  bool any_sc = false;
  bool any_ab = false;
  bool any_pu = false;
  for (int q = 0; q < ninst; ++q) {
    any_sc = any_sc || ch[q].space_charge != 0;
    any_ab = any_ab || ch[q].lateral_bc != 0;
    any_pu = any_pu || ch[q].n_pulses >= 2;
  }
  int passes_per_graph = exec && exec->check_every > 0 ? exec->check_every : 32;
  passes_per_graph += passes_per_graph & 1;  // even: the field parity repeats
  if (!z_chunk_ok(exec) || !tile_shape_ok(exec)) return IT_EINVAL;
  if (exec && exec->tile_x == 128) return IT_ENOTSUP;  // the batched kernel has no tiles of column pairs
  int T = batch_steps(ch, ninst, exec);  // steps per pass
  rc = check_batch_steps(ch, ninst, exec, T);
  if (rc) return rc;
  // every instance's time step (and a train's steps per period) before any
  // device work: a pass of T steps takes at most one pulse, so a train with
  // a shorter period needs one step per pass
  std::vector<double> dts(ninst);
  std::vector<int64_t> period_steps(ninst);
  bool short_period = false;
  for (int q = 0; q < ninst; ++q) {
    const int64_t n = track_offsets[q + 1] - track_offsets[q];
    const it_track* tq = n ? tracks + track_offsets[q] : nullptr;
    rc = compute_dt(&ch[q], tq, n, &dts[q], &period_steps[q]);
    if (rc) return rc;
    for (int64_t k = 0; k < n; ++k)
      if (deposit_step(tq[k].t_s, dts[q]) != 0) return IT_ENOTSUP;  // one pulse (or a train of it) per instance
    short_period = short_period || (ch[q].n_pulses >= 2 && period_steps[q] < T);
  }
  if (short_period) {
    if (requested_steps(exec) > 0) return IT_ENOTSUP;
    T = 1;
  }
  const int R = T > 1 ? blocked_rows(T, exec ? exec->tile_y : 0) : 0;
  const int tile_x = exec_tile_x(exec, ch, ninst, false);
  const BatchLayout B = make_batch_layout(ch, track_offsets, ninst, rows, exec, tile_x, T, R);
  if (!d_workspace || ws_bytes < B.total) return IT_EWORKSPACE;
  hipStream_t stream = (hipStream_t)stream_;
  char* ws = (char*)d_workspace;
  RunState* states = (RunState*)(ws + B.off_states);

  std::vector<BatchInstance> table(ninst);
  std::vector<int> active(ninst);
  for (int q = 0; q < ninst; ++q) active[q] = q;
  // blocked tiles: chunks of the caller's (or default) length while the
  // batch fills the machine, shorter ones when it does not (re-chosen for
  // the running instances whenever the table is rebuilt)
  const int z0 = T > 1 ? batch_blocked_z_chunk(exec) : 0;
  const int zc_run = T > 1 ? batch_blocked_retile_z(ch, active.data(), ninst, T, R, z0) : 0;
  int total_tiles = 0;
  int64_t max_steps_all = 0;
  for (int q = 0; q < ninst; ++q) {
    const it_chamber* c = &ch[q];
    const int64_t n = track_offsets[q + 1] - track_offsets[q];
    const it_track* tq = n ? tracks + track_offsets[q] : nullptr;
    const bool train = c->n_pulses >= 2;
    const int64_t m = period_steps[q];
    const InstLayout& L = B.inst[q];
    for (int f = 0; f < 4; ++f)
      HIP_TRY(hipMemsetAsync(ws + L.off_field[f], 0, L.field_elems * sizeof(double), stream));
    HIP_TRY(hipMemsetAsync(ws + L.off_counter, 0, 64 * sizeof(unsigned), stream));
    std::vector<DepTrack> dev(n);
    for (int64_t k = 0; k < n; ++k) {  // parallel tracks first, as the kernel expects
      dev[k] = prepare_track(c, tq[k]);
    }
    std::stable_partition(dev.begin(), dev.end(), [](const DepTrack& d) { return d.ux == 0.0 && d.uy == 0.0; });
    int64_t npar = 0;
    while (npar < n && dev[npar].ux == 0.0 && dev[npar].uy == 0.0) ++npar;
    if (n) HIP_TRY(hipMemcpyAsync(ws + L.off_tracks, dev.data(), n * sizeof(DepTrack), hipMemcpyHostToDevice, stream));

    const Coef cp = species_coef(c, dts[q], 0), cn = species_coef(c, dts[q], 1);
    const double dz = c->gap / c->nz, dV = c->dx * c->dy * dz;
    const Tiling ts = batch_tiling(*c, T, R, rows, exec, tile_x, zc_run);
    const Tiling td = deposit_tiling(c->nx, c->ny, c->nz);
    BatchInstance& bi = table[q];
    for (int par = 0; par < 2; ++par) {
      StepParams& sp = bi.sp[par];
      std::memset(&sp, 0, sizeof(sp));
      sp.pin = (double*)(ws + L.off_field[2 * par]);
      sp.nin = (double*)(ws + L.off_field[2 * par + 1]);
      sp.pout = (double*)(ws + L.off_field[2 * (1 - par)]);
      sp.nout = (double*)(ws + L.off_field[2 * (1 - par) + 1]);
      sp.nx = c->nx;
      sp.ny = c->ny;
      sp.nz = c->nz;
      sp.tiles_x = ts.tiles_x;
      sp.tiles_y = ts.tiles_y;
      sp.zchunks = ts.zchunks;
      sp.zc = ts.zc;
      sp.ntiles = ts.ntiles;
      sp.per_xcd = ts.per_xcd;
      sp.cp = cp;
      sp.cn = cn;
      sp.beta = c->alpha * dts[q];
      sp.gsp = screening_coef(c, dts[q], 0);
      sp.gsn = screening_coef(c, dts[q], 1);
      sp.absorbing = c->lateral_bc;
      sp.dV = dV;
      sp.stop_tol = c->stop_tol;
      sp.step0 = 0;
      sp.min_stop_step = train ? INT64_MAX : 0;  // a pulse train ends with its last period
      sp.partials = (double*)(ws + L.off_partials) + (size_t)par * L.slots * kAcc * T;
      sp.counter = (unsigned*)(ws + L.off_counter);
      sp.state = states + q;
      sp.trace = nullptr;
    }
    bi.tile_begin = total_tiles;
    bi.ntiles = ts.ntiles;
    bi.max_steps = train ? std::min<int64_t>(c->max_steps, c->n_pulses * m) : c->max_steps;
    bi.npulses = train ? c->n_pulses : 0;
    bi.period_steps = m;
    bi.pulse_pos = train ? (const double*)(ws + L.off_pulse[0]) : nullptr;
    bi.pulse_neg = train ? (const double*)(ws + L.off_pulse[1]) : nullptr;
    total_tiles += ts.ntiles;
    max_steps_all = std::max(max_steps_all, bi.max_steps);
    // the pulse: uniform pre-ionisation and the tracks, deposited before step 0
    RunState init = initial_run_state();
    init.rec_ntiles = ts.ntiles;  // the priming pass's tiles
    if (train) {
      // pulse 0 is deposited and booked here; the first two passes (steps
      // 0 .. T-1 and T .. 2T-1), whose flags no recording block sets, take
      // the pulses due at steps 1 .. T and T+1 .. 2T (a pass adds a pulse
      // at step c0 + j to the outputs of its level j)
      init.period_step = (c->n_pulses - 1) * m;
      init.pulses_counted = 1;
      init.pulses_flagged = 1;
      for (int pass = 0; pass < 2; ++pass) {
        const int64_t c0 = (int64_t)pass * T, s = (int64_t)init.pulses_flagged * m;
        if (init.pulses_flagged < c->n_pulses && s > c0 && s <= c0 + T && s < bi.max_steps) {
          init.pulse_add[pass] = (int)(s - c0);
          ++init.pulses_flagged;
        }
      }
    }
    HIP_TRY(hipMemcpyAsync(states + q, &init, sizeof(init), hipMemcpyHostToDevice, stream));
    if (n || c->uniform_n0 > 0.0) {
      DepositParams dp = base_deposit(c, dts[q], td);
      dp.pos = (double*)(ws + L.off_field[0]);
      dp.neg = (double*)(ws + L.off_field[1]);
      dp.uniform = c->uniform_n0;
      dp.par = (const DepTrack*)(ws + L.off_tracks);
      dp.npar = (int)npar;
      dp.tilt = (const DepTrack*)(ws + L.off_tracks) + npar;
      dp.ntilt = (int)(n - npar);
      dp.same_radii = same_radii(tq, n);
      dp.partials = (double*)(ws + L.off_partials);
      dp.counter = (unsigned*)(ws + L.off_counter);
      dp.state = states + q;
      HIP_TRY(launch_deposit(dp, stream));
    }
    if (train)  // the first pulse's densities (the fields held zero before it)
      for (int f = 0; f < 2; ++f)
        HIP_TRY(hipMemcpyAsync(ws + L.off_pulse[f], ws + L.off_field[f], L.field_elems * sizeof(double),
                               hipMemcpyDeviceToDevice, stream));
  }
  // The pass chain runs on the tile list of the running instances only: the
  // table is rebuilt (and the graph re-captured) whenever a quarter of its
  // instances have stopped, so finished chambers cost no dispatches.  All
  // running instances have executed the same number of passes, so they
  // share the field parity and a rebuilt table keeps the graph's pattern.
  HostSlots hs;
  host_slots(exec, ninst, hs);
  RunState* host = hs.p;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec_graph = nullptr;
  auto release_graph = [&]() {
    if (exec_graph) (void)hipGraphExecDestroy(exec_graph);
    if (graph) (void)hipGraphDestroy(graph);
    exec_graph = nullptr;
    graph = nullptr;
  };
  // Blocked tiles of the running instances in the chunk length that suits
  // them (a pass computed with the previous tiling is still reduced over its
  // own tiles: each recording block leaves its pass's tile count in the run
  // state for the next).
  auto retile = [&]() {
    if (T == 1) return;
    const int z = batch_blocked_retile_z(ch, active.data(), (int)active.size(), T, R, z0);
    for (int q : active) {
      const Tiling ts = batch_blocked_tiling(ch[q], T, R, z);
      for (int par = 0; par < 2; ++par) {
        StepParams& sp = table[q].sp[par];
        sp.tiles_x = ts.tiles_x;
        sp.tiles_y = ts.tiles_y;
        sp.zchunks = ts.zchunks;
        sp.zc = ts.zc;
        sp.ntiles = ts.ntiles;
        sp.per_xcd = ts.per_xcd;
      }
      table[q].ntiles = ts.ntiles;
    }
  };
  auto build = [&](int parity0) -> int {
    retile();
    std::vector<BatchInstance> t;
    t.reserve(active.size());
    int tiles = 0;
    for (int q : active) {
      BatchInstance bi = table[q];
      bi.tile_begin = tiles;
      tiles += bi.ntiles;
      t.push_back(bi);
    }
    if (hipMemcpyAsync(ws + B.off_table, t.data(), t.size() * sizeof(BatchInstance), hipMemcpyHostToDevice,
                       stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)  // t is pageable and local
      return IT_EHIP;
    release_graph();
    // a chain of kernel nodes, each pass depending on the one before
    if (hipGraphCreate(&graph, 0) != hipSuccess) return IT_EHIP;
    hipGraphNode_t prev = nullptr;
    for (int k = 0; k < passes_per_graph; ++k) {
      hipGraphNode_t node = nullptr;
      if (add_batch_pass_node(graph, prev, &node, ws + B.off_table, (int)t.size(), tiles, rows, tile_x, any_sc,
                              any_ab, any_pu, (parity0 + k) & 1, T, R) != hipSuccess)
        return IT_EHIP;
      prev = node;
    }
    if (hipGraphInstantiate(&exec_graph, graph, nullptr, nullptr, 0) != hipSuccess) return IT_EHIP;
    return IT_OK;
  };
  // Pass p computes step p of every running instance and records step p-1
  // (the extra blocks of its launch reduce the previous pass's partials), so
  // a first pass that only steps primes the chain; the graph's passes
  // continue from parity 1.
  rc = build(1);
  if (rc) {
    release_graph();
    return rc;
  }
  {
    int tiles = 0;
    for (int q = 0; q < ninst; ++q) tiles += table[q].ntiles;
    if (launch_batch_pass(ws + B.off_table, ninst, tiles, rows, tile_x, any_sc, any_ab, any_pu, 0, false, T, R,
                          stream) !=
        hipSuccess) {
      release_graph();
      return IT_EHIP;
    }
  }
  (void)total_tiles;
  // Replays until every instance has stopped; two replays in flight so the
  // GPU never idles on the read-back.
  const int64_t steps_per_replay = (int64_t)passes_per_graph * T;
  const int64_t max_replays = (max_steps_all + steps_per_replay - 1) / steps_per_replay + 1;
  hipEvent_t evs[2];
  HIP_TRY(hipEventCreateWithFlags(&evs[0], hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&evs[1], hipEventDisableTiming));
  int issued = 1;  // the priming pass
  int64_t replays_since_build = 0;
  rc = IT_OK;
  for (int64_t r = 0; r < max_replays; ++r) {
    if (hipGraphLaunch(exec_graph, stream) != hipSuccess) { rc = IT_EHIP; break; }
    issued += passes_per_graph;
    ++replays_since_build;
    RunState* slot = host + (r & 1) * ninst;
    if (hipMemcpyAsync(slot, states, (size_t)ninst * sizeof(RunState), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipEventRecord(evs[r & 1], stream) != hipSuccess) { rc = IT_EHIP; break; }
    if (!hs.pinned) {  // an ordinary host buffer: the copy of this replay completes first
      if (hipStreamSynchronize(stream) != hipSuccess) { rc = IT_EHIP; break; }
      bool any = false;
      for (int q : active) any = any || !slot[q].done;
      if (!any) break;
    }
    if (r >= 1) {
      RunState* prev = host + ((r - 1) & 1) * ninst;
      if (hipEventSynchronize(evs[(r - 1) & 1]) != hipSuccess) { rc = IT_EHIP; break; }
      std::vector<int> still;
      for (int q : active)
        if (!prev[q].done) still.push_back(q);
      if (still.empty()) break;
      // rebuild only once the replay in flight has finished too, so that no
      // launch still reads the table being replaced
      if (4 * still.size() <= 3 * active.size() && replays_since_build >= 2) {
        if (hipStreamSynchronize(stream) != hipSuccess) { rc = IT_EHIP; break; }
        RunState* now = host + (r & 1) * ninst;
        still.clear();
        for (int q : active)
          if (!now[q].done) still.push_back(q);
        if (still.empty()) break;
        active.swap(still);
        rc = build((int)(((int64_t)issued) & 1));
        if (rc) break;
        replays_since_build = 0;
      }
    }
  }
  if (rc == IT_OK && (hipMemcpyAsync(host, states, (size_t)ninst * sizeof(RunState), hipMemcpyDeviceToHost, stream) != hipSuccess ||
                      hipStreamSynchronize(stream) != hipSuccess))
    rc = IT_EHIP;
  (void)hipEventDestroy(evs[0]);
  (void)hipEventDestroy(evs[1]);
  release_graph();
  if (rc) return rc;
  for (int q = 0; q < ninst; ++q) {
    fill_result(host[q], dts[q], ch[q].max_steps, issued, &out[q]);
    train_result(host[q], &ch[q], period_steps[q], &out[q]);
  }
  return IT_OK;
}

int it_advance(const it_chamber* ch, double dt, int64_t nsteps, const it_exec* exec, double* d_pos,
               double* d_neg, void* d_workspace, size_t ws_bytes, void* stream_, double* h_trace) {
  clear_stale_error();
  int rc = check_chamber(ch);
  if (rc) return rc;
  // the fields come back after exactly nsteps steps with either kernel
  const int T = exec_steps(ch, exec, false);
  rc = check_exec_ws(ch, exec, T, d_workspace);
  if (rc) return rc;
  if (!d_pos || !d_neg || nsteps < 0 || nsteps > ch->max_steps) return IT_EINVAL;
  if (!(std::isfinite(dt) && dt > 0)) return IT_EINVAL;
  const Layout L = make_layout(ch, 0);
  if (!d_workspace || ws_bytes < L.total) return IT_EWORKSPACE;
  if (nsteps == 0) return IT_OK;
  hipStream_t stream = (hipStream_t)stream_;
  char* ws = (char*)d_workspace;
  const size_t plane = (size_t)ch->nx * ch->ny * sizeof(double);
  const size_t bytes = L.field_elems * sizeof(double);
  HIP_TRY(hipMemcpyAsync(ws + L.off_field[0], d_pos, bytes, hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipMemcpyAsync(ws + L.off_field[1], d_neg, bytes, hipMemcpyDeviceToDevice, stream));
  for (int f = 0; f < 2; ++f) {  // electrode planes of the input pair are zero by definition
    HIP_TRY(hipMemsetAsync(ws + L.off_field[f], 0, plane, stream));
    HIP_TRY(hipMemsetAsync(ws + L.off_field[f] + (size_t)ch->nz * plane, 0, plane, stream));
  }
  for (int f = 2; f < 4; ++f) HIP_TRY(hipMemsetAsync(ws + L.off_field[f], 0, bytes, stream));
  HIP_TRY(hipMemsetAsync(ws + L.off_counter, 0, 64 * sizeof(unsigned), stream));
  const RunState init = initial_run_state();
  HIP_TRY(hipMemcpyAsync(ws + L.off_state, &init, sizeof(init), hipMemcpyHostToDevice, stream));
  std::vector<Event> none;
  std::vector<DepTrack> nodev;
  RunState fin;
  int issued = 0;
  HostSlots hs;
  host_slots(exec, 1, hs);
  rc = run_loop(ch, dt, exec, ws, L, none, nodev, 1, nsteps, INT64_MAX, 0.0, T, stream, hs, &fin, &issued);
  if (rc) return rc;
  const int last = fin.passes & 1;
  HIP_TRY(hipMemcpyAsync(d_pos, ws + L.off_field[2 * last], bytes, hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipMemcpyAsync(d_neg, ws + L.off_field[2 * last + 1], bytes, hipMemcpyDeviceToDevice, stream));
  if (h_trace)
    HIP_TRY(hipMemcpyAsync(h_trace, ws + L.off_trace, (size_t)nsteps * IT_TRACE_COLS * sizeof(double),
                           hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return IT_OK;
}

}  // extern "C"
