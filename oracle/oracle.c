/*
 * Plain FP64 CPU oracle of the IonTracks recombination solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no source, header or table with the GPU library; the two
 * only see the same input dictionaries and track arrays.
 *
 * The arithmetic follows the paper step by step, written for clarity, not
 * speed: plain triple loops, no blocking, no fusion.  Every grid sum (the
 * per-step tallies, the released counts of a deposit) is taken plane by
 * plane into per-plane partial sums, which are then added in plane order.
 * The order of every floating-point operation is therefore fixed by the
 * grid alone: the default build is single-threaded, and a timing build with
 * OpenMP (-fopenmp: the plane loops are shared among threads) returns the
 * same bits.
 *
 *   - linear ion-pair density N0 = LET / W                    (eq. linear_density)
 *   - Gaussian radial track profile n0(r) = N0/(pi b^2) e^{-r^2/b^2}   (eq. Gaussian),
 *     optionally with a separate radius b- for the negative ions (the paper
 *     notes b- > b+ and that separate radii are a direct extension)
 *   - transport  dn/dt = D lap n -/+ mu (E . grad n + n div E) - alpha n+ n-
 *     (eq. theEquation): E in E . grad n is the uniform applied field; with
 *     space charge on, div E comes from the local net charge by the
 *     Maxwell-Gauss law, div E = q (n+ - n-) / eps0 (same section), else 0
 *   - grid x_i = i dx, ..., t_l = l dt and the weights c = mu E dt/dz,
 *     s = D dt/dx^2                                            (Appendix)
 *   - forward time difference, the drift derivative that blends a backward
 *     and a central difference with weight c, the 3-point second difference
 *                                                             (Appendix)
 *   - the largest dt obeying 2(sx+sy+sz) + cx^2+cy^2+cz^2 <= 1 and
 *     cx^2 cy^2 cz^2 <= 8 sx sy sz for both species           (eq. vNeum),
 *     optionally also (alpha + sc) dt n_ref <= rho (see orc_dt)
 *   - electrodes at z=0 and z=d hold zero density; charge reaching them is
 *     collected                                                 (Methods, Implementation)
 *   - f = N_collected / N_released                              (eq. collection_efficiency)
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - x and y are periodic by default; the transverse cell is nx*dx by
 *     ny*dy.  Optionally (lateral_bc = 1) they are absorbing instead: the
 *     nodes just outside the cell hold zero, like the electrodes, and what
 *     they would receive in a step is tallied as escaped.
 *   - c carries the sign of the drift velocity (+mu E for positive ions,
 *     -mu E for negative ions).  With that sign the paper's blended drift
 *     derivative is exactly the Lax-Wendroff update.
 *   - both species are updated from the old densities (Jacobi), so each node
 *     removes the same beta n+ n- from both species (beta = alpha dt).
 *   - "collected" in step l is what the pinned electrode plane would have
 *     received from its interior neighbour in that step.
 *   - N_released is the discrete sum of the deposited density times the
 *     voxel volume.
 *   - a track is deposited at the start of step floor(t/dt); the axis passes
 *     through (x0, y0, d/2) with direction (sin th cos ph, sin th sin ph, cos th);
 *     the transverse offset is wrapped to the nearest periodic image and the
 *     profile is cut at r <= 8b.
 *   - the run stops after the first step at which every track has been
 *     deposited and, for both species, the sum of |n| dV over the grid is
 *     <= stop_tol * N_released (the signed sum can dip below zero while
 *     Lax-Wendroff undershoots are still in flight, so it is not used).
 *   - a pulsed beam of repetition period P (Distribution of ion tracks: a
 *     beam in time as instantaneous pulses): with n_pulses = N >= 2 the
 *     chamber's deposits -- the uniform pre-ionisation and every track, all
 *     due at t = 0 -- repeat every period, N times.  A period is m =
 *     ceil(P / dt) whole steps, the time step shortened to P / m (so every
 *     period has the same steps and a periodic state can be reached
 *     exactly), and pulse k is deposited at the start of step k m.  The run
 *     covers steps 0 .. N m - 1, with no collection test.  The last period,
 *     steps (N-1) m .. N m - 1, gives the result:
 *     f = charge collected in it / charge one pulse releases (both signs),
 *     f_R = 1 - pairs recombined in it / pairs one pulse releases.  Once the
 *     pulses have reached a periodic steady state, what one pulse releases
 *     is collected or recombined within one period, so both are the
 *     collection efficiency of a pulse in the train.
 *
 * Layout: each species is an array [nz+1][ny][nx] (x fastest) whose planes
 * k = 0 and k = nz are the electrodes and always hold zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* parameter vector (mirrors the chamber dictionary) */
enum {
  P_DX, P_DY, P_GAP, P_VOLT, P_MU_POS, P_MU_NEG, P_D_POS, P_D_NEG,
  P_ALPHA, P_W, P_KAPPA, P_STOP_TOL, P_UNIFORM_N0, P_SPACE_CHARGE, P_REACTION_LIMIT,
  P_ATTACH, P_MU_E, P_D_E, P_LATERAL_BC, P_N_PULSES, P_PULSE_PERIOD, P_COUNT
};
/* result vector */
enum {
  R_F, R_KS, R_F_RECOMB, R_RELEASED, R_RECOMBINED, R_INFLIGHT_POS, R_INFLIGHT_NEG,
  R_COL_POS_ANODE, R_COL_POS_CATHODE, R_COL_NEG_ANODE, R_COL_NEG_CATHODE,
  R_DT, R_STEPS, R_FLAGS, R_MAX_BETA_N, R_SC_POS, R_SC_NEG, R_RELEASED_NEG, R_ESC_POS, R_ESC_NEG,
  R_PULSES, R_PERIOD_RELEASED, R_PERIOD_COLLECTED, R_PERIOD_RECOMBINED, R_COUNT
};
/* per-step record */
enum { T_RECOMB, T_POS_ANODE, T_POS_CATHODE, T_NEG_ANODE, T_NEG_CATHODE, T_POS_INFLIGHT, T_NEG_INFLIGHT,
       T_POS_ABS, T_NEG_ABS, T_RELEASED, T_POS_SC, T_NEG_SC, T_RELEASED_NEG, T_POS_ESC, T_NEG_ESC, T_COUNT };

/* track record: {let_keV_um, b, x0, y0, theta, phi, t, b_neg}; b_neg = 0
 * means the negative ions share the radius b */
#define TRK 8

/* elementary charge [C] and vacuum permittivity [F/cm] (CODATA 2018) */
#define Q_E 1.602176634e-19
#define EPS0 8.8541878128e-14

#define FLAG_MAX_STEPS 1
#define FLAG_NONFINITE 2
#define FLAG_REACTION 4
#define FLAG_EMPTY 8

#define IDX(k, j, i) (((size_t)(k) * (size_t)ny + (size_t)(j)) * (size_t)nx + (size_t)(i))

/* Threads the plane loops use: 1 in the default build. */
int orc_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Largest dt satisfying eq. vNeum for both species (no safety factor).
 * With the field along z only, cx = cy = 0: the product condition holds
 * trivially and the first condition is A dt + B dt^2 <= 1 with
 * A = 2 D (1/dx^2 + 1/dy^2 + 1/dz^2) and B = (mu E / dz)^2.
 * Returns INFINITY if neither species constrains dt (no drift, no diffusion). */
static double transport_dt(const double *p, int64_t nz)
{
  const double dz = p[P_GAP] / (double)nz;
  const double E = p[P_VOLT] / p[P_GAP];
  const double inv2 = 1.0 / (p[P_DX] * p[P_DX]) + 1.0 / (p[P_DY] * p[P_DY]) + 1.0 / (dz * dz);
  const double mus[2] = {p[P_MU_POS], p[P_MU_NEG]};
  const double Ds[2] = {p[P_D_POS], p[P_D_NEG]};
  double best = INFINITY;
  for (int s = 0; s < 2; ++s) {
    const double A = 2.0 * Ds[s] * inv2;
    const double v = mus[s] * E / dz;
    const double B = v * v;
    double root;
    if (B > 0.0)
      root = 2.0 / (A + sqrt(A * A + 4.0 * B)); /* positive root of B t^2 + A t - 1 */
    else if (A > 0.0)
      root = 1.0 / A;
    else
      continue;
    if (root < best) best = root;
  }
  return best;
}

/* Weights of the Appendix for species s (0 = positive, 1 = negative):
 * w = {c, sx, sy, sz}, c signed with the drift velocity along +z. */
void orc_weights(const double *p, int64_t nz, double dt, int s, double *w)
{
  const double dz = p[P_GAP] / (double)nz;
  const double E = p[P_VOLT] / p[P_GAP];
  const double mu = s == 0 ? p[P_MU_POS] : p[P_MU_NEG];
  const double D = s == 0 ? p[P_D_POS] : p[P_D_NEG];
  const double v = s == 0 ? mu * E : -mu * E;
  w[0] = v * dt / dz;
  w[1] = D * dt / (p[P_DX] * p[P_DX]);
  w[2] = D * dt / (p[P_DY] * p[P_DY]);
  w[3] = D * dt / (dz * dz);
}

static double wrap(double d, double L)
{
  return d - L * floor(d / L + 0.5);
}

/* Transverse offset of a point from a track axis: wrapped to the nearest
 * periodic image, or as it is with absorbing lateral boundaries. */
static double lateral_offset(const double *p, double d, double L)
{
  return p[P_LATERAL_BC] != 0.0 ? d : wrap(d, L);
}

/* Axis direction of a track: (sin th cos ph, sin th sin ph, cos th). */
static void track_axis(const double *tr, double *u)
{
  u[0] = sin(tr[4]) * cos(tr[5]);
  u[1] = sin(tr[4]) * sin(tr[5]);
  u[2] = cos(tr[4]);
}

/* Gaussian radius of species s (0 = positive, 1 = negative) of a track. */
static double track_radius(const double *tr, int s)
{
  return s == 1 && tr[7] > 0.0 ? tr[7] : tr[1];
}

/* Gaussian track profile of eq. Gaussian at node (i,j,k) for species s,
 * 0 beyond 8b.  u = axis direction. */
static double track_density(const double *p, int64_t nx, int64_t ny, int64_t nz,
                            const double *tr, const double *u, int s, int64_t i, int64_t j, int64_t k)
{
  const double dz = p[P_GAP] / (double)nz;
  const double N0 = tr[0] * 1.0e7 / p[P_W]; /* keV/um -> eV/cm, divided by W: pairs/cm */
  const double b = track_radius(tr, s);
  const double wx = lateral_offset(p, (double)i * p[P_DX] - tr[2], (double)nx * p[P_DX]);
  const double wy = lateral_offset(p, (double)j * p[P_DY] - tr[3], (double)ny * p[P_DY]);
  const double wz = (double)k * dz - 0.5 * p[P_GAP];
  /* squared distance from the axis: |w x u|^2 */
  const double cx = wy * u[2] - wz * u[1];
  const double cy = wz * u[0] - wx * u[2];
  const double cz = wx * u[1] - wy * u[0];
  const double r2 = cx * cx + cy * cy + cz * cz;
  if (r2 > 64.0 * b * b) return 0.0;
  return N0 / (M_PI * b * b) * exp(-r2 / (b * b));
}

/* Density that track tr deposits at the point (x, y, z) (same rule as at
 * the nodes: wrapped transverse offset, 8b cut-off). */
static double track_density_at(const double *p, int64_t nx, int64_t ny, const double *tr,
                               const double *u, int s, double x, double y, double z)
{
  const double N0 = tr[0] * 1.0e7 / p[P_W];
  const double b = track_radius(tr, s);
  const double wx = lateral_offset(p, x - tr[2], (double)nx * p[P_DX]);
  const double wy = lateral_offset(p, y - tr[3], (double)ny * p[P_DY]);
  const double wz = z - 0.5 * p[P_GAP];
  const double cx = wy * u[2] - wz * u[1];
  const double cy = wz * u[0] - wx * u[2];
  const double cz = wx * u[1] - wy * u[0];
  const double r2 = cx * cx + cy * cy + cz * cz;
  if (r2 > 64.0 * b * b) return 0.0;
  return N0 / (M_PI * b * b) * exp(-r2 / (b * b));
}

/* Reference peak density for the recombination bound on dt: the uniform
 * pre-ionisation plus, over all tracks and both species, the largest density
 * found on a track's axis at mid-gap from every track that arrives at the
 * same time. */
double orc_reference_density(const double *p, int64_t nx, int64_t ny, const double *trk, int64_t ntr)
{
  double best = 0.0;
  for (int64_t t = 0; t < ntr; ++t) {
    const double *a = trk + TRK * t;
    for (int sp = 0; sp < 2; ++sp) {
      double s = 0.0;
      for (int64_t q = 0; q < ntr; ++q) {
        const double *tr = trk + TRK * q;
        if (tr[6] != a[6]) continue;
        double u[3];
        track_axis(tr, u);
        s += track_density_at(p, nx, ny, tr, u, sp, a[2], a[3], 0.5 * p[P_GAP]);
      }
      if (s > best) best = s;
    }
  }
  return p[P_UNIFORM_N0] + best;
}

/* Time step: the largest dt of eq. vNeum, further limited (when the
 * reaction limit rho > 0) so that (alpha + sc) dt n_ref <= rho: the explicit
 * recombination sink n' = n - alpha dt n+ n- diverges once alpha dt n
 * exceeds about 1, which the transport bound alone does not prevent at
 * dense track cores.  With space charge on, sc = max(mu+, mu-) q / eps0 is
 * the rate constant of the screening term, whose explicit update
 * n' = n -/+ mu dt (q/eps0) n (n+ - n-) needs the same bound (dielectric
 * relaxation).  The safety factor kappa multiplies the result.
 * Returns 0, or -2 if nothing bounds dt. */
int orc_dt(const double *p, int64_t nx, int64_t ny, int64_t nz, const double *trk, int64_t ntr,
           double *dt)
{
  double best = transport_dt(p, nz);
  const double rho = p[P_REACTION_LIMIT];
  double rate = p[P_ALPHA];
  if (p[P_SPACE_CHARGE] != 0.0) {
    const double mu_max = p[P_MU_POS] > p[P_MU_NEG] ? p[P_MU_POS] : p[P_MU_NEG];
    rate += mu_max * Q_E / EPS0;
  }
  if (rho > 0.0 && rate > 0.0) {
    const double nref = orc_reference_density(p, nx, ny, trk, ntr);
    if (nref > 0.0) {
      const double dtr = rho / (rate * nref);
      if (dtr < best) best = dtr;
    }
  }
  if (!(best < INFINITY)) return -2;
  *dt = p[P_KAPPA] * best;
  return 0;
}

int64_t orc_deposit_step(double dt, const double *tr)
{
  const double s = floor(tr[6] / dt);
  if (s > 4.0e18) return INT64_MAX;
  return (int64_t)s;
}

/* Add every track due at step `step` (list order) to both species, or
 * every track when `all` is set (a pulse of a pulse train, whose tracks are
 * all due at its start).  released[0], released[1]: ions of each species
 * released (sum of density times dV); equal unless the track gives the
 * negative ions their own radius. */
static void deposit_tracks(const double *p, int64_t nx, int64_t ny, int64_t nz,
                           const double *trk, int64_t ntr, int64_t step, double dt, int all,
                           double *pos, double *neg, double *released)
{
  const double dV = p[P_DX] * p[P_DY] * (p[P_GAP] / (double)nz);
  released[0] = released[1] = 0.0;
  double *plane_sum = (double *)calloc((size_t)(nz + 1) * 2, sizeof(double));
  if (!plane_sum) { released[0] = released[1] = NAN; return; }
  for (int64_t t = 0; t < ntr; ++t) {
    const double *tr = trk + TRK * t;
    if (!all && orc_deposit_step(dt, tr) != step) continue;
    double u[3];
    track_axis(tr, u);
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k < nz; ++k) {
      double sp = 0.0, sn = 0.0;
      for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
          const double dp = track_density(p, nx, ny, nz, tr, u, 0, i, j, k);
          const double dn = track_density(p, nx, ny, nz, tr, u, 1, i, j, k);
          pos[IDX(k, j, i)] += dp;
          neg[IDX(k, j, i)] += dn;
          sp += dp;
          sn += dn;
        }
      plane_sum[2 * k] = sp;
      plane_sum[2 * k + 1] = sn;
    }
    double sum[2] = {0.0, 0.0};
    for (int64_t k = 1; k < nz; ++k) {
      sum[0] += plane_sum[2 * k];
      sum[1] += plane_sum[2 * k + 1];
    }
    released[0] += sum[0] * dV;
    released[1] += sum[1] * dV;
  }
  free(plane_sum);
}

/* Add every track due at step `step` (list order) to both species. */
void orc_deposit(const double *p, int64_t nx, int64_t ny, int64_t nz,
                 const double *trk, int64_t ntr, int64_t step, double dt,
                 double *pos, double *neg, double *released)
{
  deposit_tracks(p, nx, ny, nz, trk, ntr, step, dt, 0, pos, neg, released);
}

/* Uniform pre-ionisation n0 of both species at every interior node. */
double orc_uniform(const double *p, int64_t nx, int64_t ny, int64_t nz, double n0,
                   double *pos, double *neg)
{
  const double dV = p[P_DX] * p[P_DY] * (p[P_GAP] / (double)nz);
  for (int64_t k = 1; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        pos[IDX(k, j, i)] += n0;
        neg[IDX(k, j, i)] += n0;
      }
  return n0 * dV * (double)(nx * ny * (nz - 1));
}

/* Density of n at interior node (k, j, i) displaced by (dj, di) laterally:
 * the periodic image, or 0 beyond an absorbing lateral boundary. */
static double lateral_neighbour(const double *p, int64_t nx, int64_t ny, const double *n,
                                int64_t k, int64_t j, int64_t i, int64_t dj, int64_t di)
{
  int64_t jj = j + dj, ii = i + di;
  if (p[P_LATERAL_BC] != 0.0) {
    if (jj < 0 || jj >= ny || ii < 0 || ii >= nx) return 0.0;
  } else {
    jj = (jj + ny) % ny;
    ii = (ii + nx) % nx;
  }
  return n[IDX(k, jj, ii)];
}

/* One explicit step of eq. theEquation for both species from the old
 * densities (pos, neg) into (npos, nneg).  tally receives the per-step
 * record (T_*), all in ion counts (density times dV): recombined pairs,
 * collected at each electrode per species, in-flight per species (signed
 * sum of the new densities), the sum of the new |n| per species, the
 * change of each species by the space-charge term, and, with absorbing
 * lateral boundaries, what left each species through them.  The released
 * slot (released before this step) is left at 0 here; the run fills it.
 *
 * For every interior node and species, with the Appendix's derivatives:
 *   dn/dz  ~ c (n_k - n_{k-1})/dz + (1-c)(n_{k+1} - n_{k-1})/(2 dz)
 *   d2n/dx2 ~ (n_{i+1} - 2 n_i + n_{i-1})/dx^2 (and y, z)
 *   n' = n + dt [D lap n - v dn/dz] - alpha dt n+ n- -/+ mu dt n div E
 * where v is the signed drift velocity, c = v dt/dz, and, with space
 * charge on, div E = q (n+ - n-)/eps0 at the node (old densities). */
void orc_step(const double *p, int64_t nx, int64_t ny, int64_t nz, double dt,
              const double *pos, const double *neg, double *npos, double *nneg,
              double *tally)
{
  const double dz = p[P_GAP] / (double)nz;
  const double dV = p[P_DX] * p[P_DY] * dz;
  const double beta = p[P_ALPHA] * dt;
  double w[2][4];
  orc_weights(p, nz, dt, 0, w[0]);
  orc_weights(p, nz, dt, 1, w[1]);
  const double *in[2] = {pos, neg};
  double *out[2] = {npos, nneg};
  const int absorbing = p[P_LATERAL_BC] != 0.0;
  /* per-plane partial sums: recombined, then in flight, |n|, space-charge
   * change and escaped for each species */
  enum { S_REC, S_IN0, S_IN1, S_ABS0, S_ABS1, S_SC0, S_SC1, S_ESC0, S_ESC1, S_N };
  double *part = (double *)calloc((size_t)(nz + 1) * S_N, sizeof(double));
  if (!part) {
    for (int q = 0; q < T_COUNT; ++q) tally[q] = NAN;
    return;
  }
  /* mu dt q/eps0 per species, signed as the term enters n' (- for n+, + for n-) */
  const double sc_on = p[P_SPACE_CHARGE] != 0.0 ? 1.0 : 0.0;
  const double gsc[2] = {-sc_on * p[P_MU_POS] * dt * Q_E / EPS0, sc_on * p[P_MU_NEG] * dt * Q_E / EPS0};

#pragma omp parallel for schedule(static)
  for (int64_t k = 1; k < nz; ++k) {
    double recomb = 0.0, inflight[2] = {0.0, 0.0}, absolute[2] = {0.0, 0.0}, screen[2] = {0.0, 0.0};
    double escaped[2] = {0.0, 0.0};
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        const double np_ = pos[IDX(k, j, i)], nn_ = neg[IDX(k, j, i)];
        const double sink = beta * np_ * nn_;
        recomb += sink;
        /* lateral neighbours missing beyond an absorbing boundary (a node
         * of a one-node-wide cell misses both) */
        const double miss_x = absorbing ? (double)((i == 0) + (i == nx - 1)) : 0.0;
        const double miss_y = absorbing ? (double)((j == 0) + (j == ny - 1)) : 0.0;
        for (int s = 0; s < 2; ++s) {
          const double *n = in[s];
          const double c = w[s][0], sx = w[s][1], sy = w[s][2], sz = w[s][3];
          const double nc = n[IDX(k, j, i)];
          const double lap_x = lateral_neighbour(p, nx, ny, n, k, j, i, 0, 1) - 2.0 * nc
                               + lateral_neighbour(p, nx, ny, n, k, j, i, 0, -1);
          const double lap_y = lateral_neighbour(p, nx, ny, n, k, j, i, 1, 0) - 2.0 * nc
                               + lateral_neighbour(p, nx, ny, n, k, j, i, -1, 0);
          /* a missing neighbour would have received sx n (or sy n) */
          escaped[s] += (sx * miss_x + sy * miss_y) * nc;
          const double lap_z = n[IDX(k + 1, j, i)] - 2.0 * nc + n[IDX(k - 1, j, i)];
          /* c * dz * (dn/dz) with the blended derivative */
          const double drift = c * (c * (nc - n[IDX(k - 1, j, i)])
                                    + (1.0 - c) * 0.5 * (n[IDX(k + 1, j, i)] - n[IDX(k - 1, j, i)]));
          const double screening = gsc[s] * nc * (np_ - nn_);
          const double v = nc + sx * lap_x + sy * lap_y + sz * lap_z - drift - sink + screening;
          out[s][IDX(k, j, i)] = v;
          screen[s] += screening;
          inflight[s] += v;
          absolute[s] += fabs(v);
        }
      }
    double *pk = part + (size_t)k * S_N;
    pk[S_REC] = recomb;
    pk[S_IN0] = inflight[0];
    pk[S_IN1] = inflight[1];
    pk[S_ABS0] = absolute[0];
    pk[S_ABS1] = absolute[1];
    pk[S_SC0] = screen[0];
    pk[S_SC1] = screen[1];
    pk[S_ESC0] = escaped[0];
    pk[S_ESC1] = escaped[1];
  }
  /* the planes' partial sums in plane order */
  double recomb = 0.0, inflight[2] = {0.0, 0.0}, absolute[2] = {0.0, 0.0}, screen[2] = {0.0, 0.0};
  double escaped[2] = {0.0, 0.0};
  for (int64_t k = 1; k < nz; ++k) {
    const double *pk = part + (size_t)k * S_N;
    recomb += pk[S_REC];
    for (int s = 0; s < 2; ++s) {
      inflight[s] += pk[S_IN0 + s];
      absolute[s] += pk[S_ABS0 + s];
      screen[s] += pk[S_SC0 + s];
      escaped[s] += pk[S_ESC0 + s];
    }
  }
  free(part);

  /* Collected in this step: what the electrode planes would receive from
   * their interior neighbours.  Plane 0 gets the weight of n_{k+1} from node
   * k=1; plane nz gets the weight of n_{k-1} from node k=nz-1. */
  double col[2][2];
  for (int s = 0; s < 2; ++s) {
    const double c = w[s][0], sz = w[s][3];
    const double w_up = sz + 0.5 * c * c - 0.5 * c;   /* weight of n_{k+1} */
    const double w_down = sz + 0.5 * c * c + 0.5 * c; /* weight of n_{k-1} */
    double a = 0.0, b = 0.0;
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        a += in[s][IDX(1, j, i)];
        b += in[s][IDX(nz - 1, j, i)];
      }
    col[s][0] = w_up * a * dV;
    col[s][1] = w_down * b * dV;
  }
  tally[T_RECOMB] = recomb * dV;
  tally[T_POS_ANODE] = col[0][0];
  tally[T_POS_CATHODE] = col[0][1];
  tally[T_NEG_ANODE] = col[1][0];
  tally[T_NEG_CATHODE] = col[1][1];
  tally[T_POS_INFLIGHT] = inflight[0] * dV;
  tally[T_NEG_INFLIGHT] = inflight[1] * dV;
  tally[T_POS_ABS] = absolute[0] * dV;
  tally[T_NEG_ABS] = absolute[1] * dV;
  tally[T_RELEASED] = 0.0;
  tally[T_RELEASED_NEG] = 0.0;
  tally[T_POS_SC] = screen[0] * dV;
  tally[T_NEG_SC] = screen[1] * dV;
  tally[T_POS_ESC] = escaped[0] * dV;
  tally[T_NEG_ESC] = escaped[1] * dV;
}

static double field_max(int64_t n, const double *a, const double *b)
{
  double m = 0.0;
  for (int64_t q = 0; q < n; ++q) {
    if (a[q] > m) m = a[q];
    if (b[q] > m) m = b[q];
  }
  return m;
}

/* Full run: deposit, step, tally, stop (see the file header).
 * pos/neg: caller-provided (nz+1)*ny*nx arrays, overwritten; hold the final
 * densities on return.  trace: NULL or max_steps*T_COUNT doubles.
 * res: R_COUNT doubles.  Returns 0 or a negative error (-1 invalid pulse
 * train, -2 no stable dt, -3 a pulse train with a track not due at t = 0,
 * -4 out of memory). */
int orc_solve(const double *p, int64_t nx, int64_t ny, int64_t nz,
              const double *trk, int64_t ntr, int64_t max_steps,
              double *pos, double *neg, double *trace, double *res)
{
  double dt;
  int rc = orc_dt(p, nx, ny, nz, trk, ntr, &dt);
  if (rc) return rc;

  /* pulse train: m steps per period (dt shortened to P/m), pulse k at the
   * start of step k m; the run ends before step N m */
  const int64_t npulses = p[P_N_PULSES] >= 2.0 ? (int64_t)p[P_N_PULSES] : 1;
  const double period = p[P_PULSE_PERIOD];
  const int train = npulses > 1;
  int64_t end = max_steps, last_pulse = -1, m = 0;
  if (train) {
    if (!(period > 0.0) || !isfinite(period)) return -1;
    for (int64_t t = 0; t < ntr; ++t)
      if (trk[TRK * t + 6] != 0.0) return -3;
    const double per = ceil(period / dt);
    if (!(per <= 1.0e15 / (double)npulses)) return -1;  /* steps of the train beyond range */
    m = (int64_t)per;
    dt = period / (double)m;
    if (npulses * m < end) end = npulses * m;
    last_pulse = (npulses - 1) * m;
  }

  const int64_t n = (nz + 1) * ny * nx;
  double *npos = (double *)calloc((size_t)n, sizeof(double));
  double *nneg = (double *)calloc((size_t)n, sizeof(double));
  if (!npos || !nneg) { free(npos); free(nneg); return -4; }
  memset(pos, 0, (size_t)n * sizeof(double));
  memset(neg, 0, (size_t)n * sizeof(double));

  int64_t last_deposit = -1;
  for (int64_t t = 0; t < ntr; ++t) {
    int64_t s = orc_deposit_step(dt, trk + TRK * t);
    if (s < max_steps && s > last_deposit) last_deposit = s;
  }
  const double beta = p[P_ALPHA] * dt;
  double released = 0.0, released_neg = 0.0, sums[5] = {0, 0, 0, 0, 0}, screened[2] = {0, 0};
  double esc[2] = {0, 0};
  double last[T_COUNT] = {0};
  double max_beta_n = 0.0;
  /* the last period of a pulse train: running sums at its start and the
   * ions its pulse released */
  double period_sums[5] = {0, 0, 0, 0, 0}, period_rel[2] = {0, 0};
  int period_started = 0;
  int64_t next_pulse = 0;
  int flags = 0;
  int64_t steps = 0;
  for (int64_t l = 0; l < end; ++l) {
    /* what is deposited at the start of this step: pulse k of a train, or
     * the single pulse's uniform pre-ionisation and the tracks due now */
    int deposit = 0;
    if (train) {
      if (next_pulse < npulses && next_pulse * m == l) {
        deposit = 1;
        ++next_pulse;
      }
    } else {
      deposit = l == 0 && p[P_UNIFORM_N0] != 0.0;
      for (int64_t t = 0; t < ntr && !deposit; ++t)
        if (orc_deposit_step(dt, trk + TRK * t) == l) deposit = 1;
    }
    double released_now = 0.0, released_now_neg = 0.0;
    if (deposit) {
      if (p[P_UNIFORM_N0] != 0.0 && (train || l == 0)) {
        const double u0 = orc_uniform(p, nx, ny, nz, p[P_UNIFORM_N0], pos, neg);
        released_now += u0;
        released_now_neg += u0;
      }
      double rel[2];
      deposit_tracks(p, nx, ny, nz, trk, ntr, l, dt, train, pos, neg, rel);
      released_now += rel[0];
      released_now_neg += rel[1];
      const double m = beta * field_max(n, pos, neg);
      if (m > max_beta_n) max_beta_n = m;
    }
    released += released_now;
    released_neg += released_now_neg;
    if (train && l == last_pulse) {
      memcpy(period_sums, sums, sizeof(sums));
      period_rel[0] = released_now;
      period_rel[1] = released_now_neg;
      period_started = 1;
    }
    double tally[T_COUNT];
    orc_step(p, nx, ny, nz, dt, pos, neg, npos, nneg, tally);
    tally[T_RELEASED] = released_now;
    tally[T_RELEASED_NEG] = released_now_neg;
    double *tmp = pos; pos = npos; npos = tmp;
    tmp = neg; neg = nneg; nneg = tmp;
    for (int q = 0; q < 5; ++q) sums[q] += tally[q];
    screened[0] += tally[T_POS_SC];
    screened[1] += tally[T_NEG_SC];
    esc[0] += tally[T_POS_ESC];
    esc[1] += tally[T_NEG_ESC];
    memcpy(last, tally, sizeof(last));
    if (trace) memcpy(trace + T_COUNT * l, tally, sizeof(tally));
    steps = l + 1;
    int finite = 1;
    for (int q = 0; q < T_COUNT; ++q) finite &= isfinite(tally[q]) != 0;
    if (!finite) { flags |= FLAG_NONFINITE; break; }
    if (!train && l >= last_deposit && tally[T_POS_ABS] <= p[P_STOP_TOL] * released &&
        tally[T_NEG_ABS] <= p[P_STOP_TOL] * released_neg)
      break;
    if (steps == max_steps) flags |= FLAG_MAX_STEPS;
  }
  /* after an odd number of swaps the final fields sit in the scratch arrays */
  if (steps % 2 == 1) {
    memcpy(npos, pos, (size_t)n * sizeof(double));
    memcpy(nneg, neg, (size_t)n * sizeof(double));
    double *tmp = pos; pos = npos; npos = tmp;
    tmp = neg; neg = nneg; nneg = tmp;
  }
  free(npos);
  free(nneg);

  if (max_beta_n > 1.0) flags |= FLAG_REACTION;
  const double collected = sums[1] + sums[2] + sums[3] + sums[4];
  double f, f_R;
  if (released + released_neg > 0.0) {
    f = collected / (released + released_neg);
    /* recombined pairs against the mean number released per species */
    f_R = 1.0 - 2.0 * sums[0] / (released + released_neg);
  } else {
    f = 1.0;
    f_R = 1.0;
    flags |= FLAG_EMPTY;
  }
  res[R_PULSES] = 0.0;
  res[R_PERIOD_RELEASED] = res[R_PERIOD_COLLECTED] = res[R_PERIOD_RECOMBINED] = 0.0;
  if (train) {
    const int64_t delivered = (steps + m - 1) / m;  /* pulses at steps 0, m, 2m, ... below `steps` */
    res[R_PULSES] = (double)(delivered < npulses ? delivered : npulses);
  }
  if (period_started) {
    /* the last period of the train */
    double pc = 0.0;
    for (int q = 1; q < 5; ++q) pc += sums[q] - period_sums[q];
    const double prel = period_rel[0] + period_rel[1];
    const double prec = sums[0] - period_sums[0];
    res[R_PERIOD_RELEASED] = prel;
    res[R_PERIOD_COLLECTED] = pc;
    res[R_PERIOD_RECOMBINED] = prec;
    if (prel > 0.0) {
      f = pc / prel;
      f_R = 1.0 - 2.0 * prec / prel;
    }
  }
  res[R_F] = f;
  res[R_KS] = 1.0 / f;
  res[R_F_RECOMB] = f_R;
  res[R_RELEASED] = released;
  res[R_RECOMBINED] = sums[0];
  res[R_INFLIGHT_POS] = last[T_POS_INFLIGHT];
  res[R_INFLIGHT_NEG] = last[T_NEG_INFLIGHT];
  res[R_COL_POS_ANODE] = sums[1];
  res[R_COL_POS_CATHODE] = sums[2];
  res[R_COL_NEG_ANODE] = sums[3];
  res[R_COL_NEG_CATHODE] = sums[4];
  res[R_DT] = dt;
  res[R_STEPS] = (double)steps;
  res[R_FLAGS] = (double)flags;
  res[R_MAX_BETA_N] = max_beta_n;
  res[R_RELEASED_NEG] = released_neg;
  res[R_SC_POS] = screened[0];
  res[R_SC_NEG] = screened[1];
  res[R_ESC_POS] = esc[0];
  res[R_ESC_NEG] = esc[1];
  return 0;
}

/* Advance given densities by nsteps without deposits (tests of the stepping
 * alone).  trace: NULL or nsteps*T_COUNT. */
int orc_advance(const double *p, int64_t nx, int64_t ny, int64_t nz, double dt,
                int64_t nsteps, double *pos, double *neg, double *trace)
{
  const int64_t n = (nz + 1) * ny * nx;
  double *npos = (double *)calloc((size_t)n, sizeof(double));
  double *nneg = (double *)calloc((size_t)n, sizeof(double));
  if (!npos || !nneg) { free(npos); free(nneg); return -1; }
  double *a = pos, *b = neg, *c = npos, *d = nneg;
  for (int64_t l = 0; l < nsteps; ++l) {
    double tally[T_COUNT];
    orc_step(p, nx, ny, nz, dt, a, b, c, d, tally);
    if (trace) memcpy(trace + T_COUNT * l, tally, sizeof(tally));
    double *t = a; a = c; c = t;
    t = b; b = d; d = t;
  }
  if (a != pos) {
    memcpy(pos, a, (size_t)n * sizeof(double));
    memcpy(neg, b, (size_t)n * sizeof(double));
  }
  free(npos);
  free(nneg);
  return 0;
}

/* ------------------------------------------------------------------------
 * Free-electron component (sections "The free-electron component" and
 * "Implementation of the free-electron models").
 *
 *   - fraction of electrons that stay free p = (1 - e^{-a d})/(a d)
 *                                                              (eq. free_elec)
 *   - initial densities: n+ as deposited; n-(z) = n+ (1 - e^{-a z}) and
 *     n_e = n+ p, z measured from the anode                (eq. ion_elec_distribution)
 *     (applied at every node to the negative charge the deposit releases)
 *   - phase 1: the step is the largest stable one for the electrons (eq.
 *     vNeum with mu_e, D_e), all three carriers move, the positive ions
 *     recombine with both negative carriers (alpha n+ (n- + n_e)); it ends
 *     once the electrons are collected (sum |n_e| dV <= stop_tol N_e)
 *   - phase 2: the ions continue with their own step (orc_step) until
 *     collection, as without electrons
 * Only instantaneous pulses (every track at t = 0) are allowed; the
 * space-charge term is not combined with free electrons.
 * ------------------------------------------------------------------------ */

enum { E_RPN, E_RPE, E_PA, E_PC, E_NA, E_NC, E_EA, E_EC, E_SP, E_SN, E_SE, E_AP, E_AN, E_AE, E_COUNT };
enum { RE_RELEASED, RE_COLLECTED_ANODE, RE_COLLECTED_CATHODE, RE_RECOMBINED, RE_STEPS, RE_DT,
       RE_LEFT, RE_RELEASED_NEG_CHARGE, RE_COUNT };

/* p of eq. free_elec for attachment coefficient a over gap d */
double orc_free_fraction(double a, double d)
{
  const double x = a * d;
  return x == 0.0 ? 1.0 : -expm1(-x) / x;
}

/* Largest dt of eq. vNeum for the electrons (field along z): the positive
 * root of A dt + B dt^2 = 1 with A = 2 D_e (1/dx^2 + 1/dy^2 + 1/dz^2) and
 * B = (mu_e E / dz)^2, without the safety factor.  INFINITY if the electrons
 * neither drift nor diffuse. */
double orc_electron_dt(const double *p, int64_t nz)
{
  const double dz = p[P_GAP] / (double)nz;
  const double E = p[P_VOLT] / p[P_GAP];
  const double A = 2.0 * p[P_D_E] * (1.0 / (p[P_DX] * p[P_DX]) + 1.0 / (p[P_DY] * p[P_DY]) + 1.0 / (dz * dz));
  const double v = p[P_MU_E] * E / dz;
  const double B = v * v;
  if (B > 0.0) return 2.0 / (A + sqrt(A * A + 4.0 * B));
  if (A > 0.0) return 1.0 / A;
  return INFINITY;
}

/* One phase-1 step of the three carriers (n+, n-, n_e) from the old
 * densities, each with the Appendix's weights for its own signed drift
 * velocity (+mu+ E, -mu- E, -mu_e E) and diffusion constant; the positive
 * ions lose beta n+ (n- + n_e), the negative ions beta n+ n-, the electrons
 * beta n+ n_e.  tally: E_COUNT values (recombined pairs n+n- and n+n_e,
 * collected at the anode and the cathode per carrier, in flight and the sum
 * of |n| per carrier after the step), in counts (density times dV). */
void orc_step3(const double *p, int64_t nx, int64_t ny, int64_t nz, double dt,
               const double *pos, const double *neg, const double *ele,
               double *npos, double *nneg, double *nele, double *tally)
{
  const double dz = p[P_GAP] / (double)nz;
  const double dV = p[P_DX] * p[P_DY] * dz;
  const double beta = p[P_ALPHA] * dt;
  const double E = p[P_VOLT] / p[P_GAP];
  /* c (signed drift), sx, sy, sz for n+, n-, n_e */
  const double mus[3] = {p[P_MU_POS], -p[P_MU_NEG], -p[P_MU_E]};
  const double Ds[3] = {p[P_D_POS], p[P_D_NEG], p[P_D_E]};
  double w[3][4];
  for (int s = 0; s < 3; ++s) {
    w[s][0] = mus[s] * E * dt / dz;
    w[s][1] = Ds[s] * dt / (p[P_DX] * p[P_DX]);
    w[s][2] = Ds[s] * dt / (p[P_DY] * p[P_DY]);
    w[s][3] = Ds[s] * dt / (dz * dz);
  }
  const double *in[3] = {pos, neg, ele};
  double *out[3] = {npos, nneg, nele};
  /* per-plane partial sums: rpn, rpe, in flight and |n| of each carrier */
  double *part = (double *)calloc((size_t)(nz + 1) * 8, sizeof(double));
  if (!part) {
    for (int q = 0; q < E_COUNT; ++q) tally[q] = NAN;
    return;
  }
#pragma omp parallel for schedule(static)
  for (int64_t k = 1; k < nz; ++k) {
    double rpn = 0.0, rpe = 0.0, inflight[3] = {0, 0, 0}, absolute[3] = {0, 0, 0};
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        const int64_t ip = (i + 1) % nx, im = (i + nx - 1) % nx;
        const int64_t jp = (j + 1) % ny, jm = (j + ny - 1) % ny;
        const double np_ = pos[IDX(k, j, i)], nn_ = neg[IDX(k, j, i)], ne_ = ele[IDX(k, j, i)];
        const double sink_n = beta * np_ * nn_, sink_e = beta * np_ * ne_;
        rpn += sink_n;
        rpe += sink_e;
        const double sinks[3] = {sink_n + sink_e, sink_n, sink_e};
        for (int s = 0; s < 3; ++s) {
          const double *n = in[s];
          const double c = w[s][0], sx = w[s][1], sy = w[s][2], sz = w[s][3];
          const double nc = n[IDX(k, j, i)];
          const double lap_x = n[IDX(k, j, ip)] - 2.0 * nc + n[IDX(k, j, im)];
          const double lap_y = n[IDX(k, jp, i)] - 2.0 * nc + n[IDX(k, jm, i)];
          const double lap_z = n[IDX(k + 1, j, i)] - 2.0 * nc + n[IDX(k - 1, j, i)];
          const double drift = c * (c * (nc - n[IDX(k - 1, j, i)])
                                    + (1.0 - c) * 0.5 * (n[IDX(k + 1, j, i)] - n[IDX(k - 1, j, i)]));
          const double v = nc + sx * lap_x + sy * lap_y + sz * lap_z - drift - sinks[s];
          out[s][IDX(k, j, i)] = v;
          inflight[s] += v;
          absolute[s] += fabs(v);
        }
      }
    double *pk = part + (size_t)k * 8;
    pk[0] = rpn;
    pk[1] = rpe;
    for (int s = 0; s < 3; ++s) {
      pk[2 + s] = inflight[s];
      pk[5 + s] = absolute[s];
    }
  }
  double rpn = 0.0, rpe = 0.0, inflight[3] = {0, 0, 0}, absolute[3] = {0, 0, 0};
  for (int64_t k = 1; k < nz; ++k) {
    const double *pk = part + (size_t)k * 8;
    rpn += pk[0];
    rpe += pk[1];
    for (int s = 0; s < 3; ++s) {
      inflight[s] += pk[2 + s];
      absolute[s] += pk[5 + s];
    }
  }
  free(part);
  for (int s = 0; s < 3; ++s) {
    const double c = w[s][0], sz = w[s][3];
    const double w_up = sz + 0.5 * c * c - 0.5 * c, w_down = sz + 0.5 * c * c + 0.5 * c;
    double a = 0.0, b = 0.0;
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        a += in[s][IDX(1, j, i)];
        b += in[s][IDX(nz - 1, j, i)];
      }
    tally[E_PA + 2 * s] = w_up * a * dV;
    tally[E_PC + 2 * s] = w_down * b * dV;
    tally[E_SP + s] = inflight[s] * dV;
    tally[E_AP + s] = absolute[s] * dV;
  }
  tally[E_RPN] = rpn * dV;
  tally[E_RPE] = rpe * dV;
}

/* Run with a free-electron component (attachment coefficient p[P_ATTACH],
 * electron mobility p[P_MU_E] > 0 and diffusion p[P_D_E]).  pos_out,
 * neg_out: the final ion densities.  res as orc_solve (phase-2 tallies plus
 * the phase-1 ion tallies; f counts the collected electrons too, against
 * the positive plus negative charge released); res_e: RE_COUNT values of the
 * electron phase; trace: NULL or max_steps * T_COUNT phase-2 records;
 * trace_e: NULL or max_steps * E_COUNT phase-1 records.  Returns 0, -2 (no
 * step), -3 (a track not at t = 0, space charge on, absorbing lateral
 * boundaries or a pulse train) or -1. */
int orc_solve_free_electrons(const double *p, int64_t nx, int64_t ny, int64_t nz,
                             const double *trk, int64_t ntr, int64_t max_steps,
                             double *pos_out, double *neg_out, double *trace, double *res,
                             double *res_e, double *trace_e)
{
  for (int64_t t = 0; t < ntr; ++t)
    if (trk[TRK * t + 6] != 0.0) return -3;
  if (p[P_SPACE_CHARGE] != 0.0 || p[P_LATERAL_BC] != 0.0 || p[P_N_PULSES] >= 2.0) return -3;
  double dt;
  int rc = orc_dt(p, nx, ny, nz, trk, ntr, &dt);
  if (rc) return rc;
  double dt1 = p[P_KAPPA] * orc_electron_dt(p, nz);
  if (dt < dt1) dt1 = dt;
  const int64_t n = (nz + 1) * ny * nx;
  const double dz = p[P_GAP] / (double)nz;
  const double dV = p[P_DX] * p[P_DY] * dz;
  const double pf = orc_free_fraction(p[P_ATTACH], p[P_GAP]);
  double *dep = (double *)calloc((size_t)n, sizeof(double));
  double *a[6];
  int bad = !dep;
  for (int q = 0; q < 6; ++q) {
    a[q] = (double *)calloc((size_t)n, sizeof(double));
    bad |= !a[q];
  }
  if (bad) {
    free(dep);
    for (int q = 0; q < 6; ++q) free(a[q]);
    return -1;
  }
  /* deposit: positive ions into a[0], the negative charge into dep, then
   * split dep into negative ions a[1] and free electrons a[2] */
  double rel_pos = 0.0, rel_negq = 0.0;
  if (p[P_UNIFORM_N0] != 0.0) {
    const double u = orc_uniform(p, nx, ny, nz, p[P_UNIFORM_N0], a[0], dep);
    rel_pos += u;
    rel_negq += u;
  }
  double rel[2];
  orc_deposit(p, nx, ny, nz, trk, ntr, 0, dt, a[0], dep, rel);
  rel_pos += rel[0];
  rel_negq += rel[1];
  double rel_neg = 0.0, rel_e = 0.0;
  for (int64_t k = 1; k < nz; ++k) {
    const double att = -expm1(-p[P_ATTACH] * (double)k * dz); /* 1 - e^{-a z} */
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        const double d = dep[IDX(k, j, i)];
        a[1][IDX(k, j, i)] = d * att;
        a[2][IDX(k, j, i)] = d * pf;
        rel_neg += d * att;
        rel_e += d * pf;
      }
  }
  free(dep);
  rel_neg *= dV;
  rel_e *= dV;
  const double beta = p[P_ALPHA] * dt;
  double max_beta_n = 0.0;
  for (int64_t q = 0; q < n; ++q) {
    const double m = a[0][q] > a[1][q] + a[2][q] ? a[0][q] : a[1][q] + a[2][q];
    if (beta * m > max_beta_n) max_beta_n = beta * m;
  }

  /* phase 1: the three carriers at the electron step */
  double sums[5] = {0, 0, 0, 0, 0}; /* R, C+a, C+c, C-a, C-c (ions) */
  double e_col[2] = {0, 0}, e_rec = 0.0, e_left = rel_e;
  int64_t steps_e = 0;
  int flags = 0;
  int cur = 0;
  while (rel_e > 0.0 && steps_e < max_steps) {
    double tally[E_COUNT];
    orc_step3(p, nx, ny, nz, dt1, a[3 * cur], a[3 * cur + 1], a[3 * cur + 2],
          a[3 * (1 - cur)], a[3 * (1 - cur) + 1], a[3 * (1 - cur) + 2], tally);
    cur = 1 - cur;
    if (trace_e) memcpy(trace_e + E_COUNT * steps_e, tally, sizeof(tally));
    ++steps_e;
    sums[0] += tally[E_RPN];
    sums[1] += tally[E_PA];
    sums[2] += tally[E_PC];
    sums[3] += tally[E_NA];
    sums[4] += tally[E_NC];
    e_col[0] += tally[E_EA];
    e_col[1] += tally[E_EC];
    e_rec += tally[E_RPE];
    e_left = tally[E_SE];
    int finite = 1;
    for (int q = 0; q < E_COUNT; ++q) finite &= isfinite(tally[q]) != 0;
    if (!finite) { flags |= FLAG_NONFINITE; break; }
    if (tally[E_AE] <= p[P_STOP_TOL] * rel_e) break;
  }

  /* phase 2: the ions alone at their own step, from the state after phase 1 */
  double *P = a[3 * cur], *N = a[3 * cur + 1], *Q = a[3 * (1 - cur)], *M = a[3 * (1 - cur) + 1];
  double last[T_COUNT] = {0};
  int64_t steps = 0;
  int ended = 0; /* stopped by the collection criterion */
  if (!(flags & FLAG_NONFINITE)) {
    for (int64_t l = 0; steps_e + l < max_steps; ++l) {
      double t2[T_COUNT];
      orc_step(p, nx, ny, nz, dt, P, N, Q, M, t2);
      double *tmp = P; P = Q; Q = tmp;
      tmp = N; N = M; M = tmp;
      for (int q = 0; q < 5; ++q) sums[q] += t2[q];
      memcpy(last, t2, sizeof(last));
      if (trace) memcpy(trace + T_COUNT * l, t2, sizeof(t2));
      steps = l + 1;
      int finite = 1;
      for (int q = 0; q < T_COUNT; ++q) finite &= isfinite(t2[q]) != 0;
      if (!finite) { flags |= FLAG_NONFINITE; break; }
      if (t2[T_POS_ABS] <= p[P_STOP_TOL] * rel_pos && t2[T_NEG_ABS] <= p[P_STOP_TOL] * rel_neg) {
        ended = 1;
        break;
      }
    }
  }
  if (!ended && !(flags & FLAG_NONFINITE)) flags |= FLAG_MAX_STEPS;
  memcpy(pos_out, P, (size_t)n * sizeof(double));
  memcpy(neg_out, N, (size_t)n * sizeof(double));
  for (int q = 0; q < 6; ++q) free(a[q]);

  if (max_beta_n > 1.0) flags |= FLAG_REACTION;
  const double collected_ions = sums[1] + sums[2] + sums[3] + sums[4];
  const double released_q = rel_pos + rel_negq; /* positive + negative charge released */
  if (!(released_q > 0.0)) flags |= FLAG_EMPTY;
  res[R_F] = released_q > 0.0 ? (collected_ions + e_col[0] + e_col[1]) / released_q : 1.0;
  res[R_KS] = 1.0 / res[R_F];
  res[R_F_RECOMB] = released_q > 0.0 ? 1.0 - 2.0 * (sums[0] + e_rec) / released_q : 1.0;
  res[R_RELEASED] = rel_pos;
  res[R_RECOMBINED] = sums[0];
  res[R_INFLIGHT_POS] = last[T_POS_INFLIGHT];
  res[R_INFLIGHT_NEG] = last[T_NEG_INFLIGHT];
  res[R_COL_POS_ANODE] = sums[1];
  res[R_COL_POS_CATHODE] = sums[2];
  res[R_COL_NEG_ANODE] = sums[3];
  res[R_COL_NEG_CATHODE] = sums[4];
  res[R_DT] = dt;
  res[R_STEPS] = (double)steps;
  res[R_FLAGS] = (double)flags;
  res[R_MAX_BETA_N] = max_beta_n;
  res[R_SC_POS] = 0.0;
  res[R_SC_NEG] = 0.0;
  res[R_ESC_POS] = 0.0;
  res[R_ESC_NEG] = 0.0;
  res[R_RELEASED_NEG] = rel_neg;
  res_e[RE_RELEASED] = rel_e;
  res_e[RE_COLLECTED_ANODE] = e_col[0];
  res_e[RE_COLLECTED_CATHODE] = e_col[1];
  res_e[RE_RECOMBINED] = e_rec;
  res_e[RE_STEPS] = (double)steps_e;
  res_e[RE_DT] = dt1;
  res_e[RE_LEFT] = e_left;
  res_e[RE_RELEASED_NEG_CHARGE] = rel_negq;
  return 0;
}
