/*
 * iontracks.h -- C ABI of the MI355X recombination solver.
 *
 * The library computes the collection efficiency f and the recombination
 * factor k_s = 1/f of a parallel-plate ionization chamber hit by ion tracks,
 * following Christensen, Toelli & Bassler, "A general algorithm for
 * calculation of recombination losses in ionization chambers exposed to ion
 * beams" (arXiv:1610.06749):
 *
 *   - tracks release N0 = LET/W ion pairs per unit length (eq. linear_density)
 *     with Jaffe's Gaussian radial profile n0(r) = N0/(pi b^2) e^{-r^2/b^2}
 *     (eq. Gaussian) around an axis tilted by theta to the field;
 *   - positive and negative ion densities drift in the applied field, diffuse
 *     and recombine at rate alpha n+ n- (eq. theEquation), stepped by the
 *     explicit scheme of the Appendix (forward time difference, the drift
 *     derivative blending backward and central differences with weight c,
 *     3-point diffusion) at the largest time step allowed by eq. vNeum;
 *   - the electrodes at z = 0 (anode) and z = d (cathode) hold zero density
 *     and collect what reaches them (Methods, Implementation);
 *   - f = N_collected / N_released (eq. collection_efficiency).
 *
 * Units: cm, s, V, keV/um for LET, eV for W.  All arithmetic is FP64.
 *
 * Grid: nx * ny transverse nodes x_i = i dx, y_j = j dy with periodic lateral
 * boundaries (or, optionally, absorbing ones); nz gap intervals of dz = gap/nz, planes k = 0..nz, of which
 * k = 1..nz-1 are interior.  Density fields are FP64 arrays [nz+1][ny][nx]
 * with x fastest; planes 0 and nz always hold zero.
 *
 * Conventions of every entry point:
 *   - return 0 (IT_OK) on success or a negative IT_E* code; nothing is thrown
 *     across the ABI; it_strerror() names the code.  Entry points that
 *     launch device work first clear the HIP runtime's last-error state of
 *     the calling thread (hipGetLastError), so that an error an earlier,
 *     unrelated HIP call left there is not taken for one of theirs;
 *   - the caller owns every buffer.  "host" pointers are ordinary CPU memory,
 *     "device" pointers are HIP device memory of the current device.  The
 *     library allocates no memory, device or host: scratch space comes from
 *     the caller's workspace and, optionally, its page-locked host buffer
 *     (it_exec.host_buffer).  Within a call it creates and destroys HIP
 *     events and, in it_solve_batch, one HIP graph and its executable;
 *   - device work runs on the HIP stream passed as `stream` (a hipStream_t,
 *     NULL = the default stream) and on no other stream.  Calls that return
 *     host results synchronise that stream before returning;
 *   - the workspace is device memory of at least it_workspace_size() bytes;
 *     its contents need not be initialised and are clobbered.  Calls that
 *     share one workspace must not overlap in time.
 */
#ifndef IONTRACKS_H
#define IONTRACKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define IT_OK 0
#define IT_EINVAL -1      /* invalid argument: a size, a constant or a track is out of range */
#define IT_ENODT -2       /* neither drift nor diffusion bounds the time step (E = 0 and D = 0) */
#define IT_EWORKSPACE -3  /* workspace NULL or smaller than it_workspace_size() */
#define IT_EHIP -4        /* a HIP runtime call failed (no device, launch failure, ...) */
#define IT_ENOTSUP -5     /* an option or a combination of options that is not supported */

/* ---- result flags ---- */
#define IT_FLAG_MAX_STEPS 1  /* stopped by max_steps, not by the collection criterion */
#define IT_FLAG_NONFINITE 2  /* a tally became NaN or Inf; the run stopped there */
#define IT_FLAG_REACTION 4   /* alpha*dt*max(n) exceeded 1 after a deposit */
#define IT_FLAG_EMPTY 8      /* nothing was released; f is reported as 1 */

/* ---- per-step trace record: IT_TRACE_COLS doubles per step, in ion counts ---- */
#define IT_TRACE_COLS 15
/* 0 recombined pairs, 1/2 positive ions collected at anode/cathode,
 * 3/4 negative ions collected at anode/cathode, 5/6 positive/negative ions in
 * flight after the step (signed sum of n dV), 7/8 sum of |n| dV after the
 * step, 9 positive ions released by deposits made before the step, 10/11
 * change of the positive/negative ions by the space-charge term in the step
 * (0 with space charge off), 12 negative ions released by deposits made
 * before the step (equal to column 9 unless tracks give the negative ions
 * their own radius), 13/14 positive/negative ions that left through
 * absorbing lateral boundaries in the step (0 with periodic ones).  Per
 * species: in flight after = in flight before + released - collected -
 * recombined + space-charge change - escaped. */

/* Chamber, field, transport constants and run control. */
typedef struct {
  int32_t nx, ny;       /* transverse node counts (>= 1), periodic unless lateral_bc = 1 */
  int32_t nz;           /* gap intervals (>= 2): interior planes 1..nz-1 */
  int32_t space_charge; /* 1: include the space-charge screening term mu n div E of eq.
                         * theEquation, with div E = q (n+ - n-)/eps0 at each node
                         * (Maxwell-Gauss, same section); E in E . grad n stays the
                         * applied field.  0: leave it out (div E = 0). */
  double dx, dy;        /* transverse node spacing [cm] */
  double gap;           /* electrode distance d [cm]; dz = gap/nz */
  double voltage;       /* V [V]; E = V/gap along +z, anode z=0 -> cathode z=d */
  double mu_pos, mu_neg;/* ion mobilities [cm^2/(V s)] (>= 0) */
  double D_pos, D_neg;  /* ion diffusion constants [cm^2/s] (>= 0) */
  double alpha;         /* recombination constant [cm^3/s] (>= 0) */
  double W_eV;          /* mean energy per ion pair [eV] (> 0) */
  double dt_safety;     /* factor in (0, 1] on the largest stable dt (eq. vNeum) */
  double stop_tol;      /* stop once sum |n| dV <= stop_tol * released for both species (>= 0) */
  double uniform_n0;    /* uniform ion-pair density added at t = 0 [cm^-3] (>= 0) */
  double reaction_limit;/* rho >= 0: also bound dt by k dt n_ref <= rho (0 = off), see it_dt */
  /* Free-electron component (The free-electron component; Implementation of
   * the free-electron models), on when mu_e > 0: of the negative charge a
   * deposit releases, the fraction p = (1 - e^{-a d})/(a d) stays as free
   * electrons spread evenly (n_e = n+ p) and the rest forms negative ions
   * n+ (1 - e^{-a z}), z from the anode (eqs. free_elec,
   * ion_elec_distribution).  The run first steps all three carriers at the
   * electrons' largest stable step (eq. vNeum with mu_e, D_e; the positive
   * ions recombine with both negative carriers) until the electrons are
   * collected (sum |n_e| dV <= stop_tol times the electrons released), then
   * the ions alone at their own step.  Needs every track at t = 0 and
   * space_charge = 0 (else IT_ENOTSUP); it_solve_batch does not support it. */
  double attach_coeff;  /* a [1/cm] (>= 0; 0: no attachment, p = 1) */
  double mu_e;          /* electron mobility [cm^2/(V s)] (>= 0; 0 = no free electrons) */
  double D_e;           /* electron diffusion constant [cm^2/s] (>= 0) */
  int64_t max_steps;    /* hard step limit (>= 1), both phases together */
  /* Lateral (x, y) boundaries, which the paper leaves open: 0 = periodic (the
   * transverse cell repeats), 1 = absorbing: the nodes just outside the cell
   * hold zero, like the electrodes, and what they would receive in a step
   * (ax or ay times the density of each node next to the boundary, per
   * missing neighbour) leaves the chamber and is counted as escaped; track
   * offsets are then not wrapped.  Absorbing boundaries work with every
   * stepping kernel, in single runs and in batches (where they may be mixed
   * with periodic instances), not with free electrons (IT_ENOTSUP). */
  int32_t lateral_bc;
  /* Pulse train (the beam's time structure as pulses, Distribution of ion
   * tracks; a repetition rate read as a periodic train of identical
   * pulses): n_pulses >= 2 repeats the chamber's deposits -- uniform_n0 and
   * every track, each of which must be due at t = 0 (IT_ENOTSUP otherwise)
   * -- n_pulses times, one pulse every pulse_period_s seconds.  A period is
   * m = ceil(pulse_period_s / dt1) whole steps, dt1 the single-pulse step
   * (dt_safety times the bound below), and the run steps at
   * dt = pulse_period_s / m, so that every period has the same steps and
   * the train can settle into an exactly periodic state; pulse k is
   * deposited at the start of step k m.  The run covers steps
   * 0 .. n_pulses m - 1 with no collection test, and f, ks and f_R describe
   * its last period (see it_result).  0 or 1: a single pulse (the tracks at
   * their own times; pulse_period_s is ignored).  Not with free electrons
   * (IT_ENOTSUP). */
  int32_t n_pulses;
  double pulse_period_s;  /* [s], finite and > 0 when n_pulses >= 2 */
} it_chamber;

/* One ion track.  The axis passes through (x, y, gap/2) with direction
 * (sin theta cos phi, sin theta sin phi, cos theta); theta is the angle to the
 * field.  The track is deposited at the start of step floor(t/dt).  The
 * transverse offset of a node from (x, y) is wrapped to the nearest periodic
 * image (with periodic lateral boundaries) and the profile is cut at a
 * perpendicular distance of 8 b. */
typedef struct {
  double let_keV_um;    /* LET in air [keV/um] (>= 0) */
  double b_cm;          /* Gaussian track radius b [cm] (> 0) */
  double x_cm, y_cm;    /* axis position at mid-gap [cm] */
  double theta, phi;    /* polar angle to the field and azimuth [rad] */
  double t_s;           /* arrival time [s] (>= 0) */
  double b_neg_cm;      /* Gaussian radius of the negative ions [cm]; 0 = b_cm.  The
                         * paper notes that the negative ions' track is wider and
                         * that separate radii are a direct extension of its
                         * averaged radius (The charge carrier distribution). */
} it_track;

/* Result of a run (all counts in ion pairs / ions). */
typedef struct {
  double f;             /* collection efficiency: charge collected / charge released,
                         * both signs (free electrons included; charge that escapes
                         * through absorbing lateral boundaries is not collected) */
  double ks;            /* recombination factor 1/f */
  double f_R;           /* 1 - recombined pairs / mean charge released per sign */
  double n_released, n_recombined;
  double n_inflight_pos, n_inflight_neg;  /* signed in-flight counts after the last step */
  double col_pos_anode, col_pos_cathode, col_neg_anode, col_neg_cathode;
  double dt;            /* time step [s] */
  double max_beta_n;    /* max over deposits of alpha*dt*max(n) */
  double n_space_charge_pos, n_space_charge_neg;  /* change of each species by the
                         * space-charge term over the run (ions; 0 when off) */
  double n_released_neg;/* negative ions released (n_released counts the positive
                         * ions; the two differ only with separate track radii or
                         * free electrons) */
  /* free-electron phase (all 0 without free electrons) */
  double e_released;    /* free electrons released */
  double e_collected_anode, e_collected_cathode;
  double e_recombined;  /* electrons recombined with positive ions */
  double e_left;        /* electrons still in flight when the phase ended */
  double e_dt;          /* step of the electron phase [s] */
  double released_neg_charge;  /* negative charge released (ions + electrons) */
  double n_escaped_pos, n_escaped_neg;  /* ions lost through absorbing lateral
                         * boundaries over the run (0 with periodic ones) */
  int64_t e_steps;      /* steps of the electron phase */
  int64_t steps;        /* steps counted in the result */
  int32_t flags;        /* IT_FLAG_* */
  int32_t passes;       /* stepping kernel launches issued (diagnostic) */
  /* Pulse train (n_pulses >= 2; all 0 otherwise): pulses deposited, and
   * the last period, steps (n_pulses-1) m .. n_pulses m - 1, in ions of both
   * signs: period_released what its pulse released, period_collected what
   * reached the electrodes during it, period_recombined the pairs that
   * recombined during it.  f = period_collected / period_released, ks =
   * 1/f and f_R = 1 - 2 period_recombined / period_released then describe
   * one pulse of the train: in a periodic steady state one period collects
   * or recombines what one pulse releases.  The other counts cover the
   * whole run.  A run that stops before its last pulse (max_steps, a
   * non-finite tally) reports f, ks and f_R of the whole run. */
  int32_t pulses;
  int32_t reserved;
  double period_released, period_collected, period_recombined;
} it_result;

/* Kernel selection for the stepping.  NULL means "defaults". */
#define IT_KERNEL_AUTO 0     /* the library's choice: passes of 3 fused steps (the blocked kernel)
                              * on grids of at least 4e6 interior nodes, 64 x 32 nodes
                              * per plane or more, when no final fields are asked for and no
                              * one-step tile option is set; else one step per launch.  A
                              * steps_per_pass > 0 is taken as given. */
#define IT_KERNEL_PLAIN 1    /* one time step per launch */
#define IT_KERNEL_BLOCKED 2  /* steps_per_pass (default 3) fused steps per launch (temporal blocking) */
typedef struct {
  int32_t kernel;          /* IT_KERNEL_* */
  int32_t steps_per_pass;  /* T for the blocked kernel: 2..4 (1: the one-step kernel; 0 = default) */
  int32_t tile_y;          /* rows per tile of the one-step kernels, 8 or 16; with the blocked
                            * kernel the rows of its extended tiles, 24, 32, 40 or 48 (three
                            * to six rows per thread, IT_EINVAL otherwise); 0 = default */
  int32_t check_every;     /* steps between host checks of the stop criterion (0 = default) */
  /* Optional instrumentation (NULL / 0 = none): caller-created hipEvent_t
   * handles, created with timing enabled on the device of the run.  it_solve
   * and it_advance record events[2i] on the run's stream just before and
   * events[2i+1] just after the i-th stepping-kernel launch of the call, for
   * i < n_timing_events / 2 (later launches are not instrumented).  The
   * events bracket the stepping kernel launch (with one step per launch it
   * also records the previous launch's tallies in an extra block, as a blocked
   * pass does).  With
   * timing_span = 1 instead (n_timing_events >= 2), events bracket runs of
   * consecutive stepping launches, with no events inside a run: a run ends
   * where a deposit interrupts the stepping (and at the end of the call);
   * events[2r] is recorded before the first stepping launch of run r and
   * events[2r+1] after its last one, for r < n_timing_events / 2 (later runs
   * are not timed).  The computation is unchanged.  Ignored by
   * it_solve_batch. */
  void* const* timing_events;
  int32_t n_timing_events;
  int32_t z_chunk;         /* planes per tile of the one-step kernel, 4..512 (0 = default); in
                            * it_solve_batch with blocked passes, the most planes per tile
                            * (default 512): the library picks the chunk, between
                            * steps_per_pass planes and this, that runs the running instances'
                            * tiles in the fewest rounds of one block per compute unit times
                            * the planes a block marches, and picks it again as instances
                            * finish */
  int32_t timing_span;     /* see timing_events */
  int32_t tile_x;          /* columns per tile of the one-step kernels: 64, or 32 (32 x 16 tiles of
                            * 8 waves, two rows each; tile_y must then be 0 or 16, and the
                            * blocked kernel does not take it), or 128 (tiles of tile_y rows of
                            * 64 column pairs, one pair per lane: single chambers with an even
                            * nx only, IT_EINVAL otherwise; batches return IT_ENOTSUP, and the
                            * blocked kernel does not take it); 0 = default */
  /* Optional page-locked host memory (hipHostMalloc, or a pinned tensor) of
   * at least it_host_buffer_size() bytes, owned by the caller and clobbered
   * by the call: the run state the host reads back to decide when to stop
   * lands there while the device keeps stepping (two read-backs in flight).
   * NULL (or too small): the library reads into ordinary host memory, which
   * makes every read-back synchronous, so the device idles while the host
   * decides on the next launches. */
  void* host_buffer;
  size_t host_buffer_bytes;
} it_exec;

/* Bytes of it_exec.host_buffer for a single run (ninst = 1) or a batch of
 * ninst chambers.  Host only.  Errors: IT_EINVAL (ninst < 1). */
int it_host_buffer_size(int32_t ninst, size_t* bytes);

/* Time step of a run: dt_safety times the smaller of
 *   - the largest dt satisfying eq. vNeum for both species (with the field
 *     along z: 2 D dt (1/dx^2 + 1/dy^2 + 1/dz^2) + (mu E dt/dz)^2 <= 1), and
 *   - when reaction_limit > 0 and k > 0: reaction_limit / (k n_ref), with
 *     k = alpha (+ max(mu+, mu-) q/eps0 with space charge on), because the
 *     explicit recombination sink (and the screening term) diverges once
 *     k dt n exceeds about 1 at dense track cores.  n_ref is uniform_n0 plus the
 *     largest density found on any track's axis at mid-gap from all tracks
 *     with the same arrival time (host array; may be NULL if ntracks = 0).
 * With a pulse train (n_pulses >= 2) that step dt1 is shortened to
 * pulse_period_s / ceil(pulse_period_s / dt1), the step the run takes.
 * Host only: touches no device.  Errors: IT_EINVAL, IT_ENODT. */
int it_dt(const it_chamber* ch, const it_track* tracks, int64_t ntracks, double* dt);

/* Checks a chamber and a track list (host arrays; tracks may be NULL when
 * ntracks == 0).  Host only.  Errors: IT_EINVAL, IT_ENODT. */
int it_validate(const it_chamber* ch, const it_track* tracks, int64_t ntracks);

/* Device workspace bytes it_solve / it_advance need for this chamber and up
 * to ntracks tracks (includes the two double-buffered density fields and a
 * per-step trace of max_steps records).  Host only. */
int it_workspace_size(const it_chamber* ch, int64_t ntracks, size_t* bytes);

/* Full run of the method: deposit the tracks (host array, any order) and the
 * uniform pre-ionisation, step until the stop criterion or max_steps, and
 * fill *out (host).  Optional outputs:
 *   h_trace      host [max_steps][IT_TRACE_COLS]; the first out->steps rows
 *                are written;
 *   d_pos_out,   device [(nz+1)*ny*nx] each: the density fields after the
 *   d_neg_out    last executed step.  With a blocked kernel the run can
 *                execute up to steps_per_pass-1 steps beyond out->steps when
 *                it stops on the collection criterion; with stop_tol = 0 it
 *                stops exactly at max_steps.
 * Synchronises `stream` before returning.
 * Errors: IT_EINVAL, IT_ENODT, IT_EWORKSPACE, IT_EHIP. */
int it_solve(const it_chamber* ch, const it_track* tracks, int64_t ntracks,
             const it_exec* exec, void* d_workspace, size_t ws_bytes, void* stream,
             double* h_trace, double* d_pos_out, double* d_neg_out, it_result* out);

/* Advances given densities by exactly nsteps steps of size dt, without
 * deposits (the stepping of the Appendix alone).  d_pos, d_neg: device
 * [(nz+1)*ny*nx], read and overwritten in place; their electrode planes are
 * treated as zero.  h_trace: NULL or host [nsteps][IT_TRACE_COLS].  Uses the
 * chamber's constants; ch->max_steps must be >= nsteps.  Synchronises
 * `stream`.  Errors: IT_EINVAL, IT_EWORKSPACE, IT_EHIP. */
int it_advance(const it_chamber* ch, double dt, int64_t nsteps, const it_exec* exec,
               double* d_pos, double* d_neg, void* d_workspace, size_t ws_bytes,
               void* stream, double* h_trace);

/* Device workspace bytes it_solve_batch needs for ninst chambers (host
 * array ch[ninst]) with track_offsets[ninst+1] as in it_solve_batch.
 * exec may be NULL (only tile_y matters).  Host only. */
int it_workspace_size_batch(const it_chamber* ch, const int64_t* track_offsets, int32_t ninst,
                            const it_exec* exec, size_t* bytes);

/* Batched sweep: runs ninst independent chambers (uneven grids, voltages,
 * tracks, doses) to completion together, each exactly as it_solve would
 * (same time step rule, deposition, stepping, tallies and stop criterion).
 * ch: host [ninst]; tracks of instance q are tracks[track_offsets[q] ..
 * track_offsets[q+1]) (host); every track must be due at step 0 (one pulse
 * per instance, or a train of them, IT_ENOTSUP otherwise).  An instance
 * with a pulse train keeps its first pulse's densities in the workspace;
 * the pass in which each later pulse falls due adds them to the outputs of
 * the step before it.  A pass of T steps takes at most one pulse: with a
 * train whose period is shorter than T steps the library's choice is one
 * step per pass (a request for blocked passes then returns IT_ENOTSUP;
 * it_workspace_size_batch covers both).  Each pass is one launch over the
 * tiles of all running instances, plus one block per instance that records
 * the instance's previous step; the library
 * captures exec->check_every passes (default 32, rounded up to even) in a
 * HIP graph and replays it on `stream` until every instance has stopped.
 * out: host [ninst].  No per-step traces or fields are kept.
 * Synchronises `stream`.  Errors: IT_EINVAL, IT_ENODT, IT_ENOTSUP,
 * IT_EWORKSPACE, IT_EHIP. */
int it_solve_batch(const it_chamber* ch, const int64_t* track_offsets, const it_track* tracks,
                   int32_t ninst, const it_exec* exec, void* d_workspace, size_t ws_bytes, void* stream,
                   it_result* out);

/* ------------------------------------------------------------------------
 * Surrogate for ln k_s: an ensemble of `members` MLPs 6 -> 128 -> 128 -> 128
 * -> 1 (SiLU), IT_MLP_PARAMS parameters each, laid out per member as
 * W1[128][6], b1[128], W2[128][128], b2[128], W3[128][128], b3[128],
 * w4[128], b4.  Inputs per query: the six physical quantities (LET [keV/um],
 * b [cm], V [V], gap [cm], dose per pulse [mGy], pulse rate [Hz]), all > 0,
 * standardised on the device as z = (log x - mu)/sigma.  FP32 master
 * weights.  Two forward precisions, fixed when the model is initialised:
 * IT_MLP_BF16 uses BF16 copies of the weights (round to nearest even), MFMA
 * with FP32 accumulation for the 128x128 layers and BF16 hidden activations;
 * IT_MLP_FP32 uses the FP32 weights and activations throughout (FP32 MFMA).
 * The network predicts (ln k_s - t_mu)/t_sigma.
 * ------------------------------------------------------------------------ */
#define IT_MLP_PARAMS 34049
#define IT_MLP_BF16 0
#define IT_MLP_FP32 1

/* Device bytes of a model buffer for `members` members (1..64).  Host only. */
int it_mlp_model_bytes(int32_t members, size_t* bytes);

/* Initialises a model buffer: h_params host [members][IT_MLP_PARAMS] FP32
 * initial weights; h_norm host [26] = mu[6], sigma[6], box_lo[6], box_hi[6]
 * (standardised bounds of the training inputs), t_mu, t_sigma.  h_phys:
 * NULL (the network predicts ln k_s itself) or host [6] = averaged D,
 * averaged mu, alpha, W [eV], mu+ + mu-, ion pairs per cm^3 and mGy: then the
 * network predicts the residual of ln k_s over the analytic baseline
 * -ln f_Jaffe - ln f_Boag (eq. Jaffe_noangle for one track parallel to the
 * field; ln(1+u)/u for the dose), which the query adds back.  precision:
 * IT_MLP_BF16 or IT_MLP_FP32 (the forward arithmetic of training and
 * queries).  Clears the optimiser state.  Synchronises `stream`.  Errors:
 * IT_EINVAL, IT_EHIP. */
int it_mlp_init(void* d_model, int32_t members, const float* h_params, const float* h_norm,
                const double* h_phys, int32_t precision, void* stream);

/* The analytic baseline of the model (device d_X [n][6] -> d_out [n],
 * FP64), for checking.  Asynchronous on `stream`. */
int it_mlp_baseline(const void* d_model, const float* d_X, int64_t n, double* d_out, void* stream);

/* Device workspace bytes of it_mlp_train / it_mlp_grad for n samples. */
int it_mlp_train_ws_bytes(int32_t members, int64_t n, size_t* bytes);

/* Full-batch gradient of the mean squared error of every member on
 * (d_X [n][6], d_t [n] = ln k_s targets), device buffers; d_grad device
 * [members][IT_MLP_PARAMS]; h_loss NULL or host [members] (loss before any
 * update).  With IT_MLP_BF16 the casts pass gradients straight through.
 * Synchronises.
 * Errors: IT_EINVAL, IT_EWORKSPACE, IT_EHIP. */
int it_mlp_grad(const void* d_model, int32_t members, const float* d_X, const float* d_t, int64_t n,
                float* d_grad, float* h_loss, void* d_workspace, size_t ws_bytes, void* stream);

/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8) of every member on
 * (d_X [n][6], d_t [n]), device buffers.  batch: rows per step (0 = all n);
 * n must be a multiple of it, and step s (counted over the model's life)
 * uses rows [(s mod n/batch) * batch, ... + batch), so the caller shuffles
 * the data once beforehand.  The learning rate decays from lr to lr_final
 * along a half cosine over the steps of the call (lr_final = lr: constant).
 * The BF16 copies follow each update.  Workspace: it_mlp_train_ws_bytes for
 * `batch` rows (n when batch is 0).  h_loss: NULL or host
 * [ceil(steps/log_every)][members], the minibatch loss before every
 * log_every-th step.  Synchronises `stream`.
 * Errors: IT_EINVAL, IT_EWORKSPACE, IT_EHIP. */
int it_mlp_train(void* d_model, int32_t members, const float* d_X, const float* d_t, int64_t n, int64_t batch,
                 int32_t steps, float lr, float lr_final, int32_t log_every, float* h_loss, void* d_workspace,
                 size_t ws_bytes, void* stream);

/* Device workspace bytes of it_mlp_query for nq queries. */
int it_mlp_query_ws_bytes(int64_t nq, size_t* bytes);

/* Ensemble query (device buffers): d_mean[nq] = mean over members of ln k_s,
 * d_spread[nq] = max - min over members, d_fallback[nq] = 1 where a
 * standardised input lies outside the training box or the spread exceeds
 * spread_tol (such queries must be answered by the solver).  d_fallback_idx:
 * NULL or device [nq]; receives the flagged query indices in increasing
 * order.  h_nfallback: NULL or host, receives their count (synchronises
 * `stream` when given).  Errors: IT_EINVAL, IT_EWORKSPACE, IT_EHIP. */
int it_mlp_query(const void* d_model, const float* d_X, int64_t nq, float spread_tol, float* d_mean,
                 float* d_spread, unsigned char* d_fallback, int64_t* d_fallback_idx, int64_t* h_nfallback,
                 void* d_workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid device allocation): it_mlp_query
 * without a workspace argument.  The query's scratch (per-tile fallback
 * counts and offsets, their total) lives in a file-scope device array of
 * the library, about 1 MiB, one copy per GPU, held until the process ends;
 * its address is looked up once per device on the first call there.  nq
 * may be at most IT_MLP_QUERY_STATIC_MAX (IT_EINVAL beyond).  Arguments and
 * results otherwise as it_mlp_query.  Allocates nothing (no hipMalloc,
 * hipFree or allocating library call).  Every call on a GPU shares that
 * GPU's array, so calls that overlap in time on one GPU (other streams or
 * host threads) race; calls on one stream, one after the other, do not.
 * Errors: IT_EINVAL, IT_EHIP. */
#define IT_MLP_QUERY_STATIC_MAX (1 << 23)
int it_mlp_query_static(const void* d_model, const float* d_X, int64_t nq, float spread_tol, float* d_mean,
                        float* d_spread, unsigned char* d_fallback, int64_t* d_fallback_idx,
                        int64_t* h_nfallback, void* stream);

/* Message for a status code (static string). */
const char* it_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* IONTRACKS_H */
