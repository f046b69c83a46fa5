/*
 * pcmcc.h -- C ABI of the MI355X (gfx950) PIC-MCC electron library.
 *
 * Method: the particle (PIC-MCC) model of Wang, Sun & Teunissen, "A
 * comparison of particle and fluid models for positive streamer discharges
 * in air" (arXiv:2110.14494), Sec. 2.1: electrons are advanced with velocity
 * Verlet in a field interpolated from a cell-centred grid (Sec. 2.1.1
 * eq. (1)-(2), Sec. 2.1.3), collide with a neutral background through the
 * null-collision method with rates from tabulated cross sections (Sec. 2.1.1,
 * Sec. 2.1.5), and are mapped back to the grid by trilinear weighting
 * (Sec. 2.1.3).  The same mover run in a uniform field gives the flux and bulk
 * swarm coefficients that feed the fluid model (Sec. 2.2.2).
 *
 * Conventions shared by every entry point:
 *   - SI units, except energies in eV and reduced fields E/N in Td
 *     (1 Td = 1e-21 V m^2).
 *   - Every function returns an int status (PCMCC_OK or a negative code);
 *     no exception crosses the ABI.  pcmcc_last_error() gives a text for the
 *     last failing call on a context.
 *   - "device" pointers are HIP device memory of the context's device;
 *     "host" pointers are ordinary host memory.  The library never frees or
 *     keeps caller memory beyond a call.
 *   - All work is queued on the context's HIP stream.  Calls that return
 *     statistics or host results synchronise that stream before returning.
 *   - A context is not thread safe: calls on one context must not overlap.
 */
#ifndef PCMCC_H
#define PCMCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define PCMCC_OK 0
#define PCMCC_EINVAL (-1)    /* invalid argument (null pointer, size, range) */
#define PCMCC_ECAPACITY (-2) /* a step would exceed the particle capacity */
#define PCMCC_EHIP (-3)      /* a HIP runtime call failed (text in last_error) */
#define PCMCC_ESTATE (-4)    /* species or tables not initialised */
#define PCMCC_ENOMEM (-5)    /* device allocation failed */
#define PCMCC_ETABLE (-6)    /* malformed cross-section table */
#define PCMCC_ELIMIT (-7)    /* a per-step safety limit was reached */
#define PCMCC_ERANGE (-8)    /* a charge outside the deposit's fixed-point range */

/* Collision process kinds (Sec. 2.1.5).  Cumulative rates are formed in the
 * order the processes are given to pcmcc_init_tables. */
#define PCMCC_ELASTIC 0
#define PCMCC_EXCITATION 1
#define PCMCC_IONIZATION 2
#define PCMCC_ATTACHMENT 3

/* pcmcc_init_tables flags. */
#define PCMCC_EFFECTIVE_TO_ELASTIC 1 /* elastic := effective momentum transfer
                                        minus the sum of the inelastic
                                        processes, clamped at 0 (Sec. 2.1.5) */
#define PCMCC_RATES 2                /* sigma already holds collision
                                        frequencies in 1/s (no N sigma v) */

typedef struct pcmcc_ctx pcmcc_ctx;

/* Particle arrays, structure of arrays, all device memory with room for
 * `capacity` particles.  Positions in m, velocities in m/s, w = number of
 * physical electrons represented (super-particle weight, Sec. 2.1.2), id = a
 * 64-bit identity that keys the particle's random numbers.  *n_dev (device)
 * holds the live count. */
typedef struct pcmcc_particles {
  float* x;
  float* y;
  float* z;
  float* vx;
  float* vy;
  float* vz;
  float* w;
  uint64_t* id;
  int64_t* n_dev;
  int64_t capacity;
} pcmcc_particles;

/* Cell-centred uniform grid: cell (i,j,k) has centre
 * (x0 + (i+1/2) dx, y0 + (j+1/2) dx, z0 + (k+1/2) dx); E is float4 per cell
 * (Ex, Ey, Ez, unused) in V/m, x fastest, device memory. */
typedef struct pcmcc_grid {
  const float* E; /* nx*ny*nz*4 floats */
  int nx, ny, nz;
  double x0, y0, z0, dx;
} pcmcc_grid;

/* Counters of one call, summed over the committed steps. */
typedef struct pcmcc_stats {
  int64_t n;                     /* live particles after the last committed step */
  int64_t steps_done;            /* committed steps */
  uint64_t particle_steps;       /* sum over committed steps of the count at the step's start */
  uint64_t trials;               /* flight segments (one random draw each) */
  uint64_t null_collisions;      /* includes collisions rejected below threshold */
  uint64_t real_collisions[4];   /* by kind: elastic, excitation, ionization, attachment */
  uint64_t lost;                 /* removed for leaving the grid */
  uint64_t out_of_table;         /* real collisions above the last table energy */
  uint64_t errors;               /* particles dropped at the per-step segment limit */
  double step_kernel_ms;         /* device time of the step loop kernel (HIP events on the stream) */
  double deposit_kernel_ms;      /* device time of the deposit kernel, 0 if skipped */
  int32_t launch_block;          /* threads per block of the step loop kernel */
  int32_t launch_grid;           /* blocks of the step loop kernel */
  int64_t weight_updates;        /* super-particle weight updates within the call (weight control) */
  int64_t merged_pairs;          /* pairs merged by those updates */
  int64_t splits;                /* particles split by those updates */
  double weight_ms;              /* device time of those updates */
  double field_ms;               /* self-consistent steps: device time of densities, potential and field */
  int64_t mg_cycles;             /* self-consistent steps: multigrid V-cycles */
  int64_t photons;               /* photoionization: photons emitted */
  int64_t photoelectrons;        /* photoionization: photons absorbed inside the grid */
  double photo_ms;               /* photoionization: device time */
  uint64_t majorant_violations;  /* candidate collisions whose total rate exceeded the majorant of their flight
                                    segment (the null-collision method, Sec. 2.1.1, needs 0; a nonzero count
                                    means the majorant rule is wrong) */
  int32_t launch_refill;         /* refill threshold of the step loop kernel (see pcmcc_schedule) */
  int32_t launch_chunk;          /* work-counter chunk of the step loop kernel */
} pcmcc_stats;

/* Version string, static storage. */
const char* pcmcc_version(void);

/* Creates a context on HIP device `device` issuing work on `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  *out receives the
 * context.  The library owns the context, its tables and its scratch
 * buffers (ping-pong particle buffers, newborn queues, counters). */
int pcmcc_create(pcmcc_ctx** out, int device, void* hip_stream);

/* Releases everything the context owns; ctx may be NULL. */
int pcmcc_destroy(pcmcc_ctx* ctx);

/* Text of the last error on ctx (empty string if none); valid until the next
 * call on ctx.  ctx may be NULL (then a global text is returned). */
const char* pcmcc_last_error(pcmcc_ctx* ctx);

/* Particle species and background gas (Sec. 2.1.1: a = (q/m) E with q = -e
 * for electrons; Sec. 2.3: gas number density N).  target_mass_kg is the
 * neutral mass used for the elastic recoil loss 2m/M (1 - cos chi).  Calling
 * it again invalidates the tables (pcmcc_init_tables must follow). */
int pcmcc_init_species(pcmcc_ctx* ctx, double mass_kg, double charge_C, double gas_N_m3, double target_mass_kg);

/* Cross-section tables (Sec. 2.1.5).  Energies are log-spaced:
 * eps_i = eps_min (eps_max/eps_min)^(i/(n_e-1)), i = 0..n_e-1.
 * kind[n_proc], threshold_eV[n_proc] and sigma_m2[n_proc][n_e] are host
 * arrays; sigma is in m^2 (or 1/s with PCMCC_RATES).  The library forms
 * nu_k = N sigma_k v(eps) in double precision, the cumulative sums in the
 * given process order and the prefix maximum of the total, and keeps them on
 * the device in single precision.  Rates are linear in ln(eps) between nodes
 * and constant outside [eps_min, eps_max]; a collision selected below its
 * process threshold is treated as null.  1 <= n_proc <= 8, 2 <= n_e <= 4096.
 * Returns PCMCC_ETABLE for negative/non-finite values or bad kinds. */
int pcmcc_init_tables(pcmcc_ctx* ctx, int n_e, double eps_min_eV, double eps_max_eV, int n_proc, const int* kind,
                      const double* threshold_eV, const double* sigma_m2, int flags);

/* Advances the particles n_steps steps of length dt in the fixed field, then
 * adds their charge to rho by trilinear (CIC) weighting (Sec. 2.1.1-2.1.3).
 * Per step every particle is moved from t = 0 and newborn electrons from
 * their birth time, all to the end of the step; attached particles and
 * particles outside the grid at the end of the step are removed.  Random
 * numbers are Philox4x32-10 keyed by `seed` with counter (id, step0 + s,
 * segment, purpose), so results do not depend on array order and a run of
 * 10 steps equals 5 steps plus 5 steps with step0 = 5.
 *   p      : device particle arrays, updated in place; the order of the
 *            particles on return is unspecified.
 *   field  : device field, read only.
 *   rho    : device int64 array laid out like the field, or NULL to skip the
 *            deposit.  It is accumulated into (the caller zeroes it): each
 *            particle adds round(w 2^32) split over the 8 nearest cell
 *            centres, indices clamped to the grid, exactly conserving the sum.
 *            Weights must lie in [0, 2^31) and every cell sum within int64
 *            (2^31 electrons per cell); otherwise PCMCC_ERANGE is returned
 *            after the steps, with rho unspecified.
 *   stats  : host, may be NULL.
 * On PCMCC_ECAPACITY the arrays hold the state after stats->steps_done
 * committed steps and the deposit is skipped.  Synchronises the stream. */
int pcmcc_push_collide_deposit(pcmcc_ctx* ctx, const pcmcc_particles* p, const pcmcc_grid* field, double dt,
                               int n_steps, uint64_t seed, uint64_t step0, int64_t* rho, pcmcc_stats* stats);

/* ---- Schedule of the step kernel ------------------------------------------
 * How the electrons of a step are spread over the GPU; it changes the time
 * of pcmcc_push_collide_deposit (and of the calls built on it), never its
 * results (random numbers follow the electron ids, not the schedule).  A
 * zero field takes the default. */
typedef struct pcmcc_schedule {
  int block;          /* threads per block: 64, 128, 256 or 512; 0 = the size with the most resident waves per
                         compute unit (ties: the larger block), or 64 for a call that starts with fewer than
                         2^17 particles */
  int blocks_per_cu;  /* persistent blocks per compute unit; 0 = as many as fit (1 with the 64-thread default of a
                         small call) */
  int refill_min;     /* free lanes of a wave that trigger a finish-and-refill batch: 16, 24 or 32; 0 = 24 */
  int chunk;          /* electrons a wave takes from the work counter at a time: a power of two in [64, 4096];
                         0 = 512 (64 for a call that starts with fewer than 2^17 particles) */
} pcmcc_schedule;

/* Sets the schedule of later steps on ctx (s NULL: all defaults).
 * PCMCC_EINVAL for a value outside the ranges above. */
int pcmcc_set_schedule(pcmcc_ctx* ctx, const pcmcc_schedule* s);

/* The schedule the next step call on ctx uses for this field's tables and
 * block limits, every field resolved, for a call that starts with 2^17
 * particles or more (host *out). */
int pcmcc_get_schedule(pcmcc_ctx* ctx, pcmcc_schedule* out);

/* Launch-shape tuner of the step kernel: times n_steps steps (seed, step0
 * as pcmcc_push_collide_deposit, no deposit) of the particles p in `field`
 * under each candidate schedule -- the default, then block x blocks per
 * compute unit, then refill threshold x chunk at the best shape so far --
 * and sets the fastest on ctx.  p is restored to its input state (the tuner
 * allocates one copy of it).  With tune_cache (a JSON file, or NULL) a
 * schedule stored for the same workload key (particle count rounded to a
 * power of two, grid size, tables) is taken without timing, and a new one
 * is stored.  chosen (host, nullable) receives the schedule; tuned_ms and
 * default_ms (host, nullable) the step-kernel times of the chosen and the
 * default schedule (both 0 when taken from the cache).  Errors as
 * pcmcc_push_collide_deposit; synchronises the stream. */
int pcmcc_autotune_steps(pcmcc_ctx* ctx, const pcmcc_particles* p, const pcmcc_grid* field, double dt, int n_steps,
                         uint64_t seed, uint64_t step0, const char* tune_cache, pcmcc_schedule* chosen,
                         float* tuned_ms, float* default_ms);

/* ---- Batched uniform-field swarms (Sec. 2.2.2) ---------------------------
 * Swarm s starts with n0[s] electrons at rest at the origin in the field
 * E = EN_Td[s] * 1e-21 * N along +z and is advanced n_steps steps of dt with
 * the same mover as pcmcc_push_collide_deposit (newborns, attachment), all
 * swarms in one persistent launch.  Random numbers: Philox4x32-10 with key
 * (seed low word, seed high word XOR s) and counter (id, step, segment,
 * purpose); initial ids are 0..n0[s]-1.
 * Every sample_every steps, after the step's newborns, the moments of each
 * swarm are summed exactly (128-bit fixed point); then, with population
 * control on, a swarm above 2 n0 keeps each electron with probability 2^-k
 * (the smallest k that brings the expected size to 2 n0 or below) and a
 * swarm below n0/2 duplicates every electron, the weight scale 2^L of the
 * swarm following.  From the samples with t >= window_start_s:
 *   W_flux = -<v_z> (time mean),  W_bulk = -d<z>/dt,
 *   DL_flux = <dz dv_z>,  DL_bulk = (1/2) d var(z)/dt,
 *   DT_flux = (1/2) <dx dv_x + dy dv_y>,  DT_bulk = (1/4) d (var x + var y)/dt,
 *   nu_ion, nu_att = time means of the rate functions over the population,
 *   nu_eff = d ln(N 2^L)/dt (temporal growth),  mean energy,
 *   mu = W_flux/E,  alpha = nu_ion/W_flux,  eta = nu_att/W_flux,
 *   W_bulk/W_flux; slopes are least-squares fits against time; errors are
 *   batch means over n_batches contiguous sub-windows.  Drift is positive
 *   along -E (electrons). */
#define PCMCC_SWARM_NQ 14
#define PCMCC_Q_W_FLUX 0
#define PCMCC_Q_W_BULK 1
#define PCMCC_Q_DL_FLUX 2
#define PCMCC_Q_DL_BULK 3
#define PCMCC_Q_DT_FLUX 4
#define PCMCC_Q_DT_BULK 5
#define PCMCC_Q_NU_ION 6
#define PCMCC_Q_NU_ATT 7
#define PCMCC_Q_NU_EFF 8
#define PCMCC_Q_MEAN_EPS 9
#define PCMCC_Q_MU 10
#define PCMCC_Q_ALPHA 11
#define PCMCC_Q_ETA 12
#define PCMCC_Q_BULK_FLUX_RATIO 13
#define PCMCC_SWARM_NMOM 14 /* moments per sample: count, Sx, Sy, Sz, S(x^2+y^2), Sz^2, Svx, Svy,
                               Svz, S(x vx + y vy), S(z vz), S eps, S nu_ion(eps), S nu_att(eps) */

typedef struct pcmcc_swarm_opts {
  int sample_every;        /* steps between samples, >= 1 */
  double window_start_s;   /* estimators use samples at t >= this */
  int n_batches;           /* sub-windows of the batch-means error, >= 2 */
  int cap_factor;          /* slots per swarm = cap_factor * n0, >= 4 */
  int population_control;  /* 1 on, 0 off */
  int block;               /* threads per block: 64, 128, 256, 512; 0 = tuned or default */
  int blocks_per_cu;       /* persistent blocks per compute unit; 0 = tuned or default */
  int autotune;            /* 1: time the candidate shapes on this input and keep the fastest */
  const char* tune_cache;  /* JSON file the tuned shapes are read from and written to, or NULL */
  int refill_min;          /* as pcmcc_schedule; 0 = tuned or 24 */
  int chunk;               /* as pcmcc_schedule; 0 = tuned or 512 */
} pcmcc_swarm_opts;

typedef struct pcmcc_swarm_result {
  double value[PCMCC_SWARM_NQ];
  double error[PCMCC_SWARM_NQ];
} pcmcc_swarm_result;

/* EN_Td[n_swarms], n0[n_swarms] host; out[n_swarms] host.  Optional host
 * outputs (NULL to skip): moments_out[n_swarms][J][14] double sums and
 * counters_out[n_swarms][J][4] (live count, L, cumulative ionizations,
 * cumulative attachments), J = n_steps / sample_every.  1 <= n_swarms <= 4096,
 * n0[s] >= 1.  PCMCC_ECAPACITY if a swarm outgrows its slots within a step.
 * Synchronises the stream. */
int pcmcc_swarm_batch(pcmcc_ctx* ctx, int n_swarms, const double* EN_Td, const int32_t* n0, double dt, int n_steps,
                      uint64_t seed, const pcmcc_swarm_opts* opts, pcmcc_swarm_result* out, double* moments_out,
                      int64_t* counters_out, pcmcc_stats* stats);

/* ---- Coefficient surrogate ---------------------------------------------
 * A perceptron 1 -> 64 -> 64 -> 6 with tanh hidden layers maps the
 * standardised input x = (ln(E/N) - mu_x) / sd_x to six standardised log
 * swarm coefficients (ln mobility N, ln D_L N, ln alpha/N, ln eta/N, ln mean
 * energy, ln W_bulk/W_flux), i.e. the transport data of the fluid model
 * (Sec. 2.2), learned from pcmcc_swarm_batch output.  Parameters are one
 * float vector of PCMCC_MLP_PARAMS values: W1[64,1], b1[64], W2[64,64],
 * b2[64], W3[6,64], b3[6] (row-major).  Loss: masked mean squared error
 * sum(mask (y - t)^2) / sum(mask). */
#define PCMCC_MLP_PARAMS 4678
#define PCMCC_MLP_OUT 6

/* Loss and gradient for the parameters at params (single precision, fixed
 * summation order).  params[4678], x[n], t[n][6], mask[n][6], grad_out[4678]
 * and loss_out are host memory.  n >= 1, sum(mask) > 0. */
int pcmcc_mlp_grad(pcmcc_ctx* ctx, const float* params, int64_t n, const float* x, const float* t,
                   const float* mask, float* grad_out, double* loss_out);

typedef struct pcmcc_mlp_train_opts {
  int epochs;           /* full-batch Adam steps */
  double lr0, lr_min;   /* cosine schedule: lr_min + (lr0 - lr_min)(1 + cos(pi e / epochs)) / 2 */
  double beta1, beta2, eps;
} pcmcc_mlp_train_opts;

/* Trains from params_in with full-batch Adam in one persistent launch; the
 * result is bit-reproducible.  params_out[4678] host; loss_hist[epochs]
 * (host, nullable) gets the loss before each update; stats (nullable) gets
 * the kernel time. */
int pcmcc_mlp_train(pcmcc_ctx* ctx, const float* params_in, int64_t n, const float* x, const float* t,
                    const float* mask, const pcmcc_mlp_train_opts* opts, float* params_out, float* loss_hist,
                    pcmcc_stats* stats);

typedef struct pcmcc_mlp_infer_opts {
  double mu_x, sd_x;                       /* input standardisation */
  double mu_y[PCMCC_MLP_OUT], sd_y[PCMCC_MLP_OUT]; /* output un-standardisation */
  int n_cells;                             /* fallback cells uniform in ln(E/N) over [cell_lo, cell_hi); 0 = none */
  double cell_lo, cell_hi;
  const uint8_t* fallback;                 /* host [n_cells]: bit k set = output k takes the table in this cell
                                              (0x3F: every output) */
  int n_nodes;                             /* table nodes uniform in ln(E/N) from table_lo to table_hi */
  double table_lo, table_hi;
  const float* table;                      /* host [n_nodes][6] ln coefficients (linear interpolation) */
} pcmcc_mlp_infer_opts;

/* Evaluates the surrogate at n reduced fields EN_dev (device, Td) with
 * bfloat16 weights and activations and single-precision accumulation (MFMA);
 * out_dev (device) receives [6][n] ln coefficients (output-major).  The
 * outputs flagged in a point's fallback cell take the linear interpolation of
 * the table instead. */
int pcmcc_mlp_infer(pcmcc_ctx* ctx, const float* params, const pcmcc_mlp_infer_opts* opts, int64_t n,
                    const float* EN_dev, float* out_dev, pcmcc_stats* stats);

/* Training data from swarm results: x = ln(E/N / 1 Td); targets = ln(mu N),
 * ln(DL_flux N), ln(alpha / N), ln(eta / N), ln(mean energy / 1 eV),
 * ln(W_bulk / W_flux) (SI units).  An entry is masked when its value is not
 * positive and finite or its relative batch-means error exceeds max_rel_err
 * (unresolved, e.g. rare ionization or attachment events).  With
 * compute_norm = 1 the standardisation (mean, std over unmasked entries) is
 * computed into norm (mu_x, sd_x, mu_y, sd_y); otherwise norm is used as
 * given.  x_out[n], t_out[n][6], mask_out[n][6] are the standardised data;
 * ln_out[n][6] (nullable) the unstandardised ln values with masked entries
 * set to ln_floor; sig_out[n][6] (nullable) the relative batch-means error of
 * each entry, the standard error of its ln value to first order (NaN where
 * masked).  Host memory; no device work. */
int pcmcc_mlp_dataset(int n, const double* EN_Td, const pcmcc_swarm_result* res, double gas_N, double max_rel_err,
                      int compute_norm, pcmcc_mlp_infer_opts* norm, float* x_out, float* t_out, float* mask_out,
                      float* ln_out, float* sig_out, double ln_floor);

/* Held-out check of a trained surrogate: evaluates it (the bfloat16 device
 * path) at n_held reduced fields; of n_cells cells uniform in ln(E/N) over
 * [cell_lo, cell_hi), output k of cell c falls back (bit k of
 * fallback_out[c]) if, for any held-out point in the cell, that output is
 * masked or |ln y_mlp - ln y_swarm| > tol_ln + z_sig sig, sig being the
 * held-out value's own Monte Carlo standard error in ln units (sig_held NULL
 * means 0).  z_sig > 0 forgives the held-out value's noise; z_sig < 0 asks the
 * held-out evidence to show the error below tol_ln with a margin of |z_sig|
 * standard errors (an output whose sig reaches tol_ln / |z_sig| always falls
 * back).  A cell holding no held-out point falls back in every output
 * (0x3F).  ln_held, mask_held and sig_held [n_held][6] are unstandardised ln
 * targets, their mask and errors (host); fallback_out[n_cells] host;
 * err_out[n_held][6] (nullable) receives the absolute ln errors (NaN where
 * masked). */
int pcmcc_mlp_fallback(pcmcc_ctx* ctx, const float* params, const pcmcc_mlp_infer_opts* norm, int n_held,
                       const double* EN_held, const float* ln_held, const float* mask_held, const float* sig_held,
                       double tol_ln, double z_sig, int n_cells, double cell_lo, double cell_hi,
                       uint8_t* fallback_out, float* err_out);

/* ---- Super-particle weights (Sec. 2.1.2) --------------------------------
 * Desired weight of a cell: omega = n_e dV / n_ppc, n_e dV being the electrons
 * the CIC mapping puts on the cell, and at least 1.  Particles in a cell with
 * w < (2/3) omega are merged pairwise: the candidates of a cell are ordered
 * by |v|^2 (rounded to single precision), then by id, consecutive ones are
 * paired and the pair becomes one particle of weight w_a + w_b with the
 * position, velocity and id of the first with probability w_a / (w_a + w_b),
 * else of the second (an odd one out is left as it is).  Particles with
 * w > (3/2) omega are halved and copied (same position and velocity).
 * Random numbers: Philox4x32-10 keyed by `seed`, counter (id, update_index,
 * 0, purpose 3) — the smaller id of a pair decides the merge, a split copy's
 * id is the second and third words of its particle's draw.  The result does
 * not depend on the array order (the order on return is unspecified). */

/* Enables (n_ppc > 0) or disables (n_ppc = 0) weight control in
 * pcmcc_push_collide_deposit: after a committed step whose particle count
 * exceeds floor(growth * n_ref), the weights are updated with update_index =
 * the absolute index of that step, and n_ref becomes the new count; n_ref is
 * the count at the start of the first call after this one, and is kept across
 * calls.  growth >= 1 (the paper uses 1.25).  An update that fails
 * (PCMCC_ECAPACITY, PCMCC_ERANGE) ends the call with that code and the
 * particles of the last committed step. */
int pcmcc_set_weight_control(pcmcc_ctx* ctx, double n_ppc, double growth);

/* One weight update of the device particles p (in place, *p->n_dev updated)
 * on `grid` (only its geometry is used).  merged_pairs and splits (host,
 * nullable) receive the counts.  PCMCC_ECAPACITY (particles unchanged) if the
 * result exceeds p->capacity; PCMCC_ERANGE (particles unchanged) if the
 * density is outside the deposit's fixed-point range.  Synchronises the
 * stream. */
int pcmcc_update_weights(pcmcc_ctx* ctx, const pcmcc_particles* p, const pcmcc_grid* grid, double n_ppc,
                         uint64_t seed, uint64_t update_index, int64_t* merged_pairs, int64_t* splits);

/* ---- Self-consistent step (Sec. 2.5, Sec. 2.3, Sec. 2.1.4) ----------------
 * Space charge rho = e (n_+ - n_e - n_-), each density a fixed-point CIC grid
 * as above (int64, 2^-32 electrons per unit, laid out like the field).  The
 * potential of the space charge solves lap phi = -rho / eps0 (Sec. 2.5, the
 * sign read as a typo) on the cell centres with phi = 0 on the two z faces and
 * zero normal derivative on the x and y faces (Sec. 2.3): the 7-point stencil
 * with ghost cells (Dirichlet ghost = -phi of the boundary cell, Neumann ghost
 * = phi).  The caller's grid field is the applied field (it stands in for the
 * electrode and the applied voltage); the electrons see E = E_applied -
 * grad phi, central differences with the same ghosts.  Ions do not move. */

/* Geometric multigrid on phi (device, double [nz][ny][nx], the start value
 * and the result) as defect correction: the residual in double precision,
 * one single-precision V(2,2) cycle for the correction, repeated until
 * max |residual| <= tol * max |rhs| or max_cycles cycles; the grid is halved
 * while every dimension is even
 * and above 2, and the coarsest grid must hold at most 4096 cells (else
 * PCMCC_EINVAL).  n_pos, n_e, n_neg: device int64 densities.  cycles_out and
 * rel_residual_out (host, nullable) receive the cycles run and the final
 * relative residual.  Synchronises the stream. */
int pcmcc_solve_potential(pcmcc_ctx* ctx, const pcmcc_grid* grid, const int64_t* n_pos, const int64_t* n_e,
                          const int64_t* n_neg, double* phi, double tol, int max_cycles, int* cycles_out,
                          double* rel_residual_out);

/* E_out (device float4 per cell, 4th component 0) = applied->E - grad phi. */
int pcmcc_field_from_potential(pcmcc_ctx* ctx, const pcmcc_grid* applied, const double* phi, float* E_out);

/* Speed at the 90 % quantile (Sec. 2.1.4): with keys |v|^2 = (vx^2 + vy^2) +
 * vz^2 in double from the single-precision components, rounded to single
 * precision, the key of rank ceil(9 n / 10) in ascending order (exact radix
 * selection); *v90_out = its square root (0 for no particles).  Device arrays,
 * *n_dev device count. */
int pcmcc_speed_quantile(pcmcc_ctx* ctx, const float* vx, const float* vy, const float* vz, const int64_t* n_dev,
                         double* v90_out);

/* ---- Discrete photoionization (Sec. 2.4) -----------------------------------
 * Zheleznyak's model of photoionization in air with discrete photons.
 * Ionizing photons are produced in proportion to the electron-impact
 * ionizations, eta = p_q / (p + p_q) xi photons per ionization (eq. of the UV
 * source term; the paper: p_q = 40 mbar, xi = 0.075).  They fly in isotropic
 * directions without scattering and are absorbed at a distance r drawn from
 * the absorption function f(r) = (exp(-k1 r) - exp(-k2 r)) / (r ln(k2 / k1)).
 * Each absorbed photon leaves a photoelectron at rest and a positive ion at
 * the absorption point.  The paper does not give k1 and k2 (the oxygen
 * partial pressure times Zheleznyak's chi_min and chi_max): they are inputs.
 *
 * Per ionization event of weight w: lambda = eta w / w_photon photons of
 * weight w_photon (w_photon <= 0: of the event's weight, lambda = eta), and
 * the count is floor(lambda) + [U < lambda - floor(lambda)] (an event with
 * lambda >= 2^31 counts as 2^31 photons, which no capacity accepts).  Draws are
 * Philox4x32-10 with key (seed low word ^ 0x50484F54, seed high word ^ step
 * low word) and counter (bit patterns of the event's x, y, z; c), output
 * words r0..r3: c = 0 gives the count's U = (r0 + 1/2) 2^-32; c = 2j + 1
 * photon j's direction (cos theta = 1 - 2 u(r0), azimuth 2 pi u(r1),
 * u(r) = (r + 1/2) 2^-32) and distance (U = ((r2 >> 5) 2^26 + (r3 >> 6) +
 * 1/2) 2^-53, r solving F(r) = U to about 1e-14 in ln r within
 * [ln(1e-6 / k2), ln(60 / k1)], F(r) = 1 - (E1(k1 r) - E1(k2 r)) / ln(k2 / k1)
 * the distribution function of f); c = 2j + 2 its id (r0 | r1 << 32).  The
 * absorption point x + r n is rounded to single precision; a photon absorbed
 * outside [x0, x0 + nx dx) x [y0, ..) x [z0, ..) is lost. */
typedef struct pcmcc_photo_opts {
  double eta;      /* photons per ionization, p_q / (p + p_q) xi */
  double k1, k2;   /* absorption coefficients (1/m), 0 < k1 < k2 */
  double w_photon; /* weight of a photoelectron; <= 0: the ionizing event's weight */
} pcmcc_photo_opts;

/* Photoionization from n_ev ionization events at device float arrays ev_x,
 * ev_y, ev_z (positions, m) and ev_w (weights).  The photoelectrons are
 * appended to p (after its *n_dev particles, velocity 0, ids from the draws;
 * order unspecified) and, if n_pos is not null, their charge is added to the
 * device int64 grid n_pos as by pcmcc_deposit (PCMCC_ERANGE as there).  If
 * the emitted photons could exceed p->capacity, PCMCC_ECAPACITY and nothing
 * changes.  photons_out / absorbed_out (host, nullable): photons emitted and
 * photoelectrons appended.  Synchronises the stream. */
int pcmcc_photoionize(pcmcc_ctx* ctx, const pcmcc_grid* grid, const float* ev_x, const float* ev_y,
                      const float* ev_z, const float* ev_w, int64_t n_ev, const pcmcc_photo_opts* opts,
                      uint64_t seed, uint64_t step, const pcmcc_particles* p, int64_t* n_pos, int64_t* photons_out,
                      int64_t* absorbed_out);

typedef struct pcmcc_sc_opts {
  int adaptive;          /* 0: every step takes *dt_inout; 1: the Sec. 2.1.4 rule below */
  double dt_max;         /* upper bound of the adaptive step (s) */
  double cfl;            /* dt <= cfl dx / v90 (the paper: 0.5) */
  double growth_max;     /* the electron number may grow by this factor per step (the paper: 1.2) */
  int mu_n;              /* electron mobility table: mu N (1/(V m s)) at mu_n log-spaced E/N nodes */
  double mu_EN_lo, mu_EN_hi; /* (Td) first and last node; mu_n = 1: a constant */
  const double* mu_N;    /* host [mu_n] */
  double mg_tol;         /* multigrid relative residual */
  int mg_max_cycles;
  const pcmcc_photo_opts* photo; /* nullable: photoionization from each step's ionizations (host struct) */
} pcmcc_sc_opts;

/* n_steps self-consistent steps.  Before each step the field is computed from
 * the present densities (electrons deposited from p, ions from n_pos and
 * n_neg); the electrons then take one step of pcmcc_push_collide_deposit in
 * that field (weight control applies as set); every ionization adds the
 * newborn's charge to n_pos at its position and every attachment the
 * electron's charge to n_neg (device int64 grids, caller-owned, accumulated:
 * initialise n_pos with the electron density for a neutral seed, Sec. 2.3).
 * With opts->adaptive the next step is dt = min(dt_max, cfl dx / v90,
 * eps0 / (e n_e,max mu_e), dt ln(growth_max) / ln(N_new / N_old)) with v90 as
 * pcmcc_speed_quantile, n_e,max the largest electron density (first cell in
 * x-fastest order), mu_e from the table at that cell's |E|/N (linear in
 * ln E/N, clamped), N the sum of the weights (the last term only when N
 * grew).  *dt_inout: host, the first step in, the next step out; dt_hist
 * (host [n_steps], nullable) receives the steps taken.  phi (device double)
 * is the multigrid start value and holds the last potential; E_out (device
 * float4, nullable) the field of the final state.  On an error from a step
 * (PCMCC_ECAPACITY, PCMCC_ERANGE from a weight update) the particles and ion
 * grids hold the state after stats->steps_done steps; on PCMCC_ERANGE from the
 * deposit of a step's ions the particles hold the state after steps_done
 * steps and the ion grids lack (part of) that last step's ions.  With
 * opts->photo, after each step's ion deposit the step's ionizations emit
 * photons as pcmcc_photoionize (seed, step index step0 + s): photoelectrons
 * join p, their ions n_pos, before the next field; on PCMCC_ECAPACITY from it
 * the particles and ion grids hold that step without its photoelectrons.
 * stats: photons, photoelectrons, photo_ms.  Synchronises the stream. */
int pcmcc_streamer_steps(pcmcc_ctx* ctx, const pcmcc_particles* p, const pcmcc_grid* applied, int64_t* n_pos,
                         int64_t* n_neg, double* phi, float* E_out, const pcmcc_sc_opts* opts, int n_steps,
                         uint64_t seed, uint64_t step0, double* dt_inout, double* dt_hist, pcmcc_stats* stats);

/* ---- Fluid step (Sec. 2.2) -------------------------------------------------
 * Drift-diffusion-reaction model in the local field approximation: electrons
 * drift with v = -mu E, flux = v n_face - D grad n, dn_e/dt = -div(flux) +
 * (alpha - eta) mu |E| n_e; positive ions gain alpha mu |E| n_e, negative ions
 * eta mu |E| n_e; ions do not move (photoionization is not included).  Face
 * field = mean of the two cells' fields, mu and D from its magnitude, the
 * advected face density the upwind value plus half the Koren-limited slope;
 * densities have homogeneous Neumann boundaries (mirror ghosts, Sec. 2.3).
 * Heun's method with the field (as pcmcc_solve_potential, from the densities
 * in double precision) recomputed for the predicted state; per step
 * dt = min(dt_max, 0.9 min(0.5 / max(6 D / dx^2 + sum |v_i| / dx),
 * eps0 / max(e n_e mu))) (the printed CFL limit drops D from its diffusion
 * term).  Transport data: mu N, D N, alpha / N, eta / N (SI) on tab->n
 * log-spaced E/N nodes from EN_lo to EN_hi (Td), linear in ln E/N, held
 * constant outside; N is the gas density of pcmcc_init_species. */
typedef struct pcmcc_fluid_table {
  int n;
  double EN_lo, EN_hi;
  const double* muN;
  const double* DN;
  const double* alphaN;
  const double* etaN;
} pcmcc_fluid_table;

/* n_steps Heun steps.  n_e, n_pos, n_neg: device double [nz][ny][nx]
 * densities (m^-3), updated in place; phi: device double, the multigrid start
 * value and the last potential; dt_hist: host [n_steps] (nullable); E_out:
 * device float4 field of the final state (nullable).  stats: steps_done,
 * step_kernel_ms (the two stage kernels), field_ms (right-hand sides,
 * multigrid, fields), mg_cycles.  Synchronises the stream. */
int pcmcc_fluid_steps(pcmcc_ctx* ctx, const pcmcc_grid* applied, double* n_e, double* n_pos, double* n_neg,
                      double* phi, const pcmcc_fluid_table* tab, double dt_max, double mg_tol, int mg_max_cycles,
                      int n_steps, double* dt_hist, float* E_out, pcmcc_stats* stats);

/* Deposit only (Sec. 2.1.3), same fixed-point rule and range as above
 * (PCMCC_ERANGE, rho unspecified, beyond it), on n_dev particles (device
 * count) of device arrays x, y, z, w.  Synchronises the stream. */
int pcmcc_deposit(pcmcc_ctx* ctx, const float* x, const float* y, const float* z, const float* w,
                  const int64_t* n_dev, const pcmcc_grid* grid, int64_t* rho);

/* Allocation-free variant of pcmcc_deposit, for callers that cannot
 * allocate device memory (code being captured into a graph, tight serving
 * loops, harnesses that forbid allocation): the same arguments, result and
 * errors, but the call allocates nothing.  Its scratch is one file-scope
 * device array per GPU (about 50 MiB, held until the process ends) that every
 * call on that GPU shares, so calls that overlap on one GPU race.  Limits:
 * at most 2^21 particles and 2^18 tiles of 8^3 cells (a 512^3 grid); beyond
 * them PCMCC_EINVAL and rho is untouched.  Synchronises the stream. */
int pcmcc_deposit_noalloc(pcmcc_ctx* ctx, const float* x, const float* y, const float* z, const float* w,
                          const int64_t* n_dev, const pcmcc_grid* grid, int64_t* rho);

/* Philox4x32-10 (Salmon et al., SC'11) on n device counters ctr[n][4] with
 * key (seed low word, seed high word); out[n][4] device.  Self-test of the
 * generator every kernel uses. */
int pcmcc_philox4x32_10(pcmcc_ctx* ctx, int64_t n, const uint32_t* ctr, uint64_t seed, uint32_t* out);

/* Table lookups as the kernels do them, for checking the device tables:
 * cum_out[n][n_proc] = cumulative rates at eps[n] (linear in ln eps between
 * nodes, held constant outside the table); if maj_out is not NULL,
 * maj_out[n] = the collision-frequency majorant for a particle whose speed
 * stays below s_ub[n] (m/s): the prefix maximum of the total rate at the
 * energy of s_ub (inflated by 2^-16).  All arrays device. */
int pcmcc_tables_lookup(pcmcc_ctx* ctx, int64_t n, const float* eps, float* cum_out, const float* s_ub,
                        float* maj_out);

#ifdef __cplusplus
}
#endif

#endif /* PCMCC_H */
