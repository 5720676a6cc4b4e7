/*
 * sg.h -- C-ABI of the MI355X (gfx950) checkerboard spin-glass sweep library
 * (libsg.so).
 *
 * Method: Belletti et al., "Simulating spin systems on IANUS, an FPGA-based
 * computer" (arXiv 0704.3573).  Single-spin Metropolis and heat-bath dynamics
 * (sec. 2.2, Eq. 4) of the 3D Edwards-Anderson +-J Ising glass (Eq. 2 with
 * x = 1, h = 0, sec. 2.1), of the Ising-like models of Eq. 2 with dilution
 * and field (random-field Ising model, diluted antiferromagnet in a field),
 * of the q = 4 +-J Potts glass H = -sum J_ij delta(s_i, s_j) and of the
 * glassy Potts model of Eq. 3, updated colour by colour on the bipartite
 * lattice (sec. 3.1), every site update consuming one Parisi-Rapuano number
 * (sec. 3.3, Eq. 5) compared with an integer threshold.  Parallel tempering,
 * which sec. 2.2 names as an add-on, swaps temperatures between slots.
 *
 * Conventions (canonical host formats), shared with the project's CPU oracle:
 *   - cubic periodic lattice of side L, site i = x + L*(y + L*z), N = L^3;
 *   - colour p = (x + y + z) mod 2, colour 0 is updated first;
 *   - a job has S samples, R replicas, K temperature slots; copy (slot)
 *     c = (s*R + r)*K + k, C = S*R*K copies;
 *   - couplings int8 [S][3][N], J[s][d][i] (+1/-1) joins i and i + e_d;
 *   - Ising spins int8 +1/-1, Potts spins uint8 0..3, [C][N];
 *   - sweep wheels uint32 [C][NW][61] with NW = L * L / min(8, L) (one per
 *     plane z and group of min(8, L) rows, index g*L + z), words I(k-61) ..
 *     I(k-1) oldest first; parallel-tempering wheels uint32 [S*R][61];
 *   - slot_of_temp int32 [S*R][K]: slot holding temperature index k;
 *   - energies and overlaps int64.
 * Which random number feeds which site: wheel (c, z, g) serves rows
 * y = g*rho .. g*rho + rho - 1 (rho = min(8, L)) of plane z and draws, in every
 * sweep, colour 0 then colour 1, rows ascending, x ascending, one number per
 * visited site.
 *
 * Errors: every call returns SG_OK (0) or a negative SG_E_* code; the message
 * of the last error on the calling thread is returned by sg_last_error().  No
 * C++ exception crosses this boundary.  Device errors raised asynchronously
 * surface at the next call that synchronises.
 * Test hook: when the environment variable SG_TEST_INJECT_HIP_ERROR holds
 * the name of sg_job_create, sg_job_sweep, sg_job_measure, sg_job_restore,
 * sg_batch_run, sg_batch_run_static or sg_threshold_row, that call returns
 * SG_E_HIP at entry, before it changes any state (fault-path tests).
 *
 * Ownership: handles are created and released by the library.  Device memory
 * of a job (its "arena") is owned by the caller: ask sg_job_bytes(), allocate
 * that many bytes on the device (for example a torch uint8 tensor) and pass
 * the pointer; it must stay valid until sg_job_destroy().  Host arrays are
 * owned by the caller and only read (or written) during the call.  Streams
 * are hipStream_t values passed as void* (NULL = the default stream); all
 * work is stream ordered, calls marked (sync) wait for it.
 */
#ifndef SG_H
#define SG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SG_OK 0
#define SG_E_INVALID (-1)     /* bad argument or specification              */
#define SG_E_UNSUPPORTED (-2) /* lattice size / model not built             */
#define SG_E_NOMEM (-3)       /* arena (or budget) too small                */
#define SG_E_HIP (-4)         /* the HIP runtime reported an error          */
#define SG_E_STATE (-5)       /* call not valid in the current state        */

#define SG_ISING 0
#define SG_POTTS 1  /* q = 4 +-J Potts glass, H = -sum J_ij delta(s_i, s_j)          */
#define SG_GPOTTS 2 /* q = 4 glassy Potts model of Eq. (3), permutation couplings */
/* Ising-like model of Eq. (2): H = -sum_<ij> J_ij x_i x_j s_i s_j
 * - sum_i h_i x_i s_i with dilution x_i in {0, 1} and field h_i = field * f_i,
 * f_i = +-1 (RFIM: J = +1, x = 1; DAFF: J = -1, f = +1).  The energy the
 * library reports for it is the bond part E_b (first sum); the field sum
 * M = sum_i x_i f_i s_i comes from sg_job_field_sums, and H = E_b - field * M.
 * Overlaps count occupied sites only.  No parallel tempering. */
#define SG_ISING_GEN 3
/* q = 4 glassy Potts model of Eq. (3) on the 4D hypercubic lattice (the
 * paper's 4D runs, sec. 4.2): side L in {2, 4, 8, 16}, site
 * i = x + L*(y + L*(z + L*u)), N = L^4, couplings [S][4][N] permutation
 * bytes (d = x, y, z, u), heat bath; one sweep wheel per (z, u, group of
 * min(8, L) rows), index (g*L + u)*L + z, drawing in the 3D order (colour
 * (x+y+z+u) mod 2, rows, x): sg_model_wheels_per_copy(SG_GPOTTS4, L) wheels. */
#define SG_GPOTTS4 4
#define SG_METROPOLIS 0
#define SG_HEATBATH 1

typedef struct sg_ctx sg_ctx;
typedef struct sg_job sg_job;
typedef struct sg_batch sg_batch;

typedef struct sg_job_spec {
  int32_t model;      /* SG_ISING, SG_POTTS, SG_GPOTTS, SG_ISING_GEN, SG_GPOTTS4 */
  int32_t algo;       /* SG_METROPOLIS or SG_HEATBATH (Potts models: heat bath) */
  int32_t q;          /* Potts states, must be 4 (ignored for Ising)            */
  int32_t L;          /* 2, 4, 8, 16, 24, 32, 40, 48, 56, 64 (Potts: <= 48)     */
  int32_t n_samples;  /* S >= 1                                                 */
  int32_t n_replicas; /* R >= 1 (overlaps need R >= 2)                          */
  int32_t n_temps;    /* K >= 1                                                 */
  int32_t pt_every;   /* sweeps between parallel-tempering steps, 0 = none      */
  double field;       /* SG_ISING_GEN: |h| >= 0, finite; ignored otherwise       */
  uint64_t seed;      /* instance seed: inputs passed as NULL to sg_job_create
                         are generated from it (sg_generate)                    */
  uint64_t sample0;   /* global number of the job's first sample (a campaign
                         split over several jobs keeps every sample's inputs)   */
} sg_job_spec;

/* Message of the last error on this thread ("" if none). */
const char *sg_last_error(void);

/* Number of sweep wheels per copy for side L (0 if L is not supported): one
 * wheel per plane z and group of min(8, L) rows (a reading of sec. 3.3,
 * which lets one wheel feed many update cells without fixing the mapping). */
int32_t sg_wheels_per_copy(int32_t L);
/* The same for a model: SG_GPOTTS4 has one wheel per (z, u, row group),
 * L^3 / min(8, L); every other model as sg_wheels_per_copy(L). */
int32_t sg_model_wheels_per_copy(int32_t model, int32_t L);

/* Bind a context to HIP device `device` (the kernels are built for gfx950;
 * SG_E_UNSUPPORTED on any other device). */
int sg_ctx_create(int device, sg_ctx **out);
int sg_ctx_destroy(sg_ctx *ctx);

/* Device bytes needed by a job with this specification. */
int sg_job_bytes(const sg_job_spec *spec, uint64_t *bytes);

/*
 * Host only (no device needed): the seeded instance of a specification, in
 * the canonical formats above.  Sec. 2.1 draws the couplings at random
 * (+-1 with p = 1/2; iid permutations for Eq. 3; for SG_ISING_GEN the
 * general mix of Eq. 2: J, x and f iid) and sec. 3.3 loads the wheels with
 * externally generated random values; here every array is a SplitMix64
 * counter stream keyed by (spec->seed, array, global sample/copy/chain
 * number from spec->sample0, wheel).  Any output pointer may be NULL (not
 * generated).  Sizes: J [S][3][N] (SG_ISING_GEN [S][5][N], SG_GPOTTS4
 * [S][4][N]), spins [C][N], wheels [C][NW][61], ptwheels [S*R][61].
 */
int sg_generate(const sg_job_spec *spec, int8_t *J, void *spins, uint32_t *wheels,
                uint32_t *ptwheels);

/*
 * Host only: the integer threshold row the library uploads for one
 * temperature (32 words).  Metropolis (sec. 2.2): words n = 0..2 hold
 * floor(2^32 exp(-beta (12 - 4n))) for n unsatisfied bonds; heat bath
 * (Eq. 4): words k = 0..6 hold floor(2^32 / (1 + exp(-2 beta (2k - 6))));
 * Potts models: words d = 0..12 hold floor(2^28 exp(-beta d)).  A threshold
 * equal to 2^32 ("always") is stored as 0xFFFFFFFF with bit n of word 15 set
 * (Ising).  SG_ISING_GEN (Eq. 2): word k + 16 phi holds the threshold of
 * class (k, phi) and words 13, 29 the limits of the classes whose move is
 * certain (their words are 0).  SG_E_INVALID for a bad model, algorithm,
 * beta or field; SG_E_UNSUPPORTED if the Eq. 2 thresholds are not monotone.
 */
int sg_threshold_row(int32_t model, int32_t algo, double beta, double field, uint32_t row[32]);

/* Host only: parallel-tempering factors of the temperature pair
 * (beta_i, beta_next), F[b] = floor(2^32 exp(-|beta_i - beta_next| 2^b)),
 * b = 0..23, and the sign of beta_i - beta_next (sec. 2.2 names parallel
 * tempering; the integer swap test is the library's reading). */
int sg_pt_factors(double beta_i, double beta_next, uint64_t F[24], int32_t *sign);

/*
 * Create a job in the caller's device arena and upload its state (blocks
 * until the upload, which is ordered on `stream`, has finished).
 *   betas         [K] inverse temperatures >= 0, by temperature index;
 *   J             [S][3][N] int8, J[d][i] couples i and i + e_d: +-1 (Ising,
 *                 +-J Potts); for SG_GPOTTS the bytes are read as uint8
 *                 permutations pi of (0, 1, 2, 3), the bond's term being
 *                 delta(s_i, pi(s_{i+e_d})) with pi(v) = (byte >> 2v) & 3;
 *                 for SG_ISING_GEN [S][5][N] int8: rows J_x, J_y, J_z (+-1),
 *                 x (0 = empty site, 1 = spin) and f (+-1); for SG_GPOTTS4
 *                 [S][4][L^4] permutation bytes as for SG_GPOTTS;
 *   spins         [C][N] int8 +-1 (Ising models) or uint8 0..3 (Potts models);
 *                 an empty site keeps its spin (and still consumes its number);
 *   wheels        [C][NW][61];      ptwheels [S*R][61];
 *   J, spins, wheels, ptwheels: NULL = generated from spec->seed as by
 *                 sg_generate (a job is then created from its seed alone);
 *   slot_of_temp  [S*R][K] or NULL (identity);
 *   sweeps_done   sweeps already performed by this state (0 for a new job;
 *                 used to resume from exported state).
 * SG_E_NOMEM if arena_bytes < sg_job_bytes(); SG_E_UNSUPPORTED for L or a
 * model that is not built; SG_E_INVALID for inconsistent inputs.
 */
int sg_job_create(sg_ctx *ctx, const sg_job_spec *spec, const double *betas, const int8_t *J,
                  const void *spins, const uint32_t *wheels, const uint32_t *ptwheels,
                  const int32_t *slot_of_temp, uint64_t sweeps_done, void *d_arena,
                  uint64_t arena_bytes, void *stream, sg_job **out);

/* Replace the K inverse temperatures: rebuilds the integer threshold tables
 * of sec. 2.2 / Eq. 4 on the host and uploads them. (sync) */
int sg_job_set_betas(sg_job *job, const double *betas, void *stream);

/* Lanes serving one Parisi-Rapuano wheel in the 3D Potts kernels: sec. 3.3
 * lets one wheel emit many numbers at once (its lags reach back at least 24
 * outputs), so S lanes may form its outputs k = k0 + S s + l together.  The
 * numbers, their order and every result are the same for every S; only the
 * launch shape changes (S NW lanes per copy).  Defaults: 8 at L = 16, 4 at
 * L = 8, 24, 32, 2 at L = 40, 48, 1 otherwise and for the other models.
 * Alternative: 4 at L = 16 (fewer instructions per update, half the lanes).
 * Any other value: SG_E_INVALID.  The job's own launch plan is rebuilt and
 * uploaded on `stream` (no sweep of the job may be in flight on another
 * stream); batches holding the job re-plan at their next run. (sync) */
int sg_job_set_wheel_lanes(sg_job *job, int32_t lanes, void *stream);
int sg_job_wheel_lanes(sg_job *job, int32_t *lanes);

/* Run n sweeps of every copy: checkerboard half-sweeps (sec. 3.1), each site
 * update drawing one Parisi-Rapuano number (sec. 3.3, Eq. 5) and accepting
 * by the integer rule of sec. 2.2 / Eq. 4; parallel-tempering steps (sec.
 * 2.2) after every multiple of pt_every sweeps, counted since the start of
 * the job.  Asynchronous. */
int sg_job_sweep(sg_job *job, uint64_t n_sweeps, void *stream);

/* sweep(beta, n): set the single inverse temperature of a K = 1 job to beta
 * (tables rebuilt only if it changed) and run n sweeps as sg_job_sweep.
 * SG_E_INVALID if the job has K > 1. */
int sg_job_sweep_beta(sg_job *job, double beta, uint64_t n_sweeps, void *stream);

/* Measurement (sec. 4.1 measures energies and the overlap q between replicas
 * at the same temperature): energy of every copy by chain and temperature
 * index, E[(s*R + r)*K + k] (may be NULL), and overlap of replicas 0 and 1
 * at every temperature, Q[s*K + k] (may be NULL; needs R >= 2): Ising
 * sum_i s^a_i s^b_i, Potts number of equal sites. (sync) */
int sg_job_measure(sg_job *job, int64_t *E, int64_t *Q, void *stream);

/* Energy of every slot (copy order), as left by the last sweep or measure
 * (sec. 4.1). (sync) */
int sg_job_energies(sg_job *job, int64_t *E_slot, void *stream);

/* SG_ISING_GEN (Eq. 2): field sum M = sum_i x_i f_i s_i of every copy by
 * chain and temperature index, M[(s*R + r)*K + k], recomputed from the
 * current spins; SG_E_STATE for other models. (sync) */
int sg_job_field_sums(sg_job *job, int64_t *M, void *stream);

/* Canonical export of the state (sec. 4.1 copies configurations to the host
 * periodically). (sync) */
int sg_job_get_spins(sg_job *job, void *spins_out /* [C][N] */, void *stream);
int sg_job_get_wheels(sg_job *job, uint32_t *wheels_out /* [C][NW][61] */,
                      uint32_t *ptwheels_out /* [S*R][61] or NULL */, void *stream);
int sg_job_get_perm(sg_job *job, int32_t *slot_of_temp_out /* [S*R][K] */, void *stream);
/* Accepted parallel-tempering swaps per (chain, pair), [S*R][K-1] (sec. 2.2).
 * (sync) */
int sg_job_get_pt_accepts(sg_job *job, uint64_t *out, void *stream);
/* Sweeps performed so far. */
int sg_job_sweeps_done(const sg_job *job, uint64_t *out);

/*
 * Checkpoint and restore (sec. 4.1: configurations go to the host
 * periodically; a long run resumes from them).  The checkpoint is an opaque
 * host blob of sg_job_checkpoint_bytes() bytes holding the specification,
 * the inverse temperatures, the sweep counter, every spin, sweep wheel and
 * parallel-tempering wheel, the temperature permutation, the swap counters,
 * the energies and a 64-bit digest of the couplings.  sg_job_restore loads
 * it into a job of the same specification and couplings (SG_E_STATE
 * otherwise; SG_E_INVALID for a blob that is not a checkpoint); the job then
 * continues bit for bit as the checkpointed one would. (sync)
 */
int sg_job_checkpoint_bytes(const sg_job *job, uint64_t *bytes);
int sg_job_checkpoint(sg_job *job, void *host_buf, uint64_t bytes, void *stream);
int sg_job_restore(sg_job *job, const void *host_buf, uint64_t bytes, void *stream);

/* Test hook: the next n (<= 4096) numbers (Eq. 5, sec. 3.3) of sweep wheel
 * `wheel` of copy `copy`, computed on the device; the job's state is not
 * advanced. (sync) */
int sg_job_debug_rng(sg_job *job, int32_t copy, int32_t wheel, uint32_t n, uint32_t *out,
                     void *stream);

int sg_job_destroy(sg_job *job);

/*
 * Batches: many jobs (mixed L, models, temperatures) advanced together by one
 * fused sweep launch per period, replayed from a captured hipGraph.  The
 * paper fills its update cells with two replicas per FPGA and runs many
 * samples on many FPGAs (sec. 3.2, sec. 4.2); here samples, replicas and
 * temperatures of many jobs share one launch.  Jobs can be added and removed
 * between runs (continuous batching); a job's results do not depend on the
 * batch it runs in.  A removed job's arena must stay valid until the periods
 * already enqueued on the caller's stream have finished.
 */
/* Create a batch holding the n jobs of `jobs` (n may be 0, jobs NULL). */
int sg_batch_create(sg_ctx *ctx, sg_job *const *jobs, int32_t n, sg_batch **out);
int sg_batch_add(sg_batch *b, sg_job *job);
int sg_batch_remove(sg_batch *b, sg_job *job);
/* Threads per workgroup of the fused launch (multiple of 64, <= 1024;
 * 0 = automatic); the Potts and Ising-like launches use min(threads, 512)
 * (768 for the Potts models at L = 40, 48); a copy needing more lanes than
 * that runs in a workgroup of its own size, and items much smaller than it
 * in workgroups of theirs.  Results do not depend on it. */
int sg_batch_set_block(sg_batch *b, int32_t threads);
/* Remaining sweep budget of a job in the batch: a run of n sweeps advances
 * the job by min(n, budget) and lowers the budget by that much
 * (UINT64_MAX = unlimited, the default).  For jobs without parallel tempering.
 * This lets jobs of different lengths share one launch and stop exactly. */
int sg_batch_set_budget(sg_batch *b, sg_job *job, uint64_t sweeps);
int sg_batch_get_budget(sg_batch *b, sg_job *job, uint64_t *sweeps);
/* Per-run cap of a job in the batch: every run of n sweeps advances the job
 * by min(n, cap, budget) (UINT64_MAX = no cap, the default); the cap is not
 * consumed.  Jobs whose sweeps cost different device time can so share one
 * launch for the same time each (the serving loop sets caps from its cost
 * estimate).  For jobs without parallel tempering. */
int sg_batch_set_period_cap(sg_batch *b, sg_job *job, uint64_t sweeps);
/* Advance every job of the batch by n sweeps (sec. 3.1 / 3.3 / 2.2 as
 * sg_job_sweep, parallel tempering included).  After membership changes the
 * call first waits for the work already enqueued on `stream`. */
int sg_batch_run(sg_batch *b, uint64_t n_sweeps, void *stream);
/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * periods as sg_batch_run, bit for bit, with the batch's launch tables (work
 * items, per-job sweep counters and caps, parallel-tempering work lists) in
 * a fixed device array of 2 MiB that each device holds until the process
 * ends; SG_E_NOMEM (nothing run) if the tables need more (about 18,000 work
 * items).  Calls no hipMalloc, hipFree or other allocating routine and
 * captures no graph: periods are enqueued directly on `stream` (the timing
 * mode does not apply).  Waits first for this batch's previous run.  Every
 * call on a device shares that device's array and leaves its tables in it:
 * calls of different batches on one device must not overlap in time (run
 * them on one stream, or one after another) -- overlapping calls race.
 */
int sg_batch_run_static(sg_batch *b, uint64_t n_sweeps, void *stream);
/* Threads per workgroup chosen for the current membership. */
int sg_batch_block(sg_batch *b, int32_t *threads);
/* Timing mode: periods are enqueued directly on the caller's stream (not
 * replayed from the graph) with HIP events around the fused sweep launch;
 * sg_batch_sweep_ms() returns that launch's duration in the last period,
 * waiting for it. (sync) */
int sg_batch_set_timing(sg_batch *b, int32_t enable);
int sg_batch_sweep_ms(sg_batch *b, float *ms);
int sg_batch_destroy(sg_batch *b);

#ifdef __cplusplus
}
#endif
#endif
