/*
 * chromh.h -- C-ABI of the chromatic Metropolis-Hastings region sweep on
 * AMD Instinct MI355X (gfx950).
 *
 * The library infers the set of seismic events that explains a set of
 * station traces (the inference problem of Section 3 of Song & Moore,
 * "Parallel Chromatic MCMC with Spatial Partitioning"), by MH over the event
 * set, run region by region in colour phases (Section 4, Algorithm 4) with
 * the partition offset redrawn between sweeps (Section 4.3.2).
 *
 * Conventions shared by every entry point:
 *   - Every function returns an int32_t status: CMH_OK (0) or a negative
 *     CMH_E* code; it never throws.  cmh_last_error() returns a message for
 *     the last failure on the calling thread.
 *   - Pointers named *_dev are device pointers (HIP device memory on the
 *     current device), *_host are host pointers.  The caller owns every
 *     buffer: traces, workspace, feed and log arrays must outlive the state.
 *     The library never allocates device memory; it owns only the small host
 *     handle freed by cmh_destroy.
 *   - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Sweep calls only enqueue work.  Calls that return data to the host
 *     synchronise that stream first.  Errors raised on the device (event
 *     capacity, NaN) are latched in a device word and reported by the next
 *     synchronising call; the state then answers CMH_ESTATE until destroyed.
 *   - Arguments are validated before any device work.
 *
 * Model (Section 3, in the 2-D attenuating form Section 4.1 names as the
 * natural case for a spatial partition):
 *   stations on an nsx x nsy grid, cell-centred with spacing ds; domain
 *   [0, nsx ds) x [0, nsy ds); events (x, y, t, m) with Poisson(lambda) count,
 *   uniform location and onset t in [0, n_samples), m - mag_min ~
 *   Exp(mag_rate); an event reaches a station at distance d < r_c with
 *   arrival a = t + d / velocity and adds a zero-mean Gaussian signal of
 *   standard deviation m exp(-d / atten) exp(-(n - a) / env_decay) on samples
 *   n in [ceil(a), ceil(a) + t_s); the trace is Gaussian with variance
 *   sigma^2 plus the variances of all arriving signals.
 *
 * Trace layout: [station][sample], station j = iy * nsx + ix, samples
 * contiguous; dtype CMH_F32 or CMH_F64.
 */
#ifndef CHROMH_H
#define CHROMH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CMH_OK      0
#define CMH_EINVAL (-1)   /* invalid argument */
#define CMH_EHIP   (-2)   /* a HIP runtime call failed */
#define CMH_ECAP   (-3)   /* a region's event capacity was exceeded */
#define CMH_ECOLOR (-4)   /* no colouring satisfies the independence check */
#define CMH_ENAN   (-5)   /* NaN/Inf met in a likelihood evaluation */
#define CMH_ESTATE (-6)   /* state poisoned by an earlier device error */
#define CMH_ERACE  (-7)   /* debug owner check: two regions of one colour shared a sample */

#define CMH_F32 0
#define CMH_F64 1

#define CMH_BIRTH 0
#define CMH_DEATH 1
#define CMH_LOC   2
#define CMH_TIME  3
#define CMH_MAG   4
#define CMH_ARR   5   /* arrival-time move (latent arrivals) */
#define CMH_JOINT 6   /* joint two-event move (latent arrivals) */

typedef struct {
    int32_t nsx, nsy;     /* station grid */
    double  ds;           /* station spacing */
    int64_t n_samples;    /* samples per trace */
    double  sigma;        /* noise standard deviation */
    double  atten;        /* amplitude attenuation length */
    double  velocity;     /* domain units per sample */
    double  env_decay;    /* amplitude envelope decay, samples */
    int32_t t_s;          /* signal duration, samples (1..128) */
    int32_t _pad0;
    double  r_c;          /* detection cutoff, 0 < r_c < ds */
    double  lambda;       /* Poisson mean number of events */
    double  mag_min;      /* magnitude lower bound */
    double  mag_rate;     /* rate of the exponential magnitude prior */
    /* Line model (line = 1): the 1-D world of Section 3 as printed.  nsx
     * stations (1..8, nsy = 1) at station_x on a line; events (x, t) with
     * y = 0, x uniform on [0, x_max); every station detects every event at
     * a = t + |x - station_x[j]| / velocity; the signal is Gaussian with the
     * constant variance m^2 on [ceil(a), ceil(a) + t_s) (m = mag_min for
     * events the sampler creates).  The partition is in onset time
     * (Section 4.1): grid_x regions, grid_y = 0.  ds, atten, env_decay, r_c
     * and mag_rate are not used; magnitude moves are rejected; learned
     * births, anchors and training pairs are not available. */
    int32_t line;
    /* Mean-template likelihood (template_mean = 1), the alternative reading
     * of Section 3's signal model: an event adds the deterministic waveform
     * A phi(n - a) (A = m exp(-d / atten), phi(tau) = exp(-tau / env_decay),
     * or the constant m on the line) to the mean of the trace, and the trace
     * is that mean plus Gaussian noise of variance sigma^2.  The state's
     * per-sample array then holds the residual trace - mean (cmh_read_variance
     * returns it), a move's log-likelihood change is sum g (r - g / 2) /
     * sigma^2 over its footprint, and the trace is not read by the sweeps.
     * Learned births, anchors and training pairs need the variance model. */
    int32_t template_mean;
    double  x_max;
    double  station_x[8];
    /* Latent arrival times (line model only; 0 = off), Section 3's arrival
     * density: every event carries offsets da[j] (cmh_event) and arrives at
     * station j at t + |x - station_x[j]| / velocity + da[j]; each offset is
     * Gaussian with standard deviation arrival_sd, truncated to
     * |da[j]| <= 4 arrival_sd so that the colouring stays exact (every
     * region's reach widens by that bound on both sides).  Births draw the
     * offsets from this prior, location and onset moves carry them along
     * (the arrivals move with the event), and the sampler gains the
     * arrival-time move and the joint move (cmh_sampler).  Runs the
     * block-64 or block-256 forms of the chromatic schedule. */
    double  arrival_sd;
} cmh_model;

#define CMH_BLOCK_SPEC 1024
#define CMH_BLOCK_PERSIST (2048 + 64)

typedef struct {
    int32_t grid_x, grid_y;     /* regions per axis of the unshifted grid */
    int32_t dynamic;            /* 1: offset redrawn every sweep */
    int32_t period;             /* colour period p, 0 = derive */
    int32_t moves_per_region;   /* k, MH moves per region per colour phase */
    int32_t region_capacity;    /* events per region, 1..64 */
    double  p_birth, p_death, p_loc, p_time, p_mag;   /* sum to 1 */
    double  step_xy, step_t, step_m;                  /* random-walk steps */
    int32_t prior_only;         /* 1: likelihood switched off */
    int32_t block;              /* sweep kernel form: 128, 256, 512 threads per region (one
                                   scout wave, the rest evaluate; for few regions per
                                   colour), or 64: one wave per region, four regions per
                                   workgroup (for many regions per colour), or
                                   CMH_BLOCK_SPEC + 128 / 256 / 512: 2, 4 or 8 waves per
                                   region, each taking one of the region's next moves from
                                   the same state; the moves stand in order up to the
                                   first that conflicts with an earlier standing
                                   acceptance (same event, overlapping samples) or up to
                                   an accepted birth or death (the chain is the
                                   sequential one; not with latent arrivals or the naive
                                   schedule), or CMH_BLOCK_PERSIST: the
                                   one-wave-per-region form as one persistent launch per
                                   sweep over every colour, each chain's (instance's)
                                   colours ordered by its own colour counter, different
                                   chains overlapping (dynamic partitions only, not with
                                   latent arrivals or the naive schedule; cmh_sweep_color
                                   then runs the whole sweep at colour 0); 0 = 256 */
    int32_t schedule;           /* 0: chromatic (Algorithm 4).  1: naive parallel MH
                                   (Algorithm 3, the paper's negative control): every region
                                   in one phase, each evaluating against the phase-start
                                   state plus its own changes; the variance is then
                                   recomputed from the merged events.  Naive needs
                                   n_stations x n_samples <= 2048 (a private copy per
                                   region in LDS) and runs the block-64 form. */
    int32_t debug;              /* bit 0: owner check.  Every sample a move reads or writes
                                   is tagged with (sweep, colour, region) in a workspace array
                                   of 8 bytes per sample per chain; meeting another region's
                                   tag of the same colour phase latches CMH_ERACE (the
                                   colouring of Section 4.1 failed to make the regions of one
                                   colour independent).  Chromatic schedule only.  Bit 1
                                   (with bit 0 and a period): take the period without the
                                   independence check, so that a test can force a breach
                                   for the owner check to catch.  Bit 2: the persistent
                                   form's colour-counter waits give up at once (an unmet
                                   wait latches CMH_ESTATE), so that a test can reach the
                                   wait's error path.  0 for production runs. */
    /* Latent arrivals only (0 otherwise).  p_arrival: the arrival-time move
     * of Section 3 (one event, one station drawn uniformly, its offset plus
     * step_arrival times a standard normal; the offset prior enters the
     * ratio).  p_joint: the joint move of Section 3: two events of a region
     * (of equal magnitude) exchange their arrival times at the stations
     * from a uniformly drawn split s in 1..n-1 onwards (station index
     * order), each then moves to its least-squares location fit to the new
     * arrivals plus Gaussian steps (step_xy, step_t), with offsets that keep
     * its arrivals where they are; the signal is unchanged, so only the
     * offset prior and the proposal densities (around the fits of the new
     * and of the old arrivals) enter the ratio.  All seven probabilities sum
     * to 1. */
    double  p_arrival, p_joint, step_arrival;
    int32_t refresh_every;      /* > 0: after every sweep s with (s + 1) % refresh_every == 0
                                   the event variance of every chain is recomputed exactly
                                   from its events (removing the rounding that in-place
                                   updates accumulate); 0: never */
    int32_t _pad0;
} cmh_sampler;

typedef struct {
    double   x, y, t, m;
    uint64_t id;       /* (sweep << 32) | (region << 12) | move, or caller's */
    int32_t  region;   /* linear region index k * (grid_x + 1) + i */
    int32_t  _pad;
    double   da[8];    /* latent arrivals: offset per station (0 otherwise) */
} cmh_event;

typedef struct cmh_state cmh_state;

const char *cmh_last_error(void);

/* Partition and colouring (Sections 4.1 and 4.3).  Region i along x covers
 * [off_x + (i - 1) w, off_x + i w) clipped to the domain, w = domain / grid,
 * i in 0..grid_x; the offset is in [0, w).  Colour of region (i, k) is
 * (i mod p) + p (k mod p).  Static partitions use the smallest p whose
 * colouring passes the exact check (no station within r_c of two regions of
 * one colour); dynamic ones use p = ceil(2 r_c / w) + 1, which holds for
 * every offset.  Line model: regions of onset time, w = n_samples / grid_x,
 * off_x the time offset, off_y = 0, grid_y = 0; region i can touch samples
 * [ceil(t0 + dmin / v), ceil(t1 + dmax / v) + t_s) of a station at distances
 * dmin..dmax from the line (each end widened by the jitter bound e =
 * 4 arrival_sd with latent arrivals), and no two regions of one colour may
 * share a sample; dynamic p = ceil((tau_max + t_s + 2 e) / w) + 1; colour
 * i mod p.
 * color_of_region: caller array of (grid_x+1)*(grid_y+1) int32, may be NULL.
 * Pure host function.  CMH_ECOLOR if no p works. */
int32_t cmh_partition_and_color(const cmh_model *model, int32_t grid_x, int32_t grid_y,
                                double off_x, double off_y, int32_t dynamic,
                                int32_t *n_reg_x, int32_t *n_reg_y, int32_t *period,
                                int32_t *n_colors, int32_t *color_of_region);

/* Workspace bytes for n_chains chains: the per-chain event-variance
 * accumulator (n_stations x n_samples doubles), two event tables of
 * region_capacity slots per region (with latent arrivals also eight offsets
 * per slot), offsets, the sweep's per-move draw records (with latent
 * arrivals a second array for draws 8..15), statistics and flags. */
int32_t cmh_state_bytes(const cmh_model *model, const cmh_sampler *sampler,
                        int32_t n_chains, size_t *bytes);

/* Initialise n_chains chains on one trace (Algorithm 4's input: an empty
 * world, zero event variance).  trace_dev: [station][sample] of trace_dtype,
 * shared by all chains, read only.  Chain c draws from Philox4x32-10 under
 * key (seed, c).  Enqueues the workspace set-up on hip_stream. */
int32_t cmh_init_state(const cmh_model *model, const cmh_sampler *sampler,
                       const void *trace_dev, int32_t trace_dtype, int32_t n_chains,
                       uint32_t seed, void *workspace_dev, size_t workspace_bytes,
                       void *hip_stream, cmh_state **out);

/* One colour phase of sweep `sweep` on every chain (Algorithm 4's inner
 * parallel loop): every region of colour `color` runs k MH moves at once,
 * one workgroup per region.  color == 0 first lays out the sweep's partition
 * (a fresh offset when dynamic) and moves every event into the list of its
 * region.  Phases must be called in colour order. */
int32_t cmh_sweep_color(cmh_state *st, int64_t sweep, int32_t color, void *hip_stream);

/* Sweeps first_sweep .. first_sweep + n_sweeps - 1, every colour in order
 * (Algorithm 4's outer loop with Section 4.3.2's offset draw).  Replayed
 * from captured HIP graphs when no feed or log is attached. */
int32_t cmh_run_sweeps(cmh_state *st, int64_t first_sweep, int64_t n_sweeps, void *hip_stream);

/* Current events of one chain, in region order and by id within a region.
 * Synchronises.  If more than cap events exist, *n_out is set and
 * CMH_EINVAL returned. */
int32_t cmh_read_events(cmh_state *st, int32_t chain, cmh_event *out_host, int64_t cap,
                        int64_t *n_out);

/* Replace one chain's (one instance's, in a batch) events (host array, ids
 * kept) and recompute its event variance exactly.  Events must lie in the
 * model's support; a region over capacity is CMH_ECAP, with the state
 * unchanged.  Synchronises. */
int32_t cmh_write_events(cmh_state *st, int32_t chain, const cmh_event *ev_host, int64_t n);

/* Checkpoint and resume.  cmh_save copies every chain's (or batch
 * instance's) current event table (with arrival offsets under latent
 * arrivals), its event variance as the sweeps left it (not recomputed, so a
 * resumed chain continues bit for bit), its move counters and the layout
 * parity into the caller's host buffer of cmh_checkpoint_bytes bytes (about
 * n_stations x n_samples x 8 bytes per chain).  cmh_load writes such a
 * buffer back into a state made with the same model, sampler settings,
 * chain count, seed and trace (CMH_EINVAL on any other shape, before
 * anything is written).  The random draws are keyed by (seed, chain, sweep,
 * region, move), so the caller resumes with the next sweep index: N sweeps,
 * save, load into a fresh state, N more sweeps equal 2N sweeps.  Feeds,
 * logs, recordings and learned tables are not part of the checkpoint (attach
 * them again).  Both synchronise. */
int32_t cmh_checkpoint_bytes(cmh_state *st, size_t *bytes);
int32_t cmh_save(cmh_state *st, void *host_buf, size_t bytes);
int32_t cmh_load(cmh_state *st, const void *host_buf, size_t bytes);

/* Replay mode.  feed_dev: doubles [n_sweeps][regions][k][8] holding, per
 * move, the draws the sampler would otherwise take from Philox: [0] uniform
 * for the move type, [1] uniform a (index or birth x), [2] uniform b (birth
 * y), [3] uniform c (birth onset), [4] Exp(1) (birth magnitude), [5], [6]
 * standard normals, [7] log of the acceptance uniform.  With learned births
 * (cmh_set_learned) the records are [16]: the same 8, then [8] mixture
 * uniform, [9] anchor uniform, [10] component uniform, [11..13] standard
 * normals truncated to [-4, 4], [14], [15] unused.  With latent arrivals
 * they are [16] too: the same 8, then [8..15] standard normals truncated to
 * [-4, 4] (cmh_move_draws_arrivals).  width (8 or 16) states the record
 * size; a sweep whose mode needs the other size fails with CMH_EINVAL before
 * any launch.  Chain 0 only.  NULL detaches. */
int32_t cmh_set_feed(cmh_state *st, const double *feed_dev, int64_t first_sweep,
                     int64_t n_sweeps, int32_t width);

/* Sample recording (the record of Algorithm 4's output states).  After the
 * last colour phase of every sweep s in [first_sweep, first_sweep +
 * n_sweeps), each chain c's state is written to rec_dev[s - first_sweep][c]
 * [1 + 4 max_events] (binary64): [0] its event count, then (x, y, t, m) of
 * its first max_events events (regions in index order, each region's events
 * in id order); events beyond max_events are counted but not written.  Runs
 * inside captured sweep graphs (the sweep index is read on the device).
 * NULL detaches.  Drops captured graphs. */
int32_t cmh_set_record(cmh_state *st, double *rec_dev, int64_t first_sweep, int64_t n_sweeps,
                       int32_t max_events);

/* Move log.  log_dev: doubles [n_sweeps][regions][k][4] = move type,
 * status (0 rejected before the likelihood, 1 rejected, 2 accepted),
 * log-likelihood change, log acceptance ratio.  Chain 0 only.  NULL
 * detaches. */
int32_t cmh_set_log(cmh_state *st, double *log_dev, int64_t first_sweep, int64_t n_sweeps);

/* Exact recomputation of every chain's event variance from its events and,
 * when out_host is not NULL, each chain's signal log-likelihood
 * log P(s | e) (Section 3) into out_host[n_chains].  write_variance = 0 only
 * evaluates the log-likelihood.  Synchronises when out_host is given. */
int32_t cmh_refresh(cmh_state *st, int32_t write_variance, double *out_host, void *hip_stream);

/* Copy one chain's event variance for stations [station0, station0 + nsta)
 * into out_host (nsta x n_samples doubles).  Synchronises. */
int32_t cmh_read_variance(cmh_state *st, int32_t chain, int64_t station0, int64_t nsta,
                          double *out_host);

/* Per-chain move statistics since init, out_host[23]: [3 t + 0], [3 t + 1],
 * [3 t + 2] = attempted, evaluated (valid proposals) and accepted moves of
 * type t (CMH_BIRTH .. CMH_MAG); [15] footprint samples evaluated; [16]
 * footprint samples rewritten on acceptance; [17 + 3 (t - 5) + 0..2] the
 * same three counts for CMH_ARR and CMH_JOINT.  Synchronises. */
int32_t cmh_read_stats(cmh_state *st, int32_t chain, uint64_t *out_host);

/* The sweep kernel form in use (the sampler's block code, after tuning). */
int32_t cmh_get_block(cmh_state *st, int32_t *block);

/* Times each sweep-kernel form on n_trial sweeps starting at
 * first_sweep, keeps the fastest, then restores the chains' events and
 * recomputes their event variance.  Results are cached per problem shape.
 * Synchronises. */
int32_t cmh_autotune(cmh_state *st, int64_t first_sweep, int32_t n_trial, void *hip_stream);

/* Tuning while sampling, for single chains and batches alike: each
 * sweep-kernel form in turn runs one sweep (which builds its graphs) and then
 * n_trial timed sweeps of the chains themselves, starting at first_sweep;
 * the fastest form is kept.  Every form takes the chains through the same
 * states, so these are ordinary sweeps of the run (recorded, logged and fed
 * like any other) and nothing is restored; *next_sweep receives the index
 * of the first sweep not yet run.  Nothing is cached.  Synchronises.  On an
 * error the form in use before the call is kept, and the chains may have
 * run part of the trial sweeps. */
int32_t cmh_tune_running(cmh_state *st, int64_t first_sweep, int32_t n_trial, void *hip_stream,
                         int64_t *next_sweep);

/* Log-posterior of every chain (instance, in a batch) as its current
 * events stand (Section 3's joint density of events and signals, as a set
 * density, up to the constant of the signal model): out_host[3 c] = the
 * signals' log-likelihood ln p(s | X), out_host[3 c + 1] = the events' log
 * prior (-lambda + sum over events of ln lambda, the uniform location and
 * onset densities, the magnitude's exponential density, and with latent
 * arrivals each offset's truncated-normal density), out_host[3 c + 2] their
 * sum.  The variance is recomputed exactly from the events on the way
 * (written back to the state when write_variance is set).  Synchronises. */
int32_t cmh_log_posterior(cmh_state *st, int32_t write_variance, double *out_host,
                          void *hip_stream);

/* Log-probability records taken by the scheduled refresh (refresh_every >
 * 0): for each sweep s in first_sweep .. first_sweep + n_sweeps - 1 at which
 * the refresh runs, rec_dev[((s - first_sweep) n_chains + c) 2 + 0 / 1]
 * receive chain c's log-likelihood / log prior after the sweep (rows of
 * other sweeps are not written).  rec_dev: caller-owned device memory of
 * n_sweeps x n_chains x 2 doubles.  NULL switches recording off. */
int32_t cmh_set_logprob(cmh_state *st, double *rec_dev, int64_t first_sweep, int64_t n_sweeps);

/* Sweep-kernel time stamps (measurement), read live from the sweeps as they
 * run, graph replays included.  stamps_dev: caller-owned device memory of
 * n_sweeps x n_colors x 2 uint64, which the caller fills with (UINT64_MAX,
 * 0) pairs before the stamped sweeps run.  For sweep first_sweep + s, the
 * colour-c kernel folds the device's steady clock (cmh_stamp_rate ticks per
 * second) at the start of each workgroup into element 2 (s n_colors + c)
 * (minimum) and at the end into element 2 (s n_colors + c) + 1 (maximum):
 * end - start is the kernel's span from its first workgroup's start to its
 * last workgroup's end.  NULL switches stamping off.  Drops the captured
 * sweep graphs (they are rebuilt on the next cmh_run_sweeps). */
int32_t cmh_set_stamps(cmh_state *st, uint64_t *stamps_dev, int64_t first_sweep,
                       int64_t n_sweeps);
int32_t cmh_stamp_rate(int32_t device, int64_t *hz);

/* Runs sweeps first_sweep .. first_sweep + n_sweeps - 1 like cmh_run_sweeps
 * but launched one kernel at a time, with HIP events recorded on hip_stream
 * around each; ms_out[c] receives the summed milliseconds of colour c's
 * phases and ms_out[n_colors] those of the sweeps' starts (re-layout and the
 * sweep's draw records).  Synchronises.
 * Used for measurement. */
int32_t cmh_time_phases(cmh_state *st, int64_t first_sweep, int64_t n_sweeps, void *hip_stream,
                        float *ms_out);

/* Learned birth proposal (the independence proposal of Section 3's MH
 * ratio, its density entering the birth and death ratios).  A birth in a
 * region R that holds at least one station draws, with probability
 * p_learned, from q_R: an anchor a (station s in R, window i) with
 * probability w_a / W_R, W_R the total weight of R's anchors, then component
 * k of the anchor's mixture with probability pi_k, then (x, y, t) = mean +
 * sd * (independent standard normals truncated to [-4, 4]), magnitude from
 * the prior; otherwise it draws from the prior on R.  The birth and death
 * ratios carry log(b / p_R) = log((1 - p_learned) + p_learned q_R(x, y, t)
 * area(R) n_samples) at the born or dying event; the posterior is unchanged.
 *   table_dev: [n_stations * n_tau][8][8] binary64, anchor a = station *
 *     n_tau + window, per component (mean x, y, t, sd x, y, t, log pi_k,
 *     pi_1 + ... + pi_k), as cmh_mixture_table writes it;
 *   weights_dev: [n_stations * n_tau] positive anchor weights;
 *   work_dev: cmh_learned_bytes(st, n_tau) bytes for the library's derived
 *     arrays (weight running sums, component normalisers, the table's time
 *     reach, per-sweep birth proposals).
 * All three are caller-owned and must outlive their use.  p_learned in
 * [0, 1).  table_dev NULL returns to plain births.  Regions may hold at most
 * 16 stations (a larger one raises CMH_ESTATE at the next check).  Drops
 * captured sweep graphs; enqueues the preparation on hip_stream. */
int32_t cmh_learned_bytes(cmh_state *st, int32_t n_tau, size_t *bytes);
int32_t cmh_set_learned(cmh_state *st, const double *table_dev, const double *weights_dev,
                        int32_t n_tau, double p_learned, void *work_dev, size_t work_bytes,
                        void *hip_stream);

/* The same for one instance of a batch (cmh_batch_init): its own table over
 * its own stations and windows, its own weights and workspace
 * (cmh_batch_learned_bytes bytes), its own p_learned; instances without a
 * table keep plain births.  Instance q with a table follows the same chain
 * as a one-chain state of its own with that table.  Synchronises, drops
 * captured sweep graphs. */
int32_t cmh_batch_learned_bytes(cmh_state *st, int32_t instance, int32_t n_tau, size_t *bytes);
int32_t cmh_batch_set_learned(cmh_state *st, int32_t instance, const double *table_dev,
                              const double *weights_dev, int32_t n_tau, double p_learned,
                              void *work_dev, size_t work_bytes, void *hip_stream);

/* A batch of independent instances (each a model, sampler settings, trace
 * and Philox seed; chain key 0) sampled together: every colour phase is one
 * launch over the regions of that colour of every instance, so instances of
 * uneven size share the device.  All instances share k, dynamic, block and
 * the trace dtype; an instance with fewer colours simply has no regions in
 * the later phases.  The returned state works with cmh_run_sweeps,
 * cmh_sweep_color, cmh_read_events / cmh_read_stats (chain = instance
 * index), cmh_set_record (chain = instance) and cmh_destroy; the other calls
 * return CMH_EINVAL for it.  Every instance starts empty (no events, E = 0),
 * and instance q of a batch follows the same chain as a one-chain state of
 * its own with seed seeds[q].  traces_dev[q]: [nsta_q][n_samples_q]. */
int32_t cmh_batch_bytes(int32_t n_instances, const cmh_model *models,
                        const cmh_sampler *samplers, size_t *bytes);
int32_t cmh_batch_init(int32_t n_instances, const cmh_model *models,
                       const cmh_sampler *samplers, const void *const *traces_dev,
                       int32_t trace_dtype, const uint32_t *seeds, void *workspace_dev,
                       size_t workspace_bytes, void *hip_stream, cmh_state **out);

int32_t cmh_destroy(cmh_state *st);

/* Forward simulator (synthetic worlds sampled from the model, Section 5):
 * trace[j][n] = sqrt(sigma^2 + E_j[n]) z_jn with E from the given events and
 * z standard normal from Philox4x32-10 under key (seed, 0x80000001),
 * counter (n / 2, j, 0, 0), Box-Muller (even n cosine, odd n sine).
 * truth_host: n_events events (host).  workspace_dev must hold
 * cmh_simulate_bytes() bytes.  Enqueues on hip_stream and synchronises
 * before returning (the staged events live in the workspace). */
int32_t cmh_simulate_bytes(const cmh_model *model, const cmh_event *truth_host,
                           int64_t n_events, size_t *bytes);
int32_t cmh_simulate(const cmh_model *model, const cmh_event *truth_host, int64_t n_events,
                     uint32_t seed, void *trace_dev, int32_t trace_dtype,
                     void *workspace_dev, size_t workspace_bytes, void *hip_stream);

/* The same simulator for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * no workspace argument; the truth table is staged in a library-owned device
 * array of 8 MiB per device (held until the process ends), so a truth
 * layout needing more (cmh_simulate_bytes) is CMH_EINVAL.  The caller still
 * owns trace_dev.  Every call on one device uses the same array: calls that
 * overlap on one device (other host threads) race.  Synchronises. */
int32_t cmh_simulate_noalloc(const cmh_model *model, const cmh_event *truth_host,
                             int64_t n_events, uint32_t seed, void *trace_dev,
                             int32_t trace_dtype, void *hip_stream);

/* Draw records [count][width] (width 8, or 16 for learned births) that
 * chain `chain` takes for moves j0 .. j0+count-1 of region `region` in sweep
 * `sweep` (the same layout as the feed), computed on the device into
 * out_dev.  Enqueues on hip_stream. */
int32_t cmh_move_draws(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                       uint32_t j0, int32_t count, int32_t width, double *out_dev,
                       void *hip_stream);

/* The same for latent arrival times: records [count][16], the 8 above, then
 * eight standard normals truncated to [-4, 4] (a birth's offsets in station
 * order; the joint move's second event takes the first two): Box-Muller
 * pairs from counter blocks 4, 5, ... (cosine, then sine), the first eight
 * of absolute value at most 4; after blocks 4 .. 19 missing ones are 0.
 * Enqueues on hip_stream. */
int32_t cmh_move_draws_arrivals(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                                uint32_t j0, int32_t count, double *out_dev, void *hip_stream);

/* ------------------------------------------------------------------------
 * Learned birth proposal: a mixture-density network (MDN).
 *
 * Input: 576 BF16 features = the 3x3 block of stations around a centre
 * station (row-major) x 64 log-envelope values e[n] = ln(sigma^2 +
 * mean(s[n..n+3]^2)) - ln(sigma^2) from a window start (rounded to binary32,
 * then BF16).  Layers 576 -> 256 -> 256 -> 256 (GELU, erf form) -> 64 (56
 * live): 8 components x (logit, mean x, y, t, log sd x, y, t) over the
 * event's offset from the centre station in units of ds and from the window
 * start in units of 32 samples; log sds clamped to sd_xy in [0.025, 1.5],
 * sd_t in [1/64, 1].  BF16 operands on MFMA, FP32 accumulation.
 *
 * Parameter blob (caller-owned device memory, cmh_mdn_param_bytes): FP32
 * master weights and biases of the four layers (weights [out][in]) in order
 * W1 b1 W2 b2 W3 b3 W4 b4 (n_params floats), the Adam moments, then BF16
 * copies of the weights and transposed BF16 copies of W2, W3 and W4 (for
 * the backward pass).  Work buffers hold a row batch's activations.
 * ---------------------------------------------------------------------- */
#define CMH_MDN_IN 576
#define CMH_MDN_OUT 64

int32_t cmh_mdn_sizes(int64_t *n_params, int64_t *n_weights_bf16);
int32_t cmh_mdn_param_bytes(size_t *bytes);

/* Glorot-uniform weights from Philox4x32-10 under key (seed, 0x80000004),
 * counter (parameter index, 0, 0, 0); zero biases and Adam moments. */
int32_t cmh_mdn_init(void *params_dev, uint32_t seed, void *hip_stream);

/* Replace / read the FP32 master parameters (host arrays of n_params floats);
 * setting zeroes the Adam moments and refreshes the BF16 copies.
 * Synchronises. */
int32_t cmh_mdn_set_params(void *params_dev, const float *host, void *hip_stream);
int32_t cmh_mdn_get_params(const void *params_dev, float *host);

int32_t cmh_mdn_work_bytes(int32_t rows, size_t *bytes);

/* Head outputs out_dev[rows][64] (FP32) for BF16 features x_dev[rows][576].
 * x_dev and work_dev must be 16-byte aligned (CMH_EINVAL otherwise), here
 * and in cmh_mdn_gradients / cmh_mdn_train_step. */
int32_t cmh_mdn_forward(const void *params_dev, const void *x_dev, int32_t rows, float *out_dev,
                        void *work_dev, size_t work_bytes, void *hip_stream);

/* The same head outputs from one fused kernel for inference (anchor tables):
 * no work buffer, the hidden activations never leave LDS, only
 * out_dev[rows][64] (FP32) is written.  Hidden activations are rounded to
 * BF16 exactly as cmh_mdn_forward stores them.  x_dev 16-byte aligned;
 * rows in 1..2^31 - 1. */
int32_t cmh_mdn_infer(const void *params_dev, const void *x_dev, int32_t rows, float *out_dev,
                      void *hip_stream);

/* Mean mixture negative log-likelihood of targets z_dev[rows][3] and its
 * gradient w.r.t. every FP32 parameter (grad_dev[n_params]); per-row losses
 * into loss_dev[rows] when not NULL.  Mixture components are untruncated
 * Gaussians in the training loss. */
int32_t cmh_mdn_gradients(const void *params_dev, const void *x_dev, const float *z_dev,
                          int32_t rows, float *grad_dev, float *loss_dev, void *work_dev,
                          size_t work_bytes, void *hip_stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected at `step`, from
 * 1) on the gradients of cmh_mdn_gradients. */
int32_t cmh_mdn_train_step(void *params_dev, const void *x_dev, const float *z_dev, int32_t rows,
                           int32_t step, float lr, float *loss_dev, void *work_dev,
                           size_t work_bytes, void *hip_stream);

/* Training pairs from the forward simulator (synthetic local worlds, as the
 * paper's evaluation samples worlds from the model): pair p is a 3x3 block of
 * stations around a centre at the origin.  An edge class drawn from counter
 * c = 8 keeps all nine stations with probability 1/2, else (1/16 each) drops
 * the block's column and/or row beyond a domain edge that lies half a
 * spacing from the centre on that side.  A target event is uniform within
 * one spacing of the centre inside the domain with onset uniform in [-16,
 * 64) samples of the window; 3 background events are uniform within 1.5 ds +
 * r_c of the centre inside the domain, onsets in [-(t_s + 8), 64 + 8);
 * magnitudes from the prior; traces over the window's first 67 samples.
 * Draws: Philox under key (seed, 0x80000003): counter (p mod 2^32, p div
 * 2^32, 0, c) for the events (c = 0: target x, y; 1: target t, m; 2 + b and
 * 5 + b: background b's x, y and t, m), counter (p mod 2^32, p div 2^32, 1 +
 * station, n / 2) for the noise (Box-Muller, even n cosine, odd n sine).
 * Writes x_dev[count][576] BF16 (0 for a dropped station) and the target
 * offsets z_dev[count][3] = (x / ds, y / ds, t / 32). */
int32_t cmh_mdn_pairs(const cmh_model *model, uint32_t seed, int64_t first_pair, int32_t count,
                      void *x_dev, float *z_dev, void *hip_stream);

/* Training (§3's model as the simulator of the pairs; the network and loss
 * of cmh_mdn_gradients): `steps` Adam steps in one call, step s (0-based)
 * drawing rows pairs first_pair + s rows .. first_pair + (s + 1) rows - 1
 * into x_dev[rows][576] / z_dev[rows][3] (as cmh_mdn_pairs) and taking one
 * step of cmh_mdn_train_step at Adam step step0 + s.  Everything is enqueued
 * on hip_stream; the caller's buffers: x_dev (16-byte aligned), z_dev, the
 * work buffer of cmh_mdn_work_bytes(rows), and loss_dev[rows] (optional)
 * which receives the last step's per-pair losses.  Errors: CMH_EINVAL for a
 * line or mean-template model, rows outside 1..2^20, steps < 1, step0 < 1,
 * negative first_pair, NULL or misaligned buffers, a short work buffer. */
int32_t cmh_mdn_train(void *params_dev, const cmh_model *model, uint32_t seed, int64_t first_pair,
                      int32_t steps, int32_t rows, int32_t step0, float lr, void *x_dev,
                      float *z_dev, float *loss_dev, void *work_dev, size_t work_bytes,
                      void *hip_stream);

/* Anchors of an instance: every station c (row-major) times window starts
 * tau = 32 i (tau + 67 <= n_samples); anchor index = c * n_tau + i.
 * CMH_EINVAL below 67 samples. */
int32_t cmh_anchor_count(const cmh_model *model, int32_t *n_anchors, int32_t *n_tau);

/* Anchors first .. first + count - 1: their 576 BF16 features (x_dev[count]
 * [576]: the log envelopes of the 3x3 block of stations around the anchor's
 * station over the window's 64 samples, 0 for block stations beyond the
 * grid) and weights w_dev[count] = 1e-3 + mean over the features of
 * max(0, f - 1), which rank windows by how far their envelopes rise above
 * the noise.  The trace is device memory [nsta][n_samples]. */
int32_t cmh_anchor_features(const cmh_model *model, const void *trace_dev, int32_t trace_dtype,
                            int64_t first, int32_t count, void *x_dev, double *w_dev,
                            void *hip_stream);

/* Mixture table of anchors first .. first + rows - 1 from the network's head
 * outputs head_dev[rows][64] (cmh_mdn_forward): table_dev[rows][8][8] in
 * binary64, per component (mean x, mean y, mean t, sd x, sd y, sd t, log
 * weight, cumulative weight), absolute units.  Means are clamped to within
 * 2 spacings of the anchor's station and to [tau - 32, tau + 96]; sds to
 * [0.025, 1.5] spacings and [0.5, 32] samples. */
int32_t cmh_mixture_table(const cmh_model *model, const float *head_dev, int64_t first,
                          int32_t rows, double *table_dev, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
