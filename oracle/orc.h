/*
 * orc.h -- the plain FP64 CPU oracle of the chromatic Metropolis-Hastings
 * sampler (Song & Moore, "Parallel Chromatic MCMC with Spatial Partitioning").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * GPU library; the only thing the two sides have in common is the published
 * definition of the Philox4x32-10 counter-based generator, which each side
 * implements on its own.
 *
 * Everything is IEEE double precision, single-threaded, compiled with
 * -ffp-contract=off so that every integer decided by floating point (region
 * of an event, detection test, first sample of an arrival window) is
 * reproducible bit for bit.
 *
 * Model (Section 3, "Generative Model of Seismic Signals"), in the 2-D,
 * attenuating form that Section 4.1 names as the natural case for a spatial
 * partition:
 *   - stations on an nsx x nsy grid, cell-centred, spacing ds;
 *     domain D = [0, nsx*ds) x [0, nsy*ds);
 *   - events e = (x, y, t, m): uniform location, uniform onset time t in
 *     [0, N) samples, magnitude m with m - mmin ~ Exp(mrate); their number
 *     is Poisson with mean lambda (the event prior of Section 3);
 *   - distance d to a station; detected only if d < rc; arrival
 *     a = t + d / vel (the arrival model of Section 3 with zero jitter);
 *   - the event's signal at a detecting station is zero-mean Gaussian with
 *     standard deviation A * phi(n - a) on n in [ceil(a), ceil(a) + ts),
 *     A = m * exp(-d / atten), phi(tau) = exp(-tau / decay);
 *   - signal likelihood: zero-mean diagonal Gaussian whose variance at each
 *     sample is the noise variance sigma^2 plus the variances of all
 *     arriving signals (Section 3, the paragraph after the joint density).
 *
 * Line model (line = 1): the world of Section 3 as the paper states it, with
 * the time partition of Section 4.1:
 *   - stations on a line at sta_x[0 .. nsx) (nsy = 1, station y = 0);
 *     events e = (x, t) with x uniform on [0, xmax), y = 0, and a fixed
 *     amplitude: the magnitude field holds mmin for every event;
 *   - every station detects every event; d = |x - sta_x[j]|, a = t + d / vel;
 *   - the signal is iid Gaussian of constant variance mmin^2 on
 *     [ceil(a), ceil(a) + ts): a boxcar, no attenuation, no decay;
 *   - regions are intervals of onset time: region i holds onsets in
 *     [off + (i-1) w, off + i w) clipped to [0, N), w = N / gx; the
 *     colour of region i is i mod p.
 *   - latent arrival times (arr_sd > 0), Section 3's arrival density: the
 *     arrival at station j is a_j = t + d_j / vel + da[j], the offset da[j]
 *     Gaussian with standard deviation arr_sd, truncated to
 *     |da[j]| <= ORC_ARR_TRUNC arr_sd so that the colouring stays exact (the
 *     reach of a region widens by that bound on both sides).  The event
 *     stores the offsets; moves of Section 3 act on them: births draw them
 *     from the prior, the arrival-time move steps one station's arrival,
 *     the location and onset moves carry the arrivals along with the event,
 *     and the joint move exchanges two events' arrivals at the stations
 *     from a split onwards and refits both locations.
 *
 * Mean-template likelihood (tmpl = 1), the alternative reading of the
 * signal model: an event adds the deterministic waveform A phi(n - a) (not
 * a variance) on [ceil(a), ceil(a) + ts), and the trace is the sum of the
 * waveforms plus Gaussian noise of variance sigma^2.  The per-sample
 * quantity the sampler tracks is then the sum of waveforms (the mean), and
 * a move changes the log-likelihood by sum g (r - g / 2) / sigma^2 over its
 * footprint, r the residual and g the change of the mean.
 */
#ifndef ORC_H
#define ORC_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nsx, nsy;   /* station grid */
    double  ds;         /* station spacing */
    int64_t N;          /* samples per trace */
    double  sigma;      /* background noise standard deviation */
    double  atten;      /* attenuation length of the amplitude */
    double  vel;        /* wave speed, domain units per sample */
    double  decay;      /* decay of the amplitude envelope, samples */
    int32_t ts;         /* signal duration, samples */
    int32_t _pad0;
    double  rc;         /* detection cutoff distance (strict d < rc) */
    double  lambda;     /* Poisson mean number of events in the domain */
    double  mmin;       /* magnitude lower bound */
    double  mrate;      /* rate of the exponential magnitude prior */
    int32_t line;       /* 1: the line model (see above) */
    int32_t tmpl;       /* 1: mean-template likelihood (see above) */
    double  xmax;       /* line model: locations uniform on [0, xmax) */
    double  sta_x[8];   /* line model: station positions */
    double  arr_sd;     /* line model: arrival-time jitter sd (0: a = t + d / vel) */
} orc_model;

/* The arrival-time jitter is truncated at this many standard deviations. */
#define ORC_ARR_TRUNC 4.0

enum { ORC_BIRTH = 0, ORC_DEATH = 1, ORC_LOC = 2, ORC_TIME = 3, ORC_MAG = 4, ORC_ARR = 5,
       ORC_JOINT = 6 };
enum { ORC_SCHED_CHROMATIC = 0, ORC_SCHED_NAIVE = 1 };

typedef struct {
    int32_t gx, gy;       /* regions per axis of the unshifted grid */
    int32_t dynamic;      /* 0 static partition, 1 offset redrawn every sweep */
    int32_t period;       /* colour period p (0: derive it) */
    int32_t k;            /* moves per region per colour phase */
    int32_t cap;          /* per-region event capacity */
    double  pb, pd, ploc, pt, pm;  /* move-type probabilities */
    double  sxy, st, sm;  /* random-walk step sizes */
    int32_t prior_only;   /* 1: likelihood switched off */
    int32_t schedule;     /* ORC_SCHED_* */
    /* lattice mode (tests only): events live on a finite site set */
    int32_t lattice;
    int32_t kx, ky, kt, km;   /* sites per axis */
    int32_t _pad1;
    double  hm;               /* magnitude site spacing */
    /* latent arrivals (line model with arr_sd > 0): probabilities of the
     * arrival-time and joint moves (added to the five above, all seven sum
     * to 1) and the arrival step */
    double  pa, pj, sa;
} orc_sampler;

typedef struct {
    double   x, y, t, m;
    uint64_t id;
    int32_t  region;
    int32_t  _pad;
    double   da[8];    /* latent arrival offsets per station (line model) */
} orc_event;

/* ---- Philox4x32-10 and the conversions built on it ------------------- */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t w0, uint32_t w1);
void   orc_move_draws(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                      uint32_t j, double out[8]);
void   orc_offset(uint32_t seed, uint32_t chain, uint32_t sweep, double wx, double wy,
                  double *dx, double *dy);

/* ---- geometry --------------------------------------------------------- */
double orc_station_x(const orc_model *m, int32_t ix);
double orc_station_y(const orc_model *m, int32_t iy);
int32_t orc_region_axis(double x, double off, double w, int32_t g);
int32_t orc_partition_and_color(const orc_model *m, int32_t gx, int32_t gy,
                                double offx, double offy, int32_t dynamic,
                                int32_t *nrx, int32_t *nry, int32_t *period,
                                int32_t *ncolors, int32_t *color_of_region);
int64_t orc_coloring_violations(const orc_model *m, int32_t gx, int32_t gy,
                                double offx, double offy, int32_t period);
double  orc_line_tau_max(const orc_model *m);
void    orc_line_fit(const orc_model *m, const double *a, double *x, double *t);

/* ---- likelihood ------------------------------------------------------- */
typedef struct {
    double  d, a, amp;   /* distance, arrival time, amplitude */
    int64_t n0, n1;      /* affected samples [n0, n1); empty when not detected */
    int32_t in;          /* detected: d < rc */
    int32_t _pad;
} orc_arrival_t;
double orc_arrival_time(double x, double y, double t, double sx, double sy, double vel,
                        double *d_out);
void   orc_arrival(const orc_model *m, const orc_event *e, int32_t ix, int32_t iy,
                   orc_arrival_t *out);
double orc_arrival_variance(const orc_model *m, const orc_arrival_t *ar, int64_t n);
void   orc_event_variance(const orc_model *m, const orc_event *ev, int64_t nev, double *E);
void   orc_event_variance_rows(const orc_model *m, const orc_event *ev, int64_t nev, int64_t j0,
                               int64_t nrows, double *E);
double orc_loglik(const orc_model *m, const double *s, const orc_event *ev, int64_t nev);
double orc_logprior(const orc_model *m, const orc_event *ev, int64_t nev);
double orc_single_term(double sigma, double s, double e);

/* ---- forward simulator ------------------------------------------------ */
void   orc_simulate(const orc_model *m, const orc_event *truth, int64_t nev,
                    uint32_t seed, double *s_out);
void   orc_simulate_rows(const orc_model *m, const orc_event *truth, int64_t nev, uint32_t seed,
                         int64_t j0, int64_t nrows, double *s_out);
void   orc_trace_from_noise_f32(const orc_model *m, const orc_event *truth, int64_t nev,
                                const float *z, float *s_out);

/* ---- learned proposal: training pairs and anchor features -------------- */
void   orc_mdn_pair(const orc_model *m, uint32_t seed, int64_t p, double *feat, double *target);
void   orc_anchor_features(const orc_model *m, const double *s, int32_t n_tau, int32_t a,
                           double *feat);

/* ---- the sampler (serial, chromatic static/dynamic, naive) ----------- */
typedef struct orc_chain orc_chain;
orc_chain *orc_chain_new(const orc_model *m, const orc_sampler *sp, const double *s,
                         uint32_t seed, uint32_t chain);
orc_chain *orc_chain_new_f32(const orc_model *m, const orc_sampler *sp, const float *s,
                             uint32_t seed, uint32_t chain);
void    orc_chain_free(orc_chain *c);
int32_t orc_chain_begin_sweep(orc_chain *c, int64_t sweep);
int32_t orc_chain_phase(orc_chain *c, int64_t sweep, int32_t color,
                        const double *feed, double *log);
int32_t orc_chain_sweep(orc_chain *c, int64_t sweep, const double *feed, double *log);
/* threads > 1: the regions of each colour phase run on that many OpenMP
 * threads (when built with OpenMP); the chain is the same. */
void    orc_chain_set_threads(orc_chain *c, int32_t threads);
int64_t orc_chain_count(const orc_chain *c);
/* learned birth proposal: table [nsta * n_tau][8][8] of (mean x, y, t, sd x,
 * y, t, log weight, cumulative weight) and anchor weights [nsta * n_tau],
 * both kept by the caller; NULL table switches it off. */
int32_t orc_chain_set_learned(orc_chain *c, const double *table, const double *weights,
                              int32_t n_tau, double p_learned);
void    orc_move_draws16(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                         uint32_t j, double out[16]);
void    orc_move_draws_arr(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                           uint32_t j, double out[16]);
double  orc_chain_learned_q(orc_chain *c, int32_t region, double x, double y, double t);
int32_t orc_chain_learned_draw(orc_chain *c, int32_t region, const double *d, double *out);
int64_t orc_chain_events(const orc_chain *c, orc_event *out, int64_t cap);
int32_t orc_chain_set_events(orc_chain *c, const orc_event *ev, int64_t nev);
void    orc_chain_layout(const orc_chain *c, int32_t *nrx, int32_t *nry, int32_t *period,
                         int32_t *ncolors, double *offx, double *offy);
int64_t orc_chain_overflows(const orc_chain *c);
double  orc_chain_delta(orc_chain *c, int32_t region, int32_t type, int64_t idx,
                        const orc_event *proposed);

/* ---- lattice mode: brute-force enumeration of the posterior ---------- */
int64_t orc_lattice_nsites(const orc_model *m, const orc_sampler *sp);
void    orc_lattice_site(const orc_model *m, const orc_sampler *sp, int64_t site,
                         orc_event *out);
int64_t orc_enumerate(const orc_model *m, const orc_sampler *sp, const double *s,
                      int32_t nmax, int32_t *sites_out, double *logw_out, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif
