// cmh_common.hpp -- shared definitions of the chromatic MH library: the
// by-value parameter block every kernel receives, the event-table layout, and
// the small pieces of arithmetic that must give the same bits on the host and
// the device (Philox4x32-10, uniform conversion, region binning, arrival
// geometry).  Compiled with -ffp-contract=off so that no product is fused
// into an add where the result decides an integer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmh {

constexpr int kMaxCap = 64;          // events per region
constexpr int kMaxSeg = 32;          // footprint segments per move
constexpr int kMaxTs = 128;          // signal duration, samples
constexpr int kMaxFootprint = 2048;  // samples touched by one move (16 * kMaxTs)
constexpr int kDrawChunk = 64;       // moves whose draws are staged at once
constexpr int kTile = 8192;          // samples per workgroup in streaming kernels
constexpr int kRefreshU = 8;         // samples per thread per step of a streaming loop
constexpr int kMaxTileEvents = 640;  // events reaching one station tile
constexpr int kMaxRegSta = 16;       // stations of one region, learned births
constexpr int kNaiveMax = 2048;      // stations x samples of an instance, naive schedule

enum : int {
    kFlagCap = 1, kFlagNan = 2, kFlagSeg = 4, kFlagTile = 8, kFlagSta = 16, kFlagRace = 32,
    kFlagWait = 64  // persistent form: a colour-counter wait exceeded its spin limit
};

// Per-chain statistics: [3 t + 0..2] attempted / evaluated / accepted moves of
// type t < 5, [15] footprint samples evaluated, [16] footprint samples
// rewritten, [17 + 3 (t - 5) + 0..2] the same for the latent-arrival moves
// t = 5 (arrival time) and t = 6 (joint).
constexpr int kStats = 23;
__host__ __device__ constexpr int stat_base(int t) { return t < 5 ? 3 * t : 17 + 3 * (t - 5); }

// The arrival-time jitter of latent arrivals is truncated at this many
// standard deviations.
constexpr double kArrTrunc = 4.0;

// Model, partition and sampler constants (by value in every kernel).
struct Geo {
    int nsx, nsy, nsta, ts;
    int N;
    int gx, gy, nrx, nry, R;
    int period, ncolors, dynamic;
    int k, cap, prior_only;
    uint32_t seed;
    double ds, sigma2, atten, vel, decay, rc, lambda, mmin, mrate, Lx, Ly;
    double wx, wy;
    double pb, pd, ploc, pt, pm, sxy, st, sm;
    double c1, c2, c3, c4;  // cumulative move-type thresholds
    double att2, dec2;      // 2 / atten, 2 / decay (1 / atten, 1 / decay for templates)
    // Line model (the paper's 1-D world): stations at sx[0 .. nsx) on a line
    // (nsy = 1), events (x, t) with y = 0, regions of onset time along the
    // first region axis (wx is the region length in samples, wy = 0).  The
    // host sets rc, atten and decay to infinity there, so every station
    // detects every event with a constant (boxcar) signal variance m^2.
    int line;
    int tmpl;               // 1: mean-template likelihood (B is an amplitude)
    int naive, pad_naive;   // 1: the naive schedule (Algorithm 3), one phase
    double tmax;            // longest travel time from the line to a station
    double sx[8];
    // Latent arrival times (line model, arrival_sd > 0): every event carries
    // per-station offsets (Events::da), its arrival at station j is
    // t + d / vel + da[j] with |da[j]| <= arr_e, and two more move types
    // exist: 5, the arrival-time move, and 6, the joint two-event move.
    int latent, pad_latent;
    double arr_sd, arr_e, arr_2v;  // arrival_sd; kArrTrunc * arrival_sd; 2 arrival_sd^2
    double pa, pj, sa;      // arrival and joint move probabilities, arrival step
    double c5, c6;          // cumulative thresholds after the magnitude, arrival moves
    int owner, pad_owner;   // 1: the debug owner check (Slot::owner)
    double inv_ds;          // 1 / ds: candidate cells of a footprint (a cell off by one at
                            // a cell edge still leaves every station within rc in the box)
};

// Learned birth proposal: a mixture over the anchors (station, window) of
// the stations in a region, mixed with the prior birth with probability pl.
// tab and w belong to the caller; the rest is derived by the library.
struct Learned {
    const double *tab;    // [nsta * ntau][8][8]: mean x, y, t, sd x, y, t, log w, cum w
    const double *w;      // anchor weights [nsta * ntau]
    const double *cum;    // per station: running sums of its anchors' weights
    const double *norm;   // [nsta * ntau][8]: log weight minus log normaliser
    const double *reach;  // min and max over the table of mean t -/+ 4 sd t - tau
    double *birth;        // [chain][region][move][4]: birth proposal x, y, t, log b/p
    double *raw;          // [chain][region][move][8]: draws 8..15 of each record
    int ntau;
    double pl;
};

// Sweep-kernel forms (the sampler's block): 64, one wave per work item; 128,
// 256, 512, the latency form with that workgroup size; kSpecBase + 64 D,
// the speculative form with D = 2, 4 or 8 waves per work item; kPersist,
// the wave form as one persistent launch per sweep over every colour.
constexpr int kSpecBase = 1024;
constexpr int kPersist = 2048 + 64;
__host__ __device__ constexpr bool is_spec_block(int b)
{
    return b == kSpecBase + 128 || b == kSpecBase + 256 || b == kSpecBase + 512;
}

// Persistent form's queue: a ticket counter, per slot the items of the
// current sweep it has completed, per item (colour order) the count of its
// slot's items in lower colours it waits for, and the wait's spin limit.
// ticket and done are cleared before every launch.
struct PersistArg {
    int *ticket;
    unsigned *done;
    const unsigned *wait;
    long long spin_limit;
};

// Work items of the sweep kernels: region r of slot s packed as (s << 16) | r.
constexpr int kMaxItemRegions = 65536;
constexpr int kMaxSlots = 65536;

// Region-slot event table for all chains.  Slot s of region r of chain c is
// element ((c * R) + r) * cap + s of each array; cnt[c * R + r] slots are
// live, ordered by id.  off[2c], off[2c+1]: the partition offset the table
// is laid out for.
struct Events {
    double *x, *y, *t, *m;
    unsigned long long *id;
    int *cnt;
    double *off;
    double *da;  // latent arrivals: [slot][8] per-station offsets, else nullptr
};

// One chain of one instance as the sweep kernels see it: the instance's
// constants, its Philox key word (seed in g, chain here), and its own
// buffers.  The event tables are slot-local: region r's events at r * cap,
// cnt[r], the offsets at off[0..1]; draws [R][k][8]; stats [kStats].  The
// learned arrays birth and raw are slot-local too.
struct Slot {
    Geo g;
    uint32_t chain;
    int pad_;
    const void *trace;
    double *E;            // [nsta][N]
    Events ev[2];         // ping-pong tables of the dynamic re-layout
    double *draws;
    double *draws2;       // latent arrivals: draws 8..15 of each record [R][k][8]
    unsigned long long *stats;
    Learned L;
    // Debug owner check (else nullptr): per sample of E the tag
    // (phase << 16) | region of the last move that read or wrote it, with
    // phase = sweep * colours + colour + 1.  A move that finds another
    // region's tag of its own phase proves that two regions of one colour
    // share a sample, which the colouring must rule out.
    unsigned long long *owner;  // [nsta][N]
};

// Kernel time stamps (measurement): for sweeps first .. first + n - 1, the
// sweep kernel of colour `colour` folds the steady clock (wall_clock64) at
// the start of each of its workgroups into p[2 q] with a minimum and at the
// end into p[2 q + 1] with a maximum, q = (sweep - first) ncol + colour.
// The caller clears p (all ones, zeros) before the stamped sweeps run.
struct StampArg {
    unsigned long long *p;
    long long first, n;
    int colour, ncol;
};

__device__ inline void stamp_at(const StampArg &sa, long long sweep, int end)
{
    if (sa.p == nullptr || sweep < sa.first || sweep >= sa.first + sa.n) return;
    unsigned long long *q = sa.p + 2 * ((sweep - sa.first) * sa.ncol + sa.colour) + end;
    const unsigned long long t = (unsigned long long)wall_clock64();
    if (end)
        atomicMax(q, t);
    else
        atomicMin(q, t);
}

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): ten rounds, each multiplying counter
// words 0 and 2 by the Philox multipliers and mixing the high halves with the
// other words and the round key; the key advances by the Weyl constants.
__host__ __device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int round = 0; round < 10; ++round) {
        const uint64_t a = (uint64_t)0xD2511F53u * c[0];
        const uint64_t b = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t x0 = (uint32_t)(b >> 32) ^ c[1] ^ k0;
        const uint32_t x2 = (uint32_t)(a >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)b;
        c[3] = (uint32_t)a;
        c[0] = x0;
        c[2] = x2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Open-interval uniform: centre of cell k of 2^52, k from the top 26 bits of
// two words.  Exact in binary64.
__host__ __device__ inline double unit_open(uint32_t hi, uint32_t lo)
{
    const uint64_t cell = ((uint64_t)(hi >> 6) << 26) | (uint64_t)(lo >> 6);
    return (double)(cell * 2u + 1u) * 0x1p-53;
}

// Partition offset of sweep `sweep` for chain `chain`: counter
// (sweep, 0xFFFFFFFF, 0, 0) under key (seed, chain).
__host__ __device__ inline void sweep_offset(uint32_t seed, uint32_t chain, uint32_t sweep,
                                             double wx, double wy, double *ox, double *oy)
{
    uint32_t c[4] = {sweep, 0xFFFFFFFFu, 0u, 0u};
    philox10(c, seed, chain);
    *ox = unit_open(c[0], c[1]) * wx;
    *oy = unit_open(c[2], c[3]) * wy;
}

// Region index along one axis: floor((x - off) / w) + 1 clamped to [0, g].
__host__ __device__ inline int region_axis(double x, double off, double w, int g)
{
    const double f = floor((x - off) / w);
    int i = (int)f + 1;
    i = i < 0 ? 0 : i;
    return i > g ? g : i;
}

// Rectangle of region index i along one axis, clipped to [0, L).
__host__ __device__ inline void region_span(double off, double w, double L, int i, double *lo,
                                            double *hi)
{
    const double a = off + (double)(i - 1) * w;
    const double b = off + (double)i * w;
    *lo = a > 0.0 ? a : 0.0;
    *hi = b < L ? b : L;
}

// Station position on the cell-centred grid.
__host__ __device__ inline double station_pos(int i, double ds) { return ((double)i + 0.5) * ds; }

// Region of an event under offsets (offx, offy): by location on the grid, by
// onset time in the line model.
__host__ __device__ inline int event_region(const Geo &g, double offx, double offy, double x,
                                            double y, double t)
{
    if (g.line) return region_axis(t, offx, g.wx, g.gx);
    return region_axis(y, offy, g.wy, g.gy) * g.nrx + region_axis(x, offx, g.wx, g.gx);
}

// Arrival of an event at a station: distance, arrival time, first sample and
// the variance scale B = A^2 exp(-2 (n0 - a) / decay), so that the variance
// the event adds at sample n0 + q is B exp(-2 q / decay).  Under the
// mean-template likelihood B = A exp(-(n0 - a) / decay) scales the waveform
// B exp(-q / decay) the event adds to the mean.  n0 = ceil(a) is negative
// where a latent offset puts the arrival before the trace; the samples the
// event affects are then [0, n1).
struct Arrival {
    int in;       // d < rc and the window starts before the end of the trace
    int n0, n1;   // n0 = ceil(a), n1 = min(n0 + ts, N): the window, [max(n0, 0), n1) in the trace
    double B;
};

// The station sits at (px, py): station_pos of its grid cell, or its place
// on the line (y = 0) in the line model.  eps is the event's arrival offset
// at this station (latent arrivals; 0 otherwise).
__device__ inline Arrival arrive(const Geo &g, double x, double y, double t, double m, double px,
                                 double py, double eps)
{
    Arrival ar;
    const double dx = x - px;
    const double dy = y - py;
    const double d = sqrt(dx * dx + dy * dy);
    const double a = t + d / g.vel + eps;
    const double c = ceil(a);
    ar.in = 0;
    ar.n0 = 0;
    ar.n1 = 0;
    ar.B = 0.0;
    // a latent offset can put an arrival before the first sample: n0 is then
    // negative, and n1 <= 0 if the whole window precedes the trace (users of
    // the window cut it at sample 0)
    if (d < g.rc && c < (double)g.N) {
        ar.n0 = (int)c;
        ar.n1 = ar.n0 + g.ts < g.N ? ar.n0 + g.ts : g.N;
        // A^2 exp(-2 (c - a) / decay) with A = m exp(-d / atten), one exponential
        ar.B = (g.tmpl ? m : m * m) * exp(-(g.att2 * d + g.dec2 * (c - a)));
        ar.in = 1;
    }
    return ar;
}

}  // namespace cmh
