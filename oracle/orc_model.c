/*
 * orc_model.c -- oracle: random numbers, geometry, partition and colouring,
 * likelihood and forward simulator.  TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Plain FP64, no blocking, no fusion: each function states the definition it
 * follows and computes it directly.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------
 * Philox4x32-10, as defined by Salmon, Moraes, Dror and Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3" (SC'11): a 10-round Feistel-like
 * bijection of a 128-bit counter under a 64-bit key.  Each round multiplies
 * counter words 0 and 2 by the two Philox multipliers, exchanges and XORs the
 * halves with the other words and the round key; the key is bumped by the two
 * Weyl constants between rounds.
 * ---------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform on the open interval (0, 1) from two 32-bit words: the top 26 bits
 * of each word form a 52-bit integer k, and u = (2k + 1) / 2^53, the centre
 * of the k-th of 2^52 equal cells.  2k + 1 < 2^53 is exactly representable,
 * so the conversion is exact on any IEEE machine and never yields 0 or 1. */
double orc_u01(uint32_t w0, uint32_t w1)
{
    uint64_t k = ((uint64_t)(w0 >> 6) << 26) | (uint64_t)(w1 >> 6);
    return (double)(2u * k + 1u) * 0x1p-53;
}

/* Key of a sampler chain: (seed, chain).  Counter of a move's draws:
 * (sweep, region, move, block).  Four blocks per move give the record
 *   [0] uniform choosing the move type     [1] uniform a (index / birth x)
 *   [2] uniform b (birth y / direction)    [3] uniform c (birth onset time)
 *   [4] Exp(1) draw (birth magnitude)      [5],[6] two standard normals
 *   [7] log of the acceptance uniform
 * Normals use the Box-Muller transform. */
void orc_move_draws(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                    uint32_t j, double out[8])
{
    uint32_t key[2] = {seed, chain};
    uint32_t w[4];
    uint32_t ctr[4] = {sweep, region, j, 0u};

    orc_philox4x32_10(ctr, key, w);
    out[0] = orc_u01(w[0], w[1]);
    out[1] = orc_u01(w[2], w[3]);

    ctr[3] = 1u;
    orc_philox4x32_10(ctr, key, w);
    out[2] = orc_u01(w[0], w[1]);
    out[3] = orc_u01(w[2], w[3]);

    ctr[3] = 2u;
    orc_philox4x32_10(ctr, key, w);
    out[4] = -log(orc_u01(w[0], w[1]));
    out[7] = log(orc_u01(w[2], w[3]));

    ctr[3] = 3u;
    orc_philox4x32_10(ctr, key, w);
    double u1 = orc_u01(w[0], w[1]);
    double u2 = orc_u01(w[2], w[3]);
    double r = sqrt(-2.0 * log(u1));
    out[5] = r * cos(2.0 * M_PI * u2);
    out[6] = r * sin(2.0 * M_PI * u2);
}

/* Dynamic colouring (Section 4.3.2): after every full round the region
 * boundaries are shifted by an offset drawn uniformly; here one offset per
 * axis, uniform on [0, w), drawn from counter (sweep, 0xFFFFFFFF, 0, 0). */
void orc_offset(uint32_t seed, uint32_t chain, uint32_t sweep, double wx, double wy,
                double *dx, double *dy)
{
    uint32_t key[2] = {seed, chain};
    uint32_t ctr[4] = {sweep, 0xFFFFFFFFu, 0u, 0u};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    *dx = orc_u01(w[0], w[1]) * wx;
    *dy = orc_u01(w[2], w[3]) * wy;
}

/* ------------------------------------------------------------------------
 * Geometry.  Stations sit at the centres of an nsx x nsy grid of cells of
 * side ds.
 * ---------------------------------------------------------------------- */
double orc_station_x(const orc_model *m, int32_t ix)
{
    return m->line ? m->sta_x[ix] : ((double)ix + 0.5) * m->ds;
}
double orc_station_y(const orc_model *m, int32_t iy)
{
    return m->line ? 0.0 : ((double)iy + 0.5) * m->ds;
}

/* Region index along one axis (Section 4.1 partitions the latent space into
 * intervals of length l; Section 4.3.2 shifts all boundaries by an offset).
 * Region i covers [off + (i-1) w, off + i w) clipped to the domain, so an
 * offset in [0, w) gives regions 0..g. */
int32_t orc_region_axis(double x, double off, double w, int32_t g)
{
    double f = floor((x - off) / w);
    int32_t i = (int32_t)f + 1;
    if (i < 0) i = 0;
    if (i > g) i = g;
    return i;
}

static void region_bounds(double off, double w, double L, int32_t i, double *lo, double *hi)
{
    double a = off + (double)(i - 1) * w;
    double b = off + (double)i * w;
    *lo = a > 0.0 ? a : 0.0;
    *hi = b < L ? b : L;
}

/* Distance from a point to the closure of a rectangle. */
static double rect_dist(double px, double py, double x0, double x1, double y0, double y1)
{
    double dx = 0.0, dy = 0.0;
    if (px < x0) dx = x0 - px; else if (px > x1) dx = px - x1;
    if (py < y0) dy = y0 - py; else if (py > y1) dy = py - y1;
    return sqrt(dx * dx + dy * dy);
}

/* Line model: distances from station j to the nearest and farthest event
 * location in [0, xmax]. */
static void line_reach(const orc_model *m, int32_t j, double *dmin, double *dmax)
{
    double sx = m->sta_x[j];
    *dmin = sx < 0.0 ? -sx : (sx > m->xmax ? sx - m->xmax : 0.0);
    double a = fabs(sx), b = fabs(sx - m->xmax);
    *dmax = a > b ? a : b;
}

/* Line model: the longest travel time from any location to any station
 * (Section 3's tau_max, the time a wave takes to cross the world when the
 * stations sit at its ends). */
double orc_line_tau_max(const orc_model *m)
{
    double t = 0.0;
    for (int32_t j = 0; j < m->nsx; ++j) {
        double dmin, dmax;
        line_reach(m, j, &dmin, &dmax);
        if (dmax / m->vel > t) t = dmax / m->vel;
    }
    return t;
}

/* Line model (Section 4.1's time partition): region i holds onsets in
 * [t0, t1); its events arrive at station j within [t0 + dmin / vel - e,
 * t1 + dmax / vel + e), e the bound of the arrival jitter (0 without latent
 * arrivals), so the samples they can touch lie in
 * [ceil(t0 + dmin / vel - e), ceil(t1 + dmax / vel + e) + ts).  Two regions
 * of one colour conflict when these sample ranges meet at some station:
 * their events could then explain the same samples. */
static int64_t line_violations(const orc_model *m, int32_t g, double off, int32_t period)
{
    double w = (double)m->N / (double)g;
    double e = ORC_ARR_TRUNC * m->arr_sd;
    int64_t bad = 0;
    for (int32_t j = 0; j < m->nsx; ++j) {
        double dmin, dmax;
        line_reach(m, j, &dmin, &dmax);
        for (int32_t a = 0; a <= g; ++a) {
            double a0, a1;
            region_bounds(off, w, (double)m->N, a, &a0, &a1);
            if (!(a1 > a0)) continue;
            double lo_a = ceil(a0 + dmin / m->vel - e);
            double hi_a = ceil(a1 + dmax / m->vel + e) + m->ts;
            for (int32_t b = a + 1; b <= g; ++b) {
                if (a % period != b % period) continue;
                double b0, b1;
                region_bounds(off, w, (double)m->N, b, &b0, &b1);
                if (!(b1 > b0)) continue;
                double lo_b = ceil(b0 + dmin / m->vel - e);
                double hi_b = ceil(b1 + dmax / m->vel + e) + m->ts;
                if (lo_a < hi_b && lo_b < hi_a) ++bad;
            }
        }
    }
    return bad;
}

/* Line model: least-squares location and onset of an event from its arrival
 * times a[0 .. nsx) at the stations: minimise
 * F(x, t) = sum_j (a_j - t - |x - sx_j| / vel)^2 over x in [0, xmax] and t.
 * Between consecutive breakpoints (0, xmax and the station positions inside
 * (0, xmax)) every |x - sx_j| is linear in x, with sign g_j = +1 for stations
 * at or left of the interval's midpoint and -1 otherwise; there
 * c_j = a_j + g_j sx_j / vel = t + g_j x / vel is a straight-line regression
 * of c on g, whose slope gives x / vel (the midpoint when every g_j is the
 * same).  x is clamped to the interval, t is the mean of a_j - |x - sx_j| /
 * vel at that x, and the interval with the smallest F wins (the first in
 * breakpoint order on ties).  This is the geometric analysis behind the
 * joint move of Section 3: it places an event where a set of arrivals says
 * it must be. */
void orc_line_fit(const orc_model *m, const double *a, double *x_out, double *t_out)
{
    const int32_t ns = m->nsx;
    double bp[10];
    int32_t nb = 0;
    bp[nb++] = 0.0;
    for (int32_t j = 0; j < ns; ++j)
        if (m->sta_x[j] > 0.0 && m->sta_x[j] < m->xmax) bp[nb++] = m->sta_x[j];
    bp[nb++] = m->xmax;
    double best_f = INFINITY, best_x = 0.0, best_t = 0.0;
    for (int32_t q = 0; q < nb; ++q) {
        double lo = bp[q], hi = INFINITY;
        for (int32_t r = 0; r < nb; ++r)
            if (bp[r] > lo && bp[r] < hi) hi = bp[r];
        if (hi == INFINITY) continue;  /* lo is the last breakpoint */
        double mid = 0.5 * (lo + hi);
        double sgn[8], cj[8], gbar = 0.0, cbar = 0.0;
        for (int32_t j = 0; j < ns; ++j) {
            sgn[j] = m->sta_x[j] <= mid ? 1.0 : -1.0;
            cj[j] = a[j] + sgn[j] * m->sta_x[j] / m->vel;
            gbar += sgn[j];
            cbar += cj[j];
        }
        gbar /= (double)ns;
        cbar /= (double)ns;
        double sgg = 0.0, sgc = 0.0;
        for (int32_t j = 0; j < ns; ++j) {
            double dg = sgn[j] - gbar;
            sgg += dg * dg;
            sgc += dg * (cj[j] - cbar);
        }
        double x = sgg > 0.0 ? m->vel * (sgc / sgg) : mid;
        if (x < lo) x = lo;
        if (x > hi) x = hi;
        double t = 0.0;
        for (int32_t j = 0; j < ns; ++j) t += a[j] - fabs(x - m->sta_x[j]) / m->vel;
        t /= (double)ns;
        double f = 0.0;
        for (int32_t j = 0; j < ns; ++j) {
            double r = (a[j] - t) - fabs(x - m->sta_x[j]) / m->vel;
            f += r * r;
        }
        if (f < best_f) {
            best_f = f;
            best_x = x;
            best_t = t;
        }
    }
    *x_out = best_x;
    *t_out = best_t;
}

/* Number of (station, pair of same-coloured regions) conflicts: two regions
 * of one colour must not both lie within the detection cutoff of a common
 * station, otherwise their events could explain the same signal and the
 * regions would not be conditionally independent (the Markov-blanket
 * argument of Section 4.1, with the blanket given by shared stations). */
int64_t orc_coloring_violations(const orc_model *m, int32_t gx, int32_t gy,
                                double offx, double offy, int32_t period)
{
    if (m->line) return line_violations(m, gx, offx, period);
    double Lx = (double)m->nsx * m->ds, Ly = (double)m->nsy * m->ds;
    double wx = Lx / (double)gx, wy = Ly / (double)gy;
    int32_t nrx = gx + 1;
    int64_t bad = 0;
    int32_t cap = (gx + 1) * (gy + 1);
    int32_t *near = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    for (int32_t sy = 0; sy < m->nsy; ++sy) {
        for (int32_t sx = 0; sx < m->nsx; ++sx) {
            double px = orc_station_x(m, sx), py = orc_station_y(m, sy);
            int32_t nn = 0;
            for (int32_t k = 0; k <= gy; ++k) {
                double y0, y1;
                region_bounds(offy, wy, Ly, k, &y0, &y1);
                if (!(y1 > y0)) continue;
                for (int32_t i = 0; i <= gx; ++i) {
                    double x0, x1;
                    region_bounds(offx, wx, Lx, i, &x0, &x1);
                    if (!(x1 > x0)) continue;
                    if (rect_dist(px, py, x0, x1, y0, y1) < m->rc) near[nn++] = k * nrx + i;
                }
            }
            for (int32_t a = 0; a < nn; ++a) {
                for (int32_t b = a + 1; b < nn; ++b) {
                    int32_t ia = near[a] % nrx, ka = near[a] / nrx;
                    int32_t ib = near[b] % nrx, kb = near[b] / nrx;
                    int32_t ca = (ia % period) + period * (ka % period);
                    int32_t cb = (ib % period) + period * (kb % period);
                    if (ca == cb) ++bad;
                }
            }
        }
    }
    free(near);
    return bad;
}

/* Line model partition: gx regions of onset time (gy unused), colour i mod p.
 * Dynamic partitions need p - 1 region lengths to cover the longest travel
 * time plus the signal duration plus twice the jitter bound e,
 * p = ceil((tau_max + ts + 2 e) / w) + 1. */
static int32_t line_partition(const orc_model *m, int32_t gx, double offt, int32_t dynamic,
                              int32_t *nrx, int32_t *nry, int32_t *period, int32_t *ncolors,
                              int32_t *color_of_region)
{
    double w = (double)m->N / (double)gx;
    int32_t p;
    if (dynamic) {
        p = (int32_t)ceil((orc_line_tau_max(m) + (double)m->ts + 2.0 * ORC_ARR_TRUNC * m->arr_sd)
                          / w) + 1;
        if (line_violations(m, gx, offt, p) != 0) return -4;
    } else {
        for (p = 1; p <= gx + 1; ++p)
            if (line_violations(m, gx, offt, p) == 0) break;
        if (p > gx + 1) return -4;
    }
    *nrx = gx + 1;
    *nry = 1;
    *period = p;
    *ncolors = p;
    if (color_of_region)
        for (int32_t i = 0; i <= gx; ++i) color_of_region[i] = i % p;
    return 0;
}

/* Partition and colouring.  Colour of region (i, k) is (i mod p) + p (k mod p).
 * Static partitions (Section 4.3.1) use the smallest period whose colouring
 * passes the exact station check at the given offset; dynamic partitions
 * (Section 4.3.2) need a period that holds for every offset: same-coloured
 * regions are then at least (p - 1) w apart, which exceeds 2 rc when
 * p = ceil(2 rc / w) + 1.  Returns 0, or -4 when no valid colouring exists. */
int32_t orc_partition_and_color(const orc_model *m, int32_t gx, int32_t gy,
                                double offx, double offy, int32_t dynamic,
                                int32_t *nrx, int32_t *nry, int32_t *period,
                                int32_t *ncolors, int32_t *color_of_region)
{
    if (m->line)
        return line_partition(m, gx, offx, dynamic, nrx, nry, period, ncolors, color_of_region);
    double Lx = (double)m->nsx * m->ds, Ly = (double)m->nsy * m->ds;
    double wx = Lx / (double)gx, wy = Ly / (double)gy;
    double w = wx < wy ? wx : wy;
    int32_t p;
    if (dynamic) {
        p = (int32_t)ceil(2.0 * m->rc / w) + 1;
        if (orc_coloring_violations(m, gx, gy, offx, offy, p) != 0) return -4;
    } else {
        int32_t pmax = (gx > gy ? gx : gy) + 1;
        for (p = 1; p <= pmax; ++p)
            if (orc_coloring_violations(m, gx, gy, offx, offy, p) == 0) break;
        if (p > pmax) return -4;
    }
    *nrx = gx + 1;
    *nry = gy + 1;
    *period = p;
    *ncolors = p * p;
    if (color_of_region) {
        for (int32_t k = 0; k <= gy; ++k)
            for (int32_t i = 0; i <= gx; ++i)
                color_of_region[k * (gx + 1) + i] = (i % p) + p * (k % p);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Signal model (Section 3).
 * ---------------------------------------------------------------------- */

/* Arrival time of an event at a station: onset plus distance over wave speed
 * (the mean of the arrival model in Section 3; this model has no jitter). */
double orc_arrival_time(double x, double y, double t, double sx, double sy, double vel,
                        double *d_out)
{
    double dx = x - sx, dy = y - sy;
    double d = sqrt(dx * dx + dy * dy);
    if (d_out) *d_out = d;
    return t + d / vel;
}

/* Arrival of one event at station (ix, iy): distance d, detection d < rc,
 * arrival a = t + d / vel (plus the event's offset da[ix] when the line
 * model's arrivals are latent), amplitude A = m exp(-d / atten), and the samples
 * [n0, n1) = [ceil(a), ceil(a) + ts) clipped to the trace.  In the line
 * model every station detects and the amplitude does not attenuate. */
void orc_arrival(const orc_model *m, const orc_event *e, int32_t ix, int32_t iy,
                 orc_arrival_t *out)
{
    out->a = orc_arrival_time(e->x, e->y, e->t, orc_station_x(m, ix), orc_station_y(m, iy),
                              m->vel, &out->d);
    if (m->line && m->arr_sd > 0.0) out->a = out->a + e->da[ix];  /* latent arrival */
    out->in = m->line ? 1 : out->d < m->rc;
    out->amp = m->line ? e->m : e->m * exp(-out->d / m->atten);
    int64_t n0 = (int64_t)ceil(out->a);
    int64_t n1 = n0 + m->ts;
    if (n0 < 0) n0 = 0;
    if (n1 > m->N) n1 = m->N;
    if (!out->in || n0 >= n1) { n0 = 0; n1 = 0; }
    out->n0 = n0;
    out->n1 = n1;
}

/* What the event adds at sample n.  Variance model: its signal is zero-mean
 * Gaussian with standard deviation A phi(n - a), phi(tau) = exp(-tau /
 * decay), during the signal duration, and absent otherwise, so it adds the
 * variance (A phi)^2; the line model's signal is iid over its duration
 * (phi = 1).  Mean-template model: it adds the waveform value A phi(n - a)
 * to the mean. */
double orc_arrival_variance(const orc_model *m, const orc_arrival_t *ar, int64_t n)
{
    if (n < ar->n0 || n >= ar->n1) return 0.0;
    double env = m->line ? 1.0 : exp(-((double)n - ar->a) / m->decay);
    double sd = ar->amp * env;
    return m->tmpl ? sd : sd * sd;
}

/* Events whose signal reaches station (ix, iy) at all. */
static int64_t events_at_station(const orc_model *m, const orc_event *ev, int64_t nev,
                                 int32_t ix, int32_t iy, int64_t *idx)
{
    int64_t k = 0;
    double sx = orc_station_x(m, ix), sy = orc_station_y(m, iy);
    for (int64_t i = 0; i < nev; ++i) {
        double dx = ev[i].x - sx, dy = ev[i].y - sy;
        if (m->line || sqrt(dx * dx + dy * dy) < m->rc) idx[k++] = i;
    }
    return k;
}

/* One station's summed event variance: row[n] = sum over the listed events,
 * in list order, of the variance each adds at sample n. */
static void station_row(const orc_model *m, const orc_event *ev, const int64_t *idx,
                        int64_t k, int32_t ix, int32_t iy, double *row)
{
    for (int64_t n = 0; n < m->N; ++n) row[n] = 0.0;
    for (int64_t q = 0; q < k; ++q) {
        orc_arrival_t ar;
        orc_arrival(m, &ev[idx[q]], ix, iy, &ar);
        for (int64_t n = ar.n0; n < ar.n1; ++n) row[n] += orc_arrival_variance(m, &ar, n);
    }
}

/* E[j][n] = sum over events of the variance each adds (no noise term).
 * Station j = iy * nsx + ix, samples contiguous. */
void orc_event_variance(const orc_model *m, const orc_event *ev, int64_t nev, double *E)
{
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nev > 0 ? nev : 1));
    for (int32_t iy = 0; iy < m->nsy; ++iy) {
        for (int32_t ix = 0; ix < m->nsx; ++ix) {
            double *row = E + ((int64_t)iy * m->nsx + ix) * m->N;
            int64_t k = events_at_station(m, ev, nev, ix, iy, idx);
            station_row(m, ev, idx, k, ix, iy, row);
        }
    }
    free(idx);
}

/* The same for stations [j0, j0 + nrows) only. */
void orc_event_variance_rows(const orc_model *m, const orc_event *ev, int64_t nev, int64_t j0,
                             int64_t nrows, double *E)
{
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nev > 0 ? nev : 1));
    for (int64_t j = j0; j < j0 + nrows; ++j) {
        int32_t ix = (int32_t)(j % m->nsx), iy = (int32_t)(j / m->nsx);
        int64_t k = events_at_station(m, ev, nev, ix, iy, idx);
        station_row(m, ev, idx, k, ix, iy, E + (j - j0) * m->N);
    }
    free(idx);
}

/* Log density of one sample: zero-mean Gaussian with variance sigma^2 + e. */
double orc_single_term(double sigma, double s, double e)
{
    double v = sigma * sigma + e;
    return -0.5 * (log(2.0 * M_PI) + log(v) + s * s / v);
}

/* Mean-template model: Gaussian with mean e and variance sigma^2. */
static double template_term(double sigma, double s, double e)
{
    double r = s - e;
    return -0.5 * (log(2.0 * M_PI) + log(sigma * sigma) + r * r / (sigma * sigma));
}

/* Signal log-likelihood log P(s | e) summed over every station and sample. */
double orc_loglik(const orc_model *m, const double *s, const orc_event *ev, int64_t nev)
{
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nev > 0 ? nev : 1));
    double *row = (double *)malloc(sizeof(double) * (size_t)m->N);
    double total = 0.0;
    for (int32_t iy = 0; iy < m->nsy; ++iy) {
        for (int32_t ix = 0; ix < m->nsx; ++ix) {
            const double *sr = s + ((int64_t)iy * m->nsx + ix) * m->N;
            int64_t k = events_at_station(m, ev, nev, ix, iy, idx);
            station_row(m, ev, idx, k, ix, iy, row);
            for (int64_t n = 0; n < m->N; ++n)
                total += m->tmpl ? template_term(m->sigma, sr[n], row[n])
                                 : orc_single_term(m->sigma, sr[n], row[n]);
        }
    }
    free(row);
    free(idx);
    return total;
}

/* Log of the event prior (Section 3) as a set density: Poisson count with
 * mean lambda, uniform location over the domain, uniform onset over [0, N),
 * exponential magnitude above mmin. */
double orc_logprior(const orc_model *m, const orc_event *ev, int64_t nev)
{
    double Lx = (double)m->nsx * m->ds, Ly = (double)m->nsy * m->ds;
    double total = -m->lambda;
    if (m->line) {  /* uniform location on [0, xmax), no magnitude */
        for (int64_t i = 0; i < nev; ++i) {
            total += log(m->lambda) - log(m->xmax) - log((double)m->N);
            if (!(m->arr_sd > 0.0)) continue;
            /* latent arrivals: a truncated normal density per station */
            double z = ORC_ARR_TRUNC, mass = erf(z / sqrt(2.0));
            for (int32_t j = 0; j < m->nsx; ++j) {
                double u = ev[i].da[j] / m->arr_sd;
                if (fabs(u) > z) return -INFINITY;
                total += -0.5 * u * u - log(m->arr_sd * sqrt(2.0 * M_PI) * mass);
            }
        }
        return total;
    }
    for (int64_t i = 0; i < nev; ++i) {
        total += log(m->lambda) - log(Lx * Ly) - log((double)m->N) + log(m->mrate)
                 - m->mrate * (ev[i].m - m->mmin);
    }
    return total;
}

/* Forward simulator (Section 5 evaluates on worlds sampled from the model):
 * given the true events, each sample is Gaussian with the model's variance,
 * s = sqrt(sigma^2 + E) z.  The standard normal z for station j and sample n
 * comes from Philox under key (seed, 0x80000001), counter (n / 2, j, 0, 0),
 * by Box-Muller: even n take the cosine branch, odd n the sine branch. */
void orc_simulate(const orc_model *m, const orc_event *truth, int64_t nev,
                  uint32_t seed, double *s_out)
{
    orc_simulate_rows(m, truth, nev, seed, 0, (int64_t)m->nsx * m->nsy, s_out);
}

/* The same simulator restricted to stations [j0, j0 + nrows). */
void orc_simulate_rows(const orc_model *m, const orc_event *truth, int64_t nev, uint32_t seed,
                       int64_t j0, int64_t nrows, double *s_out)
{
    uint32_t key[2] = {seed, 0x80000001u};
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nev > 0 ? nev : 1));
    double *row = (double *)malloc(sizeof(double) * (size_t)m->N);
    for (int64_t j = j0; j < j0 + nrows; ++j) {
        int32_t ix = (int32_t)(j % m->nsx), iy = (int32_t)(j / m->nsx);
        double *out = s_out + (j - j0) * m->N;
        int64_t k = events_at_station(m, truth, nev, ix, iy, idx);
        station_row(m, truth, idx, k, ix, iy, row);
        for (int64_t n = 0; n < m->N; ++n) {
            uint32_t ctr[4] = {(uint32_t)(n >> 1), (uint32_t)j, 0u, 0u};
            uint32_t w[4];
            orc_philox4x32_10(ctr, key, w);
            double u1 = orc_u01(w[0], w[1]);
            double u2 = orc_u01(w[2], w[3]);
            double r = sqrt(-2.0 * log(u1));
            double z = (n & 1) ? r * sin(2.0 * M_PI * u2) : r * cos(2.0 * M_PI * u2);
            out[n] = m->tmpl ? row[n] + m->sigma * z : sqrt(m->sigma * m->sigma + row[n]) * z;
        }
    }
    free(row);
    free(idx);
}

/* The simulator with the standard normals supplied by the caller:
 * s = sqrt(sigma^2 + E) z, rounded to binary32. */
void orc_trace_from_noise_f32(const orc_model *m, const orc_event *truth, int64_t nev,
                              const float *z, float *s_out)
{
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nev > 0 ? nev : 1));
    double *row = (double *)malloc(sizeof(double) * (size_t)m->N);
    for (int32_t iy = 0; iy < m->nsy; ++iy) {
        for (int32_t ix = 0; ix < m->nsx; ++ix) {
            int64_t j = (int64_t)iy * m->nsx + ix;
            int64_t k = events_at_station(m, truth, nev, ix, iy, idx);
            station_row(m, truth, idx, k, ix, iy, row);
            for (int64_t n = 0; n < m->N; ++n)
                s_out[j * m->N + n] =
                    (float)(m->tmpl ? row[n] + m->sigma * (double)z[j * m->N + n]
                                    : sqrt(m->sigma * m->sigma + row[n]) * (double)z[j * m->N + n]);
        }
    }
    free(row);
    free(idx);
}

/* ------------------------------------------------------------------------
 * Learned birth proposal: training pairs and anchor window features.  The
 * network and its proposal density are an addition of this implementation
 * (an independence proposal corrected inside MH, so the posterior is
 * unchanged); the pair generator samples local worlds from the model of
 * Section 3, as the paper's evaluation samples worlds (Section 5).
 * ---------------------------------------------------------------------- */

/* Log envelope of one station over 64 samples from q = s^2 over 67 samples:
 * f[n] = ln(sigma^2 + (q[n] + q[n+1] + q[n+2] + q[n+3]) / 4) - ln(sigma^2). */
static void log_envelope(double sigma, const double *q, double *f)
{
    double s2 = sigma * sigma;
    for (int n = 0; n < 64; ++n)
        f[n] = log(s2 + (q[n] + q[n + 1] + q[n + 2] + q[n + 3]) * 0.25) - log(s2);
}

/* Edge classes of a training pair: class 0 has all nine stations of the 3x3
 * block; classes 1..8 drop the column (ex = -1 left, +1 right) and/or the row
 * (ey) beyond the domain edge, which lies half a spacing from the centre on
 * that side, in the order (-1,-1) (0,-1) (1,-1) (-1,0) (1,0) (-1,1) (0,1)
 * (1,1).  A uniform u gives class 0 when 16u < 8, else class 16u - 7. */
static void edge_class(double u, int *ex, int *ey)
{
    static const int tx[8] = {-1, 0, 1, -1, 1, -1, 0, 1};
    static const int ty[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
    int k = (int)floor(u * 16.0);
    if (k > 15) k = 15;
    if (k < 8) {
        *ex = 0;
        *ey = 0;
    } else {
        *ex = tx[k - 8];
        *ey = ty[k - 8];
    }
}

/* Training pair p: a 3x3 block of stations (spacing ds) around a centre at
 * the origin, with the edge class drawn under counter (p, 0, 8); one target
 * event uniform within one spacing of the centre (inside the domain) and
 * with onset in [-16, 64); three background events anywhere that reaches the
 * block; all magnitudes from the prior.  Draws from Philox under key (seed,
 * 0x80000003): counter (p mod 2^32, p div 2^32, 0, c) for the events and the
 * class, (.., .., 1 + station, n / 2) for the noise of sample n.  Features
 * [9][64]: each present station's log envelope over the window's first 67
 * samples; 0 for a missing station.  Target: offset (x/ds, y/ds, t/32). */
void orc_mdn_pair(const orc_model *m, uint32_t seed, int64_t p, double *feat, double *target)
{
    uint32_t key[2] = {seed, 0x80000003u};
    uint32_t plo = (uint32_t)p, phi = (uint32_t)((uint64_t)p >> 32);
    uint32_t cm[4] = {plo, phi, 0u, 8u}, wm[4];
    orc_philox4x32_10(cm, key, wm);
    int ex, ey;
    edge_class(orc_u01(wm[0], wm[1]), &ex, &ey);
    double ev[4][4];
    for (int e = 0; e < 4; ++e) {
        uint32_t c0[4] = {plo, phi, 0u, (uint32_t)(e == 0 ? 0 : 2 + (e - 1))};
        uint32_t c1[4] = {plo, phi, 0u, (uint32_t)(e == 0 ? 1 : 5 + (e - 1))};
        uint32_t w0[4], w1[4];
        orc_philox4x32_10(c0, key, w0);
        orc_philox4x32_10(c1, key, w1);
        double ux = orc_u01(w0[0], w0[1]), uy = orc_u01(w0[2], w0[3]);
        double ut = orc_u01(w1[0], w1[1]), um = orc_u01(w1[2], w1[3]);
        double reach = e == 0 ? m->ds : 1.5 * m->ds + m->rc;
        double xlo = ex < 0 ? -0.5 * m->ds : -reach, xhi = ex > 0 ? 0.5 * m->ds : reach;
        double ylo = ey < 0 ? -0.5 * m->ds : -reach, yhi = ey > 0 ? 0.5 * m->ds : reach;
        ev[e][0] = xlo + ux * (xhi - xlo);
        ev[e][1] = ylo + uy * (yhi - ylo);
        if (e == 0)
            ev[e][2] = -16.0 + ut * 80.0;
        else
            ev[e][2] = -(double)(m->ts + 8) + ut * (double)(64 + m->ts + 16);
        ev[e][3] = m->mmin - log(um) / m->mrate;
    }
    for (int b = 0; b < 9; ++b) {
        int dx = b % 3 - 1, dy = b / 3 - 1;
        if ((ex != 0 && dx == ex) || (ey != 0 && dy == ey)) {
            for (int n = 0; n < 64; ++n) feat[b * 64 + n] = 0.0;
            continue;
        }
        double sx = (double)dx * m->ds, sy = (double)dy * m->ds;
        double q[67];
        for (int n = 0; n < 67; ++n) {
            double E = 0.0;
            for (int e = 0; e < 4; ++e) {
                double ddx = ev[e][0] - sx, ddy = ev[e][1] - sy;
                double d = sqrt(ddx * ddx + ddy * ddy);
                if (!(d < m->rc)) continue;
                double a = ev[e][2] + d / m->vel;
                double n0 = ceil(a);
                if ((double)n < n0 || (double)n >= n0 + m->ts) continue;
                double amp = ev[e][3] * exp(-d / m->atten);
                double env = exp(-((double)n - a) / m->decay);
                E += (amp * env) * (amp * env);
            }
            uint32_t c[4] = {plo, phi, (uint32_t)(1 + b), (uint32_t)(n >> 1)};
            uint32_t w[4];
            orc_philox4x32_10(c, key, w);
            double u1 = orc_u01(w[0], w[1]), u2 = orc_u01(w[2], w[3]);
            double r = sqrt(-2.0 * log(u1));
            double z = (n & 1) ? r * sin(2.0 * M_PI * u2) : r * cos(2.0 * M_PI * u2);
            double s = sqrt(m->sigma * m->sigma + E) * z;
            q[n] = s * s;
        }
        log_envelope(m->sigma, q, feat + b * 64);
    }
    target[0] = ev[0][0] / m->ds;
    target[1] = ev[0][1] / m->ds;
    target[2] = ev[0][2] / 32.0;
}

/* Anchor a of an instance: centre station c = a div n_tau (any station,
 * row-major), window start 32 (a mod n_tau); features of the 3x3 block
 * around it from the trace, 0 for block stations off the grid. */
void orc_anchor_features(const orc_model *m, const double *s, int32_t n_tau, int32_t a,
                         double *feat)
{
    int32_t c = a / n_tau, ti = a % n_tau;
    int32_t cx = c % m->nsx, cy = c / m->nsx;
    int64_t tau = 32 * (int64_t)ti;
    for (int b = 0; b < 9; ++b) {
        int32_t ix = cx + b % 3 - 1, iy = cy + b / 3 - 1;
        if (ix < 0 || ix >= m->nsx || iy < 0 || iy >= m->nsy) {
            for (int n = 0; n < 64; ++n) feat[b * 64 + n] = 0.0;
            continue;
        }
        int64_t j = (int64_t)iy * m->nsx + ix;
        double q[67];
        for (int n = 0; n < 67; ++n) {
            double v = s[j * m->N + tau + n];
            q[n] = v * v;
        }
        log_envelope(m->sigma, q, feat + b * 64);
    }
}
