/*
 * orc_sampler.c -- oracle: the Metropolis-Hastings sampler over the event
 * set, run region by region in colour phases.  TEST INFRASTRUCTURE ONLY.
 *
 * Follows Section 4: the latent space is partitioned into regions
 * (Section 4.1), regions are coloured so that regions of one colour are
 * conditionally independent, and Algorithm 4 runs k MH moves inside every
 * region of one colour while the other regions are held at their values from
 * the start of the phase.  Section 4.3.2 (dynamic colouring) redraws the
 * partition offset after every full round of colours.  Algorithm 3 (naive
 * parallel MH) runs every region in one phase, each region accepting against
 * the posterior of its own events alone; it is kept only as a negative
 * control.
 *
 * The log-likelihood change of a move is evaluated directly: for every sample
 * the move can affect, the model variance is summed from scratch over the
 * events present before and after the move, and the two Gaussian log
 * densities are differenced.  No incremental state is kept.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    orc_event *e;
    int64_t n, capa;
} evlist;

static void ev_push(evlist *l, const orc_event *e)
{
    if (l->n == l->capa) {
        l->capa = l->capa ? 2 * l->capa : 8;
        l->e = (orc_event *)realloc(l->e, sizeof(orc_event) * (size_t)l->capa);
    }
    l->e[l->n++] = *e;
}

/* Removal keeps the remaining events in their order. */
static void ev_remove(evlist *l, int64_t i)
{
    for (int64_t q = i; q + 1 < l->n; ++q) l->e[q] = l->e[q + 1];
    l->n--;
}

static int cmp_id(const void *a, const void *b)
{
    uint64_t x = ((const orc_event *)a)->id, y = ((const orc_event *)b)->id;
    return x < y ? -1 : (x > y ? 1 : 0);
}

struct orc_chain {
    orc_model m;
    orc_sampler sp;
    const double *s;      /* trace, binary64 ... */
    const float *s32;     /* ... or binary32 */
    uint32_t seed, chain;
    double Lx, Ly, wx, wy;
    int32_t nrx, nry, period, ncolors;
    double offx, offy;
    int32_t *color;
    int64_t nreg;
    evlist *reg;        /* per region, sorted by id */
    evlist *snap;       /* per station: copies of the events that reach it */
    int64_t nsta;
    int64_t overflows;
    int32_t laid_out;
    /* learned birth proposal (off when ltab is NULL) */
    const double *ltab;   /* [nsta * ntau][8 components][8] */
    const double *lw;     /* anchor weights [nsta * ntau] */
    double *lcum;         /* per station: running sums of its anchors' weights */
    int32_t ntau;
    double plearn;
    int32_t threads;      /* host threads for the regions of one phase (1: serial) */
};

/* ---------------------------------------------------------------- lattice */
static double lat_hx(const orc_chain *c) { return c->Lx / (double)c->sp.kx; }
static double lat_hy(const orc_chain *c) { return c->Ly / (double)c->sp.ky; }
static double lat_ht(const orc_chain *c) { return (double)c->m.N / (double)c->sp.kt; }

static void lat_coords(const orc_chain *c, int32_t ix, int32_t iy, int32_t it, int32_t im,
                       orc_event *e)
{
    e->x = ((double)ix + 0.5) * lat_hx(c);
    e->y = c->m.line ? 0.0 : ((double)iy + 0.5) * lat_hy(c);
    e->t = ((double)it + 0.5) * lat_ht(c);
    e->m = c->m.line ? c->m.mmin : c->m.mmin + ((double)im + 0.5) * c->sp.hm;
}

static void lat_index(const orc_chain *c, const orc_event *e, int32_t *ix, int32_t *iy,
                      int32_t *it, int32_t *im)
{
    *ix = (int32_t)floor(e->x / lat_hx(c));
    *it = (int32_t)floor(e->t / lat_ht(c));
    if (c->m.line) {  /* one row of sites, the fixed amplitude */
        *iy = 0;
        *im = 0;
        return;
    }
    *iy = (int32_t)floor(e->y / lat_hy(c));
    *im = (int32_t)floor((e->m - c->m.mmin) / c->sp.hm);
}

/* ------------------------------------------------------------- partition */
/* Region of an event: by location on the grid, by onset time in the line
 * model (whose partition axis is time, Section 4.1). */
static int32_t region_of(const orc_chain *c, double x, double y, double t)
{
    if (c->m.line) return orc_region_axis(t, c->offx, c->wx, c->sp.gx);
    int32_t i = orc_region_axis(x, c->offx, c->wx, c->sp.gx);
    int32_t k = orc_region_axis(y, c->offy, c->wy, c->sp.gy);
    return k * c->nrx + i;
}

/* Line model: the onset interval [t0, t1) of region r. */
static void region_times(const orc_chain *c, int32_t r, double *t0, double *t1)
{
    double a = c->offx + (double)(r - 1) * c->wx, b = c->offx + (double)r * c->wx;
    *t0 = a > 0.0 ? a : 0.0;
    *t1 = b < (double)c->m.N ? b : (double)c->m.N;
}

static void region_rect(const orc_chain *c, int32_t r, double *x0, double *x1, double *y0,
                        double *y1)
{
    int32_t i = r % c->nrx, k = r / c->nrx;
    double a = c->offx + (double)(i - 1) * c->wx, b = c->offx + (double)i * c->wx;
    *x0 = a > 0.0 ? a : 0.0;
    *x1 = b < c->Lx ? b : c->Lx;
    a = c->offy + (double)(k - 1) * c->wy;
    b = c->offy + (double)k * c->wy;
    *y0 = a > 0.0 ? a : 0.0;
    *y1 = b < c->Ly ? b : c->Ly;
}

/* Lattice sites (x, y part) inside region r, in row-major order. */
static int64_t lat_region_sites(const orc_chain *c, int32_t r, int64_t want, int32_t *ix,
                                int32_t *iy)
{
    int64_t cnt = 0;
    for (int32_t b = 0; b < c->sp.ky; ++b) {
        for (int32_t a = 0; a < c->sp.kx; ++a) {
            orc_event e;
            lat_coords(c, a, b, 0, 0, &e);
            if (region_of(c, e.x, e.y, e.t) != r) continue;
            if (cnt == want) { *ix = a; *iy = b; }
            ++cnt;
        }
    }
    return cnt;
}

/* Line model: lattice sites (x, onset) inside region r, onset-major. */
static int64_t lat_line_region_sites(const orc_chain *c, int32_t r, int64_t want, int32_t *ix,
                                     int32_t *it)
{
    int64_t cnt = 0;
    for (int32_t b = 0; b < c->sp.kt; ++b) {
        orc_event e;
        lat_coords(c, 0, 0, b, 0, &e);
        if (region_of(c, e.x, e.y, e.t) != r) continue;
        for (int32_t a = 0; a < c->sp.kx; ++a) {
            if (cnt == want) { *ix = a; *it = b; }
            ++cnt;
        }
    }
    return cnt;
}

static double trace_at(const orc_chain *c, int64_t j, int64_t n)
{
    return c->s ? c->s[j * c->m.N + n] : (double)c->s32[j * c->m.N + n];
}

orc_chain *orc_chain_new_f32(const orc_model *m, const orc_sampler *sp, const float *s,
                             uint32_t seed, uint32_t chain)
{
    orc_chain *c = orc_chain_new(m, sp, NULL, seed, chain);
    c->s32 = s;
    return c;
}

orc_chain *orc_chain_new(const orc_model *m, const orc_sampler *sp, const double *s,
                         uint32_t seed, uint32_t chain)
{
    orc_chain *c = (orc_chain *)calloc(1, sizeof(orc_chain));
    c->m = *m;
    c->sp = *sp;
    c->s = s;
    c->seed = seed;
    c->chain = chain;
    if (m->line) {  /* regions of onset time along the first axis */
        c->Lx = m->xmax;
        c->Ly = 1.0;
        c->wx = (double)m->N / (double)sp->gx;
        c->wy = 0.0;
        c->nrx = sp->gx + 1;
        c->nry = 1;
    } else {
        c->Lx = (double)m->nsx * m->ds;
        c->Ly = (double)m->nsy * m->ds;
        c->wx = c->Lx / (double)sp->gx;
        c->wy = c->Ly / (double)sp->gy;
        c->nrx = sp->gx + 1;
        c->nry = sp->gy + 1;
    }
    c->nreg = (int64_t)c->nrx * c->nry;
    c->color = (int32_t *)calloc((size_t)c->nreg, sizeof(int32_t));
    c->reg = (evlist *)calloc((size_t)c->nreg, sizeof(evlist));
    c->nsta = (int64_t)m->nsx * m->nsy;
    c->snap = (evlist *)calloc((size_t)c->nsta, sizeof(evlist));
    return c;
}

void orc_chain_free(orc_chain *c)
{
    if (c) free(c->lcum);
    if (!c) return;
    for (int64_t r = 0; r < c->nreg; ++r) free(c->reg[r].e);
    for (int64_t j = 0; j < c->nsta; ++j) free(c->snap[j].e);
    free(c->reg);
    free(c->snap);
    free(c->color);
    free(c);
}

/* Lay out the partition for this sweep and move every event into the list
 * of its region, each list sorted by event id.  Returns 0, -3 when a region
 * would exceed its capacity, -4 when the colouring check fails. */
static int32_t relayout(orc_chain *c, double offx, double offy)
{
    c->offx = offx;
    c->offy = offy;
    if (!c->laid_out || c->sp.dynamic) {
        int32_t nrx, nry, p, nc;
        int32_t rc = orc_partition_and_color(&c->m, c->sp.gx, c->sp.gy, offx, offy,
                                             c->sp.dynamic, &nrx, &nry, &p, &nc, c->color);
        if (rc != 0) return rc;
        if (c->sp.period > 0) {
            if (orc_coloring_violations(&c->m, c->sp.gx, c->sp.gy, offx, offy, c->sp.period) != 0)
                return -4;
            p = c->sp.period;
            nc = c->m.line ? p : p * p;
            for (int32_t k = 0; k < nry; ++k)
                for (int32_t i = 0; i < nrx; ++i) c->color[k * nrx + i] = (i % p) + p * (k % p);
        }
        c->period = p;
        c->ncolors = nc;
        c->laid_out = 1;
    }
    evlist all = {0, 0, 0};
    for (int64_t r = 0; r < c->nreg; ++r) {
        for (int64_t q = 0; q < c->reg[r].n; ++q) ev_push(&all, &c->reg[r].e[q]);
        c->reg[r].n = 0;
    }
    int32_t status = 0;
    for (int64_t q = 0; q < all.n; ++q) {
        orc_event e = all.e[q];
        e.region = region_of(c, e.x, e.y, e.t);
        if (c->reg[e.region].n >= c->sp.cap) status = -3;
        ev_push(&c->reg[e.region], &e);
    }
    for (int64_t r = 0; r < c->nreg; ++r)
        qsort(c->reg[r].e, (size_t)c->reg[r].n, sizeof(orc_event), cmp_id);
    free(all.e);
    return status;
}

int32_t orc_chain_begin_sweep(orc_chain *c, int64_t sweep)
{
    double ox = 0.0, oy = 0.0;
    if (c->sp.dynamic) orc_offset(c->seed, c->chain, (uint32_t)sweep, c->wx, c->wy, &ox, &oy);
    return relayout(c, ox, oy);
}

int32_t orc_chain_set_events(orc_chain *c, const orc_event *ev, int64_t nev)
{
    for (int64_t r = 0; r < c->nreg; ++r) c->reg[r].n = 0;
    for (int64_t q = 0; q < nev; ++q) ev_push(&c->reg[0], &ev[q]);
    return relayout(c, c->offx, c->offy);
}

void orc_chain_layout(const orc_chain *c, int32_t *nrx, int32_t *nry, int32_t *period,
                      int32_t *ncolors, double *offx, double *offy)
{
    *nrx = c->nrx; *nry = c->nry; *period = c->period; *ncolors = c->ncolors;
    *offx = c->offx; *offy = c->offy;
}

int64_t orc_chain_count(const orc_chain *c)
{
    int64_t n = 0;
    for (int64_t r = 0; r < c->nreg; ++r) n += c->reg[r].n;
    return n;
}

/* Events in region order, each region's list in id order. */
int64_t orc_chain_events(const orc_chain *c, orc_event *out, int64_t cap)
{
    int64_t n = 0;
    for (int64_t r = 0; r < c->nreg; ++r)
        for (int64_t q = 0; q < c->reg[r].n; ++q) {
            if (n < cap) out[n] = c->reg[r].e[q];
            ++n;
        }
    return n;
}

int64_t orc_chain_overflows(const orc_chain *c) { return c->overflows; }

/* ----------------------------------------------------------- likelihood */

/* Snapshot of the event set at the start of a colour phase, indexed by the
 * stations each event reaches (Algorithm 4 holds the other regions at these
 * values for the whole phase). */
static void build_snapshot(orc_chain *c)
{
    for (int64_t j = 0; j < c->nsta; ++j) c->snap[j].n = 0;
    int32_t reach = c->m.line ? 0 : (int32_t)ceil(c->m.rc / c->m.ds) + 1;
    for (int64_t r = 0; r < c->nreg; ++r) {
        for (int64_t q = 0; q < c->reg[r].n; ++q) {
            const orc_event *e = &c->reg[r].e[q];
            if (c->m.line) {  /* every station detects every event */
                for (int64_t j = 0; j < c->nsta; ++j) ev_push(&c->snap[j], e);
                continue;
            }
            int32_t cx = (int32_t)floor(e->x / c->m.ds), cy = (int32_t)floor(e->y / c->m.ds);
            for (int32_t iy = cy - reach; iy <= cy + reach; ++iy) {
                if (iy < 0 || iy >= c->m.nsy) continue;
                for (int32_t ix = cx - reach; ix <= cx + reach; ++ix) {
                    if (ix < 0 || ix >= c->m.nsx) continue;
                    orc_arrival_t ar;
                    orc_arrival(&c->m, e, ix, iy, &ar);
                    if (ar.in) ev_push(&c->snap[(int64_t)iy * c->m.nsx + ix], e);
                }
            }
        }
    }
}

static double gauss_logpdf(double s, double v)
{
    return -0.5 * (log(2.0 * M_PI) + log(v) + s * s / v);
}

/* Log density of a sample under the model: variance c (variance model, c
 * includes sigma^2) or mean c and variance sigma^2 (mean-template model). */
static double sample_logpdf(const orc_model *m, double s, double c)
{
    if (!m->tmpl) return gauss_logpdf(s, c);
    double r = s - c;
    return -0.5 * (log(2.0 * M_PI) + log(m->sigma * m->sigma) + r * r / (m->sigma * m->sigma));
}

/* Change of log P(s | e) when, in region r, the event at index idx of the
 * region's list is removed (death), replaced by *nw (location, time and
 * magnitude moves), or *nw is added (birth).  Every other region contributes
 * its snapshot events.  Sums run over the union of the samples where the old
 * or the new event has signal; elsewhere nothing changes. */
static double move_delta(orc_chain *c, int32_t r, int32_t type, int64_t idx,
                         const orc_event *nw)
{
    const orc_model *m = &c->m;
    const evlist *own = &c->reg[r];
    const orc_event *old = (type == ORC_BIRTH) ? NULL : &own->e[idx];
    const orc_event *neu = (type == ORC_DEATH) ? NULL : nw;
    int32_t reach = m->line ? 0 : (int32_t)ceil(m->rc / m->ds) + 1;
    int32_t lo_x = m->nsx, hi_x = -1, lo_y = m->nsy, hi_y = -1;
    const orc_event *pts[2] = {old, neu};
    if (m->line) {  /* every station */
        lo_x = 0; hi_x = m->nsx - 1; lo_y = 0; hi_y = 0;
    }
    for (int q = 0; q < 2 && !m->line; ++q) {
        if (!pts[q]) continue;
        int32_t cx = (int32_t)floor(pts[q]->x / m->ds), cy = (int32_t)floor(pts[q]->y / m->ds);
        if (cx - reach < lo_x) lo_x = cx - reach;
        if (cx + reach > hi_x) hi_x = cx + reach;
        if (cy - reach < lo_y) lo_y = cy - reach;
        if (cy + reach > hi_y) hi_y = cy + reach;
    }
    if (lo_x < 0) lo_x = 0;
    if (lo_y < 0) lo_y = 0;
    if (hi_x >= m->nsx) hi_x = m->nsx - 1;
    if (hi_y >= m->nsy) hi_y = m->nsy - 1;

    double delta = 0.0;
    orc_arrival_t *others = NULL;
    int64_t others_cap = 0;
    for (int32_t iy = lo_y; iy <= hi_y; ++iy) {
        for (int32_t ix = lo_x; ix <= hi_x; ++ix) {
            orc_arrival_t ao, an;
            memset(&ao, 0, sizeof ao);
            memset(&an, 0, sizeof an);
            if (old) orc_arrival(m, old, ix, iy, &ao);
            if (neu) orc_arrival(m, neu, ix, iy, &an);
            if (!ao.in && !an.in) continue;
            int64_t lo = m->N, hi = 0;
            if (ao.n1 > ao.n0) { lo = ao.n0; hi = ao.n1; }
            if (an.n1 > an.n0) {
                if (an.n0 < lo) lo = an.n0;
                if (an.n1 > hi) hi = an.n1;
            }
            if (hi <= lo) continue;
            int64_t j = (int64_t)iy * m->nsx + ix;
            /* every other event reaching this station */
            int64_t need = c->snap[j].n + own->n;
            if (need > others_cap) {
                others_cap = need;
                others = (orc_arrival_t *)realloc(others, sizeof(orc_arrival_t) * (size_t)need);
            }
            int64_t no = 0;
            for (int64_t q = 0; q < c->snap[j].n; ++q) {
                if (c->snap[j].e[q].region == r) continue;
                orc_arrival(m, &c->snap[j].e[q], ix, iy, &others[no]);
                if (others[no].in) ++no;
            }
            for (int64_t q = 0; q < own->n; ++q) {
                if (old && q == idx) continue;
                orc_arrival(m, &own->e[q], ix, iy, &others[no]);
                if (others[no].in) ++no;
            }
            for (int64_t n = lo; n < hi; ++n) {
                double sv = trace_at(c, j, n);
                /* noise variance (variance model) plus what every other event adds */
                double base = m->tmpl ? 0.0 : m->sigma * m->sigma;
                for (int64_t q = 0; q < no; ++q) base += orc_arrival_variance(m, &others[q], n);
                double c_old = base + (old ? orc_arrival_variance(m, &ao, n) : 0.0);
                double c_new = base + (neu ? orc_arrival_variance(m, &an, n) : 0.0);
                delta += sample_logpdf(m, sv, c_new) - sample_logpdf(m, sv, c_old);
            }
        }
    }
    free(others);
    return delta;
}

double orc_chain_delta(orc_chain *c, int32_t region, int32_t type, int64_t idx,
                       const orc_event *proposed)
{
    build_snapshot(c);
    return move_delta(c, region, type, idx, proposed);
}

/* Log-likelihood change of replacing events i and k of region r (line
 * model) by ni and nk, evaluated directly like move_delta: at every station,
 * over the samples any of the four windows covers, the variance is summed
 * from scratch over the other events before and after. */
static double pair_delta(orc_chain *c, int32_t r, int64_t i, int64_t k, const orc_event *ni,
                         const orc_event *nk)
{
    const orc_model *m = &c->m;
    const evlist *own = &c->reg[r];
    double delta = 0.0;
    int64_t cap = 0;
    orc_arrival_t *others = NULL;
    for (int32_t ix = 0; ix < m->nsx; ++ix) {
        orc_arrival_t w[4];
        orc_arrival(m, &own->e[i], ix, 0, &w[0]);
        orc_arrival(m, &own->e[k], ix, 0, &w[1]);
        orc_arrival(m, ni, ix, 0, &w[2]);
        orc_arrival(m, nk, ix, 0, &w[3]);
        int64_t lo = m->N, hi = 0;
        for (int q = 0; q < 4; ++q) {
            if (w[q].n1 <= w[q].n0) continue;
            if (w[q].n0 < lo) lo = w[q].n0;
            if (w[q].n1 > hi) hi = w[q].n1;
        }
        if (hi <= lo) continue;
        int64_t need = c->snap[ix].n + own->n;
        if (need > cap) {
            cap = need;
            others = (orc_arrival_t *)realloc(others, sizeof(orc_arrival_t) * (size_t)need);
        }
        int64_t no = 0;
        for (int64_t q = 0; q < c->snap[ix].n; ++q)
            if (c->snap[ix].e[q].region != r) orc_arrival(m, &c->snap[ix].e[q], ix, 0, &others[no++]);
        for (int64_t q = 0; q < own->n; ++q)
            if (q != i && q != k) orc_arrival(m, &own->e[q], ix, 0, &others[no++]);
        for (int64_t n = lo; n < hi; ++n) {
            double sv = trace_at(c, ix, n);
            double base = m->tmpl ? 0.0 : m->sigma * m->sigma;
            for (int64_t q = 0; q < no; ++q) base += orc_arrival_variance(m, &others[q], n);
            double c_old = base + orc_arrival_variance(m, &w[0], n) + orc_arrival_variance(m, &w[1], n);
            double c_new = base + orc_arrival_variance(m, &w[2], n) + orc_arrival_variance(m, &w[3], n);
            delta += sample_logpdf(m, sv, c_new) - sample_logpdf(m, sv, c_old);
        }
    }
    free(others);
    return delta;
}

/* --------------------------------------------------------------- moves */

/* One MH move inside region r (Algorithm 2's step, confined to the region
 * as in Algorithm 4).  Move types (Section 3): birth from the region's prior
 * and death of a uniformly chosen event (Geyer-Moller birth-death for a
 * Poisson process restricted to the region), a Gaussian location offset, a
 * Gaussian time offset and a Gaussian magnitude offset; with latent arrival
 * times (line model) also the arrival-time move and the joint two-event move
 * (joint_proposal).  A proposal that leaves the region, the trace or the
 * magnitude or offset support is rejected without evaluating the
 * likelihood.  log entry: type, status (0 invalid, 1 rejected, 2 accepted),
 * delta, log alpha. */
/* ------------------------------------------------------ learned births */
/* Draw record of 16 for the learned birth proposal: the 8 of
 * orc_move_draws, then [8] mixture uniform, [9] anchor uniform, [10]
 * component uniform (counter blocks 4 and 5), [11..13] three standard
 * normals truncated to [-4, 4]: Box-Muller pairs from blocks 6, 7, ...
 * (cosine then sine), taking the first three of absolute value at most 4;
 * after 16 blocks any still missing are 0.  [14], [15] are 0. */
void orc_move_draws16(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region, uint32_t j,
                      double out[16])
{
    orc_move_draws(seed, chain, sweep, region, j, out);
    uint32_t key[2] = {seed, chain}, w[4];
    uint32_t c4[4] = {sweep, region, j, 4u}, c5[4] = {sweep, region, j, 5u};
    orc_philox4x32_10(c4, key, w);
    out[8] = orc_u01(w[0], w[1]);
    out[9] = orc_u01(w[2], w[3]);
    orc_philox4x32_10(c5, key, w);
    out[10] = orc_u01(w[0], w[1]);
    int got = 0;
    for (uint32_t blk = 6; blk < 22 && got < 3; ++blk) {
        uint32_t cb[4] = {sweep, region, j, blk};
        orc_philox4x32_10(cb, key, w);
        double u1 = orc_u01(w[0], w[1]), u2 = orc_u01(w[2], w[3]);
        double r = sqrt(-2.0 * log(u1));
        double z[2] = {r * cos(2.0 * M_PI * u2), r * sin(2.0 * M_PI * u2)};
        for (int h = 0; h < 2 && got < 3; ++h)
            if (fabs(z[h]) <= 4.0) out[11 + got++] = z[h];
    }
    while (got < 3) out[11 + got++] = 0.0;
    out[14] = 0.0;
    out[15] = 0.0;
}

/* Draw record of 16 for latent arrivals: the 8 of orc_move_draws, then
 * [8..15] eight standard normals truncated to [-4, 4] (the birth's arrival
 * offsets in station order; the joint move's second event takes [8], [9]):
 * Box-Muller pairs from counter blocks 4, 5, ... (cosine then sine), the
 * first eight of absolute value at most 4; after blocks 4 .. 19 any still
 * missing are 0. */
void orc_move_draws_arr(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                        uint32_t j, double out[16])
{
    orc_move_draws(seed, chain, sweep, region, j, out);
    uint32_t key[2] = {seed, chain}, w[4];
    int got = 0;
    for (uint32_t blk = 4; blk < 20 && got < 8; ++blk) {
        uint32_t cb[4] = {sweep, region, j, blk};
        orc_philox4x32_10(cb, key, w);
        double u1 = orc_u01(w[0], w[1]), u2 = orc_u01(w[2], w[3]);
        double r = sqrt(-2.0 * log(u1));
        double z[2] = {r * cos(2.0 * M_PI * u2), r * sin(2.0 * M_PI * u2)};
        for (int h = 0; h < 2 && got < 8; ++h)
            if (fabs(z[h]) <= 4.0) out[8 + got++] = z[h];
    }
    while (got < 8) out[8 + got++] = 0.0;
}

int32_t orc_chain_set_learned(orc_chain *c, const double *table, const double *weights,
                              int32_t n_tau, double p_learned)
{
    free(c->lcum);
    c->lcum = NULL;
    c->ltab = NULL;
    if (!table) return 0;
    if (c->m.line || c->m.tmpl) return -1;  /* anchors: grid stations, variance signals */
    if (n_tau < 1 || !weights || !(p_learned >= 0.0 && p_learned <= 1.0)) return -1;
    c->lcum = (double *)malloc(sizeof(double) * (size_t)(c->nsta * n_tau));
    for (int64_t st = 0; st < c->nsta; ++st) {
        double acc = 0.0;
        for (int32_t i = 0; i < n_tau; ++i) {
            acc = acc + weights[st * n_tau + i];
            c->lcum[st * n_tau + i] = acc;
        }
    }
    c->ltab = table;
    c->lw = weights;
    c->ntau = n_tau;
    c->plearn = p_learned;
    return 0;
}

/* Stations whose position lies in region r, ascending; returns the count. */
static int32_t region_stations(const orc_chain *c, int32_t r, int32_t *out, int32_t cap)
{
    int32_t cnt = 0;
    for (int32_t st = 0; st < (int32_t)c->nsta; ++st) {
        double sx = orc_station_x(&c->m, st % c->m.nsx), sy = orc_station_y(&c->m, st / c->m.nsx);
        if (region_of(c, sx, sy, 0.0) != r) continue;
        if (cnt < cap) out[cnt] = st;
        ++cnt;
    }
    return cnt;
}

/* Total anchor weight W_R of region r (stations ascending, anchors in
 * window order); 0 when no station lies in r. */
static double region_weight(const orc_chain *c, const int32_t *sta, int32_t ns)
{
    double W = 0.0;
    for (int32_t q = 0; q < ns; ++q) W = W + c->lcum[(int64_t)sta[q] * c->ntau + c->ntau - 1];
    return W;
}

/* Density at (x, y, t) of one mixture component truncated at 4 standard
 * deviations per axis (Gaussian of independent axes, each renormalised by
 * the mass erf(4 / sqrt 2) inside the truncation). */
static double component_density(const double *T, double x, double y, double t)
{
    double ux = (x - T[0]) / T[3], uy = (y - T[1]) / T[4], ut = (t - T[2]) / T[5];
    if (!(fabs(ux) <= 4.0 && fabs(uy) <= 4.0 && fabs(ut) <= 4.0)) return 0.0;
    double lz = log(sqrt(2.0 * M_PI) * erf(4.0 / sqrt(2.0)));
    return exp(T[6] - log(T[3]) - log(T[4]) - log(T[5]) - 3.0 * lz -
               0.5 * (ux * ux + uy * uy + ut * ut));
}

/* q_R(x, y, t): the mixture over the anchors of the stations in R, anchor a
 * weighted w_a / W_R, each anchor a mixture of 8 truncated Gaussians. */
static double learned_density(const orc_chain *c, const int32_t *sta, int32_t ns, double W,
                              double x, double y, double t)
{
    double S = 0.0;
    for (int32_t q = 0; q < ns; ++q) {
        for (int32_t i = 0; i < c->ntau; ++i) {
            int64_t a = (int64_t)sta[q] * c->ntau + i;
            double qa = 0.0;
            for (int k = 0; k < 8; ++k) qa += component_density(c->ltab + (a * 8 + k) * 8, x, y, t);
            S += c->lw[a] * qa;
        }
    }
    return S / W;
}

/* The learned branch of a birth: anchor by u_anchor * W_R against the
 * running weight sums (stations ascending, then windows), component by
 * u_comp against the cumulative mixture weights, then the component's mean
 * plus its standard deviations times the truncated normals. */
static void learned_draw(const orc_chain *c, const int32_t *sta, int32_t ns, double W,
                         const double *d, double *x, double *y, double *t)
{
    double target = d[9] * W, acc = 0.0, rem = 0.0;
    int32_t pick = -1;
    for (int32_t q = 0; q < ns; ++q) {
        double Ws = c->lcum[(int64_t)sta[q] * c->ntau + c->ntau - 1];
        double nxt = acc + Ws;
        if (target < nxt) {
            pick = sta[q];
            rem = target - acc;
            break;
        }
        acc = nxt;
    }
    if (pick < 0) {
        pick = sta[ns - 1];
        rem = c->lcum[(int64_t)pick * c->ntau + c->ntau - 1];
    }
    int32_t i = c->ntau - 1;
    for (int32_t q = 0; q < c->ntau; ++q)
        if (rem < c->lcum[(int64_t)pick * c->ntau + q]) { i = q; break; }
    int64_t a = (int64_t)pick * c->ntau + i;
    int k = 7;
    for (int q = 0; q < 8; ++q)
        if (d[10] < c->ltab[(a * 8 + q) * 8 + 7]) { k = q; break; }
    const double *T = c->ltab + (a * 8 + k) * 8;
    *x = T[0] + T[3] * d[11];
    *y = T[1] + T[4] * d[12];
    *t = T[2] + T[5] * d[13];
}

/* log(b / p_R) at (x, y, t) for the mixture b = (1 - p_L) p_R + p_L q_R. */
static double learned_log_ratio(const orc_chain *c, const int32_t *sta, int32_t ns, double W,
                                double pl, double area, double x, double y, double t)
{
    double q = learned_density(c, sta, ns, W, x, y, t);
    return log((1.0 - pl) + pl * q * area * (double)c->m.N);
}

double orc_chain_learned_q(orc_chain *c, int32_t region, double x, double y, double t)
{
    int32_t sta[64];
    int32_t ns = region_stations(c, region, sta, 64);
    if (!c->ltab || ns == 0 || ns > 64) return 0.0;
    return learned_density(c, sta, ns, region_weight(c, sta, ns), x, y, t);
}

int32_t orc_chain_learned_draw(orc_chain *c, int32_t region, const double *d, double *out)
{
    int32_t sta[64];
    int32_t ns = region_stations(c, region, sta, 64);
    if (!c->ltab || ns == 0 || ns > 64) return -1;
    learned_draw(c, sta, ns, region_weight(c, sta, ns), d, out, out + 1, out + 2);
    return 0;
}

/* Latent arrival times are on: the line model with arr_sd > 0. */
static int latent(const orc_chain *c)
{
    return c->m.line && c->m.arr_sd > 0.0 && !c->sp.lattice;
}

/* The joint move of Section 3 (line model with latent arrivals).  Events i
 * and k of region r exchange their arrival times at stations split .. nsx-1.
 * Each then moves to a Gaussian draw (steps sxy and st; normals d[5], d[6]
 * for i, d[8], d[9] for k) around the least-squares fit of its new arrivals
 * (orc_line_fit), and its offsets become whatever places its arrivals
 * exactly where they are.  The reverse move (the same pair and split)
 * exchanges them back and proposes around the fits of the original
 * arrivals.  The move is valid only for two events of equal amplitude (the
 * exchange then leaves every station's set of signals as it was), new
 * locations and onsets inside the domain and the region, offsets within the
 * jitter bound, and new windows that start at the sample of the arrival they
 * take over.  *lx receives the prior and proposal part of log alpha: the
 * change of the offsets' log prior density, summed over both events and all
 * stations, plus log q(reverse) - log q(forward). */
static int joint_proposal(const orc_chain *c, int32_t r, int64_t i, int64_t k, int32_t split,
                          const double *d, orc_event *ni, orc_event *nk, double *lx)
{
    const orc_model *m = &c->m;
    const orc_event *ev[2] = {&c->reg[r].e[i], &c->reg[r].e[k]};
    orc_event *nw[2] = {ni, nk};
    if (ev[0]->m != ev[1]->m) return 0;
    double A[2][8], B[2][8];
    for (int e = 0; e < 2; ++e)
        for (int32_t j = 0; j < m->nsx; ++j) {
            orc_arrival_t ar;
            orc_arrival(m, ev[e], j, 0, &ar);
            A[e][j] = ar.a;
        }
    for (int e = 0; e < 2; ++e)
        for (int32_t j = 0; j < m->nsx; ++j) B[e][j] = j >= split ? A[1 - e][j] : A[e][j];
    const double zx[2] = {d[5], d[8]}, zt[2] = {d[6], d[9]};
    const double bound = ORC_ARR_TRUNC * m->arr_sd, v2 = 2.0 * (m->arr_sd * m->arr_sd);
    for (int e = 0; e < 2; ++e) {
        double fx, ft;
        orc_line_fit(m, B[e], &fx, &ft);
        *nw[e] = *ev[e];
        nw[e]->x = fx + c->sp.sxy * zx[e];
        nw[e]->t = ft + c->sp.st * zt[e];
        if (!(nw[e]->x >= 0.0 && nw[e]->x < c->Lx && nw[e]->t >= 0.0 &&
              nw[e]->t < (double)m->N && region_of(c, nw[e]->x, 0.0, nw[e]->t) == r))
            return 0;
        for (int32_t j = 0; j < 8; ++j) nw[e]->da[j] = 0.0;
        for (int32_t j = 0; j < m->nsx; ++j) {
            double mean = orc_arrival_time(nw[e]->x, 0.0, nw[e]->t, m->sta_x[j], 0.0, m->vel, NULL);
            nw[e]->da[j] = B[e][j] - mean;
            if (fabs(nw[e]->da[j]) > bound) return 0;
        }
        for (int32_t j = 0; j < m->nsx; ++j) {
            orc_arrival_t ar;
            orc_arrival(m, nw[e], j, 0, &ar);
            if (ceil(ar.a) != ceil(B[e][j])) return 0;
        }
    }
    double lp = 0.0, lq = 0.0;
    for (int e = 0; e < 2; ++e)
        for (int32_t j = 0; j < m->nsx; ++j)
            lp += (ev[e]->da[j] * ev[e]->da[j] - nw[e]->da[j] * nw[e]->da[j]) / v2;
    for (int e = 0; e < 2; ++e) {
        double bx, bt;
        orc_line_fit(m, A[e], &bx, &bt);  /* the reverse move's centre */
        double rx = (ev[e]->x - bx) / c->sp.sxy, rt = (ev[e]->t - bt) / c->sp.st;
        lq += 0.5 * (zx[e] * zx[e] + zt[e] * zt[e]) - 0.5 * (rx * rx + rt * rt);
    }
    *lx = lp + lq;
    return 1;
}

static void run_move(orc_chain *c, int32_t r, uint32_t sweep, uint32_t j, const double *d,
                     double lam_r, double area, double *logentry)
{
    const orc_model *m = &c->m;
    const orc_sampler *sp = &c->sp;
    evlist *own = &c->reg[r];
    int64_t n = own->n;
    /* learned births: stations of the region, their weight, the mixing
     * probability (0 for a region without stations) */
    int32_t sta[64], ns = 0;
    double W = 0.0, pl = 0.0;
    if (c->ltab && !sp->lattice) {
        ns = region_stations(c, r, sta, 64);
        if (ns > 64) ns = 0;
        if (ns > 0) {
            W = region_weight(c, sta, ns);
            pl = c->plearn;
        }
    }
    const int lat = latent(c);
    double c1 = sp->pb, c2 = c1 + sp->pd, c3 = c2 + sp->ploc, c4 = c3 + sp->pt;
    double c5 = c4 + sp->pm, c6 = c5 + sp->pa;
    int32_t type = d[0] < c1 ? ORC_BIRTH
                 : d[0] < c2 ? ORC_DEATH
                 : d[0] < c3 ? ORC_LOC
                 : d[0] < c4 ? ORC_TIME
                 : (!lat || d[0] < c5) ? ORC_MAG
                 : d[0] < c6 ? ORC_ARR : ORC_JOINT;
    int valid = 1;
    int64_t idx = -1, idx2 = -1;
    double lx = 0.0;  /* prior and proposal part of log alpha (latent moves) */
    orc_event nw, nw2;
    memset(&nw, 0, sizeof nw);
    memset(&nw2, 0, sizeof nw2);

    if (type == ORC_BIRTH) {
        if (n >= sp->cap) {
            valid = 0;
#pragma omp atomic
            c->overflows++;
        } else if (sp->lattice && m->line) {
            int32_t ix = 0, it = 0;
            int64_t nr = lat_line_region_sites(c, r, -1, &ix, &it);
            int64_t pick = (int64_t)floor(d[1] * (double)nr);
            if (pick >= nr) pick = nr - 1;
            lat_line_region_sites(c, r, pick, &ix, &it);
            lat_coords(c, ix, 0, it, 0, &nw);
            nw.m = m->mmin;
        } else if (sp->lattice) {
            int32_t ix = 0, iy = 0;
            int64_t nr = lat_region_sites(c, r, -1, &ix, &iy);
            int64_t pick = (int64_t)floor(d[1] * (double)nr);
            if (pick >= nr) pick = nr - 1;
            lat_region_sites(c, r, pick, &ix, &iy);
            int32_t it = (int32_t)floor(d[2] * (double)sp->kt);
            int32_t im = (int32_t)floor(d[3] * (double)sp->km);
            if (it >= sp->kt) it = sp->kt - 1;
            if (im >= sp->km) im = sp->km - 1;
            lat_coords(c, ix, iy, it, im, &nw);
        } else if (m->line) {
            /* prior birth on the region: location on [0, xmax), onset in
             * the region's interval, the fixed amplitude */
            double t0, t1;
            region_times(c, r, &t0, &t1);
            nw.x = d[1] * c->Lx;
            nw.y = 0.0;
            nw.t = t0 + d[3] * (t1 - t0);
            nw.m = m->mmin;
            valid = nw.x >= 0.0 && nw.x < c->Lx && nw.t >= 0.0 && nw.t < (double)m->N &&
                    region_of(c, nw.x, nw.y, nw.t) == r;
            if (lat)  /* arrival offsets from their prior: arr_sd times truncated normals */
                for (int32_t q = 0; q < m->nsx; ++q) nw.da[q] = m->arr_sd * d[8 + q];
        } else {
            double x0, x1, y0, y1;
            region_rect(c, r, &x0, &x1, &y0, &y1);
            if (pl > 0.0 && d[8] < pl) {
                learned_draw(c, sta, ns, W, d, &nw.x, &nw.y, &nw.t);
            } else {
                nw.x = x0 + d[1] * (x1 - x0);
                nw.y = y0 + d[2] * (y1 - y0);
                nw.t = d[3] * (double)m->N;
            }
            nw.m = m->mmin + d[4] / m->mrate;
            valid = nw.x >= 0.0 && nw.x < c->Lx && nw.y >= 0.0 && nw.y < c->Ly &&
                    nw.t >= 0.0 && nw.t < (double)m->N && region_of(c, nw.x, nw.y, nw.t) == r;
        }
        nw.id = ((uint64_t)sweep << 32) | ((uint64_t)(uint32_t)r << 12) | (uint64_t)j;
        nw.region = r;
    } else if (type == ORC_JOINT) {
        if (n < 2 || m->nsx < 2) {
            valid = 0;
        } else {
            idx = (int64_t)floor(d[1] * (double)n);
            if (idx >= n) idx = n - 1;
            idx2 = (int64_t)floor(d[2] * (double)(n - 1));
            if (idx2 >= n - 1) idx2 = n - 2;
            if (idx2 >= idx) idx2 += 1;
            int32_t split = 1 + (int32_t)floor(d[3] * (double)(m->nsx - 1));
            if (split >= m->nsx) split = m->nsx - 1;
            valid = joint_proposal(c, r, idx, idx2, split, d, &nw, &nw2, &lx);
        }
    } else {
        if (n == 0) {
            valid = 0;
        } else {
            idx = (int64_t)floor(d[1] * (double)n);
            if (idx >= n) idx = n - 1;
            nw = own->e[idx];
            if (sp->lattice) {
                int32_t ix, iy, it, im;
                lat_index(c, &nw, &ix, &iy, &it, &im);
                if (type == ORC_LOC) {
                    int32_t dir = (int32_t)floor(d[2] * 4.0);
                    if (dir == 0) ix -= 1; else if (dir == 1) ix += 1;
                    else if (dir == 2) iy -= 1; else iy += 1;
                } else if (type == ORC_TIME) {
                    it += d[2] < 0.5 ? -1 : 1;
                } else if (type == ORC_MAG) {
                    im += d[2] < 0.5 ? -1 : 1;
                }
                if (type != ORC_DEATH) {
                    valid = ix >= 0 && ix < sp->kx && iy >= 0 && iy < sp->ky && it >= 0 &&
                            it < sp->kt && im >= 0 && im < sp->km;
                    if (valid) {
                        lat_coords(c, ix, iy, it, im, &nw);
                        valid = region_of(c, nw.x, nw.y, nw.t) == r;
                    }
                }
            } else if (m->line && type == ORC_LOC) {
                /* the location is not a partition axis of the line model */
                nw.x = nw.x + sp->sxy * d[5];
                valid = nw.x >= 0.0 && nw.x < c->Lx;
            } else if (m->line && type == ORC_TIME) {
                nw.t = nw.t + sp->st * d[5];
                valid = nw.t >= 0.0 && nw.t < (double)m->N && region_of(c, nw.x, nw.y, nw.t) == r;
            } else if (m->line && type == ORC_MAG) {
                valid = 0;  /* the line model's amplitude is fixed */
            } else if (type == ORC_ARR) {
                /* one station's arrival moves by a Gaussian step; the prior
                 * density of its offset enters the ratio */
                int32_t js = (int32_t)floor(d[2] * (double)m->nsx);
                if (js >= m->nsx) js = m->nsx - 1;
                double o = nw.da[js];
                nw.da[js] = o + sp->sa * d[5];
                valid = fabs(nw.da[js]) <= ORC_ARR_TRUNC * m->arr_sd;
                lx = (o * o - nw.da[js] * nw.da[js]) / (2.0 * (m->arr_sd * m->arr_sd));
            } else if (type == ORC_LOC) {
                nw.x = nw.x + sp->sxy * d[5];
                nw.y = nw.y + sp->sxy * d[6];
                valid = nw.x >= 0.0 && nw.x < c->Lx && nw.y >= 0.0 && nw.y < c->Ly &&
                        region_of(c, nw.x, nw.y, nw.t) == r;
            } else if (type == ORC_TIME) {
                nw.t = nw.t + sp->st * d[5];
                valid = nw.t >= 0.0 && nw.t < (double)m->N;
            } else if (type == ORC_MAG) {
                nw.m = nw.m + sp->sm * d[5];
                valid = nw.m >= m->mmin;
            }
        }
    }

    double delta = 0.0, la = 0.0;
    int32_t status = 0;
    if (valid) {
        if (!sp->prior_only)
            delta = type == ORC_JOINT ? pair_delta(c, r, idx, idx2, &nw, &nw2)
                                      : move_delta(c, r, type, idx, &nw);
        if (type == ORC_BIRTH) {
            la = delta + log(lam_r) + log(sp->pd) - log((double)(n + 1)) - log(sp->pb);
            if (pl > 0.0) la -= learned_log_ratio(c, sta, ns, W, pl, area, nw.x, nw.y, nw.t);
        } else if (type == ORC_DEATH) {
            la = delta + log((double)n) + log(sp->pb) - log(lam_r) - log(sp->pd);
            if (pl > 0.0) la += learned_log_ratio(c, sta, ns, W, pl, area, nw.x, nw.y, nw.t);
        } else if (type == ORC_MAG && !sp->lattice) {
            la = delta - m->mrate * (nw.m - own->e[idx].m);
        } else if (type == ORC_ARR || type == ORC_JOINT) {
            la = delta + lx;
        } else {
            la = delta;
        }
        if (d[7] < la) {
            status = 2;
            if (type == ORC_BIRTH) ev_push(own, &nw);
            else if (type == ORC_DEATH) ev_remove(own, idx);
            else if (type == ORC_JOINT) { own->e[idx] = nw; own->e[idx2] = nw2; }
            else own->e[idx] = nw;
        } else {
            status = 1;
        }
    }
    if (logentry) {
        logentry[0] = (double)type;
        logentry[1] = (double)status;
        logentry[2] = delta;
        logentry[3] = la;
    }
}

/* The k moves of region r in one phase (Algorithm 4's inner loop). */
static void run_region(orc_chain *c, int64_t r, int64_t sweep, const double *feed,
                       double *log_out)
{
    double x0, x1, y0, y1;
    region_rect(c, (int32_t)r, &x0, &x1, &y0, &y1);
    double area = (x1 - x0) * (y1 - y0);
    if (c->m.line) {  /* the region's share of the onset interval */
        double t0, t1;
        region_times(c, (int32_t)r, &t0, &t1);
        area = t1 - t0;
    }
    if (!(area > 0.0)) return;
    double lam_r;
    if (c->sp.lattice && c->m.line) {
        int32_t a, b;
        int64_t nr = lat_line_region_sites(c, (int32_t)r, -1, &a, &b);
        if (nr == 0) return;
        lam_r = c->m.lambda * (double)nr / ((double)c->sp.kx * (double)c->sp.kt);
    } else if (c->m.line) {
        lam_r = c->m.lambda * area / (double)c->m.N;
    } else if (c->sp.lattice) {
        int32_t a, b;
        int64_t nr = lat_region_sites(c, (int32_t)r, -1, &a, &b);
        if (nr == 0) return;
        lam_r = c->m.lambda * (double)nr / ((double)c->sp.kx * (double)c->sp.ky);
    } else {
        lam_r = c->m.lambda * area / (c->Lx * c->Ly);
    }
    const int64_t stride = c->ltab || latent(c) ? 16 : 8;
    for (int32_t j = 0; j < c->sp.k; ++j) {
        double d[16];
        const double *dp;
        if (feed) {
            dp = feed + ((r * c->sp.k) + j) * stride;
        } else {
            if (latent(c))
                orc_move_draws_arr(c->seed, c->chain, (uint32_t)sweep, (uint32_t)r, (uint32_t)j, d);
            else if (c->ltab)
                orc_move_draws16(c->seed, c->chain, (uint32_t)sweep, (uint32_t)r, (uint32_t)j, d);
            else
                orc_move_draws(c->seed, c->chain, (uint32_t)sweep, (uint32_t)r, (uint32_t)j, d);
            dp = d;
        }
        run_move(c, (int32_t)r, (uint32_t)sweep, (uint32_t)j, dp, lam_r, area,
                 log_out ? log_out + ((r * c->sp.k) + j) * 4 : NULL);
    }
}

/* One colour phase of Algorithm 4: every region of the colour runs k moves;
 * the other regions are held at the phase-start snapshot.  With the naive
 * schedule (Algorithm 3) every region belongs to the phase and each accepts
 * against the posterior of its own events alone (the algorithm's pi(x_m)):
 * the other regions' events are invisible to it.
 * feed (optional): draws [region][k][8] ([16] with learned births or latent
 * arrivals); log
 * (optional): [region][k][4]. */
int32_t orc_chain_phase(orc_chain *c, int64_t sweep, int32_t color, const double *feed,
                        double *log_out)
{
    if (c->sp.schedule == ORC_SCHED_NAIVE) {
        for (int64_t j = 0; j < c->nsta; ++j) c->snap[j].n = 0;
    } else {
        build_snapshot(c);
    }
    /* The regions of one colour are conditionally independent given the
     * snapshot of the others (Section 4.1), so they may run on several host
     * threads, as the paper's own implementation ran them on several cores;
     * each writes only its own event list and its own log entries, and the
     * result does not depend on the thread count. */
#pragma omp parallel for schedule(dynamic, 1) num_threads(c->threads > 1 ? c->threads : 1) if (c->threads > 1)
    for (int64_t r = 0; r < c->nreg; ++r) {
        if (c->sp.schedule == ORC_SCHED_CHROMATIC && c->color[r] != color) continue;
        run_region(c, r, sweep, feed, log_out);
    }
    return 0;
}

void orc_chain_set_threads(orc_chain *c, int32_t threads)
{
    c->threads = threads > 1 ? threads : 1;
}

/* One full sweep: lay out the partition (a fresh offset when dynamic), then
 * the colours in ascending order. */
int32_t orc_chain_sweep(orc_chain *c, int64_t sweep, const double *feed, double *log_out)
{
    int32_t rc = orc_chain_begin_sweep(c, sweep);
    if (rc != 0) return rc;
    int32_t nphase = c->sp.schedule == ORC_SCHED_NAIVE ? 1 : c->ncolors;
    for (int32_t col = 0; col < nphase; ++col) {
        rc = orc_chain_phase(c, sweep, col, feed, log_out);
        if (rc != 0) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------ enumeration */

int64_t orc_lattice_nsites(const orc_model *m, const orc_sampler *sp)
{
    (void)m;
    return (int64_t)sp->kx * sp->ky * sp->kt * sp->km;
}

void orc_lattice_site(const orc_model *m, const orc_sampler *sp, int64_t site, orc_event *out)
{
    int32_t im = (int32_t)(site % sp->km);
    int64_t rest = site / sp->km;
    int32_t it = (int32_t)(rest % sp->kt);
    rest /= sp->kt;
    int32_t iy = (int32_t)(rest % sp->ky);
    int32_t ix = (int32_t)(rest / sp->ky);
    double Lx = m->line ? m->xmax : (double)m->nsx * m->ds, Ly = (double)m->nsy * m->ds;
    memset(out, 0, sizeof *out);
    out->x = ((double)ix + 0.5) * (Lx / (double)sp->kx);
    out->y = m->line ? 0.0 : ((double)iy + 0.5) * (Ly / (double)sp->ky);
    out->t = ((double)it + 0.5) * ((double)m->N / (double)sp->kt);
    out->m = m->line ? m->mmin : m->mmin + ((double)im + 0.5) * sp->hm;
}

/* Every multiset of at most nmax sites, with its unnormalised log posterior:
 * the lattice Poisson prior (independent Poisson(lambda / S) counts on the S
 * sites, so a multiset with counts k_s has weight prod mu^k_s / k_s!) times
 * the signal likelihood.  sites_out: [count][nmax], ascending, padded -1. */
int64_t orc_enumerate(const orc_model *m, const orc_sampler *sp, const double *s,
                      int32_t nmax, int32_t *sites_out, double *logw_out, int64_t cap)
{
    int64_t S = orc_lattice_nsites(m, sp);
    double mu = m->lambda / (double)S;
    int64_t count = 0;
    int32_t *cur = (int32_t *)calloc((size_t)(nmax > 0 ? nmax : 1), sizeof(int32_t));
    orc_event *ev = (orc_event *)calloc((size_t)(nmax > 0 ? nmax : 1), sizeof(orc_event));
    for (int32_t n = 0; n <= nmax; ++n) {
        for (int32_t q = 0; q < n; ++q) cur[q] = 0;
        for (;;) {
            double lw = -m->lambda + (double)n * log(mu);
            int32_t run = 1;
            for (int32_t q = 0; q < n; ++q) {
                if (q > 0 && cur[q] == cur[q - 1]) {
                    ++run;
                    lw -= log((double)run);
                } else {
                    run = 1;
                }
                orc_lattice_site(m, sp, cur[q], &ev[q]);
            }
            if (!sp->prior_only) lw += orc_loglik(m, s, ev, n);
            if (count < cap) {
                for (int32_t q = 0; q < nmax; ++q)
                    sites_out[count * nmax + q] = q < n ? cur[q] : -1;
                logw_out[count] = lw;
            }
            ++count;
            /* next non-decreasing sequence */
            int32_t pos = n - 1;
            while (pos >= 0 && cur[pos] == S - 1) --pos;
            if (pos < 0) break;
            cur[pos]++;
            for (int32_t q = pos + 1; q < n; ++q) cur[q] = cur[pos];
        }
    }
    free(cur);
    free(ev);
    return count;
}
