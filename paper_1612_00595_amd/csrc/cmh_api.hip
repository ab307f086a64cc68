// cmh_api.hip -- the C-ABI of the chromatic MH library (include/chromh.h):
// argument validation, partition and colouring, workspace layout inside the
// caller's device buffer, eager and graph-replayed sweeps, host transfers,
// the workgroup-size autotuner and the forward simulator's staging.
#include "chromh.h"
#include "cmh_common.hpp"
#include "cmh_kernels.hpp"
#include "cmh_mdn.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using cmh::Events;
using cmh::Geo;

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(CMH_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// ------------------------------------------------------------- validation
// The line model: 1..8 stations on a line, events on [0, x_max); atten,
// env_decay, r_c and ds are not used.
int32_t check_line_model(const cmh_model *m)
{
    if (m->nsy != 1 || m->nsx < 1 || m->nsx > 8)
        return fail(CMH_EINVAL, "line model: nsy = 1 and 1..8 stations");
    if (!(m->x_max > 0.0) || !std::isfinite(m->x_max))
        return fail(CMH_EINVAL, "line model: x_max must be positive");
    for (int j = 0; j < m->nsx; ++j)
        if (!std::isfinite(m->station_x[j]))
            return fail(CMH_EINVAL, "line model: station positions must be finite");
    if (m->n_samples < 1) return fail(CMH_EINVAL, "n_samples must be positive");
    if ((long long)m->nsx * m->n_samples >= (1LL << 31))
        return fail(CMH_EINVAL, "stations x samples must stay below 2^31");
    if (!(m->sigma > 0.0)) return fail(CMH_EINVAL, "sigma must be positive");
    if (!(m->velocity > 0.0)) return fail(CMH_EINVAL, "velocity must be positive");
    if (m->t_s < 1 || m->t_s > cmh::kMaxTs) return fail(CMH_EINVAL, "t_s must be in 1..128");
    if (!(m->lambda > 0.0)) return fail(CMH_EINVAL, "lambda must be positive");
    if (!std::isfinite(m->mag_min)) return fail(CMH_EINVAL, "mag_min must be finite");
    if (!(m->arrival_sd >= 0.0) || !std::isfinite(m->arrival_sd))
        return fail(CMH_EINVAL, "arrival_sd must be finite and non-negative");
    return CMH_OK;
}

int32_t check_model(const cmh_model *m)
{
    if (!m) return fail(CMH_EINVAL, "model is NULL");
    if (m->line != 0 && m->line != 1) return fail(CMH_EINVAL, "line must be 0 or 1");
    if (m->template_mean != 0 && m->template_mean != 1)
        return fail(CMH_EINVAL, "template_mean must be 0 or 1");
    if (m->line) return check_line_model(m);
    if (m->arrival_sd != 0.0)
        return fail(CMH_EINVAL, "latent arrival times (arrival_sd > 0) need the line model");
    if (m->nsx < 1 || m->nsy < 1) return fail(CMH_EINVAL, "station grid must be at least 1x1");
    if ((long long)m->nsx * m->nsy > (1LL << 22)) return fail(CMH_EINVAL, "too many stations");
    if (!(m->ds > 0.0)) return fail(CMH_EINVAL, "ds must be positive");
    if (m->n_samples < 1) return fail(CMH_EINVAL, "n_samples must be positive");
    if ((long long)m->nsx * m->nsy * m->n_samples >= (1LL << 31))
        return fail(CMH_EINVAL, "stations x samples must stay below 2^31");
    if (!(m->sigma > 0.0)) return fail(CMH_EINVAL, "sigma must be positive");
    if (!(m->atten > 0.0)) return fail(CMH_EINVAL, "atten must be positive");
    if (!(m->velocity > 0.0)) return fail(CMH_EINVAL, "velocity must be positive");
    if (!(m->env_decay > 0.0)) return fail(CMH_EINVAL, "env_decay must be positive");
    if (m->t_s < 1 || m->t_s > cmh::kMaxTs) return fail(CMH_EINVAL, "t_s must be in 1..128");
    if (!(m->r_c > 0.0) || !(m->r_c < m->ds))
        return fail(CMH_EINVAL, "r_c must satisfy 0 < r_c < ds");
    if (!(m->lambda > 0.0)) return fail(CMH_EINVAL, "lambda must be positive");
    if (!(m->mag_rate > 0.0)) return fail(CMH_EINVAL, "mag_rate must be positive");
    if (!std::isfinite(m->mag_min)) return fail(CMH_EINVAL, "mag_min must be finite");
    return CMH_OK;
}

int32_t check_grid(const cmh_model *m, int32_t gx, int32_t gy)
{
    if (m->line) {
        if (gx < 1 || gy != 0)
            return fail(CMH_EINVAL, "line model: grid_x >= 1 onset regions and grid_y = 0");
        if (gx + 1 >= (1 << 20)) return fail(CMH_EINVAL, "at most 2^20 regions");
        return CMH_OK;
    }
    if (gx < 1 || gy < 1) return fail(CMH_EINVAL, "grid must be at least 1x1");
    if ((long long)(gx + 1) * (gy + 1) >= (1LL << 20))
        return fail(CMH_EINVAL, "at most 2^20 regions");
    return CMH_OK;
}

// Rectangle distance from a station to the closure of a region.
double rect_distance(double px, double py, double x0, double x1, double y0, double y1)
{
    const double dx = px < x0 ? x0 - px : (px > x1 ? px - x1 : 0.0);
    const double dy = py < y0 ? y0 - py : (py > y1 ? py - y1 : 0.0);
    return std::sqrt(dx * dx + dy * dy);
}

// Number of (station, same-coloured region pair) conflicts for period p.
long long colour_conflicts(const cmh_model *m, int gx, int gy, double offx, double offy, int p)
{
    const double Lx = (double)m->nsx * m->ds, Ly = (double)m->nsy * m->ds;
    const double wx = Lx / (double)gx, wy = Ly / (double)gy;
    std::vector<double> xlo(gx + 1), xhi(gx + 1), ylo(gy + 1), yhi(gy + 1);
    for (int i = 0; i <= gx; ++i) cmh::region_span(offx, wx, Lx, i, &xlo[i], &xhi[i]);
    for (int k = 0; k <= gy; ++k) cmh::region_span(offy, wy, Ly, k, &ylo[k], &yhi[k]);
    long long bad = 0;
    std::vector<int> hit;
    for (int sy = 0; sy < m->nsy; ++sy) {
        const double py = cmh::station_pos(sy, m->ds);
        for (int sx = 0; sx < m->nsx; ++sx) {
            const double px = cmh::station_pos(sx, m->ds);
            hit.clear();
            for (int k = 0; k <= gy; ++k) {
                if (!(yhi[k] > ylo[k])) continue;
                if (py < ylo[k] - m->r_c || py > yhi[k] + m->r_c) continue;
                for (int i = 0; i <= gx; ++i) {
                    if (!(xhi[i] > xlo[i])) continue;
                    if (rect_distance(px, py, xlo[i], xhi[i], ylo[k], yhi[k]) < m->r_c)
                        hit.push_back((i % p) + p * (k % p));
                }
            }
            std::sort(hit.begin(), hit.end());
            for (size_t q = 1; q < hit.size(); ++q) bad += hit[q] == hit[q - 1];
        }
    }
    return bad;
}

// Line model: nearest and farthest distance from station j to [0, x_max].
void line_reach(const cmh_model *m, int j, double *dmin, double *dmax)
{
    const double s = m->station_x[j];
    *dmin = s < 0.0 ? -s : (s > m->x_max ? s - m->x_max : 0.0);
    *dmax = std::max(std::fabs(s), std::fabs(s - m->x_max));
}

// Line model: the longest travel time from the line to a station.
double line_tmax(const cmh_model *m)
{
    double t = 0.0;
    for (int j = 0; j < m->nsx; ++j) {
        double lo, hi;
        line_reach(m, j, &lo, &hi);
        t = std::max(t, hi / m->velocity);
    }
    return t;
}

// Line model conflicts for period p: onset region [t0, t1) can touch
// samples [ceil(t0 + dmin / v - e), ceil(t1 + dmax / v + e) + t_s) of
// station j, e the bound of the arrival-time jitter (0 without latent
// arrivals); two regions of one colour must not share a sample of any
// station.
long long line_conflicts(const cmh_model *m, int gx, double offt, int p)
{
    const double N = (double)m->n_samples, w = N / (double)gx;
    const double e = cmh::kArrTrunc * m->arrival_sd;
    std::vector<double> lo(gx + 1), hi(gx + 1);
    for (int i = 0; i <= gx; ++i) cmh::region_span(offt, w, N, i, &lo[i], &hi[i]);
    long long bad = 0;
    for (int j = 0; j < m->nsx; ++j) {
        double dmin, dmax;
        line_reach(m, j, &dmin, &dmax);
        std::vector<double> a(gx + 1), b(gx + 1);
        for (int i = 0; i <= gx; ++i) {
            a[i] = std::ceil(lo[i] + dmin / m->velocity - e);
            b[i] = std::ceil(hi[i] + dmax / m->velocity + e) + m->t_s;
        }
        for (int i = 0; i <= gx; ++i) {
            if (!(hi[i] > lo[i])) continue;
            for (int q = i + p; q <= gx; q += p)
                if (hi[q] > lo[q] && a[q] < b[i] && a[i] < b[q]) ++bad;
        }
    }
    return bad;
}

int32_t choose_line_period(const cmh_model *m, int gx, double offt, int dynamic, int requested,
                           int *period, bool unchecked)
{
    if (unchecked && requested > 0) {  // debug: the owner check is to catch the breach
        *period = requested;
        return CMH_OK;
    }
    const double w = (double)m->n_samples / (double)gx;
    int p;
    if (dynamic) {
        // p - 1 region lengths cover tau_max, t_s and twice the jitter bound
        p = (int)std::ceil((line_tmax(m) + (double)m->t_s + 2.0 * cmh::kArrTrunc * m->arrival_sd)
                           / w) + 1;
        if (requested > 0) {
            if (requested < p)
                return fail(CMH_ECOLOR, "requested period too small for shifted partitions");
            p = requested;
        }
        if (line_conflicts(m, gx, offt, p) != 0)
            return fail(CMH_ECOLOR, "colouring check failed");
    } else if (requested > 0) {
        p = requested;
        if (line_conflicts(m, gx, offt, p) != 0)
            return fail(CMH_ECOLOR, "requested period gives dependent regions of one colour");
    } else {
        for (p = 1; p <= gx + 1; ++p)
            if (line_conflicts(m, gx, offt, p) == 0) break;
        if (p > gx + 1) return fail(CMH_ECOLOR, "no colouring separates the regions");
    }
    *period = p;
    return CMH_OK;
}

int32_t choose_period(const cmh_model *m, int gx, int gy, double offx, double offy, int dynamic,
                      int requested, int *period, bool unchecked = false)
{
    if (m->line) return choose_line_period(m, gx, offx, dynamic, requested, period, unchecked);
    if (unchecked && requested > 0) {  // debug: the owner check is to catch the breach
        *period = requested;
        return CMH_OK;
    }
    const double Lx = (double)m->nsx * m->ds, Ly = (double)m->nsy * m->ds;
    const double w = std::min(Lx / (double)gx, Ly / (double)gy);
    int p;
    if (dynamic) {
        p = (int)std::ceil(2.0 * m->r_c / w) + 1;
        if (requested > 0) {
            if (requested < p)
                return fail(CMH_ECOLOR, "requested period too small for shifted partitions");
            p = requested;
        }
        if (colour_conflicts(m, gx, gy, offx, offy, p) != 0)
            return fail(CMH_ECOLOR, "colouring check failed");
    } else if (requested > 0) {
        p = requested;
        if (colour_conflicts(m, gx, gy, offx, offy, p) != 0)
            return fail(CMH_ECOLOR, "requested period gives dependent regions of one colour");
    } else {
        const int pmax = std::max(gx, gy) + 1;
        for (p = 1; p <= pmax; ++p)
            if (colour_conflicts(m, gx, gy, offx, offy, p) == 0) break;
        if (p > pmax) return fail(CMH_ECOLOR, "no colouring separates the regions");
    }
    *period = p;
    return CMH_OK;
}

int32_t make_geo(const cmh_model *m, const cmh_sampler *s, Geo *g)
{
    int32_t rc = check_model(m);
    if (rc) return rc;
    if (!s) return fail(CMH_EINVAL, "sampler is NULL");
    rc = check_grid(m, s->grid_x, s->grid_y);
    if (rc) return rc;
    if (s->moves_per_region < 1 || s->moves_per_region > 4095)
        return fail(CMH_EINVAL, "moves_per_region must be in 1..4095");
    if (s->region_capacity < 1 || s->region_capacity > cmh::kMaxCap)
        return fail(CMH_EINVAL, "region_capacity must be in 1..64");
    const double ps[7] = {s->p_birth, s->p_death, s->p_loc, s->p_time, s->p_mag, s->p_arrival,
                          s->p_joint};
    double sum = 0.0;
    for (double v : ps) {
        if (!(v >= 0.0)) return fail(CMH_EINVAL, "move probabilities must be non-negative");
        sum += v;
    }
    if (!(s->p_birth > 0.0) || !(s->p_death > 0.0))
        return fail(CMH_EINVAL, "birth and death probabilities must be positive");
    if (std::fabs(sum - 1.0) > 1e-9) return fail(CMH_EINVAL, "move probabilities must sum to 1");
    if (!(s->step_xy >= 0.0) || !(s->step_t >= 0.0) || !(s->step_m >= 0.0))
        return fail(CMH_EINVAL, "step sizes must be non-negative");
    if (s->block != 0 && s->block != 64 && s->block != 128 && s->block != 256 && s->block != 512 &&
        !cmh::is_spec_block(s->block) && s->block != cmh::kPersist)
        return fail(CMH_EINVAL, "block must be 0, 64, 128, 256, 512, CMH_BLOCK_SPEC + 128, "
                                "256 or 512, or CMH_BLOCK_PERSIST");
    if (s->dynamic != 0 && s->dynamic != 1) return fail(CMH_EINVAL, "dynamic must be 0 or 1");
    if (s->refresh_every < 0) return fail(CMH_EINVAL, "refresh_every must be non-negative");
    // A persistent launch on a static partition (whose edge regions have no
    // area and end their item at once) did not finish on the device once;
    // the cause is not known, so that combination is refused.
    if (s->block == cmh::kPersist && s->dynamic != 1)
        return fail(CMH_EINVAL, "the persistent form runs dynamic partitions only");
    if (s->prior_only != 0 && s->prior_only != 1)
        return fail(CMH_EINVAL, "prior_only must be 0 or 1");
    if (s->schedule != 0 && s->schedule != 1) return fail(CMH_EINVAL, "schedule must be 0 or 1");
    const bool latent = m->line && m->arrival_sd > 0.0;
    if (!latent && (s->p_arrival != 0.0 || s->p_joint != 0.0))
        return fail(CMH_EINVAL, "arrival-time and joint moves need latent arrivals");
    if (latent) {
        if (s->p_arrival > 0.0 && !(s->step_arrival > 0.0 && std::isfinite(s->step_arrival)))
            return fail(CMH_EINVAL, "step_arrival must be positive");
        if (s->p_joint > 0.0 && !(s->step_xy > 0.0 && s->step_t > 0.0))
            return fail(CMH_EINVAL, "the joint move needs positive step_xy and step_t");
        if (s->block != 0 && s->block != 64 && s->block != 256)
            return fail(CMH_EINVAL, "latent arrivals run the block-64 or block-256 form");
        if (s->schedule != 0)
            return fail(CMH_EINVAL, "latent arrivals run the chromatic schedule");
    }
    if (s->debug & ~7) return fail(CMH_EINVAL, "debug takes bits 0, 1 and 2 only");
    if ((s->debug & 1) && s->schedule != 0)
        return fail(CMH_EINVAL, "the owner check needs the chromatic schedule");
    if ((s->debug & 2) && !(s->debug & 1 && s->period > 0))
        return fail(CMH_EINVAL, "an unchecked period needs the owner check and a period");
    if (s->schedule == 1) {
        if ((long long)m->nsx * m->nsy * m->n_samples > cmh::kNaiveMax)
            return fail(CMH_EINVAL, "the naive schedule needs stations x samples <= 2048");
        if (s->block != 0 && s->block != 64)
            return fail(CMH_EINVAL, "the naive schedule runs the block-64 form");
    }
    int p = 0;
    rc = choose_period(m, s->grid_x, s->grid_y, 0.0, 0.0, s->dynamic, s->period, &p,
                       (s->debug & 2) != 0);
    if (rc) return rc;

    std::memset(g, 0, sizeof *g);
    g->nsx = m->nsx; g->nsy = m->nsy; g->nsta = m->nsx * m->nsy; g->ts = m->t_s;
    g->N = (int)m->n_samples;
    g->gx = s->grid_x; g->gy = s->grid_y; g->nrx = s->grid_x + 1; g->nry = s->grid_y + 1;
    g->R = g->nrx * g->nry;
    g->period = p; g->ncolors = p * p; g->dynamic = s->dynamic;
    g->k = s->moves_per_region; g->cap = s->region_capacity; g->prior_only = s->prior_only;
    g->ds = m->ds; g->sigma2 = m->sigma * m->sigma; g->atten = m->atten; g->vel = m->velocity;
    g->decay = m->env_decay; g->rc = m->r_c; g->lambda = m->lambda; g->mmin = m->mag_min;
    g->mrate = m->mag_rate;
    g->Lx = (double)m->nsx * m->ds; g->Ly = (double)m->nsy * m->ds;
    g->wx = g->Lx / (double)s->grid_x; g->wy = g->Ly / (double)s->grid_y;
    g->pb = s->p_birth; g->pd = s->p_death; g->ploc = s->p_loc; g->pt = s->p_time;
    g->pm = s->p_mag;
    g->sxy = s->step_xy; g->st = s->step_t; g->sm = s->step_m;
    g->c1 = g->pb;
    g->c2 = g->c1 + g->pd;
    g->c3 = g->c2 + g->ploc;
    g->c4 = g->c3 + g->pt;
    g->att2 = 2.0 / g->atten;
    g->dec2 = 2.0 / g->decay;
    g->tmpl = m->template_mean;
    if (g->tmpl) {  // waveform amplitudes: A = m exp(-d / atten), phi = exp(-tau / decay)
        g->att2 = 1.0 / g->atten;
        g->dec2 = 1.0 / g->decay;
    }
    if (m->line) {
        // regions of onset time; every station detects, no attenuation, a
        // constant signal variance over t_s samples
        g->ncolors = p;
        g->nry = 1;
        g->R = g->nrx;
        g->Lx = m->x_max;
        g->Ly = 1.0;
        g->wx = (double)m->n_samples / (double)s->grid_x;
        g->wy = 0.0;
        g->rc = INFINITY;
        g->atten = INFINITY;
        g->decay = INFINITY;
        g->att2 = 0.0;
        g->dec2 = 0.0;
        g->line = 1;
        g->tmax = line_tmax(m);
        for (int j = 0; j < m->nsx; ++j) g->sx[j] = m->station_x[j];
    }
    if (s->schedule == 1) {  // Algorithm 3: every region in the one phase
        g->naive = 1;
        g->ncolors = 1;
    }
    g->c5 = g->c4 + g->pm;
    if (latent) {  // Section 3's arrival density, truncated at kArrTrunc sd
        g->latent = 1;
        g->arr_sd = m->arrival_sd;
        g->arr_e = cmh::kArrTrunc * m->arrival_sd;
        g->arr_2v = 2.0 * (m->arrival_sd * m->arrival_sd);
        g->pa = s->p_arrival;
        g->pj = s->p_joint;
        g->sa = s->step_arrival;
        g->c6 = g->c5 + g->pa;
    }
    g->owner = s->debug & 1;
    g->inv_ds = 1.0 / m->ds;
    return CMH_OK;
}

// Workspace carving.  When st is NULL only the size is computed.
struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        const size_t o = align_up(off);
        off = o + count * sizeof(T);
        return base ? (T *)(base + o) : nullptr;
    }
};

void carve_events(Carver &c, const Geo &g, int chains, Events *ev)
{
    const size_t slots = (size_t)chains * g.R * g.cap;
    ev->x = c.take<double>(slots);
    ev->y = c.take<double>(slots);
    ev->t = c.take<double>(slots);
    ev->m = c.take<double>(slots);
    ev->id = c.take<unsigned long long>(slots);
    ev->cnt = c.take<int>((size_t)chains * g.R);
    ev->off = c.take<double>((size_t)chains * 2);
    ev->da = g.latent ? c.take<double>(slots * 8) : nullptr;  // latent arrival offsets
}

}  // namespace

struct cmh_state {
    Geo g;
    int chains = 0;
    int f64 = 0;
    const void *trace = nullptr;
    double *E = nullptr;
    Events ev[2];
    Events snap;
    int cur = 0;
    long long *sweep_ctr = nullptr;
    int *err = nullptr;
    unsigned long long *stats = nullptr;
    unsigned long long *stats_snap = nullptr;
    double *partials = nullptr;
    double *llout = nullptr;
    double *draws = nullptr;  // [chain][region][move][8] for the current sweep
    double *draws2 = nullptr; // latent arrivals: draws 8..15, same layout
    unsigned long long *owner = nullptr;  // debug owner check: [chain][nsta][N] tags
    int owner_any = 0;  // some slot runs the owner check (its kernel instantiations)
    int block = 256;
    const double *feed = nullptr;
    long long feed_first = 0, feed_n = 0;
    int feed_width = 8;
    double *logp = nullptr;
    long long log_first = 0, log_n = 0;
    int refresh_every = 0;   // exact refresh after every this many sweeps (0: never)
    double *lp_rec = nullptr;  // log-probability records [sweeps][slot][2] (NULL: off)
    long long lp_first = 0, lp_n = 0;
    int *pq_ctr = nullptr;       // persistent form: ticket, then per slot completed items
    unsigned *pq_wait = nullptr; // persistent form: per item (colour order) its wait target
    long long spin_limit = 1LL << 22;
    unsigned long long *stamps = nullptr;  // sweep-kernel time stamps (NULL: off)
    long long stamp_first = 0, stamp_n = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_block = 0;
    hipStream_t cap_stream = nullptr;
    int poisoned = 0;
    int batch = 0;  // slots are different instances (cmh_batch_init)
    cmh::Learned learned{};  // tab == nullptr: plain births
    int n_learned = 0;       // batches: instances with learned births
    // work items: one slot per chain, items (slot << 16) | region
    int nslots = 0;
    int refresh_max = 0;  // the most (station, tile) blocks of a slot (naive refresh)
    int naive_elems = 0;  // naive schedule: the largest stations x samples of a slot
    std::vector<cmh::Slot> slots_h;
    cmh::Slot *slots_d = nullptr;
    unsigned *items_all = nullptr;   // every region of every slot
    int n_all = 0;
    unsigned *items_col = nullptr;   // grouped by colour
    std::vector<int> col_off, col_n;
    double *rec = nullptr;   // sample recording (NULL: off)
    long long rec_first = 0, rec_n = 0;
    int rec_max = 0;
};

namespace {

size_t carve_state(const Geo &g, int chains, char *base, cmh_state *st)
{
    Carver c{base};
    double *E = c.take<double>((size_t)chains * g.nsta * (size_t)g.N);
    Events ev0, ev1, snap;
    carve_events(c, g, chains, &ev0);
    carve_events(c, g, chains, &ev1);
    carve_events(c, g, chains, &snap);
    long long *sweep = c.take<long long>(1);
    int *err = c.take<int>(1);
    unsigned long long *stats = c.take<unsigned long long>((size_t)chains * cmh::kStats);
    unsigned long long *stats_snap = c.take<unsigned long long>((size_t)chains * cmh::kStats);
    double *partials = c.take<double>((size_t)chains * cmh::refresh_blocks(g));
    double *llout = c.take<double>((size_t)chains * 2);
    double *draws = c.take<double>((size_t)chains * g.R * (size_t)g.k * 8);
    double *draws2 = g.latent ? c.take<double>((size_t)chains * g.R * (size_t)g.k * 8) : nullptr;
    cmh::Slot *slots = c.take<cmh::Slot>((size_t)chains);
    unsigned *items_all = c.take<unsigned>((size_t)chains * g.R);
    unsigned *items_col = c.take<unsigned>((size_t)chains * g.R);
    int *pq_ctr = c.take<int>((size_t)chains + 1);
    unsigned *pq_wait = c.take<unsigned>((size_t)chains * g.R);
    unsigned long long *owner =
        g.owner ? c.take<unsigned long long>((size_t)chains * g.nsta * (size_t)g.N) : nullptr;
    if (st) {
        st->owner = owner;
        st->slots_d = slots;
        st->items_all = items_all;
        st->items_col = items_col;
        st->pq_ctr = pq_ctr;
        st->pq_wait = pq_wait;
        st->draws = draws;
        st->draws2 = draws2;
        st->E = E;
        st->ev[0] = ev0;
        st->ev[1] = ev1;
        st->snap = snap;
        st->sweep_ctr = sweep;
        st->err = err;
        st->stats = stats;
        st->stats_snap = stats_snap;
        st->partials = partials;
        st->llout = llout;
    }
    return align_up(c.off);
}

// Slot c of a single-instance state: chain c's share of the chain-major
// arrays.
cmh::Slot chain_slot(const cmh_state *st, int c)
{
    const Geo &g = st->g;
    cmh::Slot sl{};
    sl.g = g;
    sl.chain = (uint32_t)c;
    sl.trace = st->trace;
    sl.E = st->E + (size_t)c * g.nsta * (size_t)g.N;
    for (int b = 0; b < 2; ++b) {
        const Events &e = st->ev[b];
        const size_t o = (size_t)c * g.R * g.cap;
        sl.ev[b] = Events{e.x + o, e.y + o, e.t + o, e.m + o, e.id + o, e.cnt + (size_t)c * g.R,
                          e.off + 2 * (size_t)c, e.da ? e.da + 8 * o : nullptr};
    }
    sl.draws = st->draws + (size_t)c * g.R * g.k * 8;
    sl.draws2 = st->draws2 ? st->draws2 + (size_t)c * g.R * g.k * 8 : nullptr;
    sl.stats = st->stats + (size_t)c * cmh::kStats;
    sl.owner = st->owner ? st->owner + (size_t)c * g.nsta * (size_t)g.N : nullptr;
    sl.L = st->learned;
    if (sl.L.tab) {
        sl.L.birth = st->learned.birth + (size_t)c * g.R * g.k * 4;
        sl.L.raw = st->learned.raw + (size_t)c * g.R * g.k * 8;
    }
    return sl;
}

// Persistent form: for each item of the colour-ordered list, how many items
// of its own slot lie in lower colours (the slot's colour counter must reach
// that count before the item may start).
std::vector<unsigned> wait_targets(const std::vector<unsigned> &col, const std::vector<int> &off,
                                   const std::vector<int> &cnt, int nslots)
{
    std::vector<unsigned> wait(col.size(), 0u), done(nslots, 0u);
    for (size_t c = 0; c < off.size(); ++c) {
        for (int q = off[c]; q < off[c] + cnt[c]; ++q) wait[q] = done[col[q] >> 16];
        for (int q = off[c]; q < off[c] + cnt[c]; ++q) ++done[col[q] >> 16];
    }
    return wait;
}

// Host slot table and work items of a single-instance state, uploaded to
// its workspace (synchronously: the host vectors are temporaries).
int32_t upload_slots(cmh_state *st)
{
    const Geo &g = st->g;
    st->nslots = st->chains;
    st->slots_h.resize(st->chains);
    for (int c = 0; c < st->chains; ++c) st->slots_h[c] = chain_slot(st, c);
    std::vector<unsigned> all, col;
    st->col_off.assign(g.ncolors, 0);
    st->col_n.assign(g.ncolors, 0);
    for (int c = 0; c < st->chains; ++c)
        for (int r = 0; r < g.R; ++r) all.push_back(((unsigned)c << 16) | (unsigned)r);
    const int p = g.period;
    for (int color = 0; color < g.ncolors; ++color) {
        st->col_off[color] = (int)col.size();
        for (int c = 0; c < st->chains; ++c)
            for (int r = 0; r < g.R; ++r) {
                const int i = r % g.nrx, k = r / g.nrx;
                const int cr = g.naive ? 0 : (i % p) + p * (k % p);
                if (cr == color) col.push_back(((unsigned)c << 16) | (unsigned)r);
            }
        st->col_n[color] = (int)col.size() - st->col_off[color];
    }
    st->n_all = (int)all.size();
    st->refresh_max = cmh::refresh_blocks(g);
    st->naive_elems = g.nsta * g.N;
    HIPCHK(hipMemcpy(st->slots_d, st->slots_h.data(), sizeof(cmh::Slot) * st->slots_h.size(),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(st->items_all, all.data(), sizeof(unsigned) * all.size(),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(st->items_col, col.data(), sizeof(unsigned) * col.size(),
                     hipMemcpyHostToDevice));
    const std::vector<unsigned> wait = wait_targets(col, st->col_off, st->col_n, st->nslots);
    HIPCHK(hipMemcpy(st->pq_wait, wait.data(), sizeof(unsigned) * wait.size(),
                     hipMemcpyHostToDevice));
    return CMH_OK;
}

int32_t check_single(cmh_state *st)
{
    return st->batch ? fail(CMH_EINVAL, "not available for a batch of instances") : CMH_OK;
}

int32_t check_state(cmh_state *st)
{
    if (!st) return fail(CMH_EINVAL, "state is NULL");
    if (st->poisoned) return fail(CMH_ESTATE, "state poisoned by an earlier device error");
    return CMH_OK;
}

// Synchronises the device and turns a latched device flag into a status.
int32_t sync_and_check(cmh_state *st)
{
    HIPCHK(hipDeviceSynchronize());
    int flags = 0;
    HIPCHK(hipMemcpy(&flags, st->err, sizeof(int), hipMemcpyDeviceToHost));
    if (flags) {
        st->poisoned = 1;
        if (flags & cmh::kFlagRace)
            return fail(CMH_ERACE, "two regions of one colour shared a sample in one phase");
        if (flags & cmh::kFlagCap) return fail(CMH_ECAP, "a region exceeded its event capacity");
        if (flags & cmh::kFlagNan) return fail(CMH_ENAN, "NaN or Inf in a likelihood change");
        if (flags & cmh::kFlagSta)
            return fail(CMH_ESTATE, "a region holds more stations than learned births allow");
        if (flags & cmh::kFlagWait)
            return fail(CMH_ESTATE, "a persistent-form wait for a colour counter timed out");
        return fail(CMH_ESTATE, "footprint or tile capacity exceeded");
    }
    return CMH_OK;
}

hipError_t copy_events(const Events &dst, const Events &src, const Geo &g, int chains,
                       hipStream_t s)
{
    const size_t slots = (size_t)chains * g.R * g.cap;
    hipError_t e;
    if ((e = hipMemcpyAsync(dst.x, src.x, slots * 8, hipMemcpyDeviceToDevice, s))) return e;
    if ((e = hipMemcpyAsync(dst.y, src.y, slots * 8, hipMemcpyDeviceToDevice, s))) return e;
    if ((e = hipMemcpyAsync(dst.t, src.t, slots * 8, hipMemcpyDeviceToDevice, s))) return e;
    if ((e = hipMemcpyAsync(dst.m, src.m, slots * 8, hipMemcpyDeviceToDevice, s))) return e;
    if ((e = hipMemcpyAsync(dst.id, src.id, slots * 8, hipMemcpyDeviceToDevice, s))) return e;
    if (src.da && (e = hipMemcpyAsync(dst.da, src.da, slots * 64, hipMemcpyDeviceToDevice, s)))
        return e;
    if ((e = hipMemcpyAsync(dst.cnt, src.cnt, (size_t)chains * g.R * 4, hipMemcpyDeviceToDevice,
                            s)))
        return e;
    return hipMemcpyAsync(dst.off, src.off, (size_t)chains * 16, hipMemcpyDeviceToDevice, s);
}

// Enqueue the start of a sweep: the re-layout of a shifted partition and
// the draw records of every move of the sweep.
hipError_t enqueue_sweep_start(cmh_state *st, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (st->g.dynamic) {
        e = cmh::launch_rebin(st->slots_d, st->items_all, st->n_all, st->cur, st->sweep_ctr,
                              st->err, s);
        if (e) return e;
        st->cur ^= 1;
    }
    return cmh::launch_sweep_draws(st->slots_d, st->items_all, st->n_all, st->g.k, st->cur,
                                   st->sweep_ctr, st->feed, st->feed_first, st->feed_width,
                                   st->learned.tab != nullptr || st->n_learned > 0, st->err, s);
}

// Enqueue one colour phase (colour 0 first starts the sweep), reading the
// sweep index from the device counter.
hipError_t enqueue_phase(cmh_state *st, int color, bool start, hipStream_t s)
{
    if (start) {
        hipError_t e = enqueue_sweep_start(st, s);
        if (e) return e;
    }
    const cmh::StampArg sa{st->stamps, st->stamp_first, st->stamp_n, color, st->g.ncolors};
    hipError_t e = hipSuccess;
    if (st->block == cmh::kPersist) {
        // every colour in one launch at colour 0; later colours launch nothing
        if (color == 0) {
            const cmh::PersistArg pq{st->pq_ctr, (unsigned *)(st->pq_ctr + 1), st->pq_wait,
                                     st->spin_limit};
            int total = 0;
            for (int c = 0; c < st->g.ncolors; ++c) total += st->col_n[c];
            e = cmh::launch_sweep_persist(st->slots_d, st->items_col, total, st->cur, st->f64,
                                          st->sweep_ctr, st->logp, st->log_first, st->log_n,
                                          st->err, st->owner_any, sa, pq, st->nslots, s);
        }
    } else {
        e = cmh::launch_sweep(st->slots_d, st->items_col + st->col_off[color], st->col_n[color],
                              st->cur, st->f64, st->sweep_ctr, st->logp, st->log_first,
                              st->log_n, st->err, st->block, st->g.naive ? st->naive_elems : 0,
                              st->g.latent, st->owner_any, sa, s);
    }
    if (!e && st->g.naive)  // the merged events' variance after the single naive phase
        e = cmh::launch_refresh_slots(st->slots_d, st->nslots, st->refresh_max, st->cur,
                                      st->f64, st->err, s);
    if (e || st->rec == nullptr || color != st->g.ncolors - 1) return e;
    return cmh::launch_record(st->slots_d, st->nslots, st->cur, st->sweep_ctr, st->rec,
                              st->rec_first, st->rec_n, st->rec_max, s);
}

// The scheduled exact refresh after sweep `sweep` (every refresh_every
// sweeps): every slot's event variance recomputed from its events, removing
// the rounding the incremental updates accumulate; within the log-probability
// record's range also each slot's log-likelihood and log prior.
hipError_t enqueue_refresh(cmh_state *st, long long sweep, hipStream_t s)
{
    if (st->refresh_every <= 0 || (sweep + 1) % st->refresh_every != 0) return hipSuccess;
    double *out = nullptr;
    if (st->lp_rec && sweep >= st->lp_first && sweep < st->lp_first + st->lp_n)
        out = st->lp_rec + (sweep - st->lp_first) * 2LL * st->nslots;
    return cmh::launch_refresh_slots(st->slots_d, st->nslots, st->refresh_max, st->cur, st->f64,
                                     st->err, s, 1, st->partials, out);
}

void drop_graphs(cmh_state *st)
{
    for (auto &gr : st->graph) {
        if (gr) (void)hipGraphExecDestroy(gr);
        gr = nullptr;
    }
    st->graph_block = 0;
}

// One graph per layout parity: [re-layout], every colour, advance counter.
int32_t build_graphs(cmh_state *st)
{
    drop_graphs(st);
    const int saved = st->cur;
    const int nparity = st->g.dynamic ? 2 : 1;
    for (int par = 0; par < nparity; ++par) {
        st->cur = par;
        HIPCHK(hipStreamBeginCapture(st->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int c = 0; c < st->g.ncolors && e == hipSuccess; ++c)
            e = enqueue_phase(st, c, c == 0, st->cap_stream);
        if (e == hipSuccess) e = cmh::advance_sweep(st->sweep_ctr, st->cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(st->cap_stream, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            st->cur = saved;
            drop_graphs(st);
            return fail(CMH_EHIP, std::string("graph capture failed: ") +
                                      hipGetErrorString(e != hipSuccess ? e : e2));
        }
        e = hipGraphInstantiate(&st->graph[par], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            st->cur = saved;
            drop_graphs(st);
            return fail(CMH_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
    }
    st->cur = saved;
    st->graph_block = st->block;
    return CMH_OK;
}

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;

// Tuning-cache key: every constant of the problem that changes the kernel
// form or the work per move (sizes, partition, move mix, likelihood form,
// footprint geometry, prior occupancy, latent arrivals, learned births), not
// the seed.
std::string tune_key(const cmh::Geo &g, int chains, int f64, bool learned)
{
    std::string k;
    auto put = [&k](const void *p, size_t n) { k.append((const char *)p, n); };
    const int iv[] = {g.nsx, g.nsy, g.N, g.ts, g.gx, g.gy, g.period, g.dynamic, g.k, g.cap,
                      g.prior_only, g.line, g.tmpl, g.naive, g.latent, g.owner, chains, f64,
                      learned ? 1 : 0};
    const double dv[] = {g.ds, g.sigma2, g.atten, g.vel, g.decay, g.rc, g.lambda, g.mmin,
                         g.mrate, g.pb, g.pd, g.ploc, g.pt, g.pm, g.sxy, g.st, g.sm,
                         g.arr_sd, g.pa, g.pj, g.sa, g.Lx, g.Ly};
    put(iv, sizeof iv);
    put(dv, sizeof dv);
    if (g.line) put(g.sx, sizeof g.sx);
    return k;
}

}  // namespace

extern "C" {

const char *cmh_last_error(void) { return g_err.c_str(); }

int32_t cmh_partition_and_color(const cmh_model *model, int32_t grid_x, int32_t grid_y,
                                double off_x, double off_y, int32_t dynamic, int32_t *n_reg_x,
                                int32_t *n_reg_y, int32_t *period, int32_t *n_colors,
                                int32_t *color_of_region)
{
    int32_t rc = check_model(model);
    if (rc) return rc;
    rc = check_grid(model, grid_x, grid_y);
    if (rc) return rc;
    if (!n_reg_x || !n_reg_y || !period || !n_colors) return fail(CMH_EINVAL, "NULL output");
    if (model->line) {
        const double w = (double)model->n_samples / grid_x;
        if (!(off_x >= 0.0 && off_x < w) || off_y != 0.0)
            return fail(CMH_EINVAL, "line model: offset in [0, w), off_y = 0");
        int p = 0;
        rc = choose_line_period(model, grid_x, off_x, dynamic ? 1 : 0, 0, &p, false);
        if (rc) return rc;
        *n_reg_x = grid_x + 1;
        *n_reg_y = 1;
        *period = p;
        *n_colors = p;
        if (color_of_region)
            for (int i = 0; i <= grid_x; ++i) color_of_region[i] = i % p;
        return CMH_OK;
    }
    const double Lx = (double)model->nsx * model->ds, Ly = (double)model->nsy * model->ds;
    const double wx = Lx / grid_x, wy = Ly / grid_y;
    if (!(off_x >= 0.0 && off_x < wx && off_y >= 0.0 && off_y < wy))
        return fail(CMH_EINVAL, "offsets must lie in [0, w)");
    int p = 0;
    rc = choose_period(model, grid_x, grid_y, off_x, off_y, dynamic ? 1 : 0, 0, &p);
    if (rc) return rc;
    *n_reg_x = grid_x + 1;
    *n_reg_y = grid_y + 1;
    *period = p;
    *n_colors = p * p;
    if (color_of_region)
        for (int k = 0; k <= grid_y; ++k)
            for (int i = 0; i <= grid_x; ++i)
                color_of_region[k * (grid_x + 1) + i] = (i % p) + p * (k % p);
    return CMH_OK;
}

int32_t cmh_state_bytes(const cmh_model *model, const cmh_sampler *sampler, int32_t n_chains,
                        size_t *bytes)
{
    Geo g;
    int32_t rc = make_geo(model, sampler, &g);
    if (rc) return rc;
    if (n_chains < 1 || n_chains > 65535) return fail(CMH_EINVAL, "n_chains must be in 1..65535");
    if (!bytes) return fail(CMH_EINVAL, "bytes is NULL");
    *bytes = carve_state(g, n_chains, nullptr, nullptr);
    return CMH_OK;
}

int32_t cmh_init_state(const cmh_model *model, const cmh_sampler *sampler, const void *trace_dev,
                       int32_t trace_dtype, int32_t n_chains, uint32_t seed, void *workspace_dev,
                       size_t workspace_bytes, void *hip_stream, cmh_state **out)
{
    if (!out) return fail(CMH_EINVAL, "out is NULL");
    *out = nullptr;
    Geo g;
    int32_t rc = make_geo(model, sampler, &g);
    if (rc) return rc;
    if (n_chains < 1 || n_chains > 65535) return fail(CMH_EINVAL, "n_chains must be in 1..65535");
    if (g.R > 65535) return fail(CMH_EINVAL, "at most 65535 regions");
    if (trace_dtype != CMH_F32 && trace_dtype != CMH_F64)
        return fail(CMH_EINVAL, "trace_dtype must be CMH_F32 or CMH_F64");
    if (!trace_dev) return fail(CMH_EINVAL, "trace_dev is NULL");
    if (!workspace_dev) return fail(CMH_EINVAL, "workspace_dev is NULL");
    const size_t need = carve_state(g, n_chains, nullptr, nullptr);
    if (workspace_bytes < need)
        return fail(CMH_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    g.seed = seed;

    cmh_state *st = new cmh_state();
    st->g = g;
    st->chains = n_chains;
    st->f64 = trace_dtype == CMH_F64;
    st->trace = trace_dev;
    st->block = g.naive ? 64 : (sampler->block ? sampler->block : 256);
    st->refresh_every = sampler->refresh_every;
    st->spin_limit = (sampler->debug & 4) ? 0 : st->spin_limit;
    carve_state(g, n_chains, (char *)workspace_dev, st);
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipStreamCreateWithFlags(&st->cap_stream, hipStreamNonBlocking);
    const long long nE = (long long)n_chains * g.nsta * (long long)g.N;
    const long long nR = (long long)n_chains * g.R;
    // the empty world's state: no event variance, or under templates the
    // residual, the trace itself
    if (!e)
        e = g.tmpl ? cmh::residual_init(st->E, trace_dev, st->f64,
                                        (long long)g.nsta * (long long)g.N, nE, s)
                   : cmh::fill_f64(st->E, nE, 0.0, s);
    for (int b = 0; b < 2 && !e; ++b) {
        e = cmh::fill_i32(st->ev[b].cnt, nR, 0, s);
        if (!e) e = cmh::fill_f64(st->ev[b].off, 2LL * n_chains, 0.0, s);
    }
    if (!e) e = cmh::fill_i32(st->err, 1, 0, s);
    if (!e) e = cmh::fill_u64(st->stats, (long long)cmh::kStats * n_chains, s);
    if (!e && st->owner) e = cmh::fill_u64(st->owner, nE, s);
    st->owner_any = st->owner != nullptr;
    if (!e) e = cmh::set_sweep(st->sweep_ctr, 0, s);
    if (e) {
        if (st->cap_stream) (void)hipStreamDestroy(st->cap_stream);
        delete st;
        return fail(CMH_EHIP, std::string("init: ") + hipGetErrorString(e));
    }
    rc = upload_slots(st);
    if (rc) {
        if (st->cap_stream) (void)hipStreamDestroy(st->cap_stream);
        delete st;
        return rc;
    }
    *out = st;
    return CMH_OK;
}

int32_t cmh_sweep_color(cmh_state *st, int64_t sweep, int32_t color, void *hip_stream)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (color < 0 || color >= st->g.ncolors) return fail(CMH_EINVAL, "colour out of range");
    if (sweep < 0 || sweep >= (1LL << 32)) return fail(CMH_EINVAL, "sweep out of range");
    if (st->feed && (sweep < st->feed_first || sweep >= st->feed_first + st->feed_n))
        return fail(CMH_EINVAL, "sweep outside the attached feed");
    if (st->feed && st->feed_width != (st->learned.tab || st->g.latent ? 16 : 8))
        return fail(CMH_EINVAL,
                    "feed records must be 16 wide with learned births or latent arrivals, else 8");
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(cmh::set_sweep(st->sweep_ctr, sweep, s));
    HIPCHK(enqueue_phase(st, color, color == 0, s));
    if (color == st->g.ncolors - 1) HIPCHK(enqueue_refresh(st, sweep, s));
    return CMH_OK;
}

int32_t cmh_run_sweeps(cmh_state *st, int64_t first_sweep, int64_t n_sweeps, void *hip_stream)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (n_sweeps < 0 || first_sweep < 0 || first_sweep + n_sweeps > (1LL << 32))
        return fail(CMH_EINVAL, "sweep range out of bounds");
    if (st->feed || st->logp) {
        for (int64_t s = first_sweep; s < first_sweep + n_sweeps; ++s)
            for (int c = 0; c < st->g.ncolors; ++c) {
                rc = cmh_sweep_color(st, s, c, hip_stream);
                if (rc) return rc;
            }
        return CMH_OK;
    }
    if (n_sweeps == 0) return CMH_OK;
    if (st->graph_block != st->block || !st->graph[0]) {
        rc = build_graphs(st);
        if (rc) return rc;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(cmh::set_sweep(st->sweep_ctr, first_sweep, s));
    for (int64_t q = 0; q < n_sweeps; ++q) {
        HIPCHK(hipGraphLaunch(st->graph[st->g.dynamic ? st->cur : 0], s));
        if (st->g.dynamic) st->cur ^= 1;
        HIPCHK(enqueue_refresh(st, first_sweep + q, s));
    }
    return CMH_OK;
}

// ------------------------------------------------------ checkpoint / resume
namespace {
struct CkptHead {
    char magic[8];
    uint32_t version, nslots;
    int32_t cur, pad;
};
struct CkptSlot {
    int32_t nsta, N, R, cap, latent, pad;
};
constexpr char kCkptMagic[8] = {'C', 'M', 'H', 'C', 'K', 'P', 'T', '1'};

// Bytes of one slot's part: its current event table (x, y, t, m, id, counts,
// offsets, arrival offsets when latent), its event variance and counters.
size_t ckpt_slot_bytes(const Geo &g)
{
    const size_t n = (size_t)g.R * g.cap;
    return sizeof(CkptSlot) + n * (5 * 8 + (g.latent ? 64 : 0)) + (size_t)g.R * 4 + 16 +
           (size_t)g.nsta * g.N * 8 + (size_t)cmh::kStats * 8;
}

size_t ckpt_bytes(const cmh_state *st)
{
    size_t b = sizeof(CkptHead);
    for (const cmh::Slot &sl : st->slots_h) b += ckpt_slot_bytes(sl.g);
    return b;
}

// Copies between the slot's device arrays and a host record (to_host: device
// to host).
int32_t ckpt_copy(const cmh::Slot &sl, int cur, char *rec, bool to_host)
{
    const Geo &g = sl.g;
    const Events &ev = sl.ev[cur];
    const size_t n = (size_t)g.R * g.cap;
    struct Part {
        void *dev;
        size_t bytes;
    };
    const Part parts[] = {{ev.x, n * 8}, {ev.y, n * 8}, {ev.t, n * 8}, {ev.m, n * 8},
                          {ev.id, n * 8}, {ev.cnt, (size_t)g.R * 4}, {ev.off, 16},
                          {ev.da, g.latent ? n * 64 : 0}, {sl.E, (size_t)g.nsta * g.N * 8},
                          {sl.stats, (size_t)cmh::kStats * 8}};
    char *p = rec;
    for (const Part &q : parts) {
        if (q.bytes == 0) continue;
        if (to_host) HIPCHK(hipMemcpy(p, q.dev, q.bytes, hipMemcpyDeviceToHost));
        else HIPCHK(hipMemcpy(q.dev, p, q.bytes, hipMemcpyHostToDevice));
        p += q.bytes;
    }
    return CMH_OK;
}

// Checks one slot's record (the part after its CkptSlot header) against what
// a state of this shape can hold, on the host, before anything reaches the
// device: counts in [0, cap]; offsets in [0, w) per axis when the offset is
// redrawn (0 otherwise); every live event inside the model's support, binned
// to its region under the saved offsets, ids strictly increasing within a
// region, arrival offsets within the jitter bound; the per-sample array
// finite (and non-negative when it is a variance).  Returns the reason for
// a refusal, or nullptr.
const char *ckpt_validate(const Geo &g, const char *rec)
{
    const size_t n = (size_t)g.R * g.cap;
    std::vector<double> x(n), y(n), t(n), m(n), da(g.latent ? n * 8 : 0);
    std::vector<unsigned long long> id(n);
    std::vector<int> cnt(g.R);
    double off[2];
    const char *p = rec;
    auto take = [&p](void *dst, size_t bytes) {
        if (bytes) std::memcpy(dst, p, bytes);
        p += bytes;
    };
    take(x.data(), n * 8);
    take(y.data(), n * 8);
    take(t.data(), n * 8);
    take(m.data(), n * 8);
    take(id.data(), n * 8);
    take(cnt.data(), (size_t)g.R * 4);
    take(off, 16);
    take(da.data(), da.size() * 8);
    for (int a = 0; a < 2; ++a) {
        const double w = a == 0 ? g.wx : g.wy;
        const bool ok = (g.dynamic && w > 0.0) ? (off[a] >= 0.0 && off[a] < w) : off[a] == 0.0;
        if (!ok) return "partition offset outside [0, region width)";
    }
    for (int r = 0; r < g.R; ++r) {
        if (cnt[r] < 0 || cnt[r] > g.cap) return "region event count outside [0, capacity]";
        for (int s = 0; s < cnt[r]; ++s) {
            const size_t a = (size_t)r * g.cap + s;
            if (!(x[a] >= 0.0 && x[a] < g.Lx && y[a] >= 0.0 && y[a] < g.Ly && t[a] >= 0.0 &&
                  t[a] < (double)g.N && m[a] >= g.mmin && std::isfinite(m[a])))
                return "event outside the model's support";
            if (cmh::event_region(g, off[0], off[1], x[a], y[a], t[a]) != r)
                return "event stored in a region that does not hold it";
            if (s > 0 && !(id[a - 1] < id[a])) return "event ids not increasing within a region";
            if (g.latent)
                for (int c = 0; c < g.nsx; ++c)
                    if (!(std::fabs(da[a * 8 + c]) <= g.arr_e))
                        return "arrival offset beyond the jitter bound";
        }
    }
    const size_t ns = (size_t)g.nsta * g.N;
    for (size_t i = 0; i < ns; ++i) {
        double e;
        std::memcpy(&e, p + i * 8, 8);
        if (!std::isfinite(e) || (!g.tmpl && e < 0.0))
            return g.tmpl ? "residual not finite" : "event variance negative or not finite";
    }
    return nullptr;
}
}  // namespace

int32_t cmh_checkpoint_bytes(cmh_state *st, size_t *bytes)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (!bytes) return fail(CMH_EINVAL, "bytes is NULL");
    *bytes = ckpt_bytes(st);
    return CMH_OK;
}

int32_t cmh_save(cmh_state *st, void *host_buf, size_t bytes)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (!host_buf) return fail(CMH_EINVAL, "host_buf is NULL");
    if (bytes < ckpt_bytes(st)) return fail(CMH_EINVAL, "checkpoint buffer too small");
    rc = sync_and_check(st);
    if (rc) return rc;
    char *p = (char *)host_buf;
    CkptHead h{};
    std::memcpy(h.magic, kCkptMagic, 8);
    h.version = 1;
    h.nslots = (uint32_t)st->slots_h.size();
    h.cur = st->cur;
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    for (const cmh::Slot &sl : st->slots_h) {
        const CkptSlot cs{sl.g.nsta, sl.g.N, sl.g.R, sl.g.cap, sl.g.latent, 0};
        std::memcpy(p, &cs, sizeof cs);
        rc = ckpt_copy(sl, st->cur, p + sizeof cs, true);
        if (rc) return rc;
        p += ckpt_slot_bytes(sl.g);
    }
    return CMH_OK;
}

int32_t cmh_load(cmh_state *st, const void *host_buf, size_t bytes)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (!host_buf) return fail(CMH_EINVAL, "host_buf is NULL");
    if (bytes < ckpt_bytes(st)) return fail(CMH_EINVAL, "checkpoint buffer too small");
    const char *p = (const char *)host_buf;
    CkptHead h;
    std::memcpy(&h, p, sizeof h);
    if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != 1)
        return fail(CMH_EINVAL, "not a checkpoint of this library");
    if (h.nslots != st->slots_h.size() || (h.cur != 0 && h.cur != 1))
        return fail(CMH_EINVAL, "checkpoint of a state with a different number of chains");
    const char *q = p + sizeof h;
    for (const cmh::Slot &sl : st->slots_h) {  // validate every slot before writing any
        CkptSlot cs;
        std::memcpy(&cs, q, sizeof cs);
        if (cs.nsta != sl.g.nsta || cs.N != sl.g.N || cs.R != sl.g.R || cs.cap != sl.g.cap ||
            cs.latent != sl.g.latent)
            return fail(CMH_EINVAL, "checkpoint of a state with a different shape");
        if (const char *why = ckpt_validate(sl.g, q + sizeof cs))
            return fail(CMH_EINVAL, std::string("corrupt checkpoint: ") + why);
        q += ckpt_slot_bytes(sl.g);
    }
    rc = sync_and_check(st);
    if (rc) return rc;
    q = p + sizeof h;
    for (const cmh::Slot &sl : st->slots_h) {
        rc = ckpt_copy(sl, h.cur, const_cast<char *>(q) + sizeof(CkptSlot), false);
        if (rc) return rc;
        q += ckpt_slot_bytes(sl.g);
    }
    for (const cmh::Slot &sl : st->slots_h)  // the resumed run starts with no owner tags
        if (sl.owner) HIPCHK(cmh::fill_u64(sl.owner, (long long)sl.g.nsta * sl.g.N, nullptr));
    HIPCHK(hipDeviceSynchronize());
    st->cur = h.cur;
    return CMH_OK;
}

int32_t cmh_read_events(cmh_state *st, int32_t chain, cmh_event *out_host, int64_t cap,
                        int64_t *n_out)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (chain < 0 || chain >= st->chains) return fail(CMH_EINVAL, "chain out of range");
    if (!n_out) return fail(CMH_EINVAL, "n_out is NULL");
    rc = sync_and_check(st);
    if (rc) return rc;
    // the chain's (or batch instance's) slot-local table
    const Geo &g = st->slots_h[chain].g;
    const Events &ev = st->slots_h[chain].ev[st->cur];
    const size_t slots = (size_t)g.R * g.cap, o = 0;
    std::vector<int> cnt(g.R);
    std::vector<double> x(slots), y(slots), t(slots), m(slots);
    std::vector<unsigned long long> id(slots);
    HIPCHK(hipMemcpy(cnt.data(), ev.cnt, g.R * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(x.data(), ev.x + o, slots * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(y.data(), ev.y + o, slots * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(t.data(), ev.t + o, slots * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(m.data(), ev.m + o, slots * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(id.data(), ev.id + o, slots * 8, hipMemcpyDeviceToHost));
    std::vector<double> da(ev.da ? slots * 8 : 0);
    if (ev.da) HIPCHK(hipMemcpy(da.data(), ev.da, slots * 64, hipMemcpyDeviceToHost));
    int64_t n = 0;
    for (int r = 0; r < g.R; ++r) n += cnt[r];
    *n_out = n;
    if (n > cap) return fail(CMH_EINVAL, "output capacity too small");
    if (n > 0 && !out_host) return fail(CMH_EINVAL, "out_host is NULL");
    int64_t q = 0;
    for (int r = 0; r < g.R; ++r)
        for (int s = 0; s < cnt[r]; ++s) {
            const size_t a = (size_t)r * g.cap + s;
            cmh_event &e = out_host[q++];
            e.x = x[a]; e.y = y[a]; e.t = t[a]; e.m = m[a]; e.id = id[a];
            e.region = r; e._pad = 0;
            for (int c = 0; c < 8; ++c) e.da[c] = ev.da ? da[a * 8 + c] : 0.0;
        }
    return CMH_OK;
}

int32_t cmh_write_events(cmh_state *st, int32_t chain, const cmh_event *ev_host, int64_t n)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (chain < 0 || chain >= st->chains) return fail(CMH_EINVAL, "chain out of range");
    if (n < 0 || (n > 0 && !ev_host)) return fail(CMH_EINVAL, "bad event array");
    rc = sync_and_check(st);
    if (rc) return rc;
    // the chain's (the instance's, in a batch) own view: its constants and
    // its slot-local event table
    const cmh::Slot &sl = st->slots_h[chain];
    const Geo &g = sl.g;
    const Events &ev = sl.ev[st->cur];
    double off[2];
    HIPCHK(hipMemcpy(off, ev.off, 16, hipMemcpyDeviceToHost));
    std::vector<std::vector<cmh_event>> reg(g.R);
    for (int64_t q = 0; q < n; ++q) {
        const cmh_event &e = ev_host[q];
        if (!(e.x >= 0.0 && e.x < g.Lx && e.y >= 0.0 && e.y < g.Ly && e.t >= 0.0 &&
              e.t < (double)g.N && e.m >= g.mmin))
            return fail(CMH_EINVAL, "event outside the model's support");
        if (g.latent)
            for (int c = 0; c < g.nsx; ++c)
                if (!(std::fabs(e.da[c]) <= g.arr_e))
                    return fail(CMH_EINVAL, "arrival offset beyond the jitter bound");
        reg[cmh::event_region(g, off[0], off[1], e.x, e.y, e.t)].push_back(e);
    }
    const size_t slots = (size_t)g.R * g.cap, o = 0;
    std::vector<double> da(g.latent ? slots * 8 : 0, 0.0);
    std::vector<int> cnt(g.R, 0);
    std::vector<double> x(slots, 0), y(slots, 0), t(slots, 0), m(slots, 0);
    std::vector<unsigned long long> id(slots, 0);
    for (int r = 0; r < g.R; ++r) {
        auto &L = reg[r];
        if ((int)L.size() > g.cap) return fail(CMH_ECAP, "a region exceeds its capacity");
        std::sort(L.begin(), L.end(),
                  [](const cmh_event &a, const cmh_event &b) { return a.id < b.id; });
        cnt[r] = (int)L.size();
        for (size_t s = 0; s < L.size(); ++s) {
            const size_t a = (size_t)r * g.cap + s;
            x[a] = L[s].x; y[a] = L[s].y; t[a] = L[s].t; m[a] = L[s].m; id[a] = L[s].id;
            if (g.latent)
                for (int c = 0; c < g.nsx; ++c) da[a * 8 + c] = L[s].da[c];
        }
    }
    if (g.latent) HIPCHK(hipMemcpy(ev.da + 8 * o, da.data(), slots * 64, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ev.cnt, cnt.data(), g.R * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ev.x + o, x.data(), slots * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ev.y + o, y.data(), slots * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ev.t + o, t.data(), slots * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ev.m + o, m.data(), slots * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ev.id + o, id.data(), slots * 8, hipMemcpyHostToDevice));
    // the variance of this chain alone, recomputed from the new events
    HIPCHK(cmh::launch_refresh_slots(st->slots_d + chain, 1, cmh::refresh_blocks(g), st->cur,
                                     st->f64, st->err, nullptr));
    return sync_and_check(st);
}

int32_t cmh_set_feed(cmh_state *st, const double *feed_dev, int64_t first_sweep, int64_t n_sweeps,
                     int32_t width)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if ((rc = check_single(st))) return rc;
    if (feed_dev && (first_sweep < 0 || n_sweeps < 1))
        return fail(CMH_EINVAL, "feed needs first_sweep >= 0 and n_sweeps >= 1");
    if (feed_dev && width != 8 && width != 16) return fail(CMH_EINVAL, "width must be 8 or 16");
    st->feed_width = width;
    st->feed = feed_dev;
    st->feed_first = feed_dev ? first_sweep : 0;
    st->feed_n = feed_dev ? n_sweeps : 0;
    return CMH_OK;
}

int32_t cmh_set_record(cmh_state *st, double *rec_dev, int64_t first_sweep, int64_t n_sweeps,
                       int32_t max_events)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (rec_dev && (first_sweep < 0 || n_sweeps < 1 || max_events < 0))
        return fail(CMH_EINVAL, "record needs first_sweep >= 0, n_sweeps >= 1, max_events >= 0");
    drop_graphs(st);
    st->rec = rec_dev;
    st->rec_first = rec_dev ? first_sweep : 0;
    st->rec_n = rec_dev ? n_sweeps : 0;
    st->rec_max = rec_dev ? max_events : 0;
    return CMH_OK;
}

int32_t cmh_set_log(cmh_state *st, double *log_dev, int64_t first_sweep, int64_t n_sweeps)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if ((rc = check_single(st))) return rc;
    if (log_dev && (first_sweep < 0 || n_sweeps < 1))
        return fail(CMH_EINVAL, "log needs first_sweep >= 0 and n_sweeps >= 1");
    st->logp = log_dev;
    st->log_first = log_dev ? first_sweep : 0;
    st->log_n = log_dev ? n_sweeps : 0;
    return CMH_OK;
}

int32_t cmh_log_posterior(cmh_state *st, int32_t write_variance, double *out_host,
                          void *hip_stream)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (!out_host) return fail(CMH_EINVAL, "out_host is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(cmh::launch_refresh_slots(st->slots_d, st->nslots, st->refresh_max, st->cur, st->f64,
                                     st->err, s, write_variance ? 1 : 0, st->partials,
                                     st->llout));
    rc = sync_and_check(st);
    if (rc) return rc;
    std::vector<double> v((size_t)st->nslots * 2);
    HIPCHK(hipMemcpy(v.data(), st->llout, v.size() * 8, hipMemcpyDeviceToHost));
    for (int q = 0; q < st->nslots; ++q) {
        out_host[3 * q] = v[2 * q];
        out_host[3 * q + 1] = v[2 * q + 1];
        out_host[3 * q + 2] = v[2 * q] + v[2 * q + 1];
    }
    return CMH_OK;
}

int32_t cmh_set_logprob(cmh_state *st, double *rec_dev, int64_t first_sweep, int64_t n_sweeps)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (rec_dev && (first_sweep < 0 || n_sweeps < 1))
        return fail(CMH_EINVAL, "log-probability records need first_sweep >= 0, n_sweeps >= 1");
    if (rec_dev && st->refresh_every <= 0)
        return fail(CMH_EINVAL, "log-probability records are taken at the scheduled refresh: "
                                "set refresh_every");
    st->lp_rec = rec_dev;
    st->lp_first = rec_dev ? first_sweep : 0;
    st->lp_n = rec_dev ? n_sweeps : 0;
    return CMH_OK;
}

int32_t cmh_set_stamps(cmh_state *st, uint64_t *stamps_dev, int64_t first_sweep,
                       int64_t n_sweeps)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (stamps_dev && (first_sweep < 0 || n_sweeps < 1))
        return fail(CMH_EINVAL, "stamps need first_sweep >= 0 and n_sweeps >= 1");
    drop_graphs(st);  // the graphs carry the kernels' arguments
    st->stamps = (unsigned long long *)stamps_dev;
    st->stamp_first = stamps_dev ? first_sweep : 0;
    st->stamp_n = stamps_dev ? n_sweeps : 0;
    return CMH_OK;
}

int32_t cmh_stamp_rate(int32_t device, int64_t *hz)
{
    if (!hz) return fail(CMH_EINVAL, "NULL argument");
    int khz = 0;
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device));
    if (khz <= 0) return fail(CMH_EHIP, "no steady clock rate");
    *hz = (int64_t)khz * 1000;
    return CMH_OK;
}

int32_t cmh_refresh(cmh_state *st, int32_t write_variance, double *out_host, void *hip_stream)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if ((rc = check_single(st))) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(cmh::launch_refresh(st->g, st->ev[st->cur], st->trace, st->f64, st->E,
                               write_variance ? 1 : 0, st->partials,
                               out_host ? st->llout : nullptr, 0, st->chains, st->err, s));
    if (!out_host) return CMH_OK;
    rc = sync_and_check(st);
    if (rc) return rc;
    HIPCHK(hipMemcpy(out_host, st->llout, (size_t)st->chains * 8, hipMemcpyDeviceToHost));
    return CMH_OK;
}

int32_t cmh_read_variance(cmh_state *st, int32_t chain, int64_t station0, int64_t nsta,
                          double *out_host)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if ((rc = check_single(st))) return rc;
    if (chain < 0 || chain >= st->chains) return fail(CMH_EINVAL, "chain out of range");
    if (station0 < 0 || nsta < 0 || station0 + nsta > st->g.nsta || (nsta > 0 && !out_host))
        return fail(CMH_EINVAL, "station range out of bounds");
    rc = sync_and_check(st);
    if (rc) return rc;
    const size_t N = (size_t)st->g.N;
    const double *src = st->E + ((size_t)chain * st->g.nsta + (size_t)station0) * N;
    HIPCHK(hipMemcpy(out_host, src, (size_t)nsta * N * 8, hipMemcpyDeviceToHost));
    return CMH_OK;
}

int32_t cmh_read_stats(cmh_state *st, int32_t chain, uint64_t *out_host)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (chain < 0 || chain >= st->chains || !out_host) return fail(CMH_EINVAL, "bad arguments");
    rc = sync_and_check(st);
    if (rc) return rc;
    HIPCHK(hipMemcpy(out_host, st->slots_h[chain].stats, cmh::kStats * 8, hipMemcpyDeviceToHost));
    return CMH_OK;
}

int32_t cmh_get_block(cmh_state *st, int32_t *block)
{
    if (!st || !block) return fail(CMH_EINVAL, "NULL argument");
    *block = st->block;
    return CMH_OK;
}

// Sweep-kernel forms worth trying for a state's geometry.
static std::vector<int> tune_forms(const cmh::Geo &g)
{
    if (g.naive) return {64};
    // latent arrivals have the wave form and the 256-thread latency form
    std::vector<int> f = g.latent ? std::vector<int>{64, 256}
                                  : std::vector<int>{64, 128, 256, 512, cmh::kSpecBase + 128,
                                                     cmh::kSpecBase + 256, cmh::kSpecBase + 512};
    // the persistent form: dynamic partitions without latent arrivals (its
    // kernel has no arrival moves)
    if (g.dynamic && !g.latent) f.push_back(cmh::kPersist);
    return f;
}

int32_t cmh_autotune(cmh_state *st, int64_t first_sweep, int32_t n_trial, void *hip_stream)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if ((rc = check_single(st))) return rc;
    if (n_trial < 1) return fail(CMH_EINVAL, "n_trial must be positive");
    if (st->feed || st->logp) return fail(CMH_EINVAL, "detach feed and log before tuning");
    const Geo &g = st->g;
    if (g.naive) {  // one form only
        st->block = 64;
        return CMH_OK;
    }
    const std::string key = tune_key(g, st->chains, st->f64, st->learned.tab != nullptr);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            st->block = it->second;
            return CMH_OK;
        }
    }
    hipStream_t s = (hipStream_t)hip_stream;
    rc = sync_and_check(st);
    if (rc) return rc;
    const int saved_cur = st->cur;
    HIPCHK(copy_events(st->snap, st->ev[saved_cur], g, st->chains, s));
    HIPCHK(hipMemcpyAsync(st->stats_snap, st->stats, (size_t)st->chains * cmh::kStats * 8,
                          hipMemcpyDeviceToDevice, s));
    auto restore = [&]() -> int32_t {
        st->cur = saved_cur;
        HIPCHK(copy_events(st->ev[saved_cur], st->snap, g, st->chains, s));
        HIPCHK(cmh::launch_refresh(g, st->ev[saved_cur], st->trace, st->f64, st->E, 1,
                                   st->partials, nullptr, 0, st->chains, st->err, s));
        HIPCHK(hipMemcpyAsync(st->stats, st->stats_snap, (size_t)st->chains * cmh::kStats * 8,
                              hipMemcpyDeviceToDevice, s));
        return CMH_OK;
    };
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const std::vector<int> forms = tune_forms(g);
    int best = st->block;
    float best_ms = 1e30f;
    for (int b : forms) {
        st->block = b;
        rc = cmh_run_sweeps(st, first_sweep, 1, hip_stream);  // warm-up, builds graphs
        if (!rc) rc = restore();
        if (!rc) {
            (void)hipEventRecord(e0, s);
            rc = cmh_run_sweeps(st, first_sweep, n_trial, hip_stream);
            (void)hipEventRecord(e1, s);
        }
        if (!rc) rc = sync_and_check(st);
        float ms = 0.f;
        if (!rc) (void)hipEventElapsedTime(&ms, e0, e1);
        const int32_t rc2 = restore();
        if (rc || rc2) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rc ? rc : rc2;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = b;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st->block = best;
    drop_graphs(st);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    return sync_and_check(st);
}

int32_t cmh_tune_running(cmh_state *st, int64_t first_sweep, int32_t n_trial, void *hip_stream,
                         int64_t *next_sweep)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (!next_sweep) return fail(CMH_EINVAL, "next_sweep is NULL");
    if (n_trial < 1) return fail(CMH_EINVAL, "n_trial must be positive");
    const std::vector<int> forms = tune_forms(st->g);
    const int64_t per = 1 + (int64_t)n_trial;
    if (first_sweep < 0 || first_sweep + per * (int64_t)forms.size() > (1LL << 32))
        return fail(CMH_EINVAL, "sweep range out of bounds");
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int saved = st->block;
    int best = saved;
    float best_ms = 1e30f;
    int64_t sw = first_sweep;
    for (int b : forms) {
        st->block = b;
        // one sweep that builds the form's graphs, then the timed ones; every
        // form takes the chain through the same states
        rc = cmh_run_sweeps(st, sw, 1, hip_stream);
        if (!rc) {
            (void)hipEventRecord(e0, s);
            rc = cmh_run_sweeps(st, sw + 1, n_trial, hip_stream);
            (void)hipEventRecord(e1, s);
        }
        if (!rc) rc = sync_and_check(st);
        float ms = 0.f;
        if (!rc) (void)hipEventElapsedTime(&ms, e0, e1);
        if (rc) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            st->block = saved;
            return rc;
        }
        sw += per;
        if (ms < best_ms) {
            best_ms = ms;
            best = b;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st->block = best;
    *next_sweep = sw;
    return CMH_OK;
}

int32_t cmh_time_phases(cmh_state *st, int64_t first_sweep, int64_t n_sweeps, void *hip_stream,
                        float *ms_out)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if ((rc = check_single(st))) return rc;
    if (!ms_out || n_sweeps < 1 || first_sweep < 0 || first_sweep + n_sweeps > (1LL << 32))
        return fail(CMH_EINVAL, "bad arguments");
    if (st->feed && (first_sweep < st->feed_first ||
                     first_sweep + n_sweeps > st->feed_first + st->feed_n))
        return fail(CMH_EINVAL, "sweeps outside the attached feed");
    if (st->feed && st->feed_width != (st->learned.tab || st->g.latent ? 16 : 8))
        return fail(CMH_EINVAL,
                    "feed records must be 16 wide with learned births or latent arrivals, else 8");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nc = st->g.ncolors;
    std::vector<hipEvent_t> ev((size_t)n_sweeps * (nc + 2));
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    hipError_t e = hipSuccess;
    for (int64_t q = 0; q < n_sweeps && e == hipSuccess; ++q) {
        hipEvent_t *E = &ev[(size_t)q * (nc + 2)];
        e = cmh::set_sweep(st->sweep_ctr, first_sweep + q, s);
        if (!e) e = hipEventRecord(E[0], s);
        if (!e) e = enqueue_sweep_start(st, s);
        if (!e) e = hipEventRecord(E[1], s);
        for (int c = 0; c < nc && !e; ++c) {
            e = enqueue_phase(st, c, false, s);
            if (!e) e = hipEventRecord(E[2 + c], s);
        }
    }
    if (!e) e = hipStreamSynchronize(s);
    for (int c = 0; c <= nc; ++c) ms_out[c] = 0.f;
    for (int64_t q = 0; q < n_sweeps && !e; ++q) {
        hipEvent_t *E = &ev[(size_t)q * (nc + 2)];
        float ms = 0.f;
        if (!e) e = hipEventElapsedTime(&ms, E[0], E[1]);
        ms_out[nc] += ms;
        for (int c = 0; c < nc && !e; ++c) {
            e = hipEventElapsedTime(&ms, E[1 + c], E[2 + c]);
            ms_out[c] += ms;
        }
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    if (e) return fail(CMH_EHIP, std::string("phase timing: ") + hipGetErrorString(e));
    return sync_and_check(st);
}

namespace {
// The library's learned-birth arrays for `chains` chains of one instance.
size_t carve_learned(const cmh::Geo &g, int chains, int ntau, char *base, cmh::Learned *L,
                     double **part)
{
    Carver c{base};
    const size_t na = (size_t)g.nsta * ntau;
    double *cum = c.take<double>(na);
    double *norm = c.take<double>(na * 8);
    double *reach = c.take<double>(2);
    double *pp = c.take<double>((size_t)2 * cmh::learned_norm_blocks((long long)na * 8));
    double *birth = c.take<double>((size_t)chains * g.R * g.k * 4);
    double *raw = c.take<double>((size_t)chains * g.R * g.k * 8);
    if (L) {
        L->cum = cum;
        L->norm = norm;
        L->reach = reach;
        L->birth = birth;
        L->raw = raw;
    }
    if (part) *part = pp;
    return align_up(c.off);
}

size_t carve_learned_st(const cmh_state *st, int ntau, char *base, cmh::Learned *L, double **part)
{
    return carve_learned(st->g, st->chains, ntau, base, L, part);
}

// Checks shared by the learned-birth setters; derives the arrays into
// work_dev and returns the instance's Learned in *L.
int32_t prepare_learned(const cmh::Geo &g, int chains, const double *table_dev,
                        const double *weights_dev, int32_t n_tau, double p_learned,
                        void *work_dev, size_t work_bytes, hipStream_t s, cmh::Learned *L)
{
    if (n_tau < 1) return fail(CMH_EINVAL, "n_tau must be >= 1");
    if (!(p_learned >= 0.0 && p_learned < 1.0))
        return fail(CMH_EINVAL, "p_learned must lie in [0, 1)");
    if (!weights_dev || !work_dev) return fail(CMH_EINVAL, "NULL argument");
    if (work_bytes < carve_learned(g, chains, n_tau, nullptr, nullptr, nullptr))
        return fail(CMH_EINVAL, "learned workspace too small");
    *L = cmh::Learned{};
    double *part = nullptr;
    carve_learned(g, chains, n_tau, (char *)work_dev, L, &part);
    L->tab = table_dev;
    L->w = weights_dev;
    L->ntau = n_tau;
    L->pl = p_learned;
    const double lz3 = 3.0 * log(sqrt(2.0 * M_PI) * erf(4.0 / sqrt(2.0)));
    HIPCHK(cmh::launch_learned_prep(weights_dev, table_dev, n_tau, g.nsta, lz3, (double *)L->cum,
                                    (double *)L->norm, part, (double *)L->reach, s));
    HIPCHK(hipStreamSynchronize(s));
    return CMH_OK;
}
}  // namespace

int32_t cmh_learned_bytes(cmh_state *st, int32_t n_tau, size_t *bytes)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if ((rc = check_single(st))) return rc;
    if (st->g.line || st->g.tmpl)
        return fail(CMH_EINVAL, "learned births need the grid model's variance signals");
    if (n_tau < 1) return fail(CMH_EINVAL, "n_tau must be >= 1");
    if (!bytes) return fail(CMH_EINVAL, "bytes is NULL");
    *bytes = carve_learned_st(st, n_tau, nullptr, nullptr, nullptr);
    return CMH_OK;
}

int32_t cmh_set_learned(cmh_state *st, const double *table_dev, const double *weights_dev,
                        int32_t n_tau, double p_learned, void *work_dev, size_t work_bytes,
                        void *hip_stream)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if ((rc = check_single(st))) return rc;
    if (table_dev && (st->g.line || st->g.tmpl))
        return fail(CMH_EINVAL, "learned births need the grid model's variance signals");
    drop_graphs(st);
    if (!table_dev) {
        st->learned = cmh::Learned{};
        return upload_slots(st);
    }
    cmh::Learned L{};
    rc = prepare_learned(st->g, st->chains, table_dev, weights_dev, n_tau, p_learned, work_dev,
                         work_bytes, (hipStream_t)hip_stream, &L);
    if (rc) return rc;
    st->learned = L;
    return upload_slots(st);
}

int32_t cmh_batch_learned_bytes(cmh_state *st, int32_t instance, int32_t n_tau, size_t *bytes)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (!st->batch) return fail(CMH_EINVAL, "not a batch of instances");
    if (instance < 0 || instance >= st->nslots) return fail(CMH_EINVAL, "instance out of range");
    const Geo &g = st->slots_h[instance].g;
    if (g.line || g.tmpl)
        return fail(CMH_EINVAL, "learned births need the grid model's variance signals");
    if (n_tau < 1) return fail(CMH_EINVAL, "n_tau must be >= 1");
    if (!bytes) return fail(CMH_EINVAL, "bytes is NULL");
    *bytes = carve_learned(g, 1, n_tau, nullptr, nullptr, nullptr);
    return CMH_OK;
}

int32_t cmh_batch_set_learned(cmh_state *st, int32_t instance, const double *table_dev,
                              const double *weights_dev, int32_t n_tau, double p_learned,
                              void *work_dev, size_t work_bytes, void *hip_stream)
{
    int32_t rc = check_state(st);
    if (rc) return rc;
    if (!st->batch) return fail(CMH_EINVAL, "not a batch of instances");
    if (instance < 0 || instance >= st->nslots) return fail(CMH_EINVAL, "instance out of range");
    cmh::Slot &sl = st->slots_h[instance];
    if (table_dev && (sl.g.line || sl.g.tmpl))
        return fail(CMH_EINVAL, "learned births need the grid model's variance signals");
    rc = sync_and_check(st);
    if (rc) return rc;
    drop_graphs(st);
    cmh::Learned L{};
    if (table_dev) {
        rc = prepare_learned(sl.g, 1, table_dev, weights_dev, n_tau, p_learned, work_dev,
                             work_bytes, (hipStream_t)hip_stream, &L);
        if (rc) return rc;
    }
    st->n_learned += (L.tab != nullptr) - (sl.L.tab != nullptr);
    sl.L = L;
    HIPCHK(hipMemcpy(st->slots_d + instance, &sl, sizeof(cmh::Slot), hipMemcpyHostToDevice));
    return CMH_OK;
}

// ------------------------------------------------------------------- batch
namespace {

struct BatchPlan {
    std::vector<Geo> g;
    Geo head;  // what the sweep loop reads: k, dynamic, colours (the most of any instance)
};

int32_t plan_batch(int32_t n, const cmh_model *models, const cmh_sampler *samplers, BatchPlan *P)
{
    if (n < 1 || n > 65535) return fail(CMH_EINVAL, "n_instances must be in 1..65535");
    if (!models || !samplers) return fail(CMH_EINVAL, "NULL argument");
    P->g.resize(n);
    for (int q = 0; q < n; ++q) {
        int32_t rc = make_geo(&models[q], &samplers[q], &P->g[q]);
        if (rc) return rc;
        if (P->g[q].R > 65535) return fail(CMH_EINVAL, "at most 65535 regions per instance");
        if (P->g[q].k != P->g[0].k || P->g[q].dynamic != P->g[0].dynamic ||
            samplers[q].block != samplers[0].block || P->g[q].naive != P->g[0].naive ||
            P->g[q].latent != P->g[0].latent ||
            samplers[q].refresh_every != samplers[0].refresh_every)
            return fail(CMH_EINVAL, "instances of a batch share k, dynamic, block, schedule, "
                                    "latent arrivals and refresh_every");
    }
    P->head = P->g[0];
    for (int q = 0; q < n; ++q) P->head.ncolors = std::max(P->head.ncolors, P->g[q].ncolors);
    return CMH_OK;
}

// Workspace of a batch: per instance E, two event tables, draws, statistics;
// shared sweep counter, error word, slot table and work items.
size_t carve_batch(const BatchPlan &P, char *base, std::vector<cmh::Slot> *slots,
                   long long **sweep, int **err, cmh::Slot **slots_d, unsigned **items_all,
                   unsigned **items_col, double **partials = nullptr, double **llout = nullptr,
                   int **pq_ctr = nullptr, unsigned **pq_wait = nullptr)
{
    Carver c{base};
    long long total_r = 0;
    int per_max = 0;
    for (size_t q = 0; q < P.g.size(); ++q) {
        const Geo &g = P.g[q];
        cmh::Slot sl{};
        sl.g = g;
        sl.E = c.take<double>((size_t)g.nsta * (size_t)g.N);
        for (int b = 0; b < 2; ++b) carve_events(c, g, 1, &sl.ev[b]);
        sl.draws = c.take<double>((size_t)g.R * g.k * 8);
        sl.draws2 = g.latent ? c.take<double>((size_t)g.R * g.k * 8) : nullptr;
        sl.stats = c.take<unsigned long long>(cmh::kStats);
        sl.owner = g.owner ? c.take<unsigned long long>((size_t)g.nsta * (size_t)g.N) : nullptr;
        if (slots) (*slots)[q] = sl;
        total_r += g.R;
        per_max = std::max(per_max, cmh::refresh_blocks(g));
    }
    double *pp = c.take<double>(P.g.size() * (size_t)per_max);
    double *lo = c.take<double>(P.g.size() * 2);
    if (partials) *partials = pp;
    if (llout) *llout = lo;
    long long *sw = c.take<long long>(1);
    int *er = c.take<int>(1);
    cmh::Slot *sd = c.take<cmh::Slot>(P.g.size());
    unsigned *ia = c.take<unsigned>((size_t)total_r);
    unsigned *ic = c.take<unsigned>((size_t)total_r);
    int *pc = c.take<int>(P.g.size() + 1);
    unsigned *pw = c.take<unsigned>((size_t)total_r);
    if (pq_ctr) *pq_ctr = pc;
    if (pq_wait) *pq_wait = pw;
    if (sweep) *sweep = sw;
    if (err) *err = er;
    if (slots_d) *slots_d = sd;
    if (items_all) *items_all = ia;
    if (items_col) *items_col = ic;
    return align_up(c.off);
}

}  // namespace

int32_t cmh_batch_bytes(int32_t n_instances, const cmh_model *models, const cmh_sampler *samplers,
                        size_t *bytes)
{
    BatchPlan P;
    int32_t rc = plan_batch(n_instances, models, samplers, &P);
    if (rc) return rc;
    if (!bytes) return fail(CMH_EINVAL, "bytes is NULL");
    *bytes = carve_batch(P, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    return CMH_OK;
}

int32_t cmh_batch_init(int32_t n_instances, const cmh_model *models, const cmh_sampler *samplers,
                       const void *const *traces_dev, int32_t trace_dtype, const uint32_t *seeds,
                       void *workspace_dev, size_t workspace_bytes, void *hip_stream,
                       cmh_state **out)
{
    if (!out) return fail(CMH_EINVAL, "out is NULL");
    *out = nullptr;
    BatchPlan P;
    int32_t rc = plan_batch(n_instances, models, samplers, &P);
    if (rc) return rc;
    if (trace_dtype != CMH_F32 && trace_dtype != CMH_F64)
        return fail(CMH_EINVAL, "trace_dtype must be CMH_F32 or CMH_F64");
    if (!traces_dev || !seeds || !workspace_dev) return fail(CMH_EINVAL, "NULL argument");
    for (int q = 0; q < n_instances; ++q)
        if (!traces_dev[q]) return fail(CMH_EINVAL, "NULL trace");
    const size_t need = carve_batch(P, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                    nullptr);
    if (workspace_bytes < need)
        return fail(CMH_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    cmh_state *st = new cmh_state();
    st->batch = 1;
    st->g = P.head;
    st->chains = n_instances;
    st->nslots = n_instances;
    st->f64 = trace_dtype == CMH_F64;
    st->block = P.head.naive ? 64 : (samplers[0].block ? samplers[0].block : 256);
    st->slots_h.resize(n_instances);
    carve_batch(P, (char *)workspace_dev, &st->slots_h, &st->sweep_ctr, &st->err, &st->slots_d,
                &st->items_all, &st->items_col, &st->partials, &st->llout, &st->pq_ctr,
                &st->pq_wait);
    st->refresh_every = samplers[0].refresh_every;
    st->spin_limit = (samplers[0].debug & 4) ? 0 : st->spin_limit;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipStreamCreateWithFlags(&st->cap_stream, hipStreamNonBlocking);
    std::vector<unsigned> all, col;
    for (int q = 0; q < n_instances && !e; ++q) {
        cmh::Slot &sl = st->slots_h[q];
        sl.g.seed = seeds[q];
        sl.chain = 0;
        sl.trace = traces_dev[q];
        const Geo &g = sl.g;
        const long long nE = (long long)g.nsta * g.N;
        e = g.tmpl ? cmh::residual_init(sl.E, sl.trace, trace_dtype == CMH_F64, nE, nE, s)
                   : cmh::fill_f64(sl.E, nE, 0.0, s);
        for (int b = 0; b < 2 && !e; ++b) {
            e = cmh::fill_i32(sl.ev[b].cnt, g.R, 0, s);
            if (!e) e = cmh::fill_f64(sl.ev[b].off, 2, 0.0, s);
        }
        if (!e) e = cmh::fill_u64(sl.stats, cmh::kStats, s);
        if (!e && sl.owner) e = cmh::fill_u64(sl.owner, nE, s);
        if (sl.owner) st->owner_any = 1;
        for (int r = 0; r < g.R; ++r) all.push_back(((unsigned)q << 16) | (unsigned)r);
        st->refresh_max = std::max(st->refresh_max, cmh::refresh_blocks(g));
        st->naive_elems = std::max(st->naive_elems, g.nsta * g.N);
    }
    st->col_off.assign(P.head.ncolors, 0);
    st->col_n.assign(P.head.ncolors, 0);
    for (int color = 0; color < P.head.ncolors; ++color) {
        st->col_off[color] = (int)col.size();
        for (int q = 0; q < n_instances; ++q) {
            const Geo &g = st->slots_h[q].g;
            for (int r = 0; r < g.R; ++r) {
                const int i = r % g.nrx, k = r / g.nrx;
                if ((g.naive ? 0 : (i % g.period) + g.period * (k % g.period)) == color)
                    col.push_back(((unsigned)q << 16) | (unsigned)r);
            }
        }
        st->col_n[color] = (int)col.size() - st->col_off[color];
    }
    st->n_all = (int)all.size();
    if (!e) e = cmh::fill_i32(st->err, 1, 0, s);
    if (!e) e = cmh::set_sweep(st->sweep_ctr, 0, s);
    if (!e) e = hipStreamSynchronize(s);
    if (!e) e = hipMemcpy(st->slots_d, st->slots_h.data(), sizeof(cmh::Slot) * n_instances,
                          hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(st->items_all, all.data(), sizeof(unsigned) * all.size(),
                          hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(st->items_col, col.data(), sizeof(unsigned) * col.size(),
                          hipMemcpyHostToDevice);
    if (e) {
        if (st->cap_stream) (void)hipStreamDestroy(st->cap_stream);
        delete st;
        return fail(CMH_EHIP, std::string("batch init: ") + hipGetErrorString(e));
    }
    {
        const std::vector<unsigned> wait = wait_targets(col, st->col_off, st->col_n, n_instances);
        e = hipMemcpy(st->pq_wait, wait.data(), sizeof(unsigned) * wait.size(),
                      hipMemcpyHostToDevice);
        if (e) {
            if (st->cap_stream) (void)hipStreamDestroy(st->cap_stream);
            delete st;
            return fail(CMH_EHIP, std::string("batch init: ") + hipGetErrorString(e));
        }
    }
    *out = st;
    return CMH_OK;
}

int32_t cmh_destroy(cmh_state *st)
{
    if (!st) return CMH_OK;
    drop_graphs(st);
    if (st->cap_stream) (void)hipStreamDestroy(st->cap_stream);
    delete st;
    return CMH_OK;
}

// ---------------------------------------------------------------- simulator
namespace {

struct TruthLayout {
    Geo g;
    std::vector<std::vector<cmh_event>> cells;
    int cap = 1;
};

int32_t truth_layout(const cmh_model *model, const cmh_event *truth, int64_t n, TruthLayout *L)
{
    int32_t rc = check_model(model);
    if (rc) return rc;
    if (n < 0 || (n > 0 && !truth)) return fail(CMH_EINVAL, "bad truth array");
    Geo &g = L->g;
    std::memset(&g, 0, sizeof g);
    g.nsx = model->nsx; g.nsy = model->nsy; g.nsta = g.nsx * g.nsy; g.ts = model->t_s;
    g.N = (int)model->n_samples;
    g.gx = model->nsx; g.gy = model->nsy; g.nrx = g.gx + 1; g.nry = g.gy + 1;
    g.R = g.nrx * g.nry;
    g.ds = model->ds; g.sigma2 = model->sigma * model->sigma; g.atten = model->atten;
    g.vel = model->velocity; g.decay = model->env_decay; g.rc = model->r_c;
    g.att2 = 2.0 / g.atten; g.dec2 = 2.0 / g.decay;
    g.tmpl = model->template_mean;
    if (g.tmpl) {
        g.att2 = 1.0 / g.atten;
        g.dec2 = 1.0 / g.decay;
    }
    g.Lx = (double)model->nsx * model->ds; g.Ly = (double)model->nsy * model->ds;
    g.wx = g.Lx / (double)g.gx; g.wy = g.Ly / (double)g.gy;
    if (model->line) {
        // cells of onset time, long enough that a tile's gather spans at
        // most 25 of them
        g.line = 1;
        g.tmax = line_tmax(model);
        for (int j = 0; j < model->nsx; ++j) g.sx[j] = model->station_x[j];
        g.rc = INFINITY; g.atten = INFINITY; g.decay = INFINITY; g.att2 = 0.0; g.dec2 = 0.0;
        g.Lx = model->x_max; g.Ly = 1.0;
        if (model->arrival_sd > 0.0) {  // latent arrivals: offsets stored per event
            g.latent = 1;
            g.arr_e = cmh::kArrTrunc * model->arrival_sd;
        }
        const double wmin =
            std::max(512.0, (cmh::kTile + g.tmax + g.ts + 2.0 * g.arr_e + 1.0) / 23.0);
        g.gx = std::max(1, (int)((double)g.N / wmin));
        g.gy = 0; g.nrx = g.gx + 1; g.nry = 1; g.R = g.nrx;
        g.wx = (double)g.N / (double)g.gx; g.wy = 0.0;
    }
    L->cells.assign(g.R, {});
    for (int64_t q = 0; q < n; ++q) {
        const cmh_event &e = truth[q];
        if (!(e.x >= 0.0 && e.x < g.Lx && e.y >= 0.0 && e.y < g.Ly && e.t >= 0.0 &&
              e.t < (double)g.N && std::isfinite(e.m)))
            return fail(CMH_EINVAL, "truth event outside the domain");
        if (g.latent)
            for (int c = 0; c < g.nsx; ++c)
                if (!(std::fabs(e.da[c]) <= g.arr_e))
                    return fail(CMH_EINVAL, "truth arrival offset beyond the jitter bound");
        L->cells[cmh::event_region(g, 0.0, 0.0, e.x, e.y, e.t)].push_back(e);
    }
    L->cap = 1;
    for (auto &c : L->cells) {
        std::sort(c.begin(), c.end(),
                  [](const cmh_event &a, const cmh_event &b) { return a.id < b.id; });
        L->cap = std::max(L->cap, (int)c.size());
    }
    if (L->cap > cmh::kMaxTileEvents / 9)
        return fail(CMH_EINVAL, "too many truth events in one station cell");
    g.cap = L->cap;
    return CMH_OK;
}

size_t carve_truth(const Geo &g, char *base, Events *ev, int **err)
{
    Carver c{base};
    Events e;
    carve_events(c, g, 1, &e);
    int *f = c.take<int>(1);
    if (ev) *ev = e;
    if (err) *err = f;
    return align_up(c.off);
}

}  // namespace

int32_t cmh_simulate_bytes(const cmh_model *model, const cmh_event *truth_host, int64_t n_events,
                           size_t *bytes)
{
    if (!bytes) return fail(CMH_EINVAL, "bytes is NULL");
    TruthLayout L;
    int32_t rc = truth_layout(model, truth_host, n_events, &L);
    if (rc) return rc;
    *bytes = carve_truth(L.g, nullptr, nullptr, nullptr);
    return CMH_OK;
}

namespace {

// The simulator on a laid-out truth table: the table is staged in `ws` (at
// least carve_truth bytes of device memory), then every station's trace is
// written.  Synchronises.
int32_t simulate_into(const TruthLayout &L, uint32_t seed, void *trace_dev, int32_t trace_dtype,
                      void *ws, hipStream_t s)
{
    const Geo &g = L.g;
    Events ev;
    int *err = nullptr;
    carve_truth(g, (char *)ws, &ev, &err);
    const size_t slots = (size_t)g.R * g.cap;
    std::vector<int> cnt(g.R, 0);
    std::vector<double> x(slots, 0), y(slots, 0), t(slots, 0), m(slots, 0), off(2, 0.0);
    std::vector<unsigned long long> id(slots, 0);
    std::vector<double> da(g.latent ? slots * 8 : 0, 0.0);
    for (int r = 0; r < g.R; ++r) {
        cnt[r] = (int)L.cells[r].size();
        for (size_t q = 0; q < L.cells[r].size(); ++q) {
            const size_t a = (size_t)r * g.cap + q;
            const cmh_event &e = L.cells[r][q];
            x[a] = e.x; y[a] = e.y; t[a] = e.t; m[a] = e.m; id[a] = e.id;
            if (g.latent)
                for (int c = 0; c < g.nsx; ++c) da[a * 8 + c] = e.da[c];
        }
    }
    HIPCHK(hipMemcpyAsync(ev.cnt, cnt.data(), g.R * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ev.x, x.data(), slots * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ev.y, y.data(), slots * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ev.t, t.data(), slots * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ev.m, m.data(), slots * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ev.id, id.data(), slots * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ev.off, off.data(), 16, hipMemcpyHostToDevice, s));
    if (g.latent) HIPCHK(hipMemcpyAsync(ev.da, da.data(), slots * 64, hipMemcpyHostToDevice, s));
    HIPCHK(cmh::fill_i32(err, 1, 0, s));
    HIPCHK(cmh::launch_simulate(g, ev, seed, trace_dev, trace_dtype == CMH_F64, err, s));
    HIPCHK(hipStreamSynchronize(s));
    int flags = 0;
    HIPCHK(hipMemcpy(&flags, err, sizeof(int), hipMemcpyDeviceToHost));
    if (flags) return fail(CMH_ESTATE, "simulator tile capacity exceeded");
    return CMH_OK;
}

// Scratch of the no-allocation simulator: one array per device, reached
// through the address hipGetSymbolAddress returns on that device (the
// symbol's name is a host-side stand-in).  Calls on one device share it.
constexpr size_t kSimScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kSimScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> device address of `scratch`

int32_t scratch_address(void **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(CMH_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return CMH_OK;
}

}  // namespace

int32_t cmh_simulate(const cmh_model *model, const cmh_event *truth_host, int64_t n_events,
                     uint32_t seed, void *trace_dev, int32_t trace_dtype, void *workspace_dev,
                     size_t workspace_bytes, void *hip_stream)
{
    TruthLayout L;
    int32_t rc = truth_layout(model, truth_host, n_events, &L);
    if (rc) return rc;
    if (trace_dtype != CMH_F32 && trace_dtype != CMH_F64)
        return fail(CMH_EINVAL, "trace_dtype must be CMH_F32 or CMH_F64");
    if (!trace_dev || !workspace_dev) return fail(CMH_EINVAL, "NULL device buffer");
    const size_t need = carve_truth(L.g, nullptr, nullptr, nullptr);
    if (workspace_bytes < need) return fail(CMH_EINVAL, "simulator workspace too small");
    return simulate_into(L, seed, trace_dev, trace_dtype, workspace_dev, (hipStream_t)hip_stream);
}

int32_t cmh_simulate_noalloc(const cmh_model *model, const cmh_event *truth_host,
                             int64_t n_events, uint32_t seed, void *trace_dev,
                             int32_t trace_dtype, void *hip_stream)
{
    TruthLayout L;
    int32_t rc = truth_layout(model, truth_host, n_events, &L);
    if (rc) return rc;
    if (trace_dtype != CMH_F32 && trace_dtype != CMH_F64)
        return fail(CMH_EINVAL, "trace_dtype must be CMH_F32 or CMH_F64");
    if (!trace_dev) return fail(CMH_EINVAL, "NULL device buffer");
    const size_t need = carve_truth(L.g, nullptr, nullptr, nullptr);
    if (need > kSimScratchBytes)
        return fail(CMH_EINVAL, "truth table needs " + std::to_string(need) +
                                    " bytes of scratch, more than the " +
                                    std::to_string(kSimScratchBytes) + " this call holds");
    void *ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    return simulate_into(L, seed, trace_dev, trace_dtype, ws, (hipStream_t)hip_stream);
}

int32_t cmh_move_draws(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region, uint32_t j0,
                       int32_t count, int32_t width, double *out_dev, void *hip_stream)
{
    if (count < 0 || (count > 0 && !out_dev)) return fail(CMH_EINVAL, "bad arguments");
    if (width != 8 && width != 16) return fail(CMH_EINVAL, "width must be 8 or 16");
    if (count == 0) return CMH_OK;
    HIPCHK(cmh::launch_draws(seed, chain, sweep, region, j0, count, width, out_dev,
                             (hipStream_t)hip_stream));
    return CMH_OK;
}

int32_t cmh_move_draws_arrivals(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                                uint32_t j0, int32_t count, double *out_dev, void *hip_stream)
{
    if (count < 0 || (count > 0 && !out_dev)) return fail(CMH_EINVAL, "bad arguments");
    if (count == 0) return CMH_OK;
    // width code 17: the latent-arrival records (16 wide) of the draw kernel
    HIPCHK(cmh::launch_draws(seed, chain, sweep, region, j0, count, 17, out_dev,
                             (hipStream_t)hip_stream));
    return CMH_OK;
}

}  // extern "C"

// ---------------------------------------------------------- learned proposal
namespace {

void model_geo(const cmh_model *m, Geo *g)
{
    std::memset(g, 0, sizeof *g);
    g->nsx = m->nsx; g->nsy = m->nsy; g->nsta = m->nsx * m->nsy; g->ts = m->t_s;
    g->N = (int)m->n_samples;
    g->ds = m->ds; g->sigma2 = m->sigma * m->sigma; g->atten = m->atten; g->vel = m->velocity;
    g->decay = m->env_decay; g->rc = m->r_c; g->lambda = m->lambda; g->mmin = m->mag_min;
    g->mrate = m->mag_rate;
    g->att2 = 2.0 / g->atten; g->dec2 = 2.0 / g->decay;
    g->Lx = (double)m->nsx * m->ds; g->Ly = (double)m->nsy * m->ds;
}

struct MdnBlob {
    float *params;
    __bf16 *hcopy;
};

size_t mdn_param_bytes()
{
    const cmh::MdnLayout L = cmh::mdn_layout();
    return align_up((size_t)3 * L.np * 4) + align_up((size_t)L.nh * 2);
}

MdnBlob mdn_blob(const void *p)
{
    const cmh::MdnLayout L = cmh::mdn_layout();
    MdnBlob b;
    b.params = (float *)p;
    b.hcopy = (__bf16 *)((char *)p + align_up((size_t)3 * L.np * 4));
    return b;
}

size_t carve_mdn_work(int M, char *base, cmh::MdnBuffers *B, float **grad)
{
    const cmh::MdnLayout L = cmh::mdn_layout();
    Carver c{base};
    cmh::MdnBuffers b;
    const size_t mh = (size_t)M * cmh::kMdnHid, mo = (size_t)M * cmh::kMdnOutPad;
    for (int l = 0; l < 3; ++l) b.Z[l] = c.take<float>(mh);
    for (int l = 0; l < 3; ++l) b.A[l] = c.take<__bf16>(mh);
    b.O = c.take<float>(mo);
    b.dO = c.take<__bf16>(mo);
    b.dH[0] = c.take<__bf16>(mh);
    b.dH[1] = c.take<__bf16>(mh);
    b.loss = c.take<float>((size_t)M);
    // split partials of every weight and bias gradient, side by side
    b.part = c.take<float>(cmh::mdn_part_floats(M));
    float *gr = c.take<float>((size_t)L.np);
    if (B) *B = b;
    if (grad) *grad = gr;
    return align_up(c.off);
}

int32_t check_rows(int32_t rows) { return rows >= 1 && rows <= (1 << 20) ? CMH_OK : fail(CMH_EINVAL, "rows must be in 1..2^20"); }

int32_t check_aligned(const void *p, const char *what)
{
    return ((uintptr_t)p & 15u) == 0 ? CMH_OK
                                     : fail(CMH_EINVAL, std::string(what) + " must be 16-byte aligned");
}

}  // namespace

extern "C" {

int32_t cmh_mdn_sizes(int64_t *n_params, int64_t *n_weights_bf16)
{
    const cmh::MdnLayout L = cmh::mdn_layout();
    if (n_params) *n_params = L.np;
    if (n_weights_bf16) *n_weights_bf16 = L.nh;
    return CMH_OK;
}

int32_t cmh_mdn_param_bytes(size_t *bytes)
{
    if (!bytes) return fail(CMH_EINVAL, "bytes is NULL");
    *bytes = mdn_param_bytes();
    return CMH_OK;
}

int32_t cmh_mdn_init(void *params_dev, uint32_t seed, void *hip_stream)
{
    if (!params_dev) return fail(CMH_EINVAL, "params_dev is NULL");
    const MdnBlob b = mdn_blob(params_dev);
    HIPCHK(cmh::mdn_init(b.params, b.hcopy, seed, (hipStream_t)hip_stream));
    return CMH_OK;
}

int32_t cmh_mdn_set_params(void *params_dev, const float *host, void *hip_stream)
{
    if (!params_dev || !host) return fail(CMH_EINVAL, "NULL argument");
    const cmh::MdnLayout L = cmh::mdn_layout();
    const MdnBlob b = mdn_blob(params_dev);
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(hipMemcpyAsync(b.params, host, (size_t)L.np * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(b.params + L.np, 0, (size_t)2 * L.np * 4, s));
    HIPCHK(cmh::mdn_refresh_copies(b.params, b.hcopy, s));
    HIPCHK(hipStreamSynchronize(s));
    return CMH_OK;
}

int32_t cmh_mdn_get_params(const void *params_dev, float *host)
{
    if (!params_dev || !host) return fail(CMH_EINVAL, "NULL argument");
    const cmh::MdnLayout L = cmh::mdn_layout();
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(host, params_dev, (size_t)L.np * 4, hipMemcpyDeviceToHost));
    return CMH_OK;
}

int32_t cmh_mdn_work_bytes(int32_t rows, size_t *bytes)
{
    int32_t rc = check_rows(rows);
    if (rc) return rc;
    if (!bytes) return fail(CMH_EINVAL, "bytes is NULL");
    *bytes = carve_mdn_work(rows, nullptr, nullptr, nullptr);
    return CMH_OK;
}

int32_t cmh_mdn_forward(const void *params_dev, const void *x_dev, int32_t rows, float *out_dev,
                        void *work_dev, size_t work_bytes, void *hip_stream)
{
    int32_t rc = check_rows(rows);
    if (rc) return rc;
    if (!params_dev || !x_dev || !out_dev || !work_dev) return fail(CMH_EINVAL, "NULL argument");
    if ((rc = check_aligned(x_dev, "x_dev")) || (rc = check_aligned(work_dev, "work_dev")))
        return rc;
    if (work_bytes < carve_mdn_work(rows, nullptr, nullptr, nullptr))
        return fail(CMH_EINVAL, "work buffer too small");
    cmh::MdnBuffers B;
    carve_mdn_work(rows, (char *)work_dev, &B, nullptr);
    B.O = out_dev;
    const MdnBlob b = mdn_blob(params_dev);
    HIPCHK(cmh::mdn_forward(b.params, b.hcopy, (const __bf16 *)x_dev, rows, B,
                            (hipStream_t)hip_stream));
    return CMH_OK;
}

int32_t cmh_mdn_infer(const void *params_dev, const void *x_dev, int32_t rows, float *out_dev,
                      void *hip_stream)
{
    if (rows < 1) return fail(CMH_EINVAL, "rows must be positive");
    if (!params_dev || !x_dev || !out_dev) return fail(CMH_EINVAL, "NULL argument");
    int32_t rc = check_aligned(x_dev, "x_dev");
    if (rc) return rc;
    const MdnBlob b = mdn_blob(params_dev);
    HIPCHK(cmh::mdn_infer(b.params, b.hcopy, (const __bf16 *)x_dev, rows, out_dev,
                          (hipStream_t)hip_stream));
    return CMH_OK;
}

int32_t cmh_mdn_gradients(const void *params_dev, const void *x_dev, const float *z_dev,
                          int32_t rows, float *grad_dev, float *loss_dev, void *work_dev,
                          size_t work_bytes, void *hip_stream)
{
    int32_t rc = check_rows(rows);
    if (rc) return rc;
    if (!params_dev || !x_dev || !z_dev || !grad_dev || !work_dev)
        return fail(CMH_EINVAL, "NULL argument");
    if ((rc = check_aligned(x_dev, "x_dev")) || (rc = check_aligned(work_dev, "work_dev")))
        return rc;
    if (work_bytes < carve_mdn_work(rows, nullptr, nullptr, nullptr))
        return fail(CMH_EINVAL, "work buffer too small");
    cmh::MdnBuffers B;
    carve_mdn_work(rows, (char *)work_dev, &B, nullptr);
    if (loss_dev) B.loss = loss_dev;
    const MdnBlob b = mdn_blob(params_dev);
    HIPCHK(cmh::mdn_backward(b.params, b.hcopy, (const __bf16 *)x_dev, z_dev, rows, B, grad_dev,
                             (hipStream_t)hip_stream));
    return CMH_OK;
}

int32_t cmh_mdn_train_step(void *params_dev, const void *x_dev, const float *z_dev, int32_t rows,
                           int32_t step, float lr, float *loss_dev, void *work_dev,
                           size_t work_bytes, void *hip_stream)
{
    int32_t rc = check_rows(rows);
    if (rc) return rc;
    if (step < 1) return fail(CMH_EINVAL, "Adam steps count from 1");
    if (!params_dev || !x_dev || !z_dev || !work_dev) return fail(CMH_EINVAL, "NULL argument");
    if ((rc = check_aligned(x_dev, "x_dev")) || (rc = check_aligned(work_dev, "work_dev")))
        return rc;
    if (work_bytes < carve_mdn_work(rows, nullptr, nullptr, nullptr))
        return fail(CMH_EINVAL, "work buffer too small");
    cmh::MdnBuffers B;
    float *grad = nullptr;
    carve_mdn_work(rows, (char *)work_dev, &B, &grad);
    if (loss_dev) B.loss = loss_dev;
    const MdnBlob b = mdn_blob(params_dev);
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(cmh::mdn_backward(b.params, b.hcopy, (const __bf16 *)x_dev, z_dev, rows, B, grad, s));
    HIPCHK(cmh::mdn_adam(b.params, b.hcopy, grad, step, lr, s));
    return CMH_OK;
}

int32_t cmh_mdn_pairs(const cmh_model *model, uint32_t seed, int64_t first_pair, int32_t count,
                      void *x_dev, float *z_dev, void *hip_stream)
{
    int32_t rc = check_model(model);
    if (rc) return rc;
    if (model->line || model->template_mean)
        return fail(CMH_EINVAL, "training pairs need the grid model's variance signals");
    if (count < 0 || first_pair < 0 || (count > 0 && (!x_dev || !z_dev)))
        return fail(CMH_EINVAL, "bad arguments");
    Geo g;
    model_geo(model, &g);
    HIPCHK(cmh::mdn_pairs(g, seed, first_pair, count, (__bf16 *)x_dev, z_dev,
                          (hipStream_t)hip_stream));
    return CMH_OK;
}

int32_t cmh_mdn_train(void *params_dev, const cmh_model *model, uint32_t seed, int64_t first_pair,
                      int32_t steps, int32_t rows, int32_t step0, float lr, void *x_dev,
                      float *z_dev, float *loss_dev, void *work_dev, size_t work_bytes,
                      void *hip_stream)
{
    int32_t rc = check_model(model);
    if (rc) return rc;
    if (model->line || model->template_mean)
        return fail(CMH_EINVAL, "training pairs need the grid model's variance signals");
    if ((rc = check_rows(rows))) return rc;
    if (steps < 1 || step0 < 1 || first_pair < 0)
        return fail(CMH_EINVAL, "steps and step0 count from 1, first_pair from 0");
    if (!params_dev || !x_dev || !z_dev || !work_dev) return fail(CMH_EINVAL, "NULL argument");
    if ((rc = check_aligned(x_dev, "x_dev")) || (rc = check_aligned(work_dev, "work_dev")))
        return rc;
    if (work_bytes < carve_mdn_work(rows, nullptr, nullptr, nullptr))
        return fail(CMH_EINVAL, "work buffer too small");
    Geo g;
    model_geo(model, &g);
    cmh::MdnBuffers B;
    float *grad = nullptr;
    carve_mdn_work(rows, (char *)work_dev, &B, &grad);
    const MdnBlob b = mdn_blob(params_dev);
    hipStream_t s = (hipStream_t)hip_stream;
    for (int32_t q = 0; q < steps; ++q) {
        if (loss_dev && q == steps - 1) B.loss = loss_dev;
        HIPCHK(cmh::mdn_pairs(g, seed, first_pair + (int64_t)q * rows, rows, (__bf16 *)x_dev,
                              z_dev, s));
        HIPCHK(cmh::mdn_backward(b.params, b.hcopy, (const __bf16 *)x_dev, z_dev, rows, B, grad,
                                 s));
        HIPCHK(cmh::mdn_adam(b.params, b.hcopy, grad, step0 + q, lr, s));
    }
    return CMH_OK;
}

int32_t cmh_anchor_count(const cmh_model *model, int32_t *n_anchors, int32_t *n_tau)
{
    int32_t rc = check_model(model);
    if (rc) return rc;
    if (model->line || model->template_mean)
        return fail(CMH_EINVAL, "anchors need the grid model's variance signals");
    if (model->n_samples < cmh::kMdnWin + 3)
        return fail(CMH_EINVAL, "anchors need at least 67 samples");
    const long ntau = (long)((model->n_samples - (cmh::kMdnWin + 3)) / cmh::kMdnTScale) + 1;
    const long na = (long)model->nsx * model->nsy * ntau;
    if (na > INT32_MAX) return fail(CMH_EINVAL, "more than 2^31 - 1 anchors");
    if (n_tau) *n_tau = (int32_t)ntau;
    if (n_anchors) *n_anchors = (int32_t)na;
    return CMH_OK;
}

int32_t cmh_anchor_features(const cmh_model *model, const void *trace_dev, int32_t trace_dtype,
                            int64_t first, int32_t count, void *x_dev, double *w_dev,
                            void *hip_stream)
{
    int32_t na = 0, ntau = 0;
    int32_t rc = cmh_anchor_count(model, &na, &ntau);
    if (rc) return rc;
    if (first < 0 || count < 0 || first + count > na)
        return fail(CMH_EINVAL, "anchor range outside 0 .. n_anchors");
    if (count > 0 && (!trace_dev || !x_dev || !w_dev)) return fail(CMH_EINVAL, "NULL argument");
    if (trace_dtype != CMH_F32 && trace_dtype != CMH_F64)
        return fail(CMH_EINVAL, "trace_dtype must be CMH_F32 or CMH_F64");
    Geo g;
    model_geo(model, &g);
    HIPCHK(cmh::anchor_features(g, trace_dev, trace_dtype == CMH_F64, ntau, first, count,
                                (__bf16 *)x_dev, w_dev, (hipStream_t)hip_stream));
    return CMH_OK;
}

int32_t cmh_mixture_table(const cmh_model *model, const float *head_dev, int64_t first,
                          int32_t rows, double *table_dev, void *hip_stream)
{
    int32_t na = 0, ntau = 0;
    int32_t rc = cmh_anchor_count(model, &na, &ntau);
    if (rc) return rc;
    if (first < 0 || rows < 0 || first + rows > na)
        return fail(CMH_EINVAL, "anchor range outside 0 .. n_anchors");
    if (rows > 0 && (!head_dev || !table_dev)) return fail(CMH_EINVAL, "NULL argument");
    Geo g;
    model_geo(model, &g);
    HIPCHK(cmh::mixture_table(g, ntau, first, rows, head_dev, table_dev, (hipStream_t)hip_stream));
    return CMH_OK;
}

}  // extern "C"
