// cmh_kernels.hip -- device kernels of the chromatic MH region sweep.
//
//   k_sweep_color   one colour phase (Algorithm 4's parallel loop): one
//                   workgroup per region of the colour, k MH moves each
//   k_rebin         the sweep's partition (Section 4.3.2 offset) and the
//                   move of every event into its region's id-ordered list
//   k_refresh       exact event variance and signal log-likelihood (Section 3)
//   k_simulate      forward simulator (synthetic worlds, Section 5)
//   k_draws         the per-move draw records, for inspection
#include "cmh_common.hpp"
#include "cmh_kernels.hpp"

#include <math.h>

#include <algorithm>

namespace cmh {

// ------------------------------------------------------------------ draws
// Per-move draw record under key (seed, chain), counter (sweep, region,
// move, block): [0] move-type uniform, [1] uniform a, [2] uniform b,
// [3] uniform c, [4] Exp(1), [5] [6] standard normals (Box-Muller),
// [7] log of the acceptance uniform.
__device__ inline void move_draws(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                                  uint32_t j, double out[8])
{
    uint32_t c[4];
    c[0] = sweep; c[1] = region; c[2] = j; c[3] = 0u;
    philox10(c, seed, chain);
    out[0] = unit_open(c[0], c[1]);
    out[1] = unit_open(c[2], c[3]);
    c[0] = sweep; c[1] = region; c[2] = j; c[3] = 1u;
    philox10(c, seed, chain);
    out[2] = unit_open(c[0], c[1]);
    out[3] = unit_open(c[2], c[3]);
    c[0] = sweep; c[1] = region; c[2] = j; c[3] = 2u;
    philox10(c, seed, chain);
    out[4] = -log(unit_open(c[0], c[1]));
    out[7] = log(unit_open(c[2], c[3]));
    c[0] = sweep; c[1] = region; c[2] = j; c[3] = 3u;
    philox10(c, seed, chain);
    const double u1 = unit_open(c[0], c[1]);
    const double u2 = unit_open(c[2], c[3]);
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 2.0 * M_PI * u2;
    out[5] = rad * cos(ang);
    out[6] = rad * sin(ang);
}

// Cross-lane moves within a row of 16 lanes (DPP): a double travels as two
// 32-bit halves.
template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double lane_f64(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, the same value in every lane: quad swaps, then the
// half-row and row mirrors leave each row's sum in all its lanes; the four
// row sums are read out and added in a fixed order.
__device__ inline double wave_sum(double v)
{
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Lanes 0-31 receive the value of lanes 32-63 (v_permlane32_swap exchanges
// lanes 32-63 of its first operand with lanes 0-31 of its second).
__device__ inline int upper_half(int v)
{
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    return (int)r[1];
}

__device__ inline int wave_sum_i32(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);
    return (__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16)) +
           (__builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48));
}

// Exclusive prefix sum over the lanes of a wave of a value in [0, 2^BITS):
// bit by bit, the lanes below with that bit set, counted from a ballot
// (no LDS round trip).
template <int BITS>
__device__ inline int wave_excl_prefix_small(int v)
{
    int acc = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const unsigned long long m = __ballot((v >> b) & 1);
        const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        acc += below << b;
    }
    return acc;
}

// 1 / x for the positive, well-scaled model variances: the hardware
// reciprocal refined by two Newton steps (each squares the relative error).
__device__ inline double rcp_refined(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

// Draw record of 16 for learned births: the 8 above, then [8] mixture
// uniform, [9] anchor uniform (counter block 4), [10] component uniform
// (block 5), [11..13] standard normals truncated to [-4, 4]: Box-Muller
// pairs from blocks 6, 7, ... (cosine, then sine), the first three of
// absolute value at most 4; after 16 blocks missing ones are 0.  [14], [15]
// are 0.
__device__ inline void move_draws16(uint32_t seed, uint32_t chain, uint32_t sweep,
                                    uint32_t region, uint32_t j, double out[16])
{
    move_draws(seed, chain, sweep, region, j, out);
    uint32_t c[4] = {sweep, region, j, 4u};
    philox10(c, seed, chain);
    out[8] = unit_open(c[0], c[1]);
    out[9] = unit_open(c[2], c[3]);
    c[0] = sweep; c[1] = region; c[2] = j; c[3] = 5u;
    philox10(c, seed, chain);
    out[10] = unit_open(c[0], c[1]);
    double z[3] = {0.0, 0.0, 0.0};
    int got = 0;
    for (uint32_t blk = 6; blk < 22 && got < 3; ++blk) {
        c[0] = sweep; c[1] = region; c[2] = j; c[3] = blk;
        philox10(c, seed, chain);
        const double u1 = unit_open(c[0], c[1]), u2 = unit_open(c[2], c[3]);
        const double rad = sqrt(-2.0 * log(u1));
        const double zc = rad * cos(2.0 * M_PI * u2), zs = rad * sin(2.0 * M_PI * u2);
        if (fabs(zc) <= 4.0) z[got++] = zc;
        if (got < 3 && fabs(zs) <= 4.0) z[got++] = zs;
    }
    out[11] = z[0]; out[12] = z[1]; out[13] = z[2];
    out[14] = 0.0; out[15] = 0.0;
}

// Draw record of 16 for latent arrival times: the 8 above, then [8..15]
// eight standard normals truncated to [-4, 4] (a birth's arrival offsets in
// station order; the joint move's second event takes [8], [9]): Box-Muller
// pairs from counter blocks 4, 5, ... (cosine, then sine), the first eight
// of absolute value at most 4; after blocks 4 .. 19 missing ones are 0.
__device__ inline void move_draws_arr(uint32_t seed, uint32_t chain, uint32_t sweep,
                                      uint32_t region, uint32_t j, double out[16])
{
    move_draws(seed, chain, sweep, region, j, out);
    int got = 0;
    for (uint32_t blk = 4; blk < 20 && got < 8; ++blk) {
        uint32_t c[4] = {sweep, region, j, blk};
        philox10(c, seed, chain);
        const double u1 = unit_open(c[0], c[1]), u2 = unit_open(c[2], c[3]);
        const double rad = sqrt(-2.0 * log(u1));
        const double zc = rad * cos(2.0 * M_PI * u2), zs = rad * sin(2.0 * M_PI * u2);
        if (fabs(zc) <= 4.0) out[8 + got++] = zc;
        if (got < 8 && fabs(zs) <= 4.0) out[8 + got++] = zs;
    }
    for (; got < 8; ++got) out[8 + got] = 0.0;
}

// ------------------------------------------------ latent arrivals (line model)
// Arrival time of a line-model event at (x, t) at the station at px, with
// offset eps (the arithmetic of arrive).
__device__ inline double line_arrival(const Geo &g, double x, double t, double px, double eps)
{
    const double dx = x - px;
    const double dy = 0.0 - 0.0;
    const double d = sqrt(dx * dx + dy * dy);
    return t + d / g.vel + eps;
}

// One interval of the least-squares location fit that the joint move of
// Section 3 proposes around: minimise F(x, t) = sum_j (a_j - t - |x - sx_j|
// / vel)^2.  Breakpoints are 0, the stations strictly inside (0, x_max) in
// index order, and x_max; breakpoint q is the interval's lower end, the next
// larger breakpoint its upper end.  On the interval |x - sx_j| = g_j (x -
// sx_j), g_j = +1 for stations at or left of its midpoint, else -1, so
// c_j = a_j + g_j sx_j / vel = t + g_j x / vel is a straight-line regression
// of c on g (slope x / vel; the midpoint when all g_j agree).  x is clamped
// to the interval and t is the mean of a_j - |x - sx_j| / vel.  Returns F,
// or infinity when q names no interval.  The fit is the interval with the
// smallest F, the first on ties.
__device__ inline double fit_interval(const Geo &g, const double *lsx, const double *a, int q,
                                      double *xo, double *to)
{
    const int ns = g.nsx;
    double lo = 0.0;
    bool found = q == 0;
    int cnt = 1;
    for (int j = 0; j < ns; ++j) {
        const double sj = lsx[j];
        if (sj > 0.0 && sj < g.Lx) {
            if (cnt == q) { lo = sj; found = true; }
            ++cnt;
        }
    }
    if (!found && q == cnt) { lo = g.Lx; found = true; }
    *xo = 0.0;
    *to = 0.0;
    if (!found) return INFINITY;
    double hi = INFINITY;
    for (int j = 0; j < ns; ++j) {
        const double sj = lsx[j];
        if (sj > 0.0 && sj < g.Lx && sj > lo && sj < hi) hi = sj;
    }
    if (g.Lx > lo && g.Lx < hi) hi = g.Lx;
    if (hi == INFINITY) return INFINITY;
    const double mid = 0.5 * (lo + hi);
    double gbar = 0.0, cbar = 0.0;
    for (int j = 0; j < ns; ++j) {
        const double sg = lsx[j] <= mid ? 1.0 : -1.0;
        gbar += sg;
        cbar += a[j] + sg * lsx[j] / g.vel;
    }
    gbar /= (double)ns;
    cbar /= (double)ns;
    double sgg = 0.0, sgc = 0.0;
    for (int j = 0; j < ns; ++j) {
        const double sg = lsx[j] <= mid ? 1.0 : -1.0;
        const double cj = a[j] + sg * lsx[j] / g.vel;
        const double dg = sg - gbar;
        sgg += dg * dg;
        sgc += dg * (cj - cbar);
    }
    double x = sgg > 0.0 ? g.vel * (sgc / sgg) : mid;
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    double t = 0.0;
    for (int j = 0; j < ns; ++j) t += a[j] - fabs(x - lsx[j]) / g.vel;
    t /= (double)ns;
    double f = 0.0;
    for (int j = 0; j < ns; ++j) {
        const double r = (a[j] - t) - fabs(x - lsx[j]) / g.vel;
        f += r * r;
    }
    *xo = x;
    *to = t;
    return f;
}

// LDS scratch of the joint move: the four fits' arrivals (exchanged
// arrivals of both events, then their original arrivals) and every
// interval's result.
struct JointScratch {
    double in[4][8];
    double f[4][10], x[4][10], t[4][10];
    double bx[4], bt[4];          // each fit's best interval
    double lpt[2][8], lqt[2];     // each event's terms of the ratio
    double px[2], pt[2];          // each event's proposed location and onset
    int ok[2];
};

// Stations whose position falls in region (i, kk) of a partition with
// offsets (offx, offy), in ascending index; returns their number (only the
// first `cap` are stored in sta).  Candidates are the cells around the
// region's span, one per lane of the calling wave (every lane must take
// part), membership decided by the region binning itself, compacted in
// order by a ballot.  Every lane returns the count.
__device__ inline int region_stations_wave(const Geo &g, double offx, double offy, int i, int kk,
                                           double x0, double x1, double y0, double y1, int *sta,
                                           int cap, int lane)
{
    const int ix0 = max((int)floor(x0 / g.ds - 0.5) - 1, 0);
    const int ix1 = min((int)ceil(x1 / g.ds - 0.5) + 1, g.nsx - 1);
    const int iy0 = max((int)floor(y0 / g.ds - 0.5) - 1, 0);
    const int iy1 = min((int)ceil(y1 / g.ds - 0.5) + 1, g.nsy - 1);
    const int nx = ix1 - ix0 + 1, ny = iy1 - iy0 + 1;
    int cnt = 0;
    if (nx <= 0 || ny <= 0) return 0;
    for (int c0 = 0; c0 < nx * ny; c0 += 64) {
        const int c = c0 + lane;
        bool in = false;
        int id = 0;
        if (c < nx * ny) {
            const int iy = iy0 + c / nx, ix = ix0 + c % nx;
            in = region_axis(station_pos(iy, g.ds), offy, g.wy, g.gy) == kk &&
                 region_axis(station_pos(ix, g.ds), offx, g.wx, g.gx) == i;
            id = iy * g.nsx + ix;
        }
        const unsigned long long m = __ballot(in);
        const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (in && cnt + below < cap) sta[cnt + below] = id;
        cnt += __popcll(m);
    }
    __builtin_amdgcn_wave_barrier();
    return cnt;
}

// Windows i whose anchors can put mass at time t: tau_i + reach[0] <= t <=
// tau_i + reach[1], widened by one window each side.
__device__ inline void learned_windows(const Learned &L, double t, int *ilo, int *ihi)
{
    const double a = floor((t - L.reach[1]) / 32.0) - 1.0;
    const double b = ceil((t - L.reach[0]) / 32.0) + 1.0;
    *ilo = (int)fmax(a, 0.0);
    *ihi = (int)fmin(b, (double)(L.ntau - 1));
}

// Part of sum over anchors a of the stations sta[0..ns) and windows
// [ilo, ihi] of w_a sum_k pi_k TN_k(x, y, t): (station, window, component)
// triples first, first + stride, ...  TN_k is the component's Gaussian
// truncated at 4 sd per axis and renormalised.
__device__ inline double learned_part(const Learned &L, const int *sta, int ns, int ilo, int ihi,
                                      double x, double y, double t, int first, int stride)
{
    const int nw = ihi - ilo + 1;
    double S = 0.0;
    if (nw <= 0) return S;
    const int per = nw * 8;
    for (int p = first; p < ns * per; p += stride) {
        const int q = p / per, r = p - q * per;
        const int k = r & 7;
        const long long a = (long long)sta[q] * L.ntau + ilo + (r >> 3);
        const double *T = L.tab + a * 64 + 8 * k;
        const double ux = (x - T[0]) / T[3];
        const double uy = (y - T[1]) / T[4];
        const double ut = (t - T[2]) / T[5];
        if (fabs(ux) <= 4.0 && fabs(uy) <= 4.0 && fabs(ut) <= 4.0)
            S += L.w[a] * exp(L.norm[a * 8 + k] - 0.5 * (ux * ux + uy * uy + ut * ut));
    }
    return S;
}

// log(b / p_R) for the birth density b = (1 - pl) p_R + pl q_R, given the
// anchor sum S and the region's total anchor weight W.
__device__ inline double learned_log_ratio(double pl, double S, double W, double area, int N)
{
    return log((1.0 - pl) + pl * (S / W) * area * (double)N);
}

// One run of affected samples at one station: samples [lo, lo + len); the
// old event's window [o0, o1) with scale Bo and the new event's window
// [w0, w1) with scale Bn.  Runs are laid end to end in flat positions in
// their order in the table.
struct Seg {
    int j, lo, len, pad;
    int o0, o1, w0, w1;
    double Bo, Bn;
};

// Flat start of every run of a move's footprint and its global base (the
// station's row offset plus the run's first sample, minus the flat start),
// so that flat position f inside run t is sample gb[t] + f of E and the trace.
struct __attribute__((aligned(16))) SegIndex {
    int fs[kMaxSeg];
    int gb[kMaxSeg];
};

// Flat footprint positions f0 + q stride (q < Q): the run holding each and
// its global sample index (-1 past the footprint's S samples).  Run starts
// are read four at a time and compared without a data-dependent branch.
template <int Q>
__device__ inline void locate_runs(const SegIndex &six, int nseg, int S, int f0, int stride,
                                   int *run, int *gidx)
{
    // runs start at non-decreasing flat positions (fs[0] = 0), so the run of
    // position f is the number of runs starting at or before f, minus one
    int cnt[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) cnt[q] = 0;
    for (int t0 = 0; t0 < nseg; t0 += 4) {
        const int4 a = *(const int4 *)&six.fs[t0];
        const int fa[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool in = t0 + u < nseg;  // the same in every lane
#pragma unroll
            for (int q = 0; q < Q; ++q) cnt[q] += (in && fa[u] <= f0 + q * stride) ? 1 : 0;
        }
    }
    int gb[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {  // every table read issued before any is used
        run[q] = cnt[q] > 0 ? cnt[q] - 1 : 0;
        gb[q] = six.gb[run[q]];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int f = f0 + q * stride;
        gidx[q] = f < S ? gb[q] + f : -1;
    }
}

// Change of the event variance at sample nn of run a: the new event's
// contribution minus the old event's, envelope from the table sT.
__device__ inline double run_dvar(const Seg &a, const double *sT, int nn)
{
    const bool io = nn >= a.o0 && nn < a.o1;
    const bool iw = nn >= a.w0 && nn < a.w1;
    const double co = io ? a.Bo * sT[io ? nn - a.o0 : 0] : 0.0;
    const double cn = iw ? a.Bn * sT[iw ? nn - a.w0 : 0] : 0.0;
    return cn - co;
}

// One sample's share of the log-likelihood change, accumulated as
// -1/2 [log(prod v'/v) - sum s^2 (v' - v) / (v v')], v = sigma^2 + E (the
// Gaussian log density of Section 3 differenced); returns the new E.
__device__ inline double sample_term(double sigma2, double e0, double dc, double s, double *prod,
                                     double *lin)
{
    double en = e0 + dc;
    en = en > 0.0 ? en : 0.0;
    const double de = en - e0;
    const double v = sigma2 + e0, vp = sigma2 + en;
    const double inv = rcp_refined(v * vp);
    *prod *= de != 0.0 ? vp * vp * inv : 1.0;
    *lin += s * s * de * inv;
    return en;
}

// Mean-template likelihood: one sample's share of sum g (r - g / 2) (to be
// divided by sigma^2), g the change of the mean and r the residual s - mean
// before the move; returns the new residual.
__device__ inline double template_term(double r, double g, double *lin)
{
    *lin += g * (r - 0.5 * g);
    return r - g;
}

struct MoveHdr {
    int valid, type, n, nseg, S;
    int flags;  // error flags, raised only when the move is consumed
    double dm;  // magnitude change (magnitude move)
    double lr;  // learned births: log(b / p_R) at the born or dying event
    double lx;  // latent arrivals: prior and proposal part of log alpha (moves 5, 6)
};

// A region's learned-birth constants, staged in LDS by the sweep workgroup.
struct RegionLearned {
    int ns;          // stations in the region (at most kMaxRegSta)
    double W, pl;    // their total anchor weight; mixing probability (0: plain)
    double area;
};

// A region's learned-birth constants, computed by one whole wave (every lane
// takes part and gets the same value): its stations into sta, and W, the
// running total of their anchors' weights in station order (loads one per
// lane, additions in order).  *over: more than kMaxRegSta stations (the
// region is then taken as plain).
__device__ inline RegionLearned region_learned_wave(const Geo &g, const Learned &L, double offx,
                                                    double offy, int i, int kk, double x0,
                                                    double x1, double y0, double y1, double area,
                                                    int *sta, int lane, bool *over)
{
    RegionLearned rl;
    rl.ns = 0; rl.W = 0.0; rl.pl = 0.0; rl.area = area;
    *over = false;
    if (L.tab == nullptr) return rl;
    const int ns = region_stations_wave(g, offx, offy, i, kk, x0, x1, y0, y1, sta, kMaxRegSta,
                                        lane);
    if (ns > kMaxRegSta) {
        *over = true;
    } else if (ns > 0) {
        const double tot = lane < ns ? L.cum[(long long)sta[lane] * L.ntau + L.ntau - 1] : 0.0;
        double W = 0.0;
        for (int q = 0; q < ns; ++q) W = W + lane_f64(tot, q);
        rl.ns = ns; rl.W = W; rl.pl = L.pl;
    }
    return rl;
}

// x lies in region index `want` of one axis.  Points further than 1e-9 w
// from both edges of the region's interval are decided by comparison (the
// floor in region_axis cannot differ there); the rest by region_axis itself.
__device__ inline bool in_region_axis(double x, double lo, double hi, double off, double w, int g,
                                      int want)
{
    const double eps = 1e-9 * w;
    if (x > lo + eps && x < hi - eps) return true;
    return region_axis(x, off, w, g) == want;
}

// A region's extent and prior mean count Lambda_R.  On the grid: its
// rectangle [x0, x1) x [y0, y1).  In the line model: the whole line
// [x0, x1) = [0, x_max) and the region's onset interval [y0, y1) (time is the
// partition axis there).
struct RegionBox {
    double x0, x1, y0, y1, area, lamR;
};

__device__ inline RegionBox region_box(const Geo &g, double offx, double offy, int i, int kk)
{
    RegionBox b;
    if (g.line) {
        b.x0 = 0.0;
        b.x1 = g.Lx;
        region_span(offx, g.wx, (double)g.N, i, &b.y0, &b.y1);
        b.area = b.y1 - b.y0;
        b.lamR = g.lambda * b.area / (double)g.N;
    } else {
        region_span(offx, g.wx, g.Lx, i, &b.x0, &b.x1);
        region_span(offy, g.wy, g.Ly, kk, &b.y0, &b.y1);
        b.area = (b.x1 - b.x0) * (b.y1 - b.y0);
        b.lamR = g.lambda * b.area / (g.Lx * g.Ly);
    }
    return b;
}

// Footprint of a move, computed by the 64 lanes of wave 0: every station
// within the detection cutoff of the old or the new event, with the union of
// their sample windows.  Candidate stations are the cells around both events;
// lanes 0-31 evaluate the old event's arrival at candidate `lane`, lanes
// 32-63 the new event's at candidate `lane - 32`, so the two arrival
// computations run side by side.  A wave prefix sum then places each
// candidate's one or two sample runs.  CLIP (latent arrivals, which can
// precede the trace): windows are cut at sample 0, and one that ends there
// is absent.
template <bool CLIP = false>
__device__ __forceinline__ void footprint(const Geo &g, int lane, bool has_old, double ox, double oy, double ot,
                          double om, bool has_new, double nx, double ny, double nt, double nm,
                          Seg *segs, SegIndex *six, const double *lsx, int *nseg_out, int *S_out,
                          int *flags, const double *oda = nullptr, const double *nda = nullptr)
{
    // candidate cells: the events' cells (by a product with 1 / ds: at a cell
    // edge the cell may be off by one, and the one-cell margin still holds
    // every station within rc < ds) widened by one cell
    int cx0 = 1 << 30, cx1 = -1, cy0 = 1 << 30, cy1 = -1;
    if (has_old) {
        const int cx = (int)floor(ox * g.inv_ds), cy = (int)floor(oy * g.inv_ds);
        cx0 = min(cx0, cx); cx1 = max(cx1, cx); cy0 = min(cy0, cy); cy1 = max(cy1, cy);
    }
    if (has_new) {
        const int cx = (int)floor(nx * g.inv_ds), cy = (int)floor(ny * g.inv_ds);
        cx0 = min(cx0, cx); cx1 = max(cx1, cx); cy0 = min(cy0, cy); cy1 = max(cy1, cy);
    }
    cx0 = max(cx0 - 1, 0); cy0 = max(cy0 - 1, 0);
    cx1 = min(cx1 + 1, g.nsx - 1); cy1 = min(cy1 + 1, g.nsy - 1);
    if (g.line) {  // every station of the line
        cx0 = 0; cx1 = g.nsx - 1; cy0 = 0; cy1 = 0;
    }
    const int bw = cx1 - cx0 + 1;
    const int nbox = bw * (cy1 - cy0 + 1);
    // row of a candidate: (cidx + 1/2) / bw lies at least 1 / (2 bw) from an
    // integer, beyond the error of a float reciprocal for cidx < 2^16 and
    // bw <= 2^12 (checked exhaustively); larger boxes divide
    const float rbw = __builtin_amdgcn_rcpf((float)bw);
    const bool small_box = nbox < (1 << 16) && bw <= (1 << 12);
    const int half = lane >> 5, hl = lane & 31;
    const bool mine = half == 0 ? has_old : has_new;
    const double ex = half ? nx : ox, ey = half ? ny : oy, et = half ? nt : ot,
                 em = half ? nm : om;
    int seg_base = 0, samp_base = 0;
    for (int c0 = 0; c0 < nbox; c0 += 32) {
        const int cidx = c0 + hl;
        Arrival ar;
        ar.in = 0; ar.n0 = 0; ar.n1 = 0; ar.B = 0.0;
        int ix = 0, iy = 0;
        if (cidx < nbox) {
            const int row = small_box ? (int)(((float)cidx + 0.5f) * rbw) : cidx / bw;
            ix = cx0 + (cidx - row * bw);
            iy = cy0 + row;
            // line stations from lsx (LDS): a Geo held in registers must not
            // be indexed dynamically, which would move it to scratch memory
            if (mine) {
                // latent arrivals: the event's offset at this station (LDS)
                const double *eda = half ? nda : oda;
                ar = arrive(g, ex, ey, et, em, g.line ? lsx[ix] : station_pos(ix, g.ds),
                            g.line ? 0.0 : station_pos(iy, g.ds), eda != nullptr ? eda[ix] : 0.0);
            }
        }
        // lanes 0-31 take the new event's arrival from their partner lane
        // (the two halves of the wave swapped in registers)
        Arrival an;
        an.in = upper_half(ar.in);
        an.n0 = upper_half(ar.n0);
        an.n1 = upper_half(ar.n1);
        an.B = __hiloint2double(upper_half(__double2hiint(ar.B)), upper_half(__double2loint(ar.B)));
        Arrival ao = ar;
        if (CLIP) {
            ao.in = ao.in && ao.n1 > 0;
            an.in = an.in && an.n1 > 0;
        }
        int ns = 0, nsamp = 0;
        Seg sa, sb;
        if (half == 0 && cidx < nbox && (ao.in || an.in)) {
            const int j = iy * g.nsx + ix;
            sa.j = j;
            sa.o0 = ao.in ? ao.n0 : 0; sa.o1 = ao.in ? ao.n1 : 0;
            sa.w0 = an.in ? an.n0 : 0; sa.w1 = an.in ? an.n1 : 0;
            sa.Bo = ao.B; sa.Bn = an.B;
            sb = sa;
            // the runs start at the first sample of the trace at the
            // earliest (o0 and w0 keep the arrival's own first sample)
            const int ob = CLIP ? max(ao.n0, 0) : ao.n0, nb = CLIP ? max(an.n0, 0) : an.n0;
            if (ao.in && an.in) {
                if (max(ob, nb) <= min(ao.n1, an.n1)) {  // overlapping or touching
                    sa.lo = min(ob, nb);
                    sa.len = max(ao.n1, an.n1) - sa.lo;
                    ns = 1;
                } else {                                   // disjoint, sample order
                    sa.lo = min(ob, nb);
                    sa.len = (ob < nb ? ao.n1 : an.n1) - sa.lo;
                    sb.lo = max(ob, nb);
                    sb.len = (ob < nb ? an.n1 : ao.n1) - sb.lo;
                    ns = 2;
                }
            } else if (ao.in) {
                sa.lo = ob; sa.len = ao.n1 - ob; ns = 1;
            } else {
                sa.lo = nb; sa.len = an.n1 - nb; ns = 1;
            }
            nsamp = sa.len + (ns == 2 ? sb.len : 0);
        }
        const unsigned long long m1 = __ballot(ns >= 1), m2 = __ballot(ns == 2);
        const unsigned long long below = (1ull << lane) - 1ull;
        const int sbase = seg_base + __popcll(m1 & below) + __popcll(m2 & below);
        static_assert(2 * kMaxTs < (1 << 9), "a candidate's samples fit in 9 bits");
        const int fpos = samp_base + wave_excl_prefix_small<9>(nsamp);
        if (ns >= 1) {
            if (sbase + ns <= kMaxSeg) {
                segs[sbase] = sa;
                six->fs[sbase] = fpos;
                six->gb[sbase] = sa.j * g.N + sa.lo - fpos;
                if (ns == 2) {
                    segs[sbase + 1] = sb;
                    six->fs[sbase + 1] = fpos + sa.len;
                    six->gb[sbase + 1] = sb.j * g.N + sb.lo - (fpos + sa.len);
                }
            } else {
                *flags |= kFlagSeg;
            }
        }
        seg_base += __popcll(m1) + __popcll(m2);
        samp_base += wave_sum_i32(nsamp);
    }
    *nseg_out = seg_base;
    *S_out = samp_base;
}

// ------------------------------------------------------------ sweep colour
// Latent arrivals' per-move LDS of the latency form: the proposed offsets of
// the (up to two) changed events, the joint move's second event (x, t,
// index), and the joint move's fit scratch.
struct LatentLds {
    double pda[2][2][8];
    double prop2[2][3];
    JointScratch js;
};

// Debug owner tag of region r = (i, kk) in its colour phase of a sweep; the
// region's colour is (i mod p) + p (kk mod p) (i mod p on the line).
__device__ inline unsigned long long owner_tag(const Geo &g, long long sweep, int i, int kk, int r)
{
    const long long colour = (long long)(i % g.period) + (long long)g.period * (kk % g.period);
    return ((unsigned long long)(sweep * g.ncolors + colour + 1) << 16) | (unsigned long long)r;
}

// Wave 0 of a sweep workgroup ("scout"): builds move jj's proposal from its
// draws and the region's current events, and its footprint, into buffer
// `buf`.  Lane 0 owns the event table; the other lanes help with the
// footprint.  LAT: latent arrival times (line model), with the arrival-time
// move (type 5) and the joint two-event move (type 6); d2 holds draws 8..15
// and s_da the events' offsets.
template <bool LAT>
__device__ inline void scout_move(const Geo &g, int lane, int buf, int i, int kk, double offx,
                                  double offy, double x0, double x1, double y0, double y1, int n,
                                  const double *d, const double *s_ex, const double *s_ey,
                                  const double *s_et, const double *s_em, Seg (*s_seg)[kMaxSeg],
                                  SegIndex *s_six, const double *lsx, MoveHdr *s_hdr, double (*s_prop)[5], int max_samples,
                                  const Learned &L, const double *lb, const int *lsta,
                                  const RegionLearned &rl, const double *d2 = nullptr,
                                  const double (*s_da)[8] = nullptr, LatentLds *lat = nullptr,
                                  unsigned long long *own = nullptr, unsigned long long tag = 0)
{
    int type = 0, valid = 0, idx = -1, mflags = 0;
    double ox = 0, oy = 0, ot = 0, om = 0, nx = 0, ny = 0, nt = 0, nm = 0, lr = 0, lx = 0;
    int idx2 = -1, split = 0;
    if (lane == 0) {
        const double u = d[0];
        type = u < g.c1 ? 0 : u < g.c2 ? 1 : u < g.c3 ? 2 : u < g.c4 ? 3 : 4;
        if (LAT && type == 4 && !(u < g.c5)) type = u < g.c6 ? 5 : 6;
        if (LAT) {  // the new event's offsets start as the old one's (or none)
            double *pd = lat->pda[buf][0];
            for (int q = 0; q < 8; ++q) pd[q] = 0.0;
        }
        if (type == 0) {
            if (n >= g.cap) {
                mflags |= kFlagCap;
            } else if (g.line) {  // [y0, y1) is the region's onset interval
                nx = d[1] * g.Lx;
                ny = 0.0;
                nt = y0 + d[3] * (y1 - y0);
                nm = g.mmin;
                valid = nx >= 0.0 && nx < g.Lx && nt >= 0.0 && nt < (double)g.N &&
                        in_region_axis(nt, y0, y1, offx, g.wx, g.gx, i);
                if (LAT)  // offsets from their prior: arrival_sd times truncated normals
                    for (int q = 0; q < g.nsx; ++q) lat->pda[buf][0][q] = g.arr_sd * d2[q];
            } else {
                if (L.tab != nullptr) {  // derived for the sweep by the draw kernel
                    nx = lb[0]; ny = lb[1]; nt = lb[2]; lr = lb[3];
                } else {
                    nx = x0 + d[1] * (x1 - x0);
                    ny = y0 + d[2] * (y1 - y0);
                    nt = d[3] * (double)g.N;
                }
                nm = g.mmin + d[4] / g.mrate;
                valid = nx >= 0.0 && nx < g.Lx && ny >= 0.0 && ny < g.Ly && nt >= 0.0 &&
                        nt < (double)g.N && in_region_axis(nx, x0, x1, offx, g.wx, g.gx, i) &&
                        in_region_axis(ny, y0, y1, offy, g.wy, g.gy, kk);
            }
        } else if (LAT && type == 6) {
            // joint move: the pair and the station split; the arrivals to
            // fit go to LDS for the wave
            if (n >= 2 && g.nsx >= 2) {
                idx = (int)floor(d[1] * (double)n);
                if (idx >= n) idx = n - 1;
                idx2 = (int)floor(d[2] * (double)(n - 1));
                if (idx2 >= n - 1) idx2 = n - 2;
                if (idx2 >= idx) idx2 += 1;
                split = 1 + (int)floor(d[3] * (double)(g.nsx - 1));
                if (split >= g.nsx) split = g.nsx - 1;
                valid = s_em[idx] == s_em[idx2];
                if (valid)
                    for (int q = 0; q < g.nsx; ++q) {
                        const double ai = line_arrival(g, s_ex[idx], s_et[idx], lsx[q], s_da[idx][q]);
                        const double ak = line_arrival(g, s_ex[idx2], s_et[idx2], lsx[q], s_da[idx2][q]);
                        lat->js.in[0][q] = q >= split ? ak : ai;
                        lat->js.in[1][q] = q >= split ? ai : ak;
                        lat->js.in[2][q] = ai;
                        lat->js.in[3][q] = ak;
                    }
            }
        } else if (n > 0) {
            idx = (int)floor(d[1] * (double)n);
            if (idx >= n) idx = n - 1;
            ox = s_ex[idx]; oy = s_ey[idx]; ot = s_et[idx]; om = s_em[idx];
            nx = ox; ny = oy; nt = ot; nm = om;
            valid = 1;
            if (LAT) {  // carried along by location and onset moves
                double *pd = lat->pda[buf][0];
                for (int q = 0; q < 8; ++q) pd[q] = s_da[idx][q];
            }
            if (LAT && type == 5) {
                // arrival-time move: one station's offset takes a Gaussian
                // step; its prior density enters the ratio
                int js = (int)floor(d[2] * (double)g.nsx);
                if (js >= g.nsx) js = g.nsx - 1;
                const double o = s_da[idx][js];
                const double w = o + g.sa * d[5];
                lat->pda[buf][0][js] = w;
                valid = fabs(w) <= g.arr_e;
                lx = (o * o - w * w) / g.arr_2v;
            } else if (g.line) {  // location moves keep the region; onset moves must
                if (type == 2) {
                    nx = ox + g.sxy * d[5];
                    valid = nx >= 0.0 && nx < g.Lx;
                } else if (type == 3) {
                    nt = ot + g.st * d[5];
                    valid = nt >= 0.0 && nt < (double)g.N &&
                            in_region_axis(nt, y0, y1, offx, g.wx, g.gx, i);
                } else if (type == 4) {
                    valid = 0;  // fixed amplitude
                }
            } else if (type == 2) {
                nx = ox + g.sxy * d[5];
                ny = oy + g.sxy * d[6];
                valid = nx >= 0.0 && nx < g.Lx && ny >= 0.0 && ny < g.Ly &&
                        in_region_axis(nx, x0, x1, offx, g.wx, g.gx, i) &&
                        in_region_axis(ny, y0, y1, offy, g.wy, g.gy, kk);
            } else if (type == 3) {
                nt = ot + g.st * d[5];
                valid = nt >= 0.0 && nt < (double)g.N;
            } else if (type == 4) {
                nm = om + g.sm * d[5];
                valid = nm >= g.mmin;
            }
        }
    }
    type = __builtin_amdgcn_readlane(type, 0);
    valid = __builtin_amdgcn_readlane(valid, 0);
    if (LAT && type == 6 && valid) {
        // the four least-squares fits, one interval per lane; then one lane
        // per event builds its proposal around the fit of its exchanged
        // arrivals, and lane 0 sums the ratio's terms
        __builtin_amdgcn_wave_barrier();
        JointScratch &js = lat->js;
        if (lane < 40) {
            const int f = lane / 10, q = lane % 10;
            double fx, ft;
            const double F = fit_interval(g, lsx, js.in[f], q, &fx, &ft);
            js.f[f][q] = F;
            js.x[f][q] = fx;
            js.t[f][q] = ft;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < 4) {  // fit `lane`: its best interval, the first on ties
            double best = INFINITY, bx = 0.0, bt = 0.0;
            for (int q = 0; q < 10; ++q)
                if (js.f[lane][q] < best) {
                    best = js.f[lane][q];
                    bx = js.x[lane][q];
                    bt = js.t[lane][q];
                }
            js.bx[lane] = bx;
            js.bt[lane] = bt;
        }
        __builtin_amdgcn_wave_barrier();
        const int pi0 = __builtin_amdgcn_readlane(idx, 0), pi1 = __builtin_amdgcn_readlane(idx2, 0);
        if (lane < 2) {
            // event `lane` of the pair: a Gaussian step around the fit of its
            // exchanged arrivals, offsets that keep those arrivals, and its
            // terms of the ratio (the reverse move centres on the fit of its
            // original arrivals, fit 2 + lane)
            const int e = lane, ie = e ? pi1 : pi0;
            const double zx = e ? d2[0] : d[5], zt = e ? d2[1] : d[6];
            const double px = js.bx[e] + g.sxy * zx, pt = js.bt[e] + g.st * zt;
            int ok = px >= 0.0 && px < g.Lx && pt >= 0.0 && pt < (double)g.N &&
                     in_region_axis(pt, y0, y1, offx, g.wx, g.gx, i);
            double *pd = lat->pda[buf][e];
            for (int q = 0; q < 8; ++q) pd[q] = 0.0;
            for (int q = 0; q < g.nsx && ok; ++q) {
                const double target = js.in[e][q];
                const double w = target - line_arrival(g, px, pt, lsx[q], 0.0);
                pd[q] = w;
                // the offset stays in its support, and the window starts at
                // the sample of the arrival it takes over
                ok = fabs(w) <= g.arr_e && ceil(line_arrival(g, px, pt, lsx[q], w)) == ceil(target);
            }
            for (int q = 0; q < g.nsx; ++q) {
                const double o = s_da[ie][q], w = pd[q];
                js.lpt[e][q] = (o * o - w * w) / g.arr_2v;
            }
            const double rx = (s_ex[ie] - js.bx[2 + e]) / g.sxy;
            const double rt = (s_et[ie] - js.bt[2 + e]) / g.st;
            js.lqt[e] = 0.5 * (zx * zx + zt * zt) - 0.5 * (rx * rx + rt * rt);
            js.px[e] = px;
            js.pt[e] = pt;
            js.ok[e] = ok;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            valid = js.ok[0] && js.ok[1];
            if (valid) {  // the terms summed in event, then station order
                double lp = 0.0, lq = 0.0;
                for (int e = 0; e < 2; ++e)
                    for (int q = 0; q < g.nsx; ++q) lp += js.lpt[e][q];
                for (int e = 0; e < 2; ++e) lq += js.lqt[e];
                lx = lp + lq;
                nx = js.px[0]; ny = 0.0; nt = js.pt[0]; nm = s_em[idx];
                ox = s_ex[idx]; ot = s_et[idx]; om = nm;
                lat->prop2[buf][0] = js.px[1];
                lat->prop2[buf][1] = js.pt[1];
                lat->prop2[buf][2] = (double)idx2;
            }
        }
        valid = __builtin_amdgcn_readlane(valid, 0);
    }
    if (type == 1 && valid && rl.pl > 0.0) {
        // death under learned births: the birth density at the dying event,
        // (station, window) pairs spread over the lanes
        const double ex = lane_f64(ox, 0), ey = lane_f64(oy, 0), et = lane_f64(ot, 0);
        int ilo, ihi;
        learned_windows(L, et, &ilo, &ihi);
        const double S = wave_sum(learned_part(L, lsta, rl.ns, ilo, ihi, ex, ey, et, lane, 64));
        lr = learned_log_ratio(rl.pl, S, rl.W, rl.area, g.N);
    }
    int nseg = 0, S = 0;
    // the joint move leaves every station's set of signals unchanged: no
    // footprint, a likelihood change of zero
    if (valid && !g.prior_only && !(LAT && type == 6)) {
        ox = lane_f64(ox, 0); oy = lane_f64(oy, 0);
        ot = lane_f64(ot, 0); om = lane_f64(om, 0);
        nx = lane_f64(nx, 0); ny = lane_f64(ny, 0);
        nt = lane_f64(nt, 0); nm = lane_f64(nm, 0);
        int fl = 0;
        const double *oda = nullptr, *nda = nullptr;
        if (LAT) {
            __builtin_amdgcn_wave_barrier();  // lane 0's offsets are in LDS
            const int io = __builtin_amdgcn_readlane(idx, 0);
            oda = type != 0 ? s_da[io] : nullptr;
            nda = type != 1 ? lat->pda[buf][0] : nullptr;
        }
        footprint<LAT>(g, lane, type != 0, ox, oy, ot, om, type != 1, nx, ny, nt, nm, s_seg[buf],
                       &s_six[buf], lsx, &nseg, &S, &fl, oda, nda);
        if (__ballot(fl != 0) != 0ull || S > max_samples) {
            valid = 0;
            mflags |= kFlagSeg;
        }
    }
    if (own != nullptr && valid && nseg > 0) {
        // debug owner check: every sample the move reads (and, if accepted,
        // writes) takes this region's tag; another region's tag of this
        // phase means the colouring let two regions share the sample
        __builtin_amdgcn_wave_barrier();
        int race = 0;
        for (int t = 0; t < nseg; ++t) {
            const Seg &sg = s_seg[buf][t];
            unsigned long long *row = own + (long long)sg.j * g.N + sg.lo;
            for (int f = lane; f < sg.len; f += 64) {
                const unsigned long long old = atomicExch(row + f, tag);
                race |= (old >> 16) == (tag >> 16) && old != tag;
            }
        }
        if (__ballot(race != 0) != 0ull) mflags |= kFlagRace;
    }
    if (lane == 0) {
        MoveHdr h;
        h.valid = valid; h.type = type; h.n = n; h.nseg = nseg; h.S = S; h.flags = mflags;
        h.dm = nm - om;
        h.lr = lr;
        h.lx = lx;
        s_hdr[buf] = h;
        s_prop[buf][0] = nx; s_prop[buf][1] = ny; s_prop[buf][2] = nt; s_prop[buf][3] = nm;
        s_prop[buf][4] = (double)idx;
    }
}

// One workgroup per work item (slot, region) of one colour; k MH moves in
// sequence (Algorithm 4's inner loop).
//   Wave 0 (scout) builds each move's proposal and footprint.  While the
//   other waves evaluate move j it already builds move j + 1 on the
//   assumption that move j is rejected (the state is then unchanged); after
//   an acceptance it rebuilds move j + 1 from the updated events.  The chain
//   of states is exactly the sequential one.
//   Waves 1.. (evaluators) evaluate the log-likelihood change on a strided
//   share of the footprint samples: every load issued before any arithmetic,
//   one division per sample and one logarithm per thread (of the product of
//   the variance ratios); on acceptance they write the new event variance in
//   place.
// The event variance of other regions is read but never written: the
// colouring guarantees that no station is reached from two regions of one
// colour (the Markov-blanket argument of Section 4.1).
// LAT: latent arrival times (line model): the events' offsets live in LDS
// next to their coordinates, draws 8..15 come from the slot's draws2, and
// the scout also builds arrival-time and joint moves.
template <typename TraceT, int BLOCK, bool LAT, bool OWN = false>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(LAT ? 2 : 1)))
k_sweep_color(const Slot *__restrict__ slots, const unsigned *__restrict__ items, int par,
              const long long *__restrict__ sweep_ptr, double *__restrict__ logp,
              long long log_first, long long log_n, int *__restrict__ err, StampArg sa)
{
    static_assert(BLOCK >= 128 && BLOCK % 64 == 0, "one scout wave and at least one evaluator");
    constexpr int W = BLOCK / 64;
    constexpr int EV = BLOCK - 64;
    constexpr int QP = 4;  // footprint positions per evaluator thread per pass
    __shared__ double s_draw[2][kDrawChunk][8];
    __shared__ double s_lb[2][kDrawChunk][4];
    __shared__ int s_lsta[kMaxRegSta];
    __shared__ RegionLearned s_rl;
    __shared__ double s_T[kMaxTs];
    __shared__ double s_log[kMaxCap + 2];  // s_log[q] = log(q)
    __shared__ double s_ex[kMaxCap], s_ey[kMaxCap], s_et[kMaxCap], s_em[kMaxCap];
    __shared__ unsigned long long s_id[kMaxCap];
    __shared__ Seg s_seg[2][kMaxSeg];
    __shared__ SegIndex s_six[2];
    __shared__ double s_lsx[8];  // line model: station positions
    __shared__ MoveHdr s_hdr[2];
    __shared__ double s_prop[2][5];
    __shared__ double s_part[2][W];
    __shared__ int s_n;
    // latent arrivals only (one-element stand-ins when LAT is false)
    __shared__ double s_draw2[LAT ? 2 : 1][LAT ? kDrawChunk : 1][8];
    __shared__ double s_da[LAT ? kMaxCap : 1][8];
    __shared__ LatentLds s_lat[1];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned item = items[blockIdx.x];
    const int slot = (int)(item >> 16), r = (int)(item & 0xFFFFu);
    const Geo g = slots[slot].g;
    const Events ev = slots[slot].ev[par];
    const TraceT *__restrict__ trace = (const TraceT *)slots[slot].trace;
    double *__restrict__ E = slots[slot].E;
    const double *__restrict__ draws = slots[slot].draws;
    unsigned long long *__restrict__ stats = slots[slot].stats;
    const Learned L = slots[slot].L;
    const int chain = 0;  // every array of the slot is slot-local
    const int i = r % g.nrx, kk = r / g.nrx;
    const long long sweep = *sweep_ptr;
    if (tid == 0) stamp_at(sa, sweep, 0);
    // debug owner check (OWN: a separate instantiation, so production
    // kernels carry none of it)
    unsigned long long *const own = OWN ? slots[slot].owner : nullptr;
    const unsigned long long tag = OWN ? owner_tag(g, sweep, i, kk, r) : 0ull;

    const double offx = ev.off[2 * chain], offy = ev.off[2 * chain + 1];
    const RegionBox box = region_box(g, offx, offy, i, kk);
    const double x0 = box.x0, x1 = box.x1, y0 = box.y0, y1 = box.y1, area = box.area;
    if (!(area > 0.0)) return;
    const double lamR = box.lamR;
    const double log_lamR = log(lamR), log_pb = log(g.pb), log_pd = log(g.pd);

    const long long base = ((long long)chain * g.R + r) * g.cap;
    const long long ebase = (long long)chain * g.nsta * (long long)g.N;
    // E and the trace as global pointers: their loads are then counted apart
    // from LDS operations
    const __attribute__((address_space(1))) double *const gE =
        (const __attribute__((address_space(1))) double *)(E + ebase);
    const __attribute__((address_space(1))) TraceT *const gT =
        (const __attribute__((address_space(1))) TraceT *)trace;
    __attribute__((address_space(1))) double *const gEw =
        (__attribute__((address_space(1))) double *)(E + ebase);
    const double *dsrc = draws + ((long long)chain * g.R + r) * (long long)g.k * 8;
    const double *lsrc =
        L.tab != nullptr ? L.birth + ((long long)chain * g.R + r) * (long long)g.k * 4 : nullptr;
    int n = ev.cnt[chain * g.R + r];
    for (int s = tid; s < n; s += BLOCK) {
        s_ex[s] = ev.x[base + s]; s_ey[s] = ev.y[base + s];
        s_et[s] = ev.t[base + s]; s_em[s] = ev.m[base + s];
        s_id[s] = ev.id[base + s];
    }
    const double *dsrc2 = nullptr;
    if constexpr (LAT) {
        for (int q = tid; q < n * 8; q += BLOCK) s_da[q >> 3][q & 7] = ev.da[base * 8 + q];
        dsrc2 = slots[slot].draws2 + ((long long)chain * g.R + r) * (long long)g.k * 8;
    }
    for (int q = tid; q < g.ts; q += BLOCK) s_T[q] = exp(-(g.tmpl ? 1.0 : 2.0) * (double)q / g.decay);
    for (int q = tid; q < kMaxCap + 2; q += BLOCK) s_log[q] = log((double)q);
    if (tid < 8) s_lsx[tid] = slots[slot].g.sx[tid];
    for (int c = 0; c < 2 && 64 * c < g.k; ++c) {
        const int m = min(kDrawChunk, g.k - 64 * c) * 8;
        for (int q = tid; q < m; q += BLOCK) s_draw[c][q >> 3][q & 7] = dsrc[64LL * 8 * c + q];
        if constexpr (LAT)
            for (int q = tid; q < m; q += BLOCK) s_draw2[c][q >> 3][q & 7] = dsrc2[64LL * 8 * c + q];
        if (lsrc != nullptr)
            for (int q = tid; q < m / 2; q += BLOCK)
                s_lb[c][q >> 2][q & 3] = lsrc[64LL * 4 * c + q];
    }
    int flags = 0;
    if (tid < 64) {  // the first wave
        bool over = false;
        const RegionLearned rl = region_learned_wave(g, L, offx, offy, i, kk, x0, x1, y0, y1,
                                                     area, s_lsta, tid, &over);
        if (tid == 0) {
            if (over) flags |= kFlagSta;
            s_rl = rl;
        }
    }

    const bool use_log = logp != nullptr && slot == 0 && sweep >= log_first &&
                         sweep < log_first + log_n;
    constexpr int NT = LAT ? 7 : 5;  // move types
    unsigned int cnt_att[NT] = {}, cnt_val[NT] = {}, cnt_acc[NT] = {};
    unsigned long long samp_read = 0, samp_written = 0;
    __syncthreads();
    const RegionLearned rl = s_rl;
    if (wave == 0) {
        scout_move<LAT>(g, lane, 0, i, kk, offx, offy, x0, x1, y0, y1, n, s_draw[0][0], s_ex,
                        s_ey, s_et, s_em, s_seg, s_six, s_lsx, s_hdr, s_prop, kMaxFootprint, L,
                        s_lb[0][0], s_lsta, rl, LAT ? s_draw2[0][0] : nullptr, s_da, s_lat, own,
                        tag);
    }
    __syncthreads();

    for (int j = 0; j < g.k; ++j) {
        const int buf = j & 1;
        // moves 128, 192, ... start a chunk whose buffer held moves 128 earlier
        if (((j + 1) & 63) == 0 && j + 1 < g.k && j + 1 >= 128) {
            const int c = (j + 1) >> 6;
            const int m = min(kDrawChunk, g.k - (j + 1)) * 8;
            for (int q = tid; q < m; q += BLOCK)
                s_draw[c & 1][q >> 3][q & 7] = dsrc[(long long)(j + 1) * 8 + q];
            if constexpr (LAT)
                for (int q = tid; q < m; q += BLOCK)
                    s_draw2[c & 1][q >> 3][q & 7] = dsrc2[(long long)(j + 1) * 8 + q];
            if (lsrc != nullptr)
                for (int q = tid; q < m / 2; q += BLOCK)
                    s_lb[c & 1][q >> 2][q & 3] = lsrc[(long long)(j + 1) * 4 + q];
            __syncthreads();
        }
        const MoveHdr h = s_hdr[buf];
        const double lnu = s_draw[(j >> 6) & 1][j & 63][7];
        const bool evaluate = h.valid && !g.prior_only;

        // the first pass's samples (global index or -1) and their new variance,
        // kept for the write-back of an accepted move
        double enew[QP];
        int gidx[QP];
#pragma unroll
        for (int q = 0; q < QP; ++q) { gidx[q] = -1; enew[q] = 0.0; }
        double prod = 1.0, lin = 0.0;
        if (wave == 0) {
            if (j + 1 < g.k) {  // speculative: the state as if move j is rejected
                scout_move<LAT>(g, lane, buf ^ 1, i, kk, offx, offy, x0, x1, y0, y1, n,
                                s_draw[((j + 1) >> 6) & 1][(j + 1) & 63], s_ex, s_ey, s_et, s_em,
                                s_seg, s_six, s_lsx, s_hdr, s_prop, kMaxFootprint, L,
                                s_lb[((j + 1) >> 6) & 1][(j + 1) & 63], s_lsta, rl,
                                LAT ? s_draw2[((j + 1) >> 6) & 1][(j + 1) & 63] : nullptr, s_da,
                                s_lat, own, tag);
            }
        } else if (evaluate) {
            const int et = tid - 64;
            const Seg *sg = s_seg[buf];
            // passes of QP strided footprint positions per thread: one pass
            // unless the footprint exceeds QP * EV samples
            for (int p = 0; p * QP * EV < h.S; ++p) {
                int run[QP], gi[QP];
                locate_runs<QP>(s_six[buf], h.nseg, h.S, et + p * QP * EV, EV, run, gi);
                // every sample's variance and trace value in flight at once;
                // slots past the footprint are skipped by a block-uniform
                // test, idle lanes of a used slot read element 0
                // (raw trace elements, converted only after every load is
                // issued, through global pointers, so that no load waits for
                // another and LDS reads do not wait for the loads)
                double eo[QP], sv[QP], dc[QP];
                TraceT tv[QP];
#pragma unroll
                for (int q = 0; q < QP; ++q) {
                    eo[q] = 0.0;
                    tv[q] = (TraceT)0;
                    if ((p * QP + q) * EV < h.S) {
                        const int g0 = gi[q] >= 0 ? gi[q] : 0;
                        eo[q] = gE[g0];  // the residual, under templates
                        if (!g.tmpl) tv[q] = gT[g0];
                    }
                }
                // variance changes from the LDS tables while the loads fly
#pragma unroll
                for (int q = 0; q < QP; ++q) {
                    dc[q] = 0.0;
                    sv[q] = (double)tv[q];
                    if ((p * QP + q) * EV < h.S && gi[q] >= 0) {
                        const Seg &a = sg[run[q]];
                        dc[q] = run_dvar(a, s_T, gi[q] - a.j * g.N);
                    }
                }
#pragma unroll
                for (int q = 0; q < QP; ++q) {
                    if ((p * QP + q) * EV < h.S && gi[q] >= 0) {
                        const double en =
                            g.tmpl ? template_term(eo[q], dc[q], &lin)
                                   : sample_term(g.sigma2, eo[q], dc[q], sv[q], &prod, &lin);
                        if (p == 0) {
                            enew[q] = en;
                            gidx[q] = gi[q];
                        }
                    }
                }
            }
            double part = g.tmpl ? lin / g.sigma2 : -0.5 * (log(prod) - lin);
            part = wave_sum(part);
            if (lane == 0) s_part[buf][wave] = part;
        }
        __syncthreads();

        double delta = 0.0;
        if (evaluate) {
#pragma unroll
            for (int w = 1; w < W; ++w) delta += s_part[buf][w];
        }
        double la;
        if (h.type == 0)
            la = delta + log_lamR + log_pd - s_log[h.n + 1] - log_pb - h.lr;
        else if (h.type == 1)
            la = delta + s_log[h.n] + log_pb - log_lamR - log_pd + h.lr;
        else if (h.type == 4)
            la = delta - g.mrate * h.dm;
        else if (LAT && h.type >= 5)
            la = delta + h.lx;
        else
            la = delta;
        bool accept = h.valid && lnu < la;
        if (!(delta == delta) || delta - delta != 0.0) {  // NaN or Inf
            accept = false;
            if (tid == 0) flags |= kFlagNan;
        }
        if (tid == 0) {
            flags |= h.flags;
            cnt_att[h.type]++;
            if (h.valid) {
                cnt_val[h.type]++;
                samp_read += (unsigned long long)h.S;
            }
            if (use_log) {
                double *lg = logp + (((sweep - log_first) * g.R + r) * g.k + j) * 4;
                lg[0] = (double)h.type;
                lg[1] = h.valid ? (accept ? 2.0 : 1.0) : 0.0;
                lg[2] = h.valid ? delta : 0.0;
                lg[3] = h.valid ? la : 0.0;
            }
        }
        if (accept) {
            if (wave > 0 && !g.prior_only) {
#pragma unroll
                for (int q = 0; q < QP; ++q)
                    if (gidx[q] >= 0) gEw[gidx[q]] = enew[q];
                // later passes (footprints over QP * EV samples) recompute the
                // same new variance from the unchanged old one
                for (int p = 1; p * QP * EV < h.S; ++p) {
                    int run[QP], gi[QP];
                    locate_runs<QP>(s_six[buf], h.nseg, h.S, tid - 64 + p * QP * EV, EV, run,
                                    gi);
                    double eo[QP];
#pragma unroll
                    for (int q = 0; q < QP; ++q)
                        eo[q] = gE[gi[q] >= 0 ? gi[q] : 0];
#pragma unroll
                    for (int q = 0; q < QP; ++q) {
                        if (gi[q] >= 0) {
                            const Seg &a = s_seg[buf][run[q]];
                            const double dv = run_dvar(a, s_T, gi[q] - a.j * g.N);
                            const double en = g.tmpl ? eo[q] - dv : eo[q] + dv;
                            gEw[gi[q]] = g.tmpl || en > 0.0 ? en : 0.0;
                        }
                    }
                }
            }
            if (tid == 0) {
                cnt_acc[h.type]++;
                samp_written += (unsigned long long)h.S;
                const double *pr = s_prop[buf];
                if (h.type == 0) {
                    s_ex[n] = pr[0]; s_ey[n] = pr[1]; s_et[n] = pr[2]; s_em[n] = pr[3];
                    s_id[n] = ((unsigned long long)(uint32_t)sweep << 32) |
                              ((unsigned long long)r << 12) | (unsigned long long)j;
                    if constexpr (LAT)
                        for (int q = 0; q < 8; ++q) s_da[n][q] = s_lat->pda[buf][0][q];
                    ++n;
                } else if (h.type == 1) {
                    const int idx = (int)pr[4];
                    for (int q = idx; q + 1 < n; ++q) {
                        s_ex[q] = s_ex[q + 1]; s_ey[q] = s_ey[q + 1];
                        s_et[q] = s_et[q + 1]; s_em[q] = s_em[q + 1];
                        s_id[q] = s_id[q + 1];
                        if constexpr (LAT)
                            for (int c = 0; c < 8; ++c) s_da[q][c] = s_da[q + 1][c];
                    }
                    --n;
                } else {
                    const int idx = (int)pr[4];
                    s_ex[idx] = pr[0]; s_ey[idx] = pr[1]; s_et[idx] = pr[2]; s_em[idx] = pr[3];
                    if constexpr (LAT) {
                        for (int q = 0; q < 8; ++q) s_da[idx][q] = s_lat->pda[buf][0][q];
                        if (h.type == 6) {  // the joint move's second event
                            const double *p2 = s_lat->prop2[buf];
                            const int i2 = (int)p2[2];
                            s_ex[i2] = p2[0]; s_et[i2] = p2[1];
                            for (int q = 0; q < 8; ++q) s_da[i2][q] = s_lat->pda[buf][1][q];
                        }
                    }
                }
            }
            n = __builtin_amdgcn_readlane(n, 0);
            __syncthreads();  // the new events and variance are visible
            // The speculative move j + 1 assumed move j rejected.  After an
            // accepted change of one event (n unchanged) it still holds
            // unless it proposes to change that same event.  A birth or a
            // death changes the event count and shifts list positions: a
            // birth proposal stands with the new count (capacity aside), and
            // a move of an event stands when its draw picks the same event at
            // its new position (the count and index are patched); anything
            // else is built again.
            const MoveHdr nx = s_hdr[buf ^ 1];
            bool rebuild;
            int patch_idx = -1;
            const int n1 = h.type == 0 ? h.n + 1 : h.n - 1;
            if (LAT && (h.type == 6 || nx.type == 6)) {
                rebuild = true;  // two events involved: built again
            } else if (h.type >= 2) {
                rebuild = nx.type != 0 && s_prop[buf ^ 1][4] == s_prop[buf][4];
            } else if (nx.type == 0) {
                rebuild = !(h.n < g.cap && n1 < g.cap);
            } else if (h.n == 0 || n1 == 0) {
                rebuild = true;
            } else {
                const double u = s_draw[((j + 1) >> 6) & 1][(j + 1) & 63][1];
                int in = (int)floor(u * (double)n1);  // the scout's index rule
                if (in >= n1) in = n1 - 1;
                const int dead = (int)s_prop[buf][4];
                const int was = h.type == 0 ? in : (in >= dead ? in + 1 : in);
                rebuild = was != (int)s_prop[buf ^ 1][4];
                patch_idx = in;
            }
            if (j + 1 < g.k) {
                if (rebuild) {
                    if (wave == 0) {
                        scout_move<LAT>(g, lane, buf ^ 1, i, kk, offx, offy, x0, x1, y0, y1, n,
                                        s_draw[((j + 1) >> 6) & 1][(j + 1) & 63], s_ex, s_ey,
                                        s_et, s_em, s_seg, s_six, s_lsx, s_hdr, s_prop,
                                        kMaxFootprint, L, s_lb[((j + 1) >> 6) & 1][(j + 1) & 63],
                                        s_lsta, rl,
                                        LAT ? s_draw2[((j + 1) >> 6) & 1][(j + 1) & 63] : nullptr,
                                        s_da, s_lat, own, tag);
                    }
                    __syncthreads();
                } else if (h.type <= 1) {
                    if (tid == 0) {
                        s_hdr[buf ^ 1].n = n1;
                        if (patch_idx >= 0) s_prop[buf ^ 1][4] = (double)patch_idx;
                    }
                    __syncthreads();
                }
            }
        }
    }

    if (tid == 0) s_n = n;
    __syncthreads();
    const int nf = s_n;
    for (int s = tid; s < nf; s += BLOCK) {
        ev.x[base + s] = s_ex[s]; ev.y[base + s] = s_ey[s];
        ev.t[base + s] = s_et[s]; ev.m[base + s] = s_em[s];
        ev.id[base + s] = s_id[s];
    }
    if constexpr (LAT)
        for (int q = tid; q < nf * 8; q += BLOCK) ev.da[base * 8 + q] = s_da[q >> 3][q & 7];
    if (tid == 0) {
        ev.cnt[chain * g.R + r] = nf;
        unsigned long long *st = stats + (long long)chain * kStats;
        for (int t = 0; t < NT; ++t) {
            const int sb = stat_base(t);
            if (cnt_att[t]) atomicAdd(&st[sb + 0], (unsigned long long)cnt_att[t]);
            if (cnt_val[t]) atomicAdd(&st[sb + 1], (unsigned long long)cnt_val[t]);
            if (cnt_acc[t]) atomicAdd(&st[sb + 2], (unsigned long long)cnt_acc[t]);
        }
        if (samp_read) atomicAdd(&st[15], samp_read);
        if (samp_written) atomicAdd(&st[16], samp_written);
        if (flags) atomicOr(err, flags);
        stamp_at(sa, sweep, 1);
    }
}

// ----------------------------------------------------- sweep colour, waves
// Throughput form of a colour phase, for launches with many more work items
// than the device holds workgroups: each of the four waves of a workgroup
// runs one work item's k moves by itself, in sequence (proposal and
// footprint as the scout builds them, then the likelihood change over the
// footprint in passes of 64 kWaveQ samples, then the decision and, on
// acceptance, a second pass writing the new variance).  No speculation and
// no barrier once the tables are filled; the wave's LDS is about a quarter
// of the latency form's, so a CU holds several times as many regions.
constexpr int kWaveQ = 4;
constexpr int kWaveDraws = 16;  // moves whose draws are staged at once

// This lane's share of the log-likelihood change of a move: passes of
// 64 kWaveQ footprint samples, every load of a pass in flight at once.
// EG: E is in global memory (not the naive schedule's private copy in LDS).
template <typename TraceT, bool EG>
__device__ double wave_delta_part(const Geo &g, const TraceT *__restrict__ trace,
                                  const double *__restrict__ E, const Seg *sg,
                                  const SegIndex &six, int nseg, int S, const double *sT, int lane)
{
    double prod = 1.0, lin = 0.0;
    for (int base = 0; base < S; base += 64 * kWaveQ) {
        int run[kWaveQ], gidx[kWaveQ];
        locate_runs<kWaveQ>(six, nseg, S, base + lane, 64, run, gidx);
        // raw trace elements, converted once every load is issued; the trace
        // (always) and E (unless it is the naive schedule's LDS copy) through
        // global pointers, whose loads are counted apart from LDS operations
        const __attribute__((address_space(1))) TraceT *gT =
            (const __attribute__((address_space(1))) TraceT *)trace;
        // every load is issued, positions past the footprint reading element
        // 0 (their terms are dropped below): loads under a branch would each
        // be waited for at the join
        double eo[kWaveQ], sv[kWaveQ], dc[kWaveQ];
        TraceT tv[kWaveQ];
#pragma unroll
        for (int q = 0; q < kWaveQ; ++q) {
            const int gi = gidx[q] >= 0 ? gidx[q] : 0;
            if constexpr (EG)  // the residual, under templates
                eo[q] = ((const __attribute__((address_space(1))) double *)E)[gi];
            else
                eo[q] = E[gi];
            tv[q] = gT[g.tmpl ? 0 : gi];
        }
#pragma unroll
        for (int q = 0; q < kWaveQ; ++q) {
            dc[q] = 0.0;
            sv[q] = (double)tv[q];
            if (base + 64 * q < S && gidx[q] >= 0) {
                const Seg &a = sg[run[q]];
                dc[q] = run_dvar(a, sT, gidx[q] - a.j * g.N);
            }
        }
#pragma unroll
        for (int q = 0; q < kWaveQ; ++q)
            if (base + 64 * q < S && gidx[q] >= 0) {
                if (g.tmpl)
                    (void)template_term(eo[q], dc[q], &lin);
                else
                    (void)sample_term(g.sigma2, eo[q], dc[q], sv[q], &prod, &lin);
            }
    }
    return g.tmpl ? lin / g.sigma2 : -0.5 * (log(prod) - lin);
}

// After an acceptance: the new variance over the footprint, written in place.
// The new variance max(E + change, 0) is the one sample_term used for Delta
// (the new residual E - change under templates).
// EG: E is in global memory (not the naive schedule's private copy in LDS);
// its loads are then issued together through a global pointer.
template <bool EG>
__device__ void wave_write(const Geo &g, double *__restrict__ E, const Seg *sg,
                           const SegIndex &six, int nseg, int S, const double *sT, int lane)
{
    for (int base = 0; base < S; base += 64 * kWaveQ) {
        int run[kWaveQ], gidx[kWaveQ];
        locate_runs<kWaveQ>(six, nseg, S, base + lane, 64, run, gidx);
        double eo[kWaveQ];
#pragma unroll
        for (int q = 0; q < kWaveQ; ++q) {
            const int gi = gidx[q] >= 0 ? gidx[q] : 0;
            if constexpr (EG)
                eo[q] = ((const __attribute__((address_space(1))) double *)E)[gi];
            else
                eo[q] = E[gi];
        }
#pragma unroll
        for (int q = 0; q < kWaveQ; ++q)
            if (base + 64 * q < S && gidx[q] >= 0) {
                const Seg &a = sg[run[q]];
                const double dv = run_dvar(a, sT, gidx[q] - a.j * g.N);
                const double en = g.tmpl ? eo[q] - dv : eo[q] + dv;
                const double v = g.tmpl || en > 0.0 ? en : 0.0;
                if constexpr (EG)
                    ((__attribute__((address_space(1))) double *)E)[gidx[q]] = v;
                else
                    E[gidx[q]] = v;
            }
    }
}

// NAIVE: the naive parallel schedule of Algorithm 3, every region in one
// phase, each accepting against the posterior of its own events alone.  Each
// wave then evaluates against a private variance in LDS built from its own
// events; the shared variance is never written and is recomputed from the
// merged events after the phase.
// LAT: latent arrival times (line model), as in the latency form: each
// wave keeps its region's arrival offsets, its draws 8..15 and the joint
// move's scratch in LDS (about 27 KB more per workgroup, two waves per SIMD).
template <typename TraceT, bool NAIVE, bool LAT = false, bool OWN = false, bool PER = false>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(NAIVE ? 1 : (LAT ? 2 : 4))))
k_sweep_wave(const Slot *__restrict__ slots, const unsigned *__restrict__ items, int nitems, int par,
             const long long *__restrict__ sweep_ptr, double *__restrict__ logp,
             long long log_first, long long log_n, int *__restrict__ err, int naive_elems,
             StampArg sa, PersistArg pq)
{
    __shared__ double s_log[kMaxCap + 2];
    __shared__ double s_T[4][kMaxTs];
    __shared__ double s_draw[4][kWaveDraws][8];
    __shared__ double s_lb[4][kWaveDraws][4];
    __shared__ double s_ex[4][kMaxCap], s_ey[4][kMaxCap], s_et[4][kMaxCap], s_em[4][kMaxCap];
    __shared__ unsigned long long s_id[4][kMaxCap];
    __shared__ Seg s_seg[4][1][kMaxSeg];
    __shared__ SegIndex s_six[4][1];
    __shared__ MoveHdr s_hdr[4][1];
    __shared__ double s_prop[4][1][5];
    __shared__ int s_lsta[4][kMaxRegSta];
    __shared__ RegionLearned s_rl[4];
    // latent arrivals only (one-element stand-ins when LAT is false)
    __shared__ double s_draw2[LAT ? 4 : 1][LAT ? kWaveDraws : 1][8];
    __shared__ double s_daw[LAT ? 4 : 1][LAT ? kMaxCap : 1][8];
    __shared__ LatentLds s_latw[LAT ? 4 : 1];
    // the instance's constants live in LDS: held in registers they would
    // halve the waves a CU can hold
    __shared__ Geo s_g[4];
    __shared__ Learned s_L[4];
    __shared__ double s_rc[4][10];
    // move counters of each wave (lane 0 counts): [3 t + 0..2], then the
    // footprint samples read and written
    __shared__ unsigned long long s_cnt[4][kStats];

    const int tid = threadIdx.x, lane = tid & 63;
    // the wave's index, and everything derived from it (work item, slot,
    // region), held in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int q = tid; q < kMaxCap + 2; q += 256) s_log[q] = log((double)q);
    __syncthreads();  // the only barrier: every wave passes it before any leaves
    // one work item (slot, region) of this wave: k moves in sequence
    auto item_body = [&](const int it) {
        const unsigned item = items[it];
        const int slot = (int)(item >> 16), r = (int)(item & 0xFFFFu);
        if (lane == 0) s_g[wv] = slots[slot].g;
        __builtin_amdgcn_wave_barrier();
        const Geo &g = s_g[wv];
        const Events ev = slots[slot].ev[par];
        const TraceT *__restrict__ trace = (const TraceT *)slots[slot].trace;
        double *__restrict__ E = slots[slot].E;
        const double *__restrict__ draws = slots[slot].draws;
        unsigned long long *__restrict__ stats = slots[slot].stats;
        if (lane == 0) s_L[wv] = slots[slot].L;
        __builtin_amdgcn_wave_barrier();
        const Learned &L = s_L[wv];
        const int i = r % g.nrx, kk = r / g.nrx;
        const long long sweep = *sweep_ptr;
        if (lane == 0) stamp_at(sa, sweep, 0);
        unsigned long long *const own = OWN ? slots[slot].owner : nullptr;  // debug owner check
        const unsigned long long tag = OWN ? owner_tag(g, sweep, i, kk, r) : 0ull;
        if (lane == 0) {
            double *c = s_rc[wv];
            c[0] = ev.off[0]; c[1] = ev.off[1];
            const RegionBox b = region_box(g, c[0], c[1], i, kk);
            c[2] = b.x0; c[3] = b.x1; c[4] = b.y0; c[5] = b.y1; c[6] = b.area;
            c[7] = log(b.lamR);
            c[8] = log(g.pb); c[9] = log(g.pd);
        }
        __builtin_amdgcn_wave_barrier();
        const double *rc_ = s_rc[wv];
        const double &offx = rc_[0], &offy = rc_[1], &x0 = rc_[2], &x1 = rc_[3], &y0 = rc_[4],
                     &y1 = rc_[5], &area = rc_[6], &log_lamR = rc_[7], &log_pb = rc_[8],
                     &log_pd = rc_[9];
        if (!(area > 0.0)) return;

        double *sT = s_T[wv];
        double *ex = s_ex[wv], *ey = s_ey[wv], *et = s_et[wv], *em = s_em[wv];
        unsigned long long *eid = s_id[wv];
        const long long base = (long long)r * g.cap;
        int n = ev.cnt[r];
        for (int s = lane; s < n; s += 64) {
            ex[s] = ev.x[base + s]; ey[s] = ev.y[base + s];
            et[s] = ev.t[base + s]; em[s] = ev.m[base + s];
            eid[s] = ev.id[base + s];
        }
        double (*da)[8] = nullptr;
        LatentLds *lat = nullptr;
        const double *dsrc2 = nullptr;
        if constexpr (LAT) {
            da = s_daw[wv];
            lat = &s_latw[wv];
            for (int q = lane; q < n * 8; q += 64) da[q >> 3][q & 7] = ev.da[base * 8 + q];
            dsrc2 = slots[slot].draws2 + (long long)r * g.k * 8;
        }
        for (int q = lane; q < g.ts; q += 64) sT[q] = exp(-(g.tmpl ? 1.0 : 2.0) * (double)q / g.decay);
        int flags = 0;
        double *Ew = E;  // the variance (or residual) this wave reads and writes
        if constexpr (NAIVE) {
            // Algorithm 3: the region accepts against its own events alone, so
            // its private variance starts from no event (the trace itself as the
            // residual, under templates) and takes in each of its events in turn
            extern __shared__ double s_pe[];  // 4 x naive_elems, sized at launch
            double *pe = s_pe + (long long)wv * naive_elems;
            for (int q = lane; q < g.nsta * g.N; q += 64) pe[q] = g.tmpl ? (double)trace[q] : 0.0;
            __builtin_amdgcn_wave_barrier();
            for (int q = 0; q < n; ++q) {
                int nseg = 0, S = 0, fl = 0;
                footprint(g, lane, false, 0.0, 0.0, 0.0, 0.0, true, ex[q], ey[q], et[q], em[q],
                          s_seg[wv][0], &s_six[wv][0], g.sx, &nseg, &S, &fl);
                __builtin_amdgcn_wave_barrier();
                if (__ballot(fl != 0) != 0ull) flags |= kFlagSeg;
                else wave_write<false>(g, pe, s_seg[wv][0], s_six[wv][0], nseg, S, sT, lane);
                __builtin_amdgcn_wave_barrier();
            }
            Ew = pe;
        }
        {
            bool over = false;
            const RegionLearned rl = region_learned_wave(g, L, offx, offy, i, kk, x0, x1, y0, y1,
                                                         area, s_lsta[wv], lane, &over);
            if (lane == 0) {
                if (over) flags |= kFlagSta;
                s_rl[wv] = rl;
            }
        }
        __builtin_amdgcn_wave_barrier();
        const RegionLearned rl = s_rl[wv];
        const double *dsrc = draws + (long long)r * g.k * 8;
        const double *lsrc = L.tab != nullptr ? L.birth + (long long)r * g.k * 4 : nullptr;
        const bool use_log = logp != nullptr && slot == 0 && sweep >= log_first &&
                             sweep < log_first + log_n;
        unsigned long long *cnt = s_cnt[wv];
        if (lane < kStats) cnt[lane] = 0;
        __builtin_amdgcn_wave_barrier();

        for (int j = 0; j < g.k; ++j) {
            const int jw = j % kWaveDraws;
            if (jw == 0) {  // stage the next kWaveDraws moves' records
                const int m = min(kWaveDraws, g.k - j);
                for (int q = lane; q < 8 * m; q += 64)
                    s_draw[wv][q >> 3][q & 7] = dsrc[(long long)j * 8 + q];
                if constexpr (LAT)
                    for (int q = lane; q < 8 * m; q += 64)
                        s_draw2[wv][q >> 3][q & 7] = dsrc2[(long long)j * 8 + q];
                if (lsrc != nullptr)
                    for (int q = lane; q < 4 * m; q += 64)
                        s_lb[wv][q >> 2][q & 3] = lsrc[(long long)j * 4 + q];
                __builtin_amdgcn_wave_barrier();
            }
            scout_move<LAT>(g, lane, 0, i, kk, offx, offy, x0, x1, y0, y1, n, s_draw[wv][jw], ex, ey,
                            et, em, s_seg[wv], s_six[wv], g.sx, s_hdr[wv], s_prop[wv], kMaxFootprint, L,
                            s_lb[wv][jw], s_lsta[wv], rl, LAT ? s_draw2[wv][jw] : nullptr, da, lat,
                            own, tag);
            __builtin_amdgcn_wave_barrier();
            const MoveHdr h = s_hdr[wv][0];
            const double lnu = s_draw[wv][jw][7];
            const bool evaluate = h.valid && !g.prior_only;
            double delta = 0.0;
            if (evaluate)
                delta = wave_sum(wave_delta_part<TraceT, !NAIVE>(g, trace, Ew, s_seg[wv][0], s_six[wv][0],
                                                         h.nseg, h.S, sT, lane));
            double la;
            if (h.type == 0)
                la = delta + log_lamR + log_pd - s_log[h.n + 1] - log_pb - h.lr;
            else if (h.type == 1)
                la = delta + s_log[h.n] + log_pb - log_lamR - log_pd + h.lr;
            else if (h.type == 4)
                la = delta - g.mrate * h.dm;
            else if (LAT && h.type >= 5)
                la = delta + h.lx;
            else
                la = delta;
            bool accept = h.valid && lnu < la;
            if (!(delta == delta) || delta - delta != 0.0) {
                accept = false;
                flags |= kFlagNan;
            }
            if (lane == 0) {
                flags |= h.flags;
                cnt[stat_base(h.type)]++;
                if (h.valid) {
                    cnt[stat_base(h.type) + 1]++;
                    cnt[15] += (unsigned long long)h.S;
                }
                if (use_log) {
                    double *lg = logp + (((sweep - log_first) * g.R + r) * g.k + j) * 4;
                    lg[0] = (double)h.type;
                    lg[1] = h.valid ? (accept ? 2.0 : 1.0) : 0.0;
                    lg[2] = h.valid ? delta : 0.0;
                    lg[3] = h.valid ? la : 0.0;
                }
            }
            if (accept) {
                if (!g.prior_only)
                    wave_write<!NAIVE>(g, Ew, s_seg[wv][0], s_six[wv][0], h.nseg, h.S, sT, lane);
                if (lane == 0) {
                    cnt[stat_base(h.type) + 2]++;
                    cnt[16] += (unsigned long long)h.S;
                    const double *pr = s_prop[wv][0];
                    if (h.type == 0) {
                        ex[n] = pr[0]; ey[n] = pr[1]; et[n] = pr[2]; em[n] = pr[3];
                        eid[n] = ((unsigned long long)(uint32_t)sweep << 32) |
                                 ((unsigned long long)r << 12) | (unsigned long long)j;
                        if constexpr (LAT)
                            for (int q = 0; q < 8; ++q) da[n][q] = lat->pda[0][0][q];
                        ++n;
                    } else if (h.type == 1) {
                        const int idx = (int)pr[4];
                        for (int q = idx; q + 1 < n; ++q) {
                            ex[q] = ex[q + 1]; ey[q] = ey[q + 1];
                            et[q] = et[q + 1]; em[q] = em[q + 1];
                            eid[q] = eid[q + 1];
                            if constexpr (LAT)
                                for (int c = 0; c < 8; ++c) da[q][c] = da[q + 1][c];
                        }
                        --n;
                    } else {
                        const int idx = (int)pr[4];
                        ex[idx] = pr[0]; ey[idx] = pr[1]; et[idx] = pr[2]; em[idx] = pr[3];
                        if constexpr (LAT) {
                            for (int q = 0; q < 8; ++q) da[idx][q] = lat->pda[0][0][q];
                            if (h.type == 6) {  // the joint move's second event
                                const double *p2 = lat->prop2[0];
                                const int i2 = (int)p2[2];
                                ex[i2] = p2[0]; et[i2] = p2[1];
                                for (int q = 0; q < 8; ++q) da[i2][q] = lat->pda[0][1][q];
                            }
                        }
                    }
                }
                n = __builtin_amdgcn_readlane(n, 0);
                __builtin_amdgcn_wave_barrier();
            }
        }

        for (int s = lane; s < n; s += 64) {
            ev.x[base + s] = ex[s]; ev.y[base + s] = ey[s];
            ev.t[base + s] = et[s]; ev.m[base + s] = em[s];
            ev.id[base + s] = eid[s];
        }
        if constexpr (LAT)
            for (int q = lane; q < n * 8; q += 64) ev.da[base * 8 + q] = da[q >> 3][q & 7];
        if (lane == 0) {
            ev.cnt[r] = n;
            for (int t = 0; t < kStats; ++t)
                if (cnt[t]) atomicAdd(&stats[t], cnt[t]);
            if (flags) atomicOr(err, flags);
            stamp_at(sa, sweep, 1);
        }
    };
    if constexpr (!PER) {
        const int it = blockIdx.x * 4 + wv;
        if (it >= nitems) return;
        item_body(it);
    } else {
        // Persistent form: the launch covers every colour of the sweep.  Each
        // wave takes the next item by ticket (items in colour order); an item
        // of colour c first waits until its own slot has completed all its
        // items of colours below c (the slot's colour counter), since the
        // colour phases are ordered within a chain (Algorithm 4) but chains
        // and instances are independent.  A wave only waits on items with
        // smaller tickets, which running waves hold, so every wait ends; a
        // wait past the spin limit raises kFlagWait and skips the item.
        for (;;) {
            int t = 0;
            if (lane == 0) t = atomicAdd(pq.ticket, 1);
            t = __builtin_amdgcn_readfirstlane(t);
            if (t >= nitems) break;
            const int slot = (int)(items[t] >> 16);
            int ok = 1;
            if (lane == 0) {
                const unsigned target = pq.wait[t];
                long long spins = 0;
                while (__hip_atomic_load(pq.done + slot, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) < target) {
                    if (++spins > pq.spin_limit) {
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            ok = __builtin_amdgcn_readfirstlane(ok);
            // the earlier colours' variance writes of this slot become visible
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (ok)
                item_body(t);
            else if (lane == 0)
                atomicOr(err, kFlagWait);
            // this item's writes are visible before its completion counts
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0)
                __hip_atomic_fetch_add(pq.done + slot, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------- sweep colour, speculative
// Speculative form of a colour phase: one workgroup of D waves per work
// item.  In each round wave w takes move j + w of the region: it builds the
// proposal and footprint, evaluates the log-likelihood change over the
// footprint and decides, all from the region's state before move j.  That is
// the state the sequential chain hands to move j + w whenever moves j ..
// j + w - 1 are all rejected, and also whenever the accepted ones among them
// leave the event count, move j + w's event and the variance on its
// footprint unchanged.  The moves of a round therefore stand in move order
// up to the first one that conflicts with an earlier standing acceptance, or
// up to and including an accepted birth or death; the accepted moves among
// them are committed (their footprints are disjoint), the rest is dropped
// and built again from the new state in the next round.  The chain of
// states is exactly the sequential one (Algorithm 4's inner loop), while a
// round costs about one move's latency.
// Plain and mean-template likelihoods, grid and line models; latent arrivals
// and the naive schedule keep their own forms.
template <typename TraceT, int D, bool OWN = false>
__global__ void __launch_bounds__(64 * D) __attribute__((amdgpu_waves_per_eu(D <= 4 ? 1 : 2)))
k_sweep_spec(const Slot *__restrict__ slots, const unsigned *__restrict__ items, int par,
             const long long *__restrict__ sweep_ptr, double *__restrict__ logp,
             long long log_first, long long log_n, int *__restrict__ err, StampArg sa)
{
    static_assert(D >= 2 && D <= 16, "two to sixteen waves");
    constexpr int BLOCK = 64 * D;
    __shared__ double s_draw[2][kDrawChunk][8];
    __shared__ double s_lb[2][kDrawChunk][4];
    __shared__ int s_lsta[kMaxRegSta];
    __shared__ RegionLearned s_rl;
    __shared__ double s_T[kMaxTs];
    __shared__ double s_log[kMaxCap + 2];  // s_log[q] = log(q)
    __shared__ double s_ex[kMaxCap], s_ey[kMaxCap], s_et[kMaxCap], s_em[kMaxCap];
    __shared__ unsigned long long s_id[kMaxCap];
    __shared__ double s_lsx[8];  // line model: station positions
    // per wave and round parity: a round's tables stay readable until every
    // wave has passed the next round's first barrier
    __shared__ Seg s_seg[D][2][kMaxSeg];
    __shared__ SegIndex s_six[D][2];
    __shared__ MoveHdr s_hdr[D][2];
    __shared__ double s_prop[D][2][5];
    __shared__ int s_acc[2][D];  // per round parity: wave w's move accepted
    __shared__ int s_n;
    __shared__ unsigned long long s_cnt[D][kStats];
    __shared__ int s_flags[D];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const unsigned item = items[blockIdx.x];
    const int slot = (int)(item >> 16), r = (int)(item & 0xFFFFu);
    // the instance's constants are read where they sit (scalar loads): a
    // private copy would live in scratch memory
    const Geo &g = slots[slot].g;
    const Events ev = slots[slot].ev[par];
    const TraceT *__restrict__ trace = (const TraceT *)slots[slot].trace;
    double *__restrict__ E = slots[slot].E;
    const double *__restrict__ draws = slots[slot].draws;
    unsigned long long *__restrict__ stats = slots[slot].stats;
    const Learned L = slots[slot].L;
    const int i = r % g.nrx, kk = r / g.nrx;
    const long long sweep = *sweep_ptr;
    if (tid == 0) stamp_at(sa, sweep, 0);
    unsigned long long *const own = OWN ? slots[slot].owner : nullptr;  // debug owner check
    const unsigned long long tag = OWN ? owner_tag(g, sweep, i, kk, r) : 0ull;

    const double offx = ev.off[0], offy = ev.off[1];
    const RegionBox box = region_box(g, offx, offy, i, kk);
    const double x0 = box.x0, x1 = box.x1, y0 = box.y0, y1 = box.y1, area = box.area;
    if (!(area > 0.0)) return;  // the same for every thread of the workgroup
    const double log_lamR = log(box.lamR), log_pb = log(g.pb), log_pd = log(g.pd);

    const long long base = (long long)r * g.cap;
    const double *dsrc = draws + (long long)r * (long long)g.k * 8;
    const double *lsrc = L.tab != nullptr ? L.birth + (long long)r * (long long)g.k * 4 : nullptr;
    int n = ev.cnt[r];
    for (int s = tid; s < n; s += BLOCK) {
        s_ex[s] = ev.x[base + s]; s_ey[s] = ev.y[base + s];
        s_et[s] = ev.t[base + s]; s_em[s] = ev.m[base + s];
        s_id[s] = ev.id[base + s];
    }
    for (int q = tid; q < g.ts; q += BLOCK) s_T[q] = exp(-(g.tmpl ? 1.0 : 2.0) * (double)q / g.decay);
    for (int q = tid; q < kMaxCap + 2; q += BLOCK) s_log[q] = log((double)q);
    if (tid < 8) s_lsx[tid] = g.sx[tid];
    for (int q = tid; q < D * kStats; q += BLOCK) s_cnt[q / kStats][q % kStats] = 0ull;
    // draw records of moves 0 .. 127 (chunks of 64 in a double buffer)
    int loaded = 0;
    for (int c = 0; c < 2 && loaded < g.k; ++c) {
        const int m = min(kDrawChunk, g.k - loaded);
        for (int q = tid; q < m * 8; q += BLOCK) s_draw[c][q >> 3][q & 7] = dsrc[64LL * 8 * c + q];
        if (lsrc != nullptr)
            for (int q = tid; q < m * 4; q += BLOCK) s_lb[c][q >> 2][q & 3] = lsrc[64LL * 4 * c + q];
        loaded += m;
    }
    int flags = 0;
    if (tid < 64) {  // the first wave
        bool over = false;
        const RegionLearned rl = region_learned_wave(g, L, offx, offy, i, kk, x0, x1, y0, y1,
                                                     area, s_lsta, tid, &over);
        if (tid == 0) {
            if (over) flags |= kFlagSta;
            s_rl = rl;
        }
    }
    const bool use_log = logp != nullptr && slot == 0 && sweep >= log_first &&
                         sweep < log_first + log_n;
    __syncthreads();
    const RegionLearned rl = s_rl;
    unsigned long long *cnt = s_cnt[wv];

    int j = 0, round = 0;
    while (j < g.k) {
        const int m = min(D, g.k - j);
        if (j + m > loaded) {
            // the next chunk replaces the one two chunks back, whose moves
            // (all below j) every wave has finished with
            const int c = loaded >> 6;
            const int cm = min(kDrawChunk, g.k - loaded);
            for (int q = tid; q < cm * 8; q += BLOCK)
                s_draw[c & 1][q >> 3][q & 7] = dsrc[(long long)loaded * 8 + q];
            if (lsrc != nullptr)
                for (int q = tid; q < cm * 4; q += BLOCK)
                    s_lb[c & 1][q >> 2][q & 3] = lsrc[(long long)loaded * 4 + q];
            loaded += cm;
            __syncthreads();
        }
        const int jm = j + wv;  // this wave's move
        const int db = (jm >> 6) & 1, dj = jm & 63;
        const int pb = round & 1;
        MoveHdr h = {};
        double delta = 0.0, la = 0.0;
        bool accept = false, nan = false;
        if (wv < m) {
            scout_move<false>(g, lane, pb, i, kk, offx, offy, x0, x1, y0, y1, n, s_draw[db][dj],
                              s_ex, s_ey, s_et, s_em, s_seg[wv], s_six[wv], s_lsx, s_hdr[wv],
                              s_prop[wv], kMaxFootprint, L, s_lb[db][dj], s_lsta, rl, nullptr,
                              nullptr, nullptr, own, tag);
            __builtin_amdgcn_wave_barrier();
            h = s_hdr[wv][pb];
            const double lnu = s_draw[db][dj][7];
            if (h.valid && !g.prior_only)
                delta = wave_sum(wave_delta_part<TraceT, true>(g, trace, E, s_seg[wv][pb],
                                                               s_six[wv][pb], h.nseg, h.S, s_T,
                                                               lane));
            if (h.type == 0)
                la = delta + log_lamR + log_pd - s_log[h.n + 1] - log_pb - h.lr;
            else if (h.type == 1)
                la = delta + s_log[h.n] + log_pb - log_lamR - log_pd + h.lr;
            else if (h.type == 4)
                la = delta - g.mrate * h.dm;
            else
                la = delta;
            accept = h.valid && lnu < la;
            nan = !(delta == delta) || delta - delta != 0.0;  // NaN or Inf
            if (nan) accept = false;
            if (lane == 0) s_acc[pb][wv] = accept ? 1 : 0;
        }
        __syncthreads();
        // Which moves of the round stand.  Move w was built and decided from
        // the state before move j; it is exactly the move the sequential chain
        // makes from the state after moves j .. j + w - 1 whenever none of the
        // accepted ones among them changed the event count (a birth or death),
        // the event w acts on, or the variance on w's footprint.  The moves
        // stand in order up to the first one in conflict with an earlier
        // standing acceptance (same event, or runs at one station with
        // overlapping samples), or up to and including an accepted birth or
        // death.  Every wave finds them by itself from the round's tables.
        int l_acc = 0, l_type = 0, l_idx = -1, l_nseg = 0;
        if (lane < m) {
            l_acc = s_acc[pb][lane];
            const MoveHdr &hl = s_hdr[lane][pb];
            l_type = hl.type;
            l_idx = (int)s_prop[lane][pb][4];
            l_nseg = hl.valid ? hl.nseg : 0;
        }
        const unsigned long long acc_mask = __ballot(l_acc != 0);
        int used = m;
        unsigned stand = 0u;  // accepted moves that stand
        for (int w = 0; w < m; ++w) {
            if (stand) {
                const int tw = __builtin_amdgcn_readlane(l_type, w);
                const int iw = __builtin_amdgcn_readlane(l_idx, w);
                const int nw = __builtin_amdgcn_readlane(l_nseg, w);
                bool c = false;
                for (int v = 0; v < w && !c; ++v) {
                    if (!((stand >> v) & 1u)) continue;
                    const int tv = __builtin_amdgcn_readlane(l_type, v);
                    const int iv = __builtin_amdgcn_readlane(l_idx, v);
                    const int nv = __builtin_amdgcn_readlane(l_nseg, v);
                    c = tw >= 1 && tv >= 1 && iw == iv;
                    bool ov = false;
                    for (int p = lane; !c && p < nw * nv; p += 64) {
                        const Seg &sa = s_seg[w][pb][p / nv], &sb = s_seg[v][pb][p % nv];
                        ov = ov || (sa.j == sb.j && sa.lo < sb.lo + sb.len && sb.lo < sa.lo + sa.len);
                    }
                    c = c || __ballot(ov) != 0ull;
                }
                if (c) {
                    used = w;
                    break;
                }
            }
            if ((acc_mask >> w) & 1ull) {
                stand |= 1u << w;
                if (__builtin_amdgcn_readlane(l_type, w) <= 1) {
                    used = w + 1;
                    break;
                }
            }
        }
        if (wv < used && lane == 0) {  // this wave's move is consumed
            flags |= h.flags | (nan ? kFlagNan : 0);
            cnt[stat_base(h.type)]++;
            if (h.valid) {
                cnt[stat_base(h.type) + 1]++;
                cnt[15] += (unsigned long long)h.S;
            }
            if (use_log) {
                double *lg = logp + (((sweep - log_first) * g.R + r) * g.k + jm) * 4;
                lg[0] = (double)h.type;
                lg[1] = h.valid ? (accept ? 2.0 : 1.0) : 0.0;
                lg[2] = h.valid ? delta : 0.0;
                lg[3] = h.valid ? la : 0.0;
            }
        }
        if (stand) {
            if ((stand >> wv) & 1u) {  // this wave's accepted move stands
                if (!g.prior_only)
                    wave_write<true>(g, E, s_seg[wv][pb], s_six[wv][pb], h.nseg, h.S, s_T, lane);
                if (lane == 0) {
                    cnt[stat_base(h.type) + 2]++;
                    cnt[16] += (unsigned long long)h.S;
                }
            }
            if (tid == 0) {  // the event table, in move order
                for (int w = 0; w < used; ++w) {
                    if (!((stand >> w) & 1u)) continue;
                    const int type = s_hdr[w][pb].type;
                    const double *pr = s_prop[w][pb];
                    if (type == 0) {
                        s_ex[n] = pr[0]; s_ey[n] = pr[1]; s_et[n] = pr[2]; s_em[n] = pr[3];
                        s_id[n] = ((unsigned long long)(uint32_t)sweep << 32) |
                                  ((unsigned long long)r << 12) | (unsigned long long)(j + w);
                        ++n;
                    } else if (type == 1) {
                        const int idx = (int)pr[4];
                        for (int q = idx; q + 1 < n; ++q) {
                            s_ex[q] = s_ex[q + 1]; s_ey[q] = s_ey[q + 1];
                            s_et[q] = s_et[q + 1]; s_em[q] = s_em[q + 1];
                            s_id[q] = s_id[q + 1];
                        }
                        --n;
                    } else {
                        const int idx = (int)pr[4];
                        s_ex[idx] = pr[0]; s_ey[idx] = pr[1]; s_et[idx] = pr[2]; s_em[idx] = pr[3];
                    }
                }
                s_n = n;
            }
            __syncthreads();  // the new events and variance are visible
            n = s_n;
        }
        j += used;
        ++round;
    }

    if (lane == 0) s_flags[wv] = flags;
    __syncthreads();
    for (int s = tid; s < n; s += BLOCK) {
        ev.x[base + s] = s_ex[s]; ev.y[base + s] = s_ey[s];
        ev.t[base + s] = s_et[s]; ev.m[base + s] = s_em[s];
        ev.id[base + s] = s_id[s];
    }
    if (tid < kStats) {
        unsigned long long v = 0;
        for (int w = 0; w < D; ++w) v += s_cnt[w][tid];
        if (v) atomicAdd(&stats[tid], v);
    }
    if (tid == 0) {
        ev.cnt[r] = n;
        int f = 0;
        for (int w = 0; w < D; ++w) f |= s_flags[w];
        if (f) atomicOr(err, f);
        stamp_at(sa, sweep, 1);
    }
}

// Every move's draw record for one sweep: per slot [region][move][8], from
// Philox under the slot's key (or, for slot 0 in replay mode, copied from
// the caller's feed, records of 8, or of 16 with learned births, whose draws
// 8..15 go to the slot's L.raw for k_learned_births, or with latent
// arrivals, whose draws 8..15 go to the slot's draws2).  One thread per move
// of every region of every slot (all slots take k moves per region).
__global__ void k_sweep_draws(const Slot *__restrict__ slots, const unsigned *__restrict__ items,
                              long long nmoves, int k, const long long *__restrict__ sweep_ptr,
                              const double *__restrict__ feed, long long feed_first, int width)
{
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= nmoves) return;
    const unsigned item = items[q / k];
    const int slot = (int)(item >> 16), r = (int)(item & 0xFFFFu), j = (int)(q % k);
    const Slot &S = slots[slot];
    const long long sweep = *sweep_ptr;
    const bool learned = S.L.tab != nullptr;
    const bool latent = S.draws2 != nullptr;
    const long long mv = (long long)r * k + j;
    double d[16];
    if (feed != nullptr && slot == 0) {
        const double *row = feed + ((sweep - feed_first) * (long long)S.g.R * k + mv) * width;
        for (int c = 0; c < width; ++c) d[c] = row[c];
    } else if (latent) {
        move_draws_arr(S.g.seed, S.chain, (uint32_t)sweep, (uint32_t)r, (uint32_t)j, d);
    } else if (learned) {
        move_draws16(S.g.seed, S.chain, (uint32_t)sweep, (uint32_t)r, (uint32_t)j, d);
    } else {
        move_draws(S.g.seed, S.chain, (uint32_t)sweep, (uint32_t)r, (uint32_t)j, d);
    }
    double *out = S.draws + mv * 8;
    for (int c = 0; c < 8; ++c) out[c] = d[c];
    if (learned) {
        double *raw = S.L.raw + mv * 8;
        for (int c = 0; c < 8; ++c) raw[c] = d[8 + c];
    }
    if (latent) {
        double *d2 = S.draws2 + mv * 8;
        for (int c = 0; c < 8; ++c) d2[c] = d[8 + c];
    }
}

// Learned births of one sweep, one wave per run of mpw <= 64 consecutive
// moves of a (slot, region): each birth move's proposal depends only on its
// draws and the sweep's partition, so it is derived here, off the sweep's
// dependent chain of moves.  The wave finds the region's stations and total
// anchor weight W_R; then lane l takes move l of its run.  With probability pl
// (regions holding a station) the anchor is picked by u_anchor W_R against
// the running weight sums (stations ascending, then windows), the component
// by u_comp against the cumulative mixture weights, and (x, y, t) = mean +
// sd * (truncated normals); otherwise (x, y, t) come from the prior on the
// region.  Either way log(b / p_R) at the proposal is then summed over
// (station, window) pairs across the lanes, one birth after another.
__global__ void __launch_bounds__(64)
k_learned_births(const Slot *__restrict__ slots, const unsigned *__restrict__ items, int k,
                 int mpw, int par, int *__restrict__ err)
{
    __shared__ int s_sta[kMaxRegSta];
    const int nrun = (k + mpw - 1) / mpw;
    const unsigned item = items[blockIdx.x / nrun];
    const int jbeg = (int)(blockIdx.x % nrun) * mpw, jend = min(k, jbeg + mpw);
    const int slot = (int)(item >> 16), r = (int)(item & 0xFFFFu), lane = threadIdx.x;
    // the table's pointers in registers (no reload after the stores below)
    const Learned L = slots[slot].L;
    if (L.tab == nullptr) return;
    const Geo &g = slots[slot].g;
    const double *offs = slots[slot].ev[par].off;
    const int i = r % g.nrx, kk = r / g.nrx;
    const double offx = offs[0], offy = offs[1];
    double x0, x1, y0, y1;
    region_span(offx, g.wx, g.Lx, i, &x0, &x1);
    region_span(offy, g.wy, g.Ly, kk, &y0, &y1);
    const double area = (x1 - x0) * (y1 - y0);
    const double c1 = g.c1, N = (double)g.N;
    const int ntau = L.ntau;
    // this lane's move and its draws, loaded before the region's stations
    const int j = jbeg + lane;
    const long long q = (long long)r * k + j;
    double d[4] = {1.0, 0.0, 0.0, 0.0}, e[6] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (j < jend) {
        for (int u = 0; u < 4; ++u) d[u] = slots[slot].draws[q * 8 + u];
        for (int u = 0; u < 6; ++u) e[u] = L.raw[q * 8 + u];  // draws 8..13
    }
    const bool birth = j < jend && d[0] < c1;
    int ns = region_stations_wave(g, offx, offy, i, kk, x0, x1, y0, y1, s_sta, kMaxRegSta, lane);
    if (ns > kMaxRegSta) {
        if (lane == 0) atomicOr(err, kFlagSta);
        ns = 0;
    }
    const double pl = ns > 0 ? L.pl : 0.0;
    // the stations' total anchor weights, loaded together (lane s, station
    // s), then one running total in station order: W and the walk below
    // add the same terms in the same order
    const double tot = lane < ns ? L.cum[(long long)s_sta[lane] * ntau + ntau - 1] : 0.0;
    double W = 0.0;
    for (int s = 0; s < ns; ++s) W = W + lane_f64(tot, s);
    const bool from_net = birth && pl > 0.0 && e[0] < pl;
    // anchor: the first station whose running total exceeds u_anchor W
    // (the last one if none), then the remainder within its windows
    const double target = e[1] * W;
    int pick = -1;
    double rem = 0.0, acc = 0.0;
    for (int s = 0; s < ns; ++s) {
        const double ts = lane_f64(tot, s);
        const double nxt = acc + ts;
        if (pick < 0 && target < nxt) {
            pick = s;
            rem = target - acc;
        }
        if (s == ns - 1 && pick < 0) {
            pick = s;
            rem = ts;
        }
        acc = nxt;
    }
    double x = 0.0, y = 0.0, t = 0.0;
    if (from_net) {
        const int sta = s_sta[pick];
        // smallest window w < ntau - 1 with rem < cum[w], else ntau - 1: an
        // eight-way search whose seven probes per level load together
        const double *cum = L.cum + (long long)sta * ntau;
        int lo = 0, hi = ntau - 1;
        while (lo < hi) {
            const int dd = hi - lo;
            double c[7];
#pragma unroll
            for (int u = 0; u < 7; ++u) c[u] = cum[lo + (u + 1) * dd / 8];
            int nlo = lo, nhi = hi;
#pragma unroll
            for (int u = 0; u < 7; ++u) {
                const int pu = lo + (u + 1) * dd / 8;
                if (rem < c[u]) nhi = min(nhi, pu);
                else nlo = max(nlo, pu + 1);
            }
            lo = nlo;
            hi = nhi;
        }
        // component: the first with u_comp below its cumulative weight (the
        // last if none)
        const double *T = L.tab + ((long long)sta * ntau + lo) * 64;
        double cw[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) cw[u] = T[8 * u + 7];
        int c = 7;
#pragma unroll
        for (int u = 6; u >= 0; --u)
            if (e[2] < cw[u]) c = u;
        x = T[8 * c + 0] + T[8 * c + 3] * e[3];
        y = T[8 * c + 1] + T[8 * c + 4] * e[4];
        t = T[8 * c + 2] + T[8 * c + 5] * e[5];
    } else if (birth) {
        x = x0 + d[1] * (x1 - x0);
        y = y0 + d[2] * (y1 - y0);
        t = d[3] * N;
    }
    if (j < jend && !birth) {
        double *lb = L.birth + q * 4;
        lb[0] = 0.0; lb[1] = 0.0; lb[2] = 0.0; lb[3] = 0.0;
    }
    // each birth's density, (station, window) pairs over the lanes
    unsigned long long todo = __ballot(birth);
    while (todo) {
        const int bl = __builtin_amdgcn_readfirstlane(__builtin_ctzll(todo));
        todo &= todo - 1;
        const double bx = lane_f64(x, bl), by = lane_f64(y, bl), bt = lane_f64(t, bl);
        double lr = 0.0;
        if (pl > 0.0) {
            int ilo, ihi;
            learned_windows(L, bt, &ilo, &ihi);
            const double S = wave_sum(learned_part(L, s_sta, ns, ilo, ihi, bx, by, bt, lane, 64));
            lr = learned_log_ratio(pl, S, W, area, g.N);
        }
        if (lane == bl) {
            double *lb = L.birth + q * 4;
            lb[0] = x; lb[1] = y; lb[2] = t; lb[3] = lr;
        }
    }
}

// Sample recording: after a sweep in [first, first + n), every chain's
// events (regions in order, each region's list in id order) are appended to
// rec[sweep - first][chain]: [0] the count, then (x, y, t, m) of the first
// max_events of them.  One workgroup per chain.
__global__ void __launch_bounds__(256)
k_record(const Slot *__restrict__ slots, int par, const long long *__restrict__ sweep_ptr,
         double *__restrict__ rec, long long first, long long n, int max_events)
{
    __shared__ int s_base[256];
    const long long sweep = *sweep_ptr;
    if (sweep < first || sweep >= first + n) return;
    const int slot = blockIdx.x, tid = threadIdx.x, chain = 0;
    const Geo g = slots[slot].g;
    const Events ev = slots[slot].ev[par];
    const long long stride = 1 + 4LL * max_events;
    double *out = rec + ((sweep - first) * gridDim.x + slot) * stride;
    int base = 0;
    // regions in chunks of 256: a block prefix sum of their counts places
    // each region's events
    for (int r0 = 0; r0 < g.R; r0 += 256) {
        const int r = r0 + tid;
        const int c = r < g.R ? ev.cnt[chain * g.R + r] : 0;
        s_base[tid] = c;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const int v = tid >= o ? s_base[tid - o] : 0;
            __syncthreads();
            s_base[tid] += v;
            __syncthreads();
        }
        const int excl = base + s_base[tid] - c;
        if (r < g.R) {
            const long long src = ((long long)chain * g.R + r) * g.cap;
            for (int s = 0; s < c; ++s) {
                const int o = excl + s;
                if (o >= max_events) break;
                out[1 + 4 * o + 0] = ev.x[src + s];
                out[1 + 4 * o + 1] = ev.y[src + s];
                out[1 + 4 * o + 2] = ev.t[src + s];
                out[1 + 4 * o + 3] = ev.m[src + s];
            }
        }
        base += s_base[255];
        __syncthreads();
    }
    if (tid == 0) out[0] = (double)base;
}

// Running sums of every station's anchor weights (one thread per station,
// windows in order).
__global__ void k_learned_cum(const double *__restrict__ w, int ntau, int nsta,
                              double *__restrict__ cum)
{
    const int st = blockIdx.x * blockDim.x + threadIdx.x;
    if (st >= nsta) return;
    double acc = 0.0;
    for (int i = 0; i < ntau; ++i) {
        acc = acc + w[(long long)st * ntau + i];
        cum[(long long)st * ntau + i] = acc;
    }
}

// Per component: log weight minus the log of its normaliser (product of the
// sds times (sqrt(2 pi) erf(4 / sqrt 2))^3), given lz3 = 3 log(sqrt(2 pi)
// erf(4 / sqrt 2)); and per block the min / max over components of mean t
// -/+ 4 sd t minus the anchor's window start.
__global__ void __launch_bounds__(256)
k_learned_norm(const double *__restrict__ tab, long long ncomp, int ntau, double lz3,
               double *__restrict__ norm, double *__restrict__ part)
{
    __shared__ double s_lo[256], s_hi[256];
    double lo = 1e300, hi = -1e300;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < ncomp;
         q += (long long)gridDim.x * blockDim.x) {
        const double *T = tab + q * 8;
        norm[q] = T[6] - log(T[3]) - log(T[4]) - log(T[5]) - lz3;
        const double tau = 32.0 * (double)((q / 8) % ntau);
        lo = fmin(lo, T[2] - 4.0 * T[5] - tau);
        hi = fmax(hi, T[2] + 4.0 * T[5] - tau);
    }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + o]);
            s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s_lo[0];
        part[2 * blockIdx.x + 1] = s_hi[0];
    }
}

__global__ void k_learned_reach(const double *__restrict__ part, int nblocks,
                                double *__restrict__ reach)
{
    double lo = 1e300, hi = -1e300;
    for (int b = 0; b < nblocks; ++b) {
        lo = fmin(lo, part[2 * b]);
        hi = fmax(hi, part[2 * b + 1]);
    }
    reach[0] = lo;
    reach[1] = hi;
}

// ------------------------------------------------------------------ rebin
// Dynamic partition (Section 4.3.2): the sweep's offset comes from Philox;
// each wave owns one region of the new layout and collects, in id order,
// the events of the old layout that fall into it.  With both offsets in
// [0, w) an event's region index moves by at most one per axis, so a 5x5
// window of old regions is always enough.  The lanes take the window's
// events side by side (flattened in window order, each old list in id
// order), a ballot packs the ones that land in the region, and each packed
// event's rank by (id, window position) places it, so that the list is in
// id order as the sweep kernels expect (equal ids keep window order).
constexpr int kRebinWaves = 4;

__global__ void __launch_bounds__(64 * kRebinWaves)
k_rebin(const Slot *__restrict__ slots, const unsigned *__restrict__ items, int nitems, int par,
        const long long *__restrict__ sweep_ptr, int *__restrict__ err)
{
    __shared__ int s_off[kRebinWaves][26];  // flat start of each old region of the window
    __shared__ int s_ro[kRebinWaves][25];
    __shared__ unsigned long long s_key[kRebinWaves][kMaxCap];
    __shared__ int s_f[kRebinWaves][kMaxCap];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q = blockIdx.x * kRebinWaves + wv;
    if (q >= nitems) return;  // whole waves; no workgroup barrier follows
    const unsigned item = items[q];
    const int slot = (int)(item >> 16), r = (int)(item & 0xFFFFu);
    const Geo &g = slots[slot].g;
    const Events src = slots[slot].ev[par], dst = slots[slot].ev[par ^ 1];
    const long long sweep = *sweep_ptr;
    double offx, offy;
    sweep_offset(g.seed, slots[slot].chain, (uint32_t)sweep, g.wx, g.wy, &offx, &offy);
    if (r == 0 && lane == 0) {
        dst.off[0] = offx;
        dst.off[1] = offy;
    }
    const int i = r % g.nrx, k = r / g.nrx;
    // the window's old regions (lane w < 25: row w / 5, column w % 5)
    int cnt = 0, ro = 0;
    if (lane < 25) {
        const int ko = k - 2 + lane / 5, io = i - 2 + lane % 5;
        if (ko >= 0 && ko <= g.gy && io >= 0 && io <= g.gx) {
            ro = ko * g.nrx + io;
            cnt = src.cnt[ro];
        }
    }
    const int start = wave_excl_prefix_small<7>(cnt);
    const int total = wave_sum_i32(cnt);
    if (lane < 25) {
        s_off[wv][lane] = start;
        s_ro[wv][lane] = ro;
    }
    if (lane == 25) s_off[wv][25] = total;
    __builtin_amdgcn_wave_barrier();
    int n = 0;
    for (int base = 0; base < total; base += 64) {
        const int f = base + lane;
        bool take = false;
        unsigned long long id = 0;
        if (f < total) {
            int w = 0;
            while (w < 24 && s_off[wv][w + 1] <= f) ++w;
            const long long e = (long long)s_ro[wv][w] * g.cap + (f - s_off[wv][w]);
            take = event_region(g, offx, offy, src.x[e], src.y[e], src.t[e]) == r;
            id = src.id[e];
        }
        const unsigned long long m = __ballot(take);
        const int pos = n + __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (take && pos < kMaxCap) {
            s_key[wv][pos] = id;
            s_f[wv][pos] = f;
        }
        n += __popcll(m);
    }
    if (n > g.cap) {
        if (lane == 0) atomicOr(err, kFlagCap);
        n = g.cap;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < n) {
        const unsigned long long key = s_key[wv][lane];
        const int f = s_f[wv][lane];
        int rank = 0;
        for (int o = 0; o < n; ++o) {
            const unsigned long long ko = s_key[wv][o];
            rank += ko < key || (ko == key && s_f[wv][o] < f);
        }
        int w = 0;
        while (w < 24 && s_off[wv][w + 1] <= f) ++w;
        const long long e = (long long)s_ro[wv][w] * g.cap + (f - s_off[wv][w]);
        const long long d = (long long)r * g.cap + rank;
        dst.x[d] = src.x[e];
        dst.y[d] = src.y[e];
        dst.t[d] = src.t[e];
        dst.m[d] = src.m[e];
        dst.id[d] = key;
        if (g.latent)
            for (int c = 0; c < 8; ++c) dst.da[d * 8 + c] = src.da[e * 8 + c];
    }
    if (lane == 0) dst.cnt[r] = n;
}

// ------------------------------------------------------- refresh / loglik
// Gathers, for one station and one tile of samples [n_lo, n_hi), every event
// of the table that reaches the station with a window meeting the tile, into
// LDS as (first sample, scale), in table order (regions in index order, each
// region's slots in id order).  The events of the few regions around the
// station are flattened and their arrivals computed by the whole
// workgroup; a block-wide prefix of ballots keeps the table order.
__device__ int gather_tile(const Geo &g, const Events &ev, int chain, int j, int n_lo, int n_hi,
                           int *s_n0, double *s_B, int *s_cnt, int *flags)
{
    __shared__ int s_roff[26];     // flat offsets of the regions around (at most 5 x 5)
    __shared__ int s_rid[25];
    __shared__ int s_wcnt[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ix = j % g.nsx, iy = j / g.nsx;
    if (tid == 0) {
        const double sx = station_pos(ix, g.ds), sy = station_pos(iy, g.ds);
        const double offx = ev.off[2 * chain], offy = ev.off[2 * chain + 1];
        int i0, i1, k0, k1;
        if (g.line) {  // onsets whose signal can meet the tile at any station
            i0 = region_axis((double)n_lo - g.tmax - (double)g.ts - 1.0 - g.arr_e, offx, g.wx,
                             g.gx);
            i1 = region_axis((double)n_hi + g.arr_e, offx, g.wx, g.gx);
            k0 = 0;
            k1 = 0;
        } else {
            i0 = region_axis(sx - g.rc, offx, g.wx, g.gx);
            i1 = region_axis(sx + g.rc, offx, g.wx, g.gx);
            k0 = region_axis(sy - g.rc, offy, g.wy, g.gy);
            k1 = region_axis(sy + g.rc, offy, g.wy, g.gy);
        }
        int nr = 0, off = 0;
        for (int kk = k0; kk <= k1; ++kk)
            for (int ii = i0; ii <= i1; ++ii) {
                if (nr < 25) {
                    const int r = kk * g.nrx + ii;
                    s_rid[nr] = r;
                    s_roff[nr] = off;
                    off += ev.cnt[chain * g.R + r];
                    ++nr;
                } else {
                    *flags |= kFlagTile;
                }
            }
        for (int q = nr; q < 26; ++q) s_roff[q] = off;
        *s_cnt = 0;
    }
    __syncthreads();
    const int total = s_roff[25];
    int count = 0;
    for (int base = 0; base < total; base += 256) {
        const int f = base + tid;
        bool take = false;
        Arrival ar;
        ar.in = 0; ar.n0 = 0; ar.n1 = 0; ar.B = 0.0;
        if (f < total) {
            int q = 0;
            while (q < 24 && s_roff[q + 1] <= f) ++q;
            const long long e = ((long long)chain * g.R + s_rid[q]) * g.cap + (f - s_roff[q]);
            ar = arrive(g, ev.x[e], ev.y[e], ev.t[e], ev.m[e],
                        g.line ? g.sx[ix] : station_pos(ix, g.ds),
                        g.line ? 0.0 : station_pos(iy, g.ds),
                        ev.da != nullptr ? ev.da[e * 8 + ix] : 0.0);
            take = ar.in && ar.n0 < n_hi && ar.n1 > n_lo;
        }
        const unsigned long long mask = __ballot(take);
        if (lane == 0) s_wcnt[wave] = __popcll(mask);
        __syncthreads();
        int before = __popcll(mask & ((1ull << lane) - 1ull));
        for (int w = 0; w < wave; ++w) before += s_wcnt[w];
        if (take) {
            const int pos = count + before;
            if (pos < kMaxTileEvents) {
                s_n0[pos] = ar.n0;
                s_B[pos] = ar.B;
            } else {
                *flags |= kFlagTile;
            }
        }
        count += (s_wcnt[0] + s_wcnt[1]) + (s_wcnt[2] + s_wcnt[3]);
        __syncthreads();
    }
    return count < kMaxTileEvents ? count : kMaxTileEvents;
}

// Exact event variance for every chain, station and sample, optionally
// written to E, and per-workgroup partial sums of the signal log-likelihood
// (Section 3: zero-mean Gaussian with variance sigma^2 plus the arriving
// signals' variances).  Under the mean-template likelihood the events' sum
// is the mean, E the residual trace - mean, and each sample a Gaussian of
// variance sigma^2 around the mean.  One workgroup per (station, tile),
// blockIdx.y chain.
template <typename TraceT>
__global__ void __launch_bounds__(256)
k_refresh(Geo g, Events ev, const TraceT *__restrict__ trace, double *__restrict__ E, int write,
          double *__restrict__ partials, int chain0, int *__restrict__ err)
{
    __shared__ int s_n0[kMaxTileEvents];
    __shared__ double s_B[kMaxTileEvents];
    __shared__ double s_T[kMaxTs];
    __shared__ double s_part[4];
    __shared__ int s_cnt;
    const int tiles = (g.N + kTile - 1) / kTile;
    const int j = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const int chain = chain0 + blockIdx.y;
    const int n_lo = tile * kTile, n_hi = min(n_lo + kTile, g.N);
    const int tid = threadIdx.x;
    int flags = 0;
    for (int q = tid; q < g.ts; q += 256) s_T[q] = exp(-(g.tmpl ? 1.0 : 2.0) * (double)q / g.decay);
    const int ne = gather_tile(g, ev, chain, j, n_lo, n_hi, s_n0, s_B, &s_cnt, &flags);
    const double l2pi = log(2.0 * M_PI);
    const double null_c = -0.5 * (l2pi + log(g.sigma2));
    const double null_q = -0.5 / g.sigma2;
    const long long row = (long long)j * g.N;
    double *Erow = E + (long long)chain * g.nsta * (long long)g.N + row;
    double acc = 0.0;
    // kRefreshU samples per thread per step, every trace load in flight
    // before any is used: raw elements, loaded unconditionally (past the
    // tile's end from its first sample) and converted only when used
    constexpr int U = kRefreshU;
    for (int base = n_lo + tid; base < n_hi; base += 256 * U) {
        TraceT tv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int nn = base + 256 * u;
            tv[u] = trace[row + (nn < n_hi ? nn : n_lo)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int nn = base + 256 * u;
            if (nn >= n_hi) break;
            const double svu = (double)tv[u];
            double e = 0.0;
            for (int q = 0; q < ne; ++q) {
                const int d = nn - s_n0[q];
                if (d >= 0 && d < g.ts) e += s_B[q] * s_T[d];
            }
            if (g.tmpl) {  // e is the mean; E holds the residual
                const double rr = svu - e;
                acc += null_c + null_q * (rr * rr);
                if (write) Erow[nn] = rr;
                continue;
            }
            const double qv = svu * svu;
            if (e > 0.0) {
                const double v = g.sigma2 + e;
                acc += -0.5 * (l2pi + log(v) + qv / v);
            } else {
                acc += null_c + null_q * qv;
            }
            if (write) Erow[nn] = e;
        }
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) s_part[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        partials[(long long)blockIdx.y * gridDim.x + blockIdx.x] =
            ((s_part[0] + s_part[1]) + s_part[2]) + s_part[3];
        if (flags) atomicOr(err, flags);
    }
}

// Every slot's exact event variance (the residual, under templates),
// recomputed from its events and written to E when `write` is set, and
// per-workgroup partial sums of its log-likelihood into partials[slot *
// per_max + block] when partials is not NULL (as k_refresh does for the
// chains of one instance).  Used after a naive phase (Algorithm 3), for the
// scheduled refresh and for the log-posterior of any state.  blockIdx.y
// slot, blockIdx.x (station, tile) of that slot; the slot's constants are
// staged in LDS (station positions are indexed).
template <typename TraceT>
__global__ void __launch_bounds__(256)
k_refresh_slots(const Slot *__restrict__ slots, int par, int write, double *__restrict__ partials,
                int per_max, int *__restrict__ err)
{
    __shared__ Geo s_g;
    __shared__ int s_n0[kMaxTileEvents];
    __shared__ double s_B[kMaxTileEvents];
    __shared__ double s_T[kMaxTs];
    __shared__ double s_part[4];
    __shared__ int s_cnt;
    const int slot = blockIdx.y, tid = threadIdx.x;
    if (tid == 0) s_g = slots[slot].g;
    __syncthreads();
    const Geo &g = s_g;
    const int tiles = (g.N + kTile - 1) / kTile;
    if ((int)blockIdx.x >= g.nsta * tiles) return;  // the slot has fewer tiles (whole block)
    const int j = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const int n_lo = tile * kTile, n_hi = min(n_lo + kTile, g.N);
    const Events ev = slots[slot].ev[par];
    const TraceT *__restrict__ trace = (const TraceT *)slots[slot].trace + (long long)j * g.N;
    double *__restrict__ Erow = slots[slot].E + (long long)j * g.N;
    int flags = 0;
    for (int q = tid; q < g.ts; q += 256) s_T[q] = exp(-(g.tmpl ? 1.0 : 2.0) * (double)q / g.decay);
    const int ne = gather_tile(g, ev, 0, j, n_lo, n_hi, s_n0, s_B, &s_cnt, &flags);
    const double l2pi = log(2.0 * M_PI);
    const double null_c = -0.5 * (l2pi + log(g.sigma2));
    const double null_q = -0.5 / g.sigma2;
    double acc = 0.0;
    // kRefreshU samples per thread per step, every trace load in flight
    // before any is used
    constexpr int U = kRefreshU;
    for (int base = n_lo + tid; base < n_hi; base += 256 * U) {
        TraceT tv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int nn = base + 256 * u;
            tv[u] = trace[nn < n_hi ? nn : n_lo];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int nn = base + 256 * u;
            if (nn >= n_hi) break;
            const double svu = (double)tv[u];
            double e = 0.0;
            for (int q = 0; q < ne; ++q) {
                const int d = nn - s_n0[q];
                if (d >= 0 && d < g.ts) e += s_B[q] * s_T[d];
            }
            if (g.tmpl) {  // e is the mean; E holds the residual
                const double rr = svu - e;
                acc += null_c + null_q * (rr * rr);
                if (write) Erow[nn] = rr;
                continue;
            }
            const double qv = svu * svu;
            if (e > 0.0) {
                const double v = g.sigma2 + e;
                acc += -0.5 * (l2pi + log(v) + qv / v);
            } else {
                acc += null_c + null_q * qv;
            }
            if (write) Erow[nn] = e;
        }
    }
    if (partials != nullptr) {
        acc = wave_sum(acc);
        if ((tid & 63) == 0) s_part[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0)
            partials[(long long)slot * per_max + blockIdx.x] =
                ((s_part[0] + s_part[1]) + s_part[2]) + s_part[3];
    }
    if (tid == 0 && flags) atomicOr(err, flags);
}

// Each slot's log-likelihood: its (station, tile) partials summed in a
// fixed order into out[2 slot].
__global__ void __launch_bounds__(256)
k_sum_slots(const Slot *__restrict__ slots, const double *__restrict__ partials, int per_max,
            double *__restrict__ out)
{
    __shared__ double s[256];
    const int slot = blockIdx.x;
    const Geo &g = slots[slot].g;
    const int nb = g.nsta * ((g.N + kTile - 1) / kTile);
    const double *p = partials + (long long)slot * per_max;
    double acc = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) acc += p[q];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[2 * slot] = s[0];
}

// Each slot's log prior of its current events (Section 3's prior as a set
// density): -lambda plus, per event, log lambda and the log densities of a
// uniform location on the domain (the line [0, x_max) in the line model), a
// uniform onset on [0, N) and, on the grid, an exponential magnitude above
// m_min; with latent arrivals each offset adds the log density of a normal
// of sd arrival_sd truncated at kArrTrunc sd (-inf outside).  Per-event terms
// summed in a fixed order into out[2 slot + 1].
__global__ void __launch_bounds__(256)
k_logprior_slots(const Slot *__restrict__ slots, int par, double *__restrict__ out)
{
    __shared__ double s[256];
    const int slot = blockIdx.x;
    const Geo &g = slots[slot].g;
    const Events ev = slots[slot].ev[par];
    const double per_event = g.line ? log(g.lambda) - log(g.Lx) - log((double)g.N)
                                    : log(g.lambda) - log(g.Lx * g.Ly) - log((double)g.N) +
                                          log(g.mrate);
    const double lz = g.latent ? log(g.arr_sd * sqrt(2.0 * M_PI) * erf(kArrTrunc / sqrt(2.0)))
                               : 0.0;
    double acc = 0.0;
    for (long long q = threadIdx.x; q < (long long)g.R * g.cap; q += 256) {
        const int r = (int)(q / g.cap), c = (int)(q % g.cap);
        if (c >= ev.cnt[r]) continue;
        double t = per_event;
        if (!g.line) t -= g.mrate * (ev.m[q] - g.mmin);
        if (g.latent)
            for (int jj = 0; jj < g.nsx; ++jj) {
                const double u = ev.da[q * 8 + jj] / g.arr_sd;
                t += fabs(u) > kArrTrunc ? -INFINITY : -0.5 * u * u - lz;
            }
        acc += t;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[2 * slot + 1] = s[0] - g.lambda;
}

// Sums each chain's partials in a fixed order (deterministic result).
__global__ void __launch_bounds__(256)
k_sum_partials(const double *__restrict__ partials, int per_chain, double *__restrict__ out)
{
    __shared__ double s[256];
    const double *p = partials + (long long)blockIdx.x * per_chain;
    double acc = 0.0;
    for (int q = threadIdx.x; q < per_chain; q += 256) acc += p[q];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

// ----------------------------------------------------------------- simulate
// trace[j][n] = sqrt(sigma^2 + E_j[n]) z_jn (mean-template likelihood:
// E_j[n] + sigma z_jn, E the sum of waveforms), z from Philox under key
// (seed, 0x80000001), counter (n / 2, j, 0, 0), Box-Muller (even n cosine,
// odd n sine).  E gathered from the truth events binned like an event table.
template <typename TraceT>
__global__ void __launch_bounds__(256)
k_simulate(Geo g, Events ev, uint32_t seed, TraceT *__restrict__ trace, int *__restrict__ err)
{
    __shared__ int s_n0[kMaxTileEvents];
    __shared__ double s_B[kMaxTileEvents];
    __shared__ double s_T[kMaxTs];
    __shared__ int s_cnt;
    const int tiles = (g.N + kTile - 1) / kTile;
    const int j = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const int n_lo = tile * kTile, n_hi = min(n_lo + kTile, g.N);
    const int tid = threadIdx.x;
    int flags = 0;
    for (int q = tid; q < g.ts; q += 256) s_T[q] = exp(-(g.tmpl ? 1.0 : 2.0) * (double)q / g.decay);
    const int ne = gather_tile(g, ev, 0, j, n_lo, n_hi, s_n0, s_B, &s_cnt, &flags);
    const long long row = (long long)j * g.N;
    for (int n2 = n_lo + 2 * tid; n2 < n_hi; n2 += 512) {
        uint32_t c[4] = {(uint32_t)(n2 >> 1), (uint32_t)j, 0u, 0u};
        philox10(c, seed, 0x80000001u);
        const double u1 = unit_open(c[0], c[1]);
        const double u2 = unit_open(c[2], c[3]);
        const double rad = sqrt(-2.0 * log(u1));
        const double ang = 2.0 * M_PI * u2;
        const double z[2] = {rad * cos(ang), rad * sin(ang)};
        for (int h = 0; h < 2; ++h) {
            const int nn = n2 + h;
            if (nn >= n_hi) break;
            double e = 0.0;
            for (int q = 0; q < ne; ++q) {
                const int d = nn - s_n0[q];
                if (d >= 0 && d < g.ts) e += s_B[q] * s_T[d];
            }
            trace[row + nn] = (TraceT)(g.tmpl ? e + sqrt(g.sigma2) * z[h]
                                              : sqrt(g.sigma2 + e) * z[h]);
        }
    }
    if (tid == 0 && flags) atomicOr(err, flags);
}

// --------------------------------------------------------------- utilities
__global__ void k_draws(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                        uint32_t j0, int count, int width, double *__restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    double d[16];
    if (width == 17)  // latent-arrival records (16 wide)
        move_draws_arr(seed, chain, sweep, region, j0 + (uint32_t)q, d);
    else if (width == 16)
        move_draws16(seed, chain, sweep, region, j0 + (uint32_t)q, d);
    else
        move_draws(seed, chain, sweep, region, j0 + (uint32_t)q, d);
    const int w = width == 17 ? 16 : width;
    for (int c = 0; c < w; ++c) out[(long long)q * w + c] = d[c];
}

// Residual of an empty world under the mean-template likelihood: the trace
// itself, copied into every chain's E (chain-major, per_chain elements each).
template <typename TraceT>
__global__ void k_residual_init(double *__restrict__ E, const TraceT *__restrict__ trace,
                                long long per_chain, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        E[q] = (double)trace[q % per_chain];
}

__global__ void k_fill_f64(double *__restrict__ p, long long n, double v)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        p[q] = v;
}

__global__ void k_fill_i32(int *__restrict__ p, long long n, int v)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        p[q] = v;
}

__global__ void k_fill_u64(unsigned long long *__restrict__ p, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        p[q] = 0ull;
}

__global__ void k_set_sweep(long long *p, long long v) { *p = v; }
__global__ void k_advance_sweep(long long *p) { *p += 1; }

// ------------------------------------------------------------- launchers
// OWN: the debug owner check's instantiations (the naive schedule has none).
template <typename TraceT, bool OWN>
static hipError_t launch_sweep_t(const Slot *slots, const unsigned *items, int nitems, int par,
                                 const long long *sweep_ptr, double *logp, long long log_first,
                                 long long log_n, int *err, int block, int naive_elems, int latent,
                                 const StampArg &sa, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    if (latent) {  // latent arrivals: the wave form (block 64) or the 256-thread latency form
        if (block == 64)
            k_sweep_wave<TraceT, false, true, OWN><<<(nitems + 3) / 4, 256, 0, s>>>(
                slots, items, nitems, par, sweep_ptr, logp, log_first, log_n, err, 0, sa, PersistArg{});
        else
            k_sweep_color<TraceT, 256, true, OWN><<<nitems, 256, 0, s>>>(
                slots, items, par, sweep_ptr, logp, log_first, log_n, err, sa);
        return hipGetLastError();
    }
    if (naive_elems > 0) {
        const size_t lds = (size_t)4 * naive_elems * sizeof(double);
        hipError_t e = hipFuncSetAttribute((const void *)k_sweep_wave<TraceT, true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        k_sweep_wave<TraceT, true><<<(nitems + 3) / 4, 256, lds, s>>>(
            slots, items, nitems, par, sweep_ptr, logp, log_first, log_n, err, naive_elems, sa,
            PersistArg{});
        return hipGetLastError();
    }
    switch (block) {
    case kSpecBase + 128:  // speculative form: one region per workgroup, D waves
        k_sweep_spec<TraceT, 2, OWN><<<nitems, 128, 0, s>>>(
            slots, items, par, sweep_ptr, logp, log_first, log_n, err, sa);
        break;
    case kSpecBase + 256:
        k_sweep_spec<TraceT, 4, OWN><<<nitems, 256, 0, s>>>(
            slots, items, par, sweep_ptr, logp, log_first, log_n, err, sa);
        break;
    case kSpecBase + 512:
        k_sweep_spec<TraceT, 8, OWN><<<nitems, 512, 0, s>>>(
            slots, items, par, sweep_ptr, logp, log_first, log_n, err, sa);
        break;
    case 64:  // one wave per work item, four per workgroup
        k_sweep_wave<TraceT, false, false, OWN><<<(nitems + 3) / 4, 256, 0, s>>>(
            slots, items, nitems, par, sweep_ptr, logp, log_first, log_n, err, 0, sa, PersistArg{});
        break;
    case 512:
        k_sweep_color<TraceT, 512, false, OWN><<<nitems, 512, 0, s>>>(
            slots, items, par, sweep_ptr, logp, log_first, log_n, err, sa);
        break;
    case 128:
        k_sweep_color<TraceT, 128, false, OWN><<<nitems, 128, 0, s>>>(
            slots, items, par, sweep_ptr, logp, log_first, log_n, err, sa);
        break;
    default:
        k_sweep_color<TraceT, 256, false, OWN><<<nitems, 256, 0, s>>>(
            slots, items, par, sweep_ptr, logp, log_first, log_n, err, sa);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_sweep(const Slot *slots, const unsigned *items, int nitems, int par, int f64,
                        const long long *sweep_ptr, double *logp, long long log_first,
                        long long log_n, int *err, int block, int naive_elems, int latent,
                        int owner, const StampArg &sa, hipStream_t s)
{
    if (f64)
        return owner ? launch_sweep_t<double, true>(slots, items, nitems, par, sweep_ptr, logp,
                                                    log_first, log_n, err, block, naive_elems,
                                                    latent, sa, s)
                     : launch_sweep_t<double, false>(slots, items, nitems, par, sweep_ptr, logp,
                                                     log_first, log_n, err, block, naive_elems,
                                                     latent, sa, s);
    return owner ? launch_sweep_t<float, true>(slots, items, nitems, par, sweep_ptr, logp,
                                               log_first, log_n, err, block, naive_elems, latent,
                                               sa, s)
                 : launch_sweep_t<float, false>(slots, items, nitems, par, sweep_ptr, logp,
                                                log_first, log_n, err, block, naive_elems, latent,
                                                sa, s);
}

// The persistent form over every colour of a sweep: `blocks` workgroups of
// four waves (enough to fill the device), each wave taking items by ticket.
template <typename TraceT, bool OWN>
static hipError_t launch_persist_t(const Slot *slots, const unsigned *items, int nitems, int par,
                                   const long long *sweep_ptr, double *logp, long long log_first,
                                   long long log_n, int *err, const StampArg &sa,
                                   const PersistArg &pq, int blocks, hipStream_t s)
{
    k_sweep_wave<TraceT, false, false, OWN, true><<<blocks, 256, 0, s>>>(
        slots, items, nitems, par, sweep_ptr, logp, log_first, log_n, err, 0, sa, pq);
    return hipGetLastError();
}

hipError_t launch_sweep_persist(const Slot *slots, const unsigned *items, int nitems, int par,
                                int f64, const long long *sweep_ptr, double *logp,
                                long long log_first, long long log_n, int *err, int owner,
                                const StampArg &sa, const PersistArg &pq, int nslots,
                                hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    // the queue's counters start from zero (a fill kernel, not a memset: the
    // launch may be captured into a graph)
    hipError_t e = fill_i32(pq.ticket, 1, 0, s);
    if (!e) e = fill_i32((int *)pq.done, nslots, 0, s);
    if (e) return e;
    int dev = 0, cus = 1, per_cu = 1;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev))) return e;
    const void *fn = f64 ? (owner ? (const void *)k_sweep_wave<double, false, false, true, true>
                                  : (const void *)k_sweep_wave<double, false, false, false, true>)
                         : (owner ? (const void *)k_sweep_wave<float, false, false, true, true>
                                  : (const void *)k_sweep_wave<float, false, false, false, true>);
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0)) != hipSuccess)
        return e;
    const int blocks = std::max(1, std::min((nitems + 3) / 4, per_cu * cus));
    if (f64)
        return owner ? launch_persist_t<double, true>(slots, items, nitems, par, sweep_ptr, logp,
                                                      log_first, log_n, err, sa, pq, blocks, s)
                     : launch_persist_t<double, false>(slots, items, nitems, par, sweep_ptr, logp,
                                                       log_first, log_n, err, sa, pq, blocks, s);
    return owner ? launch_persist_t<float, true>(slots, items, nitems, par, sweep_ptr, logp,
                                                 log_first, log_n, err, sa, pq, blocks, s)
                 : launch_persist_t<float, false>(slots, items, nitems, par, sweep_ptr, logp,
                                                  log_first, log_n, err, sa, pq, blocks, s);
}

hipError_t launch_refresh_slots(const Slot *slots, int nslots, int max_blocks, int par, int f64,
                                int *err, hipStream_t s, int write, double *partials, double *out)
{
    if (nslots <= 0 || max_blocks <= 0) return hipSuccess;
    const dim3 grid(max_blocks, nslots);
    double *part = out != nullptr ? partials : nullptr;
    if (f64)
        k_refresh_slots<double><<<grid, 256, 0, s>>>(slots, par, write, part, max_blocks, err);
    else
        k_refresh_slots<float><<<grid, 256, 0, s>>>(slots, par, write, part, max_blocks, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || out == nullptr) return e;
    k_sum_slots<<<nslots, 256, 0, s>>>(slots, partials, max_blocks, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_logprior_slots<<<nslots, 256, 0, s>>>(slots, par, out);
    return hipGetLastError();
}

constexpr long long kBirthWaves = 8192;

hipError_t launch_sweep_draws(const Slot *slots, const unsigned *items_all, int nall, int k,
                              int par, const long long *sweep_ptr, const double *feed,
                              long long feed_first, int width, bool learned, int *err,
                              hipStream_t s)
{
    const long long nmoves = (long long)nall * k;
    k_sweep_draws<<<(unsigned)((nmoves + 127) / 128), 128, 0, s>>>(slots, items_all, nmoves, k,
                                                                  sweep_ptr, feed, feed_first,
                                                                  width);
    hipError_t e = hipGetLastError();
    if (e || !learned) return e;
    // runs of up to 64 moves per wave, shorter while that leaves fewer than
    // kBirthWaves waves
    const int mpw = (int)std::max(1LL, std::min(64LL, std::min((long long)k, nmoves / kBirthWaves)));
    const long long nrun = (k + mpw - 1) / mpw;
    k_learned_births<<<(unsigned)(nall * nrun), 64, 0, s>>>(slots, items_all, k, mpw, par, err);
    return hipGetLastError();
}

hipError_t launch_record(const Slot *slots, int nslots, int par, const long long *sweep_ptr,
                         double *rec, long long first, long long n, int max_events, hipStream_t s)
{
    k_record<<<nslots, 256, 0, s>>>(slots, par, sweep_ptr, rec, first, n, max_events);
    return hipGetLastError();
}

int learned_norm_blocks(long long ncomp)
{
    const long long b = (ncomp + 255) / 256;
    return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_learned_prep(const double *w, const double *tab, int ntau, int nsta, double lz3,
                               double *cum, double *norm, double *part, double *reach,
                               hipStream_t s)
{
    k_learned_cum<<<(nsta + 127) / 128, 128, 0, s>>>(w, ntau, nsta, cum);
    hipError_t e = hipGetLastError();
    if (e) return e;
    const long long ncomp = (long long)nsta * ntau * 8;
    const int nb = learned_norm_blocks(ncomp);
    k_learned_norm<<<nb, 256, 0, s>>>(tab, ncomp, ntau, lz3, norm, part);
    if ((e = hipGetLastError())) return e;
    k_learned_reach<<<1, 1, 0, s>>>(part, nb, reach);
    return hipGetLastError();
}

hipError_t launch_rebin(const Slot *slots, const unsigned *items_all, int nall, int par,
                        const long long *sweep_ptr, int *err, hipStream_t s)
{
    k_rebin<<<(nall + kRebinWaves - 1) / kRebinWaves, 64 * kRebinWaves, 0, s>>>(
        slots, items_all, nall, par, sweep_ptr, err);
    return hipGetLastError();
}

int refresh_blocks(const Geo &g) { return g.nsta * ((g.N + kTile - 1) / kTile); }

hipError_t launch_refresh(const Geo &g, const Events &ev, const void *trace, int f64, double *E,
                          int write, double *partials, double *out, int chain0, int nchains,
                          int *err, hipStream_t s)
{
    const int per = refresh_blocks(g);
    const dim3 grid(per, nchains);
    if (f64)
        k_refresh<double><<<grid, 256, 0, s>>>(g, ev, (const double *)trace, E, write, partials,
                                               chain0, err);
    else
        k_refresh<float><<<grid, 256, 0, s>>>(g, ev, (const float *)trace, E, write, partials,
                                              chain0, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || out == nullptr) return e;
    k_sum_partials<<<nchains, 256, 0, s>>>(partials, per, out);
    return hipGetLastError();
}

hipError_t launch_simulate(const Geo &g, const Events &ev, uint32_t seed, void *trace, int f64,
                           int *err, hipStream_t s)
{
    const int per = refresh_blocks(g);
    if (f64)
        k_simulate<double><<<per, 256, 0, s>>>(g, ev, seed, (double *)trace, err);
    else
        k_simulate<float><<<per, 256, 0, s>>>(g, ev, seed, (float *)trace, err);
    return hipGetLastError();
}

hipError_t launch_draws(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                        uint32_t j0, int count, int width, double *out, hipStream_t s)
{
    k_draws<<<(count + 127) / 128, 128, 0, s>>>(seed, chain, sweep, region, j0, count, width, out);
    return hipGetLastError();
}

hipError_t residual_init(double *E, const void *trace, int f64, long long per_chain,
                         long long n, hipStream_t s)
{
    const long long nb = (n + 255) / 256;
    const int blocks = (int)(nb < 65536 ? nb : 65536);
    if (n <= 0) return hipSuccess;
    if (f64)
        k_residual_init<double><<<blocks, 256, 0, s>>>(E, (const double *)trace, per_chain, n);
    else
        k_residual_init<float><<<blocks, 256, 0, s>>>(E, (const float *)trace, per_chain, n);
    return hipGetLastError();
}

hipError_t fill_f64(double *p, long long n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    k_fill_f64<<<(unsigned)(blocks < 8192 ? blocks : 8192), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t fill_i32(int *p, long long n, int v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    k_fill_i32<<<(unsigned)(blocks < 8192 ? blocks : 8192), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t fill_u64(unsigned long long *p, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    k_fill_u64<<<(unsigned)(blocks < 8192 ? blocks : 8192), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t set_sweep(long long *p, long long v, hipStream_t s)
{
    k_set_sweep<<<1, 1, 0, s>>>(p, v);
    return hipGetLastError();
}

hipError_t advance_sweep(long long *p, hipStream_t s)
{
    k_advance_sweep<<<1, 1, 0, s>>>(p);
    return hipGetLastError();
}

}  // namespace cmh
