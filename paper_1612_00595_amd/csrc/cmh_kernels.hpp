// cmh_kernels.hpp -- host-side launchers of the device kernels.
#pragma once

#include "cmh_common.hpp"

namespace cmh {

hipError_t launch_sweep(const Slot *slots, const unsigned *items, int nitems, int par, int f64,
                        const long long *sweep_ptr, double *logp, long long log_first,
                        long long log_n, int *err, int block, int naive_elems, int latent,
                        int owner, const StampArg &sa, hipStream_t s);
// Every slot's event variance recomputed (written to E when `write`); with
// out, also each slot's log-likelihood and log prior into out[2 slot],
// out[2 slot + 1] (partials: max_blocks doubles per slot).
// The persistent form: every colour of a sweep in one launch over items in
// colour order (pq.wait per item); clears the queue's counters first.
hipError_t launch_sweep_persist(const Slot *slots, const unsigned *items, int nitems, int par,
                                int f64, const long long *sweep_ptr, double *logp,
                                long long log_first, long long log_n, int *err, int owner,
                                const StampArg &sa, const PersistArg &pq, int nslots,
                                hipStream_t s);
hipError_t launch_refresh_slots(const Slot *slots, int nslots, int max_blocks, int par, int f64,
                                int *err, hipStream_t s, int write = 1,
                                double *partials = nullptr, double *out = nullptr);
hipError_t launch_sweep_draws(const Slot *slots, const unsigned *items_all, int nall, int k,
                              int par, const long long *sweep_ptr, const double *feed,
                              long long feed_first, int width, bool learned, int *err,
                              hipStream_t s);
hipError_t launch_record(const Slot *slots, int nslots, int par, const long long *sweep_ptr,
                         double *rec, long long first, long long n, int max_events, hipStream_t s);
int learned_norm_blocks(long long ncomp);
hipError_t launch_learned_prep(const double *w, const double *tab, int ntau, int nsta, double lz3,
                               double *cum, double *norm, double *part, double *reach,
                               hipStream_t s);
hipError_t launch_rebin(const Slot *slots, const unsigned *items_all, int nall, int par,
                        const long long *sweep_ptr, int *err, hipStream_t s);
int refresh_blocks(const Geo &g);
hipError_t launch_refresh(const Geo &g, const Events &ev, const void *trace, int f64, double *E,
                          int write, double *partials, double *out, int chain0, int nchains,
                          int *err, hipStream_t s);
hipError_t launch_simulate(const Geo &g, const Events &ev, uint32_t seed, void *trace, int f64,
                           int *err, hipStream_t s);
hipError_t launch_draws(uint32_t seed, uint32_t chain, uint32_t sweep, uint32_t region,
                        uint32_t j0, int count, int width, double *out, hipStream_t s);
hipError_t residual_init(double *E, const void *trace, int f64, long long per_chain,
                         long long n, hipStream_t s);
hipError_t fill_f64(double *p, long long n, double v, hipStream_t s);
hipError_t fill_i32(int *p, long long n, int v, hipStream_t s);
hipError_t fill_u64(unsigned long long *p, long long n, hipStream_t s);
hipError_t set_sweep(long long *p, long long v, hipStream_t s);
hipError_t advance_sweep(long long *p, hipStream_t s);

}  // namespace cmh
