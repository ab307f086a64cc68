"""Chromatic Metropolis-Hastings region sweep (Song & Moore, "Parallel
Chromatic MCMC with Spatial Partitioning") on AMD MI355X.

    chromh     ctypes binding of libchromh.so (include/chromh.h)
    workloads  workload constants and seeded input generators
    metrics    event matching, precision/recall/F1, location error, ESS
    build      compiles libchromh.so for gfx950
"""
