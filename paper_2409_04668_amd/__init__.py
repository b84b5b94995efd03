"""MI355X-native Monte Carlo transport hot path (fixed-source, time-dependent,
scatter + absorb) behind the C ABI of libmcdc.so.

Modules:
    mcdc       ctypes binding of libmcdc.so (raises if the library is not built)
    workloads  seeded synthetic problem descriptions
    build      hipcc build of libmcdc.so for gfx950
    learned_ww importance estimation, GPU MLP training and weight-window set-up
"""
