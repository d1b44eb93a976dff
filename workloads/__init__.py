"""Seeded synthetic workloads: the only code shared by the HIP path's callers and the oracle.

This package generates *inputs* (problem definitions, network weights, data vectors, Latin
hypercube designs, permutations).  It holds none of the sampling method's arithmetic: no
log-density, no gradient, no proposal, no accept rule.  Every array is drawn from numpy's
seeded PCG64 generator, so a (config, seed) pair always yields the same bytes.
"""
from .synth import (  # noqa: F401
    CONFIGS,
    mlp_nparams,
    mlp_layout,
    make_problem,
    spd_with_condition,
    xavier_mlp,
    latin_hypercube,
    minibatch_permutations,
    ar1_chains,
    small_problem,
    walsh_chains,
)
