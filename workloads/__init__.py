"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds no arithmetic of the completion method itself: it only
produces operator entries, observed index sets, random starting cores and
the Gaussian matrices the low-rank to butterfly conversion draws.
"""
from .generators import (  # noqa: F401
    WORKLOADS,
    batched_instances,
    gaussian_sketches,
    radon_entries,
    random_lowrank,
    Workload,
    green_line_entries,
    green_planes_entries,
    morton_decode,
    make_workload,
    num_params,
    random_cores,
    sample_pairs,
    warm_params,
    green_geom_entries,
    observed_histogram,
    WARM_N,
    WARM_L,
    WARM_R,
    WARM_HIST_BINS,
)
