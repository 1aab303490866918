"""Seeded synthetic inputs shared by the GPU path and the oracle.

This package holds no arithmetic of the sketching method itself: it only draws
the matrices that the method is run on (entry-generator tables, kernel points,
dense stand-ins) and the serving request stream.  Both sides consume exactly the
arrays produced here.
"""
from .gen import (  # noqa: F401
    MatrixSpec,
    rbf_mixture,
    lowrank_noise,
    dense_matrix,
    natural_scene_like,
    hubble_like,
    sparse_matrix,
    movie_like,
    newsgroup_like,
    block_replicated,
    exact_rank,
    config,
    CONFIGS,
    request_stream,
    request_matrix,
)
