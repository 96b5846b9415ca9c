"""Seeded synthetic inputs for the PAC stochastic-aggregation path.

This package only draws random tables (keys, foreign keys, group columns,
value columns, filter columns) with numpy's PCG64.  It holds none of the
method's arithmetic: no hashing of privacy-unit keys, no world masks, no
aggregation.  Both the CPU oracle and the GPU path read the same arrays from
here, and each side derives everything else on its own.
"""
from .gen import (  # noqa: F401
    CONFIG_SEEDS,
    FlatTable,
    StarTable,
    config1_flat,
    config2_star,
    config3_zipf,
    config4_float,
    config5_star,
    config5_queries,
    query_key,
    noise_seed,
    tiny_flat,
    tiny_star,
)
