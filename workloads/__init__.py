"""Seeded synthetic inputs for the PAW-FE R-ChFSI filter path.

This package only draws random numbers and lays them out; it holds none of
the method's arithmetic (no finite-element tables, no projector integrals, no
filter).  Both the CPU oracle (``oracle/``) and the GPU library's callers
(tests, bench) take their inputs from here, so the two sides see identical
arrays without sharing any code that computes the method.
"""

from .configs import (  # noqa: F401
    System,
    CONFIGS,
    make_system,
    random_block,
    config_names,
)
