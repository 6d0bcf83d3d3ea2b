"""Seeded synthetic warehouse inputs shared by the oracle and the HIP path.

This package only *draws* inputs: grid layouts, CSR arrays, weights, orders,
popularity samples and congestion ticks.  It contains none of the routing
arithmetic (no distances, no relaxation, no gather), so both sides of every
parity test may import it without sharing any of the method's code.
"""
from .grid import (  # noqa: F401
    GridGraph,
    rack_layout,
    cross_rows_every,
    aisle_adjacent_mask,
    build_grid_graph,
    free_mask,
)
from .orders import (  # noqa: F401
    uniform_orders,
    zipf_orders,
    poisson_arrivals,
    CongestionTicker,
)
from .configs import CONFIGS, make_config  # noqa: F401
