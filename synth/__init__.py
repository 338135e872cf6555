"""Seeded synthetic inputs (road networks, OD demand) for the QDTA hot path.

This package only draws random numbers and builds graphs.  It holds none of
the assignment arithmetic (no link costs, no shortest paths, no loading, no
line search): both the CPU oracle and the GPU library consume its arrays, and
neither side imports the other.
"""
from .networks import Network, grid_network, geometric_network, tiny_network
from .demand import Demand, poisson_all_pairs, gravity_trips, day_profile, day_demand
from .configs import config1, config2, config3, config3_day, config3_window, config4, paper_example

__all__ = [
    "Network", "grid_network", "geometric_network", "tiny_network",
    "Demand", "poisson_all_pairs", "gravity_trips", "day_profile", "day_demand",
    "config1", "config2", "config3", "config3_day", "config3_window", "config4", "paper_example",
]
