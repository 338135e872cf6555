"""The named synthetic workloads.

Each stands in for the paper's proprietary Bay Area inputs (HERE map, SFCTA
demand), which are not available: shapes, sizes and value laws follow the
workload descriptions, the values themselves are seeded draws.

Seeds: numpy SeedSequence(2104129110 + config number), spawned into five
streams (topology, link attributes, zones, OD weights, trip sampling).
"""
from __future__ import annotations

import os
from dataclasses import dataclass

import numpy as np

from .demand import Demand, day_demand, gravity_trips, poisson_all_pairs
from .networks import Network, geometric_network, grid_network

BASE_SEED = 2104129110
CACHE_VERSION = "v1"


@dataclass
class Workload:
    name: str
    net: Network
    demand: Demand | list
    alpha: float = 0.15
    beta: int = 4
    extra: dict | None = None


def _streams(config: int):
    ss = np.random.SeedSequence(BASE_SEED + config)
    return [np.random.default_rng(s) for s in ss.spawn(5)]


def _cache_path(name):
    d = os.environ.get("QDTA_SYNTH_CACHE")
    if not d:
        return None
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, f"{name}_{CACHE_VERSION}.npz")


def _save_net(path, net: Network, extra: dict):
    arrs = dict(row_ptr=net.row_ptr, col=net.col, fftt=net.fftt, cap=net.cap,
                xy=net.xy if net.xy is not None else np.zeros((0, 2)),
                tier=net.tier if net.tier is not None else np.zeros(0, np.int8))
    arrs.update(extra)
    np.savez(path, **arrs)


def _load_net(path):
    z = np.load(path, allow_pickle=False)
    net = Network(int(z["row_ptr"].shape[0] - 1), z["row_ptr"], z["col"], z["fftt"], z["cap"],
                  xy=z["xy"] if z["xy"].size else None, tier=z["tier"] if z["tier"].size else None)
    return net, z


def paper_example():
    """The four-link, five-node serial example (Tables 3-4, section 6): free-flow
    times 10, 5, 10, 10 min and capacities 200, 150, 200, 200 veh/h; demand
    175 veh/h from node 1 to 4 in the first 15-min interval and 50 veh/h from
    node 3 to 5 in the second, none afterwards.  Nodes are numbered from 0 here
    (paper node k is node k-1); minutes are converted to seconds and rates to
    trips per 15-min interval."""
    row_ptr = np.array([0, 1, 2, 3, 4, 4], dtype=np.int32)
    col = np.array([1, 2, 3, 4], dtype=np.int32)
    fftt = np.array([600.0, 300.0, 600.0, 600.0], dtype=np.float32)
    cap = np.array([200.0, 150.0, 200.0, 200.0], dtype=np.float32)
    net = Network(5, row_ptr, col, fftt, cap, meta={"kind": "paper_example"})
    e = np.zeros(0, np.int32)
    ez = np.zeros(0)
    days = [
        Demand(np.array([0], np.int32), np.array([3], np.int32), np.array([175.0 / 4]), 900.0),
        Demand(np.array([2], np.int32), np.array([4], np.int32), np.array([50.0 / 4]), 900.0),
        Demand(e, e, ez, 900.0),
        Demand(e, e, ez, 900.0),
    ]
    return Workload("paper_example", net, days, alpha=0.15, beta=4)


def config1() -> Workload:
    """Plain static assignment, 20x20 directed grid (400 nodes, 1,520 links),
    free-flow U[30,120] s, capacity from {900,1800,3600}, 40 zones, Poisson(20)
    trips (veh/h) for every ordered zone pair."""
    topo, attr, zr, odr, _ = _streams(1)
    net = grid_network(20, attr)
    zones = np.sort(zr.choice(net.n, 40, replace=False)).astype(np.int32)
    dem = poisson_all_pairs(zones, 20.0, odr, dt_s=float("inf"))
    return Workload("config1", net, dem, extra={"zones": zones, "fw_iters": 50})


def _geometric(config, n_points, w, h, m_target, bay, zones_n):
    topo, attr, zr, odr, tr = _streams(config)
    path = _cache_path(f"config{config}_net_{n_points}")
    if path and os.path.exists(path):
        net, z = _load_net(path)
        zones = z["zones"]
    else:
        net = geometric_network(n_points, w, h, topo, m_target=m_target, bay=bay)
        zones = np.sort(zr.choice(net.n, zones_n, replace=False)).astype(np.int32)
        if path:
            _save_net(path, net, {"zones": zones})
    return net, zones, odr, tr


def config2() -> Workload:
    """One 15-min interval on a 100k-node planar metro network (~254k links),
    three speed tiers, 1,000 zones, 1M trips, lognormal(1.5) x exp(-d/10km)."""
    net, zones, odr, tr = _geometric(2, 100_000, 40_000.0, 40_000.0, None, False, 1000)
    dem = gravity_trips(net.xy, zones, 1_000_000, 1.5, 10_000.0, odr, dt_s=900.0)
    return Workload("config2", net, dem, extra={"zones": zones})


def _config3_net(scale=1.0):
    n = int(round(550_000 * scale))
    w, h = 120_000.0 * np.sqrt(scale), 100_000.0 * np.sqrt(scale)
    m_target = int(round(1_000_000 * scale))
    zones_n = max(10, int(round(5000 * scale)))
    return _geometric(3 if scale == 1.0 else 30, n, w, h, m_target, True, zones_n)


PEAK_INTERVAL = 32   # 08:00-08:15


def config3(interval: int = PEAK_INTERVAL) -> Workload:
    """Bay-Area-shaped network (~550k nodes, ~1.0M directed links, 5,000
    zones); the original legs of one 15-min interval of a 19M-trip day with a
    double-peak departure profile (default: the 08:00 peak interval)."""
    net, zones, odr, tr = _config3_net(1.0)
    days = day_demand(net.xy, zones, 19_000_000, odr, intervals={interval})
    return Workload("config3", net, days[interval], extra={"zones": zones, "interval": interval})


def config3_window(first: int, last: int = PEAK_INTERVAL) -> Workload:
    """The config-3 network with the original legs of intervals first..last
    of the same 19M-trip day (a list, one Demand per interval): running the
    earlier ones carries their residual demand into the last, as in the full
    day."""
    net, zones, odr, tr = _config3_net(1.0)
    want = set(range(first, last + 1))
    days = day_demand(net.xy, zones, 19_000_000, odr, intervals=want)
    return Workload("config3_window", net, [days[i] for i in range(first, last + 1)],
                    extra={"zones": zones, "first": first, "last": last})


def config3_day(scale: float = 1.0) -> Workload:
    """Full day (96 intervals) on the config-3 network; `scale` < 1 shrinks
    nodes, links, zones and trips together (1/20 scale for oracle runs)."""
    net, zones, odr, tr = _config3_net(scale)
    days = day_demand(net.xy, zones, int(round(19_000_000 * scale)), odr)
    return Workload(f"config3_day_{scale:g}", net, days, extra={"zones": zones})


def config4(count: int = 64, k_lo: int = 51, k_hi: int = 224, z_lo: int = 100, z_hi: int = 1000):
    """Independent grids of uneven size: side k uniform in [51, 224]
    (10,200 to 199,808 links), zones uniform in [100, 1000], config-1 laws."""
    topo, attr, zr, odr, tr = _streams(4)
    ks = topo.integers(k_lo, k_hi + 1, count)
    zs = topo.integers(z_lo, z_hi + 1, count)
    out = []
    for i in range(count):
        sub = np.random.default_rng(np.random.SeedSequence([BASE_SEED + 4, i]))
        net = grid_network(int(ks[i]), sub)
        z = int(min(zs[i], net.n))
        zones = np.sort(sub.choice(net.n, z, replace=False)).astype(np.int32)
        dem = poisson_all_pairs(zones, 20.0, sub, dt_s=float("inf"))
        out.append(Workload(f"config4_{i}", net, dem, extra={"zones": zones}))
    return out
