"""Seeded OD demand generators.

A Demand is a list of trip legs (origin node p, destination node q, trips)
for one assignment interval of length dt_s seconds (dt_s = inf: plain static
assignment).  Legs with zero trips are dropped, as the assignment only visits
non-zero OD entries (Alg. 3).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Demand:
    orig: np.ndarray    # int32[P]
    dest: np.ndarray    # int32[P]
    trips: np.ndarray   # float64[P]  vehicles departing in the interval
    dt_s: float         # interval length (s); inf for plain static assignment

    @property
    def P(self) -> int:
        return int(self.orig.shape[0])

    def total(self) -> float:
        return float(self.trips.sum())


def _pairs(zones):
    Z = zones.shape[0]
    p = np.repeat(np.arange(Z), Z)
    q = np.tile(np.arange(Z), Z)
    off = p != q
    return p[off], q[off]


def poisson_all_pairs(zones: np.ndarray, mean: float, rng: np.random.Generator, dt_s: float) -> Demand:
    """Poisson(mean) trips for every ordered zone pair (p != q)."""
    p, q = _pairs(zones)
    trips = rng.poisson(mean, p.shape[0]).astype(np.float64)
    keep = trips > 0
    return Demand(zones[p[keep]].astype(np.int32), zones[q[keep]].astype(np.int32), trips[keep], dt_s)


def gravity_weights(xy: np.ndarray, zones: np.ndarray, sigma: float, decay_m: float,
                    rng: np.random.Generator):
    """Pair weights LogNormal(0, sigma) * exp(-d/decay) (Euclidean d), p != q."""
    p, q = _pairs(zones)
    d = np.sqrt(((xy[zones[p]] - xy[zones[q]]) ** 2).sum(1))
    w = rng.lognormal(0.0, sigma, p.shape[0]) * np.exp(-d / decay_m)
    return p, q, w


def gravity_trips(xy, zones, total_trips: int, sigma: float, decay_m: float,
                  rng: np.random.Generator, dt_s: float) -> Demand:
    """`total_trips` whole trips drawn multinomially over gravity weights."""
    p, q, w = gravity_weights(xy, zones, sigma, decay_m, rng)
    counts = rng.multinomial(total_trips, w / w.sum())
    keep = counts > 0
    return Demand(zones[p[keep]].astype(np.int32), zones[q[keep]].astype(np.int32),
                  counts[keep].astype(np.float64), dt_s)


def day_profile(N: int = 96, uniform: float = 0.71, peaks=((8.0, 1.5), (17.5, 1.5))) -> np.ndarray:
    """Share of the day's departures in each of N equal intervals: a uniform
    part plus equal-weight Gaussian peaks (hours), truncated to the day.
    With the defaults, 7-10 am carries about 18% of the day's trips."""
    from scipy.stats import norm
    edges = np.linspace(0.0, 24.0, N + 1)
    share = np.full(N, uniform / N)
    for mu, sd in peaks:
        cdf = norm.cdf(edges, mu, sd)
        mass = np.diff(cdf) / (cdf[-1] - cdf[0])
        share += (1.0 - uniform) / len(peaks) * mass
    return share / share.sum()


def day_demand(xy, zones, trips_per_day: int, rng: np.random.Generator, N: int = 96,
               sigma: float = 1.5, decay_m: float = 10_000.0, intervals=None) -> list:
    """Per-interval demand for a day: trips per interval = round(day * share),
    pairs drawn from the gravity weights (one weight draw for the whole day).
    `intervals` limits which intervals are materialised (others are None);
    the random stream is consumed identically either way."""
    p, q, w = gravity_weights(xy, zones, sigma, decay_m, rng)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    share = day_profile(N)
    counts = np.floor(trips_per_day * share + 0.5).astype(np.int64)
    out = []
    for i in range(N):
        u = rng.random(counts[i])
        if intervals is not None and i not in intervals:
            out.append(None)
            continue
        k = np.searchsorted(cdf, u, side="right").clip(0, p.shape[0] - 1)
        pair, c = np.unique(k, return_counts=True)
        out.append(Demand(zones[p[pair]].astype(np.int32), zones[q[pair]].astype(np.int32),
                          c.astype(np.float64), 900.0))
    return out
