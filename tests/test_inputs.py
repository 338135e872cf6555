"""The seeded generators reproduce the recorded inputs (first 16 hex digits
of a sha256 over each array's dtype and bytes), so every measurement and
parity case names the same networks and demand."""
from __future__ import annotations

import hashlib

import numpy as np
import pytest

import synth

RECORDED = {
    "config1": ("7d2ab96b8b04697f", "91b1770ee2245b88"),
    "config2": ("9a61a4aa3049f72d", "d0fd32a338b7c434"),
}


def _h(*arrs):
    m = hashlib.sha256()
    for a in arrs:
        a = np.ascontiguousarray(a)
        m.update(str(a.dtype).encode())
        m.update(a.tobytes())
    return m.hexdigest()[:16]


@pytest.mark.parametrize("name", sorted(RECORDED))
def test_generator_reproduces_recorded_inputs(name):
    w = getattr(synth, name)()
    net, dem = w.net, w.demand
    assert (_h(net.row_ptr, net.col, net.fftt, net.cap), _h(dem.orig, dem.dest, dem.trips)) == RECORDED[name]
