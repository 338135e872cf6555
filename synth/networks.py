"""Seeded road-network generators.

Every network is returned as a forward CSR (edges sorted by (tail, head)); the
edge id ("uid") of a link is its position in that CSR.  Free-flow times are in
seconds (float32) and capacities in vehicles per hour (float32), the inputs of
the BPR curve (Eq. 1, section 3.2).  Nothing here evaluates a link cost.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components, dijkstra
from scipy.spatial import Delaunay


@dataclass
class Network:
    n: int
    row_ptr: np.ndarray          # int32[n+1]
    col: np.ndarray              # int32[m]   head node of each link
    fftt: np.ndarray             # float32[m] free-flow time c_0 (s)
    cap: np.ndarray              # float32[m] capacity C_a (veh/h)
    xy: np.ndarray | None = None  # float64[n,2] node coordinates (m), unused by the method
    tier: np.ndarray | None = None  # int8[m] 0 local, 1 arterial, 2 highway
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def tails(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.row_ptr)).astype(np.int32)


def _csr_from_edges(n, tail, head, *arrays):
    order = np.lexsort((head, tail))
    tail = tail[order]
    head = head[order]
    counts = np.bincount(tail, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    out = [row_ptr.astype(np.int32), head.astype(np.int32)]
    out.extend(a[order] for a in arrays)
    return out


# --------------------------------------------------------------------------
# Grid networks (four-neighbour lattice, links both ways)
# --------------------------------------------------------------------------
def grid_network(k: int, rng: np.random.Generator, cost_lo=30.0, cost_hi=120.0,
                 caps=(900.0, 1800.0, 3600.0)) -> Network:
    """k x k grid, node r*k+c, a link each way between 4-neighbours.

    Link count 4k(k-1).  Free-flow times U[cost_lo, cost_hi] s, capacity drawn
    uniformly from `caps`.  Draws happen in CSR order, so the seed fixes them.
    """
    r, c = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    node = (r * k + c).ravel()
    right = node[(c < k - 1).ravel()]
    down = node[(r < k - 1).ravel()]
    u = np.concatenate([right, right + 1, down, down + k])
    v = np.concatenate([right + 1, right, down + k, down])
    row_ptr, col = _csr_from_edges(k * k, u, v)
    m = col.shape[0]
    fftt = rng.uniform(cost_lo, cost_hi, m).astype(np.float32)
    cap = rng.choice(np.asarray(caps, dtype=np.float32), m)
    xy = np.stack([c.ravel() * 500.0, r.ravel() * 500.0], axis=1).astype(np.float64)
    return Network(k * k, row_ptr, col, fftt, cap, xy=xy, meta={"kind": "grid", "k": k})


# --------------------------------------------------------------------------
# Geometric planar networks (relative neighbourhood graph)
# --------------------------------------------------------------------------
def _hilbert_index(ix, iy, order=16):
    """Hilbert curve position of integer points on a 2^order grid (vectorised)."""
    ix = ix.astype(np.int64).copy()
    iy = iy.astype(np.int64).copy()
    d = np.zeros_like(ix)
    s = 1 << (order - 1)
    while s > 0:
        rx = ((ix & s) > 0).astype(np.int64)
        ry = ((iy & s) > 0).astype(np.int64)
        d += s * s * ((3 * rx) ^ ry)
        # rotate quadrant
        flip = ry == 0
        swap_x = flip & (rx == 1)
        ix = np.where(swap_x, s - 1 - ix, ix)
        iy = np.where(swap_x, s - 1 - iy, iy)
        tmp = np.where(flip, ix, iy)
        ix = np.where(flip, iy, ix)
        iy = tmp
        s >>= 1
    return d


def _rng_edges(pts):
    """Edges of the relative neighbourhood graph, filtered from the Delaunay
    triangulation: (u,v) is dropped when some Delaunay neighbour w of u or v
    is strictly closer to both endpoints than they are to each other."""
    tri = Delaunay(pts)
    s = tri.simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]])
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    n = pts.shape[0]
    # undirected neighbour CSR of the triangulation
    a = np.concatenate([e[:, 0], e[:, 1]])
    b = np.concatenate([e[:, 1], e[:, 0]])
    order = np.argsort(a, kind="stable")
    a, b = a[order], b[order]
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(a, minlength=n), out=ptr[1:])
    L2 = ((pts[e[:, 0]] - pts[e[:, 1]]) ** 2).sum(1)
    witness = np.zeros(e.shape[0], dtype=bool)
    for end in (0, 1):
        src = e[:, end]
        deg = ptr[src + 1] - ptr[src]
        eid = np.repeat(np.arange(e.shape[0]), deg)
        starts = np.repeat(ptr[src], deg)
        offs = np.arange(eid.shape[0]) - np.repeat(np.cumsum(deg) - deg, deg)
        w = b[starts + offs]
        u, v = e[eid, 0], e[eid, 1]
        du = ((pts[w] - pts[u]) ** 2).sum(1)
        dv = ((pts[w] - pts[v]) ** 2).sum(1)
        hit = (w != u) & (w != v) & (np.maximum(du, dv) < L2[eid])
        witness[np.unique(eid[hit])] = True
    return e[~witness]


def _corridor_edges(pts, und, lines, axis, band, rng_len):
    """Mark a continuous corridor along each line: the shortest path (by
    length) inside a band around the line between its two extreme nodes."""
    n = pts.shape[0]
    length = np.sqrt(((pts[und[:, 0]] - pts[und[:, 1]]) ** 2).sum(1))
    marked = np.zeros(und.shape[0], dtype=bool)
    eid_of = {}
    for pos in lines:
        for widen in (1.0, 2.0, 4.0):
            in_band = np.abs(pts[:, 1 - axis] - pos) < band * widen
            sel = in_band[und[:, 0]] & in_band[und[:, 1]]
            idx = np.nonzero(sel)[0]
            if idx.size == 0:
                continue
            nodes = np.nonzero(in_band)[0]
            local = -np.ones(n, dtype=np.int64)
            local[nodes] = np.arange(nodes.size)
            uu, vv = local[und[idx, 0]], local[und[idx, 1]]
            g = coo_matrix((length[idx], (uu, vv)), shape=(nodes.size, nodes.size)).tocsr()
            ncomp, lab = connected_components(g, directed=False)
            big = np.argmax(np.bincount(lab))
            cand = np.nonzero(lab == big)[0]
            coord = pts[nodes[cand], axis]
            if coord.max() - coord.min() < 0.8 * rng_len:
                continue
            s, t = cand[np.argmin(coord)], cand[np.argmax(coord)]
            _, pred = dijkstra(g, directed=False, indices=s, return_predecessors=True)
            path = [t]
            while path[-1] != s and pred[path[-1]] >= 0:
                path.append(pred[path[-1]])
            path = nodes[np.asarray(path)]
            if not eid_of:
                key = np.minimum(und[:, 0], und[:, 1]) * n + np.maximum(und[:, 0], und[:, 1])
                eid_of["key"] = key
                eid_of["order"] = np.argsort(key)
            key = eid_of["key"]
            order = eid_of["order"]
            pk = np.minimum(path[:-1], path[1:]) * n + np.maximum(path[:-1], path[1:])
            where = order[np.searchsorted(key[order], pk)]
            marked[where] = True
            break
    return marked


def _dfs_orientation(n, und):
    """Depth-first orientation (tree edges parent->child, back edges
    descendant->ancestor) and the bridge flags of an undirected graph.
    Orienting every non-bridge edge this way and keeping bridges two-way gives
    a strongly connected digraph (Robbins' theorem)."""
    E = und.shape[0]
    a = np.concatenate([und[:, 0], und[:, 1]])
    b = np.concatenate([und[:, 1], und[:, 0]])
    eid = np.concatenate([np.arange(E), np.arange(E)])
    order = np.argsort(a, kind="stable")
    b, eid = b[order], eid[order]
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(a, minlength=n), out=ptr[1:])
    ptr_l, b_l, eid_l = ptr.tolist(), b.tolist(), eid.tolist()
    disc = [-1] * n
    low = [0] * n
    forward = [True] * E          # True: und[e,0] -> und[e,1]
    bridge = [False] * E
    used = [False] * E
    t = 0
    for root in range(n):
        if disc[root] >= 0:
            continue
        disc[root] = low[root] = t
        t += 1
        stack = [(root, -1, ptr_l[root])]
        while stack:
            u, pe, i = stack[-1]
            if i < ptr_l[u + 1]:
                stack[-1] = (u, pe, i + 1)
                w, e = b_l[i], eid_l[i]
                if used[e]:
                    continue
                used[e] = True
                forward[e] = (und[e, 0] == u)   # oriented u -> w
                if disc[w] < 0:
                    disc[w] = low[w] = t
                    t += 1
                    stack.append((w, e, ptr_l[w]))
                else:
                    if disc[w] < low[u]:
                        low[u] = disc[w]
            else:
                stack.pop()
                if stack:
                    p = stack[-1][0]
                    if low[u] < low[p]:
                        low[p] = low[u]
                    if low[u] > disc[p]:
                        bridge[pe] = True
    return np.asarray(forward), np.asarray(bridge)


def geometric_network(n_points: int, width_m: float, height_m: float, rng: np.random.Generator,
                      m_target: int | None = None, bay: bool = False,
                      highway_every_m=10_000.0, arterial_every_m=2_000.0,
                      speeds_kmh=(40.0, 60.0, 100.0), caps=(900.0, 1800.0, 3600.0)) -> Network:
    """Planar road-like network: relative neighbourhood graph of uniform points.

    Three speed tiers by corridor overlay (continuous paths along lines every
    `highway_every_m` / `arterial_every_m`).  With `m_target` below twice the
    undirected edge count, a random subset of non-bridge, non-highway edges is
    made one-way along a depth-first orientation so the result stays strongly
    connected.  Nodes are numbered along a Hilbert curve.
    """
    if bay:
        # an elliptical "water" body; draw extra points so about n_points remain
        cx, cy, ax, ay = 0.42 * width_m, 0.55 * height_m, 0.12 * width_m, 0.22 * height_m
        frac = np.pi * ax * ay / (width_m * height_m)
        pts = rng.uniform((0, 0), (width_m, height_m), size=(int(n_points / (1 - frac) * 1.02) + 16, 2))
        keep = ((pts[:, 0] - cx) / ax) ** 2 + ((pts[:, 1] - cy) / ay) ** 2 > 1.0
        pts = pts[keep][:n_points]
    else:
        pts = rng.uniform((0, 0), (width_m, height_m), size=(n_points, 2))
    und = _rng_edges(pts)
    # largest connected component (the RNG is connected, this is a guard)
    g = coo_matrix((np.ones(und.shape[0]), (und[:, 0], und[:, 1])), shape=(pts.shape[0],) * 2)
    ncomp, lab = connected_components(g, directed=False)
    if ncomp > 1:
        big = np.argmax(np.bincount(lab))
        keep = lab == big
        remap = -np.ones(pts.shape[0], dtype=np.int64)
        remap[keep] = np.arange(keep.sum())
        und = und[keep[und[:, 0]] & keep[und[:, 1]]]
        und = remap[und]
        pts = pts[keep]
    n = pts.shape[0]
    # Hilbert numbering
    scale = (1 << 16) - 1
    hx = np.floor(pts[:, 0] / width_m * scale).clip(0, scale)
    hy = np.floor(pts[:, 1] / height_m * scale).clip(0, scale)
    perm = np.argsort(_hilbert_index(hx, hy), kind="stable")
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    pts = pts[perm]
    und = inv[und]
    # speed tiers
    tier = np.zeros(und.shape[0], dtype=np.int8)
    spacing = np.sqrt(width_m * height_m / n)
    for every, tval in ((arterial_every_m, 1), (highway_every_m, 2)):
        for axis, extent, other in ((0, width_m, height_m), (1, height_m, width_m)):
            lines = np.arange(every / 2, other, every)
            mk = _corridor_edges(pts, und, lines, axis, band=2.0 * spacing, rng_len=extent)
            tier[mk] = np.maximum(tier[mk], tval)
    # directions
    E = und.shape[0]
    oneway = np.zeros(E, dtype=bool)
    forward = np.ones(E, dtype=bool)
    if m_target is not None and m_target < 2 * E:
        forward, bridge = _dfs_orientation(n, und)
        cand = np.nonzero(~bridge & (tier < 2))[0]
        k = min(2 * E - m_target, cand.size)
        oneway[rng.choice(cand, size=k, replace=False)] = True
    u0 = np.where(forward, und[:, 0], und[:, 1])
    v0 = np.where(forward, und[:, 1], und[:, 0])
    two = ~oneway
    tail = np.concatenate([u0, v0[two]])
    head = np.concatenate([v0, u0[two]])
    etier = np.concatenate([tier, tier[two]])
    length = np.sqrt(((pts[tail] - pts[head]) ** 2).sum(1))
    row_ptr, col, etier, length = _csr_from_edges(n, tail, head, etier, length)
    speed = np.asarray(speeds_kmh)[etier] / 3.6
    fftt = (length / speed).astype(np.float32)
    fftt = np.maximum(fftt, np.float32(0.5))
    cap = np.asarray(caps, dtype=np.float32)[etier]
    return Network(n, row_ptr, col, fftt, cap, xy=pts, tier=etier,
                   meta={"kind": "rng", "width_m": width_m, "height_m": height_m,
                         "undirected": int(E), "oneway": int(oneway.sum())})


# --------------------------------------------------------------------------
# Tiny networks for brute-force checks
# --------------------------------------------------------------------------
def tiny_network(n: int, extra: int, rng: np.random.Generator, costs: str = "float",
                 parallel: bool = True) -> Network:
    """Strongly connected digraph on n nodes: a random Hamiltonian cycle plus
    `extra` random links (parallel links allowed when `parallel`).

    costs: "float"  U(1, 100) float32
           "int"    integers 1..6 (many exact ties)
           "huge"   mixes 1e8-scale and O(1) costs (float32 absorption)
    """
    perm = rng.permutation(n)
    tail = list(perm)
    head = list(np.roll(perm, -1))
    seen = set(zip(tail, head))
    tries = 0
    while len(tail) < n + extra and tries < 100 * (extra + 1):
        tries += 1
        u, v = rng.integers(0, n, 2)
        if u == v:
            continue
        if not parallel and (u, v) in seen:
            continue
        seen.add((u, v))
        tail.append(u)
        head.append(v)
    tail = np.asarray(tail, dtype=np.int64)
    head = np.asarray(head, dtype=np.int64)
    m = tail.size
    if costs == "float":
        c = rng.uniform(1.0, 100.0, m)
    elif costs == "int":
        c = rng.integers(1, 7, m).astype(np.float64)
    elif costs == "huge":
        c = np.where(rng.random(m) < 0.5, rng.uniform(1e8, 4e8, m), rng.uniform(0.5, 8.0, m))
    else:
        raise ValueError(costs)
    row_ptr, col, c = _csr_from_edges(n, tail, head, c)
    cap = rng.choice(np.asarray([900.0, 1800.0, 3600.0], dtype=np.float32), m)
    return Network(n, row_ptr, col, c.astype(np.float32), cap, meta={"kind": "tiny"})
