"""Pins of the oracle's shortest paths (Section 7.2) and of the R-MAT graph
generator, without a GPU.

The oracle (Dijkstra) is checked against things it does not share code with:
scipy's Dijkstra on random graphs, a brute-force Bellman-Ford written here on
tiny graphs, hand-worked small graphs, and the two properties that define
shortest-path distances on any graph: no edge can shorten a distance
(d[v] <= d[u] + w for every edge) and every reached vertex other than the
source is reached through a tight edge (d[v] = d[u] + w for some edge).
"""
import numpy as np
import pytest

import oracle
from paper_1701_01189_amd import inputs

INF = oracle.INF


def csr(nv, src, dst, w):
    src, dst, w = (np.asarray(a, dtype=np.int64) for a in (src, dst, w))
    order = np.argsort(src, kind="stable")
    row = np.zeros(nv + 1, dtype=np.uint64)
    np.cumsum(np.bincount(src, minlength=nv), out=row[1:])
    return row, dst[order].astype(np.uint32), w[order].astype(np.uint32)


def random_graph(seed, nv, ne, wmax):
    rng = np.random.default_rng(seed)
    s, d = rng.integers(0, nv, ne), rng.integers(0, nv, ne)
    return csr(nv, s, d, rng.integers(0, wmax + 1, ne))


def check_optimality(row, col, wt, src, dist):
    """The two defining properties, vectorised over every edge."""
    nv = len(row) - 1
    u = np.repeat(np.arange(nv), np.diff(row.astype(np.int64)))
    du = dist[u].astype(np.int64)
    dv = dist[col].astype(np.int64)
    reached = dist != INF
    assert dist[src] == 0
    # an edge out of a reached vertex reaches its target, no shorter than d[u] + w
    out_reached = du != INF
    assert reached[col[out_reached]].all()
    assert (dv[out_reached] <= du[out_reached] + wt[out_reached]).all()
    # every reached vertex but the source has a tight incoming edge
    tight = out_reached & (dv == du + wt)
    has_tight = np.zeros(nv, dtype=bool)
    has_tight[col[tight]] = True
    has_tight[src] = True
    assert (has_tight == reached).all()


def bellman_ford(nv, edges, src):
    d = [None] * nv
    d[src] = 0
    for _ in range(nv):
        for u, v, w in edges:
            if d[u] is not None and (d[v] is None or d[u] + w < d[v]):
                d[v] = d[u] + w
    return np.array([INF if x is None else x for x in d], dtype=np.uint32)


def test_hand_worked_graph():
    # 0 -> 1 (5), 0 -> 2 (9), 1 -> 2 (1), 2 -> 3 (0), 4 isolated, 3 -> 0 (7)
    row, col, wt = csr(5, [0, 0, 1, 2, 3], [1, 2, 2, 3, 0], [5, 9, 1, 0, 7])
    np.testing.assert_array_equal(oracle.sssp(row, col, wt, 0), [0, 5, 6, 6, INF])
    np.testing.assert_array_equal(oracle.sssp(row, col, wt, 3), [7, 12, 13, 0, INF])
    np.testing.assert_array_equal(oracle.sssp(row, col, wt, 4), [INF, INF, INF, INF, 0])


@pytest.mark.parametrize("seed", range(6))
def test_matches_scipy_dijkstra(seed):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    nv, ne = [(50, 200), (400, 3000), (1000, 1500), (300, 9000), (2, 1), (700, 0)][seed]
    row, col, wt = random_graph(100 + seed, nv, ne, [1000, 10, 0, 100000, 5, 1][seed])
    # scipy's sparse graphs hold one weight per vertex pair and may read a
    # stored zero as "no edge": keep the lightest of repeated edges, and use
    # positive weights (zero weights are pinned by Bellman-Ford below)
    if ne and wt.min() == 0:
        wt = wt + 1
    u = np.repeat(np.arange(nv), np.diff(row.astype(np.int64)))
    best = {}
    for a, b, w in zip(u.tolist(), col.tolist(), wt.tolist()):
        best[(a, b)] = min(w, best.get((a, b), w))
    keys = list(best)
    m = csr_matrix(([best[k] for k in keys], ([k[0] for k in keys], [k[1] for k in keys])),
                   shape=(nv, nv), dtype=np.float64)
    for src in (0, nv // 2, nv - 1):
        ref = dijkstra(m, directed=True, indices=src)
        exp = np.where(np.isinf(ref), INF, ref).astype(np.uint64).astype(np.uint32)
        np.testing.assert_array_equal(oracle.sssp(row, col, wt, src), exp)


@pytest.mark.parametrize("seed", range(8))
def test_matches_brute_force_bellman_ford(seed):
    rng = np.random.default_rng(200 + seed)
    nv = int(rng.integers(1, 12))
    ne = int(rng.integers(0, 40))
    s, d = rng.integers(0, nv, ne), rng.integers(0, nv, ne)
    w = rng.integers(0, [0, 3, 50, 1000][seed % 4] + 1, ne)  # zero weights included
    row, col, wt = csr(nv, s, d, w)
    edges = list(zip(s.tolist(), d.tolist(), w.tolist()))
    for src in range(nv):
        np.testing.assert_array_equal(oracle.sssp(row, col, wt, src), bellman_ford(nv, edges, src))


def test_optimality_on_rmat_and_random_graphs():
    row, col, wt = inputs.rmat_graph(9, 14, 60_000)
    dist = oracle.sssp(row, col, wt, 0)
    assert (dist != INF).sum() > 1000
    check_optimality(row, col, wt, 0, dist)
    row, col, wt = random_graph(31, 5000, 20000, 1000)
    check_optimality(row, col, wt, 17, oracle.sssp(row, col, wt, 17))


def test_special_cases():
    # one vertex, no edges
    row = np.zeros(2, dtype=np.uint64)
    e = np.zeros(0, dtype=np.uint32)
    np.testing.assert_array_equal(oracle.sssp(row, e, e, 0), [0])
    # all weights zero: every reached vertex is at distance 0 (reachability)
    row, col, wt = random_graph(41, 300, 400, 0)
    dist = oracle.sssp(row, col, wt, 5)
    assert set(np.unique(dist).tolist()) <= {0, INF}
    check_optimality(row, col, wt, 5, dist)
    # a path: distances are prefix sums of the weights
    w = np.arange(1, 100, dtype=np.int64) * 1000
    row, col, wt = csr(100, np.arange(99), np.arange(1, 100), w)
    np.testing.assert_array_equal(oracle.sssp(row, col, wt, 0),
                                  np.concatenate([[0], np.cumsum(w)]).astype(np.uint32))
    # a shortest path that does not fit in 32 bits is refused
    row, col, wt = csr(3, [0, 1], [1, 2], [0xFFFFFFF0, 0x20])
    with pytest.raises(ValueError):
        oracle.sssp(row, col, wt, 0)


def test_rmat_generator_shape():
    row, col, wt = inputs.rmat_graph(11, 10, 5000)
    nv = 1 << 10
    assert row.dtype == np.uint64 and len(row) == nv + 1 and row[0] == 0
    assert (np.diff(row.astype(np.int64)) >= 0).all() and row[-1] == len(col)
    assert col.max() < nv and wt.max() <= 1000
    u = np.repeat(np.arange(nv), np.diff(row.astype(np.int64)))
    assert (u != col).all()  # no self loops
    # every edge is stored in both directions with the same weight
    fwd = sorted(zip(u.tolist(), col.tolist(), wt.tolist()))
    rev = sorted(zip(col.tolist(), u.tolist(), wt.tolist()))
    assert fwd == rev
    assert len(col) % 2 == 0 and len(col) <= 2 * 5000
    # skew: an endpoint's top bit is 0 with probability a + b = a + c = 0.6,
    # so the lower half of the ids holds 60 % of the edge ends
    deg = np.diff(row.astype(np.int64))
    assert abs(deg[: nv // 2].sum() / deg.sum() - 0.6) < 0.03
    # deterministic
    r2, c2, w2 = inputs.rmat_graph(11, 10, 5000)
    assert (r2 == row).all() and (c2 == col).all() and (w2 == wt).all()
