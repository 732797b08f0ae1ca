"""Pins of the oracle's aggregation (distance-2 MIS + aggregate growth).

The synchronous MIS-2 rounds with fixed priorities select exactly the
lexicographically-first maximal independent set of the squared graph G^2 in
descending (state, priority, id) order; the brute force below builds G^2 by
breadth-first search and runs the sequential greedy, which is an independent
characterisation of the same set.
"""

import collections
import os

import numpy as np
import pytest

import oracle
from workloads.q1 import config1_checkerboard_2d, layered_stack_3d, poisson_box

M64 = (1 << 64) - 1


def py_splitmix64(x):
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_splitmix64_published_sequence():
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seq0.txt")
    vals = [int(l, 16) for l in open(path) if l.strip() and not l.startswith("#")]
    for k, v in enumerate(vals):
        state = (k * 0x9E3779B97F4A7C15) & M64
        assert oracle.splitmix64(state) == v
        assert py_splitmix64(state) == v


def kept_graph(rowptr, col, mask):
    n = rowptr.shape[0] - 1
    adj = [[] for _ in range(n)]
    for i in range(n):
        for k in range(rowptr[i], rowptr[i + 1]):
            if mask[k] and col[k] != i:
                adj[i].append(int(col[k]))
    return adj


def bfs_dist(adj, s, cap=4):
    dist = {s: 0}
    q = collections.deque([s])
    while q:
        u = q.popleft()
        if dist[u] >= cap:
            continue
        for v in adj[u]:
            if v not in dist:
                dist[v] = dist[u] + 1
                q.append(v)
    return dist


def priorities(n, seed, level):
    key = py_splitmix64((seed + 1 + level) & M64)
    return [py_splitmix64(key ^ i) >> 34 for i in range(n)]


def check_aggregation(rowptr, col, mask, dirichlet, seed=0, level=0):
    n = rowptr.shape[0] - 1
    agg, nagg, rounds, roots = oracle.aggregate(rowptr, col, mask, dirichlet, seed=seed, level=level)
    adj = kept_graph(rowptr, col, mask)
    d = np.zeros(n, bool) if dirichlet is None else np.asarray(dirichlet, bool)
    # lexicographically-first MIS of G^2 in descending (priority, id) order
    pr = priorities(n, seed, level)
    order = sorted([i for i in range(n) if not d[i]], key=lambda i: (pr[i], i), reverse=True)
    chosen = np.zeros(n, bool)
    blocked = np.zeros(n, bool)
    for i in order:
        if blocked[i]:
            continue
        chosen[i] = True
        for v, dv in bfs_dist(adj, i, cap=2).items():
            blocked[v] = True
    assert np.array_equal(roots, chosen)
    # roots are numbered by ascending node index
    assert np.array_equal(agg[roots], np.arange(nagg))
    # disjoint cover of the non-Dirichlet nodes, Dirichlet excluded
    assert np.all(agg[d] == -1)
    assert np.all((agg[~d] >= 0) & (agg[~d] < nagg))
    # every aggregate is connected in the kept graph and contains its root
    for a in range(nagg):
        members = set(np.nonzero(agg == a)[0].tolist())
        r = int(np.nonzero(roots & (agg == a))[0][0])
        seen = {r}
        q = [r]
        while q:
            u = q.pop()
            for v in adj[u]:
                if v in members and v not in seen:
                    seen.add(v)
                    q.append(v)
        assert seen == members
    # phase 2: every neighbour of a root joined that root
    for r in np.nonzero(roots)[0]:
        for v in adj[r]:
            assert agg[v] == agg[r]
    return agg, nagg, roots


@pytest.mark.parametrize("seed", [0, 1, 12345])
def test_mis2_matches_lexicographic_first_mis_of_square_graph(seed):
    prob = poisson_box((9, 7), dirichlet="x0")
    sig = oracle.clement(prob.n, 2, prob.elem_nodes, prob.elem_sigma)
    d = oracle.detect_dirichlet(prob.rowptr, prob.col, prob.val)
    _, _, _, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, prob.coords, sig, dirichlet=d)
    check_aggregation(prob.rowptr, prob.col, mask, d, seed=seed)


def test_mis2_random_sparse_graph_with_isolated_nodes():
    rng = np.random.default_rng(3)
    n = 60
    A = np.zeros((n, n), bool)
    for _ in range(70):
        i, j = rng.integers(0, n, 2)
        if i != j:
            A[i, j] = A[j, i] = True
    np.fill_diagonal(A, True)
    rowptr = np.concatenate([[0], np.cumsum(A.sum(1))]).astype(np.int32)
    col = np.nonzero(A)[1].astype(np.int32)
    mask = np.ones(col.shape[0], bool)
    agg, nagg, roots = check_aggregation(rowptr, col, mask, None, seed=9, level=2)
    isolated = A.sum(1) == 1
    assert np.all(roots[isolated])          # isolated nodes become singleton aggregates


def test_phase3_joins_most_connected_phase2_aggregate():
    prob = poisson_box((12, 12), dirichlet="none")
    sig = oracle.clement(prob.n, 2, prob.elem_nodes, prob.elem_sigma)
    _, _, _, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, prob.coords, sig)
    agg, nagg, rounds, roots = oracle.aggregate(prob.rowptr, prob.col, mask, None, seed=4)
    adj = kept_graph(prob.rowptr, prob.col, mask)
    phase2 = np.full(prob.n, -1)
    for i in range(prob.n):
        if roots[i]:
            phase2[i] = agg[i]
        elif any(roots[j] for j in adj[i]):
            phase2[i] = agg[[j for j in adj[i] if roots[j]][0]]
    late = np.nonzero(phase2 < 0)[0]
    assert late.size > 0
    for i in late:
        counts = collections.Counter(int(phase2[j]) for j in adj[i] if phase2[j] >= 0)
        best = max(counts.values())
        assert agg[i] == min(a for a, c in counts.items() if c == best)


def test_aggregates_do_not_straddle_checkerboard_interfaces():
    """At theta = 0.08 the K=1 / K=1e6 interface edges are dropped, so no
    aggregate holds a node whose whole patch is low and one whose whole patch
    is high (two-domain discussion and the aggregation figure)."""
    prob = config1_checkerboard_2d(n=32, cells=4)
    h = oracle.Hierarchy(prob, max_coarse=50)
    agg = h.get(0, "agg")
    sig = oracle.clement(prob.n, 2, prob.elem_nodes, prob.elem_sigma)[:, 0]
    low = sig == 1.0
    high = sig == 1e6
    for a in range(agg.max() + 1):
        m = agg == a
        assert not (np.any(low & m) and np.any(high & m))


def test_layered_semicoarsening():
    """In a stretched layered stack the kept graph keeps (almost) no edge
    across the 1e-10 separator layers; aggregates stay inside one z-layer band."""
    prob = layered_stack_3d(n=8, repeats=2)
    h = oracle.Hierarchy(prob, max_coarse=20)
    agg = h.get(0, "agg")
    kz = prob.meta["layer_k"]
    z = np.rint(prob.coords[:, 2] * 8).astype(int)
    # nodes strictly inside a separator-adjacent plane pair never share an aggregate
    sep = np.nonzero(kz < 1e-7)[0]
    for e in sep:
        below, above = z == e, z == e + 1
        common = set(agg[below & (agg >= 0)]) & set(agg[above & (agg >= 0)])
        assert not common
