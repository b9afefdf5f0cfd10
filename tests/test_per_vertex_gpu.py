"""Per-vertex biclique counts (the output set of Algorithm 1 as membership
counts) on the device against the oracle's, vertex by vertex."""
import math

import numpy as np
import pytest

import oracle
from paper_2403_07858_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def bc():
    import torch
    assert torch.cuda.is_available()
    from paper_2403_07858_amd import bc as m
    return m


QUERIES = [(1, 2), (2, 1), (2, 2), (2, 3), (3, 2), (3, 3), (4, 3), (3, 4), (4, 4)]


@pytest.mark.parametrize("shape", [(400, 200, 8000, 2.0, 150, 71), (500, 250, 7000, 2.2, 120, 74)])
def test_per_vertex_matches_oracle(bc, shape):
    n_u, n_v, m, beta, dmax, seed = shape
    g = gg.chung_lu_bipartite(n_u, n_v, m, beta, beta, dmax, dmax, seed=seed)
    G = bc.build_graph(g)
    for p, q in QUERIES:
        want_u, want_v = oracle.count_per_vertex(g, p, q)
        got_u = bc.bc_count_per_vertex(G, p, q, bc.BC_ANCHOR_U)
        got_v = bc.bc_count_per_vertex(G, p, q, bc.BC_ANCHOR_V)
        assert got_u == want_u, ("U", p, q)
        assert got_v == want_v, ("V", p, q)
        total = bc.bc_count(G, p, q)
        assert sum(got_u) == p * total and sum(got_v) == q * total
        say(shape, (p, q), "total", total, "nonzero U", sum(1 for x in got_u if x), "V", sum(1 for x in got_v if x))


def test_per_vertex_sorted_lists_and_closed_forms(bc):
    # the sorted-list comparator gives the same counts, and so does the
    # two-kernel candidate pass (L of two vertices then takes the global-set
    # path instead of the fused pass's attribution); on K_{a,b} every vertex of
    # a side has the same count
    g = gg.chung_lu_bipartite(200, 150, 2000, 2.2, 2.2, 50, 50, seed=72)
    G = bc.build_graph(g)
    for p, q in [(3, 3), (2, 4), (2, 2)]:
        a = bc.bc_count_per_vertex(G, p, q, bc.BC_ANCHOR_U)
        b = bc.bc_count_per_vertex(G, p, q, bc.BC_ANCHOR_U, sets=bc.BC_SETS_SORTED)
        c = bc.bc_count_per_vertex(G, p, q, bc.BC_ANCHOR_U, root_build=bc.BC_ROOT_BUILD_TWO_PASS)
        assert a == b == c
        assert a == oracle.count_per_vertex(g, p, q)[0]
    a_, b_ = 9, 7
    us = [u for u in range(a_) for _ in range(b_)]
    vs = [v for _ in range(a_) for v in range(b_)]
    K = bc.build_graph(gg.graph_from_pairs(a_, b_, us, vs))
    for p, q in [(2, 2), (3, 4), (5, 2)]:
        assert bc.bc_count_per_vertex(K, p, q, bc.BC_ANCHOR_U) == [math.comb(a_ - 1, p - 1) * math.comb(b_, q)] * a_
        assert bc.bc_count_per_vertex(K, p, q, bc.BC_ANCHOR_V) == [math.comb(a_, p) * math.comb(b_ - 1, q - 1)] * b_


def test_per_vertex_on_the_2m_graph_adds_up(bc):
    # at full size, L of two vertices: the per-vertex counts of (2,3) and (2,4)
    # add up to p times the count, and sampled vertices match the oracle's
    # count over the subgraph of their neighbourhood (a vertex x of U is in
    # exactly the (p-1, q)-bicliques of the graph on U - {x} and N(x), each
    # with x added)
    g = gg.power_law_2m()
    G = bc.build_graph(g)
    for p, q in [(2, 3), (2, 4)]:
        total = bc.bc_count(G, p, q)
        cu = bc.bc_count_per_vertex(G, p, q, bc.BC_ANCHOR_U, timeout_ms=60_000)
        assert sum(cu) == p * total
        rng = gg.draws_u64(91, 1, 0, 12)
        for x in sorted({int(r % g.n_u) for r in rng}):
            nx = g.indices_u[int(g.indptr_u[x]):int(g.indptr_u[x + 1])].astype(np.int64)
            if len(nx) < q:
                assert cu[x] == 0
                continue
            # subgraph: U - {x} against N(x), N(x) relabelled 0 .. d(x)-1
            parts = [g.indices_v[int(g.indptr_v[v]):int(g.indptr_v[v + 1])].astype(np.int64) for v in nx]
            us = np.concatenate(parts)
            vs = np.concatenate([np.full(len(a), i, dtype=np.int64) for i, a in enumerate(parts)])
            keep = us != x
            sub = gg.graph_from_pairs(g.n_u, len(nx), us[keep], vs[keep])
            want = oracle.count(sub, p - 1, q) if p > 1 else math.comb(len(nx), q)
            assert cu[x] == want, (p, q, x)
        say("2m per-vertex", (p, q), "total", total)
