"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against something the paper or plain
mathematics fixes: the paper's worked examples, closed forms, a brute force
straight from Definition 1, a textbook identity computed another way, and
invariants (relabelling, side swap, vertex order, pruning).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import brute
from paper_2403_07858_amd import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _graph_from_adj(n_u, n_v, adj):
    us = [u for u in range(n_u) for _ in adj[u]]
    vs = [v for u in range(n_u) for v in adj[u]]
    return gg.graph_from_pairs(n_u, n_v, us, vs)


def _complete(a, b):
    return _graph_from_adj(a, b, [list(range(b)) for _ in range(a)])


def _crown(n):
    return _graph_from_adj(n, n, [[j for j in range(n) if j != i] for i in range(n)])


def _random_graph(n_u, n_v, density, seed):
    r = gg.draws_unit(seed, 99, 0, n_u * n_v).reshape(n_u, n_v)
    adj = [list(np.nonzero(r[u] < density)[0]) for u in range(n_u)]
    return _graph_from_adj(n_u, n_v, adj)


def _disjoint_union(g1, g2):
    us = np.concatenate([np.repeat(np.arange(g1.n_u), np.diff(g1.indptr_u).astype(np.int64)),
                         g1.n_u + np.repeat(np.arange(g2.n_u), np.diff(g2.indptr_u).astype(np.int64))])
    vs = np.concatenate([g1.indices_u.astype(np.int64), g1.n_v + g2.indices_u.astype(np.int64)])
    return gg.graph_from_pairs(g1.n_u + g2.n_u, g1.n_v + g2.n_v, us, vs)


def _permuted(g, seed):
    pu = gg._random_relabel(g.n_u, seed, 7)
    pv = gg._random_relabel(g.n_v, seed, 8)
    us = np.repeat(np.arange(g.n_u), np.diff(g.indptr_u).astype(np.int64))
    return gg.graph_from_pairs(g.n_u, g.n_v, pu[us], pv[g.indices_u.astype(np.int64)])


# --------------------------------------------------------------------------
# The paper's worked examples.

def test_paper_example_counts(oracle_lib):
    ex = json.load(open(os.path.join(GOLDEN, "paper_example.json")))
    adj = [ex["adjacency_u"][str(u)] for u in range(ex["n_u"])]
    g = _graph_from_adj(ex["n_u"], ex["n_v"], adj)
    # Example 1: shared neighbours of the named pairs
    for a, b, shared in ex["example1_shared_neighbours"]:
        assert sorted(set(adj[a]) & set(adj[b])) == shared
    assert sorted(set(adj[1]) & set(adj[2]) & set(adj[3])) == ex["example1_common_of_u2_u3_u4"]
    # Example 2: exactly two (3,2)-bicliques
    assert oracle_lib.count(g, 3, 2) == ex["example2_count_3_2"]
    assert brute.count_graph(g, 3, 2) == ex["example2_count_3_2"]
    for L, R in ex["example2_bicliques_3_2"]:
        assert all(v in adj[u] for u in L for v in R)


def test_paper_example3_candidate_sets(oracle_lib):
    ex = json.load(open(os.path.join(GOLDEN, "paper_example.json")))
    adj = [ex["adjacency_u"][str(u)] for u in range(ex["n_u"])]
    g = _graph_from_adj(ex["n_u"], ex["n_v"], adj)
    e3 = ex["example3_after_u1_u2"]
    cr, cl = oracle_lib.basic_sets(g.n_u, g.n_v, g.indptr_u, g.indices_u, e3["q"], e3["L"])
    assert cr == e3["C_R"]
    assert cl == e3["C_L"]


def test_htb_examples(oracle_lib):
    ex = json.load(open(os.path.join(GOLDEN, "htb_example.json")))
    a = oracle_lib.htb_encode(ex["list_a"], ex["word_bits"])
    b = oracle_lib.htb_encode(ex["list_b"], ex["word_bits"])
    assert a == (ex["list_a_idx"], ex["list_a_val"])
    assert b == (ex["list_b_idx"], ex["list_b_val"])
    c = oracle_lib.htb_intersect(a, b)
    assert c == (ex["and_idx"], ex["and_val"])
    ids = [i * ex["word_bits"] + j for i, w in zip(*c) for j in range(ex["word_bits"]) if (w >> j) & 1]
    assert ids == ex["and_ids"] == sorted(set(ex["list_a"]) & set(ex["list_b"]))


def test_htb_64bit_words_roundtrip(oracle_lib):
    ids = [0, 1, 63, 64, 65, 127, 128, 1000, 4095]
    idx, val = oracle_lib.htb_encode(ids, 64)
    back = [i * 64 + j for i, w in zip(idx, val) for j in range(64) if (w >> j) & 1]
    assert back == ids


# --------------------------------------------------------------------------
# Binomial table.

@pytest.mark.parametrize("n,k", [(0, 0), (5, 0), (5, 5), (6, 3), (64, 32), (968, 8), (4869, 6),
                                 (5000, 8), (130, 65), (4089, 13)])
def test_binomial_matches_math_comb(oracle_lib, n, k):
    assert oracle_lib.binom(n, k) == math.comb(n, k)


def test_binomial_overflow_is_reported(oracle_lib):
    assert math.comb(200, 100) >= 1 << 128
    with pytest.raises(oracle_lib.OracleError) as e:
        oracle_lib.binom(200, 100)
    assert e.value.code == oracle_lib.E_OVERFLOW


# --------------------------------------------------------------------------
# Closed forms.

@pytest.mark.parametrize("a,b", [(1, 1), (3, 4), (6, 5), (9, 7)])
def test_complete_bipartite(oracle_lib, a, b):
    g = _complete(a, b)
    for p in range(1, a + 1):
        for q in range(1, b + 1):
            assert oracle_lib.count(g, p, q) == math.comb(a, p) * math.comb(b, q), (p, q)


@pytest.mark.parametrize("n", [3, 5, 8])
def test_crown_graph(oracle_lib, n):
    g = _crown(n)
    for p in range(1, n + 1):
        for q in range(1, n + 1):
            assert oracle_lib.count(g, p, q) == math.comb(n, p) * math.comb(n - p, q), (p, q)


def test_single_side_closed_forms(oracle_lib):
    g = gg.small_er()
    du, dv = g.degrees_u(), g.degrees_v()
    assert oracle_lib.count(g, 1, 1) == g.n_edges
    for q in (2, 3, 4):
        assert oracle_lib.count(g, 1, q) == sum(math.comb(int(d), q) for d in du)
    for p in (2, 3, 4):
        assert oracle_lib.count(g, p, 1) == sum(math.comb(int(d), p) for d in dv)


def test_butterflies_by_matrix_product(oracle_lib):
    # (2,2)-bicliques are butterflies: sum over unordered U pairs of C(common, 2),
    # with the common-neighbour counts taken from the product A A^T.
    g = gg.small_er()
    A = np.zeros((g.n_u, g.n_v), dtype=np.int64)
    for u in range(g.n_u):
        A[u, g.indices_u[g.indptr_u[u]:g.indptr_u[u + 1]]] = 1
    C = A @ A.T
    iu = np.triu_indices(g.n_u, 1)
    c = C[iu]
    assert oracle_lib.count(g, 2, 2) == int((c * (c - 1) // 2).sum())
    # and through V: sum over unordered V pairs
    D = A.T @ A
    iv = np.triu_indices(g.n_v, 1)
    d = D[iv]
    assert oracle_lib.count(g, 2, 2) == int((d * (d - 1) // 2).sum())


def test_disjoint_union_adds(oracle_lib):
    g1 = _random_graph(9, 8, 0.5, 1)
    g2 = _random_graph(7, 10, 0.45, 2)
    g = _disjoint_union(g1, g2)
    for p, q in [(2, 2), (2, 3), (3, 2), (3, 3)]:
        assert oracle_lib.count(g, p, q) == oracle_lib.count(g1, p, q) + oracle_lib.count(g2, p, q)


def test_exact_beyond_64_bits(oracle_lib):
    # K_{3,130} at (1, 65): 3 * C(130, 65) > 2^64 but < 2^128.
    g = _complete(3, 130)
    want = 3 * math.comb(130, 65)
    assert (1 << 64) < want < (1 << 128)
    assert oracle_lib.count(g, 1, 65) == want


def test_overflow_of_sum_is_reported(oracle_lib):
    # K_{4,130} at (1, 65): every term fits, the sum 4 * C(130, 65) does not.
    g = _complete(4, 130)
    assert 4 * math.comb(130, 65) >= 1 << 128
    with pytest.raises(oracle_lib.OracleError) as e:
        oracle_lib.count(g, 1, 65)
    assert e.value.code == oracle_lib.E_OVERFLOW


# --------------------------------------------------------------------------
# Brute force on tiny graphs (Definition 1 directly).

@pytest.mark.parametrize("seed", range(6))
def test_brute_force_tiny(oracle_lib, seed):
    n_u = 5 + seed % 4
    n_v = 6 + (seed * 3) % 5
    g = _random_graph(n_u, n_v, 0.35 + 0.08 * (seed % 4), 100 + seed)
    adj = brute.adjacency_sets(g.n_u, g.indptr_u, g.indices_u)
    for p in range(1, 5):
        for q in range(1, 5):
            want = brute.count_pairs(g.n_u, g.n_v, adj, p, q)
            assert oracle_lib.count(g, p, q) == want, (p, q)
            assert oracle_lib.count(g, p, q, prune=False) == want, (p, q)


def test_empty_and_degenerate_graphs(oracle_lib):
    g = gg.graph_from_pairs(3, 4, [], [])
    for p, q in [(1, 1), (2, 2), (3, 3)]:
        assert oracle_lib.count(g, p, q) == 0
    g = _complete(2, 3)
    assert oracle_lib.count(g, 3, 1) == 0     # p > |U|
    assert oracle_lib.count(g, 1, 4) == 0     # q > |V|
    assert oracle_lib.count(g, 2, 3) == 1


# --------------------------------------------------------------------------
# Invariants.

def test_side_swap(oracle_lib):
    g = _random_graph(12, 11, 0.45, 7)
    for p, q in [(2, 3), (3, 2), (3, 4), (4, 3), (2, 5)]:
        assert oracle_lib.count(g, p, q) == oracle_lib.count(g, p, q, anchor="V")
        assert oracle_lib.count(g, p, q) == oracle_lib.count(g.transposed(), q, p)


def test_relabel_invariance(oracle_lib):
    g = _random_graph(14, 12, 0.4, 11)
    h = _permuted(g, 5)
    for p, q in [(2, 2), (3, 3), (2, 4), (4, 2)]:
        assert oracle_lib.count(g, p, q) == oracle_lib.count(h, p, q)


@pytest.mark.parametrize("key", [0, 1, 2])
def test_order_and_prune_invariance(oracle_lib, key):
    g = gg.small_er()
    base = {pq: oracle_lib.count(g, *pq, order_key=0) for pq in gg.SMALL_ER_QUERIES}
    for pq, want in base.items():
        assert oracle_lib.count(g, *pq, order_key=key) == want
    t = _random_graph(10, 9, 0.5, 3)
    for p, q in [(3, 2), (2, 3), (4, 2)]:
        assert oracle_lib.count(t, p, q, order_key=key, prune=True) == \
            oracle_lib.count(t, p, q, order_key=0, prune=False)


def test_rank_ranges_add_up(oracle_lib):
    g = gg.small_er()
    for p, q in [(2, 2), (3, 2)]:
        total = oracle_lib.count(g, p, q, order_key=1)
        parts = sum(oracle_lib.count(g, p, q, order_key=1, rank_lo=lo, rank_hi=lo + 300)
                    for lo in range(0, g.n_u, 300))
        assert parts == total
        per = oracle_lib.count_ranks(g, p, q, list(range(g.n_u)), order_key=1)
        assert sum(per) == total


def test_degree_order_rule(oracle_lib):
    g = _random_graph(30, 20, 0.3, 4)
    by_rank = oracle_lib.order(g.n_u, g.n_v, g.indptr_u, g.indices_u, 1)
    deg = g.degrees_u()
    keys = [(int(deg[u]), int(u)) for u in by_rank]
    assert keys == sorted(keys)


def test_two_hop_order_rule(oracle_lib):
    g = _random_graph(16, 12, 0.35, 9)
    q = 2
    adj = brute.adjacency_sets(g.n_u, g.indptr_u, g.indices_u)
    size = [sum(1 for w in range(g.n_u) if w != u and len(adj[u] & adj[w]) >= q) for u in range(g.n_u)]
    by_rank = oracle_lib.order(g.n_u, g.n_v, g.indptr_u, g.indices_u, 2, q)
    keys = [(size[u], int(u)) for u in by_rank]
    assert keys == sorted(keys)


def test_invalid_csr_rejected(oracle_lib):
    # duplicate neighbour
    with pytest.raises(oracle_lib.OracleError) as e:
        oracle_lib.count_csr(2, 3, np.array([0, 2, 3], dtype=np.uint64),
                             np.array([1, 1, 0], dtype=np.uint32), 1, 1)
    assert e.value.code == oracle_lib.E_CSR
    # id out of range
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.count_csr(1, 2, np.array([0, 1], dtype=np.uint64), np.array([5], dtype=np.uint32), 1, 1)


def _per_root_brute(adj, n_u, p, q, key):
    """Definition 1 split by root: every p-subset L adds C(|common N(L)|, q) to
    the member of L that comes first in the order of `key` (vertex -> sort
    key), i.e. the root that enumerates L."""
    first = {u: 0 for u in range(n_u)}
    for L in itertools.combinations(range(n_u), p):
        common = set.intersection(*(adj[x] for x in L))
        first[min(L, key=key)] += math.comb(len(common), q)
    return first


@pytest.mark.parametrize("seed", range(3))
def test_per_root_values_by_brute_force(oracle_lib, seed):
    # count_ranks entry r is the count of the root ranked r (pins the
    # rank <-> vertex mapping, not only the sum)
    g = _random_graph(11, 9, 0.5, 40 + seed)
    adj_u = brute.adjacency_sets(g.n_u, g.indptr_u, g.indices_u)
    adj_v = brute.adjacency_sets(g.n_v, g.indptr_v, g.indices_v)
    for anchor, adj, n in (("U", adj_u, g.n_u), ("V", adj_v, g.n_v)):
        deg = [len(a) for a in adj]
        by_degree = sorted(range(n), key=lambda x: (deg[x], x))
        for p, q in [(2, 2), (3, 2), (2, 3), (3, 3)]:
            pa, qa = (p, q) if anchor == "U" else (q, p)
            want = _per_root_brute(adj, n, pa, qa, key=lambda x: (deg[x], x))
            got = oracle_lib.count_ranks(g, p, q, list(range(n)), anchor=anchor, order_key=oracle_lib.ORDER_DEGREE)
            assert got == [want[by_degree[r]] for r in range(n)], (anchor, p, q)
            assert len(set(got)) > 1   # the values differ, so a permutation would show
        # the two-hop order with threshold q (Definition 2's key, ties by id)
        qa = 2
        size = [sum(1 for w in range(n) if w != x and len(adj[x] & adj[w]) >= qa) for x in range(n)]
        by_two_hop = sorted(range(n), key=lambda x: (size[x], x))
        pa = 3
        p, q = (pa, qa) if anchor == "U" else (qa, pa)
        want = _per_root_brute(adj, n, pa, qa, key=lambda x: (size[x], x))
        got = oracle_lib.count_ranks(g, p, q, list(range(n)), anchor=anchor, order_key=oracle_lib.ORDER_TWO_HOP)
        assert got == [want[by_two_hop[r]] for r in range(n)], (anchor, "two-hop")


# --------------------------------------------------------------------------
# Per-vertex counts (the output set of Algorithm 1 as membership counts).

@pytest.mark.parametrize("seed", range(4))
def test_per_vertex_by_brute_force(oracle_lib, seed):
    g = _random_graph(6 + seed % 3, 7, 0.45 + 0.05 * seed, 300 + seed)
    adj = brute.adjacency_sets(g.n_u, g.indptr_u, g.indices_u)
    for p in range(1, 4):
        for q in range(1, 4):
            want_u, want_v = brute.per_vertex_pairs(g.n_u, g.n_v, adj, p, q)
            got_u, got_v = oracle_lib.count_per_vertex(g, p, q)
            assert (got_u, got_v) == (want_u, want_v), (p, q)


@pytest.mark.parametrize("a,b", [(3, 4), (5, 2), (6, 6)])
def test_per_vertex_complete_bipartite(oracle_lib, a, b):
    # in K_{a,b} every vertex of a side is alike: x in U is in C(a-1, p-1) C(b, q)
    # bicliques, v in V in C(a, p) C(b-1, q-1)
    g = _complete(a, b)
    for p, q in [(1, 1), (2, 2), (2, 3), (3, 2)]:
        cu, cv = oracle_lib.count_per_vertex(g, p, q)
        assert cu == [math.comb(a - 1, p - 1) * math.comb(b, q)] * a
        assert cv == [math.comb(a, p) * math.comb(b - 1, q - 1)] * b


def test_per_vertex_sums_and_side_swap(oracle_lib):
    # every biclique has p members in L and q in R; swapping the sides swaps the lists
    g = gg.small_er()
    gt = gg.graph_from_pairs(g.n_v, g.n_u, g.indices_u.astype(np.int64),
                             np.repeat(np.arange(g.n_u), np.diff(g.indptr_u).astype(np.int64)))
    for p, q in [(2, 2), (3, 2), (2, 4)]:
        cu, cv = oracle_lib.count_per_vertex(g, p, q)
        total = oracle_lib.count(g, p, q)
        assert sum(cu) == p * total and sum(cv) == q * total
        tu, tv = oracle_lib.count_per_vertex(gt, q, p)
        assert (tu, tv) == (cv, cu)
