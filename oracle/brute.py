"""Brute force over every (L, R) pair -- test infrastructure only.

Counts (p,q)-bicliques straight from Definition 1 (Section II-A): every
p-subset L of U and every q-subset R of V, kept when all p*q pairs are edges.
Exponential; meant for graphs with at most a dozen vertices per side.
"""
from __future__ import annotations

from itertools import combinations


def adjacency_sets(n_u, indptr_u, indices_u):
    return [set(int(x) for x in indices_u[int(indptr_u[u]):int(indptr_u[u + 1])])
            for u in range(n_u)]


def count_pairs(n_u, n_v, adj, p, q):
    """#{(L, R): |L| = p, |R| = q, L x R within E} by testing every pair of subsets."""
    total = 0
    for L in combinations(range(n_u), p):
        for R in combinations(range(n_v), q):
            if all(v in adj[u] for u in L for v in R):
                total += 1
    return total


def count_graph(g, p, q):
    return count_pairs(g.n_u, g.n_v, adjacency_sets(g.n_u, g.indptr_u, g.indices_u), p, q)


def per_vertex_pairs(n_u, n_v, adj, p, q):
    """For every x in U and v in V, how many (L, R) with |L| = p, |R| = q and
    L x R within E hold x in L (resp. v in R), by testing every pair of subsets."""
    cu, cv = [0] * n_u, [0] * n_v
    for L in combinations(range(n_u), p):
        for R in combinations(range(n_v), q):
            if all(v in adj[u] for u in L for v in R):
                for x in L:
                    cu[x] += 1
                for v in R:
                    cv[v] += 1
    return cu, cv
