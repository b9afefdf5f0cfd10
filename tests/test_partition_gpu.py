"""BCPar (Algorithm 3): groups of roots whose closures fit a budget; each
group counted on its closure subgraph alone; the groups' counts add up to
the whole count (oracle), for several budgets and both anchors."""
import sys

import pytest

import oracle
from paper_2403_07858_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bc():
    from paper_2403_07858_amd import bc as m
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_partition_counts_add_up(bc):
    g = gg.chung_lu_bipartite(2000, 1000, 16000, 2.2, 2.2, 150, 150, seed=21)
    G = bc.build_graph(g)
    for (p, q, anchor) in ((3, 3, bc.BC_ANCHOR_U), (4, 3, bc.BC_ANCHOR_U), (3, 4, bc.BC_ANCHOR_V)):
        want = oracle.count(g, p, q, anchor="U" if p <= q else "V")
        for budget in (1 << 16, 1 << 19, 1 << 40):
            part, n = bc.bc_partition(G, p, q, anchor, budget)
            assert n >= 1 and int(part.max()) == n - 1
            total, sizes = 0, []
            for k in range(n):
                c, edges = bc.bc_count_partition(G, p, q, anchor, part, k)
                total += c
                sizes.append(edges)
            say("bcpar", (p, q), anchor, "budget", budget, "groups", n, "largest closure", max(sizes), "edges")
            assert total == want, ((p, q), anchor, budget)
            if budget == 1 << 40:
                assert n == 1


def test_partition_on_hubs(bc):
    # few groups under a budget that cuts the hub-heavy graph several ways
    g = gg.chung_lu_bipartite(20000, 1500, 200000, 2.5, 1.5, 200, 6000, 5)
    G = bc.build_graph(g)
    want = bc.bc_count(G, 2, 3, anchor=bc.BC_ANCHOR_V)   # (2,3) with L on V: depth 3
    assert want == oracle.count(g, 2, 3, anchor="U")   # same count; the shallow side for the oracle
    part, n = bc.bc_partition(G, 2, 3, bc.BC_ANCHOR_V, 1 << 18)
    total = sum(bc.bc_count_partition(G, 2, 3, bc.BC_ANCHOR_V, part, k)[0] for k in range(n))
    say("hubs bcpar groups", n)
    assert n > 1 and total == want
