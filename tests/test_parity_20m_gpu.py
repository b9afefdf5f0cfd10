"""The power-law 20M-edge graph (|U| = 1M, |V| = 400k, exponent 2.0 on U and
2.4 on V) at full size: closed forms, per-root counts of sampled roots at
(3,3) and (6,6) on both anchors against the oracle (uniform ranks, a band of
mid ranks and the dense top of the order; the oracle abandons roots over its
intersection budget and only the roots it finishes are compared), and
additivity of root ranges."""
import math
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


@pytest.fixture(scope="module")
def g20(bc):
    say("generating power_law_20m")
    g = gg.power_law_20m()
    say("building")
    return g, bc.build_graph(g)


def test_20m_closed_forms(bc, g20):
    g, G = g20
    du, dv = g.degrees_u(), g.degrees_v()
    assert bc.bc_count(G, 1, 1) == g.n_edges == 20_000_000
    assert bc.bc_count(G, 1, 6) == sum(math.comb(int(d), 6) for d in du)
    assert bc.bc_count(G, 6, 1) == sum(math.comb(int(d), 6) for d in dv)
    assert bc.bc_count(G, 2, 1) == sum(math.comb(int(d), 2) for d in dv)


def _sample_ranks(n, seed):
    r = gg.draws_u64(seed, 1, 0, 48)
    return sorted({int(x % n) for x in r[:20]} | {n // 2 + int(x % 1000) for x in r[20:30]} |
                  {n - 1 - int(x % 2000) for x in r[30:40]})


@pytest.mark.parametrize("p,q", [(3, 3), (6, 6)])
def test_20m_per_root_samples(bc, g20, p, q):
    g, G = g20
    nonzero = 0
    for anchor, n in ((bc.BC_ANCHOR_U, g.n_u), (bc.BC_ANCHOR_V, g.n_v)):
        ranks = _sample_ranks(n, 303 + anchor)
        want = oracle.count_ranks(g, p, q, ranks, anchor="U" if anchor == bc.BC_ANCHOR_U else "V",
                                  order_key=oracle.ORDER_DEGREE, max_nodes=5_000_000)
        done = [(r, w) for r, w in zip(ranks, want) if w is not None]
        assert len(done) >= len(ranks) * 2 // 3
        for r, w in done:
            assert bc.bc_count_roots(G, p, q, anchor, r, r + 1) == w, (anchor, (p, q), r)
        nonzero += sum(1 for _, w in done if w)
        say("20m per-root", (p, q), anchor, len(done), "of", len(ranks), "compared,",
            sum(1 for _, w in done if w), "nonzero")
    # (6,6) is zero at most roots the oracle can finish; some must not be
    assert nonzero >= 2


def test_20m_rank_ranges_add_up(bc, g20):
    g, G = g20
    total = bc.bc_count(G, 3, 3, anchor=bc.BC_ANCHOR_U)
    cuts = [0, 400_000, 800_000, 950_000, 990_000, g.n_u]
    parts = [bc.bc_count_roots(G, 3, 3, bc.BC_ANCHOR_U, a, b) for a, b in zip(cuts, cuts[1:])]
    say("20m (3,3) on U", total, parts)
    assert sum(parts) == total
    assert bc.bc_count(G, 3, 3) == total == bc.bc_count(G, 3, 3, anchor=bc.BC_ANCHOR_V)
    # (6,6) over the lowest eighth of the V order, split in two
    h = g.n_v // 8
    a = bc.bc_count_roots(G, 6, 6, bc.BC_ANCHOR_V, 0, h // 2, timeout_ms=60_000)
    b = bc.bc_count_roots(G, 6, 6, bc.BC_ANCHOR_V, h // 2, h, timeout_ms=60_000)
    assert bc.bc_count_roots(G, 6, 6, bc.BC_ANCHOR_V, 0, h, timeout_ms=60_000) == a + b
    say("20m (6,6) on V, lowest eighth", a, b)
