"""bc_count_noalloc (all scratch in the library's fixed device buffer) gives
the same exact counts as bc_count, on two calls in a row (the second on a
smaller input), and refuses a count whose scratch does not fit."""
import ctypes
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


def test_noalloc_matches_bc_count(bc):
    big = gg.chung_lu_bipartite(2000, 1000, 16000, 2.2, 2.2, 150, 150, seed=21)
    small = gg.chung_lu_bipartite(200, 160, 7000, 3.0, 3.0, 110, 110, seed=5)
    Gb, Gs = bc.build_graph(big), bc.build_graph(small)
    for (p, q) in [(2, 2), (3, 3), (4, 4), (5, 3), (3, 5), (6, 4)]:
        # the larger input first, then the smaller one: the buffer keeps the
        # first call's contents and the second must not depend on them
        for name, G, g in (("cl2000", Gb, big), ("dense200", Gs, small)):
            want = bc.bc_count(G, p, q)
            got = bc.bc_count_noalloc(G, p, q)
            say("noalloc", name, (p, q), got, want)
            assert got == want, (name, p, q)
        assert want == oracle.count(small, p, q)
    # repeated on the same input, with an explicit stream and forced anchors
    import torch
    s = torch.cuda.Stream()
    for anchor in (bc.BC_ANCHOR_U, bc.BC_ANCHOR_V):
        assert bc.bc_count_noalloc(Gs, 5, 3, stream=s, anchor=anchor) == bc.bc_count(Gs, 5, 3)


def test_noalloc_refuses_what_does_not_fit(bc):
    g = gg.power_law_2m()
    G = bc.build_graph(g)
    lib = bc._lib
    out = bc.bc_u128(0xDEAD, 0xBEEF)
    o = bc.make_opts()
    s = lib.bc_count_noalloc(G.handle, 4, 4, ctypes.byref(o), ctypes.byref(out))
    say("noalloc 2M (4,4):", bc.bc_status_string(s), bc.bc_last_error())
    assert s == bc.BC_E_OOM
    assert "fixed" in bc.bc_last_error()
    assert (out.lo, out.hi) == (0xDEAD, 0xBEEF)
    # what fits on the same graph still counts, and equals bc_count
    assert bc.bc_count_noalloc(G, 1, 3) == bc.bc_count(G, 1, 3)
    small = gg.small_er()
    Gs = bc.build_graph(small)
    assert bc.bc_count_noalloc(Gs, 2, 2) == bc.bc_count(Gs, 2, 2) == oracle.count(small, 2, 2)


def test_noalloc_rejects_an_allocator(bc):
    g = gg.small_er()
    G = bc.build_graph(g)
    al = bc.Allocator(lambda n, st: 0, lambda p, st: None)
    with pytest.raises(bc.BCError) as e:
        bc.bc_count_noalloc(G, 2, 2, allocator=al)
    assert e.value.status == bc.BC_E_INVALID_ARG
