"""Seeded synthetic bipartite graphs (Erdos-Renyi and Chung-Lu) in CSR form.

This module only draws inputs: it holds none of the counting arithmetic, so
both the device path and the CPU oracle can be fed from it.  Every random
number comes from one counter-based generator, SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): draw
``i`` of stream ``s`` under seed ``k`` is ``mix64(key(k, s) + (i + 1) * GAMMA)``.
Results therefore depend only on (seed, stream, index), never on numpy's own
generators or on batch sizes.

Graph recipes (the paper's datasets are real KONECT graphs and are not used;
these stand in for their regime: power-law degrees, average degrees 2..1400):

* ``er_bipartite(nU, nV, m, seed)``: m distinct (u, v) pairs drawn uniformly
  without replacement from U x V.
* ``chung_lu_bipartite(nU, nV, m, beta_u, beta_v, dmax_u, dmax_v, seed)``:
  vertex i of side X gets weight ``(i + i0_X) ** (-1 / (beta_X - 1))``, with
  ``i0_X`` found by bisection so that the heaviest vertex expects ``dmax_X``
  edges (``m * w_X[0] / sum(w_X) == dmax_X``).  Endpoints are drawn
  independently from the two weight distributions, duplicate pairs are
  rejected, and drawing stops at exactly m distinct edges.

Both recipes permute the vertex ids of each side at random before output, so
ids carry no degree information.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = z.copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _mix64_int(x: int) -> int:
    x &= _MASK64
    x ^= x >> 30
    x = (x * 0xBF58476D1CE4E5B9) & _MASK64
    x ^= x >> 27
    x = (x * 0x94D049BB133111EB) & _MASK64
    x ^= x >> 31
    return x


def stream_key(seed: int, stream: int) -> int:
    """Key of draw stream ``stream`` under ``seed``."""
    return _mix64_int(_mix64_int(seed * 0x9E3779B97F4A7C15 + 0x632BE59BD9B4E019) ^ (stream & _MASK64))


def draws_u64(seed: int, stream: int, start: int, n: int) -> np.ndarray:
    """Draws ``start .. start+n-1`` of one stream as uint64."""
    key = np.uint64(stream_key(seed, stream))
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = key + idx * _GAMMA
    return _mix64(z)


def draws_unit(seed: int, stream: int, start: int, n: int) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits each."""
    return (draws_u64(seed, stream, start, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# Stream ids: one per purpose, so that changing one step never shifts another.
_S_ER_PAIRS, _S_CL_U, _S_CL_V, _S_PERM_U, _S_PERM_V, _S_PARAMS = 1, 2, 3, 4, 5, 6


@dataclass
class BipartiteGraph:
    """A bipartite graph as two CSR matrices, one per side.

    ``indptr_u`` (uint64, n_u + 1) / ``indices_u`` (uint32, nnz) hold N(u) for
    every u in U as sorted V ids; ``indptr_v`` / ``indices_v`` hold N(v) as
    sorted U ids.  The two are transposes of each other.
    """

    n_u: int
    n_v: int
    indptr_u: np.ndarray
    indices_u: np.ndarray
    indptr_v: np.ndarray
    indices_v: np.ndarray
    manifest: dict = field(default_factory=dict)

    @property
    def n_edges(self) -> int:
        return int(self.indices_u.shape[0])

    def transposed(self) -> "BipartiteGraph":
        """The same graph with the roles of U and V exchanged."""
        man = dict(self.manifest)
        man["transposed"] = not man.get("transposed", False)
        return BipartiteGraph(self.n_v, self.n_u, self.indptr_v, self.indices_v,
                              self.indptr_u, self.indices_u, man)

    def degrees_u(self) -> np.ndarray:
        return np.diff(self.indptr_u).astype(np.int64)

    def degrees_v(self) -> np.ndarray:
        return np.diff(self.indptr_v).astype(np.int64)


def csr_from_pairs(n_rows: int, rows: np.ndarray, cols: np.ndarray):
    """CSR (indptr uint64, indices uint32) with every row sorted ascending."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    counts = np.bincount(rows, minlength=n_rows).astype(np.uint64)
    indptr = np.zeros(n_rows + 1, dtype=np.uint64)
    np.cumsum(counts, out=indptr[1:])
    return indptr, cols[order].astype(np.uint32)


def graph_from_pairs(n_u: int, n_v: int, us, vs, manifest: dict | None = None) -> BipartiteGraph:
    """Build both CSR sides from an edge list (duplicates are the caller's problem)."""
    us = np.asarray(us, dtype=np.int64)
    vs = np.asarray(vs, dtype=np.int64)
    ip_u, ix_u = csr_from_pairs(n_u, us, vs)
    ip_v, ix_v = csr_from_pairs(n_v, vs, us)
    g = BipartiteGraph(n_u, n_v, ip_u, ix_u, ip_v, ix_v, dict(manifest or {}))
    _fill_manifest(g)
    return g


def _fill_manifest(g: BipartiteGraph) -> None:
    du, dv = g.degrees_u(), g.degrees_v()
    h = hashlib.sha256()
    for a in (g.indptr_u, g.indices_u):
        h.update(np.ascontiguousarray(a).tobytes())
    g.manifest.update({
        "n_u": g.n_u, "n_v": g.n_v, "edges": g.n_edges,
        "max_deg_u": int(du.max()) if du.size else 0,
        "max_deg_v": int(dv.max()) if dv.size else 0,
        "wedges_via_v": int((dv * (dv - 1) // 2).sum()),
        "wedges_via_u": int((du * (du - 1) // 2).sum()),
        "sha256": h.hexdigest(),
    })


def _random_relabel(n: int, seed: int, stream: int) -> np.ndarray:
    """new_id[old_id]: a uniformly random permutation of 0..n-1."""
    keys = draws_u64(seed, stream, 0, n)
    order = np.argsort(keys, kind="stable")
    new_id = np.empty(n, dtype=np.int64)
    new_id[order] = np.arange(n, dtype=np.int64)
    return new_id


def _distinct_keys(m: int, draw_batch) -> np.ndarray:
    """First m distinct keys of the stream produced by ``draw_batch(start, n)``."""
    acc = np.zeros(0, dtype=np.int64)
    start = 0
    while acc.shape[0] < m:
        need = m - acc.shape[0]
        n = int(need * 1.25) + 1024
        keys = draw_batch(start, n)
        start += n
        allk = np.concatenate([acc, keys])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        acc = allk[first]
        if start > 400 * (m + 1024):
            raise RuntimeError("edge sampler made no progress; the recipe asks for too dense a graph")
    return acc[:m]


def er_bipartite(n_u: int, n_v: int, m: int, seed: int) -> BipartiteGraph:
    """Uniform random bipartite graph with exactly m distinct edges."""
    total = n_u * n_v
    if m > total:
        raise ValueError("more edges than vertex pairs")

    def batch(start, n):
        x = draws_u64(seed, _S_ER_PAIRS, start, n)
        # Lemire-free plain reduction: 64 random bits mod total (bias < total / 2^64).
        return (x % np.uint64(total)).astype(np.int64)

    keys = _distinct_keys(m, batch)
    us, vs = keys // n_v, keys % n_v
    pu = _random_relabel(n_u, seed, _S_PERM_U)
    pv = _random_relabel(n_v, seed, _S_PERM_V)
    man = {"recipe": "er", "params": {"n_u": n_u, "n_v": n_v, "m": m}, "seed": seed}
    return graph_from_pairs(n_u, n_v, pu[us], pv[vs], man)


def chung_lu_weights(n: int, m: int, beta: float, dmax: float) -> np.ndarray:
    """Power-law weights (i + i0)^(-1/(beta-1)) with the top vertex expecting dmax edges."""
    alpha = 1.0 / (beta - 1.0)
    idx = np.arange(n, dtype=np.float64)
    mean = m / n
    if dmax <= mean * 1.0001:
        return np.ones(n, dtype=np.float64)

    def top_share(i0):
        w = (idx + i0) ** (-alpha)
        return m * w[0] / w.sum()

    lo, hi = math.log(1e-9), math.log(1e12)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if top_share(math.exp(mid)) > dmax:
            lo = mid
        else:
            hi = mid
    return (idx + math.exp(0.5 * (lo + hi))) ** (-alpha)


def _sample_index(cdf: np.ndarray, r: np.ndarray) -> np.ndarray:
    i = np.searchsorted(cdf, r, side="right")
    return np.minimum(i, cdf.shape[0] - 1).astype(np.int64)


def chung_lu_bipartite(n_u: int, n_v: int, m: int, beta_u: float, beta_v: float,
                       dmax_u: float, dmax_v: float, seed: int) -> BipartiteGraph:
    """Bipartite Chung-Lu graph with exactly m distinct edges."""
    if m > n_u * n_v:
        raise ValueError("more edges than vertex pairs")
    wu = chung_lu_weights(n_u, m, beta_u, min(dmax_u, n_v))
    wv = chung_lu_weights(n_v, m, beta_v, min(dmax_v, n_u))
    cu = np.cumsum(wu)
    cu /= cu[-1]
    cv = np.cumsum(wv)
    cv /= cv[-1]

    def batch(start, n):
        u = _sample_index(cu, draws_unit(seed, _S_CL_U, start, n))
        v = _sample_index(cv, draws_unit(seed, _S_CL_V, start, n))
        return u * n_v + v

    keys = _distinct_keys(m, batch)
    us, vs = keys // n_v, keys % n_v
    pu = _random_relabel(n_u, seed, _S_PERM_U)
    pv = _random_relabel(n_v, seed, _S_PERM_V)
    man = {"recipe": "chung_lu",
           "params": {"n_u": n_u, "n_v": n_v, "m": m, "beta_u": beta_u, "beta_v": beta_v,
                      "dmax_u": dmax_u, "dmax_v": dmax_v},
           "seed": seed}
    return graph_from_pairs(n_u, n_v, pu[us], pv[vs], man)


# ---------------------------------------------------------------------------
# The named workloads.

def small_er() -> BipartiteGraph:
    """Erdos-Renyi 2000 x 1000 with 20000 edges, seed 0: counted at (3,3)."""
    return er_bipartite(2000, 1000, 20000, seed=0)


SMALL_ER_QUERIES = [(3, 3), (2, 2), (2, 3), (3, 2)]


def power_law_2m() -> BipartiteGraph:
    """Chung-Lu 100k x 50k with 2M edges, exponent 2.1 both sides, max degree 5000."""
    return chung_lu_bipartite(100_000, 50_000, 2_000_000, 2.1, 2.1, 5000, 5000, seed=2)


POWER_LAW_2M_QUERIES = [(4, 4), (5, 5), (6, 6), (7, 7), (8, 8), (4, 6), (6, 4)]


def power_law_20m() -> BipartiteGraph:
    """Chung-Lu 1M x 400k with 20M edges, exponents 2.0 (U) and 2.4 (V), max degree 5000."""
    return chung_lu_bipartite(1_000_000, 400_000, 20_000_000, 2.0, 2.4, 5000, 5000, seed=3)


def batch_spec(i: int) -> dict:
    """Parameters of graph i of the 4096-graph batched workload (seed 4000 + i)."""
    seed = 4000 + i
    r = draws_unit(seed, _S_PARAMS, 0, 4)
    n_u = int(round(math.exp(math.log(50) + r[0] * (math.log(5000) - math.log(50)))))
    n_v = n_u // 2
    dbar = 8.0 + 32.0 * r[1]
    m = min(int(round(dbar * n_u)), (n_u * n_v) // 2)
    p = 2 + int(r[2] * 5)
    q = 2 + int(r[3] * 5)
    return {"seed": seed, "n_u": n_u, "n_v": n_v, "m": m, "p": p, "q": q,
            "beta": 2.2, "dmax": min(n_v, n_u, 5000)}


def batch_graph(i: int) -> tuple[BipartiteGraph, int, int]:
    s = batch_spec(i)
    g = chung_lu_bipartite(s["n_u"], s["n_v"], s["m"], s["beta"], s["beta"],
                           s["dmax"], s["dmax"], seed=s["seed"])
    return g, s["p"], s["q"]


def served_spec(g: int) -> dict:
    """Parameters of resident graph g of the serving workload (seed 5000 + g)."""
    seed = 5000 + g
    r = draws_unit(seed, _S_PARAMS, 0, 2)
    n_u = int(round(math.exp(math.log(10_000) + r[0] * (math.log(300_000) - math.log(10_000)))))
    n_v = n_u // 2
    m = int(round(math.exp(math.log(100_000) + r[1] * (math.log(5_000_000) - math.log(100_000)))))
    m = max(min(m, 200 * n_u), 2 * n_u)
    return {"seed": seed, "n_u": n_u, "n_v": n_v, "m": m, "beta": 2.2, "dmax": 5000}


def served_graph(g: int) -> BipartiteGraph:
    s = served_spec(g)
    return chung_lu_bipartite(s["n_u"], s["n_v"], s["m"], s["beta"], s["beta"],
                              s["dmax"], s["dmax"], seed=s["seed"])


def poisson_arrivals(rate: float, n: int, n_graphs: int, pq_lo: int, pq_hi: int, seed: int):
    """Query stream: (arrival_seconds, graph_id, p, q) for n Poisson arrivals."""
    r = draws_unit(seed, _S_PARAMS, 0, 4 * n).reshape(n, 4)
    gaps = -np.log1p(-r[:, 0]) / rate
    t = np.cumsum(gaps)
    gid = np.minimum((r[:, 1] * n_graphs).astype(np.int64), n_graphs - 1)
    span = pq_hi - pq_lo + 1
    p = pq_lo + np.minimum((r[:, 2] * span).astype(np.int64), span - 1)
    q = pq_lo + np.minimum((r[:, 3] * span).astype(np.int64), span - 1)
    return t, gid, p, q
