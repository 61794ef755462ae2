"""Seeded synthetic inputs: graphs and initial placements.

This module holds none of the layout method's arithmetic.  It draws graphs
and starting placements from explicit seeds so that the HIP path and the
oracle can be handed identical inputs.  The paper's benchmark graphs are not
available; these families stand in for them at the sizes the paper motivates
(Sec. 5.1 draws starting placements uniformly on the unit square):

* ``grid_graph``        2-D lattice (the paper's "grid-*" family)
* ``erdos_renyi``       G(n, M), M distinct pairs drawn uniformly
* ``barabasi_albert``   preferential attachment, endpoint-list method of
                        Batagelj and Brandes (Phys. Rev. E 71, 036113, 2005)
* ``random_tree``       uniform labelled tree from a random Pruefer sequence
* ``uniform_positions`` i.i.d. uniform coordinates, rounded to float32 values

Graphs are returned as symmetric CSR: ``row_ptr`` int64 (n+1), ``col_idx``
int32 (2|E|), neighbours sorted, no self loops, no duplicates.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    edge_len: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def num_edges(self) -> int:
        return self.nnz // 2

    def edges(self) -> np.ndarray:
        """Undirected edge list (i < j), shape (|E|, 2)."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        keep = src < self.col_idx
        return np.stack([src[keep], self.col_idx[keep].astype(np.int64)], axis=1)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def to_csr(n: int, edges, lengths=None, name: str = "") -> Graph:
    """Symmetric CSR from an undirected edge list; drops self loops and duplicates."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    ln = None if lengths is None else np.asarray(lengths, dtype=np.float64).reshape(-1)
    if len(e):
        if e.min() < 0 or e.max() >= n:
            raise ValueError("edge endpoint out of range")
        keep = e[:, 0] != e[:, 1]
        e = e[keep]
        if ln is not None:
            ln = ln[keep]
        a, b = np.minimum(e[:, 0], e[:, 1]), np.maximum(e[:, 0], e[:, 1])
        key = a * n + b
        key, first = np.unique(key, return_index=True)
        a, b = key // n, key % n
        if ln is not None:
            ln = ln[first]
    else:
        a = b = np.zeros(0, dtype=np.int64)
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    lsym = None if ln is None else np.concatenate([ln, ln])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    col_idx = dst.astype(np.int32)
    el = None if lsym is None else np.ascontiguousarray(lsym[order], dtype=np.float32)
    return Graph(n=n, row_ptr=row_ptr, col_idx=col_idx, edge_len=el, name=name)


def grid_graph(rows: int, cols: int) -> Graph:
    """rows x cols lattice; vertex id = r*cols + c; edges to the right and below."""
    ids = np.arange(rows * cols).reshape(rows, cols)
    right = np.stack([ids[:, :-1].ravel(), ids[:, 1:].ravel()], axis=1)
    down = np.stack([ids[:-1, :].ravel(), ids[1:, :].ravel()], axis=1)
    return to_csr(rows * cols, np.concatenate([right, down]), name="grid-%dx%d" % (rows, cols))


def path_graph(n: int) -> Graph:
    return to_csr(n, np.stack([np.arange(n - 1), np.arange(1, n)], axis=1), name="path-%d" % n)


def cycle_graph(n: int) -> Graph:
    return to_csr(n, np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1), name="cycle-%d" % n)


def complete_graph(n: int) -> Graph:
    iu = np.triu_indices(n, 1)
    return to_csr(n, np.stack(iu, axis=1), name="complete-%d" % n)


def erdos_renyi(n: int, m: int, seed: int) -> Graph:
    """G(n, M): m distinct unordered pairs drawn uniformly; isolated vertices kept."""
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges")
    rng = rng_for(seed)
    chosen = {}
    while len(chosen) < m:
        k = max(2 * (m - len(chosen)), 64)
        a = rng.integers(0, n, size=k)
        b = rng.integers(0, n, size=k)
        for x, y in zip(a.tolist(), b.tolist()):
            if x == y:
                continue
            key = (x, y) if x < y else (y, x)
            if key not in chosen:
                chosen[key] = None
                if len(chosen) == m:
                    break
    return to_csr(n, np.array(list(chosen.keys()), dtype=np.int64), name="er-%d-%d" % (n, m))


def barabasi_albert(n: int, m: int, seed: int) -> Graph:
    """Preferential attachment: a complete seed graph on m+1 vertices, then every
    new vertex links to m distinct earlier vertices chosen with probability
    proportional to degree (uniform picks from the list of edge endpoints)."""
    if n <= m:
        raise ValueError("need n > m")
    rng = rng_for(seed)
    m0 = m + 1
    iu = np.triu_indices(m0, 1)
    seed_edges = np.stack(iu, axis=1)
    total = len(seed_edges) + (n - m0) * m
    ends = np.empty(2 * total, dtype=np.int64)
    ends[: 2 * len(seed_edges)] = seed_edges.ravel()
    fill = 2 * len(seed_edges)
    edges = np.empty((total, 2), dtype=np.int64)
    edges[: len(seed_edges)] = seed_edges
    ne = len(seed_edges)
    for v in range(m0, n):
        targets = []
        while len(targets) < m:
            t = int(ends[rng.integers(0, fill)])
            if t not in targets:
                targets.append(t)
        for t in targets:
            edges[ne] = (v, t)
            ne += 1
            ends[fill] = v
            ends[fill + 1] = t
            fill += 2
    return to_csr(n, edges, name="ba-%d-%d" % (n, m))


def random_tree(n: int, seed: int) -> Graph:
    """Uniform random labelled tree on n vertices (Pruefer sequence decoding)."""
    if n <= 1:
        return to_csr(max(n, 0), np.zeros((0, 2), dtype=np.int64), name="tree-%d" % n)
    if n == 2:
        return to_csr(2, [[0, 1]], name="tree-2")
    rng = rng_for(seed)
    seq = rng.integers(0, n, size=n - 2).tolist()
    degree = [1] * n
    for x in seq:
        degree[x] += 1
    leaves = [i for i in range(n) if degree[i] == 1]
    heapq.heapify(leaves)
    edges = []
    for x in seq:
        leaf = heapq.heappop(leaves)
        edges.append((leaf, x))
        degree[x] -= 1
        if degree[x] == 1:
            heapq.heappush(leaves, x)
    a, b = heapq.heappop(leaves), heapq.heappop(leaves)
    edges.append((a, b))
    return to_csr(n, edges, name="tree-%d" % n)


def uniform_positions(n: int, dim: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n x dim i.i.d. uniform coordinates on [lo, hi), drawn in double and
    rounded to float32 so both precisions see exactly the same values."""
    rng = rng_for(seed)
    x = lo + (hi - lo) * rng.random((n, dim))
    return x.astype(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# The workloads (graph family, size, start box, relaxation factors, stopping)
# --------------------------------------------------------------------------
def workload_seed(config: int, run: int = 0) -> int:
    return 1000 * config + run


def grid16(run: int = 0):
    """16 x 16 grid (n=256, 480 edges), start uniform on [0,1]^2."""
    g = grid_graph(16, 16)
    return g, uniform_positions(g.n, 2, workload_seed(1, run))


def er4096(run: int = 0):
    """G(n=4096, M=12288) (mean degree 6), start uniform on [0, 64]^2."""
    s = workload_seed(2, run)
    g = erdos_renyi(4096, 12288, s)
    return g, uniform_positions(g.n, 2, s + 500, 0.0, 64.0)


def ba65536(dim: int = 2, run: int = 0, n: int = 65536):
    """Barabasi-Albert n=65536, m=3 (196,602 edges), start uniform on [0,1]^dim."""
    s = workload_seed(3, run)
    g = barabasi_albert(n, 3, s)
    return g, uniform_positions(g.n, dim, s + 500 + dim)


def near_square_grid(n: int) -> Graph:
    """The rows x cols lattice with rows = floor(sqrt(n)), cols = n // rows."""
    rows = max(1, int(np.floor(np.sqrt(n))))
    return grid_graph(rows, max(1, n // rows))


def largest_component(g: Graph) -> Graph:
    """The largest connected component of g, vertices renumbered in order."""
    label = -np.ones(g.n, dtype=np.int64)
    best, best_size = -1, 0
    for s in range(g.n):
        if label[s] >= 0:
            continue
        stack, label[s], size = [s], s, 0
        while stack:
            u = stack.pop()
            size += 1
            for v in g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]:
                if label[v] < 0:
                    label[v] = s
                    stack.append(int(v))
        if size > best_size:
            best, best_size = s, size
    keep = np.flatnonzero(label == best)
    new_id = -np.ones(g.n, dtype=np.int64)
    new_id[keep] = np.arange(len(keep))
    e = g.edges()
    e = e[(new_id[e[:, 0]] >= 0) & (new_id[e[:, 1]] >= 0)]
    return to_csr(len(keep), new_id[e], name=g.name + "-lcc")


def batch_of_graphs(count: int = 2048, n_lo: int = 16, n_hi: int = 1024, seed: int = 4000, dim: int = 2):
    """Many small graphs: n uniform in [n_lo, n_hi], family cycling through
    near-square grids, uniform random trees and the largest component of
    G(n, 2n) (mean degree 4), each with its own start uniform on [0,1]^dim.
    Returns (graphs, X0 list).  (A two-vertex component would make the
    one-sweep Jacobi step oscillate, r -> 2d - r, for ever.)"""
    rng = rng_for(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    fam = rng.integers(0, 3, size=count)
    graphs, starts = [], []
    for k in range(count):
        n = int(ns[k])
        s = seed * 10 + k
        if fam[k] == 0:
            g = near_square_grid(n)
        elif fam[k] == 1:
            g = random_tree(n, s)
        else:
            g = largest_component(erdos_renyi(n, min(2 * n, n * (n - 1) // 2), s))
        graphs.append(g)
        starts.append(uniform_positions(g.n, dim, s + 7))
    return graphs, starts
