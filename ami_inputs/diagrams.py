"""Seeded self-energy topologies and their integer labels.

A diagram is handed to both construction paths as the integer matrices of
Sec. 2.2 (Eq. (2) and the line after it): row ``j`` of ``alpha`` holds the
coefficients of the internal frequencies (and momenta) ``nu_1 .. nu_n`` followed
by the external one (external slot last, Sec. 5.1.1), and row ``j`` of ``eps``
holds the coefficients of the energy placeholders ``E_i = -eps(k_i)``; for
every diagram built here ``eps`` is the identity, which Sec. 5.1.1 calls the
usual starting point.

Random topologies follow the graph representation of Sec. 2.5: ``2n`` vertices,
``n`` bosonic (interaction) lines pairing vertices ``(2i, 2i+1)`` -- a local
Hubbard ``U`` -- and fermionic lines given by a permutation of the vertices.
One fermionic line is cut to make the two external legs of a self-energy,
leaving ``2n - 1`` propagators.  Momentum/frequency conservation is solved with
a spanning tree that contains every bosonic line, so the ``n`` loop variables
sit on fermionic lines (they are fermionic Matsubara frequencies) and each
propagator label is a signed sum of loop variables plus the external one.

Topologies with a loop carried by a single propagator are rejected: that sum
only converges with a convergence factor, and its value depends on it.

No residue or evaluation arithmetic lives here: a candidate that the
construction rejects (a coefficient of magnitude two after a substitution, a
pole of higher order) is skipped by whoever consumes it.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np


@dataclass
class Diagram:
    """Integer labels of one starting integrand ``R0`` (Sec. 2.2, Sec. 5.1.1).

    ``alpha``     int8 [nG, nF]: frequency/momentum coefficients; the first
                  ``n_int`` columns are the summed frequencies, the rest external.
    ``eps``       int8 [nG, nE]: energy coefficients (identity here).
    ``n_int``     number of nested Matsubara sums.
    ``fermionic`` uint8 [nF]: 1 where the frequency in that slot is fermionic.
    ``graph``     the 4-column edge list (source, target, B/F, spin) of Sec. 2.5
                  with the cut external line removed; empty for hand-written R0.
    """
    alpha: np.ndarray
    eps: np.ndarray
    n_int: int
    fermionic: np.ndarray
    seed: Optional[Tuple[int, ...]] = None
    graph: List[Tuple[int, int, int, int]] = field(default_factory=list)

    @property
    def n_g(self) -> int:
        return int(self.alpha.shape[0])

    @property
    def n_freq(self) -> int:
        return int(self.alpha.shape[1])

    @property
    def n_eps(self) -> int:
        return int(self.eps.shape[1])


def order2_example() -> Diagram:
    """The second-order self-energy integrand of Sec. 5.1.1 (Eq. (7)).

    Propagators (frequency part) ``nu_1``, ``nu_2`` and ``-nu_1 + nu_2 + nu_3``
    with the external frequency ``nu_3`` in the last slot, and the identity as
    energy labels.
    """
    alpha = np.array([[1, 0, 0], [0, 1, 0], [-1, 1, 1]], dtype=np.int8)
    eps = np.eye(3, dtype=np.int8)
    return Diagram(alpha=alpha, eps=eps, n_int=2,
                   fermionic=np.ones(3, dtype=np.uint8), seed=None)


class _DSU:
    def __init__(self, n: int):
        self.p = list(range(n))

    def find(self, x: int) -> int:
        while self.p[x] != x:
            self.p[x] = self.p[self.p[x]]
            x = self.p[x]
        return x

    def union(self, a: int, b: int) -> bool:
        ra, rb = self.find(a), self.find(b)
        if ra == rb:
            return False
        self.p[ra] = rb
        return True


def _tree_path(adj, src: int, dst: int):
    """Edges (index, +1/-1 orientation) of the unique tree path src -> dst."""
    prev = {src: None}
    stack = [src]
    while stack:
        v = stack.pop()
        if v == dst:
            break
        for (w, e, orient) in adj[v]:
            if w not in prev:
                prev[w] = (v, e, orient)
                stack.append(w)
    path = []
    v = dst
    while prev[v] is not None:
        u, e, orient = prev[v]
        path.append((e, orient))
        v = u
    path.reverse()
    return path


def _try_topology(order: int, rng: np.random.Generator):
    n = order
    nv = 2 * n
    bos = [(2 * i, 2 * i + 1) for i in range(n)]
    perm = rng.permutation(nv)
    if np.any(perm == np.arange(nv)):
        return None  # a fermion line closing on its own vertex (tadpole)
    ferm = [(v, int(perm[v])) for v in range(nv)]
    dsu = _DSU(nv)
    for a, b in bos + ferm:
        dsu.union(a, b)
    if len({dsu.find(v) for v in range(nv)}) != 1:
        return None  # disconnected
    cut = int(rng.integers(nv))
    ext_out, ext_in = ferm[cut]          # external frequency enters ext_in, leaves ext_out
    lines = [f for i, f in enumerate(ferm) if i != cut]   # 2n-1 propagators
    # spanning tree through every bosonic line, then fermionic lines in random order
    dsu = _DSU(nv)
    tree_edges = []   # (u, v, kind, line index or -1)
    for a, b in bos:
        dsu.union(a, b)
        tree_edges.append((a, b, 0, -1))
    loops = []
    for li in rng.permutation(len(lines)):
        a, b = lines[li]
        if dsu.union(a, b):
            tree_edges.append((a, b, 1, int(li)))
        else:
            loops.append(int(li))
    if len(loops) != n:
        return None
    adj = {v: [] for v in range(nv)}
    for ei, (a, b, _, _) in enumerate(tree_edges):
        adj[a].append((b, ei, +1))   # traversing a -> b follows the edge
        adj[b].append((a, ei, -1))
    n_freq = n + 1
    tree_lab = np.zeros((len(tree_edges), n_freq), dtype=np.int64)
    line_lab = np.zeros((len(lines), n_freq), dtype=np.int64)
    for slot, li in enumerate(loops):
        a, b = lines[li]
        line_lab[li, slot] = 1               # loop variable flows a -> b on its own line
        for e, orient in _tree_path(adj, b, a):   # and returns b -> a through the tree
            tree_lab[e, slot] += orient
    for e, orient in _tree_path(adj, ext_in, ext_out):
        tree_lab[e, n] += orient
    for ei, (_, _, kind, li) in enumerate(tree_edges):
        if kind == 1:
            line_lab[li] = tree_lab[ei]
    # order the propagators: loop lines first (unit rows), then the others
    order_rows = list(loops) + [li for li in range(len(lines)) if li not in loops]
    alpha = line_lab[order_rows]
    if np.abs(alpha).max() > 1:
        return None
    if np.any(np.count_nonzero(alpha, axis=1) % 2 == 0):
        return None  # every propagator must carry a fermionic frequency
    if np.any(np.count_nonzero(alpha[:, :n], axis=0) < 2):
        return None  # a loop through one propagator only (Fock-type insertion)
    rows = {}
    for r in alpha:
        key = tuple(int(x) for x in r)
        neg = tuple(-x for x in key)
        if key in rows or neg in rows:
            return None  # equal lines up to sign: repeated energies, higher-order poles
        rows[key] = True
    graph = []
    for li in order_rows:
        a, b = lines[li]
        graph.append((int(a), int(b), 1, 0))
    for a, b in bos:
        graph.append((a, b, 0, 0))
    return alpha.astype(np.int8), graph


def random_self_energy(order: int, seed: Sequence[int] | int) -> Diagram:
    """A seeded random connected self-energy topology of the given order."""
    if order < 1:
        raise ValueError("order must be >= 1")
    rng = np.random.default_rng(seed)
    for _ in range(100000):
        got = _try_topology(order, rng)
        if got is None:
            continue
        alpha, graph = got
        ng = alpha.shape[0]
        return Diagram(alpha=alpha, eps=np.eye(ng, dtype=np.int8), n_int=order,
                       fermionic=np.ones(order + 1, dtype=np.uint8),
                       seed=tuple(np.atleast_1d(seed).tolist()), graph=graph)
    raise RuntimeError("no topology found")


def diagram_set(order: int, count: int, base_seed: int = 0):
    """Iterator over ``count`` candidates of the given order, seeds (base_seed, order, i)."""
    i = 0
    made = 0
    while made < count:
        yield random_self_energy(order, (base_seed, order, i))
        i += 1
        made += 1


def relabel(d: Diagram, loop_perm: Sequence[int], row_perm: Sequence[int] | None = None,
            loop_sign: Sequence[int] | None = None) -> Diagram:
    """Same integrand with the summed frequencies permuted (and optionally negated)
    and the propagators reordered; the integrand's value is unchanged."""
    n = d.n_int
    cols = list(loop_perm) + list(range(n, d.n_freq))
    alpha = d.alpha[:, cols].astype(np.int64)
    if loop_sign is not None:
        alpha[:, :n] *= np.asarray(loop_sign, dtype=np.int64)[None, :]
    eps = d.eps.copy()
    if row_perm is not None:
        alpha = alpha[list(row_perm)]
        eps = eps[list(row_perm)]
    return Diagram(alpha=alpha.astype(np.int8), eps=eps, n_int=n,
                   fermionic=d.fermionic[cols].copy(), seed=d.seed, graph=d.graph)
