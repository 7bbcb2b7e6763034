"""Distance-k graph colourings that define the probing vectors (oracle; test infrastructure only).

Sec. 2.1 (probing paragraph): the probing vectors come from a neighbour
colouring of the graph of Q^p; vertices within graph distance p of each
other in G(Q) are adjacent in G(Q^p), so a colouring of G(Q^p) is a
distance-p colouring of G(Q): no two vertices with 0 < d(i, i') <= p share a
colour.  The probe of colour j is the 0/1 indicator of that colour class;
it can be formed on the fly from the colour array.  Greedy colouring is the
algorithm the paper points to (the survey of Culberson).
"""
from collections import deque
import itertools

import numpy as np
import scipy.sparse as sp


def adjacency(Q):
    """CSR pattern (indptr, indices) of G(Q) without the diagonal."""
    A = sp.csr_matrix(Q, copy=True)
    A.setdiag(0)
    A.eliminate_zeros()
    A.sort_indices()
    return A.indptr, A.indices


def ball(indptr, indices, i, k):
    """Vertices at graph distance 1..k from vertex i (breadth-first search)."""
    dist = {i: 0}
    queue = deque([i])
    out = []
    while queue:
        u = queue.popleft()
        if dist[u] == k:
            continue
        for w in indices[indptr[u]:indptr[u + 1]]:
            w = int(w)
            if w not in dist:
                dist[w] = dist[u] + 1
                out.append(w)
                queue.append(w)
    return out


def is_valid_colouring(Q, colours, k):
    """True when no two vertices at distance 1..k in G(Q) share a colour."""
    indptr, indices = adjacency(Q)
    colours = np.asarray(colours)
    n = len(colours)
    for i in range(n):
        for w in ball(indptr, indices, i, k):
            if colours[w] == colours[i]:
                return False
    return True


def greedy_colouring(Q, k, order=None):
    """Sequential greedy distance-k colouring.

    Vertices are visited in ``order`` (default 0..n-1); each takes the smallest
    colour not already held by a vertex within distance k.  Returns the int32
    colour array.
    """
    indptr, indices = adjacency(Q)
    n = len(indptr) - 1
    if order is None:
        order = range(n)
    colours = np.full(n, -1, dtype=np.int64)
    for i in order:
        i = int(i)
        used = set()
        for w in ball(indptr, indices, i, k):
            if colours[w] >= 0:
                used.add(int(colours[w]))
        c = 0
        while c in used:
            c += 1
        colours[i] = c
    return colours.astype(np.int32)


def order_from_priority(priority):
    """Visit order for ``greedy_colouring`` from a priority array: ascending
    priority value, ties broken by the lower vertex index."""
    priority = np.asarray(priority)
    return np.lexsort((np.arange(len(priority)), priority))


def modular_colouring(shape, C, coeffs):
    """c(x, y[, z]) = (x + a y [+ b z]) mod C on a lattice (site numbering x fastest)."""
    shape = tuple(int(m) for m in shape)
    grids = np.meshgrid(*[np.arange(m) for m in reversed(shape)], indexing="ij")
    # grids[-1] is x, grids[-2] is y, grids[-3] is z
    lin = grids[-1].astype(np.int64)
    for a, g in zip(coeffs, reversed(grids[:-1])):
        lin = lin + int(a) * g.astype(np.int64)
    return (lin % C).astype(np.int32).ravel()


def _offsets(dim, radius):
    """All nonzero integer offsets d in Z^dim with |d|_1 <= radius."""
    rng = np.arange(-radius, radius + 1)
    grid = np.array(np.meshgrid(*([rng] * dim), indexing="ij")).reshape(dim, -1).T
    l1 = np.abs(grid).sum(axis=1)
    return grid[(l1 > 0) & (l1 <= radius)]


def find_modular(dim, radius):
    """Smallest C (then the lexicographically smallest coefficients) such that
    (x + a y [+ b z]) mod C separates every pair of lattice points at L1
    distance 1..radius on the infinite lattice Z^dim.

    A pair at offset d gets the same colour exactly when
    d_x + a d_y [+ b d_z] = 0 (mod C); every offset of the L1 ball is tried."""
    D = _offsets(dim, radius)
    C = 1
    while True:
        coeffs = np.array(list(itertools.product(range(C), repeat=dim - 1)), dtype=np.int64)
        coef = np.concatenate([np.ones((len(coeffs), 1), dtype=np.int64), coeffs], axis=1)
        vals = (coef @ D.T) % C                   # (#coefficient choices) x (#offsets)
        ok = np.all(vals != 0, axis=1)
        if ok.any():
            first = int(np.argmax(ok))
            return C, tuple(int(a) for a in coeffs[first])
        C += 1
