"""Choice of the colouring distance from log(Q) e_j (NEXT row f2).

Sec. 2.1, probing paragraph: the distance p of the probing colouring (the
power of Q whose graph is coloured) can be chosen with the heuristic of the
diagonal-of-the-inverse probing literature, applied to log(Q) instead of
Q^{-1}: compute x = log(Q) e_j and take p = min{d(l, j) : |x_l| < eps}, d the
graph distance of Q.  x comes from the library (f_N(Q) e_j, two Krylov
solves per site, several sites in one call); the rule itself is host
arithmetic on that vector.

Readings (the paper states the rule only in words): eps is taken relative to
|x_j| (the diagonal entry), so that the choice does not depend on the units of
Q; rule="first" is the rule as written (the nearest graph distance at which an
entry is small), rule="all" the distance beyond which every entry is small
(robust to entries that are small by a change of sign); the largest value over
the given sites is returned.  Lattice graph distances: the L1 distance for the
5- and 7-point operators, ceil(L1 / 2) for the 13-point squared operator.
"""
import numpy as np

from . import ldq


def graph_distances(shape, site, squared):
    """Graph distance of every lattice site from `site` (sites x + nx (y + ny z))."""
    shape = tuple(int(m) for m in shape)
    coords = np.unravel_index(np.arange(int(np.prod(shape))), tuple(reversed(shape)))
    c0 = np.unravel_index(site, tuple(reversed(shape)))
    l1 = sum(np.abs(a - b) for a, b in zip(coords, c0))
    return (l1 + 1) // 2 if squared else l1


def choose_distance(ctx, Q, shape, squared, eps=1e-3, sites=None, opts=None, rule="all"):
    """Colouring distance for lattice operator Q by the log(Q) e_j heuristic.
    Returns (p, details) with the per-site distances and the vectors' peak entries."""
    import torch
    shape = tuple(int(m) for m in shape)
    n = int(np.prod(shape))
    if sites is None:
        centre = [m // 2 for m in shape]
        site = centre[0]
        stride = 1
        for d in range(1, len(shape)):
            stride *= shape[d - 1]
            site += centre[d] * stride
        sites = [site]
    V = torch.zeros((len(sites), n), dtype=torch.float64, device="cuda")
    for i, s in enumerate(sites):
        V[i, s] = 1.0
    Y, info = ldq.ldq_logm_apply(ctx.handle, Q, V, opts)
    Y = Y.cpu().numpy()
    per_site = []
    for i, s in enumerate(sites):
        d = graph_distances(shape, s, squared)
        small = np.abs(Y[i]) < eps * abs(Y[i, s])
        if rule == "first":
            ds = d[small & (d > 0)]
            p = int(ds.min()) if ds.size else int(d.max())
        else:
            big = ~small & (d > 0)
            p = int(d[big].max()) + 1 if big.any() else 1
        per_site.append(p)
    return max(per_site), {"per_site": per_site, "sites": list(sites), "iters": info["iters_max"]}
