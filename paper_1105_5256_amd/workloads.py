"""Seeded synthetic inputs for the lattice GMRF workloads.

This module only draws and lays out input data (lattice shapes, kappa^2
values and fields, observation points with their bilinear weights, greedy
priorities).  It holds none of the log-determinant method's arithmetic and is
the single source of inputs for both the library's tests/benchmark and the
CPU reference, so that both see identical arrays.  Random numbers come from
numpy's PCG64 (``numpy.random.default_rng(seed)``).

The paper's experiments (Sec. 3) use simulated SPDE fields on 2-D lattices of
unstated size and a 3-D lattice with about two million sites; these inputs
are synthetic stand-ins with the same operators and scales:

* ``lattice2d_5pt``   Q = kappa2 I + L, 5-point Dirichlet Laplacian;
* ``lattice2d_sq``    Q = (kappa2 I + L)^2, the 13-point operator;
* ``lattice3d_field`` Q = diag(kappa2(s)) + L (7-point) with
                      log kappa2(s) = eta0 + eta1 z(s), z a smooth standardised
                      Gaussian field;
* ``posterior2d``     Q_p = (kappa2 I + L)^2 + tau A^T A with A the bilinear
                      interpolation at uniformly scattered points;
* ``batch2d``         many independent square fields of uneven size and
                      kappa2 ~ LogUniform(0.01, 1);
* ``lattice2d_sq_csr`` the 13-point operator written out as a CSR matrix (the
                      "CSR form" of the 512 x 512 workload);
* ``random_spd_csr``  a seeded sparse SPD matrix on a random graph of uneven
                      degree (weighted graph Laplacian plus a positive
                      diagonal), for the general sparse path;
* ``spde_field_sample`` an exact draw of the directly observed field of
                      Q = tau^2 (kappa2 I + L)^2 (the data of the
                      hyperparameter fit).
"""
import numpy as np


def lattice2d_5pt(m=64, kappa2=0.1, k=2):
    """Plain 2-D SPDE precision kappa2 I + L on an m x m lattice."""
    return dict(kind="5pt", shape=(m, m), kappa2=float(kappa2), power=1, k=int(k))


def lattice2d_sq(mx=512, my=None, kappa2=0.05, k=4):
    """Squared operator (kappa2 I + L)^2 on an mx x my lattice."""
    my = mx if my is None else my
    return dict(kind="sq", shape=(mx, my), kappa2=float(kappa2), power=2, k=int(k))


def spde_field_sample(shape, kappa2, tau, seed):
    """A draw x ~ N(0, Q^{-1}) of the directly observed 2-D SPDE field with
    Q = tau^2 (kappa2 I + L)^2 (L the 5-point Dirichlet Laplacian): L is
    diagonalised by the orthonormal DST-I, with eigenvalue
    4 sin^2(pi i / (2 (mx + 1))) + 4 sin^2(pi j / (2 (my + 1))) at frequency
    (i, j), so x = S (w / (tau (kappa2 + lambda))) with w ~ N(0, I).
    Returned flat in site order (x fastest)."""
    import scipy.fft as sfft
    mx, my = (int(m) for m in shape)
    lx = 4.0 * np.sin(np.pi * np.arange(1, mx + 1) / (2.0 * (mx + 1))) ** 2
    ly = 4.0 * np.sin(np.pi * np.arange(1, my + 1) / (2.0 * (my + 1))) ** 2
    lam = ly[:, None] + lx[None, :]                     # array shape (my, mx)
    w = np.random.default_rng(seed).standard_normal((my, mx))
    return sfft.idstn(w / (tau * (kappa2 + lam)), type=1, norm="ortho").ravel()


def smooth_field(shape, sigma, seed):
    """Standardised smooth Gaussian field: white noise N(0, 1) on the lattice,
    convolved periodically (FFT) with a Gaussian kernel of standard deviation
    ``sigma`` sites, then shifted/scaled to sample mean 0 and sd 1.
    Returned flat in site order (x fastest)."""
    rshape = tuple(reversed(tuple(int(m) for m in shape)))
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(rshape)
    freqs = np.meshgrid(*[np.fft.fftfreq(m) for m in rshape], indexing="ij")
    f2 = sum(f * f for f in freqs)
    kernel_hat = np.exp(-2.0 * np.pi ** 2 * sigma ** 2 * f2)
    z = np.real(np.fft.ifftn(np.fft.fftn(w) * kernel_hat))
    z = (z - z.mean()) / z.std()
    return z.ravel()


def lattice3d_field(m=128, eta=(np.log(0.1), 0.5), sigma=8.0, seed=3, k=2, shape=None):
    """3-D precision diag(kappa2(s)) + L with log kappa2 = eta0 + eta1 z(s).

    Returns the field z and the inputs derived from it: kappa2 (the operator's
    diagonal shift) and the two derivative diagonals d kappa2 / d eta0 = kappa2,
    d kappa2 / d eta1 = kappa2 * z (the operator is linear in kappa2)."""
    shape = (m, m, m) if shape is None else tuple(shape)
    z = smooth_field(shape, sigma, seed)
    kappa2 = np.exp(eta[0] + eta[1] * z)
    return dict(kind="3d", shape=shape, eta=tuple(float(e) for e in eta), z=z,
                kappa2_field=kappa2, dkappa2=[kappa2, kappa2 * z], power=1, k=int(k))


def observations(shape, nobs, seed):
    """Uniform points in [0, mx - 1) x [0, my - 1) with bilinear weights.

    Returns (corner (nobs x 4 int32 site ids), weight (nobs x 4 float64)) for
    the corners (x0, y0), (x0 + 1, y0), (x0, y0 + 1), (x0 + 1, y0 + 1) of the
    cell holding each point."""
    mx, my = shape
    rng = np.random.default_rng(seed)
    px = rng.uniform(0.0, mx - 1.0, nobs)
    py = rng.uniform(0.0, my - 1.0, nobs)
    ix = np.minimum(np.floor(px).astype(np.int64), mx - 2)
    iy = np.minimum(np.floor(py).astype(np.int64), my - 2)
    fx = px - ix
    fy = py - iy
    s00 = ix + mx * iy
    corner = np.stack([s00, s00 + 1, s00 + mx, s00 + mx + 1], axis=1).astype(np.int32)
    weight = np.stack([(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy], axis=1)
    return corner, weight


def posterior2d(m=1024, kappa2=0.05, tau=100.0, nobs=100_000, seed=4, k=4, shape=None):
    """Gauss-linear posterior precision (kappa2 I + L)^2 + tau A^T A."""
    shape = (m, m) if shape is None else tuple(shape)
    corner, weight = observations(shape, nobs, seed)
    return dict(kind="post", shape=shape, kappa2=float(kappa2), power=2, tau=float(tau),
                corner=corner, weight=weight, k=int(k))


def batch2d(nfields=256, side_lo=32, side_hi=256, seed=5, k=4):
    """Independent fields (kappa2_f I + L)^2 on side_f x side_f lattices with
    side_f ~ U{side_lo..side_hi} and kappa2_f ~ LogUniform(0.01, 1)."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, nfields)
    kappa2 = np.exp(rng.uniform(np.log(0.01), np.log(1.0), nfields))
    fields = [dict(kind="sq", shape=(int(s), int(s)), kappa2=float(c), power=2, k=int(k))
              for s, c in zip(sides, kappa2)]
    return dict(kind="batch", fields=fields)


def lattice2d_sq_csr(mx, my=None, kappa2=0.05, scale=1.0):
    """CSR arrays (rowptr, colind, val) of scale * (kappa2 I + L)^2 on an
    mx x my Dirichlet lattice, site index x + mx y, columns ascending.

    Entries of the product M M with M = kappa2 I + L: (kappa2 + 4)^2 plus the
    number of in-lattice axis neighbours on the diagonal, -2 (kappa2 + 4) to the
    axis neighbours, +2 to the diagonal neighbours, +1 two steps along an axis.
    """
    my = mx if my is None else my
    c4 = kappa2 + 4.0
    x, y = np.meshgrid(np.arange(mx), np.arange(my), indexing="xy")
    x, y = x.ravel(), y.ravel()
    deg = (x > 0).astype(np.int64) + (x < mx - 1) + (y > 0) + (y < my - 1)
    rows, cols, vals = [], [], []
    offsets = [(0, 0, None), (1, 0, -2 * c4), (-1, 0, -2 * c4), (0, 1, -2 * c4), (0, -1, -2 * c4),
               (1, 1, 2.0), (1, -1, 2.0), (-1, 1, 2.0), (-1, -1, 2.0),
               (2, 0, 1.0), (-2, 0, 1.0), (0, 2, 1.0), (0, -2, 1.0)]
    site = x + mx * y
    for dx, dy, v in offsets:
        xx, yy = x + dx, y + dy
        ok = (xx >= 0) & (xx < mx) & (yy >= 0) & (yy < my)
        rows.append(site[ok])
        cols.append((xx + mx * yy)[ok])
        vals.append((c4 * c4 + deg[ok]) if v is None else np.full(int(ok.sum()), v))
    return _to_csr(mx * my, np.concatenate(rows), np.concatenate(cols), scale * np.concatenate(vals))


def lattice2d_5pt_csr(mx, my=None, kappa2=0.05, scale=1.0):
    """CSR arrays of scale * (kappa2 I + L) (5-point, Dirichlet) on an mx x my
    lattice, site index x + mx y: kappa2 + 4 on the diagonal, -1 to the axis
    neighbours inside the lattice."""
    my = mx if my is None else my
    x, y = np.meshgrid(np.arange(mx), np.arange(my), indexing="xy")
    x, y = x.ravel(), y.ravel()
    site = x + mx * y
    rows, cols, vals = [site], [site], [np.full(mx * my, kappa2 + 4.0)]
    for dx, dy in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
        xx, yy = x + dx, y + dy
        ok = (xx >= 0) & (xx < mx) & (yy >= 0) & (yy < my)
        rows.append(site[ok])
        cols.append((xx + mx * yy)[ok])
        vals.append(np.full(int(ok.sum()), -1.0))
    return _to_csr(mx * my, np.concatenate(rows), np.concatenate(cols), scale * np.concatenate(vals))


def random_spd_csr(n, deg_lo=2, deg_hi=12, shift=0.05, seed=7, signs=False):
    """Sparse SPD matrix on a random graph: vertex i draws d_i ~ U{deg_lo..deg_hi}
    partners uniformly, edges get weights U(0.5, 1.5) and the pattern is
    symmetrised; Q = D - W + diag(shift * U(0.5, 2)) (weighted graph Laplacian
    plus a positive diagonal).  With signs=True, Q -> S Q S for random signs S
    (same spectrum; the all-ones vector then misses the lowest eigenvector).
    Returns (rowptr, colind, val)."""
    rng = np.random.default_rng(seed)
    d = rng.integers(deg_lo, deg_hi + 1, n)
    src = np.repeat(np.arange(n), d)
    dst = rng.integers(0, n, src.size)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    w = rng.uniform(0.5, 1.5, src.size)
    a, b = np.minimum(src, dst), np.maximum(src, dst)
    key = a.astype(np.int64) * n + b
    key, first = np.unique(key, return_index=True)
    a, b, w = a[first], b[first], w[first]
    diag = np.zeros(n)
    np.add.at(diag, a, w)
    np.add.at(diag, b, w)
    diag += shift * rng.uniform(0.5, 2.0, n)
    rows = np.concatenate([a, b, np.arange(n)])
    cols = np.concatenate([b, a, np.arange(n)])
    vals = np.concatenate([-w, -w, diag])
    if signs:
        s = rng.choice([-1.0, 1.0], n)
        vals = vals * s[rows] * s[cols]
    return _to_csr(n, rows, cols, vals)


def _to_csr(n, rows, cols, vals):
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    return np.cumsum(rowptr).astype(np.int32), cols.astype(np.int32), vals.astype(np.float64)


def priority(n, seed):
    """A seeded random permutation of 0..n-1, used as greedy colouring priority."""
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


# Full-size workloads of the benchmark configurations.
def full_configs():
    return {
        "lattice64_5pt": lattice2d_5pt(64, 0.1, k=2),
        "lattice512_sq": lattice2d_sq(512, kappa2=0.05, k=4),
        "lattice128c_field": lattice3d_field(128, k=2),
        "posterior1024": posterior2d(1024),
        "batch256": batch2d(256),
    }
