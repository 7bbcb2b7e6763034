"""Pins of oracle/colouring.py (CPU only): closed-form colour counts, validity by
breadth-first search on the real matrix graph, greedy results with known form."""
import itertools

import numpy as np
import pytest

from oracle import colouring, lattice


def l1_ball_size(dim, r):
    return sum(1 for d in itertools.product(range(-r, r + 1), repeat=dim) if sum(map(abs, d)) <= r)


@pytest.mark.parametrize("dim,radius,expect", [(2, 1, 2), (2, 2, 5), (2, 4, 13), (2, 8, 41),
                                               (3, 1, 2), (3, 2, 7), (3, 6, 70)])
def test_modular_counts(dim, radius, expect):
    C, _ = colouring.find_modular(dim, radius)
    assert C == expect
    # every pair inside an L1 ball of radius radius // 2 is within distance radius,
    # so no colouring can use fewer colours than that ball has points
    assert C >= l1_ball_size(dim, radius // 2)


@pytest.mark.parametrize("shape,power,k", [((13, 11), 1, 2), ((12, 10), 2, 2), ((9, 8), 2, 4), ((6, 5, 7), 1, 2)])
def test_modular_colouring_valid_on_matrix_graph(shape, power, k):
    dim = len(shape)
    M = lattice.shifted_laplacian(shape, 0.1)
    Q = M if power == 1 else lattice.squared(M)
    radius = k * power          # graph distance in G(M^2) is ceil(L1 / 2)
    C, coeffs = colouring.find_modular(dim, radius)
    c = colouring.modular_colouring(shape, C, coeffs)
    assert colouring.is_valid_colouring(Q, c, k)
    assert not colouring.is_valid_colouring(Q, c, k + 1)


def test_greedy_on_path_and_grid():
    n = 17
    path = lattice.laplacian((n,))
    for k in (1, 2, 3):
        c = colouring.greedy_colouring(path, k)
        assert np.array_equal(c, np.arange(n) % (k + 1))
    grid = lattice.laplacian((6, 5))
    c = colouring.greedy_colouring(grid, 1)
    xs, ys = np.arange(30) % 6, np.arange(30) // 6
    assert np.array_equal(c, (xs + ys) % 2)


def test_greedy_valid_and_order_is_permutation_invariant():
    shape = (9, 7)
    Q = lattice.squared(lattice.shifted_laplacian(shape, 0.1))
    rng = np.random.default_rng(3)
    prio = rng.permutation(63)
    order = colouring.order_from_priority(prio)
    c = colouring.greedy_colouring(Q, 2, order)
    assert colouring.is_valid_colouring(Q, c, 2)
    # the same greedy on the symmetrically permuted matrix in natural order
    P = np.eye(63)[order]
    Qp = P @ Q.toarray() @ P.T
    cp = colouring.greedy_colouring(Qp, 2)
    assert np.array_equal(c[order], cp)


def test_modular_colour_count_independent_of_resolution():
    # Sec. 3: the number of colours does not depend on the discretisation granularity
    C, coeffs = colouring.find_modular(2, 8)
    for m in (41, 64, 200):
        assert len(np.unique(colouring.modular_colouring((m, m), C, coeffs))) == C
