"""GPU parity of the batched entry point (many independent lattice fields in
one set of launches) against single-field calls and the CPU oracle.

The batched STEP launches run the same per-tile arithmetic as a single-field
call, with the same fixed reduction order, so every field's result must be
bit-identical to calling the library on that field alone; each field is also
checked against the oracle's rational-approximation estimator and probing
gradient (direct sparse solves).
"""
import sys

import numpy as np
import pytest

from oracle import colouring, estimator, gradient, lattice, shifts
from paper_1105_5256_amd import ldq, workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ldq.Context(0)
    yield c
    c.close()


def rel(a, b):
    return abs(a - b) / abs(b)


def make_fields(ctx, fields):
    Qs, dQs = [], []
    for f in fields:
        Qs.append(ctx.op(ldq.ldq_op_lattice(ctx.handle, f["shape"], ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, f["kappa2"])))
        dQs.append([ctx.op(ldq.ldq_op_lattice(ctx.handle, f["shape"], ldq.LDQ_SHIFTED_LAPLACIAN, f["kappa2"],
                                              scale=2.0))])
    return Qs, dQs


@pytest.mark.parametrize("precision,tol,gtol,bound", [(ldq.LDQ_FP64, 1e-10, 1e-10, 1e-9),
                                                      (ldq.LDQ_MIXED, 1e-5, 1e-6, 1e-4)])
def test_batched_equals_single_calls_and_oracle(ctx, precision, tol, gtol, bound):
    wl = workloads.batch2d(nfields=9, side_lo=5, side_hi=70, seed=8)
    fields = wl["fields"] + [dict(kind="sq", shape=(90, 23), kappa2=0.02, power=2, k=4)]
    say(f"batched {len(fields)} fields, sides {[f['shape'] for f in fields]}, precision={precision}")
    Qs, dQs = make_fields(ctx, fields)
    # single calls on the batched pass's tile height (not the autotuner's choice)
    opts = ldq.ldq_options_default(k=4, nshifts=20, tol=tol, grad_tol=gtol, precision=precision, tile_rows=32)
    vals, grads, infos = ldq.ldq_logdet_batched(ctx.handle, Qs, dQs, opts)
    terms = ldq.ldq_probe_terms(ctx.handle)
    C, co = colouring.find_modular(2, 8)
    first = 0
    for i, f in enumerate(fields):
        v1, g1, info1 = ldq.ldq_logdet_grad(ctx.handle, Qs[i], dQs[i], opts)
        t1 = ldq.ldq_probe_terms(ctx.handle)
        nb = infos[i]["ncolours"]
        assert nb == info1["ncolours"]
        assert vals[i] == v1 and grads[i][0] == g1[0], (i, f["shape"])
        assert np.array_equal(terms[first:first + nb], t1)
        assert infos[i]["iters_max"] == info1["iters_max"] and infos[i]["iters_total"] == info1["iters_total"]
        first += nb
        # the oracle on the same field
        shape, k2 = f["shape"], f["kappa2"]
        M = lattice.shifted_laplacian(shape, k2)
        col = colouring.modular_colouring(shape, C, co)
        s, c = shifts.log_shifts(infos[i]["lambda_min"], infos[i]["lambda_max"], 20)
        E, _ = estimator.estimator_rational_direct(lattice.squared(M), col, s, c)
        G, _ = gradient.grad_probing_dst(shape, k2, 2, col, [2 * M])
        print(f"field {i} {shape} kappa2 {k2:.3g}: rel {rel(vals[i], E):.1e} grad {rel(grads[i][0], G[0]):.1e} "
              f"iters {infos[i]['iters_max']}")
        assert rel(vals[i], E) < bound and rel(grads[i][0], G[0]) < bound
    assert first == terms.shape[0]


# graph-replayed chunks (captured again whenever the work list falls below
# half the captured grid) against launches enqueued one by one: identical
def test_batched_graph_and_direct_agree(ctx):
    wl = workloads.batch2d(nfields=12, side_lo=8, side_hi=96, seed=3)
    say(f"batched graph vs direct, {len(wl['fields'])} fields")
    Qs, dQs = make_fields(ctx, wl["fields"])
    res = []
    for mode in (ldq.LDQ_LAUNCH_DIRECT, ldq.LDQ_LAUNCH_GRAPH, ldq.LDQ_LAUNCH_AUTO):
        opts = ldq.ldq_options_default(k=4, nshifts=20, tol=1e-5, grad_tol=1e-6, precision=ldq.LDQ_MIXED,
                                       check_every=4, launch_mode=mode)
        vals, grads, infos = ldq.ldq_logdet_batched(ctx.handle, Qs, dQs, opts)
        res.append((list(vals), [g[0] for g in grads], [i["iters_total"] for i in infos],
                    ldq.ldq_probe_terms(ctx.handle)))
    for r in res[1:]:
        assert r[0] == res[0][0] and r[1] == res[0][1] and r[2] == res[0][2]
        assert np.array_equal(r[3], res[0][3])


# the tall tile in the batched pass (FP32) against the standard tile
def test_batched_tall_tile(ctx):
    wl = workloads.batch2d(nfields=10, side_lo=20, side_hi=140, seed=4)
    say(f"batched tall tile, {len(wl['fields'])} fields")
    Qs, dQs = make_fields(ctx, wl["fields"])
    out = {}
    for rows in (0, 64):
        opts = ldq.ldq_options_default(k=4, nshifts=20, tol=1e-6, grad_tol=1e-7, precision=ldq.LDQ_MIXED,
                                       tile_rows=rows)
        vals, grads, infos = ldq.ldq_logdet_batched(ctx.handle, Qs, dQs, opts)
        assert infos[0]["tile_rows"] == (64 if rows else 34)
        out[rows] = (vals, [g[0] for g in grads])
    for i in range(len(Qs)):
        assert rel(out[64][0][i], out[0][0][i]) < 1e-6 and rel(out[64][1][i], out[0][1][i]) < 1e-5, i


def test_batched_falls_back_for_mixed_operator_kinds(ctx):
    say("batched call with a lattice field and a CSR field (per-field path)")
    f = dict(shape=(30, 20), kappa2=0.3)
    Ql = ctx.op(ldq.ldq_op_lattice(ctx.handle, f["shape"], ldq.LDQ_SQUARED_SHIFTED_LAPLACIAN, f["kappa2"]))
    n = 600
    rp, ci, v = workloads.lattice2d_sq_csr(30, 20, kappa2=0.3)
    Qc = ctx.op(ldq.ldq_op_csr(ctx.handle, n, rp, ci, v))
    opts = ldq.ldq_options_default(k=2, nshifts=20, tol=1e-10)
    vals, _, infos = ldq.ldq_logdet_batched(ctx.handle, [Ql, Qc], None, opts)
    v0, _ = ldq.ldq_logdet(ctx.handle, Ql, opts)
    v1, _ = ldq.ldq_logdet(ctx.handle, Qc, opts)
    assert vals[0] == v0 and vals[1] == v1
