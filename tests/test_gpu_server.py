"""Serving loop: continuous batching of whole jobs.  Every job's result
through the server (several jobs in flight on separate streams) must be
bitwise the result of the same job run alone."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def jobs():
    out = []
    for seed, d, N, G, nf in [(1, 3, 8, 40, 21), (2, 6, 16, 33, 41), (3, 4, 8, 70, 31)]:
        K, P = W.trig_poly(seed, d, N, G, nf, cmin=1e-2)
        out.append((dict(sampler="poly", d=d, k_lo=[-N] * d, k_hi=[N] * d, poly_k=K, poly_c=P),
                    W.params(2 * nf, 3, 1e-6, relative=False), seed))
    for seed, n, prec in [(4, 16, 0), (5, 12, 1), (6, 16, 1)]:
        prob = W.pde_problem(n, 4, 12, modes="diagonal")
        out.append((prob, dict(W.params(30, 2, 1e-4), precision=prec), seed))
    # a general triangulation: the server keeps its own copy of the mesh
    out.append((W.mesh_problem(W.jittered_mesh(8, 9, 7), 4, 8), W.params(30, 2, 1e-4), 7))
    return out


def test_server_results_equal_alone(lib):
    alone = []
    for prob, par, seed in jobs():
        plan = lib.Plan(prob, par)
        r = lib.detect(plan, seed)
        alone.append((r.freqs(), r.coeffs(), r.stats["samples"]))
    srv = lib.Server(max_active=3)
    ids = [srv.submit(prob, par, seed) for prob, par, seed in jobs()]
    for (I, C, ns), jid in zip(alone, ids):
        res, st, lat, q, err = srv.poll(jid, wait=True)
        assert st == lib.OK, err
        assert np.array_equal(res.freqs(), I)
        assert np.array_equal(res.coeffs(), C)
        assert res.stats["samples"] == ns
        assert lat >= q >= 0.0
    srv.close()


def test_server_budget_and_order(lib):
    prob, par, seed = jobs()[3]
    srv = lib.Server(max_active=2, hbm_budget=1 << 20)
    with pytest.raises(lib.UsfftError) as e:
        srv.submit(prob, par, seed)
    assert e.value.status == lib.EINVAL
    srv.close()
    # a budget that fits one job at a time: admitted in order, all complete
    srv = lib.Server(max_active=4, hbm_budget=3 << 30)
    ids = [srv.submit(p, pa, s) for p, pa, s in jobs()[3:]]
    qs = []
    for jid in ids:
        res, st, lat, q, err = srv.poll(jid, wait=True)
        assert st == lib.OK, err
        qs.append(q)
    srv.close()


def test_server_reports_job_errors(lib):
    prob, par, seed = jobs()[3]
    srv = lib.Server(max_active=2)
    jid = srv.submit(prob, dict(par, pcg_maxit=2, solver_config=-2), seed)
    res, st, lat, q, err = srv.poll(jid, wait=True)
    assert res is None and st == lib.ENOCONV and "PCG" in err
    good = srv.submit(prob, par, seed)
    res, st, *_ = srv.poll(good, wait=True)
    assert st == lib.OK and res.n > 0
    srv.close()


def test_server_reuses_plans(lib):
    """Jobs that share the sampler, coefficient family, mesh and precision run
    on a pooled plan of an earlier job, with their own box, s, r and
    threshold, and still equal the job run alone on a new plan."""
    base = W.pde_problem(16, 4, 12, modes="diagonal")
    specs = [(dict(base, k_lo=[-N] * 4, k_hi=[N] * 4), dict(W.params(s, r, th), precision=1), seed)
             for N, s, r, th, seed in [(12, 30, 2, 1e-4, 11), (8, 20, 3, 1e-3, 12), (16, 40, 2, 1e-4, 13),
                                       (12, 30, 2, 1e-4, 14)]]
    alone = []
    for prob, par, seed in specs:
        r = lib.detect(lib.Plan(prob, par), seed)
        alone.append((r.freqs(), r.coeffs()))
    srv = lib.Server(max_active=1)
    reused = []
    for (prob, par, seed), (I, C) in zip(specs, alone):
        res, st, lat, q, err = srv.poll(srv.submit(prob, par, seed), wait=True)
        assert st == lib.OK, err
        assert np.array_equal(res.freqs(), I)
        assert np.array_equal(res.coeffs(), C)
        reused.append(res.stats["plan_reused"])
    srv.close()
    assert reused == [0, 1, 1, 1]
