"""usfft_detect_batch: uneven jobs (different meshes, d, boxes, s and
precisions, plus an unfused trigonometric-polynomial job and a 128^2-mesh
job whose streaming solver keeps launches of its own) run together with
their PDE solves fused into shared persistent launches; every job's result
must equal the job run alone (each solve is independent of its batch)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def uneven_jobs():
    out = []
    for n, d, N, s, prec, seed in [(16, 4, 8, 20, 1, 1), (16, 3, 12, 30, 1, 2), (16, 6, 4, 20, 1, 3),
                                   (33, 4, 8, 20, 0, 4), (33, 5, 8, 25, 0, 5), (64, 4, 8, 20, 1, 6),
                                   (128, 3, 8, 20, 1, 8)]:
        out.append((W.pde_problem(n, d, N), dict(W.params(s, 2, 1e-4), precision=prec), seed))
    K, P = W.trig_poly(7, 3, 8, 40, 21, cmin=1e-2)
    out.append((dict(sampler="poly", d=3, k_lo=[-8] * 3, k_hi=[8] * 3, poly_k=K, poly_c=P),
                W.params(42, 3, 1e-6, relative=False), 7))
    return out


def test_batch_equals_alone(lib):
    jobs = uneven_jobs()
    alone = []
    for prob, par, seed in jobs:
        r = lib.detect(lib.Plan(prob, par), seed)
        alone.append((r.freqs(), r.coeffs(), r.stats["samples"]))
    plans = [lib.Plan(prob, par) for prob, par, _ in jobs]
    res, sts, fs = lib.detect_batch(plans, [seed for _, _, seed in jobs])
    print("solver launches %d, fused launches %d, job segments %d" % fs)
    assert all(st == lib.OK for st in sts), sts
    for (I, C, ns), r in zip(alone, res):
        assert np.array_equal(r.freqs(), I)
        assert np.array_equal(r.coeffs(), C)
        assert r.stats["samples"] == ns
    # three classes share launches: mesh 16 float32 (3 jobs), mesh 33 float64 (2 jobs)
    assert fs[1] > 0 and fs[2] > fs[0]
    # the plans still run alone afterwards
    again = lib.detect(plans[0], jobs[0][2])
    assert np.array_equal(again.coeffs(), alone[0][1])


def test_batch_reports_job_errors(lib):
    jobs = uneven_jobs()[:3]
    plans = [lib.Plan(prob, dict(par, pcg_maxit=2) if i == 1 else par) for i, (prob, par, _) in enumerate(jobs)]
    res, sts, fs = lib.detect_batch(plans, [seed for _, _, seed in jobs])
    assert sts[1] == lib.ENOCONV and res[1] is None
    assert sts[0] == lib.OK and sts[2] == lib.OK
    ref = lib.detect(lib.Plan(*jobs[2][:2]), jobs[2][2])
    assert np.array_equal(res[2].coeffs(), ref.coeffs())
