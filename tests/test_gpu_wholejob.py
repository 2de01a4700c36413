"""Whole-job parity of usfft_detect against the oracle (Alg. 1 steps 1 to 3,
"Output": the set I and the coefficients of every node).

The expected values are the oracle's, written by tests/golden/make_wholejob.py
(which calls only oracle/ and workloads/) for seed 1 at two workloads with
the box [-32,32]^10, s = 200, relative threshold 1e-5 and r = 5: h = 1/64
(G = 3969, the benchmark's workload) and h = 1/16 (G = 225); and on the
h = 1/128 mesh (G = 16129, the streaming DST solver) and the h = 1/256 mesh
(G = 65025, the two-level solver) at d = 4, box [-8,8]^4, s = 30, relative
threshold 1e-4, r = 2.  The library
runs in the benchmark's configuration (pcg_rtol 1e-12) with its detection
trace on, so every intermediate set is compared:
  * float64: every set I^(t) of step 1 and I^(1..t) of step 2 identical to
    the oracle's, the same sample counts and lattices (so the same families),
    the threshold within 1e-10, coefficients within 1e-10 of the largest,
    solves within 1e-11 (nodal relative l2);
  * float32 + float64 refinement: sets identical except flips whose oracle
    keep ratio |c|^2 / threshold^2 lies within 1 % of the threshold in
    magnitude, each listed; coefficients within 1e-6 of the largest when the
    sets agree; solves within 1e-9.
A flip changes every later candidate set, so comparison stops at the first
increment that differs.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle.select import product

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BAND = (0.99 ** 2, 1.01 ** 2)  # keep ratios of squared magnitudes within 1 % of the threshold
SEED = 1


def fixture(name):
    path = os.path.join(GOLDEN, "wholejob_%s.npz" % name)
    if not os.path.exists(path):
        pytest.skip("fixture %s not generated" % path)
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def rows(a):
    return {tuple(int(v) for v in r) for r in np.asarray(a).reshape(len(a), -1)}


def compare_trace(fx, tr, d, k_lo):
    """First differing increment and its flips [(stage, k, oracle ratio, kept by oracle)]."""
    flips = []
    for t in range(d):
        got, ref = tr[t][0][:, 0], fx["s1_I_%d" % t]
        if not np.array_equal(got, ref):
            for k in sorted(set(got.tolist()) ^ set(ref.tolist())):
                flips.append(("step1 t=%d" % (t + 1), (k,), float(fx["s1_ratio_%d" % t][k - k_lo[t]]),
                              k in set(ref.tolist())))
            return flips
    prev = fx["s1_I_0"][:, None]
    for t in range(1, d):
        got, nc = tr[d + t - 1]
        assert nc == int(fx["s2_nJ_%d" % t]), "candidate count |J_%d| differs" % (t + 1)
        ref = fx["s2_I_%d" % t]
        if not np.array_equal(got, ref):
            J = product(prev, fx["s1_I_%d" % t])
            index = {tuple(int(v) for v in r): a for a, r in enumerate(J)}
            rs = rows(ref)
            for k in sorted(rows(got) ^ rs):
                flips.append(("step2 t=%d" % (t + 1), k, float(fx["s2_ratio_%d" % t][index[k]]), k in rs))
            return flips
        prev = ref
    return flips


@pytest.mark.parametrize("name,prec,autotune", [("mesh16_d10", 0, 0), ("mesh16_d10", 1, 0), ("mesh64_d10", 0, 0),
                                                ("mesh64_d10", 1, 0), ("mesh64_d10", 1, 1), ("mesh128_d4", 0, 0),
                                                ("mesh128_d4", 1, 0), ("mesh256_d4", 0, 0), ("mesh256_d4", 1, 0)])
def test_whole_job_against_oracle(lib, name, prec, autotune):
    fx = fixture(name)
    prob, par = W.WORKLOADS[name]
    d = prob["d"]
    print("whole job %s precision %d autotune %d seed %d" % (name, prec, autotune, SEED), flush=True)
    plan = lib.Plan(prob, dict(par, precision=prec, pcg_rtol=1e-12, trace=True, autotune=autotune))
    try:
        res = lib.detect(plan, SEED)
    finally:
        if autotune:
            lib.tune_clear()  # later tests keep the built-in choices
    flips = compare_trace(fx, res.trace(), d, prob["k_lo"])
    for f in flips:
        print("flip at %s: k = %s, oracle keep ratio %.6f, kept by the oracle: %s" % f)
    if prec == lib.FP64:
        assert not flips, "float64 sets differ from the oracle"
    for f in flips:
        assert BAND[0] <= f[2] <= BAND[1], "flip outside 1 %% of the threshold: %s" % (f,)
    tol_c = 1e-10 if prec == lib.FP64 else 1e-6
    st = res.stats
    assert abs(st["theta_abs"] ** 2 - float(fx["theta2"])) <= 1e-10 * float(fx["theta2"]) * (1 if prec == 0 else 1e4)
    if not flips:
        assert np.array_equal(res.freqs(), fx["I"])
        for k in ("samples", "samples_step1", "samples_step2", "samples_step3", "lattices"):
            assert st[k] == int(fx[k]), k
        C = res.coeffs()[:, fx["nodes"]]
        ref = fx["C_re"] + 1j * fx["C_im"]
        err = np.abs(C - ref).max() / float(fx["Cmax"])
        print("%s precision %d: |I| = %d, samples = %d, max coefficient error %.2e of the largest"
              % (name, prec, res.n, st["samples"], err))
        assert err <= tol_c
    # solves at seeded nodes in the same configuration
    y = torch.from_numpy(fx["y_solve"]).cuda()
    n = y.shape[0]
    U = torch.zeros((plan.G, 64), dtype=torch.float64, device="cuda")
    lib.sample(plan, y, U, 0, 64, 0)
    torch.cuda.synchronize()
    Ug = U.cpu().numpy()[:, :n].T
    ref = fx["u_solve"]
    e = (np.linalg.norm(Ug - ref, axis=1) / np.linalg.norm(ref, axis=1)).max()
    print("%s precision %d: max nodal rel. l2 error %.2e" % (name, prec, e))
    assert e <= (1e-11 if prec == lib.FP64 else 1e-9)
