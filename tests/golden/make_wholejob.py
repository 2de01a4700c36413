"""Write the whole-job fixtures of the usFFT at d = 10 (h = 1/16, 1/64) and
at d = 4 on the h = 1/128 and 1/256 meshes.

Calls only the oracle (oracle/) and the seeded workload definitions
(workloads/): Alg. 1 steps 1 to 3 in float64 on the CPU, with the solves
spread over worker processes (oracle/pool.py; every row is solved alone,
so the results do not depend on the split).  Stored per workload, seed 1:
  theta2                   squared absolute threshold of the relative theta
                           (stage t = 1, i = 1 of step 1)
  samples, samples_step1/2/3, lattices
  s1_I_<t>, s1_ratio_<t>   step 1: the 1-D set I^(t+1) and, per candidate of
                           the box, its keep ratio (max over nodes and the r
                           iterations of |c|^2 over the node's threshold;
                           kept when >= 1)
  s2_nJ_<t>, s2_I_<t>, s2_ratio_<t>, s2_M_<t>, s2_z_<t>
                           step 2, increment t+1: |J|, the detected set
                           I^(1..t+1), keep ratio per candidate of J (max
                           over the iterations), the lattice family
  I, fam3_M, fam3_z        the output set and its step-3 family
  nodes, C_re, C_im, Cmax  coefficients at 64 nodes and max |c| over all nodes
  y_solve, u_solve         8 seeded sampling nodes and their solutions (2 when
                           G > 20000)
Usage: python tests/golden/make_wholejob.py [mesh64_d10|mesh16_d10|mesh128_d4|mesh256_d4 ...]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.fem import PDESampler  # noqa: E402
from oracle.pool import PooledSampler  # noqa: E402
from oracle.usfft import usfft  # noqa: E402

SEED = 1
HERE = os.path.dirname(os.path.abspath(__file__))


def make(name, workers=None):
    prob, par = W.WORKLOADS[name]
    d = prob["d"]
    S = PDESampler(prob["mesh_n"], prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    t0 = time.time()
    with PooledSampler(S, workers) as PS:
        res = usfft(PS, d, prob["k_lo"], prob["k_hi"], par["s"], par["s_local"], par["r"], par["theta"],
                    par["theta_relative"], SEED, par["lattice_c"], par["lattice_tries"], par["lattice_max"],
                    par["lattice_mmax"])
        g = np.random.default_rng(2024)
        y_solve = g.random((8 if S.G <= 20000 else 2, d))  # fewer stored solves on the largest meshes
        u_solve = PS(y_solve)
    out = dict(theta2=np.float64(res.theta2), samples=np.int64(res.samples))
    r = par["r"]
    s1 = 0
    lattices = 0
    for t in range(d):
        st = [s for s in res.stages if s["step"] == 1 and s["t"] == t + 1]
        mask = np.zeros(len(st[0]["cand"]), dtype=bool)
        for s in st:
            mask |= s["mask"]
            s1 += len(s["cand"])
        out["s1_I_%d" % t] = st[0]["cand"][mask].astype(np.int32)
        out["s1_ratio_%d" % t] = np.max([s["ratio"] for s in st], axis=0).astype(np.float32)
    s2 = 0
    for t in range(1, d):
        st = [s for s in res.stages if s["step"] == 2 and s["t"] == t + 1]
        if not st:
            out["s2_nJ_%d" % t] = np.int64(0)
            out["s2_I_%d" % t] = np.zeros((0, t + 1), np.int32)
            continue
        J = st[0]["cand"]
        fam = st[0]["family"]
        mask = np.zeros(len(J), dtype=bool)
        for s in st:
            mask |= s["mask"]
            s2 += fam.total_samples
        out["s2_nJ_%d" % t] = np.int64(len(J))
        out["s2_I_%d" % t] = J[mask].astype(np.int32)
        out["s2_ratio_%d" % t] = np.max([s["ratio"] for s in st], axis=0).astype(np.float32)
        out["s2_M_%d" % t] = np.asarray(fam.M, np.int32)
        out["s2_z_%d" % t] = np.asarray(fam.z, np.int32).reshape(len(fam.M), t + 1)
        lattices += len(fam.M)
    fam3 = [s for s in res.stages if s["step"] == 3][0]["family"]
    I = np.asarray(res.I, np.int32).reshape(-1, d)
    out["I"] = I
    if fam3 is not None:
        out["fam3_M"] = np.asarray(fam3.M, np.int32)
        out["fam3_z"] = np.asarray(fam3.z, np.int32).reshape(len(fam3.M), d)
        lattices += len(fam3.M)
        s3 = fam3.total_samples
    else:
        s3 = 0
    out.update(samples_step1=np.int64(s1), samples_step2=np.int64(s2), samples_step3=np.int64(s3),
               lattices=np.int64(lattices))
    assert s1 + s2 + s3 == res.samples
    G = S.G
    nodes = np.unique(np.linspace(0, G - 1, 64).round().astype(np.int64))
    out["nodes"] = nodes
    out["C_re"] = res.C[:, nodes].real.copy()
    out["C_im"] = res.C[:, nodes].imag.copy()
    out["Cmax"] = np.float64(np.abs(res.C).max()) if res.C.size else np.float64(0)
    out["y_solve"] = y_solve
    out["u_solve"] = u_solve
    path = os.path.join(HERE, "wholejob_%s.npz" % name)
    np.savez_compressed(path, **out)
    print("%s: |I| = %d, samples = %d, lattices = %d, %.0f s -> %s"
          % (name, len(I), res.samples, lattices, time.time() - t0, path), flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["mesh16_d10", "mesh64_d10", "mesh128_d4", "mesh256_d4"]:
        make(nm)
