"""Stage parity at the workloads' full sizes, in the launch configuration of
the benchmark, on outputs the oracle can compute one by one (sampled solves,
sampled columns), plus the largest meshes of the streaming solver."""
import numpy as np
import pytest

import workloads as W
from oracle import dft as odft
from oracle import fem as ofem
from oracle import rng as orng
from oracle import select as osel
from oracle.usfft import tail as otail

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("name,prec,tol,check", [("mesh64_d10", 0, 1e-11, 4), ("mesh64_d10", 1, 1e-9, 4),
                                                 ("mesh128_d20", 0, 1e-11, 2), ("mesh128_d20", 1, 1e-9, 2)])
def test_first_detection_stage_full_size(lib, name, prec, tol, check):
    """Alg. 1 stage (t=1, i=1) at full size: nodes, solves, length-K DFT and
    selection through the ABI vs the oracle (solves sampled; DFT and selection
    on the oracle's own samples for sampled nodes)."""
    prob, par = W.WORKLOADS[name]
    d = prob["d"]
    K = prob["k_hi"][0] - prob["k_lo"][0] + 1
    plan = lib.Plan(prob, dict(par, precision=prec, pcg_rtol=1e-13 if prec == 0 else 1e-12))
    G = plan.G
    tail = otail(7, orng.KIND_TAIL1, 1, 1, d)
    y = torch.zeros((K, d), dtype=torch.float64, device="cuda")
    lib.nodes(d, 0, 1, [K], None, tail, y)
    Yo = np.tile(tail, (K, 1))
    Yo[:, 0] = np.arange(K) / K
    assert np.array_equal(host(y), Yo)
    ld = (K + 63) // 64 * 64
    U = torch.zeros((G, ld), dtype=torch.float64, device="cuda")
    it = torch.zeros(K, dtype=torch.int32, device="cuda")
    lib.sample(plan, y, U, 0, ld, 0, it)
    assert (host(it) > 0).all()
    S = ofem.PDESampler(prob["mesh_n"], prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    Ug = host(U)[:, :K]
    picks = np.linspace(0, K - 1, check).astype(int)
    for l in picks:
        ref = S.solve_one(Yo[l])
        assert np.linalg.norm(Ug[:, l] - ref) / np.linalg.norm(ref) <= tol
    ks = np.arange(prob["k_lo"][0], prob["k_hi"][0] + 1)
    V = torch.zeros((G, K), dtype=torch.float64, device="cuda")
    lib.line_dft(U, 0, G, ld, 0, K, ks, lib.OUT_MAG2, V, K)
    Vg = host(V)
    # the DFT stage on the GPU's samples vs the oracle's DFT of the same samples
    cols = np.linspace(0, G - 1, 9).astype(int)
    ref = np.abs(odft.dft_bins(Ug[cols].T, ks % K)) ** 2  # (K, ncols)
    assert np.abs(Vg[cols].T - ref).max() <= 1e-13 * ref.max()
    # selection on the GPU magnitudes vs the oracle's rule on the same values
    theta2 = np.array([par["theta"] ** 2 * Vg.max()])
    mask = torch.zeros((K + 31) // 32 + 1, dtype=torch.int32, device="cuda")
    thr = torch.zeros(G, dtype=torch.float64, device="cuda")
    lib.select(V, G, K, K, par["s_local"], dev(theta2), osel.TIE_REL, mask, thr)
    m_ref, thr_ref, _ = osel.detect_mask(Vg.T, par["s_local"], theta2[0])
    m = host(mask).view(np.uint32)
    bits = np.array([(m[a >> 5] >> (a & 31)) & 1 for a in range(K)], dtype=bool)
    assert np.array_equal(bits, m_ref)
    assert np.array_equal(host(thr), thr_ref)


@pytest.mark.parametrize("prec", [0, 1])
def test_solver_in_the_benchmark_launch_configuration(lib, prec):
    """h = 1/64, d = 10, 20 000 samples in one launch with the sample layout
    of a job (float32 samples on the float32 path), as in the benchmark's
    step-2 launches: every persistent workgroup solves many samples in turn,
    reusing its LDS tables, zero rings and scratch slot.  Sampled solves from
    the first and later rounds of the persistent loop against the oracle, and
    bitwise against the same parameter solved alone."""
    prob, par = W.WORKLOADS["mesh64_d10"]
    plan = lib.Plan(prob, dict(par, precision=prec, pcg_rtol=1e-12))
    ns = 20000
    fp32 = prec == 1
    Y = np.random.default_rng(5).random((ns, prob["d"]))
    U = torch.zeros((plan.G, ns), dtype=torch.float32 if fp32 else torch.float64, device="cuda")
    it = torch.zeros(ns, dtype=torch.int32, device="cuda")
    lib.sample(plan, dev(Y), U, 1 if fp32 else 0, ns, 0, it)
    its = host(it)
    assert (its > 0).all() and its.max() <= 30, (its.min(), its.max())
    Ug = host(U)
    S = ofem.PDESampler(prob["mesh_n"], prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    for s in (0, 255, 256, 511, 512, 7777, ns - 1):
        U1 = torch.zeros((plan.G, 1), dtype=torch.float64, device="cuda")
        lib.sample(plan, dev(Y[s:s + 1]), U1, 0, 1)
        u1 = host(U1)[:, 0]
        assert np.array_equal(Ug[:, s], u1.astype(np.float32) if fp32 else u1), s
        ref = S.solve_one(Y[s])
        # the float64 contract (nodal 1e-11) at the benchmark's pcg_rtol
        assert np.linalg.norm(u1 - ref) <= (1e-11 if prec == 0 else 1e-9) * np.linalg.norm(ref), s


@pytest.mark.parametrize("G,M,fp32", [(3969, 9601, 0), (3969, 9601, 1), (16129, 4801, 1), (16129, 9601, 0),
                                      (3969, 18523, 1), (16129, 18523, 1)])
def test_lattice_dft_full_size(lib, G, M, fp32):
    """Lattice DFT at the full node counts and the largest lattice size; the
    oracle checks sampled nodes (all requested bins)."""
    g = np.random.default_rng(G + M)
    Uf = (0.05 + 1e-3 * g.standard_normal((G, M))).astype(np.float32 if fp32 else np.float64)
    nb = min(2000, M)
    bins = np.sort(g.choice(M, size=nb, replace=False)).astype(np.int32)
    pos = np.arange(nb, dtype=np.int32)
    V = torch.zeros((G, nb), dtype=torch.float64, device="cuda")
    lib.lattice_dft(dev(Uf), fp32, G, M, 0, M, dev(bins), dev(pos), lib.OUT_MAG2, V, nb)
    Vg = host(V)
    cols = np.concatenate([np.arange(3), g.choice(G, 5, replace=False), [G - 1]])
    ref = np.abs(odft.dft_bins(Uf[cols].astype(np.float64).T, bins)) ** 2
    # tolerances are relative to the node's largest coefficient (here the mean,
    # bin 0): |X|^2 errors are then bounded by 3 tol Xmax^2
    xmax = max(np.abs(Uf[cols].astype(np.float64).mean(axis=1)).max(), np.sqrt(ref.max()))
    tol = 1e-6 if fp32 else 1e-12
    assert np.abs(Vg[cols].T - ref).max() <= 3 * tol * xmax ** 2


@pytest.mark.parametrize("n,d,ns,precond", [(96, 10, 6, 0), (128, 20, 5, 0), (66, 6, 4, 0), (129, 8, 4, 0),
                                            (96, 10, 6, 1), (128, 20, 3, 1), (130, 8, 3, 0), (200, 12, 3, 0),
                                            (256, 20, 3, 0), (256, 12, 2, 1), (255, 6, 2, 0)])
def test_streaming_solver_large_meshes(lib, n, d, ns, precond):
    # meshes beyond one CU: 65 < n <= 129 with the fast-Poisson preconditioner
    # (CG vectors in a global workspace, float64; n = 66 and 129 are the ends
    # of its range, 129 fills the 128-point transform); even 129 < n <= 256
    # with the two-level preconditioner (its coarse transform at n / 2: 130
    # and 256 are the ends of its range); Jacobi on request and for odd n
    # above 129
    prob = W.pde_problem(n, d, 8)
    plan = lib.Plan(prob, dict(W.params(10, 1, 1e-4), pcg_rtol=1e-13, pcg_maxit=8000, precond=precond))
    Y = np.random.default_rng(n + d).random((ns, d))
    U = torch.zeros((plan.G, ns + 1), dtype=torch.float64, device="cuda")
    it = torch.zeros(ns, dtype=torch.int32, device="cuda")
    lib.sample(plan, dev(Y), U, 0, ns + 1, 1, it)
    its = host(it)
    assert (its > 0).all()
    print("n %d d %d precond %d: iterations %s" % (n, d, precond, its.tolist()), flush=True)
    if precond == 0 and (n <= 129 or n % 2 == 0):
        assert its.max() <= 40, its
    Ug = host(U)
    S = ofem.PDESampler(n, prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    for s in range(0, ns, max(1, ns // 2)):
        ref = S.solve_one(Y[s])
        assert np.linalg.norm(Ug[:, 1 + s] - ref) / np.linalg.norm(ref) <= 1e-11
    # a sample's result does not depend on its batch
    U1 = torch.zeros((plan.G, 1), dtype=torch.float64, device="cuda")
    lib.sample(plan, dev(Y[ns - 1:ns]), U1, 0, 1)
    assert np.array_equal(host(U1)[:, 0], Ug[:, ns])


def test_errors_full_size_chunks_and_epilogue(lib):
    # h = 1/64, d = 10 job (float32 + refinement): 40 000 test points take two
    # chunks; err_p^p and err_inf of the whole set combine those of its parts,
    # and on 300 points the fused error epilogue agrees with the values of
    # usfft_eval and usfft_sample (periodic model: parameters are nodes)
    prob, par = W.WORKLOADS["mesh64_d10"]
    plan = lib.Plan(prob, dict(par, precision=1))
    res = lib.detect(plan, 1)
    G, d = res.G, prob["d"]
    Y = np.random.default_rng(23).random((40000, d))

    def errs(y, p=2.0):
        ep = torch.zeros(G, dtype=torch.float64, device="cuda")
        ei = torch.zeros(G, dtype=torch.float64, device="cuda")
        lib.errors(plan, res, dev(y), p, ep, ei)
        return host(ep), host(ei)

    ea, ia = errs(Y)
    e1, i1 = errs(Y[:30000])
    e2, i2 = errs(Y[30000:])
    assert np.allclose(ea ** 2, (30000 * e1 ** 2 + 10000 * e2 ** 2) / 40000, rtol=1e-10, atol=0)
    assert np.array_equal(ia, np.maximum(i1, i2))
    y = Y[:300]
    U = torch.zeros((G, 300), dtype=torch.float64, device="cuda")
    lib.sample(plan, dev(y), U, 0, 300)
    V = torch.zeros((300, G), dtype=torch.float64, device="cuda")
    lib.eval(res, dev(y), V)
    D = np.abs(host(U).T - host(V))
    for p in (2.0, 3.0):
        ep, ei = errs(y, p)
        assert np.allclose(ep, np.mean(D ** p, axis=0) ** (1 / p), rtol=1e-10, atol=0)
        assert np.array_equal(ei, D.max(axis=0))
