"""GPU parity: every stage of the HIP path, through the C ABI, against the oracle.

Integer work (nodes' lattice indices, masks, sets, families) must be
bit-exact; float64 results meet the stated tolerances (nodal rel-L2 <= 1e-11
for the float64 solver, <= 1e-9 after float32 + float64 refinement; DFT bins
<= 1e-12 of the column maximum in float64, <= 1e-6 in float32).
"""
import numpy as np
import pytest

import workloads as W
from oracle import dft as odft
from oracle import fem as ofem
from oracle import lattice as olat
from oracle import rng as orng
from oracle import select as osel
from oracle.usfft import TrigPolySampler, evaluate, usfft

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ------------------------------------------------------------------ nodes
def test_nodes_line_and_lattice_bit_exact(lib):
    d = 5
    tail = [orng.uniform01(3, orng.stream_code(1, 2, 1), j) for j in range(d)]
    y = torch.zeros((33, d), dtype=torch.float64, device="cuda")
    lib.nodes(d, 2, 1, [33], None, tail, y)
    ref = np.tile(tail, (33, 1))
    ref[:, 2] = np.arange(33) / 33
    assert np.array_equal(host(y), ref)
    Ms = [31, 61]
    zs = [[1, 7, 12], [5, 3, 44]]
    y = torch.zeros((sum(Ms), d), dtype=torch.float64, device="cuda")
    lib.nodes(d, -1, 3, Ms, zs, tail, y)
    ref = np.concatenate([np.hstack([olat.lattice_nodes(M, z), np.tile(tail[3:], (M, 1))]) for M, z in zip(Ms, zs)])
    assert np.array_equal(host(y), ref)


# ------------------------------------------------------------------ sampler
@pytest.mark.parametrize("precond,cfg", [(0, -2), (0, 0), (0, 1), (1, -2)],
                         ids=["dst", "dst_global_scratch", "dst_lds_resident", "jacobi"])
@pytest.mark.parametrize("n,d,modes,prec,tol", [
    (4, 2, "diagonal", 0, 1e-11), (8, 3, "diagonal", 0, 1e-11), (16, 4, "diagonal", 0, 1e-11),
    (33, 6, "split", 0, 1e-11), (34, 6, "split", 0, 1e-11), (64, 10, "split", 0, 1e-11),
    (65, 10, "split", 0, 1e-11), (16, 4, "diagonal", 1, 1e-9), (33, 6, "split", 1, 1e-9),
    (64, 10, "split", 1, 1e-9), (65, 10, "split", 1, 1e-9)])
def test_pde_solves_match_banded_cholesky(lib, n, d, modes, prec, tol, precond, cfg):
    # n = 33 and 65 fill the padded 32 / 64 transform exactly, n = 34 is the
    # first mesh padded to 64, n = 4 the smallest (Jacobi: n = 65 streams)
    prob = W.pde_problem(n, d, 4, modes=modes)
    plan = lib.Plan(prob, dict(W.params(10, 1, 1e-4), precision=prec, pcg_rtol=1e-13 if prec == 0 else 1e-12,
                               solver_config=cfg, precond=precond))
    g = np.random.default_rng(n * 10 + d + prec)
    ns = 37
    Y = g.random((ns, d))
    G = plan.G
    ld = 40
    U = torch.zeros((G, ld), dtype=torch.float64, device="cuda")
    it = torch.zeros(ns, dtype=torch.int32, device="cuda")
    lib.sample(plan, dev(Y), U, 0, ld, 2, it)
    Ug = host(U)[:, 2:2 + ns].T
    assert (host(it) > 0).all()
    S = ofem.PDESampler(n, prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    for s in range(0, ns, 6):
        ref = S.solve_one(Y[s])
        err = np.linalg.norm(Ug[s] - ref) / np.linalg.norm(ref)
        assert err <= tol, (s, err)


def test_solver_shapes_agree_and_batch_independent(lib):
    # every admissible workgroup shape gives the same float64 solution; a
    # sample's result does not depend on the batch it is solved in (bitwise)
    n, d = 16, 4
    prob = W.pde_problem(n, d, 4, modes="diagonal")
    Y = np.random.default_rng(5).random((20, d))
    outs = []
    for cfg in range(15):
        try:
            plan = lib.Plan(prob, dict(W.params(10, 1, 1e-4), pcg_rtol=1e-13, solver_config=cfg, precond=1))
        except lib.UsfftError:
            continue
        U = torch.zeros((plan.G, 20), dtype=torch.float64, device="cuda")
        lib.sample(plan, dev(Y), U, 0, 20)
        outs.append(host(U))
        U1 = torch.zeros((plan.G, 1), dtype=torch.float64, device="cuda")
        lib.sample(plan, dev(Y[7:8]), U1, 0, 1)
        assert np.array_equal(host(U1)[:, 0], outs[-1][:, 7])
    assert len(outs) >= 2
    for o in outs[1:]:
        assert np.abs(o - outs[0]).max() <= 1e-12 * np.abs(outs[0]).max()


@pytest.mark.parametrize("variant", [0, 1, 2], ids=["global_scratch", "lds_resident", "compact_fp32"])
@pytest.mark.parametrize("prec", [0, 1])
def test_dst_solver_batch_independent_and_fast(lib, prec, variant):
    # a sample's DST-PCG solution does not depend on the batch or workgroup
    # that solves it (bitwise), the fast-Poisson preconditioner keeps the
    # iteration count of the h = 1/64, d = 10 workload small, and every
    # scratch placement agrees with the direct solve (the compact one is
    # float32-only)
    prob, _ = W.WORKLOADS["mesh64_d10"]
    par = dict(W.params(10, 1, 1e-4), precision=prec, pcg_rtol=1e-12, solver_config=variant)
    if variant == 2 and prec == 0:
        with pytest.raises(lib.UsfftError):
            lib.Plan(prob, par)
        return
    plan = lib.Plan(prob, par)
    Y = np.random.default_rng(11).random((300, prob["d"]))
    U = torch.zeros((plan.G, 300), dtype=torch.float64, device="cuda")
    it = torch.zeros(300, dtype=torch.int32, device="cuda")
    lib.sample(plan, dev(Y), U, 0, 300, 0, it)
    its = host(it)
    assert (its > 0).all() and its.max() <= 30, (its.min(), its.max())
    S = ofem.PDESampler(64, prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    for s in (0, 123, 299):
        U1 = torch.zeros((plan.G, 1), dtype=torch.float64, device="cuda")
        lib.sample(plan, dev(Y[s:s + 1]), U1, 0, 1)
        assert np.array_equal(host(U1)[:, 0], host(U)[:, s])
        ref = S.solve_one(Y[s])
        # the float64 contract (nodal 1e-11) at the benchmark's pcg_rtol
        assert np.linalg.norm(host(U)[:, s] - ref) <= (1e-11 if prec == 0 else 1e-9) * np.linalg.norm(ref)


@pytest.mark.parametrize("model,n", [("pde", 5), ("pde", 16), ("pde", 17), ("pde", 33), ("pde", 34), ("pde", 48),
                                     ("pde", 64), ("pde", 65), ("lognormal", 33), ("lognormal", 65),
                                     ("affine", 40)])
def test_compact_solver_edge_meshes(lib, model, n):
    # the compact float32 solver rebuilds its float64 edge weights on the
    # matrix cores at every true residual, with the cells beyond the waves'
    # strips (column 16 (w + 1), row MP) kept from the assembly: meshes that
    # fill the padded transform exactly (n = 33, 65, where row and column MP
    # are interior), leave most of it empty (n = 5, 17, 34) or end inside a
    # strip (n = 40, 48) must all converge to the direct solve
    d = 6
    if model == "pde":
        prob = W.pde_problem(n, d, 4, modes="split")
    elif model == "affine":
        prob = W.affine_problem(n, d, 4)
    else:
        prob = W.lognormal_problem(n, d, 4, delta=0.01)
    plan = lib.Plan(prob, dict(W.params(10, 1, 1e-4), precision=1, pcg_rtol=1e-12, solver_config=2))
    T = np.random.default_rng(n + 7).random((30, d))
    U = torch.zeros((plan.G, 30), dtype=torch.float64, device="cuda")
    it = torch.zeros(30, dtype=torch.int32, device="cuda")
    lib.sample(plan, dev(T), U, 0, 30, 0, it)
    assert (host(it) > 0).all() and (model == "lognormal" or host(it).max() <= 40)
    S = oracle_sampler(prob)
    for s in range(0, 30, 5):
        ref = S.solve_one(T[s])
        err = np.linalg.norm(host(U)[:, s] - ref) / np.linalg.norm(ref)
        assert err <= 1e-9, (s, err)


@pytest.mark.parametrize("prec", [0, 1])
def test_dst_preconditioner_is_exact_for_constant_coefficient(lib, prec):
    # a = 1: the scaled operator is the 5-point Laplacian itself, which the
    # preconditioner inverts up to fp16 rounding, so a few iterations suffice
    # and the solution is the oracle's (the same for every y)
    n, d = 64, 3
    prob = dict(W.pde_problem(n, d, 4), amp=[0.0] * d)
    plan = lib.Plan(prob, dict(W.params(10, 1, 1e-4), precision=prec, pcg_rtol=1e-12))
    Y = np.random.default_rng(2).random((4, d))
    U = torch.zeros((plan.G, 4), dtype=torch.float64, device="cuda")
    it = torch.zeros(4, dtype=torch.int32, device="cuda")
    lib.sample(plan, dev(Y), U, 0, 4, 0, it)
    assert (host(it) > 0).all() and host(it).max() <= 6, host(it)
    ref = ofem.PDESampler(n, 1.0, [0.0] * d, prob["mode1"], prob["mode2"]).solve_one(Y[0])
    for s in range(4):
        assert np.linalg.norm(host(U)[:, s] - ref) <= (1e-11 if prec == 0 else 1e-10) * np.linalg.norm(ref)


@pytest.mark.parametrize("precond", [0, 1], ids=["dst", "jacobi"])
@pytest.mark.parametrize("model,n,prec,tol", [
    ("affine", 16, 0, 1e-11), ("affine", 64, 0, 1e-11), ("affine", 64, 1, 1e-9),
    ("lognormal", 16, 0, 1e-11), ("lognormal", 64, 0, 1e-11), ("lognormal", 64, 1, 1e-9)])
def test_model_solves_match_oracle(lib, model, n, prec, tol, precond):
    # affine and lognormal coefficients through their periodizations (Sec.
    # 3.2): the sampler maps the nodes t to the parameters and solves
    d = 6
    prob = W.affine_problem(n, d, 4) if model == "affine" else W.lognormal_problem(n, d, 4, delta=0.01)
    plan = lib.Plan(prob, dict(W.params(10, 1, 1e-4), precision=prec, precond=precond,
                               pcg_rtol=1e-13 if prec == 0 else 1e-12))
    T = np.random.default_rng(n + prec).random((25, d))
    T[0] = 0.25 + (0.01 if model == "lognormal" else 0.0)  # parameter y = 0
    U = torch.zeros((plan.G, 25), dtype=torch.float64, device="cuda")
    it = torch.zeros(25, dtype=torch.int32, device="cuda")
    lib.sample(plan, dev(T), U, 0, 25, 0, it)
    assert (host(it) > 0).all()
    S = oracle_sampler(prob)
    for s in range(0, 25, 4):
        ref = S.solve_one(T[s])
        err = np.linalg.norm(host(U)[:, s] - ref) / np.linalg.norm(ref)
        assert err <= tol, (s, err)


@pytest.mark.parametrize("model", ["affine", "lognormal"])
def test_detect_models_cpu_scale(lib, model):
    # whole job with the periodized affine / lognormal coefficient: the same
    # sets as the oracle, coefficients to 1e-10 of the largest; evaluation at
    # parameters y uses the inverse periodization
    from oracle import periodization as OP
    n, d, N = 16, 4, 8
    delta = OP.delta_opt(9601)
    prob = W.affine_problem(n, d, N) if model == "affine" else W.lognormal_problem(n, d, N)
    par = W.params(30, 2, 1e-4)
    res, ref = run_both(lib, prob, par, 5, sampler=oracle_sampler(prob, delta=delta))
    assert res.freqs().tolist() == ref.I.tolist()
    C = res.coeffs()
    assert np.abs(C - ref.C).max() <= 1e-10 * np.abs(ref.C).max()
    g = np.random.default_rng(9)
    Yp = g.uniform(-1.0, 1.0, (7, d)) if model == "affine" else g.standard_normal((7, d))
    out = torch.zeros((7, res.G), dtype=torch.float64, device="cuda")
    lib.eval(res, dev(Yp), out)
    mid = OP.to_node(prob["model"], Yp, prob.get("alpha", -1.0), prob.get("beta", 1.0), delta)
    want = evaluate(ref.I, ref.C, mid)
    assert np.abs(host(out) - want).max() <= 1e-9 * np.abs(want).max()


def test_model_parameters_are_checked(lib):
    prob = W.affine_problem(16, 4, 8)
    par = W.params(10, 1, 1e-4)
    for bad in (dict(model=3), dict(alpha=1.0, beta=1.0), dict(basis1=2)):
        with pytest.raises(lib.UsfftError) as e:
            lib.Plan(dict(prob, **bad), par)
        assert e.value.status == lib.EINVAL
    with pytest.raises(lib.UsfftError):
        lib.Plan(W.lognormal_problem(16, 4, 8, delta=0.7), par)


def test_trig_poly_sampler(lib):
    K, P = W.trig_poly(4, 5, 8, 70, 31)
    prob = dict(sampler="poly", d=5, k_lo=[-8] * 5, k_hi=[8] * 5, poly_k=K, poly_c=P)
    plan = lib.Plan(prob, W.params(10, 1, 1e-6, relative=False))
    Y = np.random.default_rng(1).random((19, 5))
    U = torch.zeros((70, 19), dtype=torch.float64, device="cuda")
    lib.sample(plan, dev(Y), U, 0, 19)
    ref = TrigPolySampler(K, P)(Y)
    assert np.abs(host(U).T - ref).max() <= 1e-12 * np.abs(ref).max()


# ------------------------------------------------------------------ DFTs
@pytest.mark.parametrize("K,G", [(33, 5), (65, 130), (16, 3), (1, 4)])
def test_line_dft(lib, K, G):
    U = W.sample_matrix(K + G, K, G, kind="normal")  # (K, G)
    ld = K + 3
    Ud = np.zeros((G, ld))
    Ud[:, 1:1 + K] = U.T
    ks = np.arange(-(K // 2), K - K // 2)
    Vt = torch.zeros((G, K), dtype=torch.float64, device="cuda")
    lib.line_dft(dev(Ud), 0, G, ld, 1, K, ks, lib.OUT_MAG2, Vt, K)
    ref = odft.dft_bins(U, ks % K)
    scale = np.abs(ref).max() ** 2
    assert np.abs(host(Vt) - (np.abs(ref) ** 2).T).max() <= 1e-13 * scale
    Ct = torch.zeros((K, G, 2), dtype=torch.float64, device="cuda")
    lib.line_dft(dev(Ud), 0, G, ld, 1, K, ks, lib.OUT_COMPLEX, Ct, 0)
    c = host(Ct)
    assert np.abs(c[..., 0] + 1j * c[..., 1] - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("M,G,fp32", [(3, 4, 0), (11, 7, 0), (31, 64, 0), (97, 33, 0), (1153, 9, 0),
                                      (4801, 5, 0), (9601, 3, 0), (9601, 6, 1), (211, 129, 1), (12289, 5, 1),
                                      (18523, 3, 1)])
def test_lattice_dft_rader(lib, M, G, fp32):
    assert olat.admissible(M)
    U = W.sample_matrix(M + G, M, G, kind="normal")
    g = np.random.default_rng(M)
    bins = np.arange(M) if M <= 211 else np.sort(g.choice(M, size=min(M, 700), replace=False))
    pos = g.permutation(len(bins))
    ld = M + 5
    Ud = np.zeros((G, ld))
    Ud[:, 2:2 + M] = U.T
    ut = dev(Ud, torch.float32 if fp32 else torch.float64)
    nb = len(bins)
    V = torch.zeros((G, nb), dtype=torch.float64, device="cuda")
    lib.lattice_dft(ut, fp32, G, ld, 2, M, dev(bins, torch.int32), dev(pos, torch.int32), lib.OUT_MAG2, V, nb)
    C = torch.zeros((nb, G, 2), dtype=torch.float64, device="cuda")
    lib.lattice_dft(ut, fp32, G, ld, 2, M, dev(bins, torch.int32), dev(pos, torch.int32), lib.OUT_COMPLEX, C, G)
    ref = odft.dft_bins(U.astype(np.float32).astype(np.float64) if fp32 else U, bins)  # (nb, G)
    tol = 1e-6 if fp32 else 1e-12
    cmax = np.abs(ref).max()
    got = host(C)
    got = got[..., 0] + 1j * got[..., 1]
    assert np.abs(got[pos] - ref).max() <= tol * cmax
    assert np.abs(host(V)[:, pos] - (np.abs(ref) ** 2).T).max() <= 2 * tol * cmax ** 2
    # bins b and M-b are exact conjugates (canonical half spectrum)
    if M <= 211:
        inv = np.empty(nb, int)
        inv[pos] = np.arange(nb)
        for b in range(1, M):
            assert np.array_equal(got[pos[b]], np.conj(got[pos[M - b]]))


def test_lattice_sizes_by_precision(lib):
    """Float32 samples take lattice sizes up to 19201 (one node pair's
    float32 transform in one CU's LDS), float64 samples up to 9601."""
    M, G = 18523, 2
    ut = torch.zeros((G, M), dtype=torch.float64, device="cuda")
    b = torch.zeros(1, dtype=torch.int32, device="cuda")
    V = torch.zeros((G, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.UsfftError) as e:
        lib.lattice_dft(ut, 0, G, M, 0, M, b, b, lib.OUT_MAG2, V, 1)
    assert e.value.status == lib.EINVAL
    prob = W.pde_problem(8, 2, 4)
    with pytest.raises(lib.UsfftError) as e:
        lib.Plan(prob, dict(W.params(4, 1, 1e-4), precision=lib.FP64, lattice_mmax=19201))
    assert e.value.status == lib.EINVAL
    lib.Plan(prob, dict(W.params(4, 1, 1e-4), precision=lib.FP32_REFINE, lattice_mmax=19201)).close()


# ------------------------------------------------------------------ select
@pytest.mark.parametrize("n,G,s", [(5, 3, 2), (100, 17, 10), (4500, 40, 200), (65, 9, 200), (1, 2, 1),
                                   (2000, 13, 200), (512, 5, 512), (1024, 7, 3)])
def test_select_bit_exact(lib, n, G, s):
    g = np.random.default_rng(n + G)
    V = g.exponential(1.0, (n, G)) ** 4
    V[g.random((n, G)) < 0.1] = 0.0
    if n > 3:
        V[1] = V[0]  # exact ties
        V[2] = V[0] * (1 - 1e-12)  # ties within the band
    theta2 = 1e-3
    mask_ref, thr_ref, _ = osel.detect_mask(V, s, theta2)
    ld = n + 7
    Vd = np.zeros((G, ld))
    Vd[:, :n] = V.T
    words = (n + 31) // 32 + 1
    mask = torch.zeros(words, dtype=torch.int32, device="cuda")
    thr = torch.zeros(G, dtype=torch.float64, device="cuda")
    lib.select(dev(Vd), G, n, ld, s, dev(np.array([theta2])), osel.TIE_REL, mask, thr)
    m = host(mask).view(np.uint32)
    bits = np.array([(m[a >> 5] >> (a & 31)) & 1 for a in range(n)], dtype=bool)
    assert np.array_equal(bits, mask_ref)
    assert np.array_equal(host(thr), thr_ref)


@pytest.mark.parametrize("kind,n,G,s", [("low_bits", 4500, 12, 200), ("mid_bits", 4500, 7, 200),
                                         ("duplicates", 100, 9, 30), ("duplicates", 3000, 5, 200),
                                         ("one_binade", 700, 6, 64),
                                         # more column lengths of the LDS-staged path
                                         ("low_bits", 512, 9, 100), ("mid_bits", 513, 9, 100),
                                         ("duplicates", 1024, 5, 200), ("one_binade", 1025, 6, 64),
                                         ("low_bits", 2048, 5, 200), ("mid_bits", 2049, 5, 200),
                                         # columns longer than the LDS stage: keys read from global memory
                                         ("mid_bits", 9000, 4, 200), ("duplicates", 12000, 3, 500),
                                         ("one_binade", 8193, 3, 100)])
def test_select_bit_exact_hard_keys(lib, kind, n, G, s):
    # keys that agree in their leading bytes (the radix passes run long, the
    # small-set finish starts late or never) and many equal keys (the rank
    # with multiplicity)
    g = np.random.default_rng(len(kind) + n + G)
    if kind == "low_bits":  # steps below the tie band
        V = 1.0 + g.integers(0, 300, (n, G)) * 2.0 ** -44
    elif kind == "mid_bits":  # steps above it, keys agree in their top three bytes
        V = 1.0 + g.integers(0, 300, (n, G)) * 2.0 ** -28
    elif kind == "duplicates":
        V = g.integers(1, 5, (n, G)).astype(np.float64)
    else:
        V = 1.0 + g.random((n, G))
    theta2 = 1e-3
    mask_ref, thr_ref, _ = osel.detect_mask(V, s, theta2)
    ld = n + 3
    Vd = np.zeros((G, ld))
    Vd[:, :n] = V.T
    mask = torch.zeros((n + 31) // 32 + 1, dtype=torch.int32, device="cuda")
    thr = torch.zeros(G, dtype=torch.float64, device="cuda")
    lib.select(dev(Vd), G, n, ld, s, dev(np.array([theta2])), osel.TIE_REL, mask, thr)
    m = host(mask).view(np.uint32)
    bits = np.array([(m[a >> 5] >> (a & 31)) & 1 for a in range(n)], dtype=bool)
    assert np.array_equal(bits, mask_ref)
    assert np.array_equal(host(thr), thr_ref)


@pytest.mark.parametrize("n,G,s", [(300, 64, 20), (1155, 48, 200), (9000, 6, 200)])
def test_select_bit_exact_near_theta(lib, n, G, s):
    # columns whose count of keys at or above theta^2 runs from well below s~
    # to well above it, with keys exactly at theta^2, inside the tie band just
    # above it and just below it: thresholds at theta^2 and at (1 - tie) tau^2
    # both occur, and at the switch between them
    g = np.random.default_rng(n * 7 + G)
    theta2 = 1.0
    V = g.random((n, G)) * 0.5
    for c in range(G):
        k = (c * (2 * s + 4)) // G  # keys placed at or above theta^2
        rows = g.permutation(n)[:min(k, n)]
        V[rows, c] = theta2 * (1.0 + g.random(len(rows)))
        if len(rows) > 3:
            V[rows[0], c] = theta2  # exactly theta^2
            V[rows[1], c] = theta2 * (1 + 2.0 ** -33)  # inside the tie band
            V[rows[2], c] = np.nextafter(theta2, 0.0)  # just below
    mask_ref, thr_ref, _ = osel.detect_mask(V, s, theta2)
    ld = n + 5
    Vd = np.zeros((G, ld))
    Vd[:, :n] = V.T
    mask = torch.zeros((n + 31) // 32 + 1, dtype=torch.int32, device="cuda")
    thr = torch.zeros(G, dtype=torch.float64, device="cuda")
    lib.select(dev(Vd), G, n, ld, s, dev(np.array([theta2])), osel.TIE_REL, mask, thr)
    m = host(mask).view(np.uint32)
    bits = np.array([(m[a >> 5] >> (a & 31)) & 1 for a in range(n)], dtype=bool)
    assert np.array_equal(bits, mask_ref)
    assert np.array_equal(host(thr), thr_ref)
    assert (thr_ref == theta2).any() and (thr_ref > theta2).any()


# ------------------------------------------------------------------ sets
def test_product_and_compact_bit_exact(lib):
    parent, child = W.candidate_set(2, 60, 4, 9)
    J = osel.product(parent, child)
    out = torch.zeros(J.shape, dtype=torch.int32, device="cuda")
    lib.product(dev(parent, torch.int32), len(parent), 3, dev(child, torch.int32), len(child), out)
    assert np.array_equal(host(out), J)
    keep = np.random.default_rng(0).random(len(J)) < 0.3
    words = np.zeros((len(J) + 31) // 32, dtype=np.uint32)
    for a in np.nonzero(keep)[0]:
        words[a >> 5] |= np.uint32(1 << (a & 31))
    res = torch.zeros(J.shape, dtype=torch.int32, device="cuda")
    cnt = lib.compact(dev(J, torch.int32), dev(words.view(np.int32)), len(J), 4, res)
    assert cnt == keep.sum()
    assert np.array_equal(host(res)[:cnt], J[keep])


@pytest.mark.parametrize("seed,npar,t,nch,kind", [(1, 60, 3, 9, 3), (2, 300, 6, 9, 3), (3, 9, 2, 33, 4),
                                                  (4, 1, 2, 1, 3), (5, 1500, 9, 9, 3)])
def test_family_bit_exact(lib, seed, npar, t, nch, kind):
    parent, child = W.candidate_set(seed, npar, t, nch)
    J = osel.product(parent, child)
    n = len(J)
    ref = olat.plan_family(J, 2.0, 9601, 8, 64, seed, kind, t)
    assign = torch.zeros(n, dtype=torch.int32, device="cuda")
    bins = torch.zeros(n, dtype=torch.int32, device="cuda")
    Ms, zs = lib.family(dev(J, torch.int32), n, t, 2.0, 9601, 8, 64, seed, kind, t, assign, bins)
    assert Ms == ref.M
    assert zs == ref.z
    assert np.array_equal(host(assign), ref.assign)
    assert np.array_equal(host(bins), ref.bins)


# ------------------------------------------------------------------ whole path
def oracle_sampler(prob, delta=None):
    """The oracle's sampler for a PDE problem dict, with the same model,
    basis and lognormal shift as the plan."""
    return ofem.PDESampler(prob["mesh_n"], prob["a0"], prob["amp"], prob["mode1"], prob["mode2"],
                           model=prob.get("model", 0), alpha=prob.get("alpha", -1.0), beta=prob.get("beta", 1.0),
                           delta=delta if delta is not None else prob.get("delta", 0.0),
                           basis=(prob.get("basis1", 0), prob.get("basis2", 0)))


def run_both(lib, prob, par, seed, precision=0, sampler=None, **kw):
    plan = lib.Plan(prob, dict(par, precision=precision, pcg_rtol=1e-13 if precision == 0 else 1e-12, **kw))
    res = lib.detect(plan, seed)
    res.plan = plan
    if sampler is None:
        sampler = oracle_sampler(prob)
    ref = usfft(sampler, prob["d"], prob["k_lo"], prob["k_hi"], par["s"], par["s_local"], par["r"], par["theta"],
                par["theta_relative"], seed, keep_values=True)
    return res, ref


@pytest.mark.parametrize("seed,d,N,G,nf", [(1, 3, 8, 5, 21), (2, 6, 16, 33, 61), (3, 10, 32, 129, 81)])
def test_detect_trig_poly_exact_recovery(lib, seed, d, N, G, nf):
    K, P = W.trig_poly(seed, d, N, G, nf, cmin=1e-2)
    prob = dict(sampler="poly", d=d, k_lo=[-N] * d, k_hi=[N] * d, poly_k=K, poly_c=P)
    par = W.params(2 * nf, 4, 1e-6, relative=False)
    res, ref = run_both(lib, prob, par, seed, sampler=TrigPolySampler(K, P))
    I = res.freqs()
    assert I.tolist() == ref.I.tolist()
    support = {tuple(k) for k, row in zip(K.tolist(), P) if np.abs(row).max() > 0}
    assert {tuple(k) for k in I.tolist()} == support
    idx = {tuple(k): a for a, k in enumerate(K.tolist())}
    C = res.coeffs()
    for a, k in enumerate(I.tolist()):
        assert np.abs(C[a] - P[idx[tuple(k)]]).max() <= 1e-12
    assert res.stats["samples"] == ref.samples


def test_detect_trig_poly_uneven_box(lib):
    # a different K_t per coordinate (odd and even, asymmetric boxes): the
    # step-1 lines of all coordinates share one DFT and one selection launch
    K, P = W.trig_poly(4, 4, 4, 17, 31, cmin=1e-2)
    prob = dict(sampler="poly", d=4, k_lo=[-4, -6, -5, -9], k_hi=[4, 7, 5, 9], poly_k=K, poly_c=P)
    par = W.params(62, 4, 1e-6, relative=False)
    res, ref = run_both(lib, prob, par, 4, sampler=TrigPolySampler(K, P))
    I = res.freqs()
    assert I.tolist() == ref.I.tolist()
    support = {tuple(k) for k, row in zip(K.tolist(), P) if np.abs(row).max() > 0}
    assert {tuple(k) for k in I.tolist()} == support
    idx = {tuple(k): a for a, k in enumerate(K.tolist())}
    C = res.coeffs()
    for a, k in enumerate(I.tolist()):
        assert np.abs(C[a] - P[idx[tuple(k)]]).max() <= 1e-12
    assert res.stats["samples"] == ref.samples


def test_detect_pde_cpu_scale_fp64(lib):
    prob, par = W.WORKLOADS["cpu16_d4"]
    res, ref = run_both(lib, prob, par, 7)
    assert res.freqs().tolist() == ref.I.tolist()
    C = res.coeffs()
    assert np.abs(C - ref.C).max() <= 1e-10 * np.abs(ref.C).max()
    assert res.stats["samples"] == ref.samples
    assert abs(res.stats["theta_abs"] ** 2 - ref.theta2) <= 1e-12 * ref.theta2


def set_flips(I_gpu, I_ref):
    """Frequencies that are in one of the two detected sets only."""
    a = {tuple(k) for k in I_gpu}
    b = {tuple(k) for k in I_ref}
    return sorted(a ^ b)


def test_detect_pde_cpu_scale_fp32_refine(lib):
    prob, par = W.WORKLOADS["cpu16_d4"]
    res, ref = run_both(lib, prob, par, 7, precision=1)
    I = res.freqs().tolist()
    diff = set_flips(I, ref.I.tolist())
    assert not diff, diff
    C = res.coeffs()
    assert np.abs(C - ref.C).max() <= 1e-6 * np.abs(ref.C).max()


def full_grid_coefficients(S, d, P):
    """c_k(x_g) by the plain DFT of the oracle's solves on the full grid (j / P)^d."""
    ax = np.arange(P) / P
    grid = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), -1).reshape(-1, d)
    U = S(grid)
    return np.fft.fftn(U.reshape((P,) * d + (S.G,)), axes=tuple(range(d))) / P ** d


@pytest.mark.parametrize("precision", [0, 1])
def test_detect_pde_against_full_grid_fourier_coefficients(lib, precision):
    # the HIP path's run against the coefficients it approximates (d = 2; the
    # grid coefficients fall below 1e-11 at |k|_inf = 32): step-3 values
    # within the l1 norm T_g of the coefficients outside I, kept frequencies
    # at least theta - T_g, every frequency above 10 theta detected; float32
    # samples add their rounding (the 1e-6 coefficient tolerance)
    d, N, P = 2, 12, 64
    prob = W.pde_problem(8, d, N)
    par = W.params(100, 3, 1e-5)
    plan = lib.Plan(prob, dict(par, precision=precision, pcg_rtol=1e-13 if precision == 0 else 1e-12))
    res = lib.detect(plan, 5)
    F = full_grid_coefficients(oracle_sampler(prob), d, P)
    slack = 1e-10 if precision == 0 else 1e-6 * np.abs(F).max()
    I = [tuple(k) for k in res.freqs().tolist()]
    C = res.coeffs()
    cell = lambda k: tuple(v % P for v in k)
    outside = np.ones((P,) * d, dtype=bool)
    for k in I:
        outside[cell(k)] = False
    T = np.abs(F)[outside].sum(axis=0)
    th = res.stats["theta_abs"]
    for a, k in enumerate(I):
        ck = F[cell(k)]
        assert (np.abs(C[a] - ck) <= T + slack).all(), k
        assert (np.abs(ck) + T + slack).max() >= th, k
    big = {(a - N, b - N) for a in range(2 * N + 1) for b in range(2 * N + 1)
           if np.abs(F[cell((a - N, b - N))]).max() >= 10 * th}
    assert big <= set(I) and len(big) > 10


def test_detect_is_deterministic(lib):
    prob, par = W.WORKLOADS["cpu16_d4"]
    plan = lib.Plan(prob, dict(par, pcg_rtol=1e-13))
    r1 = lib.detect(plan, 3)
    r2 = lib.detect(plan, 3)
    assert np.array_equal(r1.freqs(), r2.freqs())
    assert np.array_equal(r1.coeffs(), r2.coeffs())


def test_eval_matches_oracle(lib):
    # 130 nodes (three node tiles, the last ragged) and 203 points (four
    # point tiles, the last ragged) against the oracle's own run
    K, P = W.trig_poly(8, 4, 8, 130, 25, cmin=1e-2)
    prob = dict(sampler="poly", d=4, k_lo=[-8] * 4, k_hi=[8] * 4, poly_k=K, poly_c=P)
    res, ref = run_both(lib, prob, W.params(60, 3, 1e-6, relative=False), 2, sampler=TrigPolySampler(K, P))
    assert res.freqs().tolist() == ref.I.tolist()
    Y = np.random.default_rng(3).random((203, 4))
    out = torch.zeros((203, 130), dtype=torch.float64, device="cuda")
    lib.eval(res, dev(Y), out)
    want = evaluate(ref.I, ref.C, Y)
    assert np.abs(host(out) - want).max() <= 1e-12 * np.abs(want).max()
    assert np.abs(host(out) - TrigPolySampler(K, P)(Y)).max() <= 1e-11
    lib.eval(res, dev(np.zeros((0, 4))), torch.zeros((0, 130), dtype=torch.float64, device="cuda"))


def test_eval_workspace_reused(lib):
    # repeated evaluations and statistics of one result: the set and the
    # workspaces stay with the result, so later calls of the same or smaller
    # size allocate no device memory, and each call's output equals the first
    # call's bit for bit (eq. (3.1); Sec. 4.1)
    K, P = W.trig_poly(8, 4, 8, 130, 25, cmin=1e-2)
    prob = dict(sampler="poly", d=4, k_lo=[-8] * 4, k_hi=[8] * 4, poly_k=K, poly_c=P)
    plan = lib.Plan(prob, dict(W.params(60, 3, 1e-6, relative=False), precision=lib.FP64, pcg_rtol=1e-13))
    res = lib.detect(plan, 2)
    Y = dev(np.random.default_rng(5).random((700, 4)))
    first = torch.zeros((700, 130), dtype=torch.float64, device="cuda")
    out = torch.zeros((700, 130), dtype=torch.float64, device="cuda")
    var0 = torch.zeros(130, dtype=torch.float64, device="cuda")
    var = torch.zeros(130, dtype=torch.float64, device="cuda")
    lib.eval(res, Y, first)
    lib.statistics(res, None, var0, None)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for n in (700, 311, 700):
        out.zero_()
        lib.eval(res, Y[:n], out[:n])
        lib.statistics(res, None, var, None)
        torch.cuda.synchronize()
        assert torch.equal(out[:n], first[:n]), n
        assert torch.equal(var, var0)
    assert torch.cuda.mem_get_info()[0] == free0


def _model_case(model):
    from oracle import periodization as OP
    delta = OP.delta_opt(9601)
    if model == "periodic":
        prob, par = W.WORKLOADS["cpu16_d4"]
        return prob, par, oracle_sampler(prob), OP.PERIODIC, 0.0
    prob = W.affine_problem(16, 4, 8) if model == "affine" else W.lognormal_problem(16, 4, 8)
    code = OP.AFFINE if model == "affine" else OP.LOGNORMAL
    return prob, W.params(30, 2, 1e-4), oracle_sampler(prob, delta=delta), code, delta


@pytest.mark.parametrize("model", ["periodic", "affine", "lognormal"])
def test_statistics_match_oracle(lib, model):
    # expectation with the model's D factors, variance and sensitivity
    # indices (Sec. 4, 4.1) of the GPU result against the oracle's own run
    from oracle import evaluation as oev
    prob, par, sampler, code, delta = _model_case(model)
    res, ref = run_both(lib, prob, par, 5, sampler=sampler)
    assert res.freqs().tolist() == ref.I.tolist()
    G, d = res.G, prob["d"]
    mean = torch.zeros((G, 2), dtype=torch.float64, device="cuda")
    var = torch.zeros(G, dtype=torch.float64, device="cuda")
    gsi = torch.zeros((d, G), dtype=torch.float64, device="cuda")
    lib.statistics(res, mean, var, gsi)
    scale = np.abs(ref.C).max()
    m_ref = oev.expectation(ref.I, ref.C, code, delta)
    assert np.abs(host(mean)[:, 0] - m_ref.real).max() <= 1e-9 * scale
    assert np.abs(host(mean)[:, 1] - m_ref.imag).max() <= 1e-9 * scale
    v_ref = oev.variance(ref.I, ref.C)
    assert np.abs(host(var) - v_ref).max() <= 1e-9 * v_ref.max()
    g_ref = oev.sensitivity_indices(ref.I, ref.C)
    live = v_ref > 1e-6 * v_ref.max()
    assert np.abs(host(gsi)[:, live] - g_ref[:, live]).max() <= 1e-6
    assert np.allclose(host(gsi)[:, live].sum(axis=0), 1.0, rtol=0, atol=1e-12)
    # any output may be left out
    var2 = torch.zeros(G, dtype=torch.float64, device="cuda")
    lib.statistics(res, None, var2, None)
    assert np.array_equal(host(var2), host(var))


@pytest.mark.parametrize("model", ["periodic", "affine", "lognormal"])
def test_errors_match_oracle(lib, model):
    # err_p / err_inf of Sec. 4: FE solves at the test parameters themselves
    # and the approximation at the same parameters, against the oracle's
    # banded-Cholesky solves and its own coefficients
    from oracle import evaluation as oev
    prob, par, sampler, code, delta = _model_case(model)
    res, ref = run_both(lib, prob, par, 5, sampler=sampler)
    assert res.freqs().tolist() == ref.I.tolist()
    g = np.random.default_rng(17)
    n, d = 150, prob["d"]
    alpha, beta = prob.get("alpha", -1.0), prob.get("beta", 1.0)
    Y = {"periodic": lambda: g.random((n, d)), "affine": lambda: g.uniform(alpha, beta, (n, d)),
         "lognormal": lambda: g.standard_normal((n, d))}[model]()
    U_fe = np.array([sampler.solve_param(y) for y in Y])
    U_ap = oev.approximation(ref.I, ref.C, Y, code, alpha, beta, delta)
    for p in (2.0, 1.0, 1.5):
        ep = torch.zeros(res.G, dtype=torch.float64, device="cuda")
        ei = torch.zeros(res.G, dtype=torch.float64, device="cuda")
        lib.errors(res.plan, res, dev(Y), p, ep, ei)
        ep_ref, ei_ref = oev.errors(U_fe, U_ap, p)
        tol = 1e-9 * np.abs(U_fe).max()
        assert np.all(np.abs(host(ep) - ep_ref) <= tol + 1e-6 * ep_ref), (p, np.abs(host(ep) - ep_ref).max())
        assert np.all(np.abs(host(ei) - ei_ref) <= tol + 1e-6 * ei_ref), p
        assert np.all(host(ei) >= host(ep) * (1 - 1e-12))


def test_errors_arguments_are_checked(lib):
    prob, par = W.WORKLOADS["cpu16_d4"]
    plan = lib.Plan(prob, par)
    res = lib.detect(plan, 1)
    ep = torch.zeros(res.G, dtype=torch.float64, device="cuda")
    Y = dev(np.random.default_rng(0).random((5, prob["d"])))
    for bad in (0.5, float("inf")):
        with pytest.raises(lib.UsfftError) as e:
            lib.errors(plan, res, Y, bad, ep, ep.clone())
        assert e.value.status == lib.EINVAL
    other = lib.Plan(W.pde_problem(8, prob["d"], 4), par)
    with pytest.raises(lib.UsfftError) as e:
        lib.errors(other, res, Y, 2.0, ep, ep.clone())
    assert e.value.status == lib.EINVAL


def test_coefficients_on_a_given_set_trig_poly(lib):
    # step 3 alone on a shuffled superset of the support (Sec. 4.5): the
    # caller's order is kept, the polynomial is recovered exactly, and the
    # values equal the oracle's step 3 on the same set and seed
    from oracle.usfft import coefficients
    d, N = 4, 8
    K, P = W.trig_poly(11, d, N, 70, 31, cmin=1e-2)
    prob = dict(sampler="poly", d=d, k_lo=[-N] * d, k_hi=[N] * d, poly_k=K, poly_c=P)
    plan = lib.Plan(prob, W.params(10, 1, 1e-6, relative=False))
    I = np.unique(np.vstack([K, W.hyperbolic_cross(d, N, [4] * d)]), axis=0)
    I = I[np.random.default_rng(2).permutation(len(I))]
    res = lib.coefficients(plan, I, 5)
    assert res.freqs().tolist() == I.tolist()
    C_ref, fam, ns = coefficients(TrigPolySampler(K, P), I, 5)
    C = res.coeffs()
    assert np.abs(C - C_ref).max() <= 1e-12 * np.abs(C_ref).max()
    idx = {tuple(k): a for a, k in enumerate(K.tolist())}
    want = np.array([P[idx[tuple(k)]] if tuple(k) in idx else np.zeros(70) for k in I.tolist()])
    assert np.abs(C - want).max() <= 1e-12
    assert res.stats["samples"] == ns and res.stats["lattices"] == len(fam.M)
    assert lib.coefficients(plan, np.zeros((0, d), dtype=np.int32), 5).n == 0
    with pytest.raises(lib.UsfftError) as e:
        lib.coefficients(plan, np.vstack([I, I[:1]]), 5)
    assert e.value.status == lib.EINVAL


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-6)])
def test_coefficients_on_a_hyperbolic_cross_pde(lib, prec, tol):
    # the PDE sampler on the uniform-weight hyperbolic cross of Sec. 4.5,
    # against the oracle's step 3 with banded-Cholesky solves
    from oracle.usfft import coefficients
    prob, par = W.WORKLOADS["cpu16_d4"]
    I = W.hyperbolic_cross(prob["d"], 16, [4] * prob["d"])
    plan = lib.Plan(prob, dict(par, precision=prec, pcg_rtol=1e-13 if prec == 0 else 1e-12))
    res = lib.coefficients(plan, I, 3)
    C_ref, fam, ns = coefficients(oracle_sampler(prob), I, 3)
    assert res.freqs().tolist() == I.tolist()
    assert np.abs(res.coeffs() - C_ref).max() <= tol * np.abs(C_ref).max()
    assert res.stats["samples"] == ns


# ------------------------------------------------------------------ general triangulations
def mesh_sampler(prob, delta=0.0):
    from oracle import fem_mesh
    return fem_mesh.MeshSampler(prob["mesh_xy"], prob["mesh_tri"], prob["mesh_boundary"], prob["a0"], prob["amp"],
                                prob["mode1"], prob["mode2"], model=prob.get("model", 0),
                                alpha=prob.get("alpha", -1.0), beta=prob.get("beta", 1.0), delta=delta,
                                basis=(prob.get("basis1", 0), prob.get("basis2", 0)))


@pytest.mark.parametrize("mesh,d,model,prec", [((10, 11, 1), 4, 0, 0), ((10, 11, 2), 4, 1, 1), ((10, 11, 3), 4, 2, 0),
                                               ((26, 27, 1), 10, 0, 0), ((26, 27, 1), 10, 0, 1),
                                               ((30, 44, 6), 4, 0, 1), ((30, 46, 2), 4, 2, 0),
                                               ((40, 55, 4), 6, 0, 0)])
def test_mesh_solves_match_sparse_direct(lib, mesh, d, model, prec):
    # jittered Delaunay meshes (121 and 729 inner vertices, the latter shaped
    # like the paper's mesh; 1936, 2116 and 3025, beyond the LDS solver, on
    # the global-scratch one) against the oracle's sparse direct solves; the
    # mesh sampler solves in float64 in both precisions
    from oracle import periodization as OP
    prob = dict(W.mesh_problem(W.jittered_mesh(*mesh), d, 8), model=model)
    if model == 2:
        prob = dict(prob, a0=0.5, basis2=1)
    delta = OP.delta_opt(9601)
    plan = lib.Plan(prob, dict(W.params(10, 1, 1e-4), precision=prec, pcg_rtol=1e-13))
    S = mesh_sampler(prob, delta)
    assert plan.G == S.G
    ns = 23
    Y = np.random.default_rng(mesh[2] + d).random((ns, d))
    U = torch.zeros((S.G, ns), dtype=torch.float64, device="cuda")
    it = torch.zeros(ns, dtype=torch.int32, device="cuda")
    lib.sample(plan, dev(Y), U, 0, ns, 0, it)
    assert (host(it) > 0).all()
    Ug = host(U).T
    for s_ in range(0, ns, 5):
        ref = S.solve_one(Y[s_])
        assert np.linalg.norm(Ug[s_] - ref) <= 1e-11 * np.linalg.norm(ref), s_
    # a sample's result does not depend on the batch it is solved in
    U1 = torch.zeros((S.G, 1), dtype=torch.float64, device="cuda")
    lib.sample(plan, dev(Y[7:8]), U1, 0, 1)
    assert np.array_equal(host(U1)[:, 0], Ug[7])


def test_detect_on_a_large_mesh(lib):
    # whole job on a mesh of 3025 inner vertices (the global-scratch solver):
    # the oracle's sets and coefficients
    prob = W.mesh_problem(W.jittered_mesh(40, 55, 8), 3, 6)
    par = W.params(15, 1, 1e-3)
    res, ref = run_both(lib, prob, par, 2, sampler=mesh_sampler(prob))
    assert res.G == 3025
    assert res.freqs().tolist() == ref.I.tolist()
    assert np.abs(res.coeffs() - ref.C).max() <= 1e-10 * np.abs(ref.C).max()


def test_uniform_mesh_through_the_mesh_sampler(lib):
    # the uniform mesh written as a triangulation gives the structured
    # solvers' samples
    n, d = 16, 4
    base = W.pde_problem(n, d, 8)
    prob = dict(W.mesh_problem(W.uniform_mesh(n), d, 8), amp=base["amp"], mode1=base["mode1"], mode2=base["mode2"])
    Y = np.random.default_rng(4).random((9, d))
    outs = []
    for pr in (base, prob):
        plan = lib.Plan(pr, dict(W.params(10, 1, 1e-4), pcg_rtol=1e-13))
        U = torch.zeros((plan.G, 9), dtype=torch.float64, device="cuda")
        lib.sample(plan, dev(Y), U, 0, 9)
        outs.append(host(U))
    assert np.abs(outs[0] - outs[1]).max() <= 1e-11 * np.abs(outs[0]).max()


def test_detect_on_a_mesh_cpu_scale(lib):
    # whole job with the mesh sampler: the oracle's sets and coefficients;
    # evaluation and error measures work on the result
    from oracle import evaluation as oev
    prob = W.mesh_problem(W.jittered_mesh(10, 11, 5), 4, 8)
    par = W.params(30, 2, 1e-4)
    res, ref = run_both(lib, prob, par, 3, sampler=mesh_sampler(prob))
    assert res.freqs().tolist() == ref.I.tolist()
    assert np.abs(res.coeffs() - ref.C).max() <= 1e-10 * np.abs(ref.C).max()
    assert res.stats["solver_kind"] == 3
    Y = np.random.default_rng(6).random((40, 4))
    ep = torch.zeros(res.G, dtype=torch.float64, device="cuda")
    ei = torch.zeros(res.G, dtype=torch.float64, device="cuda")
    lib.errors(res.plan, res, dev(Y), 2.0, ep, ei)
    S = mesh_sampler(prob)
    e_ref, i_ref = oev.errors(np.array([S.solve_param(y) for y in Y]), oev.approximation(ref.I, ref.C, Y), 2.0)
    assert np.abs(host(ep) - e_ref).max() <= 1e-9 * np.abs(ref.C).max() + 1e-6 * e_ref.max()


def test_mesh_problems_are_checked(lib):
    m = W.jittered_mesh(6, 7, 1)
    par = W.params(10, 1, 1e-4)
    bad_tri = m["mesh_tri"].copy()
    bad_tri[0, 1] = bad_tri[0, 0]  # degenerate triangle
    bad_idx = m["mesh_tri"].copy()
    bad_idx[3, 2] = len(m["mesh_xy"])  # vertex out of range
    # (meshes beyond 2048 inner vertices are accepted: the global-scratch solver)
    for mesh in (dict(m, mesh_tri=bad_tri), dict(m, mesh_tri=bad_idx),
                 dict(m, mesh_boundary=np.ones(len(m["mesh_xy"]), dtype=np.uint8))):
        with pytest.raises(lib.UsfftError) as e:
            lib.Plan(W.mesh_problem(mesh, 4, 8), par)
        assert e.value.status == lib.EINVAL


@pytest.mark.parametrize("case", range(3), ids=["d1", "nothing_detected", "flat_dimension"])
def test_degenerate_jobs_match_oracle(lib, case):
    # d = 1 (no step 2), a threshold above every coefficient (empty result
    # after step 1), and a box with K_t = 1 in the middle coordinate
    name, K, P, lo, hi, theta, r = W.degenerate_trig_cases()[case]
    d = K.shape[1]
    prob = dict(sampler="poly", d=d, k_lo=lo, k_hi=hi, poly_k=K, poly_c=P)
    res, ref = run_both(lib, prob, W.params(40, r, theta, relative=False), 7, sampler=TrigPolySampler(K, P))
    assert res.freqs().tolist() == ref.I.tolist()
    assert res.stats["samples"] == ref.samples
    if name == "empty":
        assert res.n == 0
        Y = np.random.default_rng(1).random((5, d))
        out = torch.ones((5, res.G), dtype=torch.float64, device="cuda")
        lib.eval(res, dev(Y), out)
        assert np.array_equal(host(out), np.zeros((5, res.G)))
        var = torch.ones(res.G, dtype=torch.float64, device="cuda")
        gsi = torch.ones((d, res.G), dtype=torch.float64, device="cuda")
        lib.statistics(res, None, var, gsi)
        assert not host(var).any() and not host(gsi).any()
        return
    assert np.abs(res.coeffs() - ref.C).max() <= 1e-12 * np.abs(ref.C).max()


def test_error_paths(lib):
    prob, par = W.WORKLOADS["cpu16_d4"]
    with pytest.raises(lib.UsfftError) as e:
        lib.Plan(dict(prob, mesh_n=600), par)
    assert e.value.status == lib.EINVAL
    plan = lib.Plan(prob, dict(par, pcg_maxit=3, solver_config=-2))
    with pytest.raises(lib.UsfftError) as e:
        lib.detect(plan, 1)
    assert e.value.status == lib.ENOCONV
    plan = lib.Plan(prob, dict(par, lattice_max=1, lattice_tries=1, lattice_mmax=7, solver_config=-2))
    with pytest.raises(lib.UsfftError) as e:
        lib.detect(plan, 1)
    assert e.value.status == lib.ELATTICE


# ------------------------------------------------------------------ node sets given by points
@pytest.mark.parametrize("kind,prec", [("uniform", 0), ("uniform", 1), ("jittered", 0)])
def test_solves_at_points(lib, kind, prec):
    """Sec. 3.1: solves at nodes that are not mesh vertices (P1 interpolation
    from the containing triangle) against the oracle's solve followed by its
    own brute-force point location; 150 seeded points plus every corner
    region and a few vertices."""
    from oracle import interp as oi
    from oracle.fem_mesh import MeshSampler
    d = 4
    pts = np.concatenate([W.random_points(150, 8), [[0.0, 0.0], [1.0, 1.0], [0.5, 0.5], [0.25, 0.75], [1.0, 0.3]]])
    if kind == "uniform":
        n = 16
        prob = dict(W.pde_problem(n, d, 4), nodes_xy=pts)
        mesh = W.uniform_mesh(n)
        S = ofem.PDESampler(n, prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    else:
        mesh = W.jittered_mesh(12, 11, 2)
        prob = dict(W.mesh_problem(mesh, d, 4), nodes_xy=pts)
        S = MeshSampler(mesh["mesh_xy"], mesh["mesh_tri"], mesh["mesh_boundary"], prob["a0"], prob["amp"],
                        prob["mode1"], prob["mode2"])
    IS = oi.InterpolatingSampler(S, mesh["mesh_xy"], mesh["mesh_tri"], mesh["mesh_boundary"], pts)
    plan = lib.Plan(prob, dict(W.params(4, 1, 1e-4), precision=prec, pcg_rtol=1e-13 if prec == 0 else 1e-12))
    assert plan.G == len(pts)
    Y = np.random.default_rng(3).random((9, d))
    U = torch.zeros((plan.G, 16), dtype=torch.float64, device="cuda")
    lib.sample(plan, dev(Y), U, 0, 16, 3)
    Ug = host(U)[:, 3:12].T
    ref = IS(Y)
    err = (np.linalg.norm(Ug - ref, axis=1) / np.linalg.norm(ref, axis=1)).max()
    assert err <= (1e-11 if prec == 0 else 1e-9), err


def test_detect_at_points_matches_oracle(lib):
    """A whole CPU-scale job (h = 1/16, d = 4) on 90 seeded points against the
    oracle's Alg. 1 with the interpolating sampler: identical sets,
    coefficients within 1e-10 of the largest."""
    from oracle import interp as oi
    from oracle.usfft import usfft
    prob, par = W.WORKLOADS["cpu16_d4"]
    pts = W.random_points(90, 21)
    prob = dict(prob, nodes_xy=pts)
    mesh = W.uniform_mesh(prob["mesh_n"])
    S = ofem.PDESampler(prob["mesh_n"], prob["a0"], prob["amp"], prob["mode1"], prob["mode2"])
    IS = oi.InterpolatingSampler(S, mesh["mesh_xy"], mesh["mesh_tri"], mesh["mesh_boundary"], pts)
    plan = lib.Plan(prob, dict(par, precision=lib.FP64, pcg_rtol=1e-13))
    res = lib.detect(plan, 6)
    ref = usfft(IS, prob["d"], prob["k_lo"], prob["k_hi"], par["s"], par["s_local"], par["r"], par["theta"], True, 6)
    assert res.freqs().tolist() == ref.I.tolist()
    assert res.stats["samples"] == ref.samples
    err = np.abs(res.coeffs() - ref.C).max() / np.abs(ref.C).max()
    assert err <= 1e-10, err


def test_points_outside_rejected(lib):
    prob = dict(W.pde_problem(8, 2, 4), nodes_xy=[[0.5, 0.5], [1.5, 0.2]])
    with pytest.raises(lib.UsfftError) as e:
        lib.Plan(prob, W.params(4, 1, 1e-4))
    assert e.value.status == lib.EINVAL
