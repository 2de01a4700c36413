"""The boundary calls of Alg. 1's "Input"/"Output" with a caller-provided
workspace (usfft_plan_workspace, usfft_detect_ws, usfft_coefficients_ws)
and Algorithm A alone on one lattice (usfft_lattice_coeffs, App. A),
through the C ABI."""
import numpy as np
import pytest

import workloads as W
from oracle import dft as odft
from oracle import fem as ofem
from oracle import lattice as olat

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def workspace(nbytes):
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32_refine"])
def test_detect_ws_equals_detect(lib, prec):
    prob, par = W.WORKLOADS["cpu16_d4"]
    plan = lib.Plan(prob, dict(par, precision=prec, pcg_rtol=1e-12))
    ref = lib.detect(plan, 4)
    nc, ns = ref.stats["max_candidates"], ref.stats["max_batch"]
    nc = max(nc, ref.n)
    need = lib.plan_workspace(plan, nc, ns)
    print("cpu16_d4 precision %d: |J| <= %d, batch <= %d samples, workspace %d bytes" % (prec, nc, ns, need),
          flush=True)
    ws = workspace(need)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    res = lib.detect_ws(plan, 4, nc, ns, ws)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print("device memory change during detect_ws: %d bytes" % (free0 - free1))
    assert free0 - free1 <= 4 << 20
    assert res.stats["workspace_bytes"] == need
    assert np.array_equal(res.freqs(), ref.freqs())
    assert np.array_equal(res.coeffs(), ref.coeffs())
    for k in ("samples", "lattices", "max_candidates", "max_batch", "pcg_iterations"):
        assert res.stats[k] == ref.stats[k], k
    # the result's coefficients are read from the workspace by the evaluation
    y = torch.rand((57, prob["d"]), dtype=torch.float64, device="cuda")
    a = torch.zeros((57, res.G), dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    lib.eval(res, y, a)
    lib.eval(ref, y, b)
    assert torch.equal(a, b)
    # too small: the workspace, the candidate bound, the batch bound
    with pytest.raises(lib.UsfftError) as e:
        lib.detect_ws(plan, 4, nc, ns, ws, need - 1)
    assert e.value.status == lib.ENOMEM
    fam = ref.stats["max_family"]
    assert 0 < fam <= ns
    for a_nc, a_ns in ((nc - 1, ns), (nc, fam - 1)):
        small = workspace(lib.plan_workspace(plan, a_nc, a_ns))
        with pytest.raises(lib.UsfftError) as e:
            lib.detect_ws(plan, 4, a_nc, a_ns, small)
        assert e.value.status == lib.ENOMEM, (a_nc, a_ns)
    # the smallest batch bound splits the r iterations of a stage over more
    # sampler launches; every solve is independent of its batch
    one = workspace(lib.plan_workspace(plan, nc, fam))
    res2 = lib.detect_ws(plan, 4, nc, fam, one)
    assert res2.stats["max_batch"] <= max(fam, ref.stats["samples_step1"])
    assert np.array_equal(res2.freqs(), ref.freqs())
    assert np.array_equal(res2.coeffs(), ref.coeffs())
    # the plan still runs normally afterwards
    again = lib.detect(plan, 4)
    assert np.array_equal(again.coeffs(), ref.coeffs())


def test_coefficients_ws_equals_coefficients(lib):
    prob, par = W.WORKLOADS["cpu16_d4"]
    plan = lib.Plan(prob, dict(par, precision=0, pcg_rtol=1e-12))
    A = W.hyperbolic_cross(prob["d"], 8, [1, 2, 3, 4])
    ref = lib.coefficients(plan, A, 9)
    ns = ref.stats["max_batch"]
    ws = workspace(lib.plan_workspace(plan, len(A), ns))
    res = lib.coefficients_ws(plan, A, 9, len(A), ns, ws)
    assert np.array_equal(res.freqs(), ref.freqs())
    assert np.array_equal(res.coeffs(), ref.coeffs())


@pytest.mark.parametrize("M,fp32", [(1153, 0), (2593, 1), (9601, 0)])
def test_lattice_coeffs_against_oracle(lib, M, fp32):
    """Algorithm A on one lattice: bins k.z mod M computed by the call, the
    DFT at those bins against the oracle's naive DFT of the same samples;
    PDE samples at the lattice nodes (h = 1/16, d = 3)."""
    assert olat.admissible(M)
    d, t, G = 3, 3, 225
    g = np.random.default_rng(M)
    z = g.integers(1, M, size=t)
    J = np.stack(np.meshgrid(*[np.arange(-4, 5)] * 3, indexing="ij"), -1).reshape(-1, 3)[:300]
    S = ofem.PDESampler(16, 1.0, W.amplitudes(d), *W.modes_split(d))
    nodes = olat.lattice_nodes(M, z)
    U = S(nodes)  # M x G, oracle solves at the lattice nodes
    ld = M + 5
    Ud = np.zeros((G, ld))
    Ud[:, 2:2 + M] = U.T
    u = torch.from_numpy(Ud.astype(np.float32 if fp32 else np.float64)).cuda()
    Jd = torch.from_numpy(J.astype(np.int32)).cuda()
    out = torch.full((len(J), G, 2), np.nan, dtype=torch.float64, device="cuda")
    print("lattice_coeffs M = %d, z = %s, fp32 %d" % (M, z.tolist(), fp32), flush=True)
    lib.lattice_coeffs(u, fp32, G, ld, 2, M, z, Jd, out)
    got = out.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    bins = (J.astype(np.int64) @ z.astype(np.int64)) % M
    ref = odft.dft_bins(Ud[:, 2:2 + M].T.astype(np.float32 if fp32 else np.float64), bins)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= (1e-6 if fp32 else 1e-12), err


def test_progress_log_lines(lib):
    """USFFT_LOG=1 (read once per process, so the job runs in a child): one
    stderr line for step 1, one per increment t = 2 .. d and one for step 3,
    each naming its counts; without the variable a job prints nothing."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import paper_2109_04131_amd as U, workloads as W\n"
            "prob, par = W.WORKLOADS['cpu16_d4']\n"
            "r = U.detect(U.Plan(prob, par), 1)\n"
            "print('frequencies', r.n)\n")
    d = W.WORKLOADS["cpu16_d4"][0]["d"]
    runs = {}
    for flag in ("1", "0"):
        env = dict(os.environ, USFFT_LOG=flag)
        print("child job cpu16_d4 seed 1, USFFT_LOG=%s" % flag, flush=True)
        out = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                             timeout=150)
        assert out.returncode == 0, out.stderr[-2000:]
        runs[flag] = [ln for ln in out.stderr.splitlines() if ln.startswith("usfft: ")]
        n = int(out.stdout.split()[-1])
    lines = runs["1"]
    assert len(lines) == d + 1, lines
    assert lines[0].startswith("usfft: step 1: %d lines" % (d * W.WORKLOADS["cpu16_d4"][1]["r"]))
    for t in range(2, d + 1):
        assert lines[t - 1].startswith("usfft: increment %d/%d: " % (t, d)), lines[t - 1]
    assert lines[-1].startswith("usfft: step 3: %d frequencies" % n)
    assert runs["0"] == []
