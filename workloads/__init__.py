"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

Holds problem definitions (coefficient families, boxes, sparsity parameters)
and seeded random-input generators only; none of the method's arithmetic
lives here.
"""
import math

import numpy as np


def amplitudes(d):
    """0.5 j^-2, j = 1..d (all workloads)."""
    return [0.5 * j ** -2.0 for j in range(1, d + 1)]


def modes_diagonal(d):
    """sin(j pi x1) sin(j pi x2): the 4-term CPU-scale workload."""
    return list(range(1, d + 1)), list(range(1, d + 1))


def modes_split(d):
    """sin(ceil(j/2) pi x1) sin(floor(j/2 + 1) pi x2): the larger workloads."""
    return [math.ceil(j / 2) for j in range(1, d + 1)], [j // 2 + 1 for j in range(1, d + 1)]


def pde_problem(n, d, N, modes="split", a0=1.0):
    m1, m2 = (modes_diagonal if modes == "diagonal" else modes_split)(d)
    return dict(sampler="pde", mesh_n=n, d=d, k_lo=[-N] * d, k_hi=[N] * d,
                a0=a0, amp=amplitudes(d), mode1=m1, mode2=m2)


def diagonal_enumeration(j):
    """(m1(j), m2(j)) of the affine example (Sec. 4.3): k = floor(-1/2 +
    sqrt(1/4 + 2j)), m1 = j - k(k+1)/2, m2 = k - m1."""
    k = int(math.floor(-0.5 + math.sqrt(0.25 + 2 * j)))
    m1 = j - k * (k + 1) // 2
    return m1, k - m1


def affine_problem(n, d, N, c=0.5, mu=2.0, alpha=-1.0, beta=1.0):
    """Affine model shaped like the paper's affine example: a = 1 + sum_j y_j
    c j^-mu cos(2 pi m1(j) x1) cos(2 pi m2(j) x2), y uniform on [alpha, beta]^d
    (tent periodization); f = 1 as in every workload here."""
    m = [diagonal_enumeration(j) for j in range(1, d + 1)]
    return dict(sampler="pde", mesh_n=n, d=d, k_lo=[-N] * d, k_hi=[N] * d, a0=1.0,
                amp=[c * j ** -mu for j in range(1, d + 1)], mode1=[2 * a for a, _ in m],
                mode2=[2 * b for _, b in m], model=1, alpha=alpha, beta=beta, basis1=1, basis2=1)


def lognormal_problem(n, d, N, delta=0.0):
    """Lognormal model shaped like the paper's lognormal example: a =
    exp(sum_j (1/j) y_j sin(2 pi j x1) cos(2 pi (d+1-j) x2)), y ~ N(0,1)^d
    (shifted tent and inverse normal CDF); f = 1 as in every workload here."""
    return dict(sampler="pde", mesh_n=n, d=d, k_lo=[-N] * d, k_hi=[N] * d, a0=0.0,
                amp=[1.0 / j for j in range(1, d + 1)], mode1=[2 * j for j in range(1, d + 1)],
                mode2=[2 * (d + 1 - j) for j in range(1, d + 1)], model=2, delta=delta, basis1=0, basis2=1)


def params(s, r, theta, relative=True, **kw):
    p = dict(s=s, s_local=s, r=r, theta=theta, theta_relative=relative,
             lattice_c=2.0, lattice_tries=8, lattice_max=64, lattice_mmax=9601)
    p.update(kw)
    return p


# The five synthetic workloads (uniform P1 meshes, periodic coefficient with
# 0.5 j^-2 amplitudes, f = 1, zero Dirichlet data).
WORKLOADS = {
    # CPU scale: h = 1/16, d = 4, box [-16,16]^4, s = 50, rel. threshold 1e-4, r = 3
    "cpu16_d4": (pde_problem(16, 4, 16, modes="diagonal"), params(50, 3, 1e-4)),
    # h = 1/64 (3969 nodes), d = 10, box [-32,32]^10, s = 200, rel. threshold 1e-5, r = 5
    "mesh64_d10": (pde_problem(64, 10, 32), params(200, 5, 1e-5)),
    # the h = 1/64 workload's box, sparsity and threshold on the h = 1/16 mesh
    "mesh16_d10": (pde_problem(16, 10, 32), params(200, 5, 1e-5)),
    # h = 1/128 (16129 nodes), d = 20, box [-64,64]^20, s = 500, rel. threshold 1e-6, r = 5
    "mesh128_d20": (pde_problem(128, 20, 64), params(500, 5, 1e-6)),
    # a whole job on the h = 1/128 mesh small enough for the oracle (about
    # 2200 solves): d = 4, box [-8,8]^4, s = 30, rel. threshold 1e-4, r = 2
    "mesh128_d4": (pde_problem(128, 4, 8), params(30, 2, 1e-4)),
    # the same on the h = 1/256 mesh (65025 nodes, the two-level solver)
    "mesh256_d4": (pde_problem(256, 4, 8), params(30, 2, 1e-4)),
}


def uneven_batch(seed=1, jobs=12, meshes=(32, 64, 128), dims=(8, 16, 30), Ns=(16, 32, 64), ss=(100, 300, 500)):
    """Jobs mixing meshes, d, N and s (default: 12 jobs, meshes 32^2/64^2/128^2,
    d in {8,16,30}, N in {16,32,64}, s in {100,300,500}), each seeded."""
    g = np.random.default_rng(seed)
    out = []
    for _ in range(jobs):
        n = int(g.choice(list(meshes)))
        d = int(g.choice(list(dims)))
        N = int(g.choice(list(Ns)))
        s = int(g.choice(list(ss)))
        out.append((pde_problem(n, d, N), params(s, 5, 1e-5), int(g.integers(1, 2 ** 31))))
    return out


def serving_stream(seed=1, rate=4.0, jobs=20, meshes=(16, 32, 64), dims=(4, 10), Ns=(16, 32), ss=(50, 200)):
    """Poisson arrivals (mean `rate` jobs/s) of jobs with random mesh, d, N and s."""
    g = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(jobs):
        t += float(g.exponential(1.0 / rate))
        n = int(g.choice(list(meshes)))
        d = int(g.integers(dims[0], dims[1] + 1))
        N = int(g.choice([v for v in (16, 32, 64) if Ns[0] <= v <= Ns[1]]))
        s = int(g.integers(ss[0], ss[1] + 1))
        out.append((t, pde_problem(n, d, N), params(s, 5, 1e-5), int(g.integers(1, 2 ** 31))))
    return out


def trig_poly(seed, d, N, G, n_freq, max_active=4, kmax=4, cmin=1e-3, cmax=1.0, per_node=0.7):
    """Seeded real trigonometric polynomials with a shared, +-closed support.

    Returns (K, P): K (n x d) frequencies in [-N, N]^d with at most
    `max_active` non-zero components of size <= kmax, closed under k -> -k;
    P (n x G) complex coefficients with P[-k] = conj(P[k]); each node uses a
    random +-closed subset of the support (fraction `per_node`), the others
    are exactly zero.  Non-zero magnitudes lie in [cmin, cmax].
    """
    g = np.random.default_rng(seed)
    kmax = min(kmax, N)
    S = {tuple([0] * d)}
    while len(S) < n_freq:
        k = np.zeros(d, dtype=np.int64)
        act = g.choice(d, size=int(g.integers(1, min(max_active, d) + 1)), replace=False)
        k[act] = g.integers(1, kmax + 1, size=len(act)) * g.choice([-1, 1], size=len(act))
        S.add(tuple(k))
        S.add(tuple(-k))
    K = np.array(sorted(S), dtype=np.int64)
    index = {tuple(k): a for a, k in enumerate(K)}
    P = np.zeros((len(K), G), dtype=np.complex128)
    for a, k in enumerate(K):
        b = index[tuple(-k)]
        if b < a:
            continue
        use = g.random(G) < per_node
        if a == b:  # k = 0: real coefficient
            mag = g.uniform(cmin, cmax, G)
            P[a] = np.where(use, mag * g.choice([-1.0, 1.0], G), 0.0)
        else:
            mag = g.uniform(cmin, cmax, G)
            ph = g.uniform(0, 2 * np.pi, G)
            c = np.where(use, mag * np.exp(1j * ph), 0.0)
            P[a] = c
            P[b] = np.conj(c)
    return K, P


def sample_matrix(seed, M, G, kind="smooth"):
    """Seeded real test samples (M x G) for the lattice-DFT stage."""
    g = np.random.default_rng(seed)
    if kind == "smooth":
        base = 0.05 + 0.01 * g.standard_normal(G)
        return base[None, :] + 1e-3 * g.standard_normal((M, G))
    return g.standard_normal((M, G))


def candidate_set(seed, n_parent, t, n_child, kmax=4, max_active=4):
    """A +-closed parent set (sorted) and a symmetric child range, shaped like
    the detected sets of the workloads (few active dimensions, small |k_j|)."""
    g = np.random.default_rng(seed)
    S = {tuple([0] * (t - 1))}
    if (t - 1) == 1 and n_parent > 2 * kmax + 1:
        raise ValueError("a 1-D parent set holds at most 2*kmax+1 values")
    while len(S) < n_parent:
        k = np.zeros(t - 1, dtype=np.int64)
        act = g.choice(t - 1, size=int(g.integers(1, min(max_active, t - 1) + 1)), replace=False)
        k[act] = g.integers(1, kmax + 1, size=len(act)) * g.choice([-1, 1], size=len(act))
        S.add(tuple(k))
        S.add(tuple(-k))
    parent = np.array(sorted(S), dtype=np.int64)
    child = np.arange(-(n_child // 2), n_child // 2 + 1, dtype=np.int64)
    return parent, child


# ---- a-priori frequency sets (Sec. 4.5), inputs of usfft_coefficients ----
# Weights are integer multipliers m_j (weight 1/m_j), so membership is exact.

def _enumerate(d, keep_prefix):
    """All k in Z^d (lexicographic) whose every prefix passes keep_prefix."""
    out = []

    def rec(prefix):
        if len(prefix) == d:
            out.append(list(prefix))
            return
        k = 0
        # grow |k| in the next coordinate until the prefix test fails
        cands = [0]
        while True:
            k += 1
            if not keep_prefix(prefix + [k]):
                break
            cands += [k, -k]
        for v in sorted(cands):
            rec(prefix + [v])

    rec([])
    return np.array(out, dtype=np.int32).reshape(-1, d)


def axis_cross(d, N):
    """{k : at most one nonzero component, ||k||_1 <= N} (the constant term kept)."""
    return _enumerate(d, lambda p: sum(1 for v in p if v) <= 1 and sum(abs(v) for v in p) <= N)


def hyperbolic_cross(d, N, mult):
    """{k : prod_j max(1, m_j |k_j|) <= N}; m_j = 4 (uniform weight 1/4) or j^q."""
    def ok(p):
        prod = 1
        for j, v in enumerate(p):
            prod *= max(1, mult[j] * abs(v))
        return prod <= N
    return _enumerate(d, ok)


def weighted_l1_ball(d, N, mult):
    """{k : sum_j m_j |k_j| <= N}; m_j = j^q."""
    return _enumerate(d, lambda p: sum(mult[j] * abs(v) for j, v in enumerate(p)) <= N)


# ---- triangulations of the unit square for the general-mesh sampler ----

def uniform_mesh(n):
    """The uniform mesh of h = 1/n as a general triangulation: vertex
    i + (n + 1) j at (i h, j h); each cell split by its (i,j)-(i+1,j+1)
    diagonal into {(i,j),(i+1,j),(i+1,j+1)} and {(i,j),(i,j+1),(i+1,j+1)}."""
    h = 1.0 / n
    j, i = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    xy = np.stack([i.ravel() * h, j.ravel() * h], -1)
    v = lambda a, b: a + (n + 1) * b  # noqa: E731
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ci, cj = ci.ravel(), cj.ravel()
    lower = np.stack([v(ci, cj), v(ci + 1, cj), v(ci + 1, cj + 1)], -1)
    upper = np.stack([v(ci, cj), v(ci, cj + 1), v(ci + 1, cj + 1)], -1)
    tri = np.concatenate([lower, upper]).astype(np.int32)
    bnd = (i.ravel() == 0) | (i.ravel() == n) | (j.ravel() == 0) | (j.ravel() == n)
    return dict(mesh_xy=xy, mesh_tri=tri, mesh_boundary=bnd.astype(np.uint8))


def jittered_mesh(n_bnd, n_in, seed, jitter=0.3):
    """Delaunay triangulation of [0,1]^2 with n_bnd equispaced vertices per
    side (4 n_bnd boundary vertices) and an n_in x n_in grid of interior
    vertices, each moved by up to `jitter` of the grid spacing."""
    from scipy.spatial import Delaunay
    g = np.random.default_rng(seed)
    s = np.arange(n_bnd) / n_bnd
    z, o = np.zeros(n_bnd), np.ones(n_bnd)
    bpts = np.concatenate([np.stack([s, z], -1), np.stack([o, s], -1), np.stack([1 - s, o], -1),
                           np.stack([z, 1 - s], -1)])
    h = 1.0 / (n_in + 1)
    gi, gj = np.meshgrid(np.arange(1, n_in + 1), np.arange(1, n_in + 1), indexing="ij")
    ipts = np.stack([gi.ravel() * h, gj.ravel() * h], -1) + g.uniform(-jitter * h, jitter * h, (n_in * n_in, 2))
    xy = np.concatenate([bpts, ipts])
    tri = Delaunay(xy).simplices.astype(np.int32)
    P = xy[tri]
    det = (P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0])
    tri = tri[np.abs(det) > 1e-14]
    bnd = np.concatenate([np.ones(len(bpts)), np.zeros(len(ipts))]).astype(np.uint8)
    return dict(mesh_xy=xy, mesh_tri=tri, mesh_boundary=bnd)


def random_points(n, seed):
    """n seeded points uniform in the open unit square (a node set T_G)."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, (n, 2))


def mesh_problem(mesh, d, N, a0=1.0, modes="split"):
    """The periodic coefficient family of pde_problem on a general triangulation."""
    m1, m2 = (modes_diagonal if modes == "diagonal" else modes_split)(d)
    return dict(sampler="pde_mesh", d=d, k_lo=[-N] * d, k_hi=[N] * d, a0=a0, amp=amplitudes(d),
                mode1=m1, mode2=m2, **mesh)


def degenerate_trig_cases():
    """Degenerate detection inputs: d = 1; a threshold above every coefficient
    (nothing is detected); a box with a single frequency (K_t = 1) in the
    middle coordinate.  (name, K, P, k_lo, k_hi, theta, r)."""
    K1, P1 = trig_poly(3, 1, 8, 20, 9, cmin=1e-2)
    K2, P2 = trig_poly(4, 3, 8, 10, 15, cmin=1e-2)
    Kb, Pb = trig_poly(5, 2, 8, 12, 21, cmin=1e-2)
    Kb = np.insert(Kb, 1, 0, axis=1)
    return [
        ("d1", K1, P1, [-8], [8], 1e-6, 3),
        ("empty", K2, P2, [-8] * 3, [8] * 3, 1e3, 2),
        ("flat_dim", Kb, Pb, [-8, 0, -8], [8, 0, 8], 1e-6, 3),
    ]
