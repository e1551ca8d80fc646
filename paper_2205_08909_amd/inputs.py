"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
calls.  This module holds no arithmetic of the method itself: it draws random
numbers and builds index masks only.

Workload recipes (the paper's benchmark problems, Sec. 2.1 and Sec. 6, are
the CEED BP3/BP5-style scalar Laplacians on deformed hexahedral meshes; these
synthetic fields stand in for them):
  * coefficient a = exp(g), g a Gaussian random field with squared-
    exponential covariance sigma^2 exp(-|x-x'|^2 / (2 l^2)) sampled at cell
    centres; exact in distribution on the tensor grid via the Kronecker
    factorisation C = C_x (x) C_y (x) C_z,
  * right-hand sides: standard normal entries on free nodes, zero on
    Dirichlet nodes, or the parameters of a sum of Gaussian bumps.
"""
import numpy as np

MAP_AFFINE, MAP_SINE_SHEAR, MAP_SINE_PRODUCT = 0, 1, 2


def _sqrt_cov_1d(n, length):
    x = (np.arange(n) + 0.5) / n
    C = np.exp(-(x[:, None] - x[None, :]) ** 2 / (2.0 * length ** 2))
    lam, V = np.linalg.eigh(C)
    return (V * np.sqrt(np.clip(lam, 0.0, None))) @ V.T


def grf_log_coefficient(ncells, length=0.1, variance=1.0, seed=0):
    """g at cell centres, flattened with c = cx + nx (cy + ny cz)."""
    if np.isscalar(ncells):
        ncells = (ncells, ncells, ncells)
    nx, ny, nz = (int(v) for v in ncells)
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((nz, ny, nx))
    Lx, Ly, Lz = (_sqrt_cov_1d(n, length) for n in (nx, ny, nz))
    g = np.einsum("ia,abc->ibc", Lz, xi)
    g = np.einsum("jb,ibc->ijc", Ly, g)
    g = np.einsum("kc,ijc->ijk", Lx, g)
    return (np.sqrt(variance) * g).ravel()


def grf_coefficient(ncells, length=0.1, variance=1.0, seed=0):
    return np.exp(grf_log_coefficient(ncells, length, variance, seed))


def lattice(ncells, k):
    if np.isscalar(ncells):
        ncells = (ncells, ncells, ncells)
    return tuple(int(n) * int(k) + 1 for n in ncells)


def boundary_mask(ncells, k):
    """True on nodes of the domain boundary (lexicographic, x fastest)."""
    L = lattice(ncells, k)
    m = np.zeros(L[::-1], dtype=bool)
    m[0, :, :] = m[-1, :, :] = True
    m[:, 0, :] = m[:, -1, :] = True
    m[:, :, 0] = m[:, :, -1] = True
    return m.ravel()


def random_rhs(ncells, k, seed=0, dirichlet=True):
    L = lattice(ncells, k)
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(L[0] * L[1] * L[2])
    if dirichlet:
        b[boundary_mask(ncells, k)] = 0.0
    return b


def random_vector(n, seed=0):
    return np.random.default_rng(seed).standard_normal(n)


def bump_params(seed, nbumps=8):
    """[nbumps, (A, cx, cy, cz, s) * nbumps]: A ~ N(0,1), c ~ U[0.1,0.9]^3,
    s ~ U[0.03, 0.1]."""
    rng = np.random.default_rng(seed)
    p = [float(nbumps)]
    for _ in range(nbumps):
        A = rng.standard_normal()
        c = rng.uniform(0.1, 0.9, size=3)
        s = rng.uniform(0.03, 0.1)
        p += [A, c[0], c[1], c[2], s]
    return np.array(p)


def batch_draw(seed=0, nprob=32, nmin=16, nmax=96, kmin=2, kmax=6):
    """Problem list of the batched workload: side N ~ U{nmin..nmax}, degree
    k ~ U{kmin..kmax}; per-problem seeds 1000 + i."""
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(nprob):
        N = int(rng.integers(nmin, nmax + 1))
        k = int(rng.integers(kmin, kmax + 1))
        probs.append({"N": N, "k": k, "seed": 1000 + i})
    return probs


def warmstart_sample(seed, ncells=48):
    """Coefficient length ~ U[0.05, 0.2], variance 1, and bump RHS params."""
    rng = np.random.default_rng(seed)
    length = float(rng.uniform(0.05, 0.2))
    logc = grf_log_coefficient(ncells, length, 1.0, seed=seed + 7_000_000)
    return {"length": length, "log_coeff": logc, "coeff": np.exp(logc), "bumps": bump_params(seed + 9_000_000)}


def network_init(shapes, seed=0, last_scale=0.1):
    """Initial weights of the warm-start network: for each weight shape
    (c_out, c_in, kd, kh, kw) normal draws with standard deviation
    sqrt(2 / fan_in), fan_in = c_in kd kh kw (the last shape scaled by
    last_scale); biases zero.  Returns a list of (w, b) float32 arrays."""
    rng = np.random.default_rng(seed)
    out = []
    for i, sh in enumerate(shapes):
        fan_in = int(np.prod(sh[1:]))
        std = np.sqrt(2.0 / fan_in) * (last_scale if i == len(shapes) - 1 else 1.0)
        out.append((rng.standard_normal(sh).astype(np.float32) * np.float32(std), np.zeros(sh[0], np.float32)))
    return out
