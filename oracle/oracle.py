"""Python view of the CPU oracle (oracle/mfcg_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  The product package never imports it.

The oracle computes, in FP64 and by the plain definitions of the paper:
  * the Q_k stiffness matrix of the scalar Poisson problem assembled from
    brute-force element matrices (Sec. 2, Eq. 3-5) into CSR, Dirichlet nodes
    kept as identity rows/columns (Sec. 5.3, constrained unknowns),
  * its diagonal (the point-Jacobi preconditioner of Sec. 3),
  * Algorithm 1 (preconditioned CG) stopping on ||r||_2 < tol*||b||_2
    (Sec. 3.1),
  * the load vector, the L2 error to prod sin(pi x_j), and single operator
    rows evaluated cell by cell for sampled checks at large sizes.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MFCG_ORACLE_LIBRARY selects another build of the same source (the
# host-sanitizer build of the CPU tests)
_DEFAULT_LIB = os.path.join(_HERE, "liboracle.so")
LIB_PATH = os.environ.get("MFCG_ORACLE_LIBRARY") or _DEFAULT_LIB
SOURCE = os.path.join(_HERE, "mfcg_oracle.c")

MAP_AFFINE, MAP_SINE_SHEAR, MAP_SINE_PRODUCT = 0, 1, 2
BC_DIRICHLET, BC_NONE = 0, 1
F_SINE, F_BUMPS = 0, 1

_lib = None


def build(verbose=False):
    """Compile liboracle.so with gcc + OpenMP."""
    import subprocess
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", _DEFAULT_LIB + ".tmp", SOURCE, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_DEFAULT_LIB + ".tmp", _DEFAULT_LIB)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double


def _declare(L):
    L.oracle_gauss.argtypes = [_I, _P, _P]
    L.oracle_gll.argtypes = [_I, _P]
    L.oracle_gll_weights.argtypes = [_I, _P, _P]
    L.oracle_lagrange.argtypes = [_I, _P, _I, _D]
    L.oracle_lagrange.restype = _D
    L.oracle_lagrange_deriv.argtypes = [_I, _P, _I, _D]
    L.oracle_lagrange_deriv.restype = _D
    L.oracle_map.argtypes = [_I, _D, _P, _P]
    L.oracle_map_det.argtypes = [_I, _D, _P]
    L.oracle_map_det.restype = _D
    mesh = [_P, _I, _I, _I, _D, _I, _P, _I]
    L.oracle_n_nodes.argtypes = [_P, _I]
    L.oracle_n_nodes.restype = _I64
    L.oracle_element_matrix.argtypes = mesh + [_P, _P]
    L.oracle_csr_rowptr.argtypes = mesh + [_P]
    L.oracle_csr_fill.argtypes = mesh + [_P, _P, _P]
    L.oracle_rhs.argtypes = mesh + [_I, _P, _P]
    L.oracle_l2_error.argtypes = mesh + [_I, _P]
    L.oracle_l2_error.restype = _D
    L.oracle_apply_rows.argtypes = mesh + [_P, _I64, _P, _P]
    L.oracle_spmv.argtypes = [_I64, _P, _P, _P, _P, _P]
    L.oracle_pcg.argtypes = [_I64, _P, _P, _P, _P, _P, _P, _D, _I, _P, _P]
    L.oracle_csr_diag.argtypes = [_I64, _P, _P, _P, _P]
    L.oracle_max_threads.restype = _I


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def gauss(n):
    x = np.zeros(n)
    w = np.zeros(n)
    assert lib().oracle_gauss(n, _ptr(x), _ptr(w)) == 0
    return x, w


def gll_weights(k):
    """Weights of the k+1 point Gauss-Lobatto-Legendre rule on [0,1]."""
    x, w = gll(k), np.zeros(k + 1)
    assert lib().oracle_gll_weights(k, _ptr(x), _ptr(w)) == 0
    return w


def gll(k):
    x = np.zeros(k + 1)
    assert lib().oracle_gll(k, _ptr(x)) == 0
    return x


def lagrange(nodes, i, x):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    return lib().oracle_lagrange(len(nodes), _ptr(nodes), i, float(x))


def lagrange_deriv(nodes, i, x):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    return lib().oracle_lagrange_deriv(len(nodes), _ptr(nodes), i, float(x))


def map_points(kind, amp, X):
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 3)
    out = np.zeros_like(X)
    for i in range(X.shape[0]):
        lib().oracle_map(kind, amp, _ptr(X[i]), _ptr(out[i]))
    return out


def map_det(kind, amp, X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    return lib().oracle_map_det(kind, amp, _ptr(X))


class Mesh:
    """Structured n0 x n1 x n2 hexahedral mesh of [0,1]^3 under a map.

    Node numbering is lexicographic: i = gx + (n0 k + 1) (gy + (n1 k + 1) gz).
    Cell numbering: c = cx + n0 (cy + n1 cz)."""

    def __init__(self, ncells, k, nq1=None, map_kind=MAP_AFFINE, amp=0.0, bc=BC_DIRICHLET, coeff=None,
                 quad="gauss", op="laplace", geometry="exact"):
        """quad: "gauss" (Gauss-Legendre, nq1 points, default k+1) or "gll"
        (Gauss-Lobatto-Legendre on nq1 points, default k+1: collocation at
        the nodes); op: "laplace" (Eq. 5) or "mass" (a_e w_q det J phi_i
        phi_j); geometry: "exact" (the map itself) or "quadratic" (in every
        cell the map's tensor-product quadratic interpolant through 27
        points, Sec. 2.2)."""
        assert geometry in ("exact", "quadratic")
        self.geom_bit = 16 if geometry == "quadratic" else 0
        assert op in ("laplace", "mass")
        self.op = 0 if op == "laplace" else 1
        if np.isscalar(ncells):
            ncells = (ncells, ncells, ncells)
        self.ncells = np.ascontiguousarray(ncells, dtype=np.int32)
        self.k = int(k)
        self.nq1 = int(nq1) if nq1 else self.k + 1
        assert quad in ("gauss", "gll")
        if quad == "gll":
            self.nq1 = -self.nq1
        self.map_kind = int(map_kind)
        self.amp = float(amp)
        self.bc = int(bc)
        self.coeff = None if coeff is None else np.ascontiguousarray(coeff, dtype=np.float64).ravel()
        if self.coeff is not None:
            assert self.coeff.size == int(np.prod(self.ncells))

    @property
    def lattice(self):
        return tuple(int(n) * self.k + 1 for n in self.ncells)

    @property
    def n_nodes(self):
        return int(lib().oracle_n_nodes(_ptr(self.ncells), self.k))

    def args(self):
        return [_ptr(self.ncells), self.k, self.nq1, self.map_kind | self.geom_bit, self.amp, self.bc,
                _ptr(self.coeff), self.op]

    def constrained_mask(self):
        L = self.lattice
        gz, gy, gx = np.meshgrid(np.arange(L[2]), np.arange(L[1]), np.arange(L[0]), indexing="ij")
        m = np.zeros(L[::-1], dtype=bool)
        if self.bc == BC_DIRICHLET:
            m = (gx == 0) | (gx == L[0] - 1) | (gy == 0) | (gy == L[1] - 1) | (gz == 0) | (gz == L[2] - 1)
        return m.ravel()


class CSR:
    def __init__(self, rowptr, col, val):
        self.rowptr, self.col, self.val = rowptr, col, val
        self.n = rowptr.size - 1

    def matvec(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        lib().oracle_spmv(self.n, _ptr(self.rowptr), _ptr(self.col), _ptr(self.val), _ptr(x), _ptr(y))
        return y

    def diagonal(self):
        d = np.empty(self.n)
        lib().oracle_csr_diag(self.n, _ptr(self.rowptr), _ptr(self.col), _ptr(self.val), _ptr(d))
        return d

    def abs_matvec(self, x):
        """(|A| |x|): the componentwise scale used for rounding bounds."""
        a = CSR(self.rowptr, self.col, np.abs(self.val))
        return a.matvec(np.abs(x))

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def element_matrix(mesh, cell):
    nb = (mesh.k + 1) ** 3
    A = np.zeros((nb, nb))
    c = np.ascontiguousarray(cell, dtype=np.int32)
    rc = lib().oracle_element_matrix(*mesh.args(), _ptr(c), _ptr(A))
    assert rc == 0, rc
    return A


def assemble(mesh):
    n = mesh.n_nodes
    rowptr = np.zeros(n + 1, dtype=np.int64)
    assert lib().oracle_csr_rowptr(*mesh.args(), _ptr(rowptr)) == 0
    nnz = int(rowptr[-1])
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz)
    rc = lib().oracle_csr_fill(*mesh.args(), _ptr(rowptr), _ptr(col), _ptr(val))
    assert rc == 0, rc
    return CSR(rowptr, col, val)


def rhs(mesh, fkind=F_SINE, params=None):
    b = np.zeros(mesh.n_nodes)
    p = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    assert lib().oracle_rhs(*mesh.args(), int(fkind), _ptr(p), _ptr(b)) == 0
    return b


def l2_error(mesh, uh, nqe=None):
    uh = np.ascontiguousarray(uh, dtype=np.float64)
    return lib().oracle_l2_error(*mesh.args(), int(nqe or mesh.k + 3), _ptr(uh))


def apply_rows(mesh, u, rows):
    u = np.ascontiguousarray(u, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.size)
    assert lib().oracle_apply_rows(*mesh.args(), _ptr(u), rows.size, _ptr(rows), _ptr(out)) == 0
    return out


def pcg(A, diag, b, x0=None, tol=1e-10, maxit=10000):
    """Algorithm 1.  Returns (x, iters, hist, rc); rc 0 converged, -4 maxit,
    -5 breakdown."""
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    diag = np.ascontiguousarray(diag, dtype=np.float64)
    hist = np.zeros(maxit + 1)
    it = ctypes.c_int(0)
    rc = lib().oracle_pcg(A.n, _ptr(A.rowptr), _ptr(A.col), _ptr(A.val), _ptr(diag), _ptr(b), _ptr(x),
                          float(tol), int(maxit), ctypes.byref(it), _ptr(hist))
    return x, it.value, hist[: it.value + 1].copy(), rc


def interpolate(cells, k_from, k_to, src):
    """The Q_{k_from} finite-element function with lexicographic nodal
    values src (x fastest), evaluated at the nodes of the Q_{k_to} space on
    the same cells (Sec. 2: continuous Q_k, nodes at the Gauss-Lobatto
    points of every cell).  The function is a tensor product of 1D
    piecewise Lagrange interpolants, so its values at the destination
    nodes are (P_z (x) P_y (x) P_x) src with the 1D matrices P_d[g, j] = the
    Lagrange polynomial of source node j of the cell holding destination
    node g (the last cell for the right end), at g's reference position."""
    cells = tuple(int(c) for c in cells)
    xf, xt = gll(k_from), gll(k_to)
    P = []
    for N in cells:
        M = np.zeros((N * k_to + 1, N * k_from + 1))
        for g in range(N * k_to + 1):
            e = min(g // k_to, N - 1)
            t = xt[g - k_to * e]
            for j in range(k_from + 1):
                M[g, k_from * e + j] = lagrange(xf, j, t)
        P.append(M)
    U = np.asarray(src, dtype=np.float64).reshape(cells[2] * k_from + 1, cells[1] * k_from + 1,
                                                  cells[0] * k_from + 1)
    U = np.einsum("zyx,ax->zya", U, P[0])
    U = np.einsum("zya,by->zba", U, P[1])
    U = np.einsum("zba,cz->cba", U, P[2])
    return U.reshape(-1).copy()


def max_threads():
    return int(lib().oracle_max_threads())
