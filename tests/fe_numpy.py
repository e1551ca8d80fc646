"""Independent numpy constructions used to pin the oracle in tests.

Every routine here takes a different computational route from the C oracle:
numpy's Legendre roots instead of Newton iterations, exact polynomial
integration by a high-order rule instead of the (k+1)-point rule, barycentric basis
evaluation instead of the product formula, finite-difference Jacobians instead of the
analytic derivative of the map.  Test helper only.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(k):
    """GLL points on [0,1]: ends plus roots of P_k' (numpy root finder)."""
    inner = npleg.Legendre.basis(k).deriv().roots() if k > 1 else np.array([])
    t = np.concatenate([[-1.0], np.sort(inner.real), [1.0]])
    return 0.5 * (1.0 + t)


def gauss_rule(n):
    t, w = npleg.leggauss(n)
    return 0.5 * (1.0 + t), 0.5 * w


def _bary_weights(nodes):
    n = len(nodes)
    w = np.ones(n)
    for i in range(n):
        for j in range(n):
            if i != j:
                w[i] /= (nodes[i] - nodes[j])
    return w


def basis_1d(nodes, x):
    """Values and derivatives of the Lagrange basis at points x, by the
    barycentric formula and the nodal differentiation matrix."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    w = _bary_weights(nodes)
    val = np.zeros((x.size, n))
    for a, xa in enumerate(x):
        hit = np.where(xa == nodes)[0]
        if hit.size:
            val[a, hit[0]] = 1.0
            continue
        t = w / (xa - nodes)
        val[a] = t / t.sum()
    # D[m, i] = phi_i'(x_m)
    D = np.zeros((n, n))
    for m in range(n):
        for i in range(n):
            if i != m:
                D[m, i] = (w[i] / w[m]) / (nodes[m] - nodes[i])
        D[m, m] = -D[m].sum()
    der = val @ D
    return val, der


def exact_1d_matrices(k):
    """Reference 1D stiffness and mass on [0,1]; the integrands are
    polynomials of degree <= 2k, integrated exactly by a 24-point rule."""
    nodes = gll_nodes(k)
    xq, wq = gauss_rule(24)
    val, der = basis_1d(nodes, xq)
    M = (val * wq[:, None]).T @ val
    K = (der * wq[:, None]).T @ der
    return K, M


def gll_weights_exact(k):
    """GLL quadrature weights as the exact integrals of the nodal Lagrange
    basis over [0,1] (24-point Gauss rule on degree-k polynomials)."""
    xq, wq = gauss_rule(24)
    val, _ = basis_1d(gll_nodes(k), xq)
    return wq @ val


def global_1d(k, ncell, h, lumped=False):
    """Assembled 1D stiffness/mass on a uniform lattice of ncell cells of size h.
    lumped: the mass of (k+1)-point GLL quadrature at the nodes (diagonal,
    the basis integrals); the stiffness is exact under that rule too."""
    K, M = exact_1d_matrices(k)
    if lumped:
        M = np.diag(gll_weights_exact(k))
    n = ncell * k + 1
    Kg = np.zeros((n, n))
    Mg = np.zeros((n, n))
    for c in range(ncell):
        s = slice(c * k, c * k + k + 1)
        Kg[s, s] += K / h
        Mg[s, s] += M * h
    return Kg, Mg


def kronecker_laplacian(k, ncells, lumped=False):
    """A = Kz(x)My(x)Mx + Mz(x)Ky(x)Mx + Mz(x)My(x)Kx for the affine unit cube
    (lexicographic numbering, x fastest); lumped: GLL collocation."""
    nx, ny, nz = ncells
    Kx, Mx = global_1d(k, nx, 1.0 / nx, lumped)
    Ky, My = global_1d(k, ny, 1.0 / ny, lumped)
    Kz, Mz = global_1d(k, nz, 1.0 / nz, lumped)
    return (np.kron(Kz, np.kron(My, Mx)) + np.kron(Mz, np.kron(Ky, Mx))
            + np.kron(Mz, np.kron(My, Kx)))


def map_numpy(kind, amp, X):
    """The global maps (input definition), evaluated with numpy."""
    X = np.asarray(X, dtype=np.float64)
    s = np.sin(2 * np.pi * X)
    if kind == 0:
        return X.copy()
    if kind == 1:
        out = X.copy()
        for i in range(3):
            a, b = (i + 1) % 3, (i + 2) % 3
            out[..., i] += amp * s[..., a] * s[..., b]
        return out
    if kind == 2:
        return X + amp * np.prod(s, axis=-1, keepdims=True)
    raise ValueError(kind)


def fd_jacobian(kind, amp, X, h=1e-6):
    """Central-difference Jacobian dF/dX (fourth order)."""
    J = np.zeros(X.shape[:-1] + (3, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        f1 = map_numpy(kind, amp, X + e)
        f_1 = map_numpy(kind, amp, X - e)
        f2 = map_numpy(kind, amp, X + 2 * e)
        f_2 = map_numpy(kind, amp, X - 2 * e)
        J[..., :, j] = (8 * (f1 - f_1) - (f2 - f_2)) / (12 * h)
    return J


def quadratic_map_numpy(kind, amp, ncells, cell, xi):
    """The map's quadratic interpolant in one cell at reference points xi
    (shape (..., 3)): sum over the 27 points X_abd = (cell + (a, b, d)/2) / n
    of F(X_abd) N_a(xi_0) N_b(xi_1) N_d(xi_2), with the closed-form quadratic
    Lagrange basis on {0, 1/2, 1}."""
    xi = np.asarray(xi, dtype=np.float64)

    def basis(t):
        return np.stack([(2 * t - 1) * (t - 1), 4 * t * (1 - t), t * (2 * t - 1)], axis=-1)

    Nx, Ny, Nz = basis(xi[..., 0]), basis(xi[..., 1]), basis(xi[..., 2])
    out = np.zeros(xi.shape)
    n = np.asarray(ncells, dtype=np.float64)
    for d in range(3):
        for b in range(3):
            for a in range(3):
                X = (np.asarray(cell, dtype=np.float64) + np.array([a, b, d]) / 2.0) / n
                F = map_numpy(kind, amp, X)
                out += F * (Nx[..., a] * Ny[..., b] * Nz[..., d])[..., None]
    return out


def quadratic_jacobian(kind, amp, ncells, cell, xi, h=1e-2):
    """dx/dxi of the quadratic interpolant by central differences, which
    are exact for a polynomial of degree 2 in the differentiated variable."""
    J = np.zeros((3, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, j] = (quadratic_map_numpy(kind, amp, ncells, cell, xi + e)
                   - quadratic_map_numpy(kind, amp, ncells, cell, xi - e)) / (2 * h)
    return J


def kronecker_mass(k, ncells, lumped=False):
    """Mass matrix Mz(x)My(x)Mx of the affine unit cube."""
    nx, ny, nz = ncells
    _, Mx = global_1d(k, nx, 1.0 / nx, lumped)
    _, My = global_1d(k, ny, 1.0 / ny, lumped)
    _, Mz = global_1d(k, nz, 1.0 / nz, lumped)
    return np.kron(Mz, np.kron(My, Mx))


def element_mass_fd(k, ncells, cell, kind, amp, a_e=1.0, nq1=None):
    """Element mass matrix with numpy's nq1-point Gauss rule (default k+1)
    and an FD Jacobian determinant."""
    nodes = gll_nodes(k)
    nq1 = k + 1 if nq1 is None else nq1
    xq, wq = gauss_rule(nq1)
    val, _ = basis_1d(nodes, xq)
    n = k + 1
    ncells = np.asarray(ncells, dtype=np.float64)
    A = np.zeros((n ** 3, n ** 3))
    for qz in range(nq1):
        for qy in range(nq1):
            for qx in range(nq1):
                X = (np.asarray(cell) + np.array([xq[qx], xq[qy], xq[qz]])) / ncells
                det = np.linalg.det(fd_jacobian(kind, amp, X) / ncells[None, :])
                phi = np.einsum("k,j,i->kji", val[qz], val[qy], val[qx]).ravel()
                A += a_e * wq[qx] * wq[qy] * wq[qz] * det * np.outer(phi, phi)
    return A


def element_matrix_fd(k, nq1, ncells, cell, kind, amp, a_e=1.0, quad="gauss", geometry="exact"):
    """Element stiffness matrix with numpy's rules and an FD Jacobian
    (quad "gll": the k+1 nodes with the basis integrals as weights;
    geometry "quadratic": the Jacobian of the map's quadratic interpolant)."""
    nodes = gll_nodes(k)
    if quad == "gll":
        nq1 = k + 1
        xq, wq = nodes, gll_weights_exact(k)
    else:
        xq, wq = gauss_rule(nq1)
    val, der = basis_1d(nodes, xq)  # [q, i]
    n = k + 1
    nb = n ** 3
    ncells = np.asarray(ncells, dtype=np.float64)
    A = np.zeros((nb, nb))
    for qz in range(nq1):
        for qy in range(nq1):
            for qx in range(nq1):
                xi = np.array([xq[qx], xq[qy], xq[qz]])
                X = (np.asarray(cell) + xi) / ncells
                if geometry == "quadratic":
                    J = quadratic_jacobian(kind, amp, ncells, cell, xi)
                else:
                    J = fd_jacobian(kind, amp, X) / ncells[None, :]
                det = np.linalg.det(J)
                Jinv = np.linalg.inv(J)
                w = wq[qx] * wq[qy] * wq[qz] * det * a_e
                G = np.zeros((nb, 3))
                for iz in range(n):
                    for iy in range(n):
                        for ix in range(n):
                            i = ix + n * (iy + n * iz)
                            gr = np.array([der[qx, ix] * val[qy, iy] * val[qz, iz],
                                           val[qx, ix] * der[qy, iy] * val[qz, iz],
                                           val[qx, ix] * val[qy, iy] * der[qz, iz]])
                            G[i] = Jinv.T @ gr
                A += w * G @ G.T
    return A
