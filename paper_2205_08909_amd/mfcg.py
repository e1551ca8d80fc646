"""Thin ctypes binding of libmfcg.so (include/mfcg.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  Device vectors are torch CUDA (HIP) tensors of dtype float64;
streams are torch streams.  Loading fails loudly when the library is not
built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MFCG_LIBRARY selects another build of the same library (the host-sanitizer
# build of the CPU tests)
LIB_PATH = os.environ.get("MFCG_LIBRARY") or os.path.join(HERE, "libmfcg.so")

OK, EINVAL, ENOMEM, EHIP, ENOTCONV, EBREAKDOWN, ESTAGNATION = 0, -1, -2, -3, -4, -5, -6
MAP_AFFINE, MAP_SINE_SHEAR, MAP_SINE_PRODUCT = 0, 1, 2
BC_DIRICHLET0, BC_NONE = 0, 1
RHS_SINE, RHS_BUMPS = 0, 1
SOLVER_FUSED, SOLVER_ALG5_SPLIT, SOLVER_PCG_BASIC, SOLVER_PIPELINED, SOLVER_SSTEP = 0, 1, 2, 3, 4
PRECOND_JACOBI, PRECOND_NONE = 0, 1
QUAD_GAUSS, QUAD_GLL = 0, 1
OP_LAPLACE, OP_MASS = 0, 1
GEOM_STORED, GEOM_QUADRATIC = 0, 1

EXPORTED = [
    "mfcg_setup", "mfcg_n_dofs", "mfcg_vmult", "mfcg_diagonal", "mfcg_assemble_rhs", "mfcg_solve",
    "mfcg_cg_begin", "mfcg_cg_iterate", "mfcg_cg_end", "mfcg_set_timing", "mfcg_get_timing",
    "mfcg_layout_info", "mfcg_layout_permutation", "mfcg_destroy", "mfcg_error_string", "mfcg_last_error",
    "mfcg_stream_bench", "mfcg_solve_ir", "mfcg_set_solver", "mfcg_set_coefficient", "mfcg_warmstart",
    "mfcg_autotune_tile", "mfcg_batch_setup", "mfcg_batch_info", "mfcg_batch_solve", "mfcg_batch_destroy",
    "mfcg_batch_last_error", "mfcg_set_sstep", "mfcg_set_preconditioner", "mfcg_solve_vector",
    "mfcg_vmult_fp32", "mfcg_setup_batch", "mfcg_solve_batch", "mfcg_solve_multi", "mfcg_warmstart_span",
    "mfcg_interpolate",
]
MULTI_MAX = 64
SPAN_MAX = 8


class MfcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mfcg error {code}: {msg}")
        self.code = code


class Mesh(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int32 * 3), ("map_kind", ctypes.c_int32), ("map_amplitude", ctypes.c_double),
                ("bc", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("n_q_1d", ctypes.c_int32), ("tile", ctypes.c_int32 * 3), ("check_every", ctypes.c_int32),
                ("fp32", ctypes.c_int32), ("quad_rule", ctypes.c_int32), ("op", ctypes.c_int32),
                ("geometry", ctypes.c_int32), ("deterministic", ctypes.c_int32), ("tune_cache", ctypes.c_char_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2205_08909_amd.build` "
                               "(or __graft_entry__.build())")
        # torch brings its own HIP runtime; it must own the device before this
        # library's runtime (the system one) is loaded, or the latter can find
        # no device when it is the first to initialise
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.mfcg_setup.argtypes = [ctypes.POINTER(Mesh), I32, P, ctypes.POINTER(Options), P, ctypes.POINTER(P)]
        L.mfcg_n_dofs.argtypes = [P, ctypes.POINTER(I64)]
        L.mfcg_vmult.argtypes = [P, P, P, P]
        L.mfcg_diagonal.argtypes = [P, P, P]
        L.mfcg_assemble_rhs.argtypes = [P, I32, P, P, P]
        L.mfcg_solve.argtypes = [P, P, P, D, I32, ctypes.POINTER(I32), P, P, P]
        L.mfcg_cg_begin.argtypes = [P, P, P, D, I32, P]
        L.mfcg_cg_iterate.argtypes = [P, I32, P]
        L.mfcg_cg_end.argtypes = [P, P, ctypes.POINTER(I32), P, P]
        L.mfcg_set_timing.argtypes = [P, I32]
        L.mfcg_get_timing.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(I64), ctypes.POINTER(D),
                                      ctypes.POINTER(I64)]
        L.mfcg_layout_info.argtypes = [P, P, P, P, P, P, P]
        L.mfcg_layout_permutation.argtypes = [ctypes.POINTER(Mesh), I32, P, P, P, P, P]
        L.mfcg_destroy.argtypes = [P]
        L.mfcg_stream_bench.argtypes = [I32, I64, P, P, I32, P]
        L.mfcg_solve_ir.argtypes = [P, P, P, D, D, I32, I32, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), P, P, P]
        L.mfcg_set_solver.argtypes = [P, I32]
        L.mfcg_set_sstep.argtypes = [P, I32]
        L.mfcg_set_preconditioner.argtypes = [P, I32]
        L.mfcg_solve_vector.argtypes = [P, P, P, D, I32, ctypes.POINTER(I32), P, P, P]
        L.mfcg_solve_multi.argtypes = [P, I32, P, P, D, I32, P, P, P, P]
        L.mfcg_warmstart_span.argtypes = [P, P, I32, P, D, P, P, P, P, P]
        L.mfcg_interpolate.argtypes = [P, P, P, P, P]
        L.mfcg_set_coefficient.argtypes = [P, P, P]
        L.mfcg_warmstart.argtypes = [P, P, P, D, P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I32), P]
        L.mfcg_autotune_tile.argtypes = [ctypes.POINTER(Mesh), I32, I32, P, ctypes.POINTER(D), P]
        L.mfcg_batch_setup.argtypes = [I32, P, P, P, I32, P, ctypes.POINTER(P)]
        L.mfcg_setup_batch.argtypes = [I32, P, P, P, ctypes.POINTER(Options), P, ctypes.POINTER(P)]
        L.mfcg_solve_batch.argtypes = [P, P, P, D, I32, P, P, P]
        L.mfcg_vmult_fp32.argtypes = [P, P, P, P]
        L.mfcg_batch_info.argtypes = [P, I32, ctypes.POINTER(P), P]
        L.mfcg_batch_solve.argtypes = [P, P, P, D, I32, P, P, P]
        L.mfcg_batch_destroy.argtypes = [P]
        L.mfcg_batch_last_error.argtypes = [P]
        L.mfcg_batch_last_error.restype = ctypes.c_char_p
        L.mfcg_error_string.argtypes = [ctypes.c_int]
        L.mfcg_error_string.restype = ctypes.c_char_p
        L.mfcg_last_error.argtypes = [P]
        L.mfcg_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code, handle=None):
    if code != OK:
        msg = lib().mfcg_last_error(handle).decode()
        raise MfcgError(code, msg)
    return code


def make_mesh(cells, map_kind=MAP_AFFINE, amplitude=0.0, bc=BC_DIRICHLET0):
    if np.isscalar(cells):
        cells = (cells, cells, cells)
    m = Mesh()
    for d in range(3):
        m.cells[d] = int(cells[d])
    m.map_kind = int(map_kind)
    m.map_amplitude = float(amplitude)
    m.bc = int(bc)
    return m


def make_options(tile=None, check_every=0, fp32=0, quad=QUAD_GAUSS, op=OP_LAPLACE, n_q_1d=0, geometry=GEOM_STORED,
                 tune_cache=None):
    o = Options()
    o.tune_cache = None if tune_cache is None else str(tune_cache).encode()
    o.n_q_1d = int(n_q_1d)
    o.geometry = int(geometry)
    for d in range(3):
        o.tile[d] = 0 if tile is None else int(tile[d])
    o.check_every = int(check_every)
    o.fp32 = int(fp32)
    o.quad_rule = int(quad)
    o.op = int(op)
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_vec(t, n, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            and t.numel() == n):
        raise ValueError(f"{name} must be a contiguous float64 device tensor of length {n}")
    return t


def stream_bench(kind, src, dst, nblocks, stream=None):
    """Streaming reference kernel (kind 0 copy, 1 read) on float64 device tensors."""
    _check(lib().mfcg_stream_bench(int(kind), int(src.numel()), _ptr(src), _ptr(dst), int(nblocks), _stream(stream)))


def layout_permutation(cells, degree, tile=None, map_kind=MAP_AFFINE, bc=BC_DIRICHLET0):
    """Host-only: lexicographic -> internal permutation and class counts."""
    m = make_mesh(cells, map_kind, 0.0, bc)
    n = 1
    for c in (cells if not np.isscalar(cells) else (cells,) * 3):
        n *= int(c) * degree + 1
    perm = np.zeros(n, dtype=np.int64)
    t = (ctypes.c_int32 * 3)(*(tile or (0, 0, 0)))
    nI, nS, nC = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().mfcg_layout_permutation(ctypes.byref(m), int(degree), ctypes.cast(t, ctypes.c_void_p),
                                         perm.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nI), ctypes.byref(nS),
                                         ctypes.byref(nC)))
    return perm, nI.value, nS.value, nC.value


class Problem:
    """mfcg_setup on a mesh + degree + per-cell coefficient."""

    def __init__(self, cells, degree, coeff=None, map_kind=MAP_AFFINE, amplitude=0.0, bc=BC_DIRICHLET0, tile=None,
                 check_every=0, stream=None, quad=QUAD_GAUSS, op=OP_LAPLACE, n_q_1d=0, geometry=GEOM_STORED, fp32=0):
        self.mesh = make_mesh(cells, map_kind, amplitude, bc)
        self.degree = int(degree)
        self.opt = make_options(tile, check_every, fp32=fp32, quad=quad, op=op, n_q_1d=n_q_1d, geometry=geometry)
        self.h = ctypes.c_void_p()
        self._coeff = None
        if coeff is not None:
            self._coeff = np.ascontiguousarray(coeff, dtype=np.float64).ravel()
        cptr = self._coeff.ctypes.data_as(ctypes.c_void_p) if self._coeff is not None else None
        _check(lib().mfcg_setup(ctypes.byref(self.mesh), self.degree, cptr, ctypes.byref(self.opt),
                                _stream(stream), ctypes.byref(self.h)))
        n = ctypes.c_int64()
        _check(lib().mfcg_n_dofs(self.h, ctypes.byref(n)), self.h)
        self.n = n.value

    def close(self):
        if self.h:
            lib().mfcg_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self):
        import torch
        return torch.empty(self.n, dtype=torch.float64, device="cuda")

    def vmult(self, dst, src, stream=None):
        _dev_vec(dst, self.n, "dst")
        _dev_vec(src, self.n, "src")
        _check(lib().mfcg_vmult(self.h, _ptr(dst), _ptr(src), _stream(stream)), self.h)
        return dst

    def vmult_fp32(self, dst, src, stream=None):
        """dst = A32 src with the single-precision operator of the mixed-precision solver."""
        _dev_vec(dst, self.n, "dst")
        _dev_vec(src, self.n, "src")
        _check(lib().mfcg_vmult_fp32(self.h, _ptr(dst), _ptr(src), _stream(stream)), self.h)
        return dst

    def diagonal(self, out=None, stream=None):
        out = self.empty() if out is None else _dev_vec(out, self.n, "out")
        _check(lib().mfcg_diagonal(self.h, _ptr(out), _stream(stream)), self.h)
        return out

    def rhs(self, kind=RHS_SINE, params=None, out=None, stream=None):
        out = self.empty() if out is None else _dev_vec(out, self.n, "out")
        p = None
        if params is not None:
            self._params = np.ascontiguousarray(params, dtype=np.float64)
            p = self._params.ctypes.data_as(ctypes.c_void_p)
        _check(lib().mfcg_assemble_rhs(self.h, int(kind), p, _ptr(out), _stream(stream)), self.h)
        return out

    def solve(self, b, x, tol=1e-10, maxit=10000, want_hist=True, want_true_res=False, stream=None, raise_on=True):
        """Returns (code, iters, hist, true_rel_res); x is overwritten."""
        _dev_vec(b, self.n, "b")
        _dev_vec(x, self.n, "x")
        its = ctypes.c_int32()
        hist = np.zeros(maxit + 1) if want_hist else None
        tr = ctypes.c_double(float("nan"))
        code = lib().mfcg_solve(self.h, _ptr(b), _ptr(x), float(tol), int(maxit), ctypes.byref(its),
                                hist.ctypes.data_as(ctypes.c_void_p) if want_hist else None,
                                ctypes.byref(tr) if want_true_res else None, _stream(stream))
        if raise_on and code not in (OK, ENOTCONV):
            _check(code, self.h)
        h = hist[: its.value + 1].copy() if want_hist else None
        return code, its.value, h, tr.value

    def solve_vector(self, b, x, tol=1e-10, maxit=10000, want_hist=True, want_true_res=False, stream=None,
                     raise_on=True):
        """Vector Laplacian (three uncoupled components, BP4 family): b and x
        hold 3n entries, component-blocked.  Returns (code, iters, hist,
        true_rel_res); x is overwritten."""
        _dev_vec(b, 3 * self.n, "b")
        _dev_vec(x, 3 * self.n, "x")
        its = ctypes.c_int32()
        hist = np.zeros(maxit + 1) if want_hist else None
        tr = ctypes.c_double(float("nan"))
        code = lib().mfcg_solve_vector(self.h, _ptr(b), _ptr(x), float(tol), int(maxit), ctypes.byref(its),
                                       hist.ctypes.data_as(ctypes.c_void_p) if want_hist else None,
                                       ctypes.byref(tr) if want_true_res else None, _stream(stream))
        if raise_on and code not in (OK, ENOTCONV):
            _check(code, self.h)
        h = hist[: its.value + 1].copy() if want_hist else None
        return code, its.value, h, tr.value

    def solve_multi(self, bs, xs, tol=1e-10, maxit=10000, want_true_res=False, stream=None, raise_on=True):
        """m independent right-hand sides on this operator, advanced together
        (one fused launch per iteration over all (tile, right-hand side)
        pairs).  xs hold the initial guesses and are overwritten.  Returns
        (code, iters[], status[], true_rel_res[] or None)."""
        m = len(bs)
        if m != len(xs) or not 1 <= m <= MULTI_MAX:
            raise ValueError(f"need 1..{MULTI_MAX} right-hand sides and as many solution vectors")
        for i, (b, x) in enumerate(zip(bs, xs)):
            _dev_vec(b, self.n, f"b[{i}]")
            _dev_vec(x, self.n, f"x[{i}]")
        bp = (ctypes.c_void_p * m)(*[b.data_ptr() for b in bs])
        xp = (ctypes.c_void_p * m)(*[x.data_ptr() for x in xs])
        its = (ctypes.c_int32 * m)()
        st = (ctypes.c_int32 * m)()
        tr = (ctypes.c_double * m)(*([float("nan")] * m))
        code = lib().mfcg_solve_multi(self.h, m, bp, xp, float(tol), int(maxit), its, st,
                                      tr if want_true_res else None, _stream(stream))
        if raise_on and code not in (OK, ENOTCONV, EBREAKDOWN):
            _check(code, self.h)
        return code, list(its), list(st), (list(tr) if want_true_res else None)

    def solve_ir(self, b, x, tol=1e-10, inner_tol=1e-4, max_outer=20, max_inner=10000, keep_direction=False,
                 stream=None, raise_on=True):
        """FP64 iterative refinement around the FP32 fused solver.
        Returns (code, outer_its, inner_its, rel_res_hist, true_rel_res)."""
        _dev_vec(b, self.n, "b")
        _dev_vec(x, self.n, "x")
        oi, ii = ctypes.c_int32(), ctypes.c_int32()
        hist = np.zeros(max_outer + 1)
        tr = ctypes.c_double(float("nan"))
        code = lib().mfcg_solve_ir(self.h, _ptr(b), _ptr(x), float(tol), float(inner_tol), int(max_outer),
                                   int(max_inner), 1 if keep_direction else 0, ctypes.byref(oi), ctypes.byref(ii),
                                   hist.ctypes.data_as(ctypes.c_void_p), ctypes.byref(tr), _stream(stream))
        if raise_on and code != OK:
            _check(code, self.h)
        return code, oi.value, ii.value, hist[: oi.value + 1].copy(), tr.value

    # stepping interface (throughput measurement)
    def cg_begin(self, b, x0=None, tol=0.0, maxit=100, stream=None):
        _dev_vec(b, self.n, "b")
        if x0 is not None:
            _dev_vec(x0, self.n, "x0")
        _check(lib().mfcg_cg_begin(self.h, _ptr(b), _ptr(x0), float(tol), int(maxit), _stream(stream)), self.h)

    def cg_iterate(self, n, stream=None):
        _check(lib().mfcg_cg_iterate(self.h, int(n), _stream(stream)), self.h)

    def cg_end(self, x, want_hist=False, maxit=None, stream=None):
        _dev_vec(x, self.n, "x")
        its = ctypes.c_int32()
        hist = np.zeros((maxit or 100000) + 1) if want_hist else None
        code = lib().mfcg_cg_end(self.h, _ptr(x), ctypes.byref(its),
                                 hist.ctypes.data_as(ctypes.c_void_p) if want_hist else None, _stream(stream))
        return code, its.value, (hist[: its.value + 1] if want_hist else None)

    def set_coefficient(self, coeff=None, stream=None):
        """New cell coefficient (None: a = 1); rebuilds G_q and the diagonal."""
        self._coeff = None if coeff is None else np.ascontiguousarray(coeff, dtype=np.float64).ravel()
        cptr = self._coeff.ctypes.data_as(ctypes.c_void_p) if self._coeff is not None else None
        _check(lib().mfcg_set_coefficient(self.h, cptr, _stream(stream)), self.h)

    def warmstart(self, b, u, max_rel_res=float("inf"), x0=None, stream=None):
        """x0 = s u' (Galerkin-scaled, Dirichlet entries zeroed) or 0.
        Returns (x0, scale, rel_res, used)."""
        _dev_vec(b, self.n, "b")
        _dev_vec(u, self.n, "u")
        x0 = self.empty() if x0 is None else _dev_vec(x0, self.n, "x0")
        sc, rr = ctypes.c_double(), ctypes.c_double()
        used = ctypes.c_int32()
        _check(lib().mfcg_warmstart(self.h, _ptr(b), _ptr(u), float(max_rel_res), _ptr(x0), ctypes.byref(sc),
                                    ctypes.byref(rr), ctypes.byref(used), _stream(stream)), self.h)
        return x0, sc.value, rr.value, bool(used.value)

    def warmstart_span(self, b, us, max_rel_res=float("inf"), x0=None, stream=None):
        """x0 in span(us) with the A-norm optimal coefficients (Dirichlet
        entries zeroed first).  Returns (x0, coef, rel_res, used)."""
        m = len(us)
        if not 1 <= m <= SPAN_MAX:
            raise ValueError(f"need 1..{SPAN_MAX} vectors")
        _dev_vec(b, self.n, "b")
        for i, u in enumerate(us):
            _dev_vec(u, self.n, f"u[{i}]")
        x0 = self.empty() if x0 is None else _dev_vec(x0, self.n, "x0")
        up = (ctypes.c_void_p * m)(*[u.data_ptr() for u in us])
        coef = (ctypes.c_double * m)()
        rr = ctypes.c_double()
        used = ctypes.c_int32()
        _check(lib().mfcg_warmstart_span(self.h, _ptr(b), m, up, float(max_rel_res), _ptr(x0), coef, ctypes.byref(rr),
                                         ctypes.byref(used), _stream(stream)), self.h)
        return x0, list(coef), rr.value, bool(used.value)

    def interpolate_from(self, other, src, dst=None, stream=None):
        """dst = the finite-element function of handle `other` (nodal values
        src) at this handle's nodes (same cells)."""
        _dev_vec(src, other.n, "src")
        dst = self.empty() if dst is None else _dev_vec(dst, self.n, "dst")
        _check(lib().mfcg_interpolate(other.h, _ptr(src), self.h, _ptr(dst), _stream(stream)), self.h)
        return dst

    def set_solver(self, solver):
        """SOLVER_FUSED (default), SOLVER_ALG5_SPLIT, SOLVER_PCG_BASIC,
        SOLVER_PIPELINED or SOLVER_SSTEP (the last two unpreconditioned)."""
        _check(lib().mfcg_set_solver(self.h, int(solver)), self.h)

    def set_preconditioner(self, precond):
        """PRECOND_JACOBI (default) or PRECOND_NONE (fused, split and basic solvers)."""
        _check(lib().mfcg_set_preconditioner(self.h, int(precond)), self.h)

    def set_sstep(self, s):
        """Block size of SOLVER_SSTEP, 1..8 (default 6)."""
        _check(lib().mfcg_set_sstep(self.h, int(s)), self.h)

    def set_timing(self, on=True):
        _check(lib().mfcg_set_timing(self.h, 1 if on else 0), self.h)

    def get_timing(self):
        fm, sm = ctypes.c_double(), ctypes.c_double()
        fl, sl = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().mfcg_get_timing(self.h, ctypes.byref(fm), ctypes.byref(fl), ctypes.byref(sm),
                                     ctypes.byref(sl)), self.h)
        return {"fused_ms": fm.value, "fused_launches": fl.value, "shared_ms": sm.value, "shared_launches": sl.value}

    def layout_info(self):
        t = (ctypes.c_int32 * 3)()
        vals = [ctypes.c_int64() for _ in range(5)]
        _check(lib().mfcg_layout_info(self.h, ctypes.cast(t, ctypes.c_void_p), *[ctypes.byref(v) for v in vals]),
               self.h)
        return {"tile": tuple(t), "n_interior": vals[0].value, "n_shared": vals[1].value,
                "n_dirichlet": vals[2].value, "n_tiles": vals[3].value, "geometry_bytes": vals[4].value}


def autotune_tile(cells, degree, map_kind=MAP_AFFINE, amplitude=0.0, iters=6, stream=None):
    """(tile, ms_per_iter) of the fastest candidate tile for this mesh and degree."""
    m = make_mesh(cells, map_kind, amplitude)
    t = (ctypes.c_int32 * 3)()
    ms = ctypes.c_double()
    _check(lib().mfcg_autotune_tile(ctypes.byref(m), int(degree), int(iters), t, ctypes.byref(ms), _stream(stream)))
    return tuple(t), ms.value


class _View(Problem):
    """A problem owned by a Batch (no setup, no destroy)."""

    def __init__(self, h):
        self.h = h
        self.degree = None
        n = ctypes.c_int64()
        _check(lib().mfcg_n_dofs(self.h, ctypes.byref(n)), self.h)
        self.n = n.value

    def close(self):
        self.h = ctypes.c_void_p()


class Batch:
    """Independent problems solved together (mfcg_batch_*).
    problems: list of dicts with cells, degree and optional coeff, map_kind,
    amplitude, bc."""

    def __init__(self, problems, autotune=True, stream=None, tile=None, tune_cache=None):
        np_ = len(problems)
        meshes = (Mesh * np_)()
        degs = (ctypes.c_int32 * np_)()
        self._coeffs = []
        cptrs = (ctypes.c_void_p * np_)()
        for i, p in enumerate(problems):
            meshes[i] = make_mesh(p["cells"], p.get("map_kind", MAP_AFFINE), p.get("amplitude", 0.0),
                                  p.get("bc", BC_DIRICHLET0))
            degs[i] = int(p["degree"])
            c = p.get("coeff")
            if c is not None:
                c = np.ascontiguousarray(c, dtype=np.float64).ravel()
                self._coeffs.append(c)
                cptrs[i] = c.ctypes.data
            else:
                cptrs[i] = None
        self.h = ctypes.c_void_p()
        if tile is not None or tune_cache is not None:
            # the options form: a fixed tile for every problem, or the autotuner with its cache
            self._opt = make_options(tile=tile, tune_cache=tune_cache)
            code = lib().mfcg_setup_batch(np_, meshes, degs, cptrs, ctypes.byref(self._opt), _stream(stream),
                                          ctypes.byref(self.h))
        else:
            code = lib().mfcg_batch_setup(np_, meshes, degs, cptrs, 1 if autotune else 0, _stream(stream),
                                          ctypes.byref(self.h))
        if code != OK:
            raise MfcgError(code, lib().mfcg_batch_last_error(None).decode())
        self.nprob = np_
        self.problems = []
        self.tiles = []
        for i in range(np_):
            hh = ctypes.c_void_p()
            t = (ctypes.c_int32 * 3)()
            self._chk(lib().mfcg_batch_info(self.h, i, ctypes.byref(hh), t))
            self.problems.append(_View(hh))
            self.tiles.append(tuple(t))

    def _chk(self, code):
        if code != OK:
            raise MfcgError(code, lib().mfcg_batch_last_error(self.h).decode())

    def solve(self, bs, xs, tol=1e-10, maxit=10000, stream=None):
        """Returns (code, iters[], status[]); xs are overwritten."""
        for i, (b, x) in enumerate(zip(bs, xs)):
            _dev_vec(b, self.problems[i].n, f"b[{i}]")
            _dev_vec(x, self.problems[i].n, f"x[{i}]")
        bp = (ctypes.c_void_p * self.nprob)(*[b.data_ptr() for b in bs])
        xp = (ctypes.c_void_p * self.nprob)(*[x.data_ptr() for x in xs])
        its = (ctypes.c_int32 * self.nprob)()
        st = (ctypes.c_int32 * self.nprob)()
        code = lib().mfcg_batch_solve(self.h, bp, xp, float(tol), int(maxit), its, st, _stream(stream))
        if code not in (OK, ENOTCONV, EBREAKDOWN):
            self._chk(code)
        return code, list(its), list(st)

    def close(self):
        if self.h:
            for p in self.problems:
                p.close()
            lib().mfcg_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
