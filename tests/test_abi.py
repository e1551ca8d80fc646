"""Host-side checks of the C-ABI library: it loads, exports every function
that include/mfcg.h and include/mfnn.h declare, rejects invalid arguments before any HIP call,
and its enumeration of unknowns (tile interiors, shared nodes, Dirichlet
nodes; the GPU form of the paper's Sec. 5.3 numbering) is a bijection with
the class sizes given by closed forms."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2205_08909_amd import mfcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="mfcg.h", prefix="mfcg_"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = mfcg.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(mfcg.EXPORTED)


def test_network_library_exports_every_declared_symbol():
    from paper_2205_08909_amd import nn
    L = nn.lib()
    names = declared_functions("mfnn.h", "mfnn_")
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(nn.EXPORTED)


def test_network_calls_reject_bad_descriptors():
    """Validation happens on the host: no tensor is touched."""
    from paper_2205_08909_amd import nn
    L = nn.lib()
    d = nn.desc(1, 3, 32, (145, 145, 145), 4, 4, 2, 1)
    assert tuple(d.out) == (37, 37, 37)
    bad = nn.ConvDesc.from_buffer_copy(d)
    bad.out[1] = 36
    fake = ctypes.c_void_p(64)
    assert L.mfnn_conv3d_fwd(ctypes.byref(bad), fake, 0, fake, None, 0, fake, 0, None) == nn.EINVAL
    assert b"out !=" in L.mfnn_last_error()
    big = nn.desc(1, 32, 64, (16, 16, 16), 8, 1, 0, 1)  # 32*512*8 floats of LDS > 64 KiB
    assert L.mfnn_conv3d_fwd(ctypes.byref(big), fake, 0, fake, None, 0, fake, 0, None) == nn.EINVAL
    assert L.mfnn_conv3d_fwd(ctypes.byref(d), fake, 5, fake, None, 0, fake, 0, None) == nn.EINVAL
    assert L.mfnn_conv3d_fwd(ctypes.byref(d), fake, 0, fake, None, 7, fake, 0, None) == nn.EINVAL
    assert L.mfnn_conv3d_bwd_weight(ctypes.byref(d), fake, 0, fake, 0, fake, None, fake, 1, None) == nn.EINVAL
    assert L.mfnn_conv3d_bwd_weight_work(ctypes.byref(bad)) == -1
    assert L.mfnn_adam(10, fake, None, fake, fake, fake, 0, 1e-3, 0.9, 0.999, 1e-8, None) == nn.EINVAL
    assert L.mfnn_convert(10, fake, 3, fake, 0, None) == nn.EINVAL
    cells = (ctypes.c_int32 * 3)(4, 4, 0)
    assert L.mfnn_features(cells, 3, fake, fake, fake, fake, fake, None) == nn.EINVAL
    # the allocation-free weight gradient refuses a layer whose workspace exceeds its array
    wide = nn.desc(1, 256, 256, (8, 8, 8), 3, 1, 1, 1)
    assert L.mfnn_conv3d_bwd_weight_work(ctypes.byref(wide)) > nn.NOALLOC_WORK_FLOATS
    assert L.mfnn_conv3d_bwd_weight_noalloc(ctypes.byref(wide), fake, 0, fake, 0, fake, None, None) == nn.EINVAL
    assert b"workspace" in L.mfnn_last_error()
    assert L.mfnn_conv3d_bwd_weight_noalloc(ctypes.byref(bad), fake, 0, fake, 0, fake, None, None) == nn.EINVAL


def test_error_strings():
    L = mfcg.lib()
    for code in range(-6, 1):
        assert L.mfcg_error_string(code)


@pytest.mark.parametrize("cells,degree,bc,msg", [
    ((0, 4, 4), 2, 0, "cells"),
    ((4, 4, 4), 0, 0, "degree"),
    ((4, 4, 4), 9, 0, "degree"),
    ((4, 4, 4), 2, 7, "bc"),
])
def test_setup_rejects_invalid_arguments(cells, degree, bc, msg):
    L = mfcg.lib()
    m = mfcg.make_mesh(cells, 0, 0.0, bc)
    h = ctypes.c_void_p()
    rc = L.mfcg_setup(ctypes.byref(m), degree, None, None, None, ctypes.byref(h))
    assert rc == mfcg.EINVAL and not h.value
    assert msg in L.mfcg_last_error(None).decode()


def test_setup_rejects_meshes_beyond_32_bit_offsets():
    """The fused kernels index vectors with 32-bit offsets: a lattice of
    2^31 nodes or more is refused on the host, before any allocation or HIP
    call (here 1300^3 Q1 cells, 1301^3 = 2.2e9 nodes); one just below the
    limit passes the check (it then needs the GPU, so only the message of
    the first failure is compared)."""
    L = mfcg.lib()
    h = ctypes.c_void_p()
    m = mfcg.make_mesh((1300, 1300, 1300))
    assert L.mfcg_setup(ctypes.byref(m), 1, None, None, None, ctypes.byref(h)) == mfcg.EINVAL and not h.value
    assert "2^31" in L.mfcg_last_error(None).decode()
    m = mfcg.make_mesh((1290, 1290, 1290))   # 1291^3 = 2.15e9 >= 2^31
    assert L.mfcg_setup(ctypes.byref(m), 1, None, None, None, ctypes.byref(h)) == mfcg.EINVAL
    # the batch validates every problem the same way
    meshes = (mfcg.Mesh * 2)(mfcg.make_mesh((4, 4, 4)), mfcg.make_mesh((2000, 1100, 1000)))
    degs = (ctypes.c_int32 * 2)(2, 1)
    assert L.mfcg_setup_batch(2, meshes, degs, None, None, None, ctypes.byref(h)) == mfcg.EINVAL
    assert L.mfcg_batch_setup(2, meshes, degs, None, 1, None, ctypes.byref(h)) == mfcg.EINVAL


def test_interface_summary_names_are_exported():
    """The calls under the names of the interface summary (batch set-up and
    solve, the network's Adam step and MSE loss) are exported, and the batch
    set-up with options refuses operator variants a batch does not run."""
    from paper_2205_08909_amd import nn
    L = mfcg.lib()
    for name in ("mfcg_setup", "mfcg_vmult", "mfcg_diagonal", "mfcg_solve", "mfcg_solve_ir", "mfcg_setup_batch",
                 "mfcg_solve_batch", "mfcg_destroy", "mfcg_error_string", "mfcg_last_error", "mfnn_conv3d_fwd",
                 "mfnn_conv3d_bwd_data", "mfnn_conv3d_bwd_weight", "mfnn_adam_step", "mfnn_mse_loss"):
        assert hasattr(L, name), name
    meshes = (mfcg.Mesh * 1)(mfcg.make_mesh((4, 4, 4)))
    degs = (ctypes.c_int32 * 1)(2)
    h = ctypes.c_void_p()
    o = mfcg.make_options(op=mfcg.OP_MASS)
    assert L.mfcg_setup_batch(1, meshes, degs, None, ctypes.byref(o), None, ctypes.byref(h)) == mfcg.EINVAL
    o = mfcg.make_options(tile=(-1, 2, 2))
    assert L.mfcg_setup_batch(1, meshes, degs, None, ctypes.byref(o), None, ctypes.byref(h)) == mfcg.EINVAL
    fake = ctypes.c_void_p(64)
    assert nn.lib().mfnn_adam_step(10, fake, None, fake, fake, fake, 0, 1e-3, 0.9, 0.999, 1e-8, None) == nn.EINVAL
    assert nn.lib().mfnn_mse_loss(0, fake, fake, fake, fake, fake, None) == nn.EINVAL
    assert L.mfcg_vmult_fp32(None, fake, fake, None) == mfcg.EINVAL


def test_setup_rejects_bad_coefficient_and_tile():
    L = mfcg.lib()
    m = mfcg.make_mesh((2, 2, 2))
    h = ctypes.c_void_p()
    c = np.ones(8)
    c[3] = -1.0
    assert L.mfcg_setup(ctypes.byref(m), 2, c.ctypes.data_as(ctypes.c_void_p), None, None, ctypes.byref(h)) == mfcg.EINVAL
    c[3] = np.nan
    assert L.mfcg_setup(ctypes.byref(m), 2, c.ctypes.data_as(ctypes.c_void_p), None, None, ctypes.byref(h)) == mfcg.EINVAL
    o = mfcg.make_options(tile=(99, 1, 1))
    assert L.mfcg_setup(ctypes.byref(m), 2, None, ctypes.byref(o), None, ctypes.byref(h)) == mfcg.EINVAL
    o = mfcg.make_options()
    o.n_q_1d = 5
    assert L.mfcg_setup(ctypes.byref(m), 2, None, ctypes.byref(o), None, ctypes.byref(h)) == mfcg.EINVAL
    assert L.mfcg_setup(ctypes.byref(m), 2, None, None, None, None) == mfcg.EINVAL


@pytest.mark.parametrize("k", range(1, 9))
def test_setup_rejects_tiles_beyond_the_compiled_extent(k):
    """The fused kernel's LDS is sized for a compiled maximum tile extent
    per degree and direction (x and y may differ); one cell more in either
    direction is refused on the host, before any HIP call."""
    L = mfcg.lib()
    tx, ty, _ = mfcg_default_tile(k)
    m = mfcg.make_mesh((tx + 1, ty + 1, 2))
    h = ctypes.c_void_p()
    for tile in ((tx + 1, 1, 1), (1, ty + 1, 1), (tx + 1, ty + 1, 1)):
        o = mfcg.make_options(tile=tile)
        assert L.mfcg_setup(ctypes.byref(m), k, None, ctypes.byref(o), None, ctypes.byref(h)) == mfcg.EINVAL, tile


def test_null_handle_calls():
    L = mfcg.lib()
    n = ctypes.c_int64()
    assert L.mfcg_n_dofs(None, ctypes.byref(n)) == mfcg.EINVAL
    assert L.mfcg_vmult(None, None, None, None) == mfcg.EINVAL
    assert L.mfcg_solve(None, None, None, 1e-10, 10, None, None, None, None) == mfcg.EINVAL
    assert L.mfcg_destroy(None) == mfcg.OK
    # the later entry points validate on the host too
    assert L.mfcg_set_solver(None, 0) == mfcg.EINVAL
    assert L.mfcg_set_sstep(None, 6) == mfcg.EINVAL
    assert L.mfcg_set_preconditioner(None, 0) == mfcg.EINVAL
    assert L.mfcg_solve_vector(None, None, None, 1e-10, 10, None, None, None, None) == mfcg.EINVAL
    assert L.mfcg_set_coefficient(None, None, None) == mfcg.EINVAL
    d = ctypes.c_double()
    i = ctypes.c_int32()
    assert L.mfcg_warmstart(None, None, None, 1.0, None, ctypes.byref(d), ctypes.byref(d), ctypes.byref(i),
                            None) == mfcg.EINVAL
    oi, ii = ctypes.c_int32(), ctypes.c_int32()
    assert L.mfcg_solve_ir(None, None, None, 1e-10, 1e-4, 10, 10, 0, ctypes.byref(oi), ctypes.byref(ii), None, None,
                           None) == mfcg.EINVAL
    assert L.mfcg_batch_destroy(None) == mfcg.OK
    assert L.mfcg_batch_solve(None, None, None, 1e-10, 10, None, None, None) == mfcg.EINVAL
    assert L.mfcg_batch_info(None, 0, None, None) == mfcg.EINVAL
    its, st = (ctypes.c_int32 * 2)(), (ctypes.c_int32 * 2)()
    assert L.mfcg_solve_multi(None, 2, None, None, 1e-10, 10, its, st, None, None) == mfcg.EINVAL


def test_batch_and_autotune_reject_bad_arguments_on_the_host():
    L = mfcg.lib()
    out = ctypes.c_void_p()
    assert L.mfcg_batch_setup(0, None, None, None, 0, None, ctypes.byref(out)) == mfcg.EINVAL
    meshes = (mfcg.Mesh * 2)(mfcg.make_mesh(4), mfcg.make_mesh(4))
    degs = (ctypes.c_int32 * 2)(2, 9)
    assert L.mfcg_batch_setup(2, meshes, degs, None, 0, None, ctypes.byref(out)) == mfcg.EINVAL
    assert b"problem 1" in L.mfcg_batch_last_error(None)
    assert not out.value
    t = (ctypes.c_int32 * 3)()
    ms = ctypes.c_double()
    m = mfcg.make_mesh(4)
    assert L.mfcg_autotune_tile(ctypes.byref(m), 0, 4, t, ctypes.byref(ms), None) == mfcg.EINVAL
    assert L.mfcg_autotune_tile(ctypes.byref(m), 4, 0, t, ctypes.byref(ms), None) == mfcg.EINVAL


def _closed_form_counts(cells, k, tile, bc):
    n = np.prod([c * k + 1 for c in cells])
    nI = 1
    per_dim = []
    for c, t in zip(cells, tile):
        t = min(t, c)
        sizes = [min(t, c - j) for j in range(0, c, t)]
        per_dim.append(sum(s * k - 1 for s in sizes))
    nI = int(np.prod(per_dim))
    nC = int(n - np.prod([c * k - 1 for c in cells])) if bc == 0 else 0
    return int(n), nI, int(n - nI - nC), nC


@pytest.mark.parametrize("cells,k,tile,bc", [
    ((8, 8, 8), 2, (0, 0, 0), 0),
    ((5, 7, 9), 3, (2, 3, 4), 0),
    ((4, 4, 4), 4, (0, 0, 0), 1),
    ((3, 2, 5), 1, (2, 2, 2), 0),
    ((6, 5, 4), 8, (2, 1, 3), 0),
    ((1, 1, 1), 4, (0, 0, 0), 0),
    ((2, 3, 1), 5, (1, 2, 1), 1),
])
def test_enumeration_bijection_and_counts(cells, k, tile, bc):
    perm, nI, nS, nC = mfcg.layout_permutation(cells, k, tile=tile, bc=bc)
    n, cI, cS, cC = _closed_form_counts(cells, k, [t if t else 10 ** 9 for t in tile] if any(tile) else
                                        [mfcg_default_tile(k)[d] for d in range(3)], bc)
    assert (nI, nS, nC) == (cI, cS, cC)
    assert np.array_equal(np.sort(perm), np.arange(n))
    # Dirichlet nodes occupy the tail of the internal order; interior nodes the head
    L = [c * k + 1 for c in cells]
    gz, gy, gx = np.meshgrid(*[np.arange(v) for v in L[::-1]], indexing="ij")
    bnd = ((gx == 0) | (gx == L[0] - 1) | (gy == 0) | (gy == L[1] - 1) | (gz == 0) | (gz == L[2] - 1)).ravel()
    if bc == 0:
        assert np.all(perm[bnd] >= n - nC) and np.all(perm[~bnd] < n - nC)


def mfcg_default_tile(k):
    tx = {1: 8, 2: 8, 3: 8, 4: 4, 5: 4, 6: 2, 7: 2, 8: 2}[k]
    ty = {1: 8, 2: 8, 3: 4, 4: 4, 5: 3, 6: 2, 7: 2, 8: 1}[k]
    return (tx, ty, 16)


def test_tile_interior_blocks_are_contiguous():
    cells, k, tile = (4, 4, 4), 2, (2, 2, 2)
    perm, nI, nS, nC = mfcg.layout_permutation(cells, k, tile=tile)
    L = cells[0] * k + 1
    # tile (0,0,0) interior: lattice coords 1..3 in each direction -> internal 0..26, lexicographic
    idx = [perm[x + L * (y + L * z)] for z in range(1, 4) for y in range(1, 4) for x in range(1, 4)]
    assert idx == list(range(27))
