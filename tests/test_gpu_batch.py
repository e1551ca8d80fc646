"""Batches of independent problems (mfcg_batch_*) and the tile autotuner.

Checked: a batched solve gives every problem bitwise the iterates, the
iteration count and the solution of the single-problem solver with the
same tile (the batch runs the same per-problem arithmetic in the same
order); against the oracle, a down-scaled replica of the batched workload
(sides drawn from 2..7, degrees 2..6, random-field coefficient,
random-normal right-hand side) converges with iteration counts inside the
oracle's own summation-order range and solutions within 1e-10; problems
that converge early, a zero right-hand side and an iteration cap are
handled per problem.
"""
import numpy as np
import pytest

from paper_2205_08909_amd import inputs

from tests.test_gpu_solve import oracle_noise

pytestmark = pytest.mark.gpu


def _draw(seed, nprob, nmin, nmax, kmin=2, kmax=6):
    probs = inputs.batch_draw(seed, nprob, nmin, nmax, kmin, kmax)
    out = []
    for p in probs:
        N, k = p["N"], p["k"]
        out.append({"cells": (N, N, N), "degree": k, "map_kind": 1, "amplitude": 0.05,
                    "coeff": inputs.grf_coefficient(N, 0.1, 1.0, seed=p["seed"]), "seed": p["seed"]})
    return out


def test_batch_matches_single_solves_bitwise():
    import torch
    from paper_2205_08909_amd import mfcg
    probs = _draw(3, 6, 3, 12)
    B = mfcg.Batch(probs, autotune=False)
    bs = [torch.from_numpy(inputs.random_rhs(p["cells"][0], p["degree"], seed=p["seed"])).cuda() for p in probs]
    xs = [torch.zeros_like(b) for b in bs]
    code, its, st = B.solve(bs, xs, tol=1e-10, maxit=5000)
    assert code == mfcg.OK and all(s == mfcg.OK for s in st)
    for i, p in enumerate(probs):
        P = mfcg.Problem(p["cells"], p["degree"], coeff=p["coeff"], map_kind=1, amplitude=0.05, tile=B.tiles[i])
        x = torch.zeros_like(bs[i])
        c, it, _, _ = P.solve(bs[i], x, tol=1e-10, maxit=5000, want_hist=False)
        print(i, p["cells"][0], p["degree"], its[i], it)
        assert c == mfcg.OK and it == its[i]
        assert torch.equal(x, xs[i])
        P.close()
    B.close()


def test_batch_replica_against_oracle(oracle_mod):
    import torch
    from paper_2205_08909_amd import mfcg
    probs = _draw(0, 6, 2, 7)
    B = mfcg.Batch(probs, autotune=True)
    bs, refs = [], []
    for p in probs:
        m = oracle_mod.Mesh(p["cells"], p["degree"], map_kind=1, amp=0.05, coeff=p["coeff"])
        A = oracle_mod.assemble(m)
        b = inputs.random_rhs(p["cells"][0], p["degree"], seed=p["seed"])
        xo, its_o, _, _ = oracle_mod.pcg(A, A.diagonal(), b, tol=1e-10, maxit=5000)
        lo, hi, _ = oracle_noise(oracle_mod, A, b, nperm=2)
        bs.append(torch.from_numpy(b).cuda())
        refs.append((A, b, xo, lo, hi))
    xs = [torch.zeros_like(b) for b in bs]
    code, its, st = B.solve(bs, xs, tol=1e-10, maxit=5000)
    assert code == mfcg.OK
    for i, (A, b, xo, lo, hi) in enumerate(refs):
        x = xs[i].cpu().numpy()
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        res = np.linalg.norm(b - A.matvec(x)) / np.linalg.norm(b)
        print(i, probs[i]["cells"][0], probs[i]["degree"], B.tiles[i], its[i], (lo, hi), err, res)
        assert lo - 2 <= its[i] <= hi + 2
        assert err <= 1e-10 and res <= 2e-10
    B.close()


def test_batch_edge_cases():
    import torch
    from paper_2205_08909_amd import mfcg
    probs = _draw(5, 4, 3, 8)
    B = mfcg.Batch(probs, autotune=False)
    bs = [torch.from_numpy(inputs.random_rhs(p["cells"][0], p["degree"], seed=p["seed"])).cuda() for p in probs]
    bs[1].zero_()
    xs = [torch.zeros_like(b) for b in bs]
    code, its, st = B.solve(bs, xs, tol=1e-10, maxit=5000)
    assert code == mfcg.OK and its[1] == 0 and torch.count_nonzero(xs[1]).item() == 0
    # an iteration cap hits the slow problems only
    xs = [torch.zeros_like(b) for b in bs]
    cap = sorted(its)[2]
    code, its2, st2 = B.solve(bs, xs, tol=1e-10, maxit=cap)
    assert code == mfcg.ENOTCONV
    for i in range(4):
        if its[i] <= cap:
            assert st2[i] == mfcg.OK and its2[i] == its[i]
        else:
            assert st2[i] == mfcg.ENOTCONV and its2[i] == cap
    B.close()


def test_autotune_returns_a_candidate():
    from paper_2205_08909_amd import mfcg
    tile, ms = mfcg.autotune_tile(12, 4, map_kind=1, amplitude=0.05, iters=3)
    assert ms > 0
    # x/y: the compiled maximum (4) or half of it; z: 8, 12 (clipped 16/32, or 1 layer), or the
    # mesh split into 2..12 equal layers of at least 2 cells: 6, 4, 3, 2
    assert tile[:2] in ((4, 4), (2, 2)) and tile[2] in (2, 3, 4, 6, 8, 12)


@pytest.mark.parametrize("k,ext", [(3, (8, 4)), (5, (4, 3)), (8, (2, 1))])
def test_autotune_candidates_keep_the_per_axis_extents(k, ext):
    """Degrees whose compiled tile extent differs in x and y: the autotuner
    tries that extent and its half in each direction (never a square tile
    beyond either), and the tile it returns solves like the default one."""
    import torch
    from paper_2205_08909_amd import mfcg
    cells = 9
    tile, ms = mfcg.autotune_tile(cells, k, map_kind=1, amplitude=0.05, iters=2)
    print("k", k, "tile", tile, "ms", ms, flush=True)
    half = tuple((e + 1) // 2 for e in ext)
    assert ms > 0 and tile[:2] in (ext, half)
    xs, iters = [], []
    for t in (tile, None):
        P = mfcg.Problem(cells, k, map_kind=1, amplitude=0.05, tile=t)
        b = torch.from_numpy(inputs.random_rhs(cells, k, seed=7)).cuda()
        x = torch.zeros_like(b)
        code, its, _, tr = P.solve(b, x, tol=1e-10, maxit=5000, want_hist=False, want_true_res=True)
        print("tile", t, "its", its, "true res", tr, flush=True)
        assert code == mfcg.OK and tr <= 2e-10
        xs.append(x)
        iters.append(its)
        P.close()
    # the two tilings sum in different orders: the same iteration up to rounding
    assert abs(iters[0] - iters[1]) <= 3
    assert float((xs[0] - xs[1]).norm() / xs[1].norm()) <= 1e-6


def test_batch_mixed_large_and_small_problems():
    """One problem large enough to fill the device alone (>= 512 tiles)
    beside small ones of other degrees in the same work lists: still bitwise
    the single-problem results."""
    import torch
    from paper_2205_08909_amd import mfcg
    probs = [{"cells": (32, 32, 32), "degree": 6, "map_kind": 1, "amplitude": 0.05, "seed": 1},
             {"cells": (6, 6, 6), "degree": 3, "map_kind": 1, "amplitude": 0.05, "seed": 2},
             {"cells": (5, 5, 5), "degree": 2, "map_kind": 1, "amplitude": 0.05, "seed": 3}]
    for p in probs:
        p["coeff"] = inputs.grf_coefficient(p["cells"][0], 0.1, 1.0, seed=p["seed"])
    B = mfcg.Batch(probs, autotune=False)
    assert B.problems[0].layout_info()["n_tiles"] >= 512
    bs = [torch.from_numpy(inputs.random_rhs(p["cells"][0], p["degree"], seed=p["seed"])).cuda() for p in probs]
    xs = [torch.zeros_like(b) for b in bs]
    code, its, st = B.solve(bs, xs, tol=1e-10, maxit=20000)
    assert code == mfcg.OK
    for i, p in enumerate(probs):
        P = mfcg.Problem(p["cells"], p["degree"], coeff=p["coeff"], map_kind=1, amplitude=0.05, tile=B.tiles[i])
        x = torch.zeros_like(bs[i])
        c, it, _, _ = P.solve(bs[i], x, tol=1e-10, maxit=20000, want_hist=False)
        assert c == mfcg.OK and it == its[i] and torch.equal(x, xs[i])
        P.close()
    B.close()


def test_setup_batch_options_and_tune_cache(tmp_path):
    """mfcg_setup_batch: a fixed tile from the options is used for every
    problem (clipped to its mesh); with a tune cache the first set-up tunes
    and records one tile per degree, the second reads them back (same tiles,
    no tuning), and both batches solve to the same solution bitwise."""
    import json
    import time
    import torch
    from paper_2205_08909_amd import mfcg
    probs = _draw(11, 4, 4, 10, kmin=2, kmax=4)
    bs = [torch.from_numpy(inputs.random_rhs(p["cells"][0], p["degree"], seed=p["seed"])).cuda() for p in probs]
    fixed = mfcg.Batch(probs, tile=(2, 2, 4))
    for i, p in enumerate(probs):
        assert fixed.tiles[i] == tuple(min(t, c) for t, c in zip((2, 2, 4), p["cells"]))
    fixed.close()
    cache = tmp_path / "tune.json"
    t0 = time.perf_counter()
    B1 = mfcg.Batch(probs, tune_cache=str(cache))
    t1 = time.perf_counter()
    recs = json.load(open(cache))["entries"]
    assert {r["k"] for r in recs} == {p["degree"] for p in probs}
    assert all(r["precision"] == "fp64" and len(r["tile"]) == 3 and r["ms"] > 0 for r in recs)
    before = cache.read_bytes()
    B2 = mfcg.Batch(probs, tune_cache=str(cache))
    t2 = time.perf_counter()
    print(f"set-up with tuning {t1 - t0:.2f} s, from the cache {t2 - t1:.2f} s")
    assert B2.tiles == B1.tiles
    assert cache.read_bytes() == before  # read back, nothing tuned again
    xs1 = [torch.zeros_like(b) for b in bs]
    xs2 = [torch.zeros_like(b) for b in bs]
    c1, its1, _ = B1.solve(bs, xs1, tol=1e-10, maxit=5000)
    c2, its2, _ = B2.solve(bs, xs2, tol=1e-10, maxit=5000)
    assert c1 == c2 == mfcg.OK and its1 == its2
    assert all(torch.equal(a, b) for a, b in zip(xs1, xs2))
    B1.close()
    B2.close()


def test_tune_cache_record_beyond_the_compiled_extent_is_retuned(tmp_path):
    """A cached tile wider than this build's compiled x/y extent (a cache
    written by a build with other tile shapes) is not used: the degree is
    tuned again and its record replaced."""
    import re
    from paper_2205_08909_amd import mfcg
    probs = _draw(11, 4, 4, 10, kmin=2, kmax=4)
    cache = tmp_path / "tune.json"
    mfcg.Batch(probs, tune_cache=str(cache)).close()
    stale = re.sub(r'"tile": \[\d+, \d+, (\d+)\]', r'"tile": [16, 16, \1]', cache.read_text())
    assert stale.count("[16, 16,") == len({p["degree"] for p in probs})
    cache.write_text(stale)
    B = mfcg.Batch(probs, tune_cache=str(cache))
    ext = {2: (8, 8), 3: (8, 4), 4: (4, 4)}
    for p, t in zip(probs, B.tiles):
        assert t[0] <= ext[p["degree"]][0] and t[1] <= ext[p["degree"]][1], (p["degree"], t)
    assert "[16, 16," not in cache.read_text()
    B.close()
