"""The seeded input generators: reproducible, and the Gaussian random field
has the squared-exponential covariance it claims (statistical check)."""
import numpy as np

from paper_2205_08909_amd import inputs


def test_grf_reproducible_and_shaped():
    a = inputs.grf_coefficient((5, 4, 3), 0.1, 1.0, seed=4)
    b = inputs.grf_coefficient((5, 4, 3), 0.1, 1.0, seed=4)
    assert a.shape == (60,) and np.all(a == b) and np.all(a > 0)


def test_grf_covariance():
    n = (6, 5, 4)
    length = 0.3
    draws = np.stack([inputs.grf_log_coefficient(n, length, 1.0, seed=s) for s in range(2000)])
    emp = draws.T @ draws / draws.shape[0]
    cx, cy, cz = ((np.arange(m) + 0.5) / m for m in n)
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    d2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    ref = np.exp(-d2 / (2 * length ** 2))
    # sampling error of a covariance estimate ~ sqrt(2/2000) ~ 0.03
    assert np.abs(emp - ref).max() < 0.15
    assert np.abs(np.diag(emp) - 1).mean() < 0.03


def test_rhs_and_masks():
    b = inputs.random_rhs((3, 2, 4), 2, seed=1)
    m = inputs.boundary_mask((3, 2, 4), 2)
    assert b.size == 7 * 5 * 9 and np.all(b[m] == 0) and np.all(b[~m] != 0)
    assert m.sum() == 7 * 5 * 9 - 5 * 3 * 7
    p = inputs.bump_params(3)
    assert p[0] == 8 and p.size == 41


def test_batch_draw():
    probs = inputs.batch_draw(0)
    assert len(probs) == 32
    assert all(16 <= p["N"] <= 96 and 2 <= p["k"] <= 6 for p in probs)
    assert probs == inputs.batch_draw(0)
