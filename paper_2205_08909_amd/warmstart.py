"""Learned warm start for the fused CG solver.

A four-layer 3D convolutional network (32 channels, BF16 weights and
activations, FP32 accumulation) maps the coefficient field and the
right-hand side to the shape of the solution; the solver turns that shape
into an initial guess with the Galerkin-optimal scale (mfcg_warmstart),
which can only lower the A-norm of the initial error.  The network is
trained on solutions the solver itself produced.  Every tensor operation
runs in the library's kernels (include/mfnn.h); this module holds the
layer plan, the parameter buffers and the training loop.

Layers on the (nx, ny, nz) node lattice (37^3 coarse points for 145^3 nodes):
  1  conv 4^3, stride 4, pad 2     3 -> 32 channels, fine -> coarse, leaky ReLU
  2  conv 3^3, pad 1               32 -> 32, leaky ReLU
  3  conv 3^3, dilation 3, pad 3   32 -> 32, leaky ReLU
     (receptive field 9 coarse points without gaps; dilations (2, 6), with
     17 points and gaps, trained to a larger energy-norm error)
  4  transposed conv 8^3, stride 4, pad 4   32 -> 1, coarse -> fine, + bias
Input channels: mean log a around each node, b / rms(b), D^{-1} b / rms.
Target: the solver's solution divided by its rms value (only the shape
matters after the Galerkin scaling).  Loss: mean squared error of the
values and of the forward differences along x, y, z scaled by g (an
H1-type loss: the Galerkin scaling and CG measure the error in the energy
norm, which weights gradients), computed by one fixed 4-channel
convolution of prediction and target.
"""
import time

import numpy as np

from . import inputs, mfcg, nn


class Net:
    def __init__(self, nodes, channels=32, seed=0, dil=(1, 3)):
        import torch
        self.torch = torch
        nodes = tuple(int(v) for v in nodes)  # (D, H, W) = (nz, ny, nx)
        c = int(channels)
        self.nodes, self.c = nodes, c
        self.g1 = nn.desc(1, 3, c, nodes, 4, 4, 2, 1)
        coarse = tuple(self.g1.out)
        self.coarse = coarse
        self.g2 = nn.desc(1, c, c, coarse, 3, 1, dil[0], dil[0])
        self.g3 = nn.desc(1, c, c, coarse, 3, 1, dil[1], dil[1])
        self.g4 = nn.desc(1, 1, c, nodes, 8, 4, 4, 1)  # conv fine -> coarse; layer 4 applies its transpose
        assert tuple(self.g4.out) == coarse
        shapes = [(c, 3, 4, 4, 4), (c, c, 3, 3, 3), (c, c, 3, 3, 3), (c, 1, 8, 8, 8)]
        bias_n = [c, c, c, 1]
        init = inputs.network_init(shapes, seed)
        chunks, self.slices = [], []
        off = 0
        for (w, _), sh, nb in zip(init, shapes, bias_n):
            nw = int(np.prod(sh))
            self.slices.append(((off, off + nw), (off + nw, off + nw + nb), sh))
            chunks += [w.ravel(), np.zeros(nb, np.float32)]
            off += nw + nb
        self.nparam = off
        dev = "cuda"
        self.theta = torch.from_numpy(np.concatenate(chunks)).to(dev)
        self.theta_bf16 = torch.empty(off, dtype=torch.bfloat16, device=dev)
        nn.convert(self.theta, self.theta_bf16)
        self.grad = torch.zeros(off, dtype=torch.float32, device=dev)
        self.m = torch.zeros_like(self.grad)
        self.v = torch.zeros_like(self.grad)
        self.step_count = 0
        self._bufs = {}
        self.wgrad_work = torch.empty(max(nn.wgrad_work(nn.with_batch(g, 8)) for g in (self.g1, self.g2, self.g3,
                                                                                          self.g4)),
                                      dtype=torch.float32, device=dev)

    # parameter views
    def w(self, i):
        (a, b), _, _ = self.slices[i]
        return self.theta_bf16[a:b]

    def b(self, i):
        _, (a, b), _ = self.slices[i]
        return self.theta[a:b]

    def dw(self, i):
        (a, b), _, _ = self.slices[i]
        return self.grad[a:b]

    def db(self, i):
        _, (a, b), _ = self.slices[i]
        return self.grad[a:b]

    def _buffers(self, B):
        if B not in self._bufs:
            t = self.torch
            nf = int(np.prod(self.nodes))
            ncs = int(np.prod(self.coarse))
            d = {"A": [t.empty(B * self.c * ncs, dtype=t.bfloat16, device="cuda") for _ in range(3)],
                 "Y": t.empty(B * nf, dtype=t.float32, device="cuda"),
                 "dY": t.empty(B * nf, dtype=t.float32, device="cuda"),
                 "dA": t.empty(B * self.c * ncs, dtype=t.float32, device="cuda"),
                 "dZ": t.empty(B * self.c * ncs, dtype=t.float32, device="cuda"),
                 # the activation gradient in BF16 for the gradients of the
                 # 32 -> 32 layers, which run on the matrix cores
                 "dZb": t.empty(B * self.c * ncs, dtype=t.bfloat16, device="cuda"),
                 "g": [nn.with_batch(g, B) for g in (self.g1, self.g2, self.g3, self.g4)]}
            self._bufs[B] = d
            need = max(nn.wgrad_work(g) for g in d["g"])
            if need > self.wgrad_work.numel():
                self.wgrad_work = t.empty(need, dtype=t.float32, device="cuda")
        return self._bufs[B]

    def forward(self, X, B=1):
        """X: bfloat16 [B, 3, nodes] -> Y: float32 [B, 1, nodes] (a view of an internal buffer)."""
        d = self._buffers(B)
        g1, g2, g3, g4 = d["g"]
        A1, A2, A3 = d["A"]
        self._X = X
        nn.conv_fwd(g1, X, self.w(0), self.b(0), nn.ACT_LEAKY, A1)
        nn.conv_fwd(g2, A1, self.w(1), self.b(1), nn.ACT_LEAKY, A2)
        nn.conv_fwd(g3, A2, self.w(2), self.b(2), nn.ACT_LEAKY, A3)
        nn.conv_bwd_data(g4, A3, self.w(3), self.b(3), d["Y"])
        return d["Y"]

    def backward(self, dY, B=1):
        """Gradients of all parameters into self.grad from dL/dY."""
        d = self._buffers(B)
        g1, g2, g3, g4 = d["g"]
        A1, A2, A3 = d["A"]
        dA, dZ, work = d["dA"], d["dZ"], self.wgrad_work
        # layer 4 (transposed): dA3 = conv(dY), dw4 from (dY, A3), db4 = sum dY
        nn.conv_fwd(g4, dY, self.w(3), None, nn.ACT_NONE, dA)
        nn.conv_bwd_weight(g4, dY, A3, self.dw(3), None, work)
        nn.channel_sum(B, 1, self.nodes, dY, self.db(3), work)
        # layer 3
        dZb = d["dZb"]
        nn.act_bwd(dA, A3, dZ)
        nn.convert(dZ, dZb)
        nn.conv_bwd_weight(g3, A2, dZb, self.dw(2), self.db(2), work)
        nn.conv_bwd_data(g3, dZb, self.w(2), None, dA)
        # layer 2
        nn.act_bwd(dA, A2, dZ)
        nn.convert(dZ, dZb)
        nn.conv_bwd_weight(g2, A1, dZb, self.dw(1), self.db(1), work)
        nn.conv_bwd_data(g2, dZb, self.w(1), None, dA)
        # layer 1 (no gradient to the input features)
        nn.act_bwd(dA, A1, dZ)
        nn.conv_bwd_weight(g1, self._X, dZ, self.dw(0), self.db(0), work)

    def adam(self, lr):
        self.step_count += 1
        nn.adam(self.theta, self.theta_bf16, self.grad, self.m, self.v, self.step_count, lr)

    def state(self):
        return self.theta.cpu().numpy().copy()

    def load(self, theta):
        t = self.torch
        self.theta.copy_(t.from_numpy(np.ascontiguousarray(theta, dtype=np.float32)))
        nn.convert(self.theta, self.theta_bf16)


class H1Loss:
    """Fixed filter [value, g dx, g dy, g dz] (2^3 taps, forward
    differences) applied to prediction and target; the loss is the MSE of
    the four channels, its gradient maps back through the filter's adjoint."""

    def __init__(self, nodes, B, gscale=None):
        import torch
        if gscale is None:
            gscale = 2.0 ** round(np.log2(max(1.0, (max(nodes) - 1) / 8.0)))
        w = np.zeros((4, 1, 2, 2, 2), np.float32)
        w[0, 0, 0, 0, 0] = 1.0
        for c, tap in ((1, (0, 0, 1)), (2, (0, 1, 0)), (3, (1, 0, 0))):  # x, y, z (W fastest)
            w[c, 0, 0, 0, 0] = -gscale
            w[c, 0][tap] = gscale
        self.w = torch.from_numpy(w.ravel()).to(torch.bfloat16).cuda()
        self.g = nn.desc(B, 1, 4, nodes, 2, 1, 0, 1)
        m = B * 4 * int(np.prod(tuple(self.g.out)))
        self.Z = torch.empty(m, dtype=torch.float32, device="cuda")
        self.ZT = torch.empty(m, dtype=torch.float32, device="cuda")
        self.dZ = torch.empty(m, dtype=torch.float32, device="cuda")

    def __call__(self, Y, T, dY, loss, work):
        nn.conv_fwd(self.g, Y, self.w, None, nn.ACT_NONE, self.Z)
        nn.conv_fwd(self.g, T, self.w, None, nn.ACT_NONE, self.ZT)
        nn.mse(self.Z, self.ZT, self.dZ, loss, work)
        nn.conv_bwd_data(self.g, self.dZ, self.w, None, dY)


class Workspace:
    def __init__(self):
        import torch
        self.d = torch.empty(4096, dtype=torch.float64, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")


def sample_problem(P, cells, k, seed, ws):
    """Coefficient, right-hand side, diagonal and log-coefficient of one
    sample (handle P is re-used: only the coefficient changes)."""
    import torch
    smp = inputs.warmstart_sample(seed, cells)
    P.set_coefficient(smp["coeff"])
    b = P.rhs(mfcg.RHS_BUMPS, smp["bumps"])
    diag = P.diagonal()
    logc = torch.from_numpy(smp["log_coeff"]).cuda()
    return b, diag, logc, smp


def generate(P, cells, k, seeds, tol=1e-8, maxit=50000, log=None):
    """Training pairs: features X (bfloat16 [S, 3, n]) and normalised solver
    solutions T (float32 [S, n])."""
    import torch
    ws = Workspace()
    S, n = len(seeds), P.n
    X = torch.empty((S, 3 * n), dtype=torch.bfloat16, device="cuda")
    T = torch.empty((S, n), dtype=torch.float32, device="cuda")
    its = []
    cc = (cells, cells, cells)
    t0 = time.perf_counter()
    for i, seed in enumerate(seeds):
        b, diag, logc, _ = sample_problem(P, cells, k, seed, ws)
        nn.features(cc, k, logc, b, diag, ws.d, X[i])
        u = torch.zeros_like(b)
        _, it, _, _ = P.solve(b, u, tol=tol, maxit=maxit, want_hist=False)
        its.append(it)
        nn.normalize(u, ws.d, T[i])
        if log and (i + 1) % max(1, S // 10) == 0:
            torch.cuda.synchronize()
            log(f"generated {i + 1}/{S} samples in {time.perf_counter() - t0:.1f} s (mean its {np.mean(its):.0f})")
    torch.cuda.synchronize()
    return X, T, {"seconds": time.perf_counter() - t0, "mean_iters": float(np.mean(its)), "tol": tol}


def train(net, X, T, epochs=10, batch=8, lr=1e-3, seed=0, h1=True, log=None):
    """Adam on the H1-type loss (or the plain MSE with h1=False), cosine
    learning-rate decay.  Returns the mean training loss per epoch."""
    import torch
    ws = Workspace()
    S = X.shape[0]
    B = min(batch, S)
    rng = np.random.default_rng(seed)
    steps_per_epoch = S // B
    total = epochs * steps_per_epoch
    dY = net._buffers(B)["dY"]
    lossf = H1Loss(net.nodes, B) if h1 else None
    losses = []
    step = 0
    acc = torch.zeros(steps_per_epoch, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(S)).cuda()
        for j in range(steps_per_epoch):
            idx = perm[j * B:(j + 1) * B]
            xb = X.index_select(0, idx).reshape(-1)
            tb = T.index_select(0, idx).reshape(-1)
            Y = net.forward(xb, B)
            if lossf is not None:
                lossf(Y, tb, dY, acc[j:j + 1], ws.d)
            else:
                nn.mse(Y, tb, dY, acc[j:j + 1], ws.d)
            net.backward(dY, B)
            lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * step / max(1, total)))
            net.adam(lr_t)
            step += 1
        losses.append(float(acc.mean().item()))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {losses[-1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    return losses


def predict_x0(net, P, cells, k, b, diag, logc, ws, X1=None, u=None, max_rel_res=float("inf")):
    """Features -> network -> Galerkin-scaled x0.  Returns (x0, scale, rel_res, used)."""
    import torch
    n = P.n
    if X1 is None:
        X1 = torch.empty(3 * n, dtype=torch.bfloat16, device="cuda")
    if u is None:
        u = torch.empty(n, dtype=torch.float64, device="cuda")
    nn.features((cells, cells, cells), k, logc, b, diag, ws.d, X1)
    Y = net.forward(X1, 1)
    nn.convert(Y, u)
    return P.warmstart(b, u, max_rel_res)


class CoarseLevel:
    """The same problem discretised with Q1 elements on the same cells,
    solved to a loose tolerance and interpolated to the fine nodes
    (mfcg_interpolate: the Q1 space is contained in the Q_k one).  It
    carries the smooth, global part of the solution, which the network
    cannot: its receptive field covers about a quarter of the domain width,
    while the solution of an elliptic problem depends on the data
    everywhere."""

    def __init__(self, cells, map_kind, amplitude, tol=1e-2, maxit=20000):
        self.P = mfcg.Problem(cells, 1, map_kind=map_kind, amplitude=amplitude)
        self.tol, self.maxit = tol, maxit

    def guess(self, Pf, smp, out=None):
        import torch
        self.P.set_coefficient(smp["coeff"])
        bc = self.P.rhs(mfcg.RHS_BUMPS, smp["bumps"])
        uc = torch.zeros_like(bc)
        self.P.solve(bc, uc, tol=self.tol, maxit=self.maxit, want_hist=False, raise_on=False)
        return Pf.interpolate_from(self.P, uc, out)

    def close(self):
        self.P.close()


def evaluate(net, P, cells, k, seeds, tol=1e-10, maxit=50000, max_rel_res=float("inf"), log=None, coarse=None,
             ir=False):
    """Plain CG from x0 = 0 against the learned x0 (features, inference and
    scaling included in its time) on each seed.  With a CoarseLevel also
    the coarse-level guess alone and the A-norm optimal combination of the
    coarse-level and learned guesses (mfcg_warmstart_span), each timed with
    everything it computes; with ir=True also FP32-inner iterative
    refinement (mfcg_solve_ir, residual replacement) from x0 = 0 and from the
    best of those guesses."""
    import torch
    ws = Workspace()
    rows = []
    n = P.n
    X1 = torch.empty(3 * n, dtype=torch.bfloat16, device="cuda")
    u = torch.empty(n, dtype=torch.float64, device="cuda")
    Uc = torch.empty(n, dtype=torch.float64, device="cuda")

    def sync():
        torch.cuda.synchronize()
        return time.perf_counter()

    for seed in seeds:
        b, diag, logc, smp = sample_problem(P, cells, k, seed, ws)
        x = torch.zeros_like(b)
        t0 = sync()
        c0, it0, _, _ = P.solve(b, x, tol=tol, maxit=maxit, want_hist=False)
        t_zero = sync() - t0
        t0 = sync()
        x0, sc, rel0, used = predict_x0(net, P, cells, k, b, diag, logc, ws, X1, u, max_rel_res)
        x0_copy = x0.clone()
        c1, it1, _, tr = P.solve(b, x0, tol=tol, maxit=maxit, want_hist=False, want_true_res=True)
        t_warm = sync() - t0
        # energy-norm error of the guess relative to that of x0 = 0 (x: the converged solution)
        xa = torch.dot(x, P.vmult(P.empty(), x)).item()

        def enorm(v):
            e = x - v
            return float(np.sqrt(max(torch.dot(e, P.vmult(P.empty(), e)).item(), 0.0) / xa))

        row = {"seed": int(seed), "iters_zero": it0, "iters_warm": it1, "s_zero": t_zero, "s_warm": t_warm,
               "used": bool(used), "scale": sc, "rel_res0": rel0, "status": (int(c0), int(c1)),
               "true_rel_res": tr, "energy_err0": enorm(x0_copy)}
        best = x0_copy
        if coarse is not None:
            t0 = sync()
            coarse.guess(P, smp, Uc)
            xc, _, _, _ = P.warmstart(b, Uc, max_rel_res)
            xc_copy = xc.clone()
            _, itc, _, _ = P.solve(b, xc, tol=tol, maxit=maxit, want_hist=False)
            t_c = sync() - t0
            t0 = sync()
            coarse.guess(P, smp, Uc)
            nn.features((cells, cells, cells), k, logc, b, diag, ws.d, X1)
            nn.convert(net.forward(X1, 1), u)
            xs, coef, _, _ = P.warmstart_span(b, [Uc, u], max_rel_res)
            xs_copy = xs.clone()
            _, its_, _, _ = P.solve(b, xs, tol=tol, maxit=maxit, want_hist=False)
            t_s = sync() - t0
            row.update({"iters_coarse": itc, "s_coarse": t_c, "energy_err0_coarse": enorm(xc_copy),
                        "iters_span": its_, "s_span": t_s, "energy_err0_span": enorm(xs_copy),
                        "span_coef": coef})
            best = xs_copy
        if ir:
            # FP32-inner refinement (residual replacement) from x0 = 0 and from the
            # best guess, the guess recomputed inside the timed region
            for name in ("zero", "best"):
                t0 = sync()
                if name == "zero":
                    xi = torch.zeros_like(b)
                elif coarse is not None:
                    coarse.guess(P, smp, Uc)
                    nn.features((cells, cells, cells), k, logc, b, diag, ws.d, X1)
                    nn.convert(net.forward(X1, 1), u)
                    xi, _, _, _ = P.warmstart_span(b, [Uc, u], max_rel_res)
                else:
                    xi, _, _, _ = predict_x0(net, P, cells, k, b, diag, logc, ws, X1, u, max_rel_res)
                ci, outer, inner, _, tri = P.solve_ir(b, xi, tol=tol, inner_tol=1e-1, keep_direction=True,
                                                      max_outer=100)
                row[f"ir_{name}"] = {"s": sync() - t0, "outer": outer, "inner_iters": inner, "status": int(ci),
                                     "true_rel_res": tri}
        rows.append(row)
        if log:
            msg = f"seed {seed}: {it0} -> {it1} iterations (learned)"
            if coarse is not None:
                msg += f", {row['iters_coarse']} (coarse), {row['iters_span']} (coarse + learned)"
            log(msg)
    return rows


def summarize(rows):
    i0 = np.array([r["iters_zero"] for r in rows], float)
    t0 = np.array([r["s_zero"] for r in rows])

    def stats(key_it, key_s):
        it = np.array([r[key_it] for r in rows], float)
        t = np.array([r[key_s] for r in rows])
        return {"iters": {"mean": float(it.mean()), "median": float(np.median(it)), "worst": float(it.max())},
                "ms": {"mean": float(t.mean() * 1e3), "median": float(np.median(t) * 1e3)},
                "iter_ratio_mean": float((it / i0).mean()), "time_ratio_mean": float(t.mean() / t0.mean()),
                "worse_than_zero": int((it > i0).sum())}

    out = {"n": len(rows),
           "zero": {"iters": {"mean": float(i0.mean()), "median": float(np.median(i0)), "worst": float(i0.max())},
                    "ms": {"mean": float(t0.mean() * 1e3), "median": float(np.median(t0) * 1e3)}},
           "learned": stats("iters_warm", "s_warm"),
           "energy_err0_mean": float(np.mean([r["energy_err0"] for r in rows])),
           "rel_res0_mean": float(np.mean([r["rel_res0"] for r in rows])),
           "fallbacks": int(sum(1 for r in rows if not r["used"]))}
    if "iters_coarse" in rows[0]:
        out["coarse"] = stats("iters_coarse", "s_coarse")
        out["coarse"]["energy_err0_mean"] = float(np.mean([r["energy_err0_coarse"] for r in rows]))
        out["coarse_plus_learned"] = stats("iters_span", "s_span")
        out["coarse_plus_learned"]["energy_err0_mean"] = float(np.mean([r["energy_err0_span"] for r in rows]))
        out["coarse_plus_learned"]["learned_coef_mean"] = float(np.mean([r["span_coef"][1] for r in rows]))
    if "ir_zero" in rows[0]:
        tz = np.array([r["ir_zero"]["s"] for r in rows])
        tb = np.array([r["ir_best"]["s"] for r in rows])
        out["ir"] = {"ms_from_zero": float(tz.mean() * 1e3), "ms_from_best_guess": float(tb.mean() * 1e3),
                     "inner_iters_from_zero": float(np.mean([r["ir_zero"]["inner_iters"] for r in rows])),
                     "inner_iters_from_best_guess": float(np.mean([r["ir_best"]["inner_iters"] for r in rows])),
                     "speedup_vs_plain_fp64_from_zero": float(t0.mean() / tb.mean()),
                     "worst_true_rel_res": float(max(max(r["ir_zero"]["true_rel_res"], r["ir_best"]["true_rel_res"])
                                                     for r in rows))}
    return out
