"""Learned interior-point warm start on the device: solutions of seeded load
draws by the device IPM (rkkt_solve), the perceptron of rkkt_mlp.h trained on
them (loads -> primal-dual point), and warm solves (rkkt_solve_warm) from its
predictions.  Argument marshalling and the experiment's bookkeeping only:
every solve, product and update runs in librkkt.so.

Inputs: the 2 n_load loads (P then Q) of one scenario.  Outputs: x [n_x],
u [n_u], y [n_x], z [m] of the solution, the multipliers for the objective
weighted 1/N.  Both standardised per component with the training set's mean
and standard deviation (floor 1e-8); the multipliers of h are not sign
constrained in this formulation, so they are standardised like the rest
rather than taken in log space."""
from __future__ import annotations

import time

import numpy as np

from . import _lib as L


class Solver:
    """One N = 1 handle of a grid; the loads are replaced per draw."""

    def __init__(self, net, torch):
        self.torch = torch
        nl = len(net.load_bus)
        self.p = L.rkkt_create(net, np.ones((1, nl)), np.ones((1, nl)))
        d = self.p.dims
        self.nx, self.nu, self.m, self.nl = d["n_x"], d["n_u"], d["m"], nl
        z = lambda n: torch.zeros(n, dtype=torch.float64, device="cuda")  # noqa: E731
        self.x, self.u, self.y, self.zz, self.s = z(self.nx), z(self.nu), z(self.nx), z(self.m), z(self.m)
        self.pd, self.qd = z(nl), z(nl)

    def set_loads(self, pd, qd):
        self.pd.copy_(self.torch.as_tensor(pd))
        self.qd.copy_(self.torch.as_tensor(qd))
        L.rkkt_set_loads(self.p, self.pd, self.qd)

    def solve(self, tol=1e-8, warm=None, mu0=0.0, warm_duals=0):
        """Returns (result dict, solution vector [x, u, y, z] with the
        multipliers for objective weight 1 / N)."""
        if warm is None:
            r = L.rkkt_solve(self.p, self.x, self.u, self.y, self.zz, self.s, tol=tol)
        else:
            x0, u0, y0, z0 = warm
            r = L.rkkt_solve_warm(self.p, x0, u0, y0, z0, self.x, self.u, self.y, self.zz, self.s,
                                  tol=tol, mu0=mu0, warm_duals=warm_duals)
        scale = 1.0 / r["obj_weight"]   # N = 1
        sol = self.torch.cat([self.x, self.u, self.y * scale, self.zz * scale]).cpu().numpy()
        return r, sol

    def split(self, v):
        """Device tensors (x, u, y, z) from a solution-layout vector."""
        t = self.torch.as_tensor(np.ascontiguousarray(v), dtype=self.torch.float64, device="cuda")
        a, b, c = self.nx, self.nx + self.nu, 2 * self.nx + self.nu
        return t[:a].contiguous(), t[a:b].contiguous(), t[b:c].contiguous(), t[c:].contiguous()


def solve_draws(solver, pd, qd, tol=1e-8, log=None):
    """Cold solves of the draws pd, qd [n_load][K]: (solutions [K][n_out],
    iterations [K], objectives [K], converged [K]); a progress line through
    log every 1000 solves."""
    K = pd.shape[1]
    sols, its, objs, ok = [], [], [], []
    for k in range(K):
        if log and k and k % 1000 == 0:
            log(f"cold solves: {k} of {K}")
        solver.set_loads(pd[:, k], qd[:, k])
        r, sol = solver.solve(tol)
        sols.append(sol)
        its.append(r["iters"])
        objs.append(r["obj"])
        ok.append(r["status"] == "converged")
    return np.array(sols), np.array(its), np.array(objs), np.array(ok)


class Standardizer:
    def __init__(self, a):
        self.mean = a.mean(axis=0)
        self.std = np.maximum(a.std(axis=0), 1e-8)

    def fwd(self, a):
        return (a - self.mean) / self.std

    def inv(self, a):
        return a * self.std + self.mean


def init_params(sizes, seed):
    """He-style uniform initial weights, zero biases, in the rkkt_mlp.h
    parameter layout (FP32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        s = np.sqrt(6.0 / fi) / 2.0
        parts.append(rng.uniform(-s, s, fi * fo))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def fit(torch, X, Y, sizes, steps=2000, batch=256, lr=1e-3, seed=0):
    """Trains the device perceptron on X -> Y (already standardised), mini
    batches drawn with replacement; returns (mlp, loss every 100 steps)."""
    rng = np.random.default_rng(seed)
    m = L.Mlp(sizes, batch)
    m.set_params(torch.tensor(init_params(sizes, seed), device="cuda"))
    Xd = torch.tensor(X.astype(np.float32), device="cuda")
    Yd = torch.tensor(Y.astype(np.float32), device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for step in range(steps):
        idx = torch.as_tensor(rng.integers(0, X.shape[0], batch), device="cuda")
        m.train_step(Xd[idx].contiguous(), Yd[idx].contiguous(), lr, loss)
        if step % 100 == 0 or step == steps - 1:
            hist.append(float(loss.item()))
    return m, hist


def predict(torch, m, X):
    Xd = torch.tensor(X.astype(np.float32), device="cuda")
    out = torch.zeros(X.shape[0], m.sizes[-1], dtype=torch.float32, device="cuda")
    for b0 in range(0, X.shape[0], m.batch_max):
        b1 = min(X.shape[0], b0 + m.batch_max)
        m.forward(Xd[b0:b1].contiguous(), out[b0:b1])
    return out.cpu().numpy().astype(np.float64)


def warm_solves(solver, torch, pd, qd, idx, pred, objs, its, mu0, tol, warm_duals=0):
    """Warm solves of the draws idx from the predictions; (iterations with
    fallbacks counted, number of fallbacks, relative objective differences)."""
    warm_its, fallbacks, obj_err = [], 0, []
    for j, k in enumerate(idx):
        solver.set_loads(pd[:, k], qd[:, k])
        r, _ = solver.solve(tol, warm=solver.split(pred[j]), mu0=mu0, warm_duals=warm_duals)
        rel = abs(r["obj"] - objs[k]) / max(abs(objs[k]), 1e-300)
        obj_err.append(rel)
        n = r["iters"]
        if r["status"] != "converged" or rel > 1e-6:
            fallbacks += 1
            n += its[k]
        warm_its.append(n)
    return np.array(warm_its), fallbacks, np.array(obj_err)


def experiment(torch, net, pd, qd, n_train, n_val=0, mu0s=(1e-4,), tol=1e-8, steps=2000, seed=0, log=print):
    """Cold solves of every draw; training on the first n_train, the warm
    start's barrier parameter chosen among mu0s on the next n_val draws (the
    first of mu0s without validation draws), warm solves of the rest, from the
    perceptron's predictions and, as the ablation, from the mean training
    solution at the same barrier parameter.
    Iterations are counted with fallbacks: a warm solve that fails or whose
    objective differs from the cold one by more than 1e-6 relative adds the
    cold iterations."""
    solver = Solver(net, torch)
    t0 = time.time()
    sols, its, objs, ok = solve_draws(solver, pd, qd, tol, log=log)
    t_solve = time.time() - t0
    log(f"cold solves: {len(its)} in {t_solve:.1f} s, mean {its.mean():.2f} iterations, "
        f"{(~ok).sum()} not converged")
    X = np.concatenate([pd.T, qd.T], axis=1)
    tr = np.arange(n_train)[ok[:n_train]]
    va = np.arange(n_train, n_train + n_val)[ok[n_train:n_train + n_val]]
    te = np.arange(n_train + n_val, len(its))[ok[n_train + n_val:]]
    sx, sy = Standardizer(X[tr]), Standardizer(sols[tr])
    sizes = [X.shape[1], 512, 512, 512, sols.shape[1]]
    t0 = time.time()
    mlp, hist = fit(torch, sx.fwd(X[tr]), sy.fwd(sols[tr]), sizes, steps=steps, seed=seed)
    t_train = time.time() - t0
    log(f"training: {steps} steps in {t_train:.1f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    mu0 = mu0s[0]
    val = {}
    if len(va):
        pv = sy.inv(predict(torch, mlp, sx.fwd(X[va])))
        for m0 in mu0s:
            wi, fb, _ = warm_solves(solver, torch, pd, qd, va, pv, objs, its, m0, tol)
            val[m0] = float(wi.mean())
            log(f"validation: mu0 {m0:g}: warm {wi.mean():.2f} vs cold {its[va].mean():.2f}, {fb} fallbacks")
        mu0 = min(val, key=val.get)
    pred = sy.inv(predict(torch, mlp, sx.fwd(X[te])))
    warm_its, fallbacks, obj_err = warm_solves(solver, torch, pd, qd, te, pred, objs, its, mu0, tol)
    # ablation: the same warm solve from the mean training solution (no
    # network), at the same mu0, so that the gain of the perceptron is
    # separated from the gain of starting with a small barrier parameter
    mean_pred = np.repeat(sols[tr].mean(axis=0)[None, :], len(te), axis=0)
    mean_its, mean_fb, mean_err = warm_solves(solver, torch, pd, qd, te, mean_pred, objs, its, mu0, tol)
    out = {"n_train": int(len(tr)), "n_val": int(len(va)), "n_test": int(len(te)),
           "cold_mean_iters": float(its[te].mean()), "warm_mean_iters": float(warm_its.mean()),
           "fallback_rate": fallbacks / max(len(te), 1),
           "max_rel_obj_diff": float(np.max(obj_err)) if len(obj_err) else 0.0,
           "mean_start_mean_iters": float(mean_its.mean()),
           "mean_start_fallback_rate": mean_fb / max(len(te), 1),
           "train_loss": hist, "cold_solve_seconds": t_solve, "train_seconds": t_train, "mu0_warm": mu0,
           "validation_mean_iters": {f"{k:g}": v for k, v in val.items()}}
    log(f"test: cold {out['cold_mean_iters']:.2f} vs warm {out['warm_mean_iters']:.2f} mean iterations "
        f"(mu0 {mu0:g}), fallback rate {out['fallback_rate']:.3f}; from the mean training solution "
        f"{out['mean_start_mean_iters']:.2f}, fallback rate {out['mean_start_fallback_rate']:.3f}")
    return out
