"""Learned warm start of parametric QPs: solve a training set with the batched
interior-point solver, train the MLP on (theta -> x*, lambda*), then solve
fresh instances from the network's prediction.  Every numerical step runs in
the HIP library (batched solve, MLP products, loss, Adam); this module only
sequences the calls and moves arrays between them."""
import time

import numpy as np

from . import lib as L
from . import workloads as w


class ParamBatch:
    """Batched solver over `chunk` instances of one parametric QP; solving a
    set of theta re-uses the analysis and only replaces b."""

    def __init__(self, pq, chunk, precision=L.PDIPM_FP64, **opts):
        self.pq = pq
        self.chunk = chunk
        zero = np.zeros(pq.B.shape[1])
        self.solver = L.BatchSolver([pq.instance(zero) for _ in range(chunk)], precision=precision, **opts).bind()
        self.n, self.m = pq.base.n, pq.base.m

    def solve(self, thetas, starts=None, fallback=True, log=None, log_every=60.0):
        """Solve b(theta) for every row of thetas; returns per-instance
        results, x (count x n) and lambda (count x m), and the wall time.
        With starts (predicted x, lambda per row) the instances are warm
        started; any that does not reach status OK is solved again from the
        cold start (fallback, inside the timed region) and its result says
        so ("fallback": 1)."""
        count = thetas.shape[0]
        X = np.empty((count, self.n))
        Lm = np.empty((count, self.m))
        results = []
        t0 = time.time()
        t_log = t0
        for c0 in range(0, count, self.chunk):
            if log and time.time() - t_log >= log_every:
                t_log = time.time()
                log(f"[warm] solved {c0} of {count} instances in {t_log - t0:.0f}s")
            th = thetas[c0:c0 + self.chunk]
            k = th.shape[0]
            pad = np.concatenate([th, np.repeat(th[-1:], self.chunk - k, axis=0)]) if k < self.chunk else th
            self.solver.set_b((self.pq.b0[None, :] + pad @ self.pq.B.T).ravel())
            start = None
            if starts is not None:
                xs, ls = starts
                xs = xs[c0:c0 + self.chunk]
                ls = ls[c0:c0 + self.chunk]
                if k < self.chunk:
                    xs = np.concatenate([xs, np.repeat(xs[-1:], self.chunk - k, axis=0)])
                    ls = np.concatenate([ls, np.repeat(ls[-1:], self.chunk - k, axis=0)])
                start = (xs.ravel(), ls.ravel())
            res, _ = self.solver.solve(start=start)
            sol = self.solver.solution()
            failed = [i for i in range(k) if res[i]["status"] != 0] if start is not None and fallback else []
            if failed:
                cold, _ = self.solver.solve()
                csol = self.solver.solution()
                for i in failed:
                    res[i], sol[i] = dict(cold[i], fallback=1), csol[i]
            for i in range(k):
                results.append(res[i])
                X[c0 + i] = sol[i]["x"]
                Lm[c0 + i] = sol[i]["lam"]
        return results, X, Lm, time.time() - t0


def train(model, thetas, targets, steps, batch, lr, log=None):
    """Adam steps over shuffled mini-batches (fixed seed); returns the losses."""
    import torch
    rng = np.random.default_rng(w.seed_for(5, 4242))
    th = torch.as_tensor(np.ascontiguousarray(thetas, np.float32), device="cuda:0")
    tg = torch.as_tensor(np.ascontiguousarray(targets, np.float32), device="cuda:0")
    losses = []
    n = thetas.shape[0]
    perm = rng.permutation(n)
    pos = 0
    for s in range(steps):
        if pos + batch > n:
            perm = rng.permutation(n)
            pos = 0
        idx = torch.as_tensor(perm[pos:pos + batch], device="cuda:0")
        pos += batch
        want = (s % 50 == 0) or s == steps - 1
        loss = model.train_step(th.index_select(0, idx).contiguous(), tg.index_select(0, idx).contiguous(), lr,
                                want_loss=want)
        if want:
            losses.append((s, loss))
            if log:
                log(f"[warm] step {s} loss {loss:.5f}")
    return losses


def predict(model, thetas):
    """(x_hat, lambda_hat) for every row of thetas."""
    import torch
    out = []
    for c0 in range(0, thetas.shape[0], model.max_batch):
        th = torch.as_tensor(np.ascontiguousarray(thetas[c0:c0 + model.max_batch], np.float32), device="cuda:0")
        out.append(model.forward(th).cpu().numpy().astype(np.float64))
    y = np.concatenate(out)
    return y[:, :model.n_x], y[:, model.n_x:]
