"""Surrogate-accelerated coarsening runs (host orchestration of libtfan calls).

The network (include/tfan_cnn.h) predicts the solver state k lattice steps ahead.
This module strings the library calls together; every arithmetic step runs in
the HIP library:

- trajectory_pairs: solver runs from seeded initial conditions; states exported
  on the device every k steps give training pairs (x_t, x_{t+k}).
- channel_scales: input scales (RMS of each state channel) and output scales
  (RMS of each channel's k-step increment) from a sample of pairs.
- train: Adam on random mini-batches of the pairs.
- SurrogateRun: advances a solver by surrogate calls of k steps; every
  check_every-th call also runs the solver over the same k steps from the same
  state, measures the surrogate's relative L2 error on (phi, Qxx, Qxy) and
  continues from the solver's state, which becomes the new restart point.  An
  error above tol (fallback) restores the last restart point and recomputes
  the span since it with the plain solver, plus `hold` further calls.
"""
from __future__ import annotations

import time

import numpy as np

from .binding import Cnn, Sim
from .workloads import initial_fields

K_STEPS = 50


def trajectory_pairs(params: dict, seeds, t0: int, t1: int, k: int = K_STEPS, phi_mean: float = 0.0):
    """Device tensors X, T [n][7][ny][nx]: states at t = t0, t0 + k, ... < t1 and k steps later."""
    import torch
    ny, nx = int(params["ny"]), int(params["nx"])
    per = (t1 - t0) // k
    X = torch.empty((len(seeds) * per, 7, ny, nx), dtype=torch.float32, device="cuda")
    T = torch.empty_like(X)
    for i, seed in enumerate(seeds):
        s = Sim(params)
        s.init_fields(**initial_fields(nx, ny, seed=int(seed), phi_mean=phi_mean))
        s.step(t0)
        for j in range(per):
            s.export_state(X[i * per + j])
            s.step(k)
            s.export_state(T[i * per + j])
        s.sync()
        if s.diagnostics()["status"] != 0:
            raise RuntimeError(f"training trajectory of seed {seed} became unhealthy")
        s.close()
    return X, T


def channel_scales(X, T, samples: int = 16, seed: int = 0):
    """(s_in, s_out): per-channel RMS of the states and of the k-step increments,
    from a random sample of pairs (host copies)."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(X.shape[0], size=min(samples, X.shape[0]), replace=False)
    x = X[idx].cpu().numpy().astype(np.float64)
    d = T[idx].cpu().numpy().astype(np.float64) - x
    s_in = np.sqrt(np.mean(x * x, axis=(0, 2, 3))) + 1e-12
    s_out = np.sqrt(np.mean(d * d, axis=(0, 2, 3))) + 1e-12
    return s_in.astype(np.float32), s_out.astype(np.float32)


def init_params(seed: int = 0) -> np.ndarray:
    """He-style uniform weights (fan-in 9 c_in), zero biases, zero last layer (the
    untrained surrogate is the identity map), in the ABI's parameter order."""
    rng = np.random.default_rng(seed)
    dims = [7, 48, 48, 48, 48, 48, 7]
    out = []
    for i in range(6):
        ci, co = dims[i], dims[i + 1]
        lim = np.sqrt(6.0 / (9 * ci))
        W = rng.uniform(-lim, lim, size=(co, ci, 3, 3)) if i < 5 else np.zeros((co, ci, 3, 3))
        out += [W.ravel(), np.zeros(co)]
    return np.concatenate(out).astype(np.float32)


def train(net: Cnn, X, T, steps: int, lr: float = 1e-3, lr_final: float = 1e-4, seed: int = 0,
          log_every: int = 0, log=print):
    """Adam on random batches of net.batch pairs; learning rate decays
    geometrically from lr to lr_final.  Returns the loss of every step."""
    rng = np.random.default_rng(seed)
    losses = []
    for i in range(steps):
        rate = lr * (lr_final / lr) ** (i / max(1, steps - 1))
        idx = rng.choice(X.shape[0], size=net.batch, replace=False)
        losses.append(net.train_step(X, T, idx, rate))
        if log_every and (i + 1) % log_every == 0:
            log(f"train step {i + 1}: loss {np.mean(losses[-log_every:]):.5f} (lr {rate:.2e})")
    return losses


def prediction_errors(net: Cnn, X, T, channels=(0, 1, 2)):
    """Relative L2 error over the given channels of the network's prediction and of
    persistence (x_{t+k} = x_t) on every pair; net.batch must be 1."""
    import torch
    out = torch.empty((1,) + tuple(X.shape[1:]), dtype=torch.float32, device="cuda")
    e_net, e_id = [], []
    for i in range(X.shape[0]):
        x, t = X[i:i + 1], T[i:i + 1]
        net.forward(x, out)
        c = net.compare(out, t)
        e_net.append(np.sqrt(c[list(channels), 0].sum() / c[list(channels), 1].sum()))
        c = net.compare(x, t)
        e_id.append(np.sqrt(c[list(channels), 0].sum() / c[list(channels), 1].sum()))
    return np.array(e_net), np.array(e_id)


class SurrogateRun:
    """A solver advanced by surrogate calls, checked against itself, with rollback."""

    def __init__(self, sim: Sim, net: Cnn, k: int = K_STEPS, check_every: int = 10, tol: float = 5e-2,
                 hold: int = 10, channels=(0, 1, 2)):
        import torch
        if net.batch != 1 or (net.ny, net.nx) != (sim.ny, sim.nx):
            raise ValueError("the network must take one sample of the solver's grid")
        self.sim, self.net, self.k = sim, net, int(k)
        self.check_every, self.tol, self.hold = int(check_every), float(tol), int(hold)
        self.channels = list(channels)
        shape = (1, 7, sim.ny, sim.nx)
        self.x = torch.empty(shape, dtype=torch.float32, device="cuda")
        self.xp = torch.empty_like(self.x)
        self.xs = torch.empty_like(self.x)
        self.good = torch.empty_like(self.x)
        self.good_step = None
        self.since_check = 0
        self.surrogate_calls = self.solver_calls = self.checks = self.fallbacks = 0
        self.plain_left = 0
        self.errors = []  # (step, relative L2 error) of every check

    def _mark_good(self):
        self.sim.export_state(self.good[0])
        self.good_step = self.sim.step_count()
        self.since_check = 0

    def advance(self, steps: int):
        """Advance by `steps` (a multiple of k) lattice steps."""
        if steps % self.k:
            raise ValueError("steps must be a multiple of k")
        target = self.sim.step_count() + steps
        if self.good_step is None:
            self._mark_good()
        while self.sim.step_count() < target:
            if self.plain_left > 0:
                self.sim.step(self.k)
                self.solver_calls += 1
                self.plain_left -= 1
                if self.plain_left == 0:
                    self._mark_good()
                continue
            self.sim.export_state(self.x[0])
            self.net.forward(self.x, self.xp)
            self.since_check += 1
            if self.since_check == self.check_every:
                self.sim.step(self.k)
                self.sim.export_state(self.xs[0])
                c = self.net.compare(self.xp, self.xs)
                err = float(np.sqrt(c[self.channels, 0].sum() / c[self.channels, 1].sum()))
                self.errors.append((self.sim.step_count(), err))
                self.checks += 1
                self.solver_calls += 1
                if np.isfinite(err) and err <= self.tol:
                    self.good.copy_(self.xs)
                    self.good_step = self.sim.step_count()
                    self.since_check = 0
                else:
                    # restore the last checked state; redo the span with the solver
                    span = (self.sim.step_count() - self.good_step) // self.k
                    self.fallbacks += 1
                    self.sim.import_state(self.good[0], self.good_step)
                    self.plain_left = min(span, (target - self.good_step) // self.k) + self.hold
                    self.since_check = 0
            else:
                self.sim.import_state(self.xp[0], self.sim.step_count() + self.k)
                self.surrogate_calls += 1

    def summary(self) -> dict:
        errs = [e for _, e in self.errors]
        return dict(surrogate_calls=self.surrogate_calls, solver_calls=self.solver_calls, checks=self.checks,
                    fallbacks=self.fallbacks, max_check_error=max(errs) if errs else None,
                    mean_check_error=float(np.mean(errs)) if errs else None)


def timed(fn, *args, **kw):
    """(result, wall seconds) of fn after a device synchronisation on both sides."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn(*args, **kw)
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0
