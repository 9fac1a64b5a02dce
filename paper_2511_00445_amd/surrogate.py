"""Surrogate-accelerated coarsening runs (host orchestration of libtfan calls).

The network (include/tfan_cnn.h) predicts the solver state k lattice steps ahead.
This module strings the library calls together; every arithmetic step runs in
the HIP library:

- trajectory_pairs: solver runs from seeded initial conditions; states exported
  on the device every k steps give training pairs (x_t, x_{t+k}).
- channel_scales: input scales (RMS of each state channel) and output scales
  (RMS of each channel's k-step increment) from a sample of pairs.
- train: Adam on random mini-batches of the pairs; with max_unroll > 0 part of
  every batch starts from the network's own predictions (pushforward): the
  input is the network applied m times to x_t, the target the solver state at
  t + (m + 1) k, so the network learns to correct the drift of its own rollouts.
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
RELAX_STEPS = 25     # solver steps after each jump in the deploy loop
TRAIN_STEPS = 12000  # Adam steps of the standard training run (batches of 8)
# Bounds of an accepted surrogate state.  The solver's own trajectories keep |phi|
# within a few percent of 1 (the bulk values) and |u| near 0.03-0.05 on the
# deployment workload; a chain of network jumps can leave a few sites with phi
# overshoots or velocity spikes that a whole-grid L2 check does not see and from
# which the solver itself can diverge.
PHI_LIMIT = 1.15
U_LIMIT = 0.1
# Training trajectories: 256 x 256 runs, pairs from steps TRAIN_T0 to TRAIN_T1, so
# that the network has seen the early coarsening and the late, activity-arrested
# domains it meets over long deployments.
TRAIN_T0, TRAIN_T1 = 1000, 50000
TRAIN_SEEDS = tuple(range(600, 608))


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
          log_every: int = 0, log=print, per_traj: int = 0, max_unroll: int = 0, unroll_from: float = 0.3):
    """Adam on random batches of net.batch pairs; the learning rate decays
    geometrically from lr to lr_final.  With max_unroll > 0 (pairs stored as
    consecutive runs of per_traj pairs per trajectory), after the first
    unroll_from share of the steps each batch draws an unroll depth m in
    [0, max_unroll]: inputs are the network applied m times to x_t (no gradient
    through those applications), targets the trajectory state k (m + 1) steps
    after t.  Returns the loss of every step."""
    import torch
    rng = np.random.default_rng(seed)
    losses = []
    B = net.batch
    if max_unroll:
        if per_traj <= max_unroll or X.shape[0] % per_traj:
            raise ValueError("pairs must come as runs of per_traj > max_unroll pairs")
        xa = torch.empty((B,) + tuple(X.shape[1:]), dtype=X.dtype, device=X.device)
        xb, tt = torch.empty_like(xa), torch.empty_like(xa)
        ids = np.arange(B, dtype=np.int32)
    for i in range(steps):
        rate = lr * (lr_final / lr) ** (i / max(1, steps - 1))
        m = int(rng.integers(0, max_unroll + 1)) if max_unroll and i >= unroll_from * steps else 0
        if m == 0:
            idx = rng.choice(X.shape[0], size=B, replace=False)
            losses.append(net.train_step(X, T, idx, rate))
        else:
            traj = rng.integers(0, X.shape[0] // per_traj, size=B)
            j = rng.integers(0, per_traj - m, size=B)
            start = traj * per_traj + j
            xa.copy_(X[torch.as_tensor(start, device=X.device)])
            tt.copy_(T[torch.as_tensor(start + m, device=X.device)])
            for _ in range(m):
                net.forward(xa, xb)
                xa, xb = xb, xa
            losses.append(net.train_step(xa, tt, ids, rate))
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
    """A solver advanced by surrogate calls, checked against itself, with rollback.

    Every `check_every`-th call runs the solver over the jump instead and compares
    the two; a state is accepted only after a passed check and within the solver's
    bounds.  The last `depth` accepted states are kept (with their densities): a
    failed check rolls back to the newest one and the solver redoes the span plus
    `hold` calls; if the solver itself fails from there, the run rolls back one
    accepted state further."""

    def __init__(self, sim: Sim, net: Cnn, k: int = K_STEPS, check_every: int = 10, tol: float = 5e-2,
                 hold: int = 10, channels=(0, 1, 2), relax: int = 0, densities: str = "reset",
                 phi_limit: float = PHI_LIMIT, u_limit: float = U_LIMIT, depth: int = 2, device: str = "cuda"):
        import torch
        if net.batch != 1 or (net.ny, net.nx) != (sim.ny, sim.nx):
            raise ValueError("the network must take one sample of the solver's grid")
        self.sim, self.net, self.k = sim, net, int(k)
        self.check_every, self.tol, self.hold = int(check_every), float(tol), int(hold)
        self.channels = list(channels)
        self.relax = int(relax)  # solver steps after every call: a call covers k + relax steps
        if self.relax < 0:
            raise ValueError("relax must be >= 0")
        # densities after a network jump (the network predicts none): "reset" to rho0,
        # or "keep" those the solver held before the jump.  Kept densities are exact
        # for the solver's own states, but over hundreds of chained jumps they drift
        # (a growing low-density region) and phi overshoots grow until a relax span
        # diverges; the checks then roll back, so "keep" is slower and noisier.
        if densities not in ("keep", "reset"):
            raise ValueError("densities must be 'keep' or 'reset'")
        self.densities = densities
        # a state is accepted only within these bounds (see PHI_LIMIT, U_LIMIT)
        self.phi_limit, self.u_limit = float(phi_limit), float(u_limit)
        if depth < 1:
            raise ValueError("depth must be >= 1")
        shape = (1, 7, sim.ny, sim.nx)
        self.x = torch.empty(shape, dtype=torch.float32, device=device)
        self.xp = torch.empty_like(self.x)
        self.xs = torch.empty_like(self.x)
        # jump target with zero density planes, for densities = "reset"
        self.x9 = torch.zeros((9, sim.ny, sim.nx), dtype=torch.float32, device=device) if densities == "reset" else None
        # accepted states with their densities: a rollback restores all but the
        # populations' non-equilibrium part.  accepted = [(buffer index, step)], newest last
        self.ring = [torch.empty((9, sim.ny, sim.nx), dtype=torch.float32, device=device) for _ in range(depth)]
        self.accepted = []
        self.since_check = 0
        self.surrogate_calls = self.solver_calls = self.checks = self.fallbacks = 0
        self.health_rollbacks = 0  # unjudged states at the end of advance() outside the bounds
        self.relax_rollbacks = 0   # passed checks whose relax span left a state outside the bounds
        self.deep_rollbacks = 0    # solver redos that failed, rolled back one accepted state further
        self.plain_left = 0
        self.errors = []  # (step, relative L2 error) of every check

    @property
    def good_step(self):
        return self.accepted[-1][1] if self.accepted else None

    def _healthy(self) -> bool:
        return self.sim.diagnostics()["status"] == 0

    def _valid(self) -> bool:
        """Healthy, and within the bounds a solver trajectory stays in."""
        d = self.sim.diagnostics()
        return d["status"] == 0 and d["phi_absmax"] <= self.phi_limit and d["umax"] <= self.u_limit

    def _mark_good(self):
        used = {i for i, _ in self.accepted}
        i = next(j for j in range(len(self.ring)) if j not in used) if len(used) < len(self.ring) \
            else self.accepted[0][0]
        self.sim.export_state(self.ring[i])
        self.accepted = [a for a in self.accepted if a[0] != i] + [(i, self.sim.step_count())]
        self.since_check = 0

    def _redo_from(self, back: int):
        """Restore the accepted state `back` places before the newest (dropping the
        newer ones); the solver redoes the span up to now plus `hold` calls."""
        if back:
            self.accepted = self.accepted[:-back]
        i, step = self.accepted[-1]
        span = -(-(self.sim.step_count() - step) // (self.k + self.relax))  # calls since, the last one partly done
        self.sim.import_state(self.ring[i], step)
        self.plain_left = span + self.hold
        self.since_check = 0

    def _roll_back(self):
        self.fallbacks += 1
        self._redo_from(0)

    def advance(self, steps: int):
        """Advance by `steps` lattice steps (a multiple of k + relax)."""
        call = self.k + self.relax
        if steps % call:
            raise ValueError("steps must be a multiple of k + relax")
        target = self.sim.step_count() + steps
        if not self.accepted:
            if not self._healthy():
                raise RuntimeError("the solver's state is unhealthy before the first surrogate call")
            self._mark_good()
        while True:
            self._run_to(target)
            # calls since the last check have not been judged: a state handed back
            # must be within the bounds, else the solver redoes them to the target
            if self.since_check and not self._valid():
                self.health_rollbacks += 1
                i, step = self.accepted[-1]
                self.sim.import_state(self.ring[i], step)
                self.plain_left = (target - step) // call
                self.since_check = 0
                continue
            # a solver redo still under way must at least be healthy
            if self.plain_left and not self._healthy():
                self._solver_failed()
                continue
            return

    def _solver_failed(self):
        if len(self.accepted) < 2:
            raise RuntimeError("the solver became unhealthy from the oldest accepted state")
        self.deep_rollbacks += 1
        self._redo_from(1)

    def _run_to(self, target: int):
        call = self.k + self.relax
        while self.sim.step_count() < target:
            if self.plain_left > 0:
                self.sim.step(call)
                self.solver_calls += 1
                self.plain_left -= 1
                if self.plain_left == 0:
                    if self._healthy():
                        self._mark_good()
                    else:
                        self._solver_failed()
                continue
            self.sim.export_state(self.x[0])
            self.net.forward(self.x, self.x9[None, :7] if self.x9 is not None else self.xp)
            self.since_check += 1
            if self.since_check == self.check_every:
                self.sim.step(self.k)
                self.sim.export_state(self.xs[0])
                c = self.net.compare(self.x9[None, :7] if self.x9 is not None else self.xp, self.xs)
                err = float(np.sqrt(c[self.channels, 0].sum() / c[self.channels, 1].sum()))
                # the error judges (phi, Q) over the whole grid; the bounds catch
                # what a few sites of the chained jumps carry (the solver keeps them)
                if not self._valid():
                    err = float("nan")
                self.errors.append((self.sim.step_count(), err))
                self.checks += 1
                self.solver_calls += 1
                if np.isfinite(err) and err <= self.tol:
                    if self.relax:
                        self.sim.step(self.relax)
                    if self._valid():
                        self._mark_good()
                    else:
                        self.relax_rollbacks += 1
                        self._roll_back()
                else:
                    self._roll_back()
            else:
                self.sim.import_state(self.x9 if self.x9 is not None else self.xp[0], self.sim.step_count() + self.k)
                self.surrogate_calls += 1
                if self.relax:  # the solver smooths what the jump leaves at the grid scale
                    self.sim.step(self.relax)

    def summary(self) -> dict:
        errs = [e for _, e in self.errors]
        return dict(surrogate_calls=self.surrogate_calls, solver_calls=self.solver_calls, checks=self.checks,
                    fallbacks=self.fallbacks, health_rollbacks=self.health_rollbacks,
                    relax_rollbacks=self.relax_rollbacks, deep_rollbacks=self.deep_rollbacks, failed_checks=sum(1 for e in errs if not e <= self.tol),
                    nonfinite_checks=sum(1 for e in errs if not np.isfinite(e)),
                    max_check_error=float(np.nanmax(errs)) if np.isfinite(errs).any() else None,
                    mean_check_error=float(np.nanmean(errs)) if np.isfinite(errs).any() else None)


def train_surrogate(params: dict, seeds, t0: int, t1: int, steps: int, batch: int = 8, k: int = K_STEPS,
                    lr: float = 1e-3, lr_final: float = 1e-5, seed: int = 0, velocity_weight: float = 1.0 / 9.0,
                    max_unroll: int = 0, log=None):
    """Pairs from solver trajectories of `params`, scales, and a trained network.
    velocity_weight scales the loss of the four velocity channels (through
    their output scales); the deploy checks judge (phi, Q).
    Returns (theta, s_in, s_out, losses, seconds of training)."""
    X, T = trajectory_pairs(params, seeds, t0, t1, k)
    s_in, s_out = channel_scales(X, T, samples=32, seed=seed)
    s_out[3:] /= np.float32(np.sqrt(velocity_weight))
    net = Cnn(batch, int(params["ny"]), int(params["nx"]), train=True)
    net.set_params(init_params(seed))
    net.set_scales(s_in, s_out)
    losses, secs = timed(train, net, X, T, steps, lr, lr_final, seed, (steps // 10) if log else 0,
                         log or print, per_traj=(t1 - t0) // k, max_unroll=max_unroll)
    theta = net.get_params()
    net.close()
    del X, T
    return theta, s_in, s_out, losses, secs


def deploy_compare(params: dict, seed: int, theta, s_in, s_out, t_start: int, t_end: int, every: int,
                   k: int = K_STEPS, check_every: int = 10, tol: float = 5e-2, hold: int = 10, relax: int = 0,
                   densities: str = "reset", noise_floor: bool = False, log=None):
    """The plain solver and the surrogate-accelerated run from the same state at
    t_start to t_end.  Domain length L(t) every `every` steps (host analysis of phi,
    outside the timed spans).  Returns a dict of the two L records, the stepping
    wall times, simulated steps per second and the maximum relative L deviation.
    noise_floor: also run the plain solver from the same state after one export /
    import round trip (the reconstruction the surrogate applies, without the
    network: only the populations' non-equilibrium part is lost) and return its L
    record and largest relative deviation, the chaotic spread against which the
    surrogate's deviation is read."""
    import torch
    from .analysis import domain_length
    ny, nx = int(params["ny"]), int(params["nx"])
    sim = Sim(params)
    sim.init_fields(**initial_fields(nx, ny, seed=int(seed)))
    sim.step(t_start)
    sim.sync()
    start = sim.get_state()
    samples = (t_end - t_start) // every

    def phi_length():
        f = sim.get_fields()
        return domain_length(f["phi"])

    plain_L, plain_s = [], 0.0
    for _ in range(samples):
        _, dt = timed(sim.step, every)
        plain_s += dt
        plain_L.append(phi_length())
    if sim.diagnostics()["status"] != 0:
        raise RuntimeError("plain run became unhealthy")
    extra = {}
    if noise_floor:
        sim.set_state(start)
        x = torch.empty((7, ny, nx), dtype=torch.float32, device="cuda")
        sim.export_state(x)
        sim.import_state(x, t_start)
        floor_L = []
        for _ in range(samples):
            sim.step(every)
            floor_L.append(phi_length())
        extra = dict(L_round_trip=floor_L,
                     max_L_dev_round_trip=float(np.max(np.abs(np.array(floor_L) / np.array(plain_L) - 1))))
    sim.set_state(start)
    net = Cnn(1, ny, nx)
    net.set_params(theta)
    net.set_scales(s_in, s_out)
    run = SurrogateRun(sim, net, k=k, check_every=check_every, tol=tol, hold=hold, relax=relax, densities=densities)
    sur_L, sur_s = [], 0.0
    for _ in range(samples):
        _, dt = timed(run.advance, every)
        sur_s += dt
        sur_L.append(phi_length())
        if log:
            log(f"step {sim.step_count()}: L plain {plain_L[len(sur_L) - 1]:.3f} surrogate {sur_L[-1]:.3f}")
    status = sim.diagnostics()["status"]
    dev = np.abs(np.array(sur_L) - np.array(plain_L)) / np.array(plain_L)
    span = t_end - t_start
    out = dict(t=list(range(t_start + every, t_end + 1, every)), L_plain=plain_L, L_surrogate=sur_L,
               max_L_dev=float(dev.max()), plain_seconds=plain_s, surrogate_seconds=sur_s,
               plain_steps_per_s=span / plain_s, surrogate_steps_per_s=span / sur_s, speedup=plain_s / sur_s,
               status=status, **extra, **run.summary())
    net.close()
    sim.close()
    return out


def timed(fn, *args, **kw):
    """(result, wall seconds) of fn after a device synchronisation on both sides."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn(*args, **kw)
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0
