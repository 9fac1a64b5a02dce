"""The surrogate run's bookkeeping on the host: checks, rollbacks to accepted
states, the solver's redo, and the deeper rollback when the solver fails from the
newest accepted state.  A scripted stand-in solver and network carry one number
per state (its "taint"), so every branch runs without a GPU:

  taint 0: a clean state;
  taint 1: healthy but outside the accepted bounds (|phi| too large);
  taint 2: within the bounds now, but the solver diverges once it has advanced
           the state by DIVERGE_AFTER steps;
  taint 3: diverged (non-finite).
"""
import numpy as np
import pytest
import torch

from paper_2511_00445_amd import surrogate as S

DIVERGE_AFTER = 120


class FakeSim:
    ny = nx = 4

    def __init__(self):
        self.t, self.taint, self.age = 0, 0.0, 0
        self.imports = []

    def step(self, n):
        self.t += n
        if self.taint == 2:
            self.age += n
            if self.age >= DIVERGE_AFTER:
                self.taint = 3.0

    def step_count(self):
        return self.t

    def export_state(self, buf):
        buf.view(-1)[0] = self.taint

    def import_state(self, buf, step):
        self.t, self.taint, self.age = int(step), float(buf.view(-1)[0]), 0
        self.imports.append((step, self.taint))

    def diagnostics(self):
        return {"status": -4 if self.taint == 3 else 0, "phi_absmax": 1.5 if self.taint == 1 else 1.0,
                "umax": 0.01}


class FakeNet:
    batch, ny, nx = 1, 4, 4

    def __init__(self, script=None, errors=None):
        self.script = script or {}    # forward call number -> taint of the prediction
        self.errors = errors or {}    # forward call number -> check error when that call is a check
        self.calls = 0

    def forward(self, x, out):
        self.calls += 1
        out.view(-1)[0] = self.script.get(self.calls, float(x.view(-1)[0]))

    def compare(self, a, b):
        e = self.errors.get(self.calls, 0.01)
        c = np.zeros((7, 2))
        c[:, 0], c[:, 1] = e * e, 1.0
        return c


def run(net, calls, **kw):
    sim = FakeSim()
    r = S.SurrogateRun(sim, net, k=50, check_every=5, hold=1, device="cpu", **kw)
    r.advance(50 * calls)
    return sim, r


def test_clean_run_jumps_and_checks():
    sim, r = run(FakeNet(), 20)
    assert sim.t == 1000 and sim.taint == 0
    assert (r.surrogate_calls, r.checks, r.fallbacks) == (16, 4, 0)
    assert [s for _, s in r.accepted] == [750, 1000]


def test_failed_check_rolls_back_and_the_solver_redoes_the_span():
    # the check of the first five calls fails: back to step 0, the solver redoes
    # the five calls plus one held call, then the network takes over again
    sim, r = run(FakeNet(errors={5: 0.2}), 12)
    assert sim.imports[4] == (0, 0.0)                # after the jumps at steps 50-200
    assert r.accepted[0][1] == 300
    assert r.fallbacks == 1 and r.summary()["failed_checks"] == 1
    assert r.checks == 2 and r.solver_calls == 2 + 6   # two checks, six redone calls
    assert sim.t == 600 and sim.taint == 0


def test_state_outside_the_bounds_fails_its_check():
    # a jump leaves phi outside the bounds; the check's error is small but the
    # state is not accepted
    sim, r = run(FakeNet(script={2: 1.0}), 10)
    assert r.fallbacks == 1 and np.isnan(r.errors[0][1])
    assert sim.taint == 0


def test_unjudged_state_at_the_end_is_redone_by_the_solver():
    # the last calls before the end are jumps; one leaves the bounds, so advance()
    # hands back the solver's state instead
    sim, r = run(FakeNet(script={7: 1.0}), 8)
    assert r.health_rollbacks == 1
    assert sim.t == 400 and sim.taint == 0
    assert r.accepted[-1][1] == 400


def test_solver_failing_from_the_newest_accepted_state_rolls_back_further():
    # call 3 leaves a latent state that passes the check at call 5 (accepted at
    # step 250) and the next check fails; the solver's redo from step 250 diverges,
    # so the run goes back to step 0 and the solver takes it from there
    sim, r = run(FakeNet(script={3: 2.0}, errors={10: 0.2}), 16)
    assert r.fallbacks == 1 and r.deep_rollbacks == 1
    assert (0, 0.0) in sim.imports
    assert sim.taint == 0 and sim.t == 800


def test_no_older_state_left_raises():
    sim = FakeSim()
    net = FakeNet(script={1: 2.0}, errors={5: 0.2})
    r = S.SurrogateRun(sim, net, k=50, check_every=5, hold=1, depth=1, device="cpu")
    sim.taint = 2.0  # the starting state itself is latent
    with pytest.raises(RuntimeError):
        r.advance(50 * 20)


def test_arguments():
    with pytest.raises(ValueError):
        S.SurrogateRun(FakeSim(), FakeNet(), relax=-1, device="cpu")
    with pytest.raises(ValueError):
        S.SurrogateRun(FakeSim(), FakeNet(), densities="other", device="cpu")
    with pytest.raises(ValueError):
        S.SurrogateRun(FakeSim(), FakeNet(), depth=0, device="cpu")
    r = S.SurrogateRun(FakeSim(), FakeNet(), relax=25, device="cpu")
    with pytest.raises(ValueError):
        r.advance(50)
    assert torch.all(r.x9 == 0)
