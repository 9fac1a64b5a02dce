"""The convolutional surrogate end to end on the GPU: trained by the library's own
forward and backward kernels on solver trajectories, it must predict the state
50 steps ahead better than the method without it (persistence, x_{t+50} = x_t),
and the deploy loop's solver checks must catch a bad network and fall back to
the solver from the last checked state."""
import sys

import numpy as np
import pytest

from paper_2511_00445_amd.workloads import base_params, workload_params

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_trained_surrogate_beats_persistence(gpu):
    from paper_2511_00445_amd import Cnn
    from paper_2511_00445_amd import surrogate as S
    say("case: surrogate training 128x128, seeds 11-13, held-out seed 14")
    p = base_params(128, 128, zeta=0.01)  # the 512x512 active workload's parameters
    X, T = S.trajectory_pairs(p, [11, 12, 13], 1000, 4000)
    Xh, Th = S.trajectory_pairs(p, [14], 2000, 3000)
    s_in, s_out = S.channel_scales(X, T)
    net = Cnn(4, 128, 128, train=True)
    net.set_params(S.init_params(seed=3))
    net.set_scales(s_in, s_out)
    losses = S.train(net, X, T, steps=400, lr=1e-3, lr_final=1e-4, seed=1)
    inf = Cnn(1, 128, 128)
    inf.set_params(net.get_params())
    inf.set_scales(s_in, s_out)
    e_net, e_id = S.prediction_errors(inf, Xh, Th)
    say(f"loss {np.mean(losses[:20]):.4f} -> {np.mean(losses[-20:]):.4f}; held-out relative L2 on "
        f"(phi, Q): surrogate {e_net.mean():.4f}, persistence {e_id.mean():.4f}")
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:20])
    assert e_net.mean() < 0.7 * e_id.mean()


def test_failed_checks_roll_back_to_the_solver(gpu):
    from paper_2511_00445_amd import Cnn, Sim
    from paper_2511_00445_amd import surrogate as S
    from paper_2511_00445_amd.workloads import initial_fields
    say("case: surrogate fallback 64x64")
    p = workload_params("small_64")
    bad = S.init_params(seed=5)
    bad[-(48 * 7 * 9 + 7):] = np.random.default_rng(6).uniform(-0.5, 0.5, 48 * 7 * 9 + 7)
    net = Cnn(1, 64, 64)
    net.set_params(bad)
    net.set_scales(np.ones(7), np.full(7, 0.2))
    sim = Sim(p)
    sim.init_fields(**initial_fields(64, 64, seed=0))
    sim.step(200)
    run = S.SurrogateRun(sim, net, k=50, check_every=2, tol=5e-2, hold=2)
    run.advance(1000)
    sm = run.summary()
    say(f"summary {sm}")
    assert sim.step_count() == 1200
    assert sm["fallbacks"] >= 1 and sm["max_check_error"] > 5e-2
    assert sim.diagnostics()["status"] == 0
    # identity network (zero last layer): checks pass, every other call is the surrogate
    net.set_params(S.init_params(seed=5))
    run2 = S.SurrogateRun(sim, net, k=50, check_every=2, tol=10.0, hold=2)
    run2.advance(400)
    sm2 = run2.summary()
    say(f"identity summary {sm2}")
    assert sm2["fallbacks"] == 0 and sm2["surrogate_calls"] == 4 and sm2["checks"] == 4
