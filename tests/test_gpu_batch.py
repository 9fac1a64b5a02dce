"""Launch-shape tuning and batched simulations through the C ABI."""
import sys

import numpy as np
import pytest

from oracle.coracle import COracle
from paper_2511_00445_amd.workloads import base_params, initial_fields

pytestmark = pytest.mark.gpu
# collide_rows 1, 2: rows of sites per thread on the default tile width, 11, 12: the same
# on half-width tiles; fd_shape 1, 2, 4: one launch per sub-step; 16, 32: all sub-steps in
# one launch; 162, 163: blocks of 2 or 3 sub-steps per launch; 165, 166: up to 5 sub-steps
# per launch on 40- or 32-row tiles, phi and Q in separate thread blocks of one launch
SHAPES = [(c, f) for c in (1, 2, 11, 12) for f in (1, 2, 4, 16, 32, 162, 163, 165, 166)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def single(p, ic, steps, shape=(2, 4)):
    from paper_2511_00445_amd import Sim
    s = Sim(p)
    s.set_tuning(*shape)
    s.init_fields(**ic)
    s.step(steps)
    return s


@pytest.mark.parametrize("storage", [0, 1])
def test_results_independent_of_launch_shape(gpu, storage):
    """Bitwise identical states for every launch shape (LDS/halo races or tile-edge
    errors would show up as differences)."""
    say(f"case: launch shapes, storage {storage}")
    p = dict(base_params(300, 170, zeta=0.03, lam=1.5), storage=storage)
    ic = initial_fields(300, 170, seed=9, phi_noise=0.4, S0=0.3)
    ref = single(p, ic, 15, SHAPES[0]).get_state()
    for shape in SHAPES[1:]:
        assert np.array_equal(single(p, ic, 15, shape).get_state(), ref), shape


@pytest.mark.parametrize("n_sub,nx,ny", [(1, 8, 8), (2, 13, 70), (3, 130, 9), (4, 64, 64), (5, 8, 33),
                                         (6, 40, 24), (8, 24, 40)])
def test_fused_substeps_match_per_substep_launches(gpu, n_sub, nx, ny):
    """All sub-steps in one launch (temporal blocking) against one launch per
    sub-step: bitwise equal for every n_sub, on grids smaller than a tile and with
    ragged edges (n_sub > 5 runs the per-sub-step path under either setting)."""
    say(f"case: fused sub-steps n_sub {n_sub}, {nx}x{ny}")
    p = base_params(nx, ny, zeta=0.03, lam=1.2, n_sub=n_sub)
    ic = initial_fields(nx, ny, seed=30 + n_sub, phi_noise=0.5, S0=0.3)
    ref = single(p, ic, 12, (2, 4)).get_state()
    for shape in ((2, 16), (2, 32), (2, 162), (2, 163), (2, 165), (1, 165), (12, 166), (11, 165)):
        assert np.array_equal(single(p, ic, 12, shape).get_state(), ref), shape


def test_default_tuning_by_grid_size(gpu):
    """One row of sites per collision thread below 2^21 sites, two from there."""
    from paper_2511_00445_amd import Sim
    say("case: default launch shape by grid size")
    for (nx, ny), rows in (((64, 64), 1), ((1024, 1024), 1), ((2048, 1024), 2), ((2048, 2048), 2)):
        s = Sim(base_params(nx, ny))
        assert s.get_tuning() == (rows, 165), (nx, ny, s.get_tuning())
        s.close()


def test_autotune_keeps_state(gpu):
    from paper_2511_00445_amd import Sim
    say("case: autotune")
    p = base_params(200, 120, zeta=0.02)
    s = Sim(p)
    s.init_fields(**initial_fields(200, 120, seed=2, phi_noise=0.2))
    s.step(3)
    before = s.get_state()
    ms = s.autotune(steps=3)
    assert ms > 0 and s.get_tuning() in SHAPES
    assert np.array_equal(s.get_state(), before) and s.step_count() == 3


def _members():
    return [dict(p=base_params(40, 40, zeta=0.02), ic=initial_fields(40, 40, seed=1, phi_noise=0.2)),
            dict(p=base_params(64, 32, lam=1.5, K=0.08), ic=initial_fields(64, 32, seed=2, phi_mean=0.3)),
            dict(p=base_params(70, 90, gamma=0.3, zeta=0.01), ic=initial_fields(70, 90, seed=3, S0=0.3)),
            dict(p=base_params(128, 128, tau_a=0.8, tau_p=1.3), ic=initial_fields(128, 128, seed=4, phi_mean=-0.3))]


@pytest.mark.parametrize("shape", [(2, 4), (1, 1), (2, 32), (1, 16), (2, 162), (1, 163), (2, 165), (12, 166), (11, 4)])
def test_batch_members_match_single_runs(gpu, shape):
    from paper_2511_00445_amd import Batch
    say(f"case: batch vs single, shape {shape}")
    ms = _members()
    b = Batch([m["p"] for m in ms])
    b.set_tuning(*shape)
    for i, m in enumerate(ms):
        b.init_fields(i, **m["ic"])
    b.step(20)
    for i, m in enumerate(ms):
        g = b.get_fields(i)
        s = single(m["p"], m["ic"], 20, shape).get_fields()
        for k in g:
            assert np.array_equal(g[k], s[k]), (i, k)


@pytest.mark.parametrize("shape", [(2, 165), (1, 4), (2, 162), (11, 166)])
def test_batch_binary16_members_match_single_runs(gpu, shape):
    """Binary16 population storage in the batched launches: each member bitwise
    equal to its own single run."""
    from paper_2511_00445_amd import Batch
    say(f"case: binary16 batch vs single, shape {shape}")
    ms = [dict(m, p=dict(m["p"], storage=1)) for m in _members()]
    b = Batch([m["p"] for m in ms])
    b.set_tuning(*shape)
    for i, m in enumerate(ms):
        b.init_fields(i, **m["ic"])
    b.step(20)
    for i, m in enumerate(ms):
        g = b.get_fields(i)
        s = single(m["p"], m["ic"], 20, shape).get_fields()
        for k in g:
            assert np.array_equal(g[k], s[k]), (i, k)
    assert all(b.diagnostics(i)["status"] == 0 for i in range(len(ms)))


def test_batch_member_reinit_and_oracle(gpu):
    from paper_2511_00445_amd import Batch
    say("case: batch re-init and oracle")
    ms = _members()
    b = Batch([m["p"] for m in ms])
    for i, m in enumerate(ms):
        b.init_fields(i, **m["ic"])
    b.step(5)
    ic2 = initial_fields(64, 32, seed=22, phi_noise=0.3)
    b.init_fields(1, **ic2)       # member 1 restarts while the others continue
    b.step(5)
    np.testing.assert_array_equal(b.get_fields(1)["phi"], single(ms[1]["p"], ic2, 5).get_fields()["phi"])
    np.testing.assert_array_equal(b.get_fields(2)["qxx"], single(ms[2]["p"], ms[2]["ic"], 10).get_fields()["qxx"])
    o = COracle(ms[2]["p"])
    o.init_fields(**ms[2]["ic"])
    o.step(10)
    of, g = o.get_fields(), b.get_fields(2)
    for k in ("phi", "qxx", "qxy", "u_a", "u_p"):
        assert np.linalg.norm(g[k] - of[k]) <= 1e-4 * np.linalg.norm(of[k]), k
    assert b.diagnostics(2)["step"] == 10 and b.diagnostics(1)["step"] == 5


def test_batch_autotune_and_errors(gpu):
    import paper_2511_00445_amd as T
    say("case: batch autotune and errors")
    ms = _members()
    b = T.Batch([m["p"] for m in ms])
    for i, m in enumerate(ms):
        b.init_fields(i, **m["ic"])
    b.step(2)
    before = [b.get_fields(i)["phi"] for i in range(len(ms))]
    assert b.autotune(steps=2) > 0 and b.get_tuning() in SHAPES
    for i in range(len(ms)):
        np.testing.assert_array_equal(b.get_fields(i)["phi"], before[i])
    with pytest.raises(T.TfanError) as e:
        T.Batch([base_params(32, 32), base_params(32, 32, n_sub=3)])
    assert e.value.code == T.TFAN_EINVAL
    with pytest.raises(T.TfanError):
        b.init_fields(7, *[np.zeros((40, 40))] * 3)


@pytest.mark.parametrize("storage", [0, 1])
def test_persistent_launch_matches_per_phase_launches(gpu, storage):
    """One persistent launch for all members and steps gives bitwise the states of
    the per-phase launches, also when the two are interleaved (buffer parity)."""
    from paper_2511_00445_amd import Batch
    say(f"case: persistent batch launch, storage {storage}")
    ms = [dict(m, p=dict(m["p"], storage=storage)) for m in _members()]
    a, b = Batch([m["p"] for m in ms]), Batch([m["p"] for m in ms])
    a.set_tuning(2, 165)
    for i, m in enumerate(ms):
        a.init_fields(i, **m["ic"])
        b.init_fields(i, **m["ic"])
    a.step(12)
    b.step_persistent(5)
    b.step(2)
    b.step_persistent(5)
    assert b.persistent_blocks() > 0 and b.persistent_blocks() % 8 == 0
    for i in range(len(ms)):
        ga, gb = a.get_fields(i), b.get_fields(i)
        for k in ga:
            assert np.array_equal(ga[k], gb[k]), (i, k)
        assert b.diagnostics(i)["step"] == 12


@pytest.mark.parametrize("n_sub", [1, 3])
def test_persistent_launch_other_substep_counts(gpu, n_sub):
    from paper_2511_00445_amd import Batch
    say(f"case: persistent batch launch, n_sub {n_sub}")
    ms = [dict(m, p=dict(m["p"], n_sub=n_sub)) for m in _members()]
    a, b = Batch([m["p"] for m in ms]), Batch([m["p"] for m in ms])
    for i, m in enumerate(ms):
        a.init_fields(i, **m["ic"])
        b.init_fields(i, **m["ic"])
    a.step(7)
    b.step_persistent(7)
    for i in range(len(ms)):
        assert np.array_equal(a.get_fields(i)["phi"], b.get_fields(i)["phi"])
        assert np.array_equal(a.get_fields(i)["u_a"], b.get_fields(i)["u_a"])


def test_persistent_launch_rejects_more_than_five_substeps(gpu):
    import paper_2511_00445_amd as T
    say("case: persistent batch launch, n_sub 6")
    b = T.Batch([base_params(32, 24, n_sub=6), base_params(40, 40, n_sub=6)])
    for i, (nx, ny) in enumerate(((32, 24), (40, 40))):
        b.init_fields(i, **initial_fields(nx, ny, seed=i))
    with pytest.raises(T.TfanError) as e:
        b.step_persistent(1)
    assert e.value.code == T.TFAN_EINVAL
