"""The surrogate network's HIP kernels (through the C ABI) against the FP64 oracle
oracle/cnn_oracle.py, which applies the same bfloat16 quantisation points.

Tolerances.  Every stored activation and back-propagated gradient is a bfloat16
rounding of an fp32 value that differs from the oracle's fp64 value by about
1e-5 relative (fp32 sums of up to 432 products); the rounding then lands on a
different bfloat16 neighbour for a small fraction of elements (~1e-3), each off
by one bfloat16 unit (2^-8 relative).  Over six layers this gives a relative L2
difference of a few 1e-4; the bounds below are 2e-3 (network output) and 5e-3
(weight and bias gradients).
"""
import sys

import numpy as np
import pytest

from oracle import cnn_oracle as C
from paper_2511_00445_amd.workloads import base_params, initial_fields

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


def setup(seed, nsamp, H, W, zero_last=False):
    rng = np.random.default_rng(seed)
    layers = C.init_params(seed=seed, zero_last=zero_last)
    theta = C.flatten(layers).astype(np.float32)
    layers = C.unflatten(theta.astype(np.float64))  # the oracle sees the fp32 parameters
    s_in = rng.uniform(0.5, 2.0, size=7).astype(np.float32)
    s_out = rng.uniform(0.05, 0.2, size=7).astype(np.float32)
    X = (rng.normal(size=(nsamp, 7, H, W)) * s_in[None, :, None, None]).astype(np.float32)
    T = (X + rng.normal(size=X.shape) * s_out[None, :, None, None]).astype(np.float32)
    return layers, theta, (s_in, s_out), X, T


def inv(s):
    """The reciprocal the library forms (fp32), as float64 broadcastable over [B][7][H][W]."""
    return (1.0 / s.astype(np.float32)).astype(np.float64)[None, :, None, None]


def test_forward_matches_oracle(gpu):
    import torch
    from paper_2511_00445_amd import Cnn
    say("case: cnn forward B=2 32x48")
    layers, theta, scales, X, _ = setup(1, 2, 32, 48)
    net = Cnn(2, 32, 48)
    net.set_params(theta)
    net.set_scales(*scales)
    x = torch.from_numpy(X).cuda()
    out = torch.empty_like(x)
    net.forward(x, out)
    net.sync()
    got = out.cpu().numpy().astype(np.float64)
    so = scales[1].astype(np.float64)[None, :, None, None]
    y_gpu = (got - X) / so
    y_ref, _ = C.forward(layers, X.astype(np.float64) * inv(scales[0]))
    e = rel(y_gpu, y_ref)
    say(f"forward: relative L2 of the network output {e:.2e}")
    assert e <= 2e-3
    ref = C.predict(layers, X.astype(np.float64), scales[0].astype(np.float64), scales[1].astype(np.float64))
    assert rel(got - X, ref - X) <= 2e-3


def test_forward_matches_oracle_when_blocks_walk_several_tiles(gpu):
    """Three 256 x 256 samples: 768 tiles of 16 x 16 sites, more than the
    persistent grid's 512 blocks, so blocks walk two tiles and take the path that
    loads the next tile while the matrix cores work on the current one; tiles of
    different samples share blocks."""
    import torch
    from paper_2511_00445_amd import Cnn
    say("case: cnn forward B=3 256x256 (blocks walk several tiles)")
    layers, theta, scales, X, _ = setup(3, 3, 256, 256)
    net = Cnn(3, 256, 256)
    net.set_params(theta)
    net.set_scales(*scales)
    x = torch.from_numpy(X).cuda()
    out = torch.empty_like(x)
    net.forward(x, out)
    net.sync()
    got = out.cpu().numpy().astype(np.float64)
    so = scales[1].astype(np.float64)[None, :, None, None]
    y_ref, _ = C.forward(layers, X.astype(np.float64) * inv(scales[0]))
    e = rel((got - X) / so, y_ref)
    say(f"forward 3 x 256^2: relative L2 of the network output {e:.2e}")
    assert e <= 2e-3
    for b in range(3):  # each sample on its own, so that no sample is mixed up with another
        assert rel((got[b] - X[b]) / so[0], y_ref[b]) <= 2e-3, b


def test_gradients_match_oracle(gpu):
    import torch
    from paper_2511_00445_amd import Cnn
    say("case: cnn gradients B=2 32x48")
    layers, theta, scales, X, T = setup(2, 3, 32, 48)
    net = Cnn(2, 32, 48, train=True)
    net.set_params(theta)
    net.set_scales(*scales)
    idx = [2, 0]
    loss, g = net.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), idx)
    xn = X[idx].astype(np.float64) * inv(scales[0])
    tn = (T[idx].astype(np.float32) - X[idx].astype(np.float32)).astype(np.float64) * inv(scales[1])
    lref, gref = C.loss_and_grads(layers, xn, tn)
    say(f"loss gpu {loss:.8e} oracle {lref:.8e}")
    assert abs(loss - lref) <= 1e-4 * lref
    gg = C.unflatten(g.astype(np.float64))
    for li in range(C.LAYERS):
        ew, eb = rel(gg[li][0], gref[li][0]), rel(gg[li][1], gref[li][1])
        say(f"layer {li + 1}: dW rel L2 {ew:.2e}, db rel L2 {eb:.2e}")
        assert ew <= 5e-3 and eb <= 5e-3, (li, ew, eb)


def test_gradients_match_oracle_when_blocks_walk_several_tiles(gpu):
    """Three 256 x 256 samples (768 tiles): the convolutions' persistent blocks
    (512) and the weight-gradient blocks (256) each walk several tiles, and the
    block partials of every layer's weight gradient are reduced over 256 blocks."""
    import torch
    from paper_2511_00445_amd import Cnn
    say("case: cnn gradients B=3 256x256 (blocks walk several tiles)")
    layers, theta, scales, X, T = setup(4, 3, 256, 256)
    net = Cnn(3, 256, 256, train=True)
    net.set_params(theta)
    net.set_scales(*scales)
    idx = [1, 2, 0]
    loss, g = net.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), idx)
    xn = X[idx].astype(np.float64) * inv(scales[0])
    tn = (T[idx].astype(np.float32) - X[idx].astype(np.float32)).astype(np.float64) * inv(scales[1])
    lref, gref = C.loss_and_grads(layers, xn, tn)
    say(f"loss gpu {loss:.8e} oracle {lref:.8e}")
    assert abs(loss - lref) <= 1e-4 * lref
    gg = C.unflatten(g.astype(np.float64))
    for li in range(C.LAYERS):
        ew, eb = rel(gg[li][0], gref[li][0]), rel(gg[li][1], gref[li][1])
        say(f"layer {li + 1}: dW rel L2 {ew:.2e}, db rel L2 {eb:.2e}")
        assert ew <= 5e-3 and eb <= 5e-3, (li, ew, eb)


def test_adam_step_closed_form(gpu):
    """First Adam step: bias-corrected moments are g and g^2, so each parameter
    moves by lr g / (|g| + eps) with g the batch gradient."""
    import torch
    from paper_2511_00445_amd import Cnn
    say("case: cnn adam step")
    _, theta, scales, X, T = setup(3, 2, 16, 32)
    net = Cnn(2, 16, 32, train=True)
    net.set_params(theta)
    net.set_scales(*scales)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    _, g = net.gradients(Xd, Td, [0, 1])
    lr = 1e-3
    net.train_step(Xd, Td, [0, 1], lr)
    th1 = net.get_params().astype(np.float64)
    g = g.astype(np.float64)
    want = theta.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(th1 - want) - 1e-6 * lr - 2e-7 * np.abs(want)) <= 0.0


def test_training_reduces_the_loss(gpu):
    import torch
    from paper_2511_00445_amd import Cnn
    say("case: cnn fits one batch")
    _, theta, scales, X, T = setup(4, 2, 32, 32, zero_last=True)
    net = Cnn(2, 32, 32, train=True)
    net.set_params(theta)
    net.set_scales(*scales)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    losses = [net.train_step(Xd, Td, [0, 1], 2e-3) for _ in range(60)]
    say(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.6 * losses[0]


@pytest.mark.parametrize("storage", [0, 1], ids=["f32", "f16"])
def test_state_import_reproduces_the_exported_state(gpu, storage):
    """export -> import -> export gives the exported state back: phi and Q exactly,
    the velocities (the next step's half-force solve with the implicit drag, under
    the imported fields' forces) up to the rounding of the rebuilt populations; the
    densities are those the handle held (rho0 on a handle without a state)."""
    import torch
    from paper_2511_00445_amd import Sim
    say(f"case: solver state export/import 48x32 storage {storage}")
    p = dict(base_params(48, 32, zeta=0.02), storage=storage)
    a = Sim(p)
    a.init_fields(**initial_fields(48, 32, seed=5, phi_noise=0.3, S0=0.2))
    a.step(25)
    x = torch.empty((7, 32, 48), dtype=torch.float32, device="cuda")
    a.export_state(x)
    a.sync()
    f = a.get_fields()
    xh = x.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(xh[0], f["phi"])
    np.testing.assert_array_equal(xh[1], f["qxx"])
    np.testing.assert_array_equal(xh[3:5], f["u_a"])
    np.testing.assert_array_equal(xh[5:7], f["u_p"])
    assert np.abs(f["rho_a"] - 1).max() > 1e-5  # densities that an import must keep
    x9 = torch.empty((9, 32, 48), dtype=torch.float32, device="cuda")
    a.export_state(x9)
    x9h = x9.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(x9h[:7], xh)
    np.testing.assert_allclose(x9h[7] + 1.0, f["rho_a"], rtol=0, atol=1e-7)
    np.testing.assert_allclose(x9h[8] + 1.0, f["rho_p"], rtol=0, atol=1e-7)
    # binary16 rounds each of the 9 rebuilt populations (|f - w rho0| < 5e-3 here)
    # to 2^-11 of its size: at most ~2e-5 on a density or a momentum
    utol, rtol = (1e-6, 1e-7) if storage == 0 else (5e-5, 3e-5)
    for sim, rho in ((a, f), (Sim(p), None)):
        sim.import_state(x, 25)
        assert sim.step_count() == 25
        y = torch.empty_like(x)
        sim.export_state(y)
        g = sim.get_fields()
        yh = y.cpu().numpy().astype(np.float64)
        np.testing.assert_array_equal(yh[:3], xh[:3])
        err = np.abs(yh[3:] - xh[3:]).max()
        say(f"largest velocity change over the round trip {err:.2e} (|u| up to {np.abs(xh[3:]).max():.2e})")
        assert err <= utol
        for key in ("rho_a", "rho_p"):
            want = rho[key] if rho is not None else np.ones_like(g[key])
            np.testing.assert_allclose(g[key], want, rtol=0, atol=rtol)
    # nine planes carry the densities: a fresh handle takes them from the array
    b = Sim(p)
    b.import_state(x9, 25)
    y9 = torch.empty_like(x9)
    b.export_state(y9)
    y9h = y9.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(y9h[:3], x9h[:3])
    assert np.abs(y9h[3:7] - x9h[3:7]).max() <= utol
    assert np.abs(y9h[7:] - x9h[7:]).max() <= rtol


def test_cnn_argument_errors(gpu):
    import torch
    import paper_2511_00445_amd as T
    say("case: cnn argument errors")
    with pytest.raises(T.TfanError):
        T.Cnn(1, 40, 32)
    net = T.Cnn(1, 16, 16)
    X = torch.zeros((2, 7, 16, 16), device="cuda")
    with pytest.raises(T.TfanError) as e:
        net.gradients(X, X, [0])
    assert e.value.code == T.TFAN_EINVAL
    tr = T.Cnn(1, 16, 16, train=True)
    with pytest.raises(T.TfanError):
        tr.gradients(X, X, [5])
    with pytest.raises(T.TfanError):
        tr.set_scales([1, 1, 1, 0, 1, 1, 1], np.ones(7))
