"""The pins of the surrogate and observables oracles are sharp: a plausible mistake
planted (with monkeypatch, on the CPU) in oracle/cnn_oracle.py or
oracle/analysis_oracle.py makes the named pin fail."""
import numpy as np
import pytest

from oracle import analysis_oracle as A
from oracle import cnn_oracle as C
import tests.test_analysis_oracle as TA
import tests.test_cnn_oracle as TC


def conv_flipped(a, W, b=None):
    return ORIG_C["conv3x3"](a, W[:, :, ::-1, ::-1], b)


def conv_rolled_wrong(a, W, b=None):
    z = np.zeros((a.shape[0], W.shape[0]) + a.shape[2:])
    for dy in range(3):
        for dx in range(3):
            z += np.einsum("oc,nchw->nohw", W[:, :, dy, dx], np.roll(a, shift=(dy - 1, dx - 1), axis=(2, 3)))
    return z if b is None else z + b[None, :, None, None]


def input_grad_wrong(g, W):
    ga = np.zeros((g.shape[0], W.shape[1]) + g.shape[2:])
    for dy in range(3):
        for dx in range(3):
            ga += np.einsum("oc,nohw->nchw", W[:, :, dy, dx], np.roll(g, shift=(1 - dy, 1 - dx), axis=(2, 3)))
    return ga


def weight_grad_wrong(g, a):
    gW = np.zeros((g.shape[1], a.shape[1], 3, 3))
    for dy in range(3):
        for dx in range(3):
            gW[:, :, dy, dx] = np.einsum("nohw,nchw->oc", g, np.roll(a, shift=(dy - 1, dx - 1), axis=(2, 3)))
    return gW


def bf16_truncate(x):
    f = np.asarray(x, dtype=np.float32)
    u = (f.view(np.uint32) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def adam_no_bias_correction(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    return theta - lr * m / (np.sqrt(v) + eps), m, v


def loss_without_silu_grad(layers, xn, tn, quantise=True):
    saved = C.silu_grad
    C.silu_grad = lambda z: np.ones_like(z)
    try:
        return ORIG_C["loss_and_grads"](layers, xn, tn, quantise)
    finally:
        C.silu_grad = saved


def loss_half_gradient(layers, xn, tn, quantise=True):
    loss, grads = ORIG_C["loss_and_grads"](layers, xn, tn, quantise)
    return loss, [(0.5 * gw, 0.5 * gb) for gw, gb in grads]


def shell_floor(N):
    f = np.fft.fftfreq(N, d=1.0 / N)
    return np.floor(np.sqrt(f[:, None] ** 2 + f[None, :] ** 2)).astype(np.int64)


def spectra_no_half(x):
    out = ORIG_A["spectra"](x)
    out["E"] = 2.0 * out["E"]
    return out


def vorticity_sign(u):
    return A.central_dy(u[0]) - A.central_dx(u[1])


def correlations_no_mean(x):
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[-1]
    u = A.mixed_velocity(x)
    w = A.vorticity(u)
    cnt = A.shell_counts(N)
    out = {}
    for name, comps in (("uu", [u[0], u[1]]), ("ww", [w - w.mean()]), ("QQ", [x[1], x[2]])):
        c = A._autocorrelation(comps)
        out[name] = A.shell_sum(c / c[0, 0], N) / cnt
    out["count"] = cnt
    return out


def defects_full_wrap(x):
    qxx = np.asarray(x[1], dtype=np.float32)
    qxy = np.asarray(x[2], dtype=np.float32)
    th = np.float32(0.5) * np.arctan2(qxy, qxx)
    pi = np.float32(np.pi)

    def wrap(d):  # into [-pi, pi): wrong for a headless director
        d = np.where(d >= pi, d - 2 * pi, d)
        return np.where(d < -pi, d + 2 * pi, d)

    t10, t01 = np.roll(th, -1, axis=1), np.roll(th, -1, axis=0)
    t11 = np.roll(t10, -1, axis=0)
    s = wrap(t10 - th) + wrap(t11 - t10) + wrap(t01 - t11) + wrap(th - t01)
    return int(np.count_nonzero(s > pi / 2)), int(np.count_nonzero(s < -pi / 2))


def length_without_two_pi(S, N):
    k = 2.0 * np.pi * np.arange(S.size) / N
    return float(S[1:].sum() / (k[1:] * S[1:]).sum())


def overlaps_without_two(x0, x1):
    o = ORIG_A["temporal_overlaps"](x0, x1)
    o[4:] *= 0.5
    return o


ORIG_C = {k: getattr(C, k) for k in ("loss_and_grads", "conv3x3")}
ORIG_A = {k: getattr(A, k) for k in ("spectra", "temporal_overlaps")}

MUTATIONS = [
    (C, "conv: kernel flipped", "conv3x3", conv_flipped, TC.test_conv_delta_response_orientation),
    (C, "conv: roll in the wrong direction", "conv3x3", conv_rolled_wrong, TC.test_conv_matches_brute_force_loops),
    (C, "input gradient: taps not reversed", "conv3x3_input_grad", input_grad_wrong,
     TC.test_conv_gradients_are_adjoints),
    (C, "weight gradient: roll in the wrong direction", "conv3x3_weight_grad", weight_grad_wrong,
     TC.test_conv_gradients_are_adjoints),
    (C, "SiLU': dropped z (1 - s) term", "silu_grad", lambda z: C.sigmoid(z), TC.test_silu_and_sigmoid),
    (C, "sigmoid with the wrong sign", "sigmoid", lambda z: 1.0 / (1.0 + np.exp(z)), TC.test_silu_and_sigmoid),
    (C, "bfloat16 truncation instead of rounding", "bf16", bf16_truncate, TC.test_bf16_rounding_values),
    (C, "Adam without bias correction", "adam", adam_no_bias_correction, TC.test_adam_closed_forms),
    (C, "back-propagation without SiLU'", "loss_and_grads", loss_without_silu_grad,
     TC.test_loss_gradients_against_finite_differences),
    (C, "loss gradient missing the factor 2", "loss_and_grads", loss_half_gradient,
     TC.test_loss_gradients_against_finite_differences),
    (A, "shell = floor(|n|)", "shell_index", shell_floor, TA.test_shell_index_values),
    (A, "E without the 1/2", "spectra", spectra_no_half, TA.test_single_mode_spectra_and_length),
    (A, "hat without 1/N^2", "hat", lambda f: np.fft.fft2(f), TA.test_parseval_for_a_random_state),
    (A, "vorticity with the wrong sign", "vorticity", vorticity_sign, TA.test_vorticity_of_shear_modes),
    (A, "C_uu without removing the mean flow", "correlations", correlations_no_mean,
     TA.test_correlations_against_brute_force),
    (A, "defect angles wrapped into [-pi, pi)", "defects", defects_full_wrap, TA.test_constructed_defects),
    (A, "L without 2 pi", "domain_length_from_spectrum", length_without_two_pi,
     TA.test_single_mode_spectra_and_length),
    (A, "Q:Q without the factor 2", "temporal_overlaps", overlaps_without_two, TA.test_overlap_norms_closed_form),
]


@pytest.mark.parametrize("module,name,attr,wrong,pin", MUTATIONS, ids=[m[1] for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, module, name, attr, wrong, pin):
    pin()  # the unmutated oracle passes the pin
    monkeypatch.setattr(module, attr, wrong)
    with np.errstate(all="ignore"), pytest.raises(AssertionError):
        pin()
