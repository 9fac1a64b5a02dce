"""FP64 CPU oracle of the convolutional surrogate (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU baseline may import this
module; the product path never does.

The surrogate of the Numerical Simulation / Results workflow advances the solver
state (phi, Qxx, Qxy, u_a, u_p: 7 channels) by k lattice steps.  Its network:
six 3x3 convolutions on the periodic grid, 7 -> 48 -> 48 -> 48 -> 48 -> 48 -> 7
channels, SiLU (x sigmoid(x)) after the first five, acting on the state divided
by fixed per-channel input scales s_in; the last layer's output y is the
increment in units of per-channel output scales s_out, prediction = x + s_out y.
Loss: mean over samples, channels and sites of (y - (x_target - x) / s_out)^2.
Optimiser: Adam (Kingma and Ba, 2015).

Quantisation points (quantise=True) follow the stated precision of the GPU
path: the network input, the weights, every stored activation and every
back-propagated pre-activation gradient are rounded to bfloat16 (round to
nearest, ties to even); sums are exact here (float64) where the GPU accumulates
in float32.  With quantise=False every function is the plain float64 definition.

Arrays: a batch is [B][C][H][W]; weights W[co][ci][dy][dx] with tap offset
(dy - 1, dx - 1); bias b[co].
"""
from __future__ import annotations

import numpy as np

CHANNELS, HIDDEN, LAYERS = 7, 48, 6


def layer_shapes():
    """(c_out, c_in) of each layer."""
    dims = [CHANNELS] + [HIDDEN] * (LAYERS - 1) + [CHANNELS]
    return [(dims[i + 1], dims[i]) for i in range(LAYERS)]


def param_count():
    return sum(co * ci * 9 + co for co, ci in layer_shapes())


def unflatten(theta):
    """Flat parameter vector -> [(W, b)] per layer (W then b, layer by layer)."""
    out, o = [], 0
    for co, ci in layer_shapes():
        W = np.asarray(theta[o:o + co * ci * 9], dtype=np.float64).reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = np.asarray(theta[o:o + co], dtype=np.float64)
        o += co
        out.append((W, b))
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16(x):
    """Round to the nearest bfloat16 (8 significant bits, ties to even), via the
    binary32 value of x, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def conv3x3(a, W, b=None):
    """Periodic 3x3 convolution: z[n,o,y,x] = b[o] + sum_{c,dy,dx} W[o,c,dy,dx] a[n,c,y+dy-1,x+dx-1]."""
    z = np.zeros((a.shape[0], W.shape[0]) + a.shape[2:])
    for dy in range(3):
        for dx in range(3):
            # np.roll(a, s)[i] = a[i - s]; the tap reads a[i + d] with d = dy - 1
            sh = np.roll(a, shift=(1 - dy, 1 - dx), axis=(2, 3))
            z += np.einsum("oc,nchw->nohw", W[:, :, dy, dx], sh)
    if b is not None:
        z += b[None, :, None, None]
    return z


def conv3x3_input_grad(g, W):
    """Gradient of sum(g * conv3x3(a, W)) with respect to a:
    ga[n,c,y,x] = sum_{o,dy,dx} W[o,c,dy,dx] g[n,o,y-dy+1,x-dx+1]."""
    ga = np.zeros((g.shape[0], W.shape[1]) + g.shape[2:])
    for dy in range(3):
        for dx in range(3):
            sh = np.roll(g, shift=(dy - 1, dx - 1), axis=(2, 3))
            ga += np.einsum("oc,nohw->nchw", W[:, :, dy, dx], sh)
    return ga


def conv3x3_weight_grad(g, a):
    """Gradient of sum(g * conv3x3(a, W)) with respect to W:
    gW[o,c,dy,dx] = sum_{n,y,x} g[n,o,y,x] a[n,c,y+dy-1,x+dx-1]."""
    gW = np.zeros((g.shape[1], a.shape[1], 3, 3))
    for dy in range(3):
        for dx in range(3):
            sh = np.roll(a, shift=(1 - dy, 1 - dx), axis=(2, 3))
            gW[:, :, dy, dx] = np.einsum("nohw,nchw->oc", g, sh)
    return gW


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(layers, xn, quantise=True):
    """Network on normalised input xn [B][7][H][W]; returns y and the cache
    (stored activations a_0..a_5 and pre-activations z_1..z_6)."""
    q = bf16 if quantise else (lambda v: v)
    a = q(xn)
    acts, pre = [a], []
    for i, (W, b) in enumerate(layers):
        z = conv3x3(a, q(W), b)
        pre.append(z)
        if i < LAYERS - 1:
            a = q(silu(z))
            acts.append(a)
    return pre[-1], dict(acts=acts, pre=pre)


def loss_and_grads(layers, xn, tn, quantise=True):
    """Loss mean((y - tn)^2) and its gradients [(gW, gb)] for input xn and
    target increment tn (both normalised)."""
    q = bf16 if quantise else (lambda v: v)
    y, cache = forward(layers, xn, quantise)
    d = y - tn
    loss = float(np.mean(d * d))
    g = q(2.0 * d / d.size)                      # dL/dz of the last layer
    grads = [None] * LAYERS
    for i in range(LAYERS - 1, -1, -1):
        W, _ = layers[i]
        a_in = cache["acts"][i]
        grads[i] = (conv3x3_weight_grad(g, a_in), g.sum(axis=(0, 2, 3)))
        if i > 0:
            ga = conv3x3_input_grad(g, q(W))
            g = q(ga * silu_grad(cache["pre"][i - 1]))
    return loss, grads


def adam(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(layers, x, s_in, s_out, quantise=True):
    """State after k steps from state x [B][7][H][W] (physical units)."""
    si = np.asarray(s_in, dtype=np.float64)[None, :, None, None]
    so = np.asarray(s_out, dtype=np.float64)[None, :, None, None]
    y, _ = forward(layers, x / si, quantise)
    return x + so * y


def init_params(seed=0, gain=1.0, zero_last=True):
    """He-style uniform initial weights (fan-in 9 c_in), zero biases; with
    zero_last the last layer starts at zero, so the untrained surrogate is the
    identity map."""
    rng = np.random.default_rng(seed)
    layers = []
    for i, (co, ci) in enumerate(layer_shapes()):
        lim = gain * np.sqrt(6.0 / (9 * ci))
        W = rng.uniform(-lim, lim, size=(co, ci, 3, 3))
        if i == LAYERS - 1 and zero_last:
            W[:] = 0.0
        layers.append((W, np.zeros(co)))
    return layers
