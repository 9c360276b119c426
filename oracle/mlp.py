"""CPU reference of the learned surrogate's network (test infrastructure only: imported by
tests/, never by the library).

The surrogate maps four inputs (separation L/R, log10 of the shear modulus, film height
over the capsule diameter, contact angle) to two outputs (lateral capillary force,
meniscus deformation) with a multilayer perceptron 4 -> 64 -> 64 -> 64 -> 2, tanh on the
hidden layers, 8770 parameters.  Training minimises the mean squared error
L = (1 / 2n) sum over the n weighted samples and the outputs of (y - t)^2 with Adam
(Kingma & Ba, 2015).

Precision: "mixed" is the arithmetic of the GPU kernels written out plainly: every matrix
product rounds both operands to bfloat16 (round to nearest even) and sums the exact
products in float64 (the kernels sum in float32); biases, tanh, the loss and Adam are
float64.  mixed=False is plain float64 throughout (used to pin the gradient by finite
differences).

Parameter vector layout: W1 [4][64], b1 [64], W2 [64][64], b2, W3 [64][64], b3,
W4 [64][2], b4 [2]; every W is [inputs][outputs], row-major, y = x W + b.
"""
import numpy as np

DIMS = (4, 64, 64, 64, 2)
N_PARAMS = sum(DIMS[i] * DIMS[i + 1] + DIMS[i + 1] for i in range(len(DIMS) - 1))


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even); returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    """Parameter vector -> [(W, b)] per layer (views)."""
    out, o = [], 0
    for i in range(len(DIMS) - 1):
        k, n = DIMS[i], DIMS[i + 1]
        W = theta[o:o + k * n].reshape(k, n)
        o += k * n
        b = theta[o:o + n]
        o += n
        out.append((W, b))
    assert o == len(theta) == N_PARAMS
    return out


def _mm(a, b, mixed):
    if mixed:
        return bf16(a) @ bf16(b)
    return a @ b


def forward(theta, x, mixed=True):
    """Outputs y [n][2] and the activations (input, then each hidden layer's tanh)."""
    layers = unpack(np.asarray(theta, dtype=np.float64))
    acts = [np.asarray(x, dtype=np.float64)]
    h = acts[0]
    for i, (W, b) in enumerate(layers):
        z = _mm(h, W, mixed) + b
        if i < len(layers) - 1:
            h = np.tanh(z)
            acts.append(h)
        else:
            h = z
    return h, acts


def loss_and_grad(theta, x, t, w=None, mixed=True):
    """Loss and its gradient with respect to the parameter vector (back-propagation, with
    the same rounding points as the forward pass in mixed mode).  w: per-sample weights
    (default 1); the mean runs over sum(w)."""
    theta = np.asarray(theta, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    w = np.ones(len(x)) if w is None else np.asarray(w, dtype=np.float64)
    n = w.sum()
    layers = unpack(theta)
    y, acts = forward(theta, x, mixed)
    r = (y - t) * w[:, None]
    loss = 0.5 * float(np.sum(r * (y - t))) / n
    d = r / n                                   # dL/dy
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        a = acts[i]
        gW = _mm(a.T, d, mixed)
        gb = d.sum(axis=0)
        grads.append((gW, gb))
        if i > 0:
            d = _mm(d, W.T, mixed) * (1.0 - a * a)
    g = []
    for gW, gb in reversed(grads):
        g.append(gW.ravel())
        g.append(gb)
    return loss, np.concatenate(g)


def adam(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
