"""Step-size proposer network: forward, analytic backward, Adam (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper closes (Sec. 4) by expecting better step-size controllers to help;
the proposer is a learned controller of that kind.  A 20-64-64-1 tanh network
maps features of the accepted state to y = log(h_next / h):

    x  = [log10(E_b / E + 1e-30), b = 0..15]      (shell spectrum, Sec. 3.3)
       + [log10(max(err_i, 1e-30)), last 4 accepted errors, padded with 1.0]
    z  = (x - mean) / std                         (training-set statistics)
    a1 = tanh(W1 z + b1);  a2 = tanh(W2 a1 + b2);  y = W3 a2 + b3

Parameters are one flat vector: W1 (64x20, row-major), b1 (64), W2 (64x64),
b2 (64), W3 (1x64), b3 (1): 5569 values.  The loss is the mean squared error
over a minibatch; Adam uses beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
"""
import numpy as np

NIN, NH = 20, 64
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
         ("W3", (1, NH)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out = {}
    off = 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = p[off:off + size].reshape(shape)
        off += size
    return out


def init_params(rng):
    """Glorot-uniform weights, zero biases (rng: numpy Generator)."""
    p = np.zeros(NPARAM)
    d = unpack(p)
    for name, shape in SIZES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            d[name][...] = rng.uniform(-lim, lim, size=shape)
    return p


def features(shells16, energy, accepted_errs):
    e = max(energy, 1e-300)
    x = [np.log10(s / e + 1e-30) for s in shells16]
    last = ([1.0] * 4 + list(accepted_errs))[-4:]
    x += [np.log10(max(v, 1e-30)) for v in last]
    return np.array(x)


def forward(p, z):
    """z: (B, 20) normalised features.  Returns y (B,) and the activations."""
    d = unpack(p)
    a1 = np.tanh(z @ d["W1"].T + d["b1"])
    a2 = np.tanh(a1 @ d["W2"].T + d["b2"])
    y = (a2 @ d["W3"].T + d["b3"])[:, 0]
    return y, (z, a1, a2)


def loss_and_grad(p, z, target):
    """MSE loss (1/B) sum (y - t)^2 and its gradient w.r.t. p (chain rule)."""
    d = unpack(p)
    y, (z, a1, a2) = forward(p, z)
    bsz = z.shape[0]
    r = y - target
    loss = float(np.mean(r * r))
    dy = (2.0 / bsz) * r                      # dL/dy, (B,)
    g = np.zeros_like(p)
    gd = unpack(g)
    gd["W3"][...] = dy @ a2                   # (1, 64)
    gd["b3"][...] = np.sum(dy)
    da2 = dy[:, None] * d["W3"]               # (B, 64)
    dz2 = da2 * (1.0 - a2 * a2)
    gd["W2"][...] = dz2.T @ a1
    gd["b2"][...] = np.sum(dz2, axis=0)
    da1 = dz2 @ d["W2"]
    dz1 = da1 * (1.0 - a1 * a1)
    gd["W1"][...] = dz1.T @ z
    gd["b1"][...] = np.sum(dz1, axis=0)
    return loss, g


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
