"""FP64 CPU oracle of the sizing network (test infrastructure only).

A 32-64-64-2 multilayer perceptron with ReLU hidden layers, mean-squared-error
loss and Adam (Kingma & Ba, 2015).  This network is not in the paper; it is
the learned sizing component that picks the sketch size and power count.
Parameter packing (shared *format* with the GPU side, not code): W1 (64x32),
b1 (64), W2 (64x64), b2 (64), W3 (2x64), b3 (2), each row-major, W[out][in],
concatenated in that order (6402 values).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.
"""
import numpy as np

DIMS = (32, 64, 64, 2)


def n_params(dims=DIMS):
    return sum(dims[i + 1] * dims[i] + dims[i + 1] for i in range(len(dims) - 1))


def unpack(theta, dims=DIMS):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for i in range(len(dims) - 1):
        fi, fo = dims[i], dims[i + 1]
        W = theta[o:o + fo * fi].reshape(fo, fi)
        o += fo * fi
        b = theta[o:o + fo]
        o += fo
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def forward(theta, X, dims=DIMS):
    """Y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 for each row x of X."""
    layers = unpack(theta, dims)
    acts = [np.asarray(X, dtype=np.float64)]
    pre = []
    h = acts[0]
    for i, (W, b) in enumerate(layers):
        z = h @ W.T + b
        pre.append(z)
        h = np.maximum(z, 0.0) if i < len(layers) - 1 else z
        acts.append(h)
    return h, (acts, pre)


def loss(theta, X, T, dims=DIMS):
    """Mean over the batch of the squared error summed over outputs, / 2."""
    Y, _ = forward(theta, X, dims)
    d = Y - T
    return 0.5 * float(np.sum(d * d)) / X.shape[0]


def grad(theta, X, T, dims=DIMS):
    """Gradient of loss() with respect to the packed parameters (backprop)."""
    layers = unpack(theta, dims)
    Y, (acts, pre) = forward(theta, X, dims)
    B = X.shape[0]
    g = (Y - T) / B
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        if i < len(layers) - 1:
            g = g * (pre[i] > 0)
        grads[i] = (g.T @ acts[i], g.sum(axis=0))
        g = g @ W
    return pack(grads)


def adam_step(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; step counts from 1.  Returns (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
