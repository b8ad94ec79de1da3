"""Test infrastructure (oracle): the tree-shape perceptron in float64.

Only tests, smoke() and the CPU-baseline leg of the bench use this module.
A two-hidden-layer ReLU perceptron, y = relu(relu(x W1 + b1) W2 + b2) W3 + b3,
its weighted squared error L = (1/B) sum_b sum_o w_o (y_bo - t_bo)^2, the
gradient of L by the chain rule written out layer by layer (ReLU'(0) = 0),
and one Adam step (Kingma and Ba 2015, bias-corrected).  Parameters are one
flat array, row-major with the input index first: W1, b1, W2, b2, W3, b3.
"""
import numpy as np


def sizes(d_in, h, d_out):
    return [(d_in, h), (h,), (h, h), (h,), (h, d_out), (d_out,)]


def unpack(p, d_in, h, d_out):
    out, o = [], 0
    for shp in sizes(d_in, h, d_out):
        k = int(np.prod(shp))
        out.append(np.asarray(p[o:o + k], np.float64).reshape(shp))
        o += k
    assert o == len(p)
    return out


def pack(parts):
    return np.concatenate([np.asarray(a, np.float64).ravel() for a in parts])


def forward(p, x, d_in, h, d_out):
    W1, b1, W2, b2, W3, b3 = unpack(p, d_in, h, d_out)
    x = np.asarray(x, np.float64)
    a1 = x @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    return h2 @ W3 + b3


def loss(p, x, t, w, d_in, h, d_out):
    y = forward(p, x, d_in, h, d_out)
    return float(np.sum(np.asarray(w) * (y - t) ** 2) / x.shape[0])


def loss_grad(p, x, t, w, d_in, h, d_out):
    W1, b1, W2, b2, W3, b3 = unpack(p, d_in, h, d_out)
    x = np.asarray(x, np.float64)
    B = x.shape[0]
    a1 = x @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ W3 + b3
    dy = 2.0 * np.asarray(w) * (y - t) / B
    gW3 = h2.T @ dy
    gb3 = dy.sum(0)
    dh2 = (dy @ W3.T) * (a2 > 0)
    gW2 = h1.T @ dh2
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ W2.T) * (a1 > 0)
    gW1 = x.T @ dh1
    gb1 = dh1.sum(0)
    L = float(np.sum(np.asarray(w) * (y - t) ** 2) / B)
    return L, pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
