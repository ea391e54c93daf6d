"""FP64 reference of the warm-start multilayer perceptron (test infrastructure only).

n_in -> width (tanh) -> width (tanh) -> n_out (linear); parameters packed as
(W1 [width][n_in], b1, W2 [width][width], b2, W3 [n_out][width], b3); loss = mean
squared error over all outputs.  Gradients by reverse-mode differentiation
written out layer by layer; pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np


def unpack(theta, n_in, width, n_out):
    o = 0
    out = []
    for shape in ((width, n_in), (width,), (width, width), (width,), (n_out, width), (n_out,)):
        size = int(np.prod(shape))
        out.append(np.asarray(theta[o:o + size], dtype=np.float64).reshape(shape))
        o += size
    return out


def forward(theta, X, n_in, width, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, width, n_out)
    A1 = np.tanh(X @ W1.T + b1)
    A2 = np.tanh(A1 @ W2.T + b2)
    return A2 @ W3.T + b3, (A1, A2)


def loss_grad(theta, X, T, n_in, width, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, width, n_out)
    X = np.asarray(X, dtype=np.float64)
    Y, (A1, A2) = forward(theta, X, n_in, width, n_out)
    D = Y - T
    loss = np.mean(D * D)
    dY = 2.0 * D / D.size
    gW3 = dY.T @ A2
    gb3 = dY.sum(0)
    dZ2 = (dY @ W3) * (1.0 - A2 * A2)
    gW2 = dZ2.T @ A1
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * (1.0 - A1 * A1)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(0)
    return loss, np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])
