"""FP64 reference of the learned subdomain correction network (oracle; test infrastructure only).

Not in the paper: the network is the learned addition to the method.  Three affine
layers in -> h -> h -> out with ReLU after the first two; loss = mean squared error
over all outputs.  Parameter layout (one flat array): W1[in][h] b1[h] W2[h][h] b2[h]
W3[h][out] b3[out].  The gradient is pinned by central finite differences.
"""
import numpy as np


def unpack(theta, n_in, h, n_out):
    o = 0
    parts = []
    for shape in ((n_in, h), (h,), (h, h), (h,), (h, n_out), (n_out,)):
        size = int(np.prod(shape))
        parts.append(theta[o:o + size].reshape(shape))
        o += size
    return parts


def forward(theta, X, n_in, h, n_out):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64), n_in, h, n_out)
    Z1 = X @ W1 + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2 + b2
    H2 = np.maximum(Z2, 0.0)
    return H2 @ W3 + b3, (Z1, H1, Z2, H2)


def loss_and_grad(theta, X, T, n_in, h, n_out):
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64), n_in, h, n_out)
    Y, (Z1, H1, Z2, H2) = forward(theta, X, n_in, h, n_out)
    N = Y.size
    loss = np.sum((Y - T) ** 2) / N
    dY = 2.0 * (Y - T) / N
    gW3 = H2.T @ dY
    gb3 = dY.sum(axis=0)
    dH2 = (dY @ W3.T) * (Z2 > 0)
    gW2 = H1.T @ dH2
    gb2 = dH2.sum(axis=0)
    dH1 = (dH2 @ W2.T) * (Z1 > 0)
    gW1 = X.T @ dH1
    gb1 = dH1.sum(axis=0)
    return loss, np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])
