"""CPU reference of the quartet-contribution network (test infrastructure).

Plain numpy in FP64.  With ``bf16=True`` the layer inputs, weights and the
back-propagated signals are rounded to BF16 (round to nearest even) at the same
points as the GPU kernels, so GPU and CPU differ only by FP32-vs-FP64 summation;
with ``bf16=False`` it is the exact FP64 network, which the finite-difference pin
checks.

Network: x[16] -> relu(W1 x + b1)[64] -> relu(W2 h1 + b2)[64] -> w3 . h2 + b3;
loss = mean over samples of (pred - y)^2.  Flat weight vector layout:
W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3.
"""
import numpy as np

IN, H = 16, 64
O_W1, O_B1 = 0, H * IN
O_W2 = O_B1 + H
O_B2 = O_W2 + H * H
O_W3 = O_B2 + H
O_B3 = O_W3 + H
NW = O_B3 + 1


def bf16(a):
    """Round float values to the nearest BF16 (ties to even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    return (w[O_W1:O_B1].reshape(H, IN), w[O_B1:O_W2], w[O_W2:O_B2].reshape(H, H), w[O_B2:O_W3],
            w[O_W3:O_B3], w[O_B3])


def forward(w, X, bf=True):
    W1, b1, W2, b2, w3, b3 = unpack(w)
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    x = r(X)
    z1 = x @ r(W1).T + b1
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ r(W2).T + b2
    h2 = np.maximum(z2, 0.0)
    return h2 @ w3 + b3, (x, h1, h2)


def loss_and_grad(w, X, Y, bf=True):
    """Mean squared error and its gradient with respect to the flat weight vector."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    r = bf16 if bf else (lambda v: np.asarray(v, dtype=np.float64))
    n = X.shape[0]
    pred, (x, h1, h2) = forward(w, X, bf)
    e = pred - np.asarray(Y, dtype=np.float64)
    loss = float(np.mean(e * e))
    dout = 2.0 * e / n
    g = np.zeros(NW)
    g[O_W3:O_B3] = h2.T @ dout
    g[O_B3] = dout.sum()
    dz2 = np.outer(dout, w3) * (h2 > 0)
    g[O_B2:O_W3] = dz2.sum(0)
    dz2r = r(dz2)
    g[O_W2:O_B2] = (dz2r.T @ h1).reshape(-1)
    dh1 = dz2r @ r(W2)
    dz1 = r(dh1 * (h1 > 0))
    g[O_B1:O_W2] = dz1.sum(0)
    g[O_W1:O_B1] = (dz1.T @ x).reshape(-1)
    return loss, g
