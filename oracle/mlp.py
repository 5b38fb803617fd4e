"""CPU fp64 reference of the scheduler's order-cost network (test infrastructure).

Only tests, the smoke check and the benchmark's CPU baseline use this module;
the library never does. The network is not from the paper (the paper computes
one static matching order per start edge, Section VI); it is the library's
learned addition, defined here in plain numpy:

    h1 = relu(x W1 + b1)      W1: 24 x 64
    h2 = relu(h1 W2 + b2)     W2: 64 x 64
    y  = h2 . W3 + b3         W3: 64

with the weights flattened as W1, b1, W2, b2, W3, b3 (row-major), 5,825
values. Training minimises the mean squared error over a minibatch with Adam
(Kingma and Ba, "Adam: A method for stochastic optimization", ICLR 2015,
Algorithm 1: beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments).

Pins (tests/test_oracle_mlp.py): the analytic gradient equals central finite
differences; closed forms for networks whose hidden units are all off or all
linear; Adam's first step moves every weight with a nonzero gradient by
lr * g / (|g| + eps); bfloat16 rounding against exactly representable values
and ties, and the half-unit error bound; bf16 inference rounds the inputs
and both hidden layers (a one-path network whose activations sit just off,
on, and past bfloat16 midpoints, with hand-derived outputs).
"""
import numpy as np

N_IN, N_HID = 24, 64
N_WEIGHTS = N_IN * N_HID + N_HID + N_HID * N_HID + N_HID + N_HID + 1


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (N_WEIGHTS,)
    o = 0
    W1 = w[o:o + N_IN * N_HID].reshape(N_IN, N_HID)
    o += N_IN * N_HID
    b1 = w[o:o + N_HID]
    o += N_HID
    W2 = w[o:o + N_HID * N_HID].reshape(N_HID, N_HID)
    o += N_HID * N_HID
    b2 = w[o:o + N_HID]
    o += N_HID
    W3 = w[o:o + N_HID]
    o += N_HID
    b3 = w[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, W3, [b3]]).astype(np.float64)


def forward(w, X):
    """Outputs y (n,) for inputs X (n, 24)."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ W3 + b3


def loss_and_grad(w, X, T):
    """Mean squared error over the samples and its gradient (flat, like w),
    by the chain rule through each layer."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    n = len(X)
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    err = y - T
    loss = float(np.mean(err * err))
    dy = 2.0 * err / n                      # dL/dy
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    dz2 = np.outer(dy, W3) * (z2 > 0)       # through relu of layer 2
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * (z1 > 0)           # through relu of layer 1
    gW1 = X.T @ dz1
    gb1 = dz1.sum(axis=0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(w, m1, m2, g, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1). Returns new (w, m1, m2)."""
    m1 = beta1 * m1 + (1.0 - beta1) * g
    m2 = beta2 * m2 + (1.0 - beta2) * g * g
    mhat = m1 / (1.0 - beta1 ** step)
    vhat = m2 / (1.0 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


def bf16_round(a):
    """Rounds float32 values to the nearest bfloat16 (ties to even), as float64.
    The bfloat16 of a float32 keeps its top 16 bits; rounding adds half of the
    dropped part's unit plus the kept part's lowest bit (for ties) first."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    keep_odd = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + keep_odd) & np.uint64(0xFFFF0000)).astype(np.uint32)
    finite = np.isfinite(a)
    out = np.where(finite, r.view(np.float32), a)
    return out.astype(np.float64)


def forward_bf16(w, X):
    """bf16 inference, by the usual mixed-precision convention: every operand
    of every product is bfloat16 (all weights and biases, the inputs, and
    both hidden layers' activations, each rounded to nearest-even from
    float32), and every sum is taken in wider precision (exact fp64 here).
    The output is not rounded."""
    W1, b1, W2, b2, W3, b3 = unpack(bf16_round(np.asarray(w, dtype=np.float32)))
    Xr = bf16_round(np.asarray(X, dtype=np.float32))
    h1 = np.maximum(Xr @ W1 + b1, 0.0)
    h1r = bf16_round(h1.astype(np.float32))
    h2 = np.maximum(h1r @ W2 + b2, 0.0)
    h2r = bf16_round(h2.astype(np.float32))
    return h2r @ W3 + b3
