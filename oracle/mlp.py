"""FP64 reference for the learned warm start's network (not in the paper).

The paper names block Arnoldi or randomised subspace iteration as future
work for a cheaper setup (Sec. 6).  The learned warm start feeds such a
block iteration with a predicted starting basis Y (s x k) produced node by
node from per-interface-node features X (s x F) by a 3-layer perceptron

    a1 = tanh(X W1 + b1),  a2 = tanh(a1 W2 + b2),  Y = a2 W3 + b3

trained against the Arnoldi basis W (s x k, orthonormal columns) with the
rotation-invariant subspace loss

    loss = ||Y^T Y||_F^2 - 2 ||W^T Y||_F^2 + k  =  ||Y Y^T - W W^T||_F^2,

zero exactly when Y Y^T = W W^T.  dloss/dY = 4 Y (Y^T Y) - 4 W (W^T Y).
Weights are row-major (in x out); parameters are updated by Adam
(Kingma & Ba 2015) with bias correction.
"""
import numpy as np


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    a1 = np.tanh(X @ W1 + b1)
    a2 = np.tanh(a1 @ W2 + b2)
    Y = a2 @ W3 + b3
    return Y, (X, a1, a2)


def loss(Y, W):
    k = W.shape[1]
    return (np.sum((Y.T @ Y) ** 2) - 2.0 * np.sum((W.T @ Y) ** 2) + k)


def loss_grad_Y(Y, W):
    return 4.0 * Y @ (Y.T @ Y) - 4.0 * W @ (W.T @ Y)


def backward(params, cache, dY):
    W1, b1, W2, b2, W3, b3 = params
    X, a1, a2 = cache
    gW3 = a2.T @ dY
    gb3 = dY.sum(axis=0)
    d2 = (dY @ W3.T) * (1.0 - a2 ** 2)
    gW2 = a1.T @ d2
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2.T) * (1.0 - a1 ** 2)
    gW1 = X.T @ d1
    gb1 = d1.sum(axis=0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def loss_and_grad(params, X, W):
    Y, cache = forward(params, X)
    return loss(Y, W), backward(params, cache, loss_grad_Y(Y, W))


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p, g, mi, vi in zip(params, grads, m, v):
        mi = b1 * mi + (1.0 - b1) * g
        vi = b2 * vi + (1.0 - b2) * g * g
        mh = mi / (1.0 - b1 ** t)
        vh = vi / (1.0 - b2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mi)
        out_v.append(vi)
    return out_p, out_m, out_v
