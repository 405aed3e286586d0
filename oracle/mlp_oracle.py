"""Plain FP64 CPU oracle of the neural-network surrogate for the 4-body energy.

Test infrastructure, not product code.  Only the test suite, the smoke check
and the benchmark's CPU leg import this module; the HIP library and its
binding never call it, and it shares no code with them.

The network follows the neural-network regression of arXiv:2212.14446,
Sec. IV.D, eqs. (671a)-(673a): hidden layers D^l = sigma(W^l D^(l-1) + b^l),
an energy that is linear in the last hidden layer, and forces by reverse
differentiation through the layers and then through the descriptors.  Here
it stands in for the 4-body part of the linear POD energy only:

    E_i = c23 . D23_i + y(x_i),   x_i = (D23_i[1:] - mu) * inv_sigma

with D23_i the constant, 2- and 3-body descriptors of atom i (eqs. (12b),
(26a)), two hidden layers of width 64, sigma = SiLU, and
y = w3 . h2 + b3.  Training minimises the per-atom energy part of the loss of
Sec. IV.C, eq. (63b) (mean squared error against exact 4-body energies) with
Adam (Kingma and Ba, 2015, Algorithm 1).

Precision model of the device kernels, reproduced here when bf16=True: the
standardised inputs, both weight matrices, the first hidden activation and
the two back-propagated pre-activation gradients are rounded to bfloat16
(round to nearest even) where they enter a matrix product; every product
accumulates in higher precision (FP32 on the device, FP64 here); the output
layer, biases and activation functions stay in full precision.  With
bf16=False the same functions are the exact FP64 network, pinned by finite
differences.
"""
from __future__ import annotations

import numpy as np

N_HIDDEN = 64


def n_params(n_in: int) -> int:
    """Parameter count; layout of theta: W1 [64, n_in], b1 [64], W2 [64, 64],
    b2 [64], w3 [64], b3 [1] (row-major, concatenated)."""
    H = N_HIDDEN
    return H * n_in + H + H * H + H + H + 1


def unpack(theta, n_in: int):
    H = N_HIDDEN
    t = np.asarray(theta, dtype=np.float64)
    if t.size != n_params(n_in):
        raise ValueError("wrong parameter count")
    o = 0
    W1 = t[o:o + H * n_in].reshape(H, n_in); o += H * n_in
    b1 = t[o:o + H]; o += H
    W2 = t[o:o + H * H].reshape(H, H); o += H * H
    b2 = t[o:o + H]; o += H
    w3 = t[o:o + H]; o += H
    b3 = t[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(w3),
                           np.atleast_1d(b3)]).astype(np.float64)


def bf16_round(x):
    """Round to bfloat16 (8 significant bits, round to nearest, ties to even)
    by integer arithmetic on the float32 bit pattern; returns float64.
    Values are taken to float32 first, as the device holds them."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(f.shape)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_prime(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _round(x, on):
    return bf16_round(x) if on else np.asarray(x, dtype=np.float64)


def forward(theta, X, mu, inv_sigma, bf16: bool = True):
    """Network output y [N] for raw inputs X [N, n_in], with the
    intermediate values the backward passes need."""
    X = np.asarray(X, dtype=np.float64)
    n_in = X.shape[1]
    W1, b1, W2, b2, w3, b3 = unpack(theta, n_in)
    x = _round((X - np.asarray(mu)) * np.asarray(inv_sigma), bf16)
    W1r, W2r = _round(W1, bf16), _round(W2, bf16)
    z1 = x @ W1r.T + b1
    h1 = silu(z1)
    h1r = _round(h1, bf16)
    z2 = h1r @ W2r.T + b2
    h2 = silu(z2)
    y = h2 @ w3 + b3
    return {"y": y, "x": x, "z1": z1, "h1r": h1r, "z2": z2, "h2": h2, "W1r": W1r, "W2r": W2r, "w3": w3}


def input_gradient(theta, X, mu, inv_sigma, bf16: bool = True):
    """(y [N], dy/dX [N, n_in]) by reverse differentiation (eq. (673a))."""
    f = forward(theta, X, mu, inv_sigma, bf16)
    dz2 = _round(f["w3"][None, :] * silu_prime(f["z2"]), bf16)
    dh1 = dz2 @ f["W2r"]
    dz1 = _round(dh1 * silu_prime(f["z1"]), bf16)
    dx = dz1 @ f["W1r"]
    return f["y"], dx * np.asarray(inv_sigma)[None, :]


def loss_and_grad(theta, X, target, mu, inv_sigma, bf16: bool = True):
    """Mean squared error over the batch and its gradient with respect to
    theta (same layout as theta)."""
    f = forward(theta, X, mu, inv_sigma, bf16)
    N = X.shape[0]
    r = f["y"] - np.asarray(target, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / N
    db3 = dy.sum()
    dw3 = f["h2"].T @ dy
    dz2 = _round(dy[:, None] * f["w3"][None, :] * silu_prime(f["z2"]), bf16)
    dW2 = dz2.T @ f["h1r"]
    db2 = dz2.sum(0)
    dh1 = dz2 @ f["W2r"]
    dz1 = _round(dh1 * silu_prime(f["z1"]), bf16)
    dW1 = dz1.T @ f["x"]
    db1 = dz1.sum(0)
    return loss, pack(dW1, db1, dW2, db2, dw3, db3)


def adam_step(theta, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1); step counts from 1.
    Returns new (theta, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return np.asarray(theta, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v


def forces_from_atom_weights(pos, cell, offsets, nbr_j, shift, p, Q, C):
    """Forces and virial of an energy whose derivative with respect to the
    descriptors of atom i is the row C_i (eq. (673a) with the descriptor
    derivatives of eqs. (26c), (24c) from the POD oracle):
    dE_i/dr_ij = sum_k C_ik dD_ik/dr_ij, F_n = -dE/dr_n,
    W_ab = -sum_pairs r_ij,a dE_i/dr_ij,b."""
    from oracle import pod_oracle as po
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    C = np.asarray(C, dtype=np.float64)
    dD, centre, pidx = po.descriptor_derivatives(pos, cell, offsets, nbr_j, shift, p, Q)
    F = np.zeros((N, 3))
    W = np.zeros((3, 3))
    if len(pidx):
        g = np.einsum("pm,pmd->pd", C[centre], dD)
        np.add.at(F, centre, g)
        np.add.at(F, np.asarray(nbr_j)[pidx], -g)
        _, pidx2, d = po.pair_vectors(pos, cell, offsets, nbr_j, shift)
        dmap = np.zeros((len(nbr_j), 3))
        dmap[pidx2] = d
        W -= dmap[pidx].T @ g
    return F, W


def surrogate_energy_forces(pos, cell, offsets, nbr_j, shift, p23, Q, c23, theta, mu, inv_sigma,
                            bf16: bool = True):
    """Energies, forces and virial of E_i = c23 . D23_i + y(x_i).

    p23 is a 2/3-body parameter set (K4 = 0) of the POD oracle; the network
    input is D23_i without its constant column.  Forces follow eq. (673a)
    with the per-atom weights C_i = c23 + (0, dy/dX_i)."""
    from oracle import pod_oracle as po
    pos = np.asarray(pos, dtype=np.float64)
    N = pos.shape[0]
    D = po.descriptors_fast(pos, cell, offsets, nbr_j, shift, p23, Q)
    y, dydx = input_gradient(theta, D[:, 1:], mu, inv_sigma, bf16)
    c23 = np.asarray(c23, dtype=np.float64)
    E_atom = D @ c23 + y
    C = c23[None, :] + np.concatenate([np.zeros((N, 1)), dydx], axis=1)
    F, W = forces_from_atom_weights(pos, cell, offsets, nbr_j, shift, p23, Q, C)
    return {"E_atom": E_atom, "E": float(E_atom.sum()), "F": F, "W": W, "y": y, "dydx": dydx, "D": D}
