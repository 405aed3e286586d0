"""Network surrogate of the 4-body energy: parameters on the device and the
training driver around pod_mlp_train_step.

The network (Sec. IV.D, eqs. (671a)-(673a)) reads the 2/3-body descriptors
of an atom, standardised, and returns its 4-body energy.  Training fits the
per-atom 4-body energies of the exact model (the energy part of eq. (63b))
with Adam; every forward, backward and update step runs in the library's
kernels, this module only shuffles minibatches and schedules the learning
rate.  Outputs are trained in standardised units and the scale is folded
into the output layer afterwards.
"""
from __future__ import annotations

import math

import numpy as np

from . import pod

HIDDEN = pod.POD_MLP_HIDDEN


class Network:
    """theta (FP32, layout of pod.h), Adam moments, input standardisation."""

    def __init__(self, n_in: int, seed: int = 0, device="cuda"):
        import torch
        self.n_in = int(n_in)
        self.n_params = pod.pod_mlp_num_params(n_in)
        rng = np.random.default_rng(seed)
        H = HIDDEN
        W1 = rng.normal(0.0, math.sqrt(2.0 / n_in), size=(H, n_in))
        W2 = rng.normal(0.0, math.sqrt(2.0 / H), size=(H, H))
        w3 = rng.normal(0.0, math.sqrt(1.0 / H), size=H)
        theta = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), w3, [0.0]])
        assert theta.size == self.n_params
        self.device = device
        self.theta = torch.tensor(theta, dtype=torch.float32, device=device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.mu = torch.zeros(n_in, dtype=torch.float32, device=device)
        self.inv_sigma = torch.ones(n_in, dtype=torch.float32, device=device)
        self.step = 0

    def set_standardisation(self, X):
        """mu and 1/sigma of the columns of X (device tensor, rows = atoms)."""
        import torch
        Xd = X.double()
        self.mu = Xd.mean(0).float().contiguous()
        sd = Xd.std(0)
        self.inv_sigma = torch.where(sd > 0, 1.0 / sd, torch.ones_like(sd)).float().contiguous()

    def fold_output_scale(self, scale: float, shift: float):
        """y -> scale * y + shift, by rescaling w3 and b3."""
        o_w3 = self.n_params - 1 - HIDDEN
        self.theta[o_w3:o_w3 + HIDDEN] *= float(scale)
        self.theta[-1] = self.theta[-1] * float(scale) + float(shift)

    def forward(self, h: pod.Handle, X, x_col: int = 0, ldx: int | None = None, grad: bool = True):
        """(y, dy/dX) for the rows of X (device tensor in the handle dtype)."""
        import torch
        n = X.shape[0]
        ldx = X.shape[1] if ldx is None else ldx
        y = torch.empty(n, dtype=torch.float32, device=self.device)
        g = torch.empty((n, self.n_in), dtype=torch.float32, device=self.device) if grad else None
        pod.pod_mlp_forward(h, n, self.n_in, X, ldx, self.theta, self.mu, self.inv_sigma, y, g, x_col=x_col)
        return y, g


def fit(h: pod.Handle, net: Network, X, target, epochs: int = 20, batch: int = 8192, lr: float = 3e-3,
        lr_min: float = 1e-4, seed: int = 0, log_every: int = 0):
    """Train net on rows X (FP32 device, n x n_in) against target (n).
    Targets are standardised for training and the scale folded back into the
    output layer at the end.  Returns the loss of the last batch of every
    epoch (standardised units)."""
    import torch
    n = X.shape[0]
    net.set_standardisation(X)
    t64 = target.double()
    t_mean, t_std = float(t64.mean()), float(t64.std())
    t_std = t_std if t_std > 0 else 1.0
    ts = ((t64 - t_mean) / t_std).float().contiguous()
    loss = torch.zeros(1, dtype=torch.float32, device=net.device)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    history = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen).to(net.device)
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            xb = X.index_select(0, idx).contiguous()
            tb = ts.index_select(0, idx).contiguous()
            k += 1
            net.step += 1
            # cosine decay from lr to lr_min
            cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * (k - 1) / max(total - 1, 1)))
            pod.pod_mlp_train_step(h, xb.shape[0], net.n_in, xb, net.n_in, tb, net.mu, net.inv_sigma, net.theta,
                                   net.m, net.v, net.step, cur, loss=loss)
        history.append(float(loss.item()))      # loss of the epoch's last batch
        if log_every and (ep + 1) % log_every == 0:
            print(f"[fit] epoch {ep + 1}/{epochs} loss {history[-1]:.4e}", flush=True)
    net.fold_output_scale(t_std, t_mean)
    return history


def four_body_dataset(model, boxes, c, n_in: int, input_model=None):
    """Training rows from full 2/3/4-body systems: inputs are 2/3-body
    descriptors (columns 1..n_in of the per-atom descriptors of input_model,
    by default of model itself) and labels the exact per-atom 4-body energies
    sum_{k in 4-body} c_k D_ik of model, both computed by the library
    (pod_descriptors, and pod_energy_forces with the 4-body coefficients
    only).  model: FP64 PodModel with 4-body terms; input_model: FP64
    2/3-body PodModel, e.g. with a higher 3-body degree; boxes: iterable of
    (pos, cell, neighbour list).  Returns (X FP32 [n, n_in], E4 FP32 [n])."""
    import torch
    m_by = model.M_by_order
    n23 = 1 + m_by[1] + m_by[2]
    if input_model is None and n_in != n23 - 1:
        raise ValueError("n_in differs from the model's 2/3-body descriptor count")
    if input_model is not None and n_in > input_model.M - 1:
        raise ValueError("n_in exceeds the input model's descriptors")
    c4 = np.array(c, dtype=np.float64)
    c4[:n23] = 0.0
    src = model if input_model is None else input_model
    Xs, Ts = [], []
    for pos, cell, nl in boxes:
        nb = pod.DeviceNeighbors.from_list(nl)
        D = src.descriptors(pos, cell, nb)
        o = model.energy_forces(pos, cell, nb, c4, forces=False, virial=False, global_desc=False)
        Xs.append(D[:, 1:n_in + 1].float())
        Ts.append(o["E_atom"].float())
        del D, o
    return torch.cat(Xs).contiguous(), torch.cat(Ts).contiguous()
