"""Network kernels (bfloat16 MFMA, FP32 accumulation) and the surrogate energy
path against the FP64 network oracle with the same bfloat16 rounding points.

Tolerance: the device accumulates in FP32 and the oracle in FP64, so a value
that the oracle rounds to bfloat16 can land on the other side of a rounding
boundary on the device (probability ~1e-7 / 2^-9 per rounded value).  Such a
flip moves one activation by one bfloat16 step (2^-8 relative), which moves
that atom's output by at most ~1e-3 relative; every other atom agrees to FP32
accumulation error.  The tests therefore bound the worst atom at 2e-3
(normwise) and allow at most 5% of atoms above 1e-4."""
import numpy as np
import pytest

from gpu_common import oracle_params, relerr, say
from oracle import mlp_oracle as mo
from oracle import pod_oracle as po
from paper_2212_14446_amd import pod, surrogate, workloads as wl

pytestmark = pytest.mark.gpu

WORST, TYPICAL = 2e-3, 1e-4


def per_row_rel(x, ref):
    x = np.asarray(x, dtype=np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(len(ref), -1)
    scale = np.max(np.abs(ref))
    return np.max(np.abs(x - ref), axis=1) / scale


def check(x, ref, name):
    r = per_row_rel(x, ref)
    frac = float(np.mean(r > TYPICAL))
    say(f"[gpu]   {name}: worst {r.max():.2e}, median {np.median(r):.2e}, rows above {TYPICAL:g}: {frac:.1%}")
    assert r.max() < WORST, name
    assert frac <= 0.05, name


def rand_case(n, n_in, seed):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, 1.0, size=mo.n_params(n_in))
    theta[: 64 * n_in] *= np.sqrt(2.0 / n_in)
    theta[64 * n_in + 64: 64 * n_in + 64 + 4096] *= np.sqrt(2.0 / 64)
    theta[-65:] *= 0.2
    X = rng.normal(0.5, 2.0, size=(n, n_in))
    mu = rng.normal(0.5, 0.1, size=n_in)
    inv_sigma = rng.uniform(0.3, 0.7, size=n_in)
    # the device reads FP32 parameters: the oracle uses the same values
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return f32(theta), X, f32(mu), f32(inv_sigma)


def handle(dtype="f64"):
    return pod.PodModel(pod.setup_from_workload(wl.SETUP_CFG1), dtype)


@pytest.mark.parametrize("n,n_in,dtype", [(1000, 36, "f64"), (1000, 36, "f32"), (77, 7, "f64"), (300, 64, "f32"),
                                          (16, 50, "f64"), (1, 36, "f32")])
def test_mlp_forward_vs_oracle(n, n_in, dtype):
    import torch
    theta, X, mu, isg = rand_case(n, n_in, 100 + n + n_in)
    td = torch.float64 if dtype == "f64" else torch.float32
    Xd = X if dtype == "f64" else X.astype(np.float32).astype(np.float64)
    m = handle(dtype)
    f = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    # rows with a stride: the inputs sit at columns 2.. of a wider matrix
    Xw = np.zeros((n, n_in + 3))
    Xw[:, 2:2 + n_in] = Xd
    Xt = torch.tensor(Xw, dtype=td, device="cuda")
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    g = torch.empty((n, n_in), dtype=torch.float32, device="cuda")
    say(f"[gpu] mlp forward n={n} n_in={n_in} {dtype}")
    pod.pod_mlp_forward(m.h, n, n_in, Xt, n_in + 3, f(theta), f(mu), f(isg), y, g, x_col=2)
    torch.cuda.synchronize()
    y_ref, g_ref = mo.input_gradient(theta, Xd, mu, isg, bf16=True)
    check(y.cpu().numpy(), y_ref, "y")
    check(g.cpu().numpy(), g_ref, "dy/dX")


def test_mlp_train_step_vs_oracle():
    import torch
    n, n_in = 2000, 36
    theta, X, mu, isg = rand_case(n, n_in, 7)
    X = X.astype(np.float32).astype(np.float64)
    t = np.random.default_rng(8).normal(size=n).astype(np.float32).astype(np.float64)
    m = handle("f32")
    f = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    th, mm, vv, loss = f(theta), f(np.zeros_like(theta)), f(np.zeros_like(theta)), torch.zeros(1, device="cuda")
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    pod.pod_mlp_train_step(m.h, n, n_in, f(X), n_in, f(t), f(mu), f(isg), th, mm, vv, 1, lr, b1, b2, eps, loss)
    torch.cuda.synchronize()
    L_ref, g_ref = mo.loss_and_grad(theta, X, t, mu, isg, bf16=True)
    # the device holds beta1, beta2 in FP32: 1 - beta in FP32 arithmetic
    c1 = float(np.float32(1.0) - np.float32(b1))
    c2 = float(np.float32(1.0) - np.float32(b2))
    g_dev = mm.double().cpu().numpy() / c1
    say(f"[gpu] train step: loss {float(loss.item()):.6e} ref {L_ref:.6e}; grad rel {relerr(g_dev, g_ref):.2e}")
    assert float(loss.item()) == pytest.approx(L_ref, rel=1e-4)
    assert relerr(g_dev, g_ref) < WORST
    # second moment and the update itself, from the device's own moments
    assert relerr(vv.double().cpu().numpy(), c2 * g_dev ** 2) < 1e-5
    mh, vh = mm.double().cpu().numpy() / c1, vv.double().cpu().numpy() / c2
    t_ref = theta - lr * mh / (np.sqrt(vh) + eps)
    assert np.max(np.abs(th.double().cpu().numpy() - t_ref)) < 1e-6


def test_mlp_train_step_deterministic():
    import torch
    n, n_in = 1500, 36
    theta, X, mu, isg = rand_case(n, n_in, 9)
    t = np.random.default_rng(10).normal(size=n)
    m = handle("f32")
    f = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    out = []
    for _ in range(2):
        th, mm, vv = f(theta), f(np.zeros_like(theta)), f(np.zeros_like(theta))
        for step in (1, 2, 3):
            pod.pod_mlp_train_step(m.h, n, n_in, f(X), n_in, f(t), f(mu), f(isg), th, mm, vv, step, 1e-3)
        torch.cuda.synchronize()
        out.append(th.cpu().numpy().copy())
    assert np.array_equal(out[0], out[1])


def _oracle_fit(theta, X, target, epochs, batch, lr, seed, lr_min=1e-4):
    """The training schedule of surrogate.fit written out on the FP64 network
    oracle (same bfloat16 rounding points): the FP32-rounded inputs, the
    same standardisation, the same minibatch permutations (torch's CPU
    generator with the same seed), Adam with the same cosine decay.
    Returns the loss of every epoch's last batch."""
    import math

    import torch
    n = X.shape[0]
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    X = f32(X)
    mu = f32(X.mean(0))
    isg = f32(1.0 / X.std(0, ddof=1))
    t = f32(target)
    ts = f32((t - t.mean()) / t.std(ddof=1))
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    spe = max(1, n // batch)
    total = epochs * spe
    th, m, v = f32(theta), np.zeros_like(theta), np.zeros_like(theta)
    hist, k = [], 0
    for _ in range(epochs):
        perm = torch.randperm(n, generator=gen).numpy()
        for s in range(spe):
            idx = perm[s * batch:(s + 1) * batch]
            k += 1
            cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * (k - 1) / max(total - 1, 1)))
            loss, g = mo.loss_and_grad(th, X[idx], ts[idx], mu, isg)
            th, m, v = mo.adam_step(th, m, v, g, k, cur)
        hist.append(loss)
    return hist


def test_mlp_training_reduces_loss():
    """A teacher network labels random inputs and a student is trained on
    them by the device kernels.  The expectation is the oracle's own
    training run on the same minibatches (it ends at ~0.11 of the untrained
    loss after 15 epochs on this problem): the device's loss must track it
    epoch by epoch, and the trained student must fit the teacher."""
    import torch
    n, n_in = 20000, 36
    teacher, X, mu, isg = rand_case(n, n_in, 11)
    y_t, _ = mo.input_gradient(teacher, X, mu, isg, bf16=False)
    m = handle("f32")
    net = surrogate.Network(n_in, seed=3)
    theta0 = net.theta.double().cpu().numpy()
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    tt = torch.tensor(y_t, dtype=torch.float32, device="cuda")
    # loss of the untrained network in the standardised units fit() uses
    net.set_standardisation(Xt)
    y0, _ = net.forward(m.h, Xt, grad=False)
    ts = (y_t - y_t.mean()) / y_t.std()
    loss0 = float(np.mean((y0.double().cpu().numpy() - ts) ** 2))
    hist = surrogate.fit(m.h, net, Xt, tt, epochs=15, batch=1024, lr=3e-3, seed=4)
    ref = _oracle_fit(theta0, X, y_t, epochs=15, batch=1024, lr=3e-3, seed=4)
    y, _ = net.forward(m.h, Xt)
    r = y.double().cpu().numpy() - y_t
    rmse = np.sqrt(np.mean(r ** 2))
    dev = max(abs(a - b) / b for a, b in zip(hist, ref))
    say(f"[gpu] training loss: untrained {loss0:.3e}; device {hist[0]:.4e} ... {hist[-1]:.4e}; "
        f"oracle {ref[0]:.4e} ... {ref[-1]:.4e}; worst epoch deviation {dev:.2e}; rmse/std {rmse / np.std(y_t):.3f}")
    assert ref[-1] < 0.15 * loss0          # what 15 epochs reach on this problem
    assert dev < 0.05                       # the device follows the oracle's trajectory
    assert rmse < 0.5 * np.std(y_t)


def test_mlp_argument_errors():
    import torch
    m = handle("f32")
    z = torch.zeros(8, device="cuda")
    for n_in in (0, 65):
        with pytest.raises(pod.PodError):
            pod.pod_mlp_num_params(n_in)
        with pytest.raises(pod.PodError):
            pod.pod_mlp_forward(m.h, 4, n_in, z, max(n_in, 1), z, z, z, z, None)
    with pytest.raises(pod.PodError):                     # ldx < n_in
        pod.pod_mlp_forward(m.h, 1, 4, z, 3, z, z, z, z, None)
    with pytest.raises(pod.PodError):                     # step counts from 1
        pod.pod_mlp_train_step(m.h, 1, 4, z, 4, z, z, z, z, z, z, 0, 1e-3)


# --------------------------------------------------------------------------
# surrogate energy / forces
# --------------------------------------------------------------------------
SETUP23 = wl.PodSetup(rin=0.5, rcut=5.0, L=8, K2=6, K3=6, K4=0, P3=4, P4=0)


@pytest.fixture(scope="module")
def sur_case():
    w = wl.small_bcc(3, sigma=0.15, seed=21, setup=SETUP23)
    op = oracle_params(SETUP23)
    Q, _ = po.pod_basis(op)
    args = (w.pos, w.cell, w.nl.offsets.astype(np.int64), w.nl.nbr_j, w.nl.shift3, op, Q)
    D = po.descriptors_fast(*args)
    rng = np.random.default_rng(22)
    c23 = rng.normal(size=D.shape[1]) / (D.std(0) + 1e-3) * 0.1
    n_in = D.shape[1] - 1
    theta, _, _, _ = rand_case(1, n_in, 23)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    mu = f32(D[:, 1:].mean(0))
    isg = f32(1.0 / (D[:, 1:].std(0) + 1e-6))
    return w, op, Q, args, c23, theta, mu, isg


def run_surrogate(w, Q, c, theta, mu, isg, dtype, gather=False):
    import torch
    m = pod.PodModel(pod.setup_from_workload(SETUP23), dtype, Q=Q[:, :6])
    net = surrogate.Network(len(mu), seed=0)
    f = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    net.theta, net.mu, net.inv_sigma = f(theta), f(mu), f(isg)
    nb = pod.DeviceNeighbors.from_list(w.nl)
    if gather:
        nb.build_reverse(m)
    pos = w.pos if dtype == "f64" else w.pos.astype(np.float32).astype(np.float64)
    o = m.energy_forces_surrogate(pos, w.cell, nb, c, net)
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in o.items()}, m, nb


@pytest.mark.parametrize("dtype,gather", [("f64", False), ("f64", True), ("f32", False)])
def test_surrogate_energy_forces_vs_oracle(sur_case, dtype, gather):
    """Stage by stage.  (1) The network on the device's own descriptors
    against the oracle network: the bfloat16 flip bound of this module.
    (2) The POD adjoint with the device's own per-atom weights c + dy/dX
    against the oracle's forces for those weights: FP64 rounding on the FP64
    path, the FP32 force tolerance (1e-4) on the FP32 path.  (3) End to end:
    a flip in one atom's network moves the forces of all its neighbours, so
    only the worst-case bound applies to the forces (in a 54-atom periodic
    cell every atom neighbours every other)."""
    import torch
    w, op, Q, args, c23, theta, mu, isg = sur_case
    c = c23 if dtype == "f64" else c23.astype(np.float32).astype(np.float64)
    pos = w.pos if dtype == "f64" else w.pos.astype(np.float32).astype(np.float64)
    say(f"[gpu] surrogate {dtype} gather={gather} N={w.N}")
    got, m, nb = run_surrogate(w, Q, c, theta, mu, isg, dtype, gather)
    # (1) network stage, recomputed with the same kernels on the same inputs
    net = surrogate.Network(len(mu), seed=0)
    f = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    net.theta, net.mu, net.inv_sigma = f(theta), f(mu), f(isg)
    Dd = m.descriptors(pos, w.cell, nb)
    y_dev, g_dev = net.forward(m.h, Dd, x_col=1, ldx=m.M)
    torch.cuda.synchronize()
    Dd = Dd.double().cpu().numpy()
    y_dev, g_dev = y_dev.double().cpu().numpy(), g_dev.double().cpu().numpy()
    y_ref, g_ref = mo.input_gradient(theta, Dd[:, 1:], mu, isg, bf16=True)
    check(y_dev, y_ref, "network y")
    check(g_dev, g_ref, "network dy/dX")
    # (2) POD adjoint stage with the device's weights
    C = c[None, :] + np.concatenate([np.zeros((w.N, 1)), g_dev], axis=1)
    F_C, W_C = mo.forces_from_atom_weights(pos, *args[1:], C)
    tol2 = 1e-10 if dtype == "f64" else 1e-4
    e2 = relerr(got["F"], F_C)
    say(f"[gpu]   adjoint with device weights: F rel {e2:.2e}, W rel {relerr(got['W'], W_C):.2e}")
    assert e2 < tol2 and relerr(got["W"], W_C) < tol2
    assert relerr(got["E_atom"], Dd @ c + y_dev) < (1e-12 if dtype == "f64" else 1e-5)
    # (3) end to end against the oracle surrogate
    ref = mo.surrogate_energy_forces(pos, *args[1:], c, theta, mu, isg, bf16=True)
    for k in ("E_atom", "F"):
        r = per_row_rel(got[k], ref[k])
        say(f"[gpu]   end to end {k}: worst {r.max():.2e}, 99th pct {np.quantile(r, 0.99):.2e}")
        assert r.max() < WORST, k
    assert relerr(got["W"], ref["W"]) < WORST
    assert abs(got["E"][0] - ref["E"]) < WORST * np.abs(ref["E_atom"]).max()


@pytest.mark.parametrize("K,P3", [(3, 4), (1, 4), (8, 6)])
def test_surrogate_several_network_tiles_per_wave(K, P3):
    """With K = 3 (21 atoms per wavefront, two wavefronts per workgroup in
    FP64: 42 atoms in three tiles of 16, the first wavefront taking two in
    turn, and the last workgroup holding a group past the end of the list)
    and K = 1 (64 atoms, four tiles in turn) the per-atom kernel runs the
    network on several tiles per wavefront; K = 8 at P3 = 6 gives the
    largest input, 64 descriptors (all four input groups filled).  The
    network's outputs must equal those of the network kernel on the
    device's own descriptors (same products, same rounding: the energies to
    FP64 rounding of the linear part), and the forces those of the oracle's
    adjoint with these per-atom weights to 1e-10."""
    import torch
    S = wl.PodSetup(rin=0.5, rcut=5.0, L=8, K2=K, K3=K, K4=0, P3=P3, P4=0)
    w = wl.small_bcc(3, sigma=0.15, seed=31 + K, setup=S)
    op = oracle_params(S)
    Q, _ = po.pod_basis(op)
    args = (w.pos, w.cell, w.nl.offsets.astype(np.int64), w.nl.nbr_j, w.nl.shift3, op, Q)
    D = po.descriptors_fast(*args)
    rng = np.random.default_rng(32 + K)
    c = rng.normal(size=D.shape[1]) / (D.std(0) + 1e-3) * 0.1
    n_in = D.shape[1] - 1
    theta, _, _, _ = rand_case(1, n_in, 33 + K)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    mu = f32(D[:, 1:].mean(0))
    isg = f32(1.0 / (D[:, 1:].std(0) + 1e-6))
    m = pod.PodModel(pod.setup_from_workload(S), "f64", Q=Q[:, :K])
    net = surrogate.Network(n_in, seed=0)
    f = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    net.theta, net.mu, net.inv_sigma = f(theta), f(mu), f(isg)
    nb = pod.DeviceNeighbors.from_list(w.nl)
    nb.build_reverse(m)
    say(f"[gpu] surrogate K={K}: {64 // K} atoms per wavefront, N={w.N}, n_in={n_in}")
    o = m.energy_forces_surrogate(w.pos, w.cell, nb, c, net)
    Dd = m.descriptors(w.pos, w.cell, nb)
    y_dev, g_dev = net.forward(m.h, Dd, x_col=1, ldx=m.M)
    torch.cuda.synchronize()
    got = {k: v.double().cpu().numpy() for k, v in o.items()}
    Dd = Dd.double().cpu().numpy()
    y_dev, g_dev = y_dev.double().cpu().numpy(), g_dev.double().cpu().numpy()
    assert relerr(got["E_atom"], Dd @ c + y_dev) < 1e-12
    C = c[None, :] + np.concatenate([np.zeros((w.N, 1)), g_dev], axis=1)
    F_C, W_C = mo.forces_from_atom_weights(w.pos, *args[1:], C)
    assert relerr(got["F"], F_C) < 1e-10 and relerr(got["W"], W_C) < 1e-10
    # energy only (no adjoint rows, no pair kernel): the same energies
    e = m.energy_forces_surrogate(w.pos, w.cell, nb, c, net, forces=False, virial=False)
    torch.cuda.synchronize()
    assert np.array_equal(e["E_atom"].cpu().numpy(), got["E_atom"]) and e["E"].item() == got["E"][0]


@pytest.mark.parametrize("K,P3,cells", [(6, 4, 4), (8, 6, 3)])
def test_surrogate_f32_workgroup_of_several_wavefronts(K, P3, cells):
    """FP32, where the per-atom kernel's workgroup is several wavefronts that
    share the network tiles: K = 6 on 128 atoms (three wavefronts of 10
    atoms, 13 atom groups: the last workgroup holds two groups past the end
    of the list) and K = 8 at P3 = 6 on 54 atoms (two wavefronts of 8 atoms,
    7 groups, one past the end).  Energies against the linear part on the
    device's own descriptors plus the network kernel's outputs (FP32
    rounding of the linear part: 1e-5), forces and virial against the
    oracle's adjoint with the device's per-atom weights (the FP32 force
    tolerance, 1e-4), and the energy-only launch bit for bit."""
    import torch
    S = wl.PodSetup(rin=0.5, rcut=5.0, L=8, K2=K, K3=K, K4=0, P3=P3, P4=0)
    w = wl.small_bcc(cells, sigma=0.15, seed=41 + K, setup=S)
    pos = w.pos.astype(np.float32).astype(np.float64)
    nl = wl.neighbor_list(pos, w.cell, S.rcut)   # listed on the rounded positions
    op = oracle_params(S)
    Q, _ = po.pod_basis(op)
    args = (pos, w.cell, nl.offsets.astype(np.int64), nl.nbr_j, nl.shift3, op, Q)
    D = po.descriptors_fast(*args)
    rng = np.random.default_rng(42 + K)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    c = f32(rng.normal(size=D.shape[1]) / (D.std(0) + 1e-3) * 0.1)
    n_in = D.shape[1] - 1
    theta, _, _, _ = rand_case(1, n_in, 43 + K)
    mu = f32(D[:, 1:].mean(0))
    isg = f32(1.0 / (D[:, 1:].std(0) + 1e-6))
    m = pod.PodModel(pod.setup_from_workload(S), "f32", Q=Q[:, :K])
    net = surrogate.Network(n_in, seed=0)
    f = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    net.theta, net.mu, net.inv_sigma = f(theta), f(mu), f(isg)
    nb = pod.DeviceNeighbors.from_list(nl)
    nb.build_reverse(m)
    say(f"[gpu] surrogate f32 K={K}: N={len(pos)}, {-(-len(pos) // (64 // K))} atom groups, n_in={n_in}")
    o = m.energy_forces_surrogate(pos, w.cell, nb, c, net)
    Dd = m.descriptors(pos, w.cell, nb)
    y_dev, g_dev = net.forward(m.h, Dd, x_col=1, ldx=m.M)
    torch.cuda.synchronize()
    got = {k: v.double().cpu().numpy() for k, v in o.items()}
    Dd = Dd.double().cpu().numpy()
    y_dev, g_dev = y_dev.double().cpu().numpy(), g_dev.double().cpu().numpy()
    e1 = relerr(got["E_atom"], Dd @ c + y_dev)
    C = c[None, :] + np.concatenate([np.zeros((len(pos), 1)), g_dev], axis=1)
    F_C, W_C = mo.forces_from_atom_weights(pos, *args[1:], C)
    e2, e3 = relerr(got["F"], F_C), relerr(got["W"], W_C)
    say(f"[gpu]   E_atom rel {e1:.2e}, F rel {e2:.2e}, W rel {e3:.2e}")
    assert e1 < 1e-5 and e2 < 1e-4 and e3 < 1e-4
    e = m.energy_forces_surrogate(pos, w.cell, nb, c, net, forces=False, virial=False)
    torch.cuda.synchronize()
    assert np.array_equal(e["E_atom"].double().cpu().numpy(), got["E_atom"]) and e["E"].item() == got["E"][0]


def test_surrogate_largest_box_f32():
    """The surrogate benchmark's box, 1,024,000 atoms (FP32 POD, the 2/3-body
    model with the network inside the per-atom kernel: 102,400 atom groups in
    workgroups of three wavefronts, the last holding two groups past the end
    of the list).  Every atom's energy against the descriptor kernel's linear
    part plus the network kernel's output on the same descriptors: within the
    FP32 rounding of the linear part (1e-5), where one bfloat16 rounding flip
    between the two paths would show as ~1e-3; the energy-only launch bit for
    bit; the total force of the periodic box zero to FP32 rounding."""
    import torch
    w = wl.config5_infer()
    S = wl.SETUP_CFG5_23
    pos = w.pos.astype(np.float32).astype(np.float64)
    nl = wl.neighbor_list(pos, w.cell, S.rcut)
    m = pod.PodModel(pod.setup_from_workload(S), "f32")
    nb = pod.DeviceNeighbors.from_list(nl)
    nb.build_reverse(m)
    say(f"[gpu] surrogate f32 largest box: N={len(pos)} P={nl.n_pairs}")
    Dd = m.descriptors(pos, w.cell, nb)
    D = Dd.double().cpu().numpy()
    n_in = S.M - 1
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    rng = np.random.default_rng(52)
    c = f32(rng.normal(size=S.M) / (D.std(0) + 1e-3) * 0.1)
    theta, _, _, _ = rand_case(1, n_in, 53)
    mu = f32(D[:, 1:].mean(0))
    isg = f32(1.0 / (D[:, 1:].std(0) + 1e-6))
    net = surrogate.Network(n_in, seed=0)
    f = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    net.theta, net.mu, net.inv_sigma = f(theta), f(mu), f(isg)
    o = m.energy_forces_surrogate(pos, w.cell, nb, c, net)
    y_dev, _ = net.forward(m.h, Dd, x_col=1, ldx=m.M)
    e = m.energy_forces_surrogate(pos, w.cell, nb, c, net, forces=False, virial=False)
    torch.cuda.synchronize()
    E_atom = o["E_atom"].double().cpu().numpy()
    F = o["F"].double().cpu().numpy()
    e1 = relerr(E_atom, D @ c + y_dev.double().cpu().numpy())
    say(f"[gpu]   E_atom rel {e1:.2e} against descriptors + network kernel (every atom)")
    assert e1 < 1e-5
    assert np.array_equal(e["E_atom"].double().cpu().numpy(), E_atom)
    assert np.isfinite(F).all() and np.abs(F.sum(0)).max() <= 1e-4 * np.abs(F).max() * np.sqrt(len(pos))


def test_surrogate_silent_network_equals_linear_path(sur_case):
    """w3 = 0, b3 = 0: the surrogate path must reproduce pod_energy_forces
    with the 2/3-body coefficients to FP64 rounding (the network adds exact
    zeros)."""
    w, op, Q, args, c23, theta, mu, isg = sur_case
    t0 = theta.copy()
    t0[-65:] = 0.0
    got, m, nb = run_surrogate(w, Q, c23, t0, mu, isg, "f64")
    lin = m.energy_forces(w.pos, w.cell, nb, c23)
    for k in ("E_atom", "F", "W"):
        assert relerr(got[k], lin[k].cpu().numpy()) < 1e-12, k


def test_surrogate_rejects_four_body_handle(sur_case):
    import torch
    w, op, Q, args, c23, theta, mu, isg = sur_case
    m = pod.PodModel(pod.setup_from_workload(wl.SETUP_CFG2), "f64")
    net = surrogate.Network(36, seed=0)
    nb = pod.DeviceNeighbors.from_list(w.nl)
    with pytest.raises(pod.PodError) as e:
        m.energy_forces_surrogate(w.pos, w.cell, nb, np.zeros(m.M), net)
    assert e.value.code == -1
    torch.cuda.synchronize()


def test_surrogate_learns_four_body_forces():
    """Trained on the exact 4-body energies of six displaced BCC boxes, the
    surrogate's forces on a seventh box are much closer to the exact 2/3/4-body
    forces than the 2/3-body model without it."""
    import torch
    S, S23 = wl.SETUP_CFG5, wl.SETUP_CFG5_23
    m64 = pod.PodModel(pod.setup_from_workload(S), "f64")
    boxes = []
    for k, sig in enumerate((0.08, 0.15, 0.25, 0.12, 0.2, 0.28, 0.17)):
        pos, cell = wl.bcc(10)
        pos = wl.displace(pos, sig, 300 + k)
        boxes.append((pos, cell, wl.neighbor_list(pos, cell, S.rcut)))
    nb0 = pod.DeviceNeighbors.from_list(boxes[0][2])
    c = wl.standardised_coefficients(m64.descriptors(boxes[0][0], boxes[0][1], nb0).cpu().numpy(), S, seed=31)
    X, T = surrogate.four_body_dataset(m64, boxes[:-1], c, 36)
    m23 = pod.PodModel(pod.setup_from_workload(S23), "f64")
    net = surrogate.Network(36, seed=5)
    surrogate.fit(m23.h, net, X, T, epochs=60, batch=512, lr=3e-3, seed=6)
    pos, cell, nl = boxes[-1]
    nb = pod.DeviceNeighbors.from_list(nl)
    ex = m64.energy_forces(pos, cell, nb, c)["F"]
    su = m23.energy_forces_surrogate(pos, cell, nb, c[:37], net)["F"]
    n4 = m23.energy_forces(pos, cell, nb, c[:37])["F"]
    rm = lambda a, b: float(torch.sqrt(((a - b) ** 2).mean()))
    say(f"[gpu] learned surrogate: force rmse {rm(su, ex):.4f} eV/A, without 4-body {rm(n4, ex):.4f} eV/A")
    assert rm(su, ex) < 0.3 * rm(n4, ex)
