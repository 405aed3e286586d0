"""Pins of the FP64 network oracle (Sec. IV.D, eqs. (671a)-(673a); loss of
Sec. IV.C, eq. (63b); Adam): bfloat16 rounding against torch's own
conversion and hand-worked ties, SiLU closed forms, every gradient against
central differences, Adam's first-step and convergence properties, and the
surrogate's forces and virial against finite differences of its energy."""
import numpy as np
import pytest

from oracle import mlp_oracle as mo
from oracle import pod_oracle as po
from paper_2212_14446_amd import workloads as wl

N_IN = 7


def rand_net(seed, n_in=N_IN, scale=0.4):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, scale, size=mo.n_params(n_in))
    mu = rng.normal(size=n_in)
    inv_sigma = rng.uniform(0.5, 2.0, size=n_in)
    return theta, mu, inv_sigma, rng


def test_param_count_and_layout():
    assert mo.n_params(36) == 6593          # 36 -> 64 -> 64 -> 1
    theta = np.arange(mo.n_params(3), dtype=float)
    W1, b1, W2, b2, w3, b3 = mo.unpack(theta, 3)
    assert W1.shape == (64, 3) and W1[0, 1] == 1.0 and b1[0] == 192.0
    assert W2.shape == (64, 64) and W2[0, 0] == 256.0
    assert b3 == theta[-1]
    assert np.array_equal(mo.pack(W1, b1, W2, b2, w3, b3), theta)


def test_bf16_round_hand_values():
    one = 1.0
    ulp = 2.0 ** -7                          # spacing of bfloat16 in [1, 2)
    cases = {one: one, one + ulp: one + ulp,
             one + ulp / 2: one,                       # tie, even neighbour is 1
             one + 3 * ulp / 2: one + 2 * ulp,         # tie, even neighbour is 1 + 2 ulp
             one + ulp / 2 + 2.0 ** -20: one + ulp,    # just above the tie
             -(one + ulp / 2): -one, 0.0: 0.0, 3.0: 3.0}
    for x, want in cases.items():
        assert mo.bf16_round(np.array([x]))[0] == want, x


def test_bf16_round_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=20000).astype(np.float32),
                        (rng.normal(size=2000) * 1e-30).astype(np.float32),
                        (rng.normal(size=2000) * 1e30).astype(np.float32)])
    # exact ties: 1 + k * 2^-8 with k odd
    x = np.concatenate([x, (1.0 + (2 * np.arange(100) + 1) * 2.0 ** -8).astype(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(mo.bf16_round(x), ref)


def test_silu_closed_forms():
    assert mo.silu(0.0) == 0.0
    assert mo.silu_prime(0.0) == 0.5
    assert mo.silu(40.0) == pytest.approx(40.0, rel=1e-15)
    assert abs(mo.silu(-40.0)) < 1e-15
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (mo.silu(z + h) - mo.silu(z - h)) / (2 * h)
    assert np.allclose(mo.silu_prime(z), fd, rtol=1e-8, atol=1e-10)


def test_input_gradient_fd():
    theta, mu, inv_sigma, rng = rand_net(5)
    X = rng.normal(size=(6, N_IN))
    y, g = mo.input_gradient(theta, X, mu, inv_sigma, bf16=False)
    h = 1e-6
    for k in range(N_IN):
        Xp, Xm = X.copy(), X.copy()
        Xp[:, k] += h
        Xm[:, k] -= h
        fd = (mo.forward(theta, Xp, mu, inv_sigma, False)["y"] - mo.forward(theta, Xm, mu, inv_sigma, False)["y"]) / (2 * h)
        assert np.allclose(g[:, k], fd, rtol=1e-7, atol=1e-9)


def test_parameter_gradient_fd():
    theta, mu, inv_sigma, rng = rand_net(6)
    X = rng.normal(size=(9, N_IN))
    t = rng.normal(size=9)
    loss, grad = mo.loss_and_grad(theta, X, t, mu, inv_sigma, bf16=False)
    H = mo.N_HIDDEN
    # entries from every block: W1, b1, W2, b2, w3, b3
    starts = [0, H * N_IN, H * N_IN + H, H * N_IN + H + H * H, H * N_IN + 2 * H + H * H, mo.n_params(N_IN) - 1]
    idx = sorted(set([s for s in starts] + [s + 5 for s in starts[:-1]] + list(rng.integers(0, theta.size, 20))))
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mo.loss_and_grad(tp, X, t, mu, inv_sigma, False)[0] - mo.loss_and_grad(tm, X, t, mu, inv_sigma, False)[0]) / (2 * h)
        assert grad[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i
    assert loss == pytest.approx(np.mean((mo.forward(theta, X, mu, inv_sigma, False)["y"] - t) ** 2))


def test_degenerate_networks():
    theta, mu, inv_sigma, rng = rand_net(7)
    W1, b1, W2, b2, w3, b3 = mo.unpack(theta, N_IN)
    X = rng.normal(size=(5, N_IN))
    # zero second layer: h2 = SiLU(0) = 0, so y = b3 and dy/dX = 0
    t0 = mo.pack(W1, b1, 0 * W2, 0 * b2, w3, b3)
    for bf in (False, True):
        y, g = mo.input_gradient(t0, X, mu, inv_sigma, bf)
        assert np.all(y == b3) and np.all(g == 0.0)
    # identical hidden units: the network is a function of W1[0] . x only
    W1s = np.repeat(W1[:1], 64, axis=0)
    t1 = mo.pack(W1s, np.full(64, b1[0]), W2, b2, w3, b3)
    y, g = mo.input_gradient(t1, X, mu, inv_sigma, False)
    dirn = W1s[0] * inv_sigma
    ratio = g / dirn[None, :]
    assert np.allclose(ratio, ratio[:, :1], rtol=1e-10)


def test_adam_first_step_and_convergence():
    rng = np.random.default_rng(8)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    g[3] = 0.0
    lr = 1e-3
    t1, m, v = mo.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, lr, eps=0.0 + 1e-12)
    step = theta - t1
    nz = g != 0
    # with bias correction, the first step is lr * sign(g)
    assert np.allclose(step[nz], lr * np.sign(g[nz]), rtol=1e-8)
    assert step[3] == 0.0
    # convergence on a quadratic 0.5 |theta - a|^2
    a = rng.normal(size=50)
    th, m, v = np.zeros(50), np.zeros(50), np.zeros(50)
    for s in range(1, 3001):
        th, m, v = mo.adam_step(th, m, v, th - a, s, 0.05)
    assert np.max(np.abs(th - a)) < 1e-3


@pytest.fixture(scope="module")
def sur_system():
    p = po.make_params(0.5, 5.0, 8, 4, 4, 0, 3, 0)          # 2/3-body only
    Q, _ = po.pod_basis(p)
    pos, cell = wl.bcc(2)
    pos = wl.displace(pos, 0.15, 51)
    off, nj, sh = po.neighbors_bruteforce(pos, cell, p.rcut)
    M, _ = po.num_descriptors(p)
    rng = np.random.default_rng(52)
    c23 = rng.normal(size=M)
    D = po.descriptors_fast(pos, cell, off, nj, sh, p, Q)
    mu = D[:, 1:].mean(0)
    inv_sigma = 1.0 / (D[:, 1:].std(0) + 1e-3)
    theta = rng.normal(0.0, 0.3, size=mo.n_params(M - 1))
    return p, Q, pos, cell, off, nj, sh, c23, theta, mu, inv_sigma


def _sur_energy(pos, s):
    p, Q, _, cell, off, nj, sh, c23, theta, mu, inv_sigma = s
    D = po.descriptors_fast(pos, cell, off, nj, sh, p, Q)
    return float((D @ c23).sum() + mo.forward(theta, D[:, 1:], mu, inv_sigma, False)["y"].sum())


def test_surrogate_forces_fd(sur_system):
    p, Q, pos, cell, off, nj, sh, c23, theta, mu, inv_sigma = sur_system
    out = mo.surrogate_energy_forces(pos, cell, off, nj, sh, p, Q, c23, theta, mu, inv_sigma, bf16=False)
    assert out["E"] == pytest.approx(_sur_energy(pos, sur_system), rel=1e-13)
    h = 1e-5
    scale = np.abs(out["F"]).max()
    for a in (0, 5, 13):
        for d in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[a, d] += h
            pm[a, d] -= h
            fd = -(_sur_energy(pp, sur_system) - _sur_energy(pm, sur_system)) / (2 * h)
            assert abs(out["F"][a, d] - fd) < 1e-7 * scale
    assert np.max(np.abs(out["F"].sum(0))) < 1e-11 * scale


def test_surrogate_virial_strain_fd(sur_system):
    p, Q, pos, cell, off, nj, sh, c23, theta, mu, inv_sigma = sur_system
    out = mo.surrogate_energy_forces(pos, cell, off, nj, sh, p, Q, c23, theta, mu, inv_sigma, bf16=False)
    h = 1e-6
    W = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            Ep = _sur_energy(pos @ (np.eye(3) + e).T, (p, Q, None, cell @ (np.eye(3) + e).T, off, nj, sh, c23,
                                                         theta, mu, inv_sigma))
            Em = _sur_energy(pos @ (np.eye(3) - e).T, (p, Q, None, cell @ (np.eye(3) - e).T, off, nj, sh, c23,
                                                         theta, mu, inv_sigma))
            W[a, b] = -(Ep - Em) / (2 * h)
    assert np.allclose(out["W"], W, rtol=1e-6, atol=1e-6 * np.abs(W).max())


def test_surrogate_with_silent_network_is_the_linear_model(sur_system):
    """w3 = 0, b3 = 0: the surrogate reduces to the linear POD model, whose
    forces the POD oracle computes by its own adjoint route."""
    p, Q, pos, cell, off, nj, sh, c23, theta, mu, inv_sigma = sur_system
    W1, b1, W2, b2, w3, b3 = mo.unpack(theta, len(mu))
    t0 = mo.pack(W1, b1, W2, b2, 0 * w3, 0.0)
    out = mo.surrogate_energy_forces(pos, cell, off, nj, sh, p, Q, c23, t0, mu, inv_sigma, bf16=True)
    lin = po.energy_forces(pos, cell, off, nj, sh, p, Q, c23)
    assert np.allclose(out["E_atom"], lin["E_atom"], rtol=1e-12, atol=1e-12)
    assert np.allclose(out["F"], lin["F"], rtol=1e-10, atol=1e-10 * np.abs(lin["F"]).max())
    assert np.allclose(out["W"], lin["W"], rtol=1e-10, atol=1e-10 * np.abs(lin["W"]).max())
