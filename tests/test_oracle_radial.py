"""Oracle radial functions (Sec. II.B): closed-form limits, zeros, derivative
checks by finite differences and the POD basis against an SVD."""
import numpy as np
import pytest

from oracle import pod_oracle as po

P6 = po.make_params(0.5, 5.0, 6, 4, 4, 0, 3, 0)
P8 = po.make_params(0.5, 5.0, 8, 6, 6, 6, 4, 4)


def test_scaled_distance_endpoints_and_small_beta():
    rin, rc = 0.5, 5.0
    x, _ = po.scaled_distance(np.array([rin, rc]), rin, rc, 3.0)
    assert abs(x[0]) < 1e-15 and abs(x[1] - 1.0) < 1e-14
    r = np.linspace(rin, rc, 101)
    x3, _ = po.scaled_distance(r, rin, rc, 3.0)
    assert np.all(np.diff(x3) > 0)
    # beta -> 0: x -> t = (r - rin)/(rc - rin), first correction O(beta)
    xs, _ = po.scaled_distance(r, rin, rc, 1e-8)
    t = (r - rin) / (rc - rin)
    assert np.max(np.abs(xs - t)) < 1e-8
    # x > t for beta > 0 (exp(-beta t) is convex)
    assert np.all(x3[1:-1] > t[1:-1])


def test_bessel_snapshot_limit_at_rin():
    # sin(alpha pi x)/(r - rin) -> alpha pi dx/dr(rin) = alpha pi beta / ((rc-rin)(1-e^-beta))
    rin, rc, beta = 0.5, 5.0, 3.0
    p = po.PodParams(rin, rc, np.array([2.0]), np.array([beta]), np.array([0.0]),
                     np.array([1.0]), 1, 0, 0, 0, 0)
    r = rin + 1e-7
    Phi, _ = po.snapshots(np.array([r]), p)
    fc, _ = po.cutoff(np.array([r]), rin, rc)
    want = 2.0 * np.pi * beta / ((rc - rin) * (1 - np.exp(-beta)))
    assert Phi[0, 0] / fc[0] == pytest.approx(want, rel=1e-5)


@pytest.mark.parametrize("alpha", [1, 2, 3, 4])
def test_bessel_snapshot_zeros(alpha):
    # sin(alpha pi x) vanishes where x(r) = k/alpha; invert x to find those r
    rin, rc, beta = 0.5, 5.0, 3.0
    p = po.PodParams(rin, rc, np.array([float(alpha)]), np.array([beta]), np.array([0.0]),
                     np.array([1.0]), 1, 0, 0, 0, 0)
    for k in range(1, alpha):
        xk = k / alpha
        t = -np.log1p(xk * np.expm1(-beta)) / beta
        r = rin + t * (rc - rin)
        Phi, _ = po.snapshots(np.array([r]), p)
        assert abs(Phi[0, 0]) < 1e-12


def test_inverse_power_snapshot():
    rin, rc = 0.5, 5.0
    p = po.PodParams(rin, rc, np.zeros(2), np.zeros(2), np.array([1.0, 2.0]),
                     np.zeros(2), 1, 0, 0, 0, 0)
    r = np.linspace(0.6, 4.9, 17)
    Phi, _ = po.snapshots(r, p)
    fc, _ = po.cutoff(r, rin, rc)
    assert np.allclose(Phi[:, 0] * r / fc, 1.0, rtol=1e-14)
    assert np.allclose(Phi[:, 1] * r * r / fc, 1.0, rtol=1e-14)


def test_cutoff_endpoints_and_shape():
    rin, rc = 0.5, 5.0
    fc, dfc = po.cutoff(np.array([rin, rc]), rin, rc)
    # at rin: exp(1 - (1 + eps)^(-1/2)) = 1 + eps/2 + O(eps^2)
    assert fc[0] - 1.0 == pytest.approx(po.EPS_FC / 2, rel=1e-5)
    assert dfc[0] == 0.0
    # at rc: exp(1 - eps^(-1/2)) = exp(-999) underflows; slope vanishes too
    assert fc[1] == 0.0 and dfc[1] == 0.0
    r = np.linspace(rin, rc, 401)
    f, _ = po.cutoff(r, rin, rc)
    assert np.all(np.diff(f) <= 0)
    assert np.all((f >= 0) & (f <= 1.0 + 1e-6))


def test_cutoff_interior_values():
    """Eq. (8) at interior points, values worked out by hand in 40-digit
    decimal arithmetic (rin = 0.5, rc = 5, eps = 1e-6, t = (r - rin)/(rc - rin)):
    * t^3 = 1/2: y = 1 - t^3 = 1/2, s = y^2 + eps = 0.250001,
      f_c = exp(1 - s^(-1/2)) = exp(-0.999996000012) = 0.36788091268773549;
      df/dr = -3 f_c y t^2 s^(-3/2) / (rc - rin) = -0.61799749967771510;
    * t = 1/2: y = 7/8, s = 0.765626, f_c = 0.86687854674903807;
    * r = rc - 0.01: t = 4.49/4.5, y = 1 - t^3 = 6.6519e-3,
      f_c = 7.4241044166644240e-65 (a cubic written as a square would give
      1e-95 there and 0.182 at t^3 = 1/2)."""
    rin, rc = 0.5, 5.0
    h = rc - rin
    r = np.array([rin + h * 0.5 ** (1.0 / 3.0), rin + 0.5 * h, rc - 0.01])
    fc, dfc = po.cutoff(r, rin, rc)
    assert fc[0] == pytest.approx(0.36788091268773549, rel=1e-14)
    assert dfc[0] == pytest.approx(-0.61799749967771510, rel=1e-13)
    assert fc[1] == pytest.approx(0.86687854674903807, rel=1e-14)
    assert fc[2] == pytest.approx(7.4241044166644240e-65, rel=1e-9)


@pytest.mark.parametrize("p", [P6, P8])
def test_snapshot_derivative_fd(p):
    r = np.linspace(0.7, 4.8, 23)
    _, dPhi = po.snapshots(r, p)
    h = 1e-6
    Pp, _ = po.snapshots(r + h, p)
    Pm, _ = po.snapshots(r - h, p)
    fd = (Pp - Pm) / (2 * h)
    scale = np.max(np.abs(dPhi), axis=0)
    assert np.max(np.abs(fd - dPhi) / scale) < 1e-7


def test_domain_errors():
    with pytest.raises(ValueError):
        po.snapshots(np.array([0.5]), P6)
    with pytest.raises(ValueError):
        po.snapshots(np.array([5.0]), P6)
    with pytest.raises(ValueError):
        po.snapshots(np.array([np.nan]), P6)


@pytest.mark.parametrize("p", [P6, P8])
def test_pod_basis_against_svd(p):
    # method of snapshots: the eigenpairs of Phi^T Phi / n are the squared
    # singular values and right singular vectors of Phi / sqrt(n)
    Q, lam = po.pod_basis(p, n_quad=2000)
    rs = po.quadrature_nodes(p, 2000)
    Phi, _ = po.snapshots(rs, p)
    _, s, Vt = np.linalg.svd(Phi / np.sqrt(len(rs)), full_matrices=False)
    assert np.allclose(lam, s ** 2, rtol=1e-9, atol=1e-12 * lam[0])
    for k in range(p.K):
        v = Vt[k]
        assert min(np.max(np.abs(v - Q[:, k])), np.max(np.abs(v + Q[:, k]))) < 1e-8
        assert Q[np.argmax(np.abs(Q[:, k])), k] > 0
    assert np.all(np.diff(lam) <= 0)


@pytest.mark.parametrize("p", [P6, P8])
def test_radial_basis_orthogonal_on_grid(p):
    Q, lam = po.pod_basis(p, n_quad=2000)
    rs = po.quadrature_nodes(p, 2000)
    R, _ = po.radial_basis(rs, p, Q)
    Gm = R.T @ R / len(rs)
    assert np.allclose(Gm, np.diag(lam[: p.K]), atol=1e-12 * lam[0])
