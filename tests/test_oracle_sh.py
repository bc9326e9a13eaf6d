"""Pins of the oracle's view-dependent features (Eq. 2 inside Eq. 5): the real
SH basis against orthonormality on the sphere and its values on the axes, the
H = 1 render against the plain render, and a single voxel against the closed
form with a rotated canonical direction."""
import math

import numpy as np
import pytest

import oracle
from oracle import render_sh, sh_basis


def _sphere_quadrature(nt=24, nphi=48):
    """Gauss-Legendre in cos(theta) x uniform in phi: exact for the products of
    two harmonics of degree <= 2."""
    x, w = np.polynomial.legendre.leggauss(nt)
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    ct = np.repeat(x, nphi)
    st = np.sqrt(1 - ct ** 2)
    ph = np.tile(phi, nt)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    wts = np.repeat(w, nphi) * (2 * math.pi / nphi)
    return dirs, wts


@pytest.mark.parametrize("H", [1, 4, 9])
def test_sh_basis_is_orthonormal(H):
    dirs, wts = _sphere_quadrature()
    Y = sh_basis(H, dirs)
    G = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(H), atol=1e-12)


def test_sh_basis_on_the_axes():
    Y = sh_basis(9, np.eye(3))   # x, y, z axes
    c1 = math.sqrt(3 / (4 * math.pi))
    assert Y[0, 0] == pytest.approx(0.5 / math.sqrt(math.pi))
    np.testing.assert_allclose(Y[:, 1:4], [[0, 0, c1], [c1, 0, 0], [0, c1, 0]], atol=1e-15)
    # l = 2 on the axes: only the zonal (3z^2 - 1) and the x^2 - y^2 terms survive
    np.testing.assert_allclose(Y[:, [4, 5, 7]], 0.0, atol=1e-15)
    z = 0.25 * math.sqrt(5 / math.pi)
    np.testing.assert_allclose(Y[:, 6], [-z, -z, 2 * z], rtol=1e-15)
    q = 0.25 * math.sqrt(15 / math.pi)
    np.testing.assert_allclose(Y[:, 8], [q, -q, 0.0], atol=1e-15)


def test_render_sh_degree0_is_the_plain_render_scaled():
    rng = np.random.default_rng(21)
    depth = 2
    G = 1 << (depth + 1)
    cells = np.stack(np.nonzero(rng.random((G, G, G)) < 0.2), axis=1)[:, ::-1]   # (x, y, z)
    lin = (cells[:, 2] * G + cells[:, 1]) * G + cells[:, 0]
    order = np.argsort(lin)
    lin = lin[order]
    n = len(lin)
    sig = rng.uniform(0.5, 10.0, n)
    k0 = rng.normal(size=(n, 1, 3))
    o = rng.uniform(-2, 2, (200, 3))
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    B = np.zeros((2, 3, 4))
    B[:, :, :3] = np.eye(3)
    dom = rng.integers(0, 2, n).astype(np.int32)
    sh = render_sh(o, d, depth, lin, np.arange(n), sig, k0, 1, dom, B, 0.01)
    pl = oracle.render(o, d, depth, lin, np.arange(n), sig, k0[:, 0, :], 0.01)
    np.testing.assert_allclose(sh["F"], pl["F"] * 0.5 / math.sqrt(math.pi), rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(sh["A"], pl["A"])


def test_render_sh_single_voxel_closed_form():
    # one voxel [0, h)^3 of the posed lattice (depth 1: h = 1/2, cell (2, 2, 2)),
    # crossed by a ray along a unit direction u through its centre
    depth = 1
    G = 4
    h = 0.5
    key = np.array([(2 * G + 2) * G + 2])
    u = np.array([0.48, 0.6, 0.64])          # unit
    centre = np.full(3, 0.25)
    o = centre - 3.0 * u
    # chord through the cube [0, 0.5]^3 along u through its centre
    t_in = max((0.0 - o[a]) / u[a] for a in range(3))
    t_out = min((0.5 - o[a]) / u[a] for a in range(3))
    delta = t_out - t_in
    sigma = 3.0
    rng = np.random.default_rng(22)
    k = rng.normal(size=(1, 9, 2))
    # dominant bone: a rotation by 90 degrees about z (x -> y, y -> -x)
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    B = np.zeros((1, 3, 4))
    B[0, :, :3] = R
    out = render_sh(o[None], u[None], depth, key, np.array([0]), np.array([sigma]), k, 9,
                    np.array([0], dtype=np.int32), B, 0.0)
    x, y, z = R.T @ u                        # d^c = R^T d = (u_y, -u_x, u_z)
    pi = math.pi
    Y = np.array([0.5 / math.sqrt(pi),
                  math.sqrt(3 / (4 * pi)) * y, math.sqrt(3 / (4 * pi)) * z, math.sqrt(3 / (4 * pi)) * x,
                  0.5 * math.sqrt(15 / pi) * x * y, 0.5 * math.sqrt(15 / pi) * y * z,
                  0.25 * math.sqrt(5 / pi) * (3 * z * z - 1), 0.5 * math.sqrt(15 / pi) * x * z,
                  0.25 * math.sqrt(15 / pi) * (x * x - y * y)])
    alpha = 1 - math.exp(-sigma * delta)
    np.testing.assert_allclose(out["F"][0], alpha * (Y @ k[0]), rtol=1e-12)
    assert out["A"][0] == pytest.approx(alpha, rel=1e-14)
