"""Pins of the oracle's spherical-harmonic colour basis.

The paper uses SH for view-dependent colour with 4 bands (Sec. 3, Sec. 5, Sec. 7.1)
and fixes no basis. The oracle builds real SH from the general closed form of the
solid harmonics; these tests pin that construction to properties every real
orthonormal SH basis has: orthonormality on the sphere, harmonicity
(zero Laplacian of each homogeneous polynomial), the addition theorem, and the
closed-form degree-0 constant. The sign convention (no Condon-Shortley phase:
Y_1,-1 ~ +y, Y_1,0 ~ +z, Y_1,1 ~ +x) is a reading the paper does not pin.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

from oracle.gaussians import sh_basis, sh_basis_grad, sh_polynomials


def sphere_quadrature(n_theta=24, n_phi=48):
    x, w = leggauss(n_theta)           # cos(theta) nodes
    phi = np.arange(n_phi) * 2 * np.pi / n_phi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, :]).ravel()
    return dirs, wts


def test_orthonormal_on_sphere():
    dirs, w = sphere_quadrature()
    Y = sh_basis(3, dirs)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_polynomials_are_harmonic():
    for poly in sh_polynomials(3):
        lap = {}
        for (a, b, c), v in poly.items():
            for e, idx in ((a, 0), (b, 1), (c, 2)):
                if e >= 2:
                    key = [a, b, c]
                    key[idx] -= 2
                    lap[tuple(key)] = lap.get(tuple(key), 0.0) + v * e * (e - 1)
        assert all(abs(v) < 1e-12 for v in lap.values())


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_addition_theorem(l):
    rng = np.random.default_rng(l)
    a = rng.standard_normal((20, 3))
    b = rng.standard_normal((20, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    sl = slice(l * l, (l + 1) ** 2)
    lhs = (sh_basis(3, a)[:, sl] * sh_basis(3, b)[:, sl]).sum(1)
    x = (a * b).sum(1)
    Pl = np.polynomial.legendre.legval(x, [0] * l + [1])
    np.testing.assert_allclose(lhs, (2 * l + 1) / (4 * np.pi) * Pl, atol=1e-13)


def test_degree0_constant_and_band1_convention():
    d = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    Y = sh_basis(1, d)
    np.testing.assert_allclose(Y[:, 0], 1 / (2 * math.sqrt(math.pi)), rtol=1e-15)
    c1 = math.sqrt(3 / (4 * math.pi))
    # k = 1, 2, 3 are m = -1, 0, 1  ->  y, z, x
    np.testing.assert_allclose(Y[:, 1:], np.array([[0, 0, c1], [c1, 0, 0], [0, c1, 0]]),
                               atol=1e-15)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    d = rng.standard_normal((30, 3))
    g = sh_basis_grad(3, d)
    h = 1e-6
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        num = (sh_basis(3, d + e) - sh_basis(3, d - e)) / (2 * h)
        np.testing.assert_allclose(g[:, :, ax], num, atol=1e-8)
