"""Pins of the oracle's reconstruction (WENO-JS, linear stencils) against quadrature, textbook
formulas and polynomial exactness. Section 2 (fifth-order WENO, dimension-by-dimension reconstruction
to the Gauss points)."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import (GAUSS_XI, linear_point, poly_weights, smoothness_rules, weno_linear_weights,
                    weno_point)

HERE = os.path.dirname(__file__)
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))


def cell_average_by_quadrature(coeffs, o):
    """Average of sum_p coeffs[p] xi^p over [o-1/2, o+1/2] by 8-point Gauss-Legendre (independent of
    the oracle's closed-form monomial averages)."""
    xg, wg = np.polynomial.legendre.leggauss(8)
    x = o + xg / 2.0
    return float(np.sum(wg / 2.0 * np.polyval(coeffs[::-1], x)))


def poly_val(coeffs, x, deriv=0):
    p = np.polynomial.Polynomial(coeffs)
    return float(p.deriv(deriv)(x)) if deriv else float(p(x))


@pytest.mark.parametrize("offsets", [(-2, -1, 0), (-1, 0, 1), (0, 1, 2), (-1, 0, 1, 2), (-2, -1, 0, 1, 2)])
@pytest.mark.parametrize("xi", [0.5, -0.5, GAUSS_XI[0], GAUSS_XI[1], 0.1])
@pytest.mark.parametrize("deriv", [0, 1])
def test_poly_weights_exact_for_degree(offsets, xi, deriv):
    rng = np.random.default_rng(7)
    deg = len(offsets) - 1
    for _ in range(5):
        coeffs = rng.standard_normal(deg + 1)
        qb = [cell_average_by_quadrature(coeffs, o) for o in offsets]
        w = poly_weights(offsets, xi, deriv)
        assert abs(np.dot(w, qb) - poly_val(coeffs, xi, deriv)) < 1e-12


def test_face_linear_weights_textbook():
    _, g = weno_linear_weights(0.5)
    assert np.allclose(g, GOLD["weno_js_face_linear_weights"]["value"], atol=1e-14)
    _, gm = weno_linear_weights(-0.5)
    assert np.allclose(gm, GOLD["weno_js_face_linear_weights"]["value"][::-1], atol=1e-14)


def test_gauss_linear_weights_positive_and_mirror():
    _, gm = weno_linear_weights(GAUSS_XI[0])
    _, gp = weno_linear_weights(GAUSS_XI[1])
    assert min(gm) > 0 and min(gp) > 0
    assert abs(sum(gm) - 1) < 1e-14
    assert np.allclose(gm, gp[::-1], atol=1e-14)


def test_smoothness_indicators_match_jiang_shu():
    rng = np.random.default_rng(3)
    for _ in range(20):
        a, b, c = rng.standard_normal(3)
        js = [
            13.0 / 12.0 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2,
            13.0 / 12.0 * (a - 2 * b + c) ** 2 + 0.25 * (a - c) ** 2,
            13.0 / 12.0 * (a - 2 * b + c) ** 2 + 0.25 * (3 * a - 4 * b + c) ** 2,
        ]
        for k in range(3):
            beta = sum(w * (d[0] * a + d[1] * b + d[2] * c) ** 2 for w, d in smoothness_rules(k))
            assert abs(beta - js[k]) < 1e-12 * max(1.0, js[k])


@pytest.mark.parametrize("xi", [0.5, -0.5, GAUSS_XI[0], GAUSS_XI[1]])
def test_weno_exact_for_quadratics(xi):
    rng = np.random.default_rng(11)
    for _ in range(10):
        coeffs = rng.standard_normal(3)
        q5 = [torch.tensor(cell_average_by_quadrature(coeffs, o), dtype=torch.float64) for o in range(-2, 3)]
        v = weno_point(q5, xi, 1e-6)
        assert abs(float(v) - poly_val(coeffs, xi)) < 1e-12


@pytest.mark.parametrize("xi", [0.5, -0.5, GAUSS_XI[0], GAUSS_XI[1]])
def test_weno_linear_limit_is_quartic(xi):
    # a huge epsilon makes every nonlinear weight equal to its linear weight: the scheme is the quartic
    rng = np.random.default_rng(12)
    for _ in range(10):
        coeffs = rng.standard_normal(5)
        q5 = [torch.tensor(cell_average_by_quadrature(coeffs, o), dtype=torch.float64) for o in range(-2, 3)]
        v = weno_point(q5, xi, 1e30)
        assert abs(float(v) - poly_val(coeffs, xi)) < 1e-10


def test_weno_fifth_order_at_face():
    # smooth data: error of the face value drops like h^5
    errs = []
    for n in (10, 20, 40):
        h = 2 * math.pi / n / 7.0
        xc = 0.3
        q5 = []
        for o in range(-2, 3):
            a, b = xc + (o - 0.5) * h, xc + (o + 0.5) * h
            q5.append(torch.tensor((-math.cos(b) + math.cos(a)) / h, dtype=torch.float64))
        v = float(weno_point(q5, 0.5, 1e-6 * h * h))
        errs.append(abs(v - math.sin(xc + 0.5 * h)))
    rate = math.log2(errs[1] / errs[2])
    assert rate > 4.5


def test_weno_nonoscillatory_on_step():
    q5 = [torch.tensor(v, dtype=torch.float64) for v in (0.0, 0.0, 0.0, 1.0, 1.0)]
    v = float(weno_point(q5, 0.5, 1e-6))
    assert -1e-6 < v < 0.02


def test_normal_derivative_stencil_exact_for_cubics():
    rng = np.random.default_rng(5)
    w = poly_weights((-1, 0, 1, 2), 0.5, deriv=1)
    assert np.allclose(w, np.array([1.0, -15.0, 15.0, -1.0]) / 12.0, atol=1e-13)
    for _ in range(5):
        coeffs = rng.standard_normal(4)
        qb = [cell_average_by_quadrature(coeffs, o) for o in (-1, 0, 1, 2)]
        assert abs(np.dot(w, qb) - poly_val(coeffs, 0.5, 1)) < 1e-12


def test_linear_point_quartic_value_and_derivative():
    rng = np.random.default_rng(6)
    for xi in GAUSS_XI:
        for _ in range(5):
            coeffs = rng.standard_normal(5)
            q5 = [cell_average_by_quadrature(coeffs, o) for o in range(-2, 3)]
            assert abs(linear_point(q5, xi) - poly_val(coeffs, xi)) < 1e-12
            assert abs(linear_point(q5, xi, 1) - poly_val(coeffs, xi, 1)) < 1e-11
