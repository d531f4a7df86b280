"""Pins of the partial-wave reference (Section 4): library Bessel functions
(also at ka = n pi, where j_0 vanishes), the optical theorem, the Born limit
and the hard-sphere limit."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import partial_waves as pw


@pytest.mark.parametrize("x", [0.3, 2.0, 4.712, 7.3, 18.85, 40.0, 3 * math.pi, 6 * math.pi, 1.5 * math.pi])
def test_bessel_functions_match_library(x):
    l = np.arange(31)
    ref = special.spherical_jn(l, x)
    # j_0 vanishes at x = n pi: compare there on the scale of the largest j_l
    assert np.allclose(pw.sph_jn(30, x), ref, rtol=1e-11, atol=1e-14 * np.abs(ref).max())
    yy = special.spherical_yn(l[:20], x)
    assert np.allclose(pw.sph_yn(19, x), yy, rtol=1e-11)
    assert np.allclose(pw.sph_in(30, x), special.spherical_in(l, x), rtol=1e-11, atol=1e-300)


@pytest.mark.parametrize("s", [0.5, 1.0, -0.5, -1.0, 2.0])
def test_optical_theorem(s):
    k = 1.0
    a = 4 * math.pi
    V0 = s * k * k / 2
    sigma = pw.total_cross_section(k, a, V0)
    f0 = pw.amplitude(k, a, V0, 0.0)
    assert 4 * math.pi / k * f0.imag == pytest.approx(sigma, rel=1e-12)


def test_born_limit():
    k, a = 2.0, 1.3
    th = np.linspace(0.1, 3.0, 9)
    for eps in (1e-3, 1e-4):
        f = pw.amplitude(k, a, eps, th)
        fb = pw.born_amplitude(k, a, eps, th)
        assert np.abs(f - fb).max() < 30 * eps ** 2 + 1e-14


def test_hard_sphere_limit():
    k, a = 1.7, 1.1
    # a barrier far above E: beta_l ~ q, so tan d_l -> j_l/y_l with an O(1/q)
    # error; Richardson extrapolation over q and 2q removes the first order
    ref = special.spherical_jn(np.arange(7), k * a) / special.spherical_yn(np.arange(7), k * a)
    t = []
    for qa in (100.0, 200.0):
        q = qa / a
        t.append(np.tan(pw.phase_shifts(k, a, k * k / 2 + q * q / 2, 6)))
    err1 = np.abs(t[0] / ref - 1)
    err_ex = np.abs((2 * t[1] - t[0]) / ref - 1)
    assert err1.max() < 0.15
    assert (err_ex < 0.1 * err1).all()


def test_equal_energy_branch_is_continuous():
    k, a = 1.3, 2.0
    E = k * k / 2
    d0 = pw.phase_shifts(k, a, E, 8)
    for V0 in (E * (1 - 1e-9), E * (1 + 1e-9)):
        assert np.allclose(np.tan(pw.phase_shifts(k, a, V0, 8)), np.tan(d0), rtol=1e-6, atol=1e-8)


def test_scattered_wave_tends_to_the_amplitude():
    """r e^{-ikr} psi_sc(r) -> f(theta) at large kr (the neglected terms are
    of order l^2 / kr for the partial waves that carry the amplitude)."""
    k, a, V0 = 1.0, 2.0, 0.3
    th = np.linspace(0.0, math.pi, 13)
    r = 4.0e5
    lim = r * np.exp(-1j * k * r) * pw.scattered_wave(k, a, V0, r, th)
    f = pw.amplitude(k, a, V0, th)
    assert np.abs(lim - f).max() <= 2e-4 * np.abs(f).max()


def test_scattered_wave_is_the_born_integral_for_a_weak_potential():
    """At finite r (kr = 6, outside the ball) and weak V0 the exact scattered
    wave equals the first-Born integral -(2m/hbar^2)(V0 / 4 pi) int_ball
    e^{ik|r - r'|} / |r - r'| e^{ikz'} d^3r', evaluated here by a product
    Gauss-Legendre rule over the ball, to O(V0)."""
    k, a = 1.0, 1.5
    E = 0.5 * k * k
    V0 = 1e-3 * E
    rr = 6.0
    th = np.array([0.0, 0.7, 1.6, 2.5, math.pi])
    xr, wr = np.polynomial.legendre.leggauss(28)
    xc, wc = np.polynomial.legendre.leggauss(36)
    rp = 0.5 * a * (xr + 1)
    wrp = 0.5 * a * wr * rp ** 2
    nph = 48
    php = 2 * math.pi * np.arange(nph) / nph
    R, C, Ph = np.meshgrid(rp, xc, php, indexing="ij")
    W = wrp[:, None, None] * wc[None, :, None] * (2 * math.pi / nph)
    S = np.sqrt(1 - C * C)
    Xp, Yp, Zp = R * S * np.cos(Ph), R * S * np.sin(Ph), R * C
    born = []
    for t in th:
        x, z = rr * math.sin(t), rr * math.cos(t)
        dist = np.sqrt((x - Xp) ** 2 + Yp ** 2 + (z - Zp) ** 2)
        integ = np.sum(W * np.exp(1j * k * dist) / dist * np.exp(1j * k * Zp))
        born.append(-(2 * V0) / (4 * math.pi) * integ)
    born = np.array(born)
    exact = pw.scattered_wave(k, a, V0, rr, th)
    assert np.abs(exact - born).max() <= 5e-3 * np.abs(born).max()


def test_stored_square_potential_reference_is_the_oracle():
    """tests/golden/square_potential_reference.json (read by the benchmark)
    holds what the oracle gives now."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "square_potential_reference.json")
    gold = json.load(open(path))
    th = np.deg2rad(np.asarray(gold["angles_deg"]))
    k, a = gold["k0"], gold["radius"]
    for s in ("1.0", "-1.0"):
        V0 = float(s) * k * k / 2
        f = pw.amplitude(k, a, V0, th)
        re_, im_ = gold["potentials"][s]["far"]
        assert np.allclose(np.asarray(re_) + 1j * np.asarray(im_), f, rtol=1e-12, atol=1e-14)
        v = pw.scattered_wave(k, a, V0, 100.0 / k, th)
        re_, im_ = gold["potentials"][s]["r100"]
        assert np.allclose(np.asarray(re_) + 1j * np.asarray(im_), v, rtol=1e-12, atol=1e-14)
