"""Pins of the spherical-surface oracle: quadrature against the library
Gauss-Legendre rule and the sphere's area, Lagrange weights against
polynomials, the Kirchhoff integral against analytic outgoing and regular
fields, and the grid interpolation at the benchmark spacing."""
import math

import numpy as np
import pytest

import synth
from oracle import sphere as osph


def test_gauss_legendre_matches_library_rule():
    for n in (5, 32, 64):
        x, w = osph.gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.abs(x - xr).max() < 1e-14 and np.abs(w - wr).max() < 1e-14


def test_lagrange_reproduces_polynomials():
    rng = np.random.default_rng(0)
    for _ in range(20):
        u = rng.uniform(10, 20)
        i0, L, dL = osph.lagrange(u, 8)
        xs = i0 + np.arange(8)
        assert xs[3] <= u < xs[4]
        c = rng.normal(size=8)  # degree 7
        f = np.polyval(c, xs - 15.0)
        assert abs(L @ f - np.polyval(c, u - 15.0)) < 1e-9 * np.abs(f).max()
        assert abs(dL @ f - np.polyval(np.polyder(c), u - 15.0)) < 1e-8 * np.abs(f).max()


@pytest.fixture(scope="module")
def sph():
    prob, _ = synth.square_barrier_160()
    return prob, osph.Sphere(prob, 5.0, n_theta=64, n_phi=128)


def point_source(x, x0, k=1.0):
    d = x - x0
    rho = np.sqrt(np.sum(d * d, axis=-1))
    f = np.exp(1j * k * rho) / rho
    grad = (f * (1j * k - 1 / rho))[..., None] * d / rho[..., None]
    return f, grad


def test_quadrature_area(sph):
    _, s = sph
    assert abs(s.weights.sum() - 4 * math.pi * s.R ** 2) < 1e-10 * 4 * math.pi * s.R ** 2
    assert np.allclose(np.linalg.norm(s.nodes, axis=1), s.R)


@pytest.mark.parametrize("k", [1.0, 1.3, 0.7])
def test_kirchhoff_reproduces_outgoing_field(sph, k):
    """An outgoing point-source wave of wavenumber k (the central wave, or a
    phasor of a pulsed run) from inside: the integral with G = exp(ikR)/(4
    pi R) gives it back outside, and its far field exp(-ik r_hat . x0)."""
    prob, s = sph
    x0 = np.array([2.0, -1.5, 3.0])                     # reduced, inside (R = 39.3)
    f, g = point_source(s.nodes, x0, k)
    dn = np.sum(s.normal * g, axis=1)
    rng = np.random.default_rng(1)
    pts = rng.normal(size=(12, 3))
    pts = pts / np.linalg.norm(pts, axis=1, keepdims=True) * rng.uniform(45, 120, size=(12, 1))
    got = s.project(f, dn, pts, k=k)
    ref, _ = point_source(pts, x0, k)
    assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()
    dirs = rng.normal(size=(12, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    ff = s.far_field(f, dn, dirs, k=k)
    assert np.abs(ff - np.exp(-1j * k * (dirs @ x0)) / prob.k0).max() < 1e-9 / prob.k0


def test_kirchhoff_of_regular_field_vanishes_outside(sph):
    _, s = sph
    kh = np.array([0.3, -0.4, math.sqrt(1 - 0.25)])
    f = np.exp(1j * s.nodes @ kh)
    dn = 1j * (s.normal @ kh) * f
    pts = np.array([[0, 0, 60.0], [50.0, 10.0, -20.0]])
    assert np.abs(s.project(f, dn, pts)).max() < 1e-9


def test_grid_interpolation_at_benchmark_spacing(sph):
    """Node values and normal derivatives of an outgoing field interpolated
    from its samples on the grid (8 points per wavelength, 8-point stencils),
    and the far field they give."""
    prob, s = sph
    x0 = np.array([1.0, 0.5, -2.0])
    n = prob.n
    field = np.zeros((n[2], n[1], n[0]), np.complex128)
    for (k, j, i) in s.shell:
        x = np.array([(i - n[0] // 2) * s.dxb[0], (j - n[1] // 2) * s.dxb[1], (k - n[2] // 2) * s.dxb[2]])
        field[k, j, i] = point_source(x[None, :], x0)[0][0]
    v, dn = s.node_values(field)
    fe, ge = point_source(s.nodes, x0)
    dne = np.sum(s.normal * ge, axis=1)
    ev = np.abs(v - fe).max() / np.abs(fe).max()
    ed = np.abs(dn - dne).max() / np.abs(dne).max()
    print("interpolation max rel err: value", ev, "normal derivative", ed)
    assert ev < 2e-4 and ed < 2e-3
    dirs = np.array([[0, 0, 1.0], [1, 0, 0], [0.6, 0.0, -0.8]])
    ff = s.far_field(v, dn, dirs)
    ref = np.exp(-1j * dirs @ x0) / prob.k0
    assert np.abs(ff - ref).max() < 2e-3 * np.abs(ref).max()


def test_shell_dft_removes_the_incident_part_exactly():
    """Feeding the shell DFT the incident part zeta psi_inc alone (ramped,
    oblique) leaves zero scattered phasor."""
    from oracle import pstd as opstd
    prob, _ = synth.tiny(n=(24, 24, 32), P=3, transition=3, theta=0.5, phi=0.8, steps=60, dft=(0, 60))
    prob = prob.replace(ramp_periods=0.5)
    V = np.zeros((prob.n[2], prob.n[1], prob.n[0]))
    m = opstd.build(prob, V)
    s = osph.Sphere(prob, 0.6, n_theta=8, n_phi=16, order=4)
    sd = osph.ShellDFT(m, s)
    for n in range(60):
        tau = n * m.dtau
        sd.accumulate(m.zeta * m.phase * opstd.ramp(tau, m.tau_r) * np.exp(-1j * tau), n)
    assert np.abs(sd.normalized()).max() < 1e-13
    assert (m.zeta[s.shell_mask()] > 0).any()   # the stencils do reach into the taper
