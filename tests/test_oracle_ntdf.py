"""Pins of the oracle's NTDF projection (Sections 3.1-3.2): analytic waves
whose surface data and outside values are known in closed form."""
import math

import numpy as np
import pytest

from oracle import ntdf, pstd


def window(N, lo):
    """1 on the box surface (plus margin), a smooth xi ramp to 0 at the plane
    edges: stands in for the absorber's decay of the plane data."""
    a = lo - 3
    w = np.ones(N)
    for t in range(N):
        d = min(t, N - 1 - t)
        if d < a:
            w[t] = pstd.xi(d / a)
    return w


def surface_data(box, field, lo):
    """field(r[3, ...]) -> (psi, grad psi components) on each face plane."""
    phi, dphi = [], []
    N = box.n[0]
    for f in range(6):
        a, b, c, idx, _ = box.face(f)
        xb = box.coord(b, np.arange(box.n[b]))
        xc = box.coord(c, np.arange(box.n[c]))
        XC, XB = np.meshgrid(xc, xb, indexing="ij")
        r = np.zeros((3,) + XC.shape)
        r[a] = box.coord(a, idx)
        r[b] = XB
        r[c] = XC
        psi, grad = field(r)
        W = window(box.n[c], lo)[:, None] * window(box.n[b], lo)[None, :]
        phi.append(psi * W)
        dphi.append(grad[a] * W)
    return phi, dphi


def point_source(src):
    def field(r):
        d = r - np.asarray(src)[:, None, None]
        rho = np.sqrt((d ** 2).sum(0))
        psi = np.exp(1j * rho) / rho
        return psi, [(1j - 1 / rho) * psi * d[a] / rho for a in range(3)]
    return field


def plane_wave(kh):
    def field(r):
        psi = np.exp(1j * np.tensordot(kh, r, axes=(0, 0)))
        return psi, [1j * kh[a] * psi for a in range(3)]
    return field


@pytest.mark.parametrize("N,lo,dx,tol", [(24, 6, math.pi / 4, 4e-3), (32, 8, math.pi / 6, 2e-3)])
def test_spherical_wave_is_reconstructed(N, lo, dx, tol):
    """Section 3.4's test: surface data of exp(ir)/r reproduce it outside S."""
    box = ntdf.Box((N,) * 3, [dx] * 3, (lo,) * 3, (N - lo,) * 3)
    src = np.array([0.05, -0.1, 0.07])
    phi, dphi = surface_data(box, point_source(src), lo)
    pts = np.array([[0, 0, 30.0], [20, 10, -15], [0, 40, 3], [100, 0, 0]])
    got = ntdf.project_direct(box, phi, dphi, pts)
    rho = np.linalg.norm(pts - src, axis=1)
    ref = np.exp(1j * rho) / rho
    assert (np.abs(got - ref) / np.abs(ref)).max() < tol


def test_taylor_form_matches_direct_cell_sums():
    N, lo = 20, 5
    box = ntdf.Box((N, 18, 22), [math.pi / 4, math.pi / 5, math.pi / 4.5], (lo, 4, 6), (N - lo, 14, 16))
    rng = np.random.default_rng(2)
    phi = [rng.normal(size=s) + 1j * rng.normal(size=s) for s in
           [(22, 18), (22, 18), (22, 20), (22, 20), (18, 20), (18, 20)]]
    dphi = [rng.normal(size=x.shape) + 1j * rng.normal(size=x.shape) for x in phi]
    pts = np.array([[0.3, 0.2, 25.0], [-30, 12, 4], [8, -9, -14], [300, 200, 100]])
    direct = ntdf.project_direct(box, phi, dphi, pts)
    tay = ntdf.TaylorTables(box, phi, dphi, order=8).project(pts)
    assert np.abs(tay - direct).max() <= 1e-9 * np.abs(direct).max()
    # a low order is visibly worse: the expansion is what carries the accuracy
    low = ntdf.TaylorTables(box, phi, dphi, order=1).project(pts)
    assert np.abs(low - direct).max() > 1e-5 * np.abs(direct).max()


def test_far_field_of_point_sources():
    """f(r_hat) of exp(i|r - s|)/|r - s| is exp(-i r_hat . s)."""
    N, lo = 32, 8
    box = ntdf.Box((N,) * 3, [math.pi / 6] * 3, (lo,) * 3, (N - lo,) * 3)
    for src in ([0.0, 0.0, 0.0], [1.5, -0.7, 2.2]):
        phi, dphi = surface_data(box, point_source(src), lo)
        dirs = np.array([[0, 0, 1.0], [0.6, 0, 0.8], [0, -1, 0], [0.48, 0.6, 0.64], [-0.36, 0.48, -0.8]])
        f = ntdf.far_field(box, phi, dphi, dirs)
        ref = np.exp(-1j * dirs @ np.asarray(src))
        assert np.abs(f - ref).max() < 3e-3


def test_far_field_factored_equals_direct():
    N, lo = 16, 4
    box = ntdf.Box((N, 14, 18), [0.8, 0.7, 0.75], (lo, 3, 5), (N - lo, 11, 13))
    rng = np.random.default_rng(4)
    phi = [rng.normal(size=s) + 1j * rng.normal(size=s) for s in
           [(18, 14), (18, 14), (18, 16), (18, 16), (14, 16), (14, 16)]]
    dphi = [rng.normal(size=x.shape) + 1j * rng.normal(size=x.shape) for x in phi]
    d = rng.normal(size=(7, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    a = ntdf.far_field_direct(box, phi, dphi, d)
    b = ntdf.far_field(box, phi, dphi, d)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_plane_wave_on_surface_projects_to_zero():
    """A source-free field that is regular inside S contributes nothing
    outside: the surface integral of a plane wave vanishes there."""
    N, lo = 32, 8
    box = ntdf.Box((N,) * 3, [math.pi / 6] * 3, (lo,) * 3, (N - lo,) * 3)
    kh = np.array([0.36, 0.48, 0.8])
    phi, dphi = surface_data(box, plane_wave(kh), lo)
    pts = np.array([[0, 0, 40.0], [30, -20, 5], [-60, 10, 10]])
    got = ntdf.project_direct(box, phi, dphi, pts)
    assert np.abs(got).max() < 5e-3


def test_sinc_taylor_coefficients():
    x = np.linspace(-1.6, 1.6, 13)
    s = ntdf.sinc_taylor_coeffs(x, 3)
    assert np.allclose(s[0], ntdf.sinc(x), atol=1e-15)
    xs = np.where(x == 0, 1e-300, x)
    d1 = np.where(x == 0, 0.0, (xs * np.cos(xs) - np.sin(xs)) / xs ** 2)
    assert np.allclose(s[1], -d1, atol=1e-14)
    # sinc(x - alpha) reconstructed from the series at a finite shift
    alpha = 0.35
    full = ntdf.sinc_taylor_coeffs(x, 10)
    approx = sum(full[p] * alpha ** p for p in range(11))
    assert np.abs(approx - ntdf.sinc(x - alpha)).max() < 1e-11
