"""Pins of the FDTD-variant oracle (Section 2.2.1, bound of Section 2.3.1: Eqs. y_stencil,
stencil_alpha, FDTDupdatePsi and the consistency terms of the walls)."""
import math

import numpy as np
import pytest

import synth
from oracle import fdtd
from oracle import pstd


def box_problem(n, box, v_over_E0=0.0, U0=0.0, P=0, theta=0.0, phi=0.0, dt=0.0):
    h = 0.1
    k0 = 2 * math.pi / (8 * h)
    E0 = k0 * k0 / 2
    tf = tuple((lo - 1, lo, hi, hi + 1) for (lo, hi) in box)
    p = synth.Problem(n=n, h=(h, h, h), k0=k0, theta=theta, phi=phi, abc_cells=(P,) * 3, abc_U0=U0,
                      tfsf=tf, v_max=abs(v_over_E0) * E0, dt=dt, ramp_periods=1.0)
    return p, E0


def test_stencil_coefficients_are_eighth_order():
    """The printed coefficients make a second-derivative stencil exact on
    polynomials up to degree 9: sum_l l^{2p} alpha_l (both sides) = 2 for
    p = 1 and 0 for p = 0, 2, 3, 4 (x^{2p} has second derivative 2 delta_p1 at 0)."""
    a = fdtd.ALPHA
    mom = [(a[0] if p == 0 else 0.0) + 2 * sum(a[l] * l ** (2 * p) for l in range(1, 5)) for p in range(5)]
    assert mom[0] == pytest.approx(0.0, abs=1e-15)
    assert mom[1] == pytest.approx(2.0, rel=1e-15)
    for p in (2, 3, 4):
        assert mom[p] == pytest.approx(0.0, abs=1e-12)
    # and the ninth-order term is the first that survives
    assert abs(2 * sum(a[l] * l ** 10 for l in range(1, 5))) > 1.0


@pytest.mark.parametrize("mvec,v", [((2, -1, 1), 0.3), ((4, 3, -2), 0.0), ((-8, 6, 4), -0.2)])
def test_discrete_plane_wave_dispersion(mvec, v):
    """A grid plane wave with constant v evolves as exp(i(k.x - W n)) with
    sin W = dtau (-sum_a symbol(k_a dxb_a) / dxb_a^2 + v), exactly."""
    n = (16, 12, 16)
    p, E0 = box_problem(n, ((0, 15), (0, 11), (0, 15)), v_over_E0=abs(v) + 0.5)
    V = np.full((16, 12, 16), v * E0)
    m = fdtd.build(p, V)
    dxb = m.dxb
    kv = [2 * math.pi * mvec[a] / (n[a] * dxb[a]) for a in range(3)]
    X = [pstd._bcast(pstd.coords(n[a], dxb[a]), a) for a in range(3)]
    sp = np.exp(1j * (kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2])) * np.ones((16, 12, 16))
    lam = -sum(float(fdtd.stencil_symbol(kv[a] * dxb[a])) / dxb[a] ** 2 for a in range(3)) + v
    W = math.asin(m.dtau * lam)
    prev, cur = sp * np.exp(1j * W), sp.copy()
    for s in range(1000):
        prev, cur = cur, fdtd.step(m, prev, cur, s, with_source=False)
    assert np.abs(cur - sp * np.exp(-1j * W * 1000)).max() < 1e-11


def test_leapfrog_invariant_with_random_potential():
    n = (12, 10, 8)
    p, E0 = box_problem(n, ((0, 11), (0, 9), (0, 7)), v_over_E0=0.5)
    rng = np.random.default_rng(1)
    m = fdtd.build(p, rng.uniform(-0.5, 0.5, size=(8, 10, 12)) * E0)
    prev = synth.random_state(n, 7)
    cur = synth.random_state(n, 8)
    q0 = np.vdot(cur, prev).real
    for s in range(400):
        prev, cur = cur, fdtd.step(m, prev, cur, s, with_source=False)
    assert abs(np.vdot(cur, prev).real - q0) <= 1e-12 * np.vdot(cur, cur).real


@pytest.mark.parametrize("factor", [0.99, 1.02])
def test_growth_above_the_bound(factor):
    """The Nyquist-corner mode is the stiffest: below dtau lambda = 1 it stays
    bounded, above it grows by theta + sqrt(theta^2 - 1) per step."""
    n = (8, 8, 8)
    p0, E0 = box_problem(n, ((0, 7), (0, 7), (0, 7)))
    lam = abs(float(fdtd.stencil_symbol(math.pi))) * float(np.sum(1 / pstd.dxbar(p0) ** 2))
    assert fdtd.critical_dtau(pstd.dxbar(p0), 0.0) == pytest.approx(1 / lam, rel=1e-15)
    p, _ = box_problem(n, ((0, 7), (0, 7), (0, 7)), dt=factor / lam / E0)
    m = fdtd.build(p, np.zeros((8, 8, 8)))
    x = np.arange(8)
    nyq = ((-1.0) ** x)[None, None, :] * ((-1.0) ** x)[None, :, None] * ((-1.0) ** x)[:, None, None] + 0j
    prev, cur = np.zeros_like(nyq), nyq.copy()
    for s in range(60):
        prev, cur = cur, fdtd.step(m, prev, cur, s, with_source=False)
    ratio = np.abs(cur).max() / np.abs(prev).max()
    theta = m.dtau * lam
    if theta > 1:
        assert ratio == pytest.approx(theta + math.sqrt(theta * theta - 1), rel=1e-2)
    else:
        assert np.abs(cur).max() < 10.0


def test_walls_are_exact_for_a_discrete_plane_wave():
    """With an incident wave that solves the free discrete scheme exactly (a
    grid plane wave at its discrete frequency, no ramp), the total-field box
    holds the incident wave and the scattered-field region stays zero, to
    rounding, after 300 steps: every wall term and every corner is right."""
    n = (24, 20, 28)
    box = ((7, 15), (6, 13), (9, 18))
    p, E0 = box_problem(n, box)
    m = fdtd.build(p, np.zeros((28, 20, 24)))
    mvec = (2, -1, 3)
    dxb = m.dxb
    kv = [2 * math.pi * mvec[a] / (n[a] * dxb[a]) for a in range(3)]
    X = [pstd._bcast(pstd.coords(n[a], dxb[a]), a) for a in range(3)]
    sp = np.exp(1j * (kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2])) * np.ones((28, 20, 24))
    lam = -sum(float(fdtd.stencil_symbol(kv[a] * dxb[a])) / dxb[a] ** 2 for a in range(3))
    W = math.asin(m.dtau * lam)
    T = fdtd.total_field_mask(m)
    inc = lambda s: sp * np.exp(-1j * W * s)  # noqa: E731
    prev, cur = T * inc(-1), T * inc(0)
    for s in range(300):
        prev, cur = cur, fdtd.step(m, prev, cur, s, psi_inc=inc(s))
    assert np.abs(cur - T * inc(300)).max() < 1e-12
    assert np.abs(cur * (1 - T)).max() < 1e-12


def test_wall_terms_equal_the_compact_form():
    """Accumulated wall by wall (the paper's scheme) the terms equal, at every
    cell, sum_a sum_l alpha_l sum_pm [T(c) - T(c pm l e_a)] psi_inc(c pm l e_a)
    / dxb_a^2, corners included."""
    n = (20, 24, 18)
    box = ((5, 13), (8, 15), (4, 12))
    p, E0 = box_problem(n, box, theta=0.7, phi=2.2)
    m = fdtd.build(p, np.zeros((18, 24, 20)))
    inc = synth.random_state(n, 9)
    T = fdtd.total_field_mask(m)
    compact = np.zeros_like(inc)
    for a in range(3):
        ax = pstd.NPAX[a]
        for l in range(1, 5):
            for sgn in (1, -1):
                Tn = np.roll(T, -sgn * l, axis=ax)
                In = np.roll(inc, -sgn * l, axis=ax)
                compact += fdtd.ALPHA[l] * (T - Tn) * In / m.dxb[a] ** 2
    assert np.abs(fdtd.wall_terms(m, inc) - compact).max() < 1e-12 * np.abs(compact).max()


def test_walls_hold_the_analytic_wave_at_the_discrete_frequency():
    """Started exactly after the ramp, the incident plane wave of any
    direction (not a grid mode) driven at the discrete frequency stays in the
    box and out of the scattered-field region to rounding: the walls only
    reach cells near the box, where the plane wave solves the stencil."""
    prob, V = synth.tiny(n=(32, 32, 32), P=4, transition=2, v0=0.0, radius_cells=0, steps=400,
                         theta=0.9, phi=0.4, dft=(0, 0))
    prob = prob.replace(scheme=1, ramp_periods=0.5)
    m = fdtd.build(prob, V)
    assert m.omega == pytest.approx(1.0, abs=1e-3) and m.omega != 1.0
    T = fdtd.total_field_mask(m)
    n0 = int(m.tau_r / m.dtau) + 2
    prev, cur = T * fdtd.incident(m, n0 - 1), T * fdtd.incident(m, n0)
    for s in range(n0, n0 + 300):
        prev, cur = cur, fdtd.step(m, prev, cur, s)
    assert np.abs(cur - T * fdtd.incident(m, n0 + 300)).max() < 1e-12


def test_shell_dft_removes_the_incident_wave_exactly():
    """Started exactly after the ramp with no scatterer, the field is T psi_inc
    at every step, so the normalised shell phasors vanish to rounding on a
    sphere whose shell crosses the walls of the total-field box; weights at
    the continuum frequency 1 instead of W leave a visible residue."""
    from oracle import sphere as osph
    prob, V = synth.tiny(n=(32, 32, 32), P=4, transition=2, v0=0.0, radius_cells=0, steps=400,
                         theta=0.9, phi=0.4, dft=(0, 0))
    prob = prob.replace(scheme=1, ramp_periods=0.5)
    m = fdtd.build(prob, V)
    # total-field box 8..24 around the centre 16: a sphere of 9 cells crosses its walls
    assert m.box == ((8, 24),) * 3
    sph = osph.Sphere(prob, 9 * prob.h[0], n_theta=8, n_phi=16)
    sd = fdtd.ShellDFT(m, sph)
    T = fdtd.total_field_mask(m)
    assert T[sph.shell_mask()].min() == 0.0 and T[sph.shell_mask()].max() == 1.0
    n0 = int(m.tau_r / m.dtau) + 2
    prev, cur = T * fdtd.incident(m, n0 - 1), T * fdtd.incident(m, n0)
    raw1 = np.zeros_like(sd.phi)
    for s in range(n0, n0 + 300):
        sd.accumulate(cur, s)
        raw1[sd.mask] += np.exp(1j * s * m.dtau) * cur[sd.mask]
        prev, cur = cur, fdtd.step(m, prev, cur, s)
    out = sd.normalized()
    assert np.abs(out).max() < 1e-12
    resid1 = np.abs(np.where(sd.mask, raw1 / sd.inc - T * m.phase, 0.0)).max()
    assert resid1 > 1e-4
