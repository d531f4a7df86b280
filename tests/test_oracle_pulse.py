"""Pins of the pulsed-incidence oracle (Section 2.2.3, calculation of the
incident wave: Eqs. Oinc, inc_d, pstd_psiinc, pstd_dpsiinc; Section 3.3
phasors at several frequencies)."""
import math

import numpy as np
import pytest

import synth
from oracle import pstd
from oracle import pulse


def test_1d_leapfrog_follows_each_modes_physical_root():
    """Started from psi^0 and the one-step-back state, the 1D leapfrog keeps
    every mode on its physical root: F[psi^n]_l = F[psi^0]_l exp(-i theta_l
    n), sin(theta_l) = dtau eta k_l^2 (the closed form of the two-step
    recursion)."""
    N, delta, dtau = 64, math.pi / 4, 0.02
    eta = math.sin(dtau) / dtau
    rng = np.random.default_rng(4)
    psi0 = rng.normal(size=N) + 1j * rng.normal(size=N)
    p = pulse.Pulse1D(psi0, delta, dtau, eta)
    for _ in range(500):
        p.step()
    th = pulse.scheme_frequency(pulse.kbar1d(N, delta), dtau, eta) * dtau
    want = np.fft.fft(psi0) * np.exp(-1j * th * 500)
    assert np.abs(np.fft.fft(p.cur) - want).max() < 1e-10 * np.abs(want).max()
    # the central wavenumber oscillates at exactly 1 per unit tau (eta)
    assert pulse.scheme_frequency(1.0, dtau, eta) == pytest.approx(1.0, rel=1e-13)


def test_spectral_interpolation():
    """Eqs. pstd_psiinc / pstd_dpsiinc reproduce the grid values at the grid
    points, and a trigonometric polynomial of the grid's modes (value and
    derivative) anywhere between them."""
    N, delta = 48, 0.37
    L = N * delta
    modes = {3: 0.7 - 0.2j, -5: 0.4j, 11: -0.3, -17: 0.1 + 0.1j}
    f = lambda d: sum(c * np.exp(2j * math.pi * m * d / L) for m, c in modes.items())  # noqa: E731
    df = lambda d: sum(c * 2j * math.pi * m / L * np.exp(2j * math.pi * m * d / L) for m, c in modes.items())  # noqa: E731
    dj = np.arange(N) * delta
    p = pulse.Pulse1D(f(dj), delta, 1e-3, 1.0)
    v, _ = p.at(dj)
    assert np.abs(v - f(dj)).max() < 1e-13
    d = np.random.default_rng(5).uniform(-3 * L, 3 * L, size=200)
    v, dv = p.at(d)
    assert np.abs(v - f(d)).max() < 1e-12
    assert np.abs(dv - df(d)).max() < 1e-11


def test_origin_corner_and_axis_coordinate():
    """Eq. Oinc picks the corner of the taper box the front meets first, so
    every cell of the taper box has d >= 0 and the corner itself d = 0."""
    for theta, phi in ((0.3, 0.4), (2.5, 1.9), (1.1, 3.6), (2.0, 5.5)):
        prob, V = synth.tiny(n=(20, 16, 24), P=3, transition=3, v0=0.0, radius_cells=0, theta=theta, phi=phi)
        m = pstd.build(prob, V)
        O = pulse.origin_corner(prob, m.kh)
        d = pulse.axis_coordinate(m, O)
        box = tuple(slice(prob.tfsf[a][0], prob.tfsf[a][3] + 1) for a in (2, 1, 0))
        assert d[box].min() == pytest.approx(0.0, abs=1e-12)
        assert d[O[2], O[1], O[0]] == 0.0


def test_single_mode_pulse_is_the_monochromatic_run():
    """A pulse made of the single 1D mode k = 1 (the 1D grid's length a
    multiple of 2 pi) is the plane wave of the monochromatic scheme without
    ramp, times the constant phase exp(-i k_hat . x_O): the pulsed run (1D
    leapfrog, spectral interpolation, Eqs. Oinc and inc_d) and the
    monochromatic run (analytic incident wave) agree to rounding, and so do
    their normalised phasors at k = 1."""
    prob, V = synth.tiny(n=(20, 24, 16), P=3, transition=3, v0=0.8, radius_cells=2, steps=120,
                         theta=0.6, phi=2.0, dft=(0, 0))
    prob = prob.replace(ramp_periods=0.0)
    m = pstd.build(prob, V)
    delta = m.dxb[0]
    N = 64                                   # N delta = 16 pi: k = 1 is mode 8
    psi0 = np.exp(1j * np.arange(N) * delta)
    pm, _, cur, _ = pulse.run(prob, V, psi0, delta)
    _, _, ref, _ = pstd.run(prob, V)
    xO = np.array([(pm.O[a] - prob.n[a] // 2) * m.dxb[a] for a in range(3)])
    ph = np.exp(-1j * (m.kh @ xO))
    assert np.abs(cur - ph * ref).max() < 1e-11 * np.abs(ref).max()
    assert np.abs(ref).max() > 0.5
    # phasors at k = 1 over the last 60 steps on the scattered-field cells
    mask = (m.zeta == 0) & (m.Gamma == 1)

    class Cells:
        def shell_mask(self):
            return mask
    prob = prob.replace(dft_begin=60, dft_end=120)
    pm, _, _, sd = pulse.run(prob, V, psi0, delta, sphere=Cells(), kbars=[1.0])
    prev = np.zeros_like(ref)
    cw = np.zeros_like(ref)
    cur = np.zeros_like(ref)
    for n in range(120):
        if n >= 60:
            cw += np.exp(1j * n * m.dtau) * cur
        prev, cur = cur, pstd.step(m, prev, cur, n)
    got = sd.normalized(0)[mask]
    want = cw[mask] / 60.0
    assert np.abs(got - want).max() < 1e-11 * np.abs(want).max()
    # and on the box planes (values and normal derivatives)
    _, _, _, bd = pulse.run(prob, V, psi0, delta, kbars=[1.0], box=True)
    _, _, _, cwd = pstd.run(prob, V)
    got_p, got_d = bd.normalized(0)
    want_p, want_d = cwd.normalized()
    for f in range(6):
        assert np.abs(got_p[f] - want_p[f]).max() < 1e-11 * np.abs(want_p[f]).max()
        assert np.abs(got_d[f] - want_d[f]).max() < 1e-11 * np.abs(want_d[f]).max()


def test_pulse_without_potential_crosses_the_box():
    """With V = 0 a Gaussian packet centred on k = 1 enters through the taper
    and leaves the scattered-field region nearly empty: mid-way, the total
    field in the TF core is the packet and the scattered-field region holds
    only the taper's leakage (measured about 1e-2 of the packet at 8 points
    per wavelength through a 6-cell taper, like the monochromatic scheme)."""
    prob, V = synth.tiny(n=(32, 32, 32), P=6, transition=6, v0=0.0, radius_cells=0, theta=0.5, phi=0.7,
                         dft=(0, 0))
    m = pstd.build(prob, V)
    delta = m.dxb[0]
    N = 256
    psi0 = synth.gaussian_pulse_1d(N, delta, 1.0, 6.0, -20.0)
    pm = pulse.PulseModel(prob, V, psi0, delta)
    prev = np.zeros(m.v.shape, np.complex128)
    cur = np.zeros_like(prev)
    # the centre moves 2 per unit tau: from d = -20 to the core (d about 10)
    steps = int(round(15.0 / m.dtau))
    for n in range(steps):
        prev, cur = cur, pm.step(prev, cur, n)
        pm.pulse.step()
    inc, _ = pm.pulse.at(pm.d)
    tf = prob.tfsf[0]
    core = (slice(tf[1], tf[2] + 1),) * 3
    amp = np.abs(inc[core]).max()
    assert amp > 0.3
    assert np.abs(cur[core] - inc[core]).max() < 2e-2 * amp
    sf = (m.zeta == 0)
    inner = np.zeros_like(sf)
    inner[6:-6, 6:-6, 6:-6] = True
    assert np.abs(cur[sf & inner]).max() < 2e-2 * amp
