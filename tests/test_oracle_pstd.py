"""Pins of the oracle's PSTD step (Eq. PSTDupdating) and running surface DFT
(Eqs. psiphasor-scaleddpsiphasor) against closed forms and invariants."""
import math

import numpy as np
import pytest

import synth
from oracle import pstd


def periodic_problem(n, v_over_E0, dt=0.0):
    h = 0.1
    k0 = 2 * math.pi / (8 * h)
    E0 = k0 * k0 / 2
    p = synth.Problem(n=n, h=(h, h, h), k0=k0, abc_cells=(0, 0, 0), abc_U0=0.0,
                      tfsf=((0, 1, 2, 3),) * 3, v_max=abs(v_over_E0) * E0, dt=dt)
    return p, E0


def plane_wave(model, n, mvec):
    dxb = model.dxb
    kv = [2 * math.pi * mvec[a] / (n[a] * dxb[a]) for a in range(3)]
    X = [pstd._bcast(pstd.coords(n[a], dxb[a]), a) for a in range(3)]
    sp = np.exp(1j * (kv[0] * X[0] + kv[1] * X[1] + kv[2] * X[2])) * np.ones((n[2], n[1], n[0]))
    return sp, sum(k * k for k in kv)


@pytest.mark.parametrize("mvec,v", [((2, -1, 1), 0.3), ((0, 0, 0), -0.4), ((4, 3, -2), 0.0), ((-8, 6, 4), 0.1)])
def test_discrete_plane_wave_dispersion(mvec, v):
    """A grid plane wave with constant V, no absorber and no source stays an
    exact leapfrog mode: sin(w dtau) = dtau (eta kbar^2 + v)."""
    n = (16, 12, 8)
    p, E0 = periodic_problem(n, v)
    m = pstd.build(p, np.full((n[2], n[1], n[0]), v * E0))
    sp, k2 = plane_wave(m, n, mvec)
    w = math.asin(m.dtau * (m.eta * k2 + v)) / m.dtau
    prev, cur = sp * np.exp(1j * w * m.dtau), sp.copy()
    steps = 1500
    for s in range(steps):
        prev, cur = cur, pstd.step(m, prev, cur, s, with_source=False)
    assert np.abs(cur - sp * np.exp(-1j * w * m.dtau * steps)).max() < 1e-11


def test_central_wave_has_exact_frequency():
    """With eta = sin(dtau)/dtau the |kbar| = 1 wave oscillates at exactly
    frequency 1 (Section 2.4)."""
    n = (8, 8, 8)
    p, E0 = periodic_problem(n, 0.0)
    m = pstd.build(p, np.zeros((8, 8, 8)))
    sp, k2 = plane_wave(m, n, (0, 0, 1))  # 8 points per wavelength -> kbar = 1
    assert k2 == pytest.approx(1.0, rel=1e-14)
    prev, cur = sp * np.exp(1j * m.dtau), sp.copy()
    for s in range(1000):
        prev, cur = cur, pstd.step(m, prev, cur, s, with_source=False)
    assert np.abs(cur - sp * np.exp(-1j * m.dtau * 1000)).max() < 1e-11


def test_leapfrog_invariant_with_random_potential():
    """For Hermitian H (real V, no mask, no source) Re<psi^{n+1}, psi^n> is
    conserved exactly by the leapfrog."""
    n = (12, 10, 8)
    p, E0 = periodic_problem(n, 0.5)
    rng = np.random.default_rng(0)
    V = rng.uniform(-0.5, 0.5, size=(8, 10, 12)) * E0
    m = pstd.build(p, V)
    prev = synth.random_state(n, 1)
    cur = synth.random_state(n, 2)
    q0 = np.vdot(cur, prev).real
    for s in range(400):
        prev, cur = cur, pstd.step(m, prev, cur, s, with_source=False)
    assert abs(np.vdot(cur, prev).real - q0) <= 1e-12 * np.vdot(cur, cur).real


@pytest.mark.parametrize("factor", [1.01, 1.05])
def test_growth_above_the_bound(factor):
    """Above the exact threshold dtau * lambda_max = 1 the Nyquist-corner mode
    grows by |q| = theta + sqrt(theta^2 - 1) per step, theta = dtau lambda."""
    n = (8, 8, 8)
    p0, E0 = periodic_problem(n, 0.0)
    m0 = pstd.build(p0, np.zeros((8, 8, 8)))
    lam_paper = math.pi ** 2 * float(np.sum(1 / m0.dxb ** 2))  # kinetic part of Eq. dtau_stability
    dtau = factor / lam_paper
    p, _ = periodic_problem(n, 0.0, dt=dtau / E0)
    m = pstd.build(p, np.zeros((8, 8, 8)))
    theta = m.dtau * m.eta * lam_paper
    x = np.arange(8)
    nyq = ((-1.0) ** x)[None, None, :] * ((-1.0) ** x)[None, :, None] * ((-1.0) ** x)[:, None, None] + 0j
    prev, cur = np.zeros_like(nyq), nyq.copy()
    for s in range(60):
        prev, cur = cur, pstd.step(m, prev, cur, s, with_source=False)
    ratio = np.abs(cur).max() / np.abs(prev).max()
    if theta > 1:
        assert ratio == pytest.approx(theta + math.sqrt(theta * theta - 1), rel=1e-2)
    else:
        # eta < 1 can pull a slightly-too-large step back under the exact threshold
        assert ratio < 1.0 + 1e-9 or theta <= 1


def test_growth_at_the_literal_workload_step():
    """dt = 0.1 dx^2 (the plain-method workload's literal step) exceeds the
    bound: the corner mode grows by about 2.6 per step."""
    prob, _ = synth.plain_barrier()
    E0 = pstd.central_energy(prob)
    dtau = E0 * 0.1 * 0.1 ** 2
    lam = math.pi ** 2 * float(np.sum(1 / pstd.dxbar(prob) ** 2)) + 0.5
    assert dtau > pstd.critical_dtau(pstd.dxbar(prob), 0.5)
    theta = dtau * (pstd.eta_of(dtau) * (lam - 0.5) + 0.5)
    assert theta + math.sqrt(theta * theta - 1) == pytest.approx(2.61, abs=0.01)


def test_absorber_removes_outgoing_packet():
    """A packet launched towards the layer loses most of its norm there."""
    prob, V = synth.tiny(n=(32, 8, 8), P=8, v0=0.0, radius_cells=0)
    prob = prob.replace(abc_cells=(8, 0, 0))
    m = pstd.build(prob, V)
    x = pstd.coords(32, m.dxb[0])
    g = np.exp(-0.5 * (x / 3.0) ** 2) * np.exp(1j * x)  # moves towards +x
    w = 1.0 + 1.0 / 2  # not needed exactly: start both levels from the packet
    cur = np.broadcast_to(g[None, None, :], (8, 8, 32)).astype(np.complex128)
    prev = np.broadcast_to((g * np.exp(1j * m.dtau))[None, None, :], (8, 8, 32)).astype(np.complex128)
    n0 = np.vdot(cur, cur).real
    for s in range(1600):
        prev, cur = cur, pstd.step(m, prev, cur, s, with_source=False)
    assert np.vdot(cur, cur).real < 0.05 * n0


def test_tfsf_reproduces_incident_wave_without_potential():
    """With V = 0 the total field in the TF core is the incident wave and the
    scattered-field region stays nearly empty; the leakage through a 6-cell
    taper at 8 points per wavelength is about 1e-2 (measured, not a paper
    number)."""
    prob, V = synth.tiny(n=(32, 32, 32), P=6, transition=6, steps=2600, v0=0.0,
                         radius_cells=0, dft=(0, 0))
    model, prev, cur, _ = pstd.run(prob, V)
    inc, _ = pstd.incident(model, prob.n_steps)
    tf = prob.tfsf[0]
    core = (slice(tf[1], tf[2] + 1),) * 3
    assert np.abs(cur[core] - inc[core]).max() < 2e-2
    sf = model.zeta == 0
    inner = np.zeros_like(sf)
    inner[6:-6, 6:-6, 6:-6] = True
    assert np.abs(cur[sf & inner]).max() < 2e-2
    # linear in the incident amplitude: the source is the only drive
    assert np.abs(cur).max() > 0.5


def test_source_is_laplacian_of_product_minus_product_of_laplacian():
    """The source of Eq. dimlesstildeSchrodinger is what the taper adds to the
    free equation: S = lap(zeta psi_inc) - zeta lap(psi_inc).  Check it at
    every wall cell of an oblique-incidence grid against that right-hand
    side differentiated numerically (Richardson-extrapolated central
    differences of the continuous taper of Eq. zeta_y times the plane wave),
    so a wrong coefficient, sign, index shift or length scale in the
    oracle's analytic derivatives fails by O(1)."""
    prob, V = synth.tiny(n=(24, 20, 28), P=3, transition=4, theta=0.7, phi=2.1, v0=0.0, radius_cells=0)
    prob = prob.replace(ramp_periods=0.0)
    m = pstd.build(prob, V)
    dxb = m.dxb
    kh = m.kh

    def zeta_c(a, u):
        """Eq. zeta_y at the continuous index position u of axis a."""
        y0, y1, y2, y3 = prob.tfsf[a]
        if u <= y0 or u >= y3:
            return 0.0
        if u < y1:
            return float(pstd.xi((u - y0) / (y1 - y0)))
        if u <= y2:
            return 1.0
        return 1.0 - float(pstd.xi((u - y2) / (y3 - y2)))

    def f(xb):
        """zeta(x_bar) exp(i k_hat . x_bar) at a reduced position."""
        z = 1.0
        for a in range(3):
            z *= zeta_c(a, xb[a] / dxb[a] + prob.n[a] // 2)
        return z * np.exp(1j * float(np.dot(kh, xb)))

    def lap(xb, h):
        out = 0.0
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            out += (f(xb + e) - 2 * f(xb) + f(xb - e)) / h ** 2
        return out

    n = 123
    S = pstd.source(m, n) / np.exp(-1j * n * m.dtau)   # ramp off: R = 1
    wall = (m.zeta > 0) & (m.zeta < 1)
    ks, js, is_ = np.nonzero(wall)
    rng = np.random.default_rng(8)
    pick = rng.choice(ks.size, size=60, replace=False)
    smax = np.abs(S).max()
    worst = 0.0
    for p_ in pick:
        k, j, i = ks[p_], js[p_], is_[p_]
        xb = np.array([(i - prob.n[0] // 2) * dxb[0], (j - prob.n[1] // 2) * dxb[1], (k - prob.n[2] // 2) * dxb[2]])
        h = 4e-3
        d = (4 * lap(xb, h / 2) - lap(xb, h)) / 3
        expect = d - f(xb) * (-1.0)            # lap(psi_inc) = -|k_hat|^2 psi_inc
        worst = max(worst, abs(S[k, j, i] - expect) / smax)
    assert worst < 1e-6, worst


def test_surface_dft_of_monochromatic_field():
    """psi^n = A exp(-i tau_n) over M steps gives Phi = M A; the normalised
    phasor (incident phasor at the origin, R = 1) is A."""
    prob, V = synth.tiny(n=(16, 16, 16), P=2, transition=2, v0=0.0, radius_cells=0)
    prob = prob.replace(ramp_periods=0.0)
    m = pstd.build(prob, V)
    sd = pstd.SurfaceDFT(m)
    A = synth.random_state(prob.n, 9)
    for n in range(37):
        sd.accumulate(A * np.exp(-1j * n * m.dtau), n)
    phi, dphi = sd.normalized()
    for f in range(6):
        a, _ = pstd.FACES[f]
        idx = pstd.face_index(prob, f)
        assert np.abs(phi[f] - pstd.plane(A, a, idx)).max() < 1e-13
        assert np.abs(dphi[f] - pstd.plane(pstd.derivative(m, A, a), a, idx)).max() < 1e-12
    assert sd.inc == pytest.approx(37.0)


def test_step_at_matches_full_step():
    prob, V = synth.tiny(n=(20, 16, 24), P=3, transition=3, v0=0.4, radius_cells=3)
    prob = prob.replace(theta=0.7, phi=2.1, ramp_periods=0.5)
    m = pstd.build(prob, V)
    prev = synth.random_state(prob.n, 3)
    cur = synth.random_state(prob.n, 4)
    full = pstd.step(m, prev, cur, 17)
    rng = np.random.default_rng(5)
    pts = [(int(rng.integers(20)), int(rng.integers(16)), int(rng.integers(24))) for _ in range(30)]
    pts += [(7, 8, 9), (6, 6, 6), (5, 5, 5)]
    got = pstd.step_at(m, prev, cur, 17, pts)
    ref = np.array([full[k, j, i] for (i, j, k) in pts])
    assert np.abs(got - ref).max() < 1e-12
