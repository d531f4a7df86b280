"""Pins of the oracle's scalar and 1D-table helpers (Sections 2.1-2.5)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import pstd

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_xi_closed_forms():
    assert pstd.xi(0.0) == 0.0
    assert abs(pstd.xi(0.5) - 0.5) < 1e-15
    assert abs(pstd.xi(1.0) - 1.0) < 1e-15
    rho = np.linspace(0, 1, 101)
    assert np.abs(pstd.xi(rho) + pstd.xi(1 - rho) - 1).max() < 1e-15
    # xi(1/4) = 1/4 - 2/(3 pi): the first taper weight of Eq. weight with n_t = 3
    assert abs(pstd.xi(0.25) - (0.25 - 2 / (3 * math.pi))) < 1e-15
    assert abs(pstd.xi(0.25) - 0.0377934092) < 1e-10
    assert abs(pstd.xi(0.75) - 0.9622065908) < 1e-10
    # xi' = (8/3) sin^4(pi rho) >= 0: monotone
    assert np.abs(pstd.dxi(rho) - 8 / 3 * np.sin(math.pi * rho) ** 4).max() < 1e-14
    assert (pstd.dxi(rho) >= -1e-15).all()


def test_xi_derivatives_match_finite_differences_and_vanish_at_ends():
    h = 1e-4
    rho = np.linspace(0.05, 0.95, 19)
    fd1 = (pstd.xi(rho + h) - pstd.xi(rho - h)) / (2 * h)
    fd2 = (pstd.dxi(rho + h) - pstd.dxi(rho - h)) / (2 * h)
    assert np.abs(fd1 - pstd.dxi(rho)).max() < 1e-6
    assert np.abs(fd2 - pstd.d2xi(rho)).max() < 1e-5
    # orders 1..4 vanish at both ends (golden: Eq. xi remark)
    assert GOLDEN["taper"]["vanishing_derivative_orders"] == [1, 2, 3, 4]
    for end in (0.0, 1.0):
        assert abs(pstd.dxi(end)) < 1e-15 and abs(pstd.d2xi(end)) < 1e-13
        # xi'' ~ (32 pi^4/3) (rho - end)^3 near the ends, so the third and
        # fourth derivatives vanish there too
        for e in (1e-2, 1e-3):
            r = end + (e if end == 0 else -e)
            assert abs(abs(pstd.d2xi(r)) / e ** 3 / (32 * math.pi ** 4 / 3) - 1) < 2 * e


def test_zeta_table():
    N, dxb = 40, math.pi / 4
    y = (8, 14, 25, 31)
    z, dz, d2z = pstd.zeta_1d(N, y, dxb)
    assert (z[:9] == 0).all() and (z[31:] == 0).all()
    assert (z[14:26] == 1).all()
    assert np.allclose(z[9:14], pstd.xi((np.arange(9, 14) - 8) / 6))
    assert np.allclose(z[26:31], 1 - pstd.xi((np.arange(26, 31) - 25) / 6))
    # analytic derivatives against a dense-sampled finite difference of the ramp
    for i in range(9, 14):
        rho = (i - 8) / 6
        hh = 1e-5
        fd = (pstd.xi(rho + hh) - pstd.xi(rho - hh)) / (2 * hh) / (6 * dxb)
        assert abs(fd - dz[i]) < 1e-8
    assert (dz[26:31] <= 0).all() and (dz[9:14] >= 0).all()


def test_absorber_table():
    g = pstd.absorber_gamma(20, 5, 3.0, 0.7)
    for i in range(20):
        d = min(i, 19 - i)
        assert g[i] == (3.0 / math.cosh(0.7 * d) ** 2 if d < 5 else 0.0)
    m = pstd.mask_1d(20, 5, 3.0, 0.7, 0.02)
    assert (m <= 1).all() and (m[5:15] == 1).all() and m[0] == pytest.approx(math.exp(-0.06))


@pytest.mark.parametrize("N", [8, 10, 12, 48])
def test_kbar_eigenfunctions(N):
    """exp(2 pi i m x / L) is an eigenfunction of F^-1 kbar^2 F with eigenvalue
    kbar_m^2; the Nyquist mode (-1)^i has (pi/dxb)^2."""
    from oracle import fft
    dxb = 0.7
    kb = pstd.kbar(N, dxb)
    x = np.arange(N)
    for m in range(N):
        e = np.exp(2j * math.pi * m * x / N)
        L = fft.ifft(kb ** 2 * fft.fft(e))
        mp = m if m < N // 2 else m - N
        assert np.abs(L - (2 * math.pi * mp / (N * dxb)) ** 2 * e).max() < 1e-11
    nyq = (-1.0) ** x
    assert np.abs(fft.ifft(kb ** 2 * fft.fft(nyq)) - (math.pi / dxb) ** 2 * nyq).max() < 1e-11
    assert kb[N // 2] == pytest.approx(-math.pi / dxb)


def test_stability_bound_paper_example():
    """Section 4: dtau = pi/1000 at dxb = pi/10 meets Eq. dtau_stability for
    s = +-1, +-0.5 (|V|max = |s| E0)."""
    g = GOLDEN["square_potential_run"]
    dxb = math.pi / 10
    for s in g["s_values"]:
        bound = pstd.critical_dtau([dxb] * 3, abs(s))
        assert math.pi / 1000 <= bound
    assert 0.94 < (math.pi / 1000) / pstd.critical_dtau([dxb] * 3, 1.0) < 0.95


def test_pstd_bound_smaller_than_fdtd8():
    """Section 2.3.2: pi^2/2 > 1024/315, so the PSTD critical step is smaller."""
    assert math.pi ** 2 / 2 > 1024 / 315


def test_physical_and_reduced_bounds_agree():
    prob, _ = synth.plain_barrier()
    E0 = pstd.central_energy(prob)
    dt = pstd.critical_dt(prob, prob.v_max)
    dtau = pstd.critical_dtau(pstd.dxbar(prob), prob.v_max / E0)
    assert E0 * dt / prob.hbar == pytest.approx(dtau, rel=1e-14)
    # 0.9 of the bound is the default step of every workload
    assert pstd.dtau_of(prob) == pytest.approx(0.9 * dtau, rel=1e-15)


def test_khat_and_contact_corner():
    lo, hi = (3, 4, 5), (20, 21, 22)
    corners = list(itertools.product(*[(lo[a], hi[a]) for a in range(3)]))
    rng = np.random.default_rng(1)
    for _ in range(200):
        th, ph = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi)
        kh = pstd.khat(th, ph)
        assert abs(np.linalg.norm(kh) - 1) < 1e-15
        # first contact = the corner with the smallest projection on k_hat
        best = min(corners, key=lambda c: float(np.dot(kh, c)))
        assert pstd.o_inc(kh, lo, hi) == best
    assert np.allclose(pstd.khat(0, 0), [0, 0, 1])


def test_ntdf_validation_geometry():
    """Section 3.4: the faces are at half-integer multiples of the spacing and
    the printed corner distance and far-field threshold follow from them."""
    g = GOLDEN["ntdf_validation"]
    d = math.pi / 10
    assert abs(g["x_plane"] - 131.5 * d) < 1e-4
    assert abs(g["y_plane"] - 116.5 * d) < 1e-4
    corner = math.sqrt(g["x_plane"] ** 2 + g["y_plane"] ** 2 + g["z_plane"] ** 2)
    assert abs(corner - g["corner_distance"]) < 1e-3
    assert abs((2 * g["x_plane"]) ** 2 / g["far_field_threshold_approx"] - 1) < 0.01
