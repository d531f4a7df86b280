"""Partial-wave reference for the central square potential (Section 4,
Eq. sphericalV), FP64, library-free spherical Bessel functions.

For V = V0 inside r <= a and 0 outside, the phase shift of partial wave l
follows from matching the logarithmic derivative beta_l of the interior
solution at r = a:

    tan d_l = [k j_l'(ka) - beta_l j_l(ka)] / [k y_l'(ka) - beta_l y_l(ka)],
    beta_l = k' j_l'(k'a)/j_l(k'a)   (E > V0, k' = sqrt(2m(E - V0))/hbar)
           = q i_l'(qa)/i_l(qa)      (E < V0, q = sqrt(2m(V0 - E))/hbar)
           = l / a                   (E = V0),

and the amplitude is f(theta) = (1/k) sum_l (2l+1) e^{i d_l} sin d_l P_l(cos theta).
"""
from __future__ import annotations

import math

import numpy as np


def sph_jn(lmax, x):
    """j_0..j_lmax at x > 0 by Miller's downward recurrence
    j_{l-1} = (2l+1)/x j_l - j_{l+1}, normalised by the sum rule."""
    start = lmax + 20 + int(x) + int(2 * math.sqrt(max(x, 1.0)) * 4)
    jp1, j = 0.0, 1e-300
    vals = [0.0] * (start + 1)
    vals[start] = j
    for l in range(start, 0, -1):
        jm1 = (2 * l + 1) / x * j - jp1
        jp1, j = j, jm1
        vals[l - 1] = j
        if abs(j) > 1e250:  # rescale to stay finite
            vals = [v * 1e-250 for v in vals]
            j *= 1e-250
            jp1 *= 1e-250
    # normalise with the sum rule sum_l (2l+1) j_l(x)^2 = 1 (j_0 = sin x / x
    # vanishes at x = n pi, so it cannot fix the scale there); the sign comes
    # from whichever of j_0, j_1 is larger in magnitude
    v = np.array(vals)
    v = v / np.abs(v).max()
    scale = 1.0 / math.sqrt(float(np.sum((2 * np.arange(len(v)) + 1) * v * v)))
    j0 = math.sin(x) / x
    j1 = math.sin(x) / (x * x) - math.cos(x) / x
    if abs(j0) >= abs(j1):
        scale = math.copysign(scale, j0 * v[0])
    else:
        scale = math.copysign(scale, j1 * v[1])
    return v[:lmax + 1] * scale


def sph_yn(lmax, x):
    """y_0..y_lmax by the upward recurrence (stable for y)."""
    y = [0.0] * (lmax + 1)
    y[0] = -math.cos(x) / x
    if lmax >= 1:
        y[1] = -math.cos(x) / x ** 2 - math.sin(x) / x
    for l in range(1, lmax):
        y[l + 1] = (2 * l + 1) / x * y[l] - y[l - 1]
    return np.array(y)


def sph_in(lmax, x):
    """Modified spherical Bessel i_0..i_lmax (first kind), downward recurrence
    i_{l-1} = i_{l+1} + (2l+1)/x i_l normalised with i_0 = sinh x / x."""
    start = lmax + 20 + int(x) + int(8 * math.sqrt(max(x, 1.0)))
    ip1, i = 0.0, 1e-300
    vals = [0.0] * (start + 1)
    vals[start] = i
    for l in range(start, 0, -1):
        im1 = ip1 + (2 * l + 1) / x * i
        ip1, i = i, im1
        vals[l - 1] = i
        if abs(i) > 1e250:
            vals = [v * 1e-250 for v in vals]
            i *= 1e-250
            ip1 *= 1e-250
    scale = (math.sinh(x) / x) / vals[0]
    return np.array(vals[:lmax + 1]) * scale


def _deriv(f, x, sign_l0):
    """f_l' = f_{l-1} - (l+1)/x f_l for l >= 1; f_0' = sign_l0 * f_1
    (-1 for j and y, +1 for i)."""
    lmax = len(f) - 2
    d = np.zeros(lmax + 1)
    d[0] = sign_l0 * f[1]
    for l in range(1, lmax + 1):
        d[l] = f[l - 1] - (l + 1) / x * f[l]
    return d


def phase_shifts(k, a, V0, lmax, hbar=1.0, mass=1.0):
    E = hbar ** 2 * k ** 2 / (2 * mass)
    ka = k * a
    j = sph_jn(lmax + 1, ka)
    y = sph_yn(lmax + 1, ka)
    jd = _deriv(j, ka, -1.0)
    yd = _deriv(y, ka, -1.0)
    if E > V0:
        kp = math.sqrt(2 * mass * (E - V0)) / hbar
        ji = sph_jn(lmax + 1, kp * a)
        jid = _deriv(ji, kp * a, -1.0)
        beta = kp * jid / ji[:lmax + 1]
    elif E < V0:
        q = math.sqrt(2 * mass * (V0 - E)) / hbar
        ii = sph_in(lmax + 1, q * a)
        iid = _deriv(ii, q * a, +1.0)
        beta = q * iid / ii[:lmax + 1]
    else:
        beta = np.arange(lmax + 1) / a
    num = k * jd - beta * j[:lmax + 1]
    den = k * yd - beta * y[:lmax + 1]
    return np.arctan(num / den)  # defined modulo pi, which e^{i d} sin d ignores


def legendre(lmax, x):
    x = np.asarray(x, dtype=np.float64)
    P = [np.ones_like(x), x.copy()]
    for l in range(1, lmax):
        P.append(((2 * l + 1) * x * P[l] - l * P[l - 1]) / (l + 1))
    return np.array(P[:lmax + 1])


def amplitude(k, a, V0, theta, lmax=None, hbar=1.0, mass=1.0):
    """f(theta) of the square potential (physical units of length)."""
    if lmax is None:
        lmax = int(math.ceil(k * a)) + 25
    d = phase_shifts(k, a, V0, lmax, hbar, mass)
    l = np.arange(lmax + 1)
    coef = (2 * l + 1) * np.exp(1j * d) * np.sin(d) / k
    P = legendre(lmax, np.cos(np.asarray(theta, dtype=np.float64)))
    return np.tensordot(coef, P, axes=(0, 0))


def scattered_wave(k, a, V0, r, theta, lmax=None, hbar=1.0, mass=1.0):
    """Exact scattered wave at radius r > a and polar angle theta (from the
    incident direction) for a unit incident wave e^{ikz}.  Outside the
    potential the total field is sum_l (2l+1) i^l e^{i d_l} [cos d_l j_l(kr)
    - sin d_l y_l(kr)] P_l; subtracting the incident sum_l (2l+1) i^l j_l P_l
    leaves
        psi_sc = sum_l (2l+1) i^{l+1} e^{i d_l} sin d_l h_l(kr) P_l(cos theta),
    h_l = j_l + i y_l, whose large-r limit is f(theta) e^{ikr} / r."""
    if lmax is None:
        lmax = int(math.ceil(k * a)) + 25
    d = phase_shifts(k, a, V0, lmax, hbar, mass)
    l = np.arange(lmax + 1)
    x = k * r
    h = np.asarray(sph_jn(lmax, x))[:lmax + 1] + 1j * np.asarray(sph_yn(lmax, x))[:lmax + 1]
    coef = (2 * l + 1) * (1j ** (l + 1)) * np.exp(1j * d) * np.sin(d) * h
    P = legendre(lmax, np.cos(np.asarray(theta, dtype=np.float64)))
    return np.tensordot(coef, P, axes=(0, 0))


def total_cross_section(k, a, V0, lmax=None, hbar=1.0, mass=1.0):
    """sigma = (4 pi / k^2) sum (2l+1) sin^2 d_l."""
    if lmax is None:
        lmax = int(math.ceil(k * a)) + 25
    d = phase_shifts(k, a, V0, lmax, hbar, mass)
    l = np.arange(lmax + 1)
    return 4 * math.pi / k ** 2 * float(np.sum((2 * l + 1) * np.sin(d) ** 2))


def born_amplitude(k, a, V0, theta, hbar=1.0, mass=1.0):
    """First Born approximation for the square potential:
    f_B(q) = -(2m V0 / hbar^2) (sin qa - qa cos qa) / q^3, q = 2k sin(theta/2)."""
    q = 2 * k * np.sin(np.asarray(theta, dtype=np.float64) / 2)
    q = np.where(q == 0, 1e-300, q)
    small = q * a < 1e-3
    val = (np.sin(q * a) - q * a * np.cos(q * a)) / q ** 3
    val = np.where(small, a ** 3 / 3.0, val)
    return -(2 * mass * V0 / hbar ** 2) * val
