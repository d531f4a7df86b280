"""FP64 oracle of the near-to-distant-field projection (Sections 3.1-3.2).

Everything is in reduced units (k = 1, lengths x_bar = k0 x).  The scattered
wave at r outside a closed surface S is, Eq. NTDF with G = -exp(ikR)/(4 pi R)
(the 1/(4 pi) that Eq. G omits restored, as Eq. NTDF requires):

    Psi(r) = -(1/4pi) oint ds'. [ grad' Psi + (ik - 1/R) R_hat Psi ] e^{ikR}/R,
    R = r - r', R_hat = R/|R|.

For a box, each face is split into cells between consecutive grid points; the
plane data are replaced by their trigonometric interpolant (Eq. AnBottomPsi)
and the Green function's phase is linearised inside each cell, which yields the
two sinc factors of Eqs. bottomPsi_lm, topPsi_lm, backfrontPsi_mn and
leftrightPsi_ln; Eq. Psi sums all faces.  Sign: + on faces whose outward normal
is -axis (low index), - on the others.

Plane arrays follow the surface-DFT layout: the x-faces are [k][j], the y-faces
[k][i], the z-faces [j][i]; the in-plane axes are called (b, c) with c the slow
one (so x-faces have b = y, c = z).
"""
from __future__ import annotations

import math

import numpy as np

from . import fft as _fft
from .pstd import FACES

# in-plane (b, c) axes per normal axis, c = slow array axis
INPLANE = {0: (1, 2), 1: (0, 2), 2: (0, 1)}


def signed_index(N):
    m = np.arange(N)
    return np.where(m < N // 2, m, m - N)


def sinc(x):
    """Unnormalised sinc, sin(x)/x."""
    return np.sinc(np.asarray(x) / math.pi)


def sinc_taylor_coeffs(x, order):
    """s_p(x), p = 0..order, with sinc(x - alpha) = sum_p s_p(x) alpha^p, i.e.
    s_p = (-1)^p sinc^(p)(x) / p!, from the power series of sinc
    (sum_j (-1)^j x^(2j) / (2j+1)!) differentiated term by term."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((order + 1,) + x.shape)
    J = 40
    for p in range(order + 1):
        acc = np.zeros_like(x)
        for j in range(J):
            if 2 * j < p:
                continue
            c = (-1) ** j * math.factorial(2 * j) / (math.factorial(2 * j - p) * math.factorial(2 * j + 1))
            acc = acc + c * x ** (2 * j - p)
        out[p] = (-1) ** p * acc / math.factorial(p)
    return out


class Box:
    """Geometry of the virtual box: grid sizes n, reduced spacings dxb, face
    indices lo/hi per axis."""

    def __init__(self, n, dxb, lo, hi):
        self.n = tuple(int(v) for v in n)
        self.dxb = np.asarray(dxb, dtype=np.float64)
        self.lo = tuple(lo)
        self.hi = tuple(hi)

    def coord(self, a, i):
        return (i - self.n[a] // 2) * self.dxb[a]

    def face(self, f):
        a, side = FACES[f]
        b, c = INPLANE[a]
        idx = self.lo[a] if side == 0 else self.hi[a]
        sign = 1.0 if side == 0 else -1.0
        return a, b, c, idx, sign

    def cell_centres(self, ax):
        l = np.arange(self.lo[ax], self.hi[ax])
        return self.coord(ax, l) + 0.5 * self.dxb[ax]


def _uvec(box, ax, alpha_or_none, xc):
    """(-1)^b' exp(2 pi i b' xc / L) [sinc(pi b'/N - alpha)] for one cell centre."""
    N = box.n[ax]
    L = N * box.dxb[ax]
    bp = signed_index(N)
    u = np.where(bp % 2 == 0, 1.0, -1.0) * np.exp(2j * math.pi * bp * xc / L)
    if alpha_or_none is not None:
        u = u * sinc(math.pi * bp / N - alpha_or_none)
    return u


def project_direct(box, phi, dphi, points, k=1.0):
    """Eq. Psi by the literal cell sums of Eqs. bottomPsi_lm ... leftrightPsi_ln
    (O(cells * N^2) per point; small planes only).  phi/dphi: per-face plane
    arrays of psi and of its derivative along the face normal."""
    points = np.atleast_2d(np.asarray(points, dtype=np.float64))
    out = np.zeros(len(points), np.complex128)
    for f in range(6):
        a, b, c, idx, sign = box.face(f)
        Fp = _fft.fft2(phi[f])   # [c', b']
        Fd = _fft.fft2(dphi[f])
        Nb, Nc = box.n[b], box.n[c]
        db, dc = box.dxb[b], box.dxb[c]
        xa = box.coord(a, idx)
        xb = box.cell_centres(b)
        xc = box.cell_centres(c)
        pref = sign * db * dc / (4 * math.pi * Nb * Nc)
        for pi_, r in enumerate(points):
            acc = 0.0 + 0.0j
            for m, yc in enumerate(xc):
                for l, yb in enumerate(xb):
                    R = np.zeros(3)
                    R[a] = r[a] - xa
                    R[b] = r[b] - yb
                    R[c] = r[c] - yc
                    Rn = float(np.linalg.norm(R))
                    Rh = R / Rn
                    ub = _uvec(box, b, k * db * Rh[b] / 2, yb)
                    uc = _uvec(box, c, k * dc * Rh[c] / 2, yc)
                    Sd = uc @ Fd @ ub
                    Sp = uc @ Fp @ ub
                    acc += np.exp(1j * k * Rn) / Rn * (Sd + (1j * k - 1.0 / Rn) * Rh[a] * Sp)
            out[pi_] += pref * acc
    return out


class TaylorTables:
    """Q_pq(cell) = sum_{b'c'} u_p(b') F[c', b'] v_q(c'): the spectral sum of
    the cell formula with each sinc expanded to the given order in its shift
    alpha = k d R_hat / 2.  Exact up to the truncation of the two series."""

    def __init__(self, box, phi, dphi, order=8):
        self.box = box
        self.order = order
        self.faces = []
        for f in range(6):
            a, b, c, idx, sign = box.face(f)
            Fp = _fft.fft2(phi[f])
            Fd = _fft.fft2(dphi[f])
            tabs = []
            for ax in (b, c):
                N = box.n[ax]
                L = N * box.dxb[ax]
                bp = signed_index(N)
                s = sinc_taylor_coeffs(math.pi * bp / N, order)  # [p, N]
                xcs = box.cell_centres(ax)
                base = np.where(bp % 2 == 0, 1.0, -1.0)[None, :] * \
                    np.exp(2j * math.pi * xcs[:, None] * bp[None, :] / L)  # [cells, N]
                tabs.append(base[None, :, :] * s[:, None, :])  # [p, cells, N]
            U, Vt = tabs
            # Q[p, q, m, l] = sum_{c', b'} V[q, m, c'] F[c', b'] U[p, l, b']
            Qp = np.einsum("qmc,cb,plb->pqml", Vt, Fp, U, optimize=True)
            Qd = np.einsum("qmc,cb,plb->pqml", Vt, Fd, U, optimize=True)
            self.faces.append((Qp, Qd))

    def project(self, points, k=1.0):
        box = self.box
        points = np.atleast_2d(np.asarray(points, dtype=np.float64))
        out = np.zeros(len(points), np.complex128)
        P = self.order
        for f in range(6):
            a, b, c, idx, sign = box.face(f)
            Qp, Qd = self.faces[f]
            Nb, Nc = box.n[b], box.n[c]
            db, dc = box.dxb[b], box.dxb[c]
            xa = box.coord(a, idx)
            yb = box.cell_centres(b)[None, :]   # [1, L]
            yc = box.cell_centres(c)[:, None]   # [M, 1]
            pref = sign * db * dc / (4 * math.pi * Nb * Nc)
            for i, r in enumerate(points):
                Ra = r[a] - xa
                Rb = r[b] - yb
                Rc = r[c] - yc
                Rn = np.sqrt(Ra * Ra + Rb * Rb + Rc * Rc)
                ab = k * db * (Rb / Rn) / 2
                ac = k * dc * (Rc / Rn) / 2
                Sp = np.zeros(Rn.shape, np.complex128)
                Sd = np.zeros(Rn.shape, np.complex128)
                for p in range(P + 1):
                    for q in range(P + 1):
                        w = ab ** p * ac ** q
                        Sp = Sp + w * Qp[p, q]
                        Sd = Sd + w * Qd[p, q]
                term = np.exp(1j * k * Rn) / Rn * (Sd + (1j * k - 1.0 / Rn) * (Ra / Rn) * Sp)
                out[i] += pref * term.sum()
        return out


def far_field_direct(box, phi, dphi, dirs, k=1.0):
    """Far-field amplitude f(r_hat) = lim r e^{-ikr} Psi(r) (Eq.
    FDTDfarfieldapprox applied to the cell formula): e^{ikR}/R ->
    e^{-ik r_hat . r_cell}, (ik - 1/R) R_hat -> ik r_hat, sinc shifts with r_hat.
    Literal cell sums (small planes only)."""
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    out = np.zeros(len(dirs), np.complex128)
    for f in range(6):
        a, b, c, idx, sign = box.face(f)
        Fp = _fft.fft2(phi[f])
        Fd = _fft.fft2(dphi[f])
        Nb, Nc = box.n[b], box.n[c]
        db, dc = box.dxb[b], box.dxb[c]
        xa = box.coord(a, idx)
        pref = sign * db * dc / (4 * math.pi * Nb * Nc)
        for di, rh in enumerate(dirs):
            acc = 0.0 + 0.0j
            for yc in box.cell_centres(c):
                for yb in box.cell_centres(b):
                    ub = _uvec(box, b, k * db * rh[b] / 2, yb)
                    uc = _uvec(box, c, k * dc * rh[c] / 2, yc)
                    ph = np.exp(-1j * k * (rh[a] * xa + rh[b] * yb + rh[c] * yc))
                    acc += ph * (uc @ Fd @ ub + 1j * k * rh[a] * (uc @ Fp @ ub))
            out[di] += pref * acc
    return out


def far_field(box, phi, dphi, dirs, k=1.0):
    """Same quantity as far_field_direct with the cell sums factored: in the
    far-field limit each cell term is a product of a b-factor and a c-factor,
    so sum_cells = g_c^T F g_b with g_b(b') = (-1)^b' sinc(pi b'/N - k d r_b/2)
    sum_l exp(i (2 pi b'/L - k r_b) x_l)."""
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    out = np.zeros(len(dirs), np.complex128)
    for f in range(6):
        a, b, c, idx, sign = box.face(f)
        Fp = _fft.fft2(phi[f])
        Fd = _fft.fft2(dphi[f])
        Nb, Nc = box.n[b], box.n[c]
        db, dc = box.dxb[b], box.dxb[c]
        xa = box.coord(a, idx)
        pref = sign * db * dc / (4 * math.pi * Nb * Nc)

        def g(ax, rcomp):
            N = box.n[ax]
            L = N * box.dxb[ax]
            bp = signed_index(N)
            xcs = box.cell_centres(ax)
            geo = np.exp(1j * (2 * math.pi * bp[None, :] / L - k * rcomp) * xcs[:, None]).sum(axis=0)
            return np.where(bp % 2 == 0, 1.0, -1.0) * sinc(math.pi * bp / N - k * box.dxb[ax] * rcomp / 2) * geo

        for di, rh in enumerate(dirs):
            gb = g(b, rh[b])
            gc = g(c, rh[c])
            ph = np.exp(-1j * k * rh[a] * xa)
            out[di] += pref * ph * (gc @ Fd @ gb + 1j * k * rh[a] * (gc @ Fp @ gb))
    return out


def sphere_directions(n_theta=181, n_phi=360):
    """r_hat on the theta = 0..180 deg, phi = 0..359 deg (1 deg) grid, theta-major."""
    th = np.deg2rad(np.linspace(0.0, 180.0, n_theta))
    ph = np.deg2rad(np.arange(n_phi) * (360.0 / n_phi))
    T, P = np.meshgrid(th, ph, indexing="ij")
    return np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=-1).reshape(-1, 3), th, ph
