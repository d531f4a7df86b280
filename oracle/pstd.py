"""FP64 oracle of the PSTD internal model (Sections 2.1-2.5 and 3.3).

Everything is in the paper's reduced units (Section 2.5, Eq. rescaled_var):
x_bar = k0 x, tau = E0 t / hbar, E0 = hbar^2 k0^2 / 2m, so the central wave has
|k_bar| = 1 and angular frequency 1.  Arrays are [k][j][i] (x fastest); grid
point i of an axis of N points and spacing dxb sits at x_bar = (i - N/2) dxb.

Readings where the paper is silent (each also listed in the design notes):
  * the absorber depth d counts cells from the outermost grid point and gamma
    acts only for d < width;
  * the taper walls use grid indices y0 < y1 <= y2 < y3 and analytic
    derivatives of xi;
  * the source carries no eta factor unless eta_on_source is set;
  * the incident wave is switched on with the temporal ramp R(tau) =
    xi(min(tau / tau_r, 1)), tau_r = 2 pi * ramp_periods;
  * phasors are normalised by the incident phasor at the coordinate origin.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import fft as _fft

# numpy axis holding physical axis a (x=0, y=1, z=2) in a [k][j][i] array
NPAX = (2, 1, 0)


# ----------------------------------------------------------------------------
# scalars: reduced units, stability, phase-velocity correction
# ----------------------------------------------------------------------------

def central_energy(prob):
    """E0 = hbar^2 k0^2 / 2m (Section 2.5)."""
    return prob.hbar ** 2 * prob.k0 ** 2 / (2.0 * prob.mass)


def dxbar(prob):
    """Reduced grid spacings, x_bar = x / lambdabar0 = k0 x (Eq. rescaled_var)."""
    return np.array([prob.k0 * h for h in prob.h], dtype=np.float64)


def critical_dtau(dxb, vmax_over_E0):
    """Largest stable reduced step, Eq. dtau_stability:
    dtau <= [pi^2 sum_a 1/dxb_a^2 + |V|max/E0]^-1."""
    return 1.0 / (math.pi ** 2 * float(np.sum(1.0 / np.asarray(dxb) ** 2)) + vmax_over_E0)


def critical_dt(prob, vmax):
    """The same bound in physical time, Eq. PSTDstability:
    dt <= hbar / (hbar^2 pi^2/2m sum 1/dx^2 + |V|max)."""
    lam = prob.hbar ** 2 * math.pi ** 2 / (2 * prob.mass) * sum(1.0 / h ** 2 for h in prob.h)
    return prob.hbar / (lam + vmax)


def dtau_of(prob):
    """Reduced step: the given dt, or 0.9 of the critical one for the largest
    |v| of the model, max(v_max / E0, the real part of the absorbing potential
    where the layers of all axes overlap); V vanishes in the layers, so the
    two never add."""
    E0 = central_energy(prob)
    if prob.dt > 0:
        return E0 * prob.dt / prob.hbar
    return 0.9 * critical_dtau(dxbar(prob), max(prob.v_max / E0, absorber_real_max(prob)))


def eta_of(dtau):
    """Phase-velocity correction eta = sinc(E0 dt / hbar) = sin(dtau)/dtau,
    unnormalised sinc (Eq. numdis2 with E = E0)."""
    return math.sin(dtau) / dtau


# ----------------------------------------------------------------------------
# 1D tables
# ----------------------------------------------------------------------------

def kbar(N, dxb):
    """Spectral wavenumbers of an N-point axis with the FFT index m shifted
    back to m' in [-N/2, N/2) (note under Eq. PSTDupdating)."""
    m = np.arange(N)
    mp = np.where(m < N // 2, m, m - N)
    return 2.0 * math.pi * mp / (N * dxb)


def xi(rho):
    """Optimal taper, Eq. xi."""
    rho = np.asarray(rho, dtype=np.float64)
    return rho - 2.0 / (3.0 * math.pi) * np.sin(2 * math.pi * rho) \
        + 1.0 / (12.0 * math.pi) * np.sin(4 * math.pi * rho)


def dxi(rho):
    """d xi / d rho, differentiated from Eq. xi."""
    rho = np.asarray(rho, dtype=np.float64)
    return 1.0 - 4.0 / 3.0 * np.cos(2 * math.pi * rho) + 1.0 / 3.0 * np.cos(4 * math.pi * rho)


def d2xi(rho):
    """d^2 xi / d rho^2, differentiated from Eq. xi."""
    rho = np.asarray(rho, dtype=np.float64)
    return 8.0 * math.pi / 3.0 * np.sin(2 * math.pi * rho) \
        - 4.0 * math.pi / 3.0 * np.sin(4 * math.pi * rho)


def zeta_1d(N, y, dxb):
    """One factor of the separable taper, Eq. zeta_y, with its first and
    second derivatives with respect to the reduced coordinate."""
    y0, y1, y2, y3 = y
    z = np.zeros(N)
    dz = np.zeros(N)
    d2z = np.zeros(N)
    for i in range(N):
        if i <= y0 or i >= y3:
            continue
        if y1 <= i <= y2:
            z[i] = 1.0
        elif i < y1:
            w = (y1 - y0) * dxb
            rho = (i - y0) / (y1 - y0)
            z[i] = xi(rho)
            dz[i] = dxi(rho) / w
            d2z[i] = d2xi(rho) / w ** 2
        else:
            w = (y3 - y2) * dxb
            rho = (i - y2) / (y3 - y2)
            z[i] = 1.0 - xi(rho)
            dz[i] = -dxi(rho) / w
            d2z[i] = -d2xi(rho) / w ** 2
    return z, dz, d2z


def absorber_gamma(N, width, U0, alpha):
    """Poschl-Teller absorption rate per grid index, Eq. Poshcl-Teller:
    gamma(d) = U0 / cosh^2(alpha d), d = cells from the outermost grid point,
    inside the absorbing layer only."""
    g = np.zeros(N)
    for i in range(N):
        d = min(i, N - 1 - i)
        if d < width:
            g[i] = U0 / math.cosh(alpha * d) ** 2
    return g


def mask_1d(N, width, U0, alpha, dtau):
    """exp(-gamma dtau) along one axis (one factor of Eq. Gamma)."""
    return np.exp(-absorber_gamma(N, width, U0, alpha) * dtau)


def absorber_real(N, width, UR, alphaR):
    """Real part of a complex absorbing potential along one axis (the remark
    after Eq. Poshcl-Teller: the absorbing potential may be complex as long as
    its imaginary part, here -gamma, stays non-positive).  Same shape as
    gamma, in units of E0: w(d) = UR / cosh^2(alphaR d) inside the layer.
    It enters the step like v, summed over the axes."""
    return absorber_gamma(N, width, UR, alphaR)


def absorber_alpha_real(prob):
    """Decay of the real part: abc_alphaR, or abc_alpha when that is 0."""
    a = getattr(prob, "abc_alphaR", 0.0)
    return a if a > 0 else prob.abc_alpha


def absorber_real_max(prob):
    """max |sum_a w_a| over the grid: at the corners where the layers of all
    axes with a layer meet, |UR| per such axis."""
    UR = getattr(prob, "abc_UR", 0.0)
    return abs(UR) * sum(1 for a in range(3) if prob.abc_cells[a] > 0)


def khat(theta, phi):
    """Unit incident direction, Eq. khat."""
    return np.array([math.sin(theta) * math.cos(phi),
                     math.sin(theta) * math.sin(phi),
                     math.cos(theta)])


def o_inc(kh, box_lo, box_hi):
    """Grid indices of the corner of the taper box that the incident front
    reaches first (Eq. Oinc, read by the sign of each component of k_hat:
    the low index when k_hat_a >= 0, else the high one)."""
    return tuple(box_lo[a] if kh[a] >= 0 else box_hi[a] for a in range(3))


def ramp(tau, tau_r):
    """Temporal switch-on R(tau) = xi(min(tau/tau_r, 1)); R = 1 when tau_r = 0."""
    if tau_r <= 0:
        return 1.0
    return float(xi(min(max(tau / tau_r, 0.0), 1.0)))


def coords(N, dxb):
    return (np.arange(N) - N // 2) * dxb


# ----------------------------------------------------------------------------
# the model
# ----------------------------------------------------------------------------

@dataclass
class Model:
    prob: object
    dtau: float
    eta: float
    dxb: np.ndarray
    v: np.ndarray          # V / E0 plus the absorber's real part, [k][j][i]
    kb2: list              # per axis kbar^2
    kb: list               # per axis kbar
    Gamma: np.ndarray      # 3D mask, Eq. Gamma
    zeta: np.ndarray       # 3D taper
    grad_zeta: list        # 3 arrays
    lap_zeta: np.ndarray
    phase: np.ndarray      # exp(i k_hat . r_bar)
    kh: np.ndarray
    tau_r: float


def _bcast(vec, a):
    shape = [1, 1, 1]
    shape[NPAX[a]] = vec.shape[0]
    return vec.reshape(shape)


def absorber_real_3d(prob):
    """sum_a w_a(d_a) broadcast to [k][j][i] (0.0 without a real part)."""
    UR = getattr(prob, "abc_UR", 0.0)
    if UR == 0.0:
        return 0.0
    aR = absorber_alpha_real(prob)
    w = np.zeros((prob.n[2], prob.n[1], prob.n[0]))
    for a in range(3):
        w = w + _bcast(absorber_real(prob.n[a], prob.abc_cells[a], UR, aR), a)
    return w


def build(prob, V):
    """All step-invariant quantities of Eq. PSTDupdating (plain 3D arrays)."""
    E0 = central_energy(prob)
    dxb = dxbar(prob)
    dtau = dtau_of(prob)
    eta = eta_of(dtau)
    n = prob.n
    v = np.asarray(V, dtype=np.float64) / E0
    v = v + absorber_real_3d(prob)
    kb = [kbar(n[a], dxb[a]) for a in range(3)]
    kb2 = [k * k for k in kb]
    G = np.ones((n[2], n[1], n[0]))
    for a in range(3):
        G = G * _bcast(mask_1d(n[a], prob.abc_cells[a], prob.abc_U0, prob.abc_alpha, dtau), a)
    zs = [zeta_1d(n[a], prob.tfsf[a], dxb[a]) for a in range(3)]
    Z = [_bcast(zs[a][0], a) for a in range(3)]
    dZ = [_bcast(zs[a][1], a) for a in range(3)]
    d2Z = [_bcast(zs[a][2], a) for a in range(3)]
    zeta = Z[0] * Z[1] * Z[2]
    grad = [dZ[0] * Z[1] * Z[2], Z[0] * dZ[1] * Z[2], Z[0] * Z[1] * dZ[2]]
    lap = d2Z[0] * Z[1] * Z[2] + Z[0] * d2Z[1] * Z[2] + Z[0] * Z[1] * d2Z[2]
    kh = khat(prob.theta, prob.phi)
    X = [_bcast(coords(n[a], dxb[a]), a) for a in range(3)]
    phase = np.exp(1j * (kh[0] * X[0] + kh[1] * X[1] + kh[2] * X[2]))
    tau_r = 2 * math.pi * prob.ramp_periods
    return Model(prob, dtau, eta, dxb, v, kb2, kb, G, zeta * np.ones_like(G),
                 [g * np.ones_like(G) for g in grad], lap * np.ones_like(G),
                 phase * np.ones_like(G, dtype=np.complex128), kh, tau_r)


def check_potential(model, tol=0.0):
    """(zeta - 1) V = 0 everywhere (Section 2.2.2): V must vanish wherever the
    taper is below 1 (the absorber's real part is not part of V)."""
    V = model.v - absorber_real_3d(model.prob)
    return bool(np.all(np.abs((model.zeta - 1.0) * V) <= tol))


def incident(model, n):
    """psi_inc and grad psi_inc at step n: R(tau_n) exp(i(k_hat.r - tau_n)),
    grad = i k_hat psi_inc (|k_bar| = 1 in reduced units)."""
    tau = n * model.dtau
    amp = ramp(tau, model.tau_r) * np.exp(-1j * tau)
    psi = amp * model.phase
    grad = [1j * model.kh[a] * psi for a in range(3)]
    return psi, grad


def source(model, n):
    """Transition-layer source of Eq. dimlesstildeSchrodinger:
    lap(zeta) psi_inc + 2 grad(zeta) . grad(psi_inc)."""
    psi, grad = incident(model, n)
    return model.lap_zeta * psi + 2.0 * (model.grad_zeta[0] * grad[0]
                                         + model.grad_zeta[1] * grad[1]
                                         + model.grad_zeta[2] * grad[2])


def kinetic(model, psi):
    """sum_a F_a^-1[ kbar_a^2 F_a[psi] ] (the bracket of Eq. PSTDupdating)."""
    out = np.zeros_like(psi, dtype=np.complex128)
    for a in range(3):
        ax = NPAX[a]
        out += _fft.ifft(_bcast(model.kb2[a], a) * _fft.fft(psi, axis=ax), axis=ax)
    return out


def derivative(model, psi, a):
    """Spectral first derivative along axis a, F^-1[i kbar F[psi]], the
    Nyquist index kept at m' = -N/2 as in Eq. pstd_dpsiinc."""
    ax = NPAX[a]
    return _fft.ifft(1j * _bcast(model.kb[a], a) * _fft.fft(psi, axis=ax), axis=ax)


def step(model, psi_prev, psi_cur, n, with_source=True):
    """One leapfrog step, Eq. PSTDupdating (with the mask of Eq. expmask):
    psi^{n+1} = Gamma { psi^{n-1} - 2i eta dtau K psi^n - 2i dtau v psi^n
                        - 2i dtau S^n }."""
    dt = model.dtau
    rhs = psi_prev - 2j * model.eta * dt * kinetic(model, psi_cur) - 2j * dt * model.v * psi_cur
    if with_source:
        S = source(model, n)
        if model.prob.eta_on_source:
            S = model.eta * S
        rhs = rhs - 2j * dt * S
    return model.Gamma * rhs


# ----------------------------------------------------------------------------
# running surface DFT (Section 3.3)
# ----------------------------------------------------------------------------

FACES = ((0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1))  # (axis, side)


def face_index(prob, f):
    a, side = FACES[f]
    return prob.surf_lo[a] if side == 0 else prob.surf_hi[a]


def plane(arr, a, idx):
    """Full cross-section of a [k][j][i] array at index idx along axis a:
    x -> [k][j], y -> [k][i], z -> [j][i]."""
    return np.take(arr, idx, axis=NPAX[a])


class SurfaceDFT:
    """Eqs. psiphasor and dpsiphasor: Phi += exp(i omega n dt) psi^n on the six
    virtual planes, for psi and its normal derivative (omega = E0/hbar, so the
    weight is exp(i tau_n)); plus the incident phasor at the origin,
    Eq. incpsiphasor."""

    def __init__(self, model):
        self.m = model
        p = model.prob
        self.phi = [np.zeros(plane(model.v, FACES[f][0], 0).shape, np.complex128) for f in range(6)]
        self.dphi = [np.zeros_like(x) for x in self.phi]
        self.inc = 0.0 + 0.0j
        self.count = 0

    def accumulate(self, psi, n):
        m = self.m
        tau = n * m.dtau
        w = np.exp(1j * tau)
        ders = {}
        for f in range(6):
            a, _ = FACES[f]
            if a not in ders:
                ders[a] = derivative(m, psi, a)
            idx = face_index(m.prob, f)
            self.phi[f] += w * plane(psi, a, idx)
            self.dphi[f] += w * plane(ders[a], a, idx)
        self.inc += w * ramp(tau, m.tau_r) * np.exp(-1j * tau)
        self.count += 1

    def normalized(self):
        """Eqs. scaledphsiphasor / scaleddpsiphasor (normalised at the origin)."""
        return ([x / self.inc for x in self.phi], [x / self.inc for x in self.dphi])


def run(prob, V, n_steps=None, state=None, start=0, dft=True):
    """March Eq. PSTDupdating from psi^{-1} = psi^0 = 0 (or a given state) and
    accumulate the surface DFT over [dft_begin, dft_end)."""
    model = build(prob, V)
    n_steps = prob.n_steps if n_steps is None else n_steps
    shape = (prob.n[2], prob.n[1], prob.n[0])
    if state is None:
        prev = np.zeros(shape, np.complex128)
        cur = np.zeros(shape, np.complex128)
    else:
        prev, cur = (np.array(s, dtype=np.complex128) for s in state)
    sd = SurfaceDFT(model)
    for n in range(start, start + n_steps):
        if dft and prob.dft_begin <= n < prob.dft_end:
            sd.accumulate(cur, n)
        prev, cur = cur, step(model, prev, cur, n)
    return model, prev, cur, sd


def step_at(model, psi_prev, psi_cur, n, points):
    """psi^{n+1} of Eq. PSTDupdating at selected cells only, evaluating each
    axis term on the single pencil through the cell.  points: iterable of
    (i, j, k).  Returns a complex array."""
    out = []
    dt = model.dtau
    for (i, j, k) in points:
        kin = 0.0 + 0.0j
        pen = (psi_cur[k, j, :], psi_cur[k, :, i], psi_cur[:, j, i])
        pos = (i, j, k)
        for a in range(3):
            kin += _fft.ifft(model.kb2[a] * _fft.fft(pen[a]))[pos[a]]
        tau = n * dt
        amp = ramp(tau, model.tau_r) * np.exp(-1j * tau)
        ph = model.phase[k, j, i]
        pinc = amp * ph
        S = model.lap_zeta[k, j, i] * pinc + 2.0 * sum(
            model.grad_zeta[a][k, j, i] * 1j * model.kh[a] * pinc for a in range(3))
        if model.prob.eta_on_source:
            S *= model.eta
        rhs = psi_prev[k, j, i] - 2j * model.eta * dt * kin - 2j * dt * model.v[k, j, i] * psi_cur[k, j, i] \
            - 2j * dt * S
        out.append(model.Gamma[k, j, i] * rhs)
    return np.array(out)
