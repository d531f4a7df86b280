"""GPU parity of the FDTD variant (Section 2.2.1, bound of Section 2.3.1: eighth-order stencil, wall
consistency terms, mask) against the FP64 oracle `oracle/fdtd.py`, through
the C ABI, and its far field through the spherical surface.  Tolerances as
for the spectral step: one FP32 step within 1e-5 of max|psi|, runs and
phasors within 1e-4 rel-L2."""
import math

import numpy as np
import pytest

import synth
from oracle import fdtd as ofdtd
from oracle import partial_waves as pw
from oracle import pstd as opstd
from oracle import sphere as osph

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


def fdtd_problem(n, P_=4, transition=2, theta=0.6, phi=2.0, steps=200, v0=0.5, radius=3):
    prob, V = synth.tiny(n=n, P=P_, transition=transition, v0=v0, radius_cells=radius, steps=steps,
                         theta=theta, phi=phi, dft=(0, 0))
    return prob.replace(scheme=1, ramp_periods=0.5), V.astype(np.float32).astype(np.float64)


# cubic; ragged in every direction of the 32 x 8 tile and 16-plane chunks
CASES = {"cube": (24, 24, 32), "ragged": (40, 36, 28)}


@pytest.mark.parametrize("case", list(CASES))
def test_fdtd_single_step_matches_oracle(P, case):
    n = CASES[case]
    prob, V = fdtd_problem(n)
    print(f"FDTD single step, {case}: grid {n}", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    prev = synth.random_state(n, 11).astype(np.complex64)
    cur = synth.random_state(n, 12).astype(np.complex64)
    step = 37
    s.set_state(prev, cur, step)
    s.run(1)
    got = s.psi(0).cpu().numpy()
    m = ofdtd.build(prob, V)
    ref = ofdtd.step(m, prev.astype(np.complex128), cur.astype(np.complex128), step)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("  max err / max|psi|", err, flush=True)
    assert err < 1e-5
    s.close()


@pytest.mark.parametrize("case", list(CASES))
def test_fdtd_run_from_rest_matches_oracle(P, case):
    """200 steps from rest: incident wave through the walls, barrier, mask."""
    n = CASES[case]
    prob, V = fdtd_problem(n)
    print(f"FDTD run, {case}: grid {n}", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    s.run(prob.n_steps)
    got = s.psi(0).cpu().numpy()
    _, _, ref = ofdtd.run(prob, V)
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("  rel-L2", rel, flush=True)
    assert rel < 1e-4
    s.close()


def test_fdtd_walls_hold_the_incident_wave(P):
    """Started exactly after the ramp (psi = T psi_inc at two levels, T the
    total-field box), the walls keep the incident wave in the box and the
    scattered-field region empty, to FP32 rounding, over 300 steps: the
    consistency terms of all six walls and their corners, at the discrete
    frequency, on the GPU."""
    n = (32, 32, 32)
    prob, V = fdtd_problem(n, P_=4, transition=2, theta=0.9, phi=0.4, steps=400, v0=0.0, radius=0)
    m = ofdtd.build(prob, V)
    T = ofdtd.total_field_mask(m)
    n0 = int(m.tau_r / m.dtau) + 2
    s = P.Solver(prob)
    s.set_potential(V)
    s.set_state((T * ofdtd.incident(m, n0 - 1)).astype(np.complex64),
                (T * ofdtd.incident(m, n0)).astype(np.complex64), n0)
    s.run(300)
    got = s.psi(0).cpu().numpy()
    want = T * ofdtd.incident(m, n0 + 300)
    err_box = np.abs(got - want).max()
    err_sf = (np.abs(got) * (1 - T)).max()
    print("  box |psi - psi_inc| max", err_box, " scattered region max", err_sf, flush=True)
    assert err_box < 1e-4 and err_sf < 1e-4
    s.close()


@pytest.mark.parametrize("n", [160, 288])
def test_fdtd_full_size_single_step(P, n):
    """One step of the benchmark's grid (160^3 and 288^3 square barrier) from
    seeded random states, every cell against the oracle."""
    prob, V = synth.square_barrier_160(n_fft=n)
    prob = prob.replace(scheme=1, dft_begin=0, dft_end=0)
    V = V.astype(np.float32).astype(np.float64)
    print(f"FDTD full-size single step: grid {prob.n}", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    s.autotune(reps=3)
    prev = synth.random_state(prob.n, 21).astype(np.complex64)
    cur = synth.random_state(prob.n, 22).astype(np.complex64)
    step = 300  # inside the ramp: the wall terms carry a fraction of the wave
    s.set_state(prev, cur, step)
    s.run(1)
    got = s.psi(0).cpu().numpy()
    s.close()
    ref = ofdtd.step(ofdtd.build(prob, V), prev.astype(np.complex128), cur.astype(np.complex128), step)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("  max err / max|psi|", err, flush=True)
    assert err < 1e-5


def sphere_problem(v0=1.0, theta=0.5, phi=0.8):
    """48^3 at 8 points per wavelength, total-field box 19..29, a barrier of
    radius 3 cells, a sphere of radius 0.95 (9.5 cells) around the box whose
    shell crosses its walls."""
    h = 0.1
    k0 = 2 * math.pi / (8 * h)
    E0 = k0 * k0 / 2
    alpha = 1.0
    prob = synth.Problem(n=(48, 48, 48), h=(h,) * 3, k0=k0, theta=theta, phi=phi, abc_cells=(4,) * 3,
                         abc_alpha=alpha, abc_U0=synth.paper_u0(alpha, k0 * h, 4), tfsf=((16, 19, 29, 32),) * 3,
                         v_max=max(abs(v0), 1e-9) * E0, ramp_periods=0.5, n_steps=160, dft_begin=80, dft_end=160,
                         surf_lo=(14,) * 3, surf_hi=(34,) * 3, surface_kind=1, sphere_radius=0.95,
                         sphere_nodes=(16, 32), scheme=1)
    V = np.zeros((48, 48, 48))
    x = np.arange(48) - 24
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    V[X * X + Y * Y + Z * Z <= 9] = v0 * E0
    return prob, V.astype(np.float32).astype(np.float64)


def test_fdtd_sphere_phasors_match_oracle(P):
    """The shell DFT at the discrete frequency with the incident part T
    psi_inc removed, interpolated to the nodes, against the oracle."""
    prob, V = sphere_problem()
    print(f"FDTD sphere phasors: grid {prob.n}", flush=True)
    s = P.Solver(prob)
    s.set_potential(V)
    s.run(prob.n_steps)
    v, d = (x.cpu().numpy() for x in s.sphere_phasors())
    s.close()
    sph = osph.Sphere(prob, prob.sphere_radius, n_theta=16, n_phi=32)
    _, _, sd = ofdtd.run_sphere(prob, V, sph)
    ref_v, ref_d = sph.node_values(sd.normalized())
    ev = np.linalg.norm(v - ref_v) / np.linalg.norm(ref_v)
    ed = np.linalg.norm(d - ref_d) / np.linalg.norm(ref_d)
    print(f"  rel-L2: psi {ev:.2e}, d psi/dn {ed:.2e}", flush=True)
    assert ev < 1e-4 and ed < 1e-4


def test_fdtd_validation(P):
    prob, _ = sphere_problem()
    for bad in (dict(surface_kind=0), dict(sub_core=(16, 0, 0), sub_halo=8, sub_taper=3)):
        with pytest.raises(P.PstdError) as e:
            P.Solver(prob.replace(**bad))
        assert e.value.name == "PSTD_EUNSUPPORTED"
    s = P.Solver(prob)
    with pytest.raises(P.PstdError) as e:
        s.misfit(prob.n_steps, np.array([[0.0, 0.0, 3.0]]), np.ones(1))
    assert e.value.name == "PSTD_EUNSUPPORTED"
    s.close()


def test_fdtd_square_barrier_far_field(P):
    """The 160^3 square-barrier workload advanced by the FDTD step over the
    same physical time as the spectral run (the DFT window the last 4
    periods at W), far field from the sphere of radius 5 against the
    partial-wave series and against the spectral solve."""
    base, V = synth.square_barrier_160()
    # the barrier lies inside the total-field box 56..104 of every axis
    lo, hi = base.tfsf[0][1], base.tfsf[0][2]
    inside = np.zeros(base.n[0], bool)
    inside[lo:hi + 1] = True
    assert np.abs(V[~inside, :, :]).max() == 0 and np.abs(V[:, ~inside, :]).max() == 0
    assert np.abs(V[:, :, ~inside]).max() == 0
    sph = dict(surface_kind=1, sphere_radius=5.0, sphere_nodes=(64, 128))
    fd = base.replace(scheme=1, **sph)
    dt_p, dt_f = opstd.dtau_of(base), ofdtd.dtau_of(fd)
    W = ofdtd.discrete_frequency(opstd.khat(fd.theta, fd.phi), opstd.dxbar(fd), dt_f)
    steps = int(round(base.n_steps * dt_p / dt_f))
    win = int(round(4 * 2 * math.pi / (W * dt_f)))
    fd = fd.replace(n_steps=steps, dft_begin=steps - win, dft_end=steps)
    print(f"FDTD square barrier: grid {fd.n}, {steps} steps, window {win}", flush=True)
    th = np.deg2rad(np.arange(0, 181, 3.0))
    ph = np.deg2rad(np.arange(0, 360, 30.0))
    T, F = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1).reshape(-1, 3)
    out = {}
    for name, prob in (("fdtd", fd), ("pstd", base.replace(**sph))):
        s = P.Solver(prob)
        s.set_potential(V)
        s.run(prob.n_steps)
        out[name] = s.far_field(d).cpu().numpy().reshape(T.shape)
        s.close()
    ref = pw.amplitude(base.k0, 2.4, 0.5 * base.k0 ** 2 / 2, th)[:, None] * np.ones_like(F)
    w = np.sin(T) + 1e-3

    def rel(a, b):
        return math.sqrt(np.sum(w * np.abs(a - b) ** 2) / np.sum(w * np.abs(b) ** 2))
    r_fp, r_sp, r_fs = rel(out["fdtd"], ref), rel(out["pstd"], ref), rel(out["fdtd"], out["pstd"])
    print(f"  vs partial waves: FDTD {r_fp:.4f}, PSTD {r_sp:.4f}; FDTD vs PSTD {r_fs:.4f}", flush=True)
    assert r_fp < 0.05
