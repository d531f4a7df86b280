"""GPU parity of the FDTD variant (Section 2.3: eighth-order stencil, wall
consistency terms, mask) against the FP64 oracle `oracle/fdtd.py`, through
the C ABI.  Tolerances as for the spectral step: one FP32 step within 1e-5 of
max|psi|, runs within 1e-4 rel-L2."""
import math

import numpy as np
import pytest

import synth
from oracle import fdtd as ofdtd

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
