"""GPU parity of the misfit gradient (discrete adjoint with checkpointed
recompute) against the FP64 oracle adjoint, itself pinned by dot-product
tests and finite differences (tests/test_oracle_adjoint.py)."""
import numpy as np
import pytest

import synth
from oracle import adjoint as oadj

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_STEPS = 60


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2403_04053_amd as mod
    return mod


def detector(z, n=5, half=0.6):
    g = np.linspace(-half, half, n)
    X, Y = np.meshgrid(g, g, indexing="xy")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1)


@pytest.fixture(scope="module")
def setup():
    prob, V = synth.tiny(n=(20, 20, 24), P=3, transition=3, v0=1.5, radius_cells=2, steps=N_STEPS, dft=(20, N_STEPS))
    prob = prob.replace(ramp_periods=0.5)
    V = V.astype(np.float32).astype(np.float64)
    pts = np.vstack([detector(1.5), [[0.0, 0.0, -1.5]]])
    target = oadj.intensity(prob, 0.5 * V, pts)
    J, grad = oadj.gradient(prob, V, pts, target)
    return prob, V, pts, target, J, grad


def solver_for(P, prob, V):
    s = P.Solver(prob)
    s.set_potential(V)
    return s


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n_ck", [8, 1, N_STEPS])
def test_gradient_matches_oracle(P, setup, n_ck):
    prob, V, pts, target, J_ref, g_ref = setup
    print(f"adjoint parity: grid {prob.n}, {N_STEPS} steps, {n_ck} checkpoints", flush=True)
    s = solver_for(P, prob, V)
    J = s.misfit(N_STEPS, pts, target, n_checkpoints=n_ck)
    g = s.misfit_gradient().cpu().numpy().astype(np.float64)
    print(f"  J rel err {abs(J - J_ref) / J_ref:.2e}, gradient rel L2 {rel_l2(g, g_ref):.2e}", flush=True)
    assert J == pytest.approx(J_ref, rel=1e-4)
    assert rel_l2(g, g_ref) <= 1e-3
    s.close()


def test_checkpoint_count_does_not_change_the_gradient(P, setup):
    prob, V, pts, target, _, _ = setup
    s = solver_for(P, prob, V)
    out = []
    for n_ck in (1, 7, 13, N_STEPS):
        s.misfit(N_STEPS, pts, target, n_checkpoints=n_ck)
        out.append(s.misfit_gradient().cpu().numpy())
    for g in out[1:]:
        assert rel_l2(g, out[0]) <= 1e-6
    s.close()


def test_backward_restores_the_forward_state_and_repeats(P, setup):
    prob, V, pts, target, _, _ = setup
    s = solver_for(P, prob, V)
    s.misfit(N_STEPS, pts, target, n_checkpoints=6)
    cur, prev = s.psi(0).clone(), s.psi(1).clone()
    ph = s.phasors().clone()
    g1 = s.misfit_gradient()
    assert s.step == N_STEPS
    assert torch.equal(s.psi(0), cur) and torch.equal(s.psi(1), prev)
    assert torch.equal(s.phasors(), ph)
    g2 = s.misfit_gradient()
    assert torch.equal(g1, g2)
    # the forward run equals a plain run of the same steps
    s2 = solver_for(P, prob, V)
    s2.run(N_STEPS)
    assert torch.equal(s2.psi(0), cur)
    s.close()
    s2.close()


def test_state_errors(P, setup):
    prob, V, pts, target, _, _ = setup
    s = solver_for(P, prob, V)
    with pytest.raises(P.PstdError) as e:
        s.misfit_gradient()
    assert e.value.name == "PSTD_ESTATE"
    with pytest.raises(P.PstdError) as e:
        s.misfit(N_STEPS, pts, target, n_checkpoints=0)
    assert e.value.name == "PSTD_EINVAL"
    with pytest.raises(P.PstdError) as e:
        s.misfit(N_STEPS, pts, target, n_checkpoints=N_STEPS + 1)
    assert e.value.name == "PSTD_EINVAL"
    with pytest.raises(P.PstdError) as e:  # no window step before step 10
        s.misfit(10, pts, target)
    assert e.value.name == "PSTD_EINVAL"
    with pytest.raises(P.PstdError) as e:  # a point inside the box
        s.misfit(N_STEPS, np.zeros((1, 3)), np.zeros(1))
    assert e.value.name == "PSTD_EINVAL"
    s.misfit(N_STEPS, pts, target)
    s.run(1)
    with pytest.raises(P.PstdError) as e:
        s.misfit_gradient()
    assert e.value.name == "PSTD_ESTATE"
    s.misfit(N_STEPS, pts, target)
    s.set_potential(V)
    with pytest.raises(P.PstdError) as e:
        s.misfit_gradient()
    assert e.value.name == "PSTD_ESTATE"
    s.close()


def test_autograd_function(P, setup):
    prob, V, pts, target, J_ref, g_ref = setup
    s = P.Solver(prob)
    Vt = torch.tensor(V, dtype=torch.float32, device="cuda", requires_grad=True)
    J = P.FresnelMisfit.apply(Vt, s, N_STEPS, pts, target, 5)
    assert J.dtype == torch.float64 and J.dim() == 0
    (3.0 * J).backward()
    g = Vt.grad.cpu().numpy().astype(np.float64)
    assert float(J) == pytest.approx(J_ref, rel=1e-4)
    assert rel_l2(g, 3.0 * g_ref) <= 1e-3
    s.close()


def test_autograd_refuses_a_replaced_misfit_run(P, setup):
    """Two misfit terms on one solver: the first term's backward would read
    the second run's checkpoints, so it raises; one solver per term works."""
    prob, V, pts, target, _, g_ref = setup
    s = P.Solver(prob)
    V1 = torch.tensor(V, dtype=torch.float32, device="cuda", requires_grad=True)
    J1 = P.FresnelMisfit.apply(V1, s, N_STEPS, pts, target, 5)
    J2 = P.FresnelMisfit.apply(V1 * 0.5, s, N_STEPS, pts, target, 5)
    with pytest.raises(RuntimeError, match="another misfit"):
        (J1 + J2).backward()
    s.close()
    s1, s2 = P.Solver(prob), P.Solver(prob)
    V2 = torch.tensor(V, dtype=torch.float32, device="cuda", requires_grad=True)
    J = P.FresnelMisfit.apply(V2, s1, N_STEPS, pts, target, 5) + P.FresnelMisfit.apply(V2, s2, N_STEPS, pts, target, 5)
    J.backward()
    assert rel_l2(V2.grad.cpu().numpy().astype(np.float64), 2.0 * g_ref) <= 1e-3
    s1.close()
    s2.close()


def test_gradient_matches_gpu_finite_differences(P, setup):
    """Central differences of the GPU misfit itself at core voxels where the
    gradient is large (FP32 forward runs: a large step, 2e-2 E0)."""
    prob, V, pts, target, _, g_ref = setup
    s = solver_for(P, prob, V)
    s.misfit(N_STEPS, pts, target)
    g = s.misfit_gradient().cpu().numpy().astype(np.float64)
    c0, c1 = prob.tfsf[0][1], prob.tfsf[0][2]
    core = np.zeros_like(g, dtype=bool)
    core[c0:c1 + 1, c0:c1 + 1, c0:c1 + 1] = True
    core &= V == 0  # room for the +-eps step below v_max
    order = np.argsort(-np.abs(np.where(core, g, 0.0)).ravel())[:4]
    eps = 2e-2 * prob.k0 ** 2 / 2
    for flat in order:
        idx = np.unravel_index(flat, g.shape)
        Vp = V.copy()
        Vp[idx] += eps
        Vm = V.copy()
        Vm[idx] -= eps
        s.set_potential(Vp)
        Jp = s.misfit(N_STEPS, pts, target)
        s.set_potential(Vm)
        Jm = s.misfit(N_STEPS, pts, target)
        fd = (Jp - Jm) / (2 * eps)
        print(f"  voxel {tuple(int(i) for i in idx)}: adjoint {g[idx]:.6e}, FD {fd:.6e}, oracle {g_ref[idx]:.6e}",
              flush=True)
        assert abs(g[idx] - fd) <= 1e-2 * abs(fd), (idx, g[idx], fd)
    s.close()


# ---------------------------------------------------------------------------
# the voxel-potential workload at its configured length (6000 steps)
# ---------------------------------------------------------------------------

def test_voxel_recipe_full_length_matches_oracle_adjoint(P):
    """The voxel-potential recipe on a 48^3 grid over the configured 6000
    steps (window all, 32 x 32 detector at z = 3.0): J and dJ/dV of the FP32
    GPU path against the FP64 oracle's discrete adjoint, stored by
    golden/make_voxel_adjoint_reference.py (which calls only oracle/)."""
    import math
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "voxel_adjoint_48.npz")
    if not os.path.exists(path):
        pytest.skip("voxel_adjoint_48.npz not written yet")
    ref = np.load(path)
    prob, V0, _ = synth.voxel_potential_48()
    N = prob.n_steps
    assert int(ref["steps"]) == N
    print(f"adjoint vs FP64 oracle: grid {prob.n}, {N} steps", flush=True)
    s = P.Solver(prob)
    s.set_potential(V0.astype(np.float32))
    J = s.misfit(N, ref["points"], ref["target"], math.ceil(math.sqrt(N)))
    g = s.misfit_gradient().cpu().numpy().astype(np.float64)
    eJ = abs(J - float(ref["J"])) / float(ref["J"])
    eg = rel_l2(g, ref["grad"])
    print(f"  J {J:.10e} (oracle {float(ref['J']):.10e}, rel {eJ:.2e}), gradient rel-L2 {eg:.2e}", flush=True)
    assert eJ <= 1e-4
    assert eg <= 1e-3
    s.close()


FD_DELTAS = (0.1, 0.2)           # steps of the central differences, units of E0
FD_CHUNKS = 4                    # the 64 voxels in four tests of 16


@pytest.fixture(scope="module")
def voxel160(P):
    """The 160^3 voxel-potential workload as configured: 6000 steps with the
    window over all of them, 128 x 128 detector points at z = 39.2, sqrt(N)
    checkpoints; target = total-field intensity of the hidden potential; the
    adjoint gradient at the 64 seed-555 core voxels; and the rounding noise
    eps_J of the FP32 misfit, the spread of J over six perturbations of one
    voxel by 1e-7 E0 (linear change below 1e-9 of J)."""
    import math
    prob, V0, Vh = synth.voxel_potential_160()
    N = prob.n_steps
    pts = synth.fresnel_plane(128, prob.h[0], 39.2)
    print(f"adjoint full size: grid {prob.n}, {N} steps, {len(pts)} points", flush=True)
    s = P.Solver(prob)
    s.autotune(reps=5)
    s.set_potential(Vh.astype(np.float32))
    s.run(N)
    psi = s.project(pts).cpu().numpy()
    target = np.abs(np.exp(1j * prob.k0 * pts[:, 2]) + psi) ** 2
    V = V0.astype(np.float32)
    s.set_potential(V)
    J = s.misfit(N, pts, target, math.ceil(math.sqrt(N)))
    g = s.misfit_gradient().cpu().numpy().astype(np.float64)
    vox = synth.fd_voxels(prob, 64, 555)
    E0 = prob.k0 ** 2 / 2

    def J_at(v, d):
        Vp = V.copy()
        Vp[v] += d
        s.set_potential(Vp)
        return s.misfit(N, pts, target, 1)

    js = [J_at(vox[0], k * 1e-7 * E0) for k in range(-3, 3)]
    eps_J = float(np.std(js, ddof=1))
    print(f"  J {J:.10e}, |g| max {np.abs(g).max():.3e}, FP32 noise of J {eps_J:.2e}", flush=True)
    yield dict(prob=prob, s=s, J=J, g=g, vox=vox, J_at=J_at, eps_J=eps_J, E0=E0, gmax=[])
    s.close()


@pytest.mark.parametrize("chunk", range(FD_CHUNKS))
def test_full_size_gradient_finite_differences(P, voxel160, chunk):
    """Central differences of the GPU misfit at 16 of the 64 seed-555 core
    voxels, Richardson-extrapolated from steps of 0.1 and 0.2 E0 (the O(delta^2)
    term cancels; what is left is O(delta^4) and rounding).  Bar, per voxel:
    |g_adj - g_fd| <= 1e-3 max(|g_fd|, 1e-3 max|g_adj|) + 4 sigma, where sigma
    is the rounding noise the extrapolated difference carries from the FP32
    run's measured scatter eps_J of J: each central difference at step d has
    sqrt(2) eps_J / (2 d), and (4 f(d) - f(2d)) / 3 has sqrt(16 + 1/4) / 3 =
    1.344 times that of f(d) (the noise dominates only at voxels whose
    gradient is below about 3 % of the largest)."""
    import math
    d = voxel160
    s, g, vox, E0 = d["s"], d["g"], d["vox"], d["E0"]
    per = len(vox) // FD_CHUNKS
    mine = vox[chunk * per:(chunk + 1) * per]
    gscale = float(np.max(np.abs([g[v] for v in vox])))
    d1, d2 = FD_DELTAS[0] * E0, FD_DELTAS[1] * E0
    sigma = 1.344 * math.sqrt(2.0) * d["eps_J"] / (2 * d1)
    n_bar = 0
    for v in mine:
        f1 = (d["J_at"](v, d1) - d["J_at"](v, -d1)) / (2 * d1)
        f2 = (d["J_at"](v, d2) - d["J_at"](v, -d2)) / (2 * d2)
        fd = (4 * f1 - f2) / 3
        err = abs(g[v] - fd)
        bar = 1e-3 * max(abs(fd), 1e-3 * gscale)
        n_bar += err <= bar
        print(f"  voxel {v}: adjoint {g[v]:+.6e} fd {fd:+.6e} err {err:.2e} (1e-3 bar {bar:.2e}, noise {sigma:.2e})",
              flush=True)
        assert err <= bar + 4 * sigma, (v, g[v], fd, err, bar, sigma)
    print(f"  chunk {chunk}: {n_bar} of {len(mine)} within 1e-3 without the noise allowance", flush=True)
