"""Python binding of libpstd (the C ABI in include/pstd.h).

Argument marshalling only: every step of the method runs in the HIP library.
Functions keep the C names; device buffers are passed as torch tensors (or raw
integer addresses), streams as torch streams (or raw hipStream_t integers).
Importing the package fails loudly when libpstd.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "PstdError", "pstd_problem", "problem_from", "lib",
    "pstd_problem_init_defaults", "pstd_critical_dt", "pstd_reduced_step", "pstd_create",
    "pstd_set_potential", "pstd_set_state", "pstd_run", "pstd_run_timed", "pstd_step_index",
    "pstd_get_psi", "pstd_surface_size", "pstd_get_surface_phasors", "pstd_project",
    "pstd_far_field", "pstd_set_pulse", "pstd_get_surface_phasors_k", "pstd_get_sphere_phasors_k", "pstd_project_k", "pstd_far_field_k",
    "pstd_pass_time", "pstd_check_state", "pstd_check_state_noalloc", "pstd_sphere_size", "pstd_get_sphere_phasors", "pstd_state_size", "pstd_save_state", "pstd_load_state", "pstd_misfit_forward", "pstd_misfit_backward", "FresnelMisfit", "pstd_destroy", "pstd_autotune", "pstd_tile_info", "pstd_set_tile",
    "pstd_tile_variants", "pstd_batch_create",
    "pstd_batch_size", "pstd_batch_solver", "pstd_batch_set_potential", "pstd_batch_autotune",
    "pstd_batch_run", "pstd_batch_destroy", "pstd_batch_last_error", "Batch", "pstd_status_string", "pstd_last_error", "Solver",
    "EXPORTED",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpstd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2403_04053_amd/build.py`")

# torch ships its own HIP runtime under the same soname as the system one
# libpstd.so links against; whichever is loaded first serves the process.
# Loading torch first makes the library and torch share torch's runtime (two
# runtimes in one process do not see the same devices).
import torch as _torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

STATUS = {0: "PSTD_OK", 1: "PSTD_EINVAL", 2: "PSTD_EUNSTABLE", 3: "PSTD_ENONFINITE",
          4: "PSTD_ENOMEM", 5: "PSTD_EHIP", 6: "PSTD_ESTATE", 7: "PSTD_EUNSUPPORTED"}


class PstdError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


class pstd_problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("h", ctypes.c_double * 3),
        ("hbar", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("k0", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("phi", ctypes.c_double),
        ("abc_cells", ctypes.c_int32 * 3),
        ("abc_U0", ctypes.c_double),
        ("abc_alpha", ctypes.c_double),
        ("tfsf", (ctypes.c_int32 * 4) * 3),
        ("v_max", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("force_dt", ctypes.c_int32),
        ("ramp_periods", ctypes.c_double),
        ("dft_begin", ctypes.c_int64),
        ("dft_end", ctypes.c_int64),
        ("surf_lo", ctypes.c_int32 * 3),
        ("surf_hi", ctypes.c_int32 * 3),
        ("eta_on_source", ctypes.c_int32),
        ("sub_core", ctypes.c_int32 * 3),
        ("sub_halo", ctypes.c_int32),
        ("sub_taper", ctypes.c_int32),
        ("surface_kind", ctypes.c_int32),
        ("sphere_nodes", ctypes.c_int32 * 2),
        ("sphere_radius", ctypes.c_double),
        ("abc_UR", ctypes.c_double),
        ("abc_alphaR", ctypes.c_double),
        ("scheme", ctypes.c_int32),
    ]


def problem_from(obj) -> pstd_problem:
    """Fill a pstd_problem from any object with the same attribute names
    (tfsf as three 4-tuples; booleans for force_dt / eta_on_source)."""
    p = pstd_problem()
    for a in range(3):
        p.n[a] = int(obj.n[a])
        p.h[a] = float(obj.h[a])
        p.abc_cells[a] = int(obj.abc_cells[a])
        for q in range(4):
            p.tfsf[a][q] = int(obj.tfsf[a][q])
        p.surf_lo[a] = int(obj.surf_lo[a])
        p.surf_hi[a] = int(obj.surf_hi[a])
    for name in ("hbar", "mass", "k0", "theta", "phi", "abc_U0", "abc_alpha", "v_max", "dt", "ramp_periods"):
        setattr(p, name, float(getattr(obj, name)))
    p.abc_UR = float(getattr(obj, "abc_UR", 0.0))
    p.abc_alphaR = float(getattr(obj, "abc_alphaR", 0.0))
    p.scheme = int(getattr(obj, "scheme", 0))
    p.force_dt = int(bool(getattr(obj, "force_dt", False)))
    p.eta_on_source = int(bool(getattr(obj, "eta_on_source", False)))
    p.dft_begin = int(obj.dft_begin)
    p.dft_end = int(obj.dft_end)
    sub = getattr(obj, "sub_core", None)
    if sub:
        for a in range(3):
            p.sub_core[a] = int(sub[a])
        p.sub_halo = int(obj.sub_halo)
        p.sub_taper = int(obj.sub_taper)
    p.surface_kind = int(getattr(obj, "surface_kind", 0))
    nodes = getattr(obj, "sphere_nodes", (0, 0))
    p.sphere_nodes[0] = int(nodes[0])
    p.sphere_nodes[1] = int(nodes[1])
    p.sphere_radius = float(getattr(obj, "sphere_radius", 0.0))
    return p


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_PP = ctypes.POINTER(pstd_problem)

_SIGS = {
    "pstd_problem_init_defaults": [_PP],
    "pstd_critical_dt": [_PP, ctypes.c_double, ctypes.POINTER(ctypes.c_double)],
    "pstd_reduced_step": [_PP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "pstd_create": [_PP, _vp, ctypes.POINTER(_vp)],
    "pstd_set_potential": [_vp, _vp, _i64],
    "pstd_set_state": [_vp, _vp, _vp, _i64, _i64],
    "pstd_run": [_vp, _i64],
    "pstd_run_timed": [_vp, _i64, ctypes.POINTER(ctypes.c_double)],
    "pstd_step_index": [_vp, ctypes.POINTER(_i64)],
    "pstd_get_psi": [_vp, ctypes.c_int32, _vp, _i64],
    "pstd_surface_size": [_vp, ctypes.POINTER(_i64)],
    "pstd_get_surface_phasors": [_vp, _vp, _i64],
    "pstd_project": [_vp, _vp, _i64, _vp],
    "pstd_far_field": [_vp, _vp, _i64, _vp],
    "pstd_set_pulse": [_vp, _vp, ctypes.c_int32, ctypes.c_double, _vp, ctypes.c_int32],
    "pstd_get_sphere_phasors_k": [_vp, ctypes.c_int32, _vp, _i64],
    "pstd_get_surface_phasors_k": [_vp, ctypes.c_int32, _vp, _i64],
    "pstd_project_k": [_vp, ctypes.c_int32, _vp, _i64, _vp],
    "pstd_far_field_k": [_vp, ctypes.c_int32, _vp, _i64, _vp],
    "pstd_misfit_forward": [_vp, _i64, _vp, _i64, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
    "pstd_misfit_backward": [_vp, _vp, _i64],
    "pstd_state_size": [_vp, ctypes.POINTER(_i64)],
    "pstd_sphere_size": [_vp, ctypes.POINTER(_i64)],
    "pstd_get_sphere_phasors": [_vp, _vp, _i64],
    "pstd_save_state": [_vp, _vp, _i64],
    "pstd_load_state": [_vp, _vp, _i64],
    "pstd_destroy": [_vp],
    "pstd_autotune": [_vp, ctypes.c_int32],
    "pstd_pass_time": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
    "pstd_check_state": [_vp, ctypes.POINTER(ctypes.c_double)],
    "pstd_check_state_noalloc": [_vp, ctypes.POINTER(ctypes.c_double)],
    "pstd_tile_info": [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "pstd_set_tile": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "pstd_tile_variants": [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                           ctypes.POINTER(ctypes.c_int32)],
    "pstd_batch_create": [ctypes.c_void_p, ctypes.c_int32, _vp, ctypes.POINTER(_vp)],
    "pstd_batch_size": [_vp, ctypes.POINTER(ctypes.c_int32)],
    "pstd_batch_solver": [_vp, ctypes.c_int32, ctypes.POINTER(_vp)],
    "pstd_batch_set_potential": [_vp, ctypes.c_int32, _vp, _i64],
    "pstd_batch_autotune": [_vp, ctypes.c_int32],
    "pstd_batch_run": [_vp, ctypes.POINTER(_i64)],
    "pstd_batch_destroy": [_vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
lib.pstd_status_string.argtypes = [ctypes.c_int]
lib.pstd_status_string.restype = ctypes.c_char_p
lib.pstd_last_error.argtypes = [_vp]
lib.pstd_last_error.restype = ctypes.c_char_p
lib.pstd_batch_last_error.argtypes = [_vp]
lib.pstd_batch_last_error.restype = ctypes.c_char_p

# every symbol include/pstd.h declares
EXPORTED = tuple(_SIGS) + ("pstd_status_string", "pstd_last_error", "pstd_batch_last_error")


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def _check(st, solver=None):
    if st != 0:
        msg = lib.pstd_last_error(solver).decode(errors="replace")
        raise PstdError(st, msg)


def pstd_status_string(st):
    return lib.pstd_status_string(int(st)).decode()


def pstd_last_error(solver=None):
    return lib.pstd_last_error(solver).decode(errors="replace")


def pstd_problem_init_defaults():
    p = pstd_problem()
    _check(lib.pstd_problem_init_defaults(ctypes.byref(p)))
    return p


def pstd_critical_dt(problem, vmax):
    out = ctypes.c_double()
    _check(lib.pstd_critical_dt(ctypes.byref(problem), float(vmax), ctypes.byref(out)))
    return out.value


def pstd_reduced_step(problem):
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib.pstd_reduced_step(ctypes.byref(problem), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def pstd_create(problem, stream=None):
    h = _vp()
    _check(lib.pstd_create(ctypes.byref(problem), _stream(stream), ctypes.byref(h)))
    return h.value


def pstd_set_potential(solver, V_dev, n_cells):
    _check(lib.pstd_set_potential(solver, _ptr(V_dev), int(n_cells)), solver)


def pstd_set_state(solver, prev_dev, cur_dev, n_cells, step):
    _check(lib.pstd_set_state(solver, _ptr(prev_dev), _ptr(cur_dev), int(n_cells), int(step)), solver)


def pstd_run(solver, n_steps):
    _check(lib.pstd_run(solver, int(n_steps)), solver)


def pstd_run_timed(solver, n_steps):
    out = (ctypes.c_double * 3)()
    _check(lib.pstd_run_timed(solver, int(n_steps), out), solver)
    return [out[0], out[1], out[2]]


def pstd_step_index(solver):
    out = _i64()
    _check(lib.pstd_step_index(solver, ctypes.byref(out)), solver)
    return out.value


def pstd_get_psi(solver, level, psi_dev, n_cells):
    _check(lib.pstd_get_psi(solver, int(level), _ptr(psi_dev), int(n_cells)), solver)


def pstd_surface_size(solver):
    out = _i64()
    _check(lib.pstd_surface_size(solver, ctypes.byref(out)), solver)
    return out.value


def pstd_get_surface_phasors(solver, out_dev, n):
    _check(lib.pstd_get_surface_phasors(solver, _ptr(out_dev), int(n)), solver)


def pstd_project(solver, obs_dev, n_obs, out_dev):
    _check(lib.pstd_project(solver, _ptr(obs_dev), int(n_obs), _ptr(out_dev)), solver)


def pstd_far_field(solver, dir_dev, n_dir, out_dev):
    _check(lib.pstd_far_field(solver, _ptr(dir_dev), int(n_dir), _ptr(out_dev)), solver)


def pstd_set_pulse(solver, psi0, delta, kbars):
    """psi0: complex packet on the 1D grid (host); kbars: reduced wavenumbers (host)."""
    import numpy as np
    p = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128))
    k = np.ascontiguousarray(np.asarray(kbars, dtype=np.float64))
    _check(lib.pstd_set_pulse(solver, p.ctypes.data_as(_vp), int(p.size), float(delta),
                              k.ctypes.data_as(_vp), int(k.size)), solver)


def pstd_get_surface_phasors_k(solver, ik, out_dev, n):
    _check(lib.pstd_get_surface_phasors_k(solver, int(ik), _ptr(out_dev), int(n)), solver)


def pstd_get_sphere_phasors_k(solver, ik, out_dev, n):
    _check(lib.pstd_get_sphere_phasors_k(solver, int(ik), _ptr(out_dev), int(n)), solver)


def pstd_project_k(solver, ik, obs_dev, n_obs, out_dev):
    _check(lib.pstd_project_k(solver, int(ik), _ptr(obs_dev), int(n_obs), _ptr(out_dev)), solver)


def pstd_far_field_k(solver, ik, dir_dev, n_dir, out_dev):
    _check(lib.pstd_far_field_k(solver, int(ik), _ptr(dir_dev), int(n_dir), _ptr(out_dev)), solver)


def pstd_sphere_size(solver):
    out = _i64()
    _check(lib.pstd_sphere_size(solver, ctypes.byref(out)), solver)
    return out.value


def pstd_get_sphere_phasors(solver, out_dev, n):
    _check(lib.pstd_get_sphere_phasors(solver, _ptr(out_dev), int(n)), solver)


def pstd_state_size(solver):
    out = _i64()
    _check(lib.pstd_state_size(solver, ctypes.byref(out)), solver)
    return out.value


def pstd_save_state(solver, buf_dev, nbytes):
    _check(lib.pstd_save_state(solver, _ptr(buf_dev), int(nbytes)), solver)


def pstd_load_state(solver, buf_dev, nbytes):
    _check(lib.pstd_load_state(solver, _ptr(buf_dev), int(nbytes)), solver)


def pstd_misfit_forward(solver, n_steps, obs_dev, n_obs, target_dev, n_checkpoints):
    J = ctypes.c_double()
    _check(lib.pstd_misfit_forward(solver, int(n_steps), _ptr(obs_dev), int(n_obs), _ptr(target_dev),
                                   int(n_checkpoints), ctypes.byref(J)), solver)
    return J.value


def pstd_misfit_backward(solver, out_dev, n_cells):
    _check(lib.pstd_misfit_backward(solver, _ptr(out_dev), int(n_cells)), solver)


def pstd_check_state(solver):
    out = ctypes.c_double()
    _check(lib.pstd_check_state(solver, ctypes.byref(out)), solver)
    return out.value


def pstd_check_state_noalloc(solver):
    out = ctypes.c_double()
    _check(lib.pstd_check_state_noalloc(solver, ctypes.byref(out)), solver)
    return out.value


def pstd_pass_time(solver, axis, reps=50):
    out = ctypes.c_double()
    _check(lib.pstd_pass_time(solver, int(axis), int(reps), ctypes.byref(out)), solver)
    return out.value


def pstd_autotune(solver, reps=5):
    _check(lib.pstd_autotune(solver, int(reps)), solver)


def pstd_tile_info(solver, axis):
    """(N, N1, N2, pencils, M1) of the pass along `axis`."""
    out = (ctypes.c_int32 * 5)()
    _check(lib.pstd_tile_info(solver, int(axis), out), solver)
    return tuple(out)


def pstd_set_tile(solver, axis, n1, pencils, m1=0):
    _check(lib.pstd_set_tile(solver, int(axis), int(n1), int(pencils), int(m1)), solver)


def pstd_tile_variants(n, segmented=False):
    cnt = ctypes.c_int32()
    buf = (ctypes.c_int32 * 64)()
    _check(lib.pstd_tile_variants(int(n), int(bool(segmented)), buf, 16, ctypes.byref(cnt)))
    return [tuple(buf[4 * k:4 * k + 4]) for k in range(min(cnt.value, 16))]


def pstd_destroy(solver):
    _check(lib.pstd_destroy(solver))


def _bcheck(st, batch=None):
    if st != 0:
        raise PstdError(st, lib.pstd_batch_last_error(batch).decode(errors="replace"))


def pstd_batch_create(problems, stream=None):
    arr = (pstd_problem * len(problems))(*problems)
    h = _vp()
    _bcheck(lib.pstd_batch_create(ctypes.cast(arr, ctypes.c_void_p), len(problems), _stream(stream), ctypes.byref(h)))
    return h.value


def pstd_batch_size(batch):
    out = ctypes.c_int32()
    _bcheck(lib.pstd_batch_size(batch, ctypes.byref(out)), batch)
    return out.value


def pstd_batch_solver(batch, idx):
    h = _vp()
    _bcheck(lib.pstd_batch_solver(batch, int(idx), ctypes.byref(h)), batch)
    return h.value


def pstd_batch_set_potential(batch, idx, V_dev, n_cells):
    _bcheck(lib.pstd_batch_set_potential(batch, int(idx), _ptr(V_dev), int(n_cells)), batch)


def pstd_batch_autotune(batch, reps=5):
    _bcheck(lib.pstd_batch_autotune(batch, int(reps)), batch)


def pstd_batch_run(batch, n_steps):
    arr = (_i64 * len(n_steps))(*[int(v) for v in n_steps])
    _bcheck(lib.pstd_batch_run(batch, arr), batch)


def pstd_batch_destroy(batch):
    _bcheck(lib.pstd_batch_destroy(batch))


def pstd_batch_last_error(batch=None):
    return lib.pstd_batch_last_error(batch).decode(errors="replace")


class Solver:
    """Owning wrapper around a pstd_solver handle; buffers are torch tensors."""

    def __init__(self, problem, stream=None, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.problem = problem if isinstance(problem, pstd_problem) else problem_from(problem)
        self.n = tuple(self.problem.n[a] for a in range(3))
        self.cells = self.n[0] * self.n[1] * self.n[2]
        self.stream = stream
        if self.device.type == "cuda":
            torch.cuda.init()  # torch's runtime first: it owns the buffers passed in
        self.handle = pstd_create(self.problem, stream)

    def close(self):
        if self.handle:
            pstd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shape(self):
        return (self.n[2], self.n[1], self.n[0])

    def set_potential(self, V):
        t = self.torch.as_tensor(V, dtype=self.torch.float32, device=self.device).contiguous()
        assert t.numel() == self.cells
        pstd_set_potential(self.handle, t, self.cells)

    def set_state(self, prev, cur, step):
        c64 = self.torch.complex64
        a = self.torch.as_tensor(prev, dtype=c64, device=self.device).contiguous()
        b = self.torch.as_tensor(cur, dtype=c64, device=self.device).contiguous()
        pstd_set_state(self.handle, a, b, self.cells, step)

    def run(self, n_steps):
        pstd_run(self.handle, n_steps)

    def autotune(self, reps=5):
        pstd_autotune(self.handle, reps)
        return [pstd_tile_info(self.handle, a) for a in range(3)]

    def set_tile(self, axis, n1, pencils, m1=0):
        pstd_set_tile(self.handle, axis, n1, pencils, m1)

    def tiles(self):
        return [pstd_tile_info(self.handle, a) for a in range(3)]

    def check_state(self):
        """sum |psi|^2 (FP64); raises PstdError ENONFINITE on NaN / Inf."""
        return pstd_check_state(self.handle)

    def pass_time(self, axis, reps=50):
        """Average microseconds per launch of one axis pass (pstd_pass_time)."""
        return pstd_pass_time(self.handle, axis, reps)

    def run_timed(self, n_steps):
        return pstd_run_timed(self.handle, n_steps)

    @property
    def step(self):
        return pstd_step_index(self.handle)

    def psi(self, level=0):
        out = self.torch.empty(self._shape(), dtype=self.torch.complex64, device=self.device)
        pstd_get_psi(self.handle, level, out, self.cells)
        return out

    def phasors(self, ik=0):
        """Normalised box phasors (flat complex128 CUDA tensor); ik selects a
        pulsed run's wavenumber."""
        n = pstd_surface_size(self.handle)
        out = self.torch.empty(n, dtype=self.torch.complex128, device=self.device)
        pstd_get_surface_phasors_k(self.handle, ik, out, n)
        return out

    def split_phasors(self, flat):
        """flat phasor vector -> ([psi plane per face], [dpsi plane per face])"""
        nx, ny, nz = self.n
        shapes = [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2
        phi, dphi = [], []
        off = 0
        for s in shapes:
            m = s[0] * s[1]
            phi.append(flat[off:off + m].reshape(s))
            dphi.append(flat[off + m:off + 2 * m].reshape(s))
            off += 2 * m
        return phi, dphi

    def project(self, points, ik=0):
        """Psi at physical points; ik selects a pulsed run's wavenumber."""
        pts = self.torch.as_tensor(points, dtype=self.torch.float64, device=self.device).contiguous()
        out = self.torch.empty(pts.shape[0], dtype=self.torch.complex128, device=self.device)
        pstd_project_k(self.handle, ik, pts, pts.shape[0], out)
        return out

    def far_field(self, dirs, ik=0):
        """f(r_hat); ik selects a pulsed run's wavenumber."""
        d = self.torch.as_tensor(dirs, dtype=self.torch.float64, device=self.device).contiguous()
        out = self.torch.empty(d.shape[0], dtype=self.torch.complex128, device=self.device)
        pstd_far_field_k(self.handle, ik, d, d.shape[0], out)
        return out

    def set_pulse(self, psi0, delta, kbars):
        """Pulsed incidence (pstd_set_pulse): the packet psi0 on the 1D grid of
        spacing delta (reduced) and the wavenumbers of the phasors."""
        pstd_set_pulse(self.handle, psi0, delta, kbars)

    def sphere_phasors(self, ik=0):
        """(psi, d psi/d n) at the sphere's nodes (complex128 CUDA tensors)."""
        n = pstd_sphere_size(self.handle)
        out = self.torch.empty(2 * n, dtype=self.torch.complex128, device=self.device)
        pstd_get_sphere_phasors_k(self.handle, ik, out, 2 * n)
        return out[:n], out[n:]

    def save_state(self):
        """The solver state as a uint8 CUDA tensor (pstd_save_state)."""
        n = pstd_state_size(self.handle)
        buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        pstd_save_state(self.handle, buf, n)
        return buf

    def load_state(self, buf):
        pstd_load_state(self.handle, buf, buf.numel() * buf.element_size())

    def misfit(self, n_steps, points, target, n_checkpoints=None):
        """J of the detector-plane intensity misfit (pstd_misfit_forward)."""
        import math
        torch = self.torch
        pts = torch.as_tensor(points, dtype=torch.float64, device=self.device).contiguous()
        tgt = torch.as_tensor(target, dtype=torch.float64, device=self.device).contiguous()
        if n_checkpoints is None:
            n_checkpoints = max(1, math.ceil(math.sqrt(n_steps)))
        # the library keeps one misfit run per solver: a new run replaces it
        self._misfit_run = getattr(self, "_misfit_run", 0) + 1
        return pstd_misfit_forward(self.handle, n_steps, pts, pts.shape[0], tgt, n_checkpoints)

    def misfit_gradient(self):
        """dJ/dV of the last misfit run (pstd_misfit_backward), [k][j][i] float32."""
        out = self.torch.empty(self._shape(), dtype=self.torch.float32, device=self.device)
        pstd_misfit_backward(self.handle, out, self.cells)
        return out


def _fresnel_misfit_class():
    import torch

    class FresnelMisfit(torch.autograd.Function):
        """J(V) with dJ/dV from the library's adjoint run.

        apply(V, solver, n_steps, points, target, n_checkpoints) -> 0-d float64
        tensor; V is a float32 [nz, ny, nx] CUDA tensor in energy units.
        """

        @staticmethod
        def forward(ctx, V, solver, n_steps, points, target, n_checkpoints=None):
            solver.set_potential(V.detach())
            J = solver.misfit(n_steps, points, target, n_checkpoints)
            ctx.solver = solver
            ctx.run = solver._misfit_run
            return torch.tensor(J, dtype=torch.float64, device=V.device)

        @staticmethod
        def backward(ctx, grad_out):
            # the solver holds only its latest misfit run's checkpoints: a
            # later forward on the same solver would answer for another V
            if getattr(ctx.solver, "_misfit_run", None) != ctx.run:
                raise RuntimeError("FresnelMisfit.backward: the solver has run another misfit since this "
                                   "forward; use one solver per misfit term of a graph")
            g = ctx.solver.misfit_gradient()
            return (g * grad_out.to(g.dtype)).reshape(g.shape), None, None, None, None, None

    return FresnelMisfit


def __getattr__(name):
    if name == "FresnelMisfit":
        cls = _fresnel_misfit_class()
        globals()["FresnelMisfit"] = cls
        return cls
    raise AttributeError(name)


class _BorrowedSolver(Solver):
    """View of one batch instance (not destroyed by Python)."""

    def __init__(self, batch, idx, problem):
        import torch
        self.torch = torch
        self.device = torch.device("cuda")
        self.problem = problem
        self.n = tuple(problem.n[a] for a in range(3))
        self.cells = self.n[0] * self.n[1] * self.n[2]
        self.stream = batch.stream
        self.handle = pstd_batch_solver(batch.handle, idx)
        self._batch = batch

    def close(self):
        self.handle = None


class Batch:
    """Owning wrapper around a pstd_batch handle."""

    def __init__(self, problems, stream=None):
        import torch
        self.problems = [p if isinstance(p, pstd_problem) else problem_from(p) for p in problems]
        self.stream = stream
        torch.cuda.init()  # torch's runtime first: it owns the buffers passed in
        self.handle = pstd_batch_create(self.problems, stream)
        self.count = len(self.problems)

    def close(self):
        if self.handle:
            pstd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def instance(self, idx):
        return _BorrowedSolver(self, idx, self.problems[idx])

    def set_potential(self, idx, V):
        import torch
        t = torch.as_tensor(V, dtype=torch.float32, device="cuda").contiguous()
        pstd_batch_set_potential(self.handle, idx, t, t.numel())

    def autotune(self, reps=5):
        pstd_batch_autotune(self.handle, reps)

    def run(self, n_steps):
        if isinstance(n_steps, int):
            n_steps = [n_steps] * self.count
        pstd_batch_run(self.handle, n_steps)
