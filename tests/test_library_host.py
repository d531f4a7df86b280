"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/pstd.h declares, and its host arithmetic and validation
agree with the oracle and the paper."""
import math
import os
import re

import pytest

import synth
from oracle import pstd as opstd

lib_mod = pytest.importorskip("paper_2403_04053_amd")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pstd.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pstd_status|const char\*)\s+(pstd_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib_mod.lib, n), n
    assert set(names) == set(lib_mod.EXPORTED)


def test_status_strings():
    for code, name in lib_mod.STATUS.items():
        assert lib_mod.pstd_status_string(code) == name


@pytest.mark.parametrize("make", [
    synth.plain_barrier, lambda: synth.tiny(n=(24, 20, 32), P=3, transition=2),
    # complex absorbing potentials: a shallow real part (the bound keeps v_max)
    # and a deep one (the layers' |UR| x 3 sets the bound)
    lambda: (synth.plain_barrier()[0].replace(abc_UR=-0.1, abc_alphaR=0.4), None),
    lambda: (synth.tiny(n=(24, 20, 32), P=3)[0].replace(abc_UR=-30.0), None)])
def test_reduced_step_matches_oracle(make):
    prob = make()[0]
    p = lib_mod.problem_from(prob)
    dtau, eta = lib_mod.pstd_reduced_step(p)
    assert dtau == pytest.approx(opstd.dtau_of(prob), rel=1e-14)
    assert eta == pytest.approx(opstd.eta_of(opstd.dtau_of(prob)), rel=1e-14)
    assert lib_mod.pstd_critical_dt(p, prob.v_max) == pytest.approx(opstd.critical_dt(prob, prob.v_max), rel=1e-14)


def test_defaults_are_valid_plain_method_geometry():
    p = lib_mod.pstd_problem_init_defaults()
    assert list(p.n) == [48, 48, 48]
    dtau, eta = lib_mod.pstd_reduced_step(p)
    # 0.9 of Eq. dtau_stability at dxb = pi/4, |V|max = E0/2
    assert dtau == pytest.approx(0.9 / (3 * 16 + 0.5), rel=1e-12)


def test_fdtd_scheme_step_bound_and_limits():
    """The FDTD variant's step (0.9 of its bound, no eta) matches the oracle;
    what it does not run (a DFT window on the box surface, subdomains) is
    refused before any device work; the spherical surface is accepted."""
    from oracle import fdtd as ofdtd
    prob, _ = synth.tiny(n=(24, 24, 32), P=4, transition=2, dft=(0, 0))
    prob = prob.replace(scheme=1)
    dtau, eta = lib_mod.pstd_reduced_step(lib_mod.problem_from(prob))
    assert dtau == pytest.approx(ofdtd.dtau_of(prob), rel=1e-14)
    lib_mod.pstd_reduced_step(lib_mod.problem_from(prob.replace(surface_kind=1, sphere_radius=0.5,
                                                                dft_begin=0, dft_end=10)))
    for bad in (dict(dft_begin=0, dft_end=10), dict(sub_core=(12, 0, 0), sub_halo=8, sub_taper=3)):
        with pytest.raises(lib_mod.PstdError) as e:
            lib_mod.pstd_reduced_step(lib_mod.problem_from(prob.replace(**bad)))
        assert e.value.name == "PSTD_EUNSUPPORTED"
    with pytest.raises(lib_mod.PstdError) as e:
        lib_mod.pstd_reduced_step(lib_mod.problem_from(prob.replace(scheme=2)))
    assert e.value.name == "PSTD_EINVAL"


def test_complex_absorber_fields_are_validated():
    prob, _ = synth.plain_barrier()
    for bad in (dict(abc_UR=float("inf")), dict(abc_UR=float("nan")), dict(abc_alphaR=-0.1)):
        with pytest.raises(lib_mod.PstdError) as e:
            lib_mod.pstd_reduced_step(lib_mod.problem_from(prob.replace(**bad)))
        assert e.value.name == "PSTD_EINVAL"


def _expect(status_name, prob):
    with pytest.raises(lib_mod.PstdError) as e:
        lib_mod.pstd_create(lib_mod.problem_from(prob))
    assert e.value.name == status_name


def test_create_rejects_bad_geometry_before_touching_the_device():
    prob, _ = synth.plain_barrier()
    _expect("PSTD_EINVAL", prob.replace(n=(47, 48, 48)))
    _expect("PSTD_EINVAL", prob.replace(surf_lo=(13, 10, 10)))       # face inside the taper
    _expect("PSTD_EINVAL", prob.replace(surf_hi=(38, 35, 38)))
    _expect("PSTD_EINVAL", prob.replace(surf_lo=(5, 10, 10)))        # inside the absorber
    _expect("PSTD_EINVAL", prob.replace(tfsf=((12, 11, 30, 36),) * 3))
    _expect("PSTD_EINVAL", prob.replace(k0=0.0))
    _expect("PSTD_EUNSUPPORTED", prob.replace(n=(50, 48, 48), tfsf=((12, 18, 30, 36),) * 3))


def test_create_rejects_unstable_step():
    """The plain-method workload's literal dt = 0.1 dx^2 is above the bound of
    Eq. PSTDstability and is refused unless forced."""
    prob, _ = synth.plain_barrier()
    _expect("PSTD_EUNSTABLE", prob.replace(dt=0.1 * 0.1 ** 2))
    ok = lib_mod.problem_from(prob.replace(dt=0.99 * opstd.critical_dt(prob, prob.v_max)))
    assert lib_mod.pstd_reduced_step(ok)[0] > 0


def test_subdomain_validation():
    prob, _ = synth.bumps_288()
    p = lib_mod.problem_from(prob)
    assert list(p.sub_core) == [48, 48, 48] and p.sub_halo == 8 and p.sub_taper == 3
    _expect("PSTD_EINVAL", prob.replace(sub_taper=4))                       # halo < taper + 5
    _expect("PSTD_EINVAL", prob.replace(sub_core=(50, 48, 48)))            # does not tile 288
    _expect("PSTD_EUNSUPPORTED", prob.replace(sub_core=(72, 48, 48)))      # local length 88


def test_binding_argument_kinds_match_the_header():
    """Every function the binding declares takes, in the header, the same
    number of parameters of the same kinds (pointer, int64, int32, double):
    a mismatch would pass garbage through ctypes without an error."""
    import ctypes
    text = open(HEADER).read()
    decls = {}
    for m in re.finditer(r"^\s*pstd_status\s+(pstd_\w+)\s*\(([^;]*?)\)\s*;", text, re.M | re.S):
        decls[m.group(1)] = [p.strip() for p in m.group(2).split(",") if p.strip()]

    def kind_c(p):
        if "*" in p:
            return "ptr"
        if p.startswith("int64_t"):
            return "i64"
        if p.startswith("int32_t"):
            return "i32"
        if p.startswith("double"):
            return "f64"
        return "?" + p

    def kind_py(t):
        if t in (ctypes.c_void_p,) or hasattr(t, "_type_") and isinstance(t._type_, type):
            return "ptr"
        return {ctypes.c_int64: "i64", ctypes.c_int32: "i32", ctypes.c_double: "f64"}.get(t, "?" + repr(t))

    sigs = lib_mod._SIGS
    assert len(sigs) >= 30
    for name, args in sigs.items():
        assert name in decls, name
        want = [kind_c(p) for p in decls[name]]
        got = [kind_py(t) for t in args]
        assert got == want, (name, got, want)


def test_tile_variants_cover_every_workload_length():
    """pstd_tile_variants (host only) lists (N1, N2, pencils, M1) for every
    compiled length: N1 * N2 = N, a stage-B split M1 divides N2 with both M1
    and N2 / M1 dividing N1, and the subdomain length has a segmented
    instance; lengths without a compiled pass list nothing."""
    for n in (8, 12, 16, 20, 24, 32, 40, 48, 64, 80, 96, 100, 108, 120, 128, 144, 150, 160, 162, 180, 192, 256, 288):
        shapes = lib_mod.pstd_tile_variants(n)
        assert shapes, n
        for n1, n2, pencils, m1 in shapes:
            assert n1 * n2 == n and pencils in (8, 16, 32, 64), (n, n1, n2, pencils)
            if m1:
                assert n2 % m1 == 0 and n1 % m1 == 0 and n1 % (n2 // m1) == 0, (n, n1, n2, m1)
    assert any(m1 for *_, m1 in lib_mod.pstd_tile_variants(288))
    assert lib_mod.pstd_tile_variants(64, segmented=True)
    assert lib_mod.pstd_tile_variants(72) == [] and lib_mod.pstd_tile_variants(290) == []
