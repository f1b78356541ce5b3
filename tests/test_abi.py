"""Host-side checks of libpfmi: it loads, exports every declared symbol, and
its host logic (weights, stability limit, footprint, descriptor validation)
agrees with the oracle and the paper's table.  No device calls."""
import ctypes
import math
import os
import re
from fractions import Fraction

import pytest

import oracle
import paper_2511_10508_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pfmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    names = _declared()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(P.SIGNATURES), set(names) ^ set(P.SIGNATURES)


def test_single_hip_runtime_and_version():
    P.lib()
    assert len(P.hip_runtimes_mapped()) == 1
    assert P.lib().pf_abi_version() == 1
    assert P.lib().pf_status_str(2) == b"time step above the stability limit"


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 14, 16])
def test_fornberg_matches_exact_weights(order):
    w = P.weights(order)
    exact = oracle.second_derivative_weights_exact(order)
    for a, e in zip(w, exact):
        assert abs(Fraction(float(a)) - e) <= 8 * Fraction(math.ulp(float(e)) or 2.0 ** -1074) + Fraction(1, 10 ** 14) * abs(e)


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12, 14, 16])
def test_fornberg_fourth_derivative_matches_exact_weights(order):
    w = P.weights4(order)
    exact = oracle.fourth_derivative_weights_exact(order)
    assert len(w) == len(exact) == order // 2 + 2
    for a, e in zip(w, exact):
        assert abs(Fraction(float(a)) - e) <= 8 * Fraction(math.ulp(float(e)) or 2.0 ** -1074) + Fraction(1, 10 ** 13) * abs(e)


def test_weights_reject_bad_order():
    with pytest.raises(P.PfError):
        P.weights(3)
    with pytest.raises(P.PfError):
        P.weights(18)


@pytest.mark.parametrize("kind,ndim,order,params", [
    (P.PF_AC, 2, 2, [1.0, 1.0]), (P.PF_CH, 2, 4, [1.0, 1.0]), (P.PF_CH, 3, 6, [1.0, 1.0]),
    (P.PF_GS, 3, 2, [0.2, 0.1, 0.04, 0.06]), (P.PF_AC, 3, 8, [0.7, 1.3]),
    (P.PF_MC, 2, 4, [1.0, 1.0, 0.5]), (P.PF_MC, 3, 2, [0.8, 1.2, 0.5]),
])
def test_stability_matches_oracle(kind, ndim, order, params):
    n = (16,) * ndim
    d = P.make_desc(kind, n, dx=0.9, order=order, params=params)
    assert math.isclose(P.stability(d), oracle.dt_max(kind, ndim, 0.9, order, params), rel_tol=1e-12)


@pytest.mark.parametrize("ndim,order", [(1, 2), (1, 4), (2, 4), (2, 6), (3, 2), (3, 8)])
def test_stability_direct_biharmonic_matches_oracle(ndim, order):
    d = P.make_desc(P.PF_CH, (16,) * ndim, dx=1.1, order=order, params=[0.9, 1.0],
                    flags=P.PF_BIHARMONIC_DIRECT)
    ref = oracle.dt_max(oracle.CH, ndim, 1.1, order, [0.9, 1.0], biharmonic="direct")
    assert math.isclose(P.stability(d), ref, rel_tol=1e-12)


@pytest.mark.parametrize("kind,params", [(P.PF_AC, [1.0, 1.0]), (P.PF_CH, [1.0, 1.0]),
                                         (P.PF_GS, [0.2, 0.1, 0.04, 0.06]), (P.PF_MC, [1.0, 1.0, 0.5])])
def test_stability_1d_matches_oracle(kind, params):
    d = P.make_desc(kind, (100,), dx=0.8, order=4, params=params)
    assert d.ndim == 1 and list(d.n) == [100, 1, 1]
    assert math.isclose(P.stability(d), oracle.dt_max(kind, 1, 0.8, 4, params), rel_tol=1e-12)


@pytest.mark.parametrize("kind,n,flags", [
    (P.PF_AC, (64, 64), 16),        # the direct biharmonic is Cahn-Hilliard only
    (P.PF_GS, (64,), 16),
    (P.PF_MC, (64, 64, 8), 16),
])
def test_direct_biharmonic_flag_needs_cahn_hilliard(kind, n, flags):
    d = P.make_desc(kind, n, dt=1e-3, order=4, flags=flags)
    h = ctypes.c_void_p()
    assert P.lib().pf_create(ctypes.byref(d), None, ctypes.byref(h)) == P.PF_ERR_ARG
    assert b"Cahn-Hilliard" in P.lib().pf_last_error()


def test_1d_descriptor_checks():
    for ndim, n in ((1, (64, 2, 1)), (1, (64, 1, 2)), (2, (64, 8, 2)), (0, (64, 1, 1))):
        d = P.make_desc(P.PF_AC, (64,), dt=0.01)
        d.ndim = ndim
        for a in range(3):
            d.n[a] = n[a]
        h = ctypes.c_void_p()
        assert P.lib().pf_create(ctypes.byref(d), None, ctypes.byref(h)) == P.PF_ERR_ARG


def test_footprint_against_paper_table():
    """Paper Table memory-footprint: m = 2f + f0.  The fused kernels keep no
    temporary (f0 = 0), so Model A stays m = 2 and Model B drops from 3 to 2."""
    rows = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "memory_footprint.txt")):
        if line.strip() and not line.startswith("#"):
            name, f, f0, m = line.split()
            rows[name] = (int(f), int(f0), int(m))
    assert rows["A"] == (1, 0, 2) and rows["B"] == (1, 1, 3)
    for kind, name, P_ in ((P.PF_AC, "A", 8), (P.PF_CH, "B", 8), (P.PF_AC, "A", 4)):
        prec = P.PF_FP64 if P_ == 8 else P.PF_FP32
        d = P.make_desc(kind, (1024, 1024), precision=prec)
        f, f0, m = rows[name]
        per_site = P.footprint_bytes(d) / (1024 * 1024 * P_)
        assert 2 * f <= per_site < 2 * f + 0.2
    d = P.make_desc(P.PF_GS, (256, 256, 256))
    assert 4 <= P.footprint_bytes(d) / (256 ** 3 * 8) < 4.2
    # Model C: the paper's two-pass design holds 5 arrays, the fused kernels 2f = 4
    assert rows["C"] == (2, 1, 5)
    d = P.make_desc(P.PF_MC, (1024, 1024))
    assert 4 <= P.footprint_bytes(d) / (1024 * 1024 * 8) < 4.2


def test_model_c_descriptor_checks():
    d = P.make_desc(P.PF_MC, (64, 64), dt=0.01, order=4)
    assert d.nfields == 2 and d.nparams == 3
    for field, value in (("nfields", 1), ("nparams", 2)):
        bad = P.make_desc(P.PF_MC, (64, 64), dt=0.01, order=4)
        setattr(bad, field, value)
        h = ctypes.c_void_p()
        assert P.lib().pf_create(ctypes.byref(bad), None, ctypes.byref(h)) == P.PF_ERR_ARG


def test_padded_pitch_and_buffer_elems():
    d = P.make_desc(P.PF_AC, (13, 7), precision=P.PF_FP64)
    assert P.buffer_elems(d) == 14 * 7
    d = P.make_desc(P.PF_AC, (13, 7), precision=P.PF_FP32)
    assert P.buffer_elems(d) == 16 * 7


@pytest.mark.parametrize("mutate,status", [
    (lambda d: setattr(d, "kind", 9), P.PF_ERR_ARG),
    (lambda d: setattr(d, "nfields", 2), P.PF_ERR_ARG),
    (lambda d: setattr(d, "order", 3), P.PF_ERR_ARG),
    (lambda d: setattr(d, "order", 18), P.PF_ERR_ARG),
    (lambda d: setattr(d, "dt", -1.0), P.PF_ERR_ARG),
    (lambda d: setattr(d, "dx", 0.0), P.PF_ERR_ARG),
    (lambda d: setattr(d, "ndim", 4), P.PF_ERR_ARG),
    (lambda d: setattr(d, "nparams", 3), P.PF_ERR_ARG),
    (lambda d: setattr(d, "struct_size", 8), P.PF_ERR_ARG),
    (lambda d: setattr(d, "precision", 7), P.PF_ERR_ARG),
    (lambda d: setattr(d, "dt", 1.0), P.PF_ERR_UNSTABLE),
])
def test_create_rejects_bad_descriptors_before_touching_the_device(mutate, status):
    d = P.make_desc(P.PF_CH, (64, 64), dt=0.01, order=4)
    mutate(d)
    h = ctypes.c_void_p()
    assert P.lib().pf_create(ctypes.byref(d), None, ctypes.byref(h)) == status
    assert not h.value
    assert P.lib().pf_last_error()


def test_gray_scott_dt1_in_3d_is_refused():
    d = P.make_desc(P.PF_GS, (512, 512, 512), dt=1.0)
    h = ctypes.c_void_p()
    assert P.lib().pf_create(ctypes.byref(d), None, ctypes.byref(h)) == P.PF_ERR_UNSTABLE
    assert P.stability(d) > 0.5  # the proposed dt = 0.5 is accepted


def test_footprint_counts_generic_temporaries():
    """The per-site kernels hold field-sized temporaries where the fused ones
    do not apply: one for Cahn-Hilliard, ndim for the direct biharmonic."""
    n3, n2 = (64, 64, 64), (256, 256)
    base3 = P.footprint_bytes(P.make_desc(P.PF_CH, n3, dt=1e-3, order=4))
    per3 = P.buffer_elems(P.make_desc(P.PF_CH, n3)) * 8
    d = P.make_desc(P.PF_CH, n3, dt=1e-5, order=8, flags=P.PF_BIHARMONIC_DIRECT)
    base3_8 = P.footprint_bytes(P.make_desc(P.PF_CH, n3, dt=1e-5, order=8))
    assert P.footprint_bytes(d) == base3_8 + 2 * per3  # radius 4: no fused 3D direct kernel
    for order in (4, 6):  # the fused 3D direct kernel covers r <= 3
        d = P.make_desc(P.PF_CH, n3, dt=1e-4, order=order, flags=P.PF_BIHARMONIC_DIRECT)
        assert P.footprint_bytes(d) == base3
    d = P.make_desc(P.PF_CH, n3, dt=1e-3, order=8)  # radius 4: no fused 3D CH kernel
    assert P.footprint_bytes(d) == base3 + per3
    base2 = P.footprint_bytes(P.make_desc(P.PF_CH, n2, dt=1e-3, order=4))
    d = P.make_desc(P.PF_CH, n2, dt=1e-3, order=4, flags=P.PF_BIHARMONIC_DIRECT)
    assert P.footprint_bytes(d) == base2  # fused 2D direct kernel: no temporaries


def test_spectral_host_logic():
    """PF_SPECTRAL: Models A and B only, no explicit limit, two half spectra
    in the footprint; refused combinations fail before touching the device."""
    d = P.make_desc(P.PF_CH, (100, 64), dt=1.0, params=[0.8, 1.0], flags=P.PF_SPECTRAL)
    assert math.isclose(P.stability(d), oracle.spectral.dt_max(2, [0.8, 1.0]), rel_tol=1e-15)
    d = P.make_desc(P.PF_AC, (100, 64), dt=1.0, params=[0.8, 1.0], flags=P.PF_SPECTRAL)
    assert math.isclose(P.stability(d), oracle.spectral.dt_max(1, [0.8, 1.0]), rel_tol=1e-15)
    d = P.make_desc(P.PF_CH, (100, 64), dt=1.0, params=[0.0, 1.0], flags=P.PF_SPECTRAL)
    assert math.isinf(P.stability(d))
    d = P.make_desc(P.PF_CH, (100, 64), dt=1.0, flags=P.PF_SPECTRAL)
    h = ctypes.c_void_p()
    d.dt = 2.5  # above 2 / c1^2
    assert P.lib().pf_create(ctypes.byref(d), None, ctypes.byref(h)) == P.PF_ERR_UNSTABLE
    d.dt = 1.0
    plain = P.footprint_bytes(P.make_desc(P.PF_CH, (100, 64), dt=1e-3))
    assert P.footprint_bytes(d) == plain + 2 * 51 * 64 * 16
    d32 = P.make_desc(P.PF_AC, (100, 64), dt=0.5, precision=P.PF_FP32, flags=P.PF_SPECTRAL)
    plain32 = P.footprint_bytes(P.make_desc(P.PF_AC, (100, 64), dt=1e-3, precision=P.PF_FP32))
    assert P.footprint_bytes(d32) == plain32 + 2 * 51 * 64 * 8
    for kind, flags in ((P.PF_GS, 0), (P.PF_MC, 0), (P.PF_CH, P.PF_BIHARMONIC_DIRECT),
                        (P.PF_CH, P.PF_USE_GRAPH), (P.PF_AC, P.PF_FORCE_GENERIC)):
        bad = P.make_desc(kind, (32, 32), dt=1e-3, flags=P.PF_SPECTRAL | flags)
        h = ctypes.c_void_p()
        assert P.lib().pf_create(ctypes.byref(bad), None, ctypes.byref(h)) == P.PF_ERR_ARG
        assert b"PF_SPECTRAL" in P.lib().pf_last_error()


def test_model_h_descriptor_and_host_logic():
    for n in ((64,), (64, 64), (16, 16, 16)):
        d = P.make_desc(P.PF_MH, n, dt=1e-3, order=4)
        assert d.nfields == 1 + len(n) and d.nparams == 3
        ref = oracle.dt_max(oracle.MH, len(n), 1.0, 4, [1.0, 1.0, 0.5])
        assert math.isclose(P.stability(d), ref, rel_tol=1e-12)
        per = P.buffer_elems(d) * 8
        plain = P.footprint_bytes(P.make_desc(P.PF_AC, n, dt=1e-3))
        # 2 (1 + ndim) field buffers; no temporary (one fused pass in 1D, 2D
        # and 3D at order 4), one (mu) for the per-site kernels
        assert P.footprint_bytes(d) == plain + 2 * len(n) * per
        g = P.make_desc(P.PF_MH, n, dt=1e-3, order=4, flags=P.PF_FORCE_GENERIC)
        assert P.footprint_bytes(g) == P.footprint_bytes(d) + per
    d8 = P.make_desc(P.PF_MH, (16, 16, 16), dt=1e-4, order=8)
    assert P.footprint_bytes(d8) == (P.footprint_bytes(P.make_desc(P.PF_AC, (16, 16, 16), dt=1e-4, order=8))
                                     + 7 * P.buffer_elems(d8) * 8)
    bad = P.make_desc(P.PF_MH, (64, 64), dt=1e-3)
    bad.nfields = 2
    h = ctypes.c_void_p()
    assert P.lib().pf_create(ctypes.byref(bad), None, ctypes.byref(h)) == P.PF_ERR_ARG


@pytest.mark.parametrize("order", [2, 4, 6, 8, 12, 16])
def test_fornberg_first_derivative_matches_exact_weights(order):
    """The library's first-derivative weights (Model H's gradient and
    divergence) equal the oracle's exact ones to rounding."""
    w = P.weights1(order)
    exact = oracle.first_derivative_weights_exact(order)
    assert len(w) == len(exact)
    for a, e in zip(w, exact):
        assert abs(Fraction(float(a)) - e) <= 8 * Fraction(math.ulp(float(e)) or 2.0 ** -1074) + Fraction(1, 10 ** 14) * abs(e)


def test_step_noalloc_refusals_precede_any_device_call():
    """pf_step_noalloc checks its arguments and the reduction scratch it needs
    (against the static 16 MiB) on the host before any HIP call; here, with
    no GPU, each refusal is its own status rather than a device error.  The
    pointers are never dereferenced: every case is refused first."""
    ptrs = [16 * (i + 1) for i in range(4)]
    red = P.PF_REDUCE_EACH_STEP
    big = P.make_desc(P.PF_GS, (128, 4096, 6144), dt=0.5, order=2, precision=P.PF_FP32, flags=red)
    with pytest.raises(P.PfError) as e:
        P.step_noalloc(big, None, ptrs, 0, 1, 4096)
    assert e.value.status == P.PF_ERR_ARG and "16 MiB" in str(e.value)
    generic = P.make_desc(P.PF_CH, (20, 20, 20), dt=1e-4, order=10)
    with pytest.raises(P.PfError) as e:
        P.step_noalloc(generic, None, ptrs[:2], 0, 1, None)
    assert e.value.status == P.PF_ERR_UNSUPPORTED
    small = P.make_desc(P.PF_CH, (20, 20), dt=0.01, order=4, flags=red)
    for args, status in (((ptrs[:2], 2, 1, 4096), P.PF_ERR_ARG),       # parity
                         ((ptrs[:1], 0, 1, 4096), P.PF_ERR_ARG),       # nbufs
                         ((ptrs[:2], 0, 1, None), P.PF_ERR_ARG),       # history
                         ((ptrs[:2], 0, -1, 4096), P.PF_ERR_ARG),      # nsteps
                         (([16, 40], 0, 1, 4096), P.PF_ERR_ARG)):      # alignment
        with pytest.raises(P.PfError) as e:
            P.step_noalloc(small, None, *args)
        assert e.value.status == status
    for flag in (P.PF_USE_GRAPH, P.PF_FORCE_GENERIC):
        d = P.make_desc(P.PF_CH, (20, 20), dt=0.01, order=4, flags=flag)
        with pytest.raises(P.PfError) as e:
            P.step_noalloc(d, None, ptrs[:2], 0, 1, None)
        assert e.value.status == P.PF_ERR_ARG
    unstable = P.make_desc(P.PF_GS, (16, 16, 16), dt=1.0, order=2)
    with pytest.raises(P.PfError) as e:
        P.step_noalloc(unstable, None, ptrs, 0, 1, None)
    assert e.value.status == P.PF_ERR_UNSTABLE
