"""The C ABI library loads, exports every symbol the header declares, and its
host-only table / quantum routines agree with the oracle (no GPU needed)."""
import os
import re

import numpy as np
import pytest

import paper_2401_02896_amd as L
from oracle import quanta
from tests.golden.make_knot_tables import TABLES, load

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KIND_ID = {"cubic": 0, "wendland": 1, "wendland_c4": 2, "wendland_c6": 3, "wendland_grad": 4,
           "wendland_c4_grad": 5, "wendland_c6_grad": 6}


def test_every_declared_symbol_is_exported():
    hdr = open(os.path.join(ROOT, "include", "sph_hoa.h")).read()
    names = sorted(set(re.findall(r"\b(sph_hoa_[a-z_]+)\s*\(", hdr)))
    assert len(names) >= 12
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(L.EXPORTS) <= set(names)


def test_status_strings():
    lib = L.lib()
    for s in range(9):
        assert lib.sph_hoa_status_string(s)
        assert lib.sph_hoa_status_string(s) != b"unknown status"


def test_build_rejects_bad_params_before_device_work():
    """Parameter checks run on the host before any device call: both table precisions at once,
    unknown flag bits, and an out-of-range degree are refused with E_INVALID_ARG."""
    import ctypes

    lib = L.lib()
    buf = (ctypes.c_float * 12)()
    for flags, degree in ((L.FLAG_LUT_FP32 | L.FLAG_LUT_BF16, 2), (L.FLAG_LUT_BF16 | L.FLAG_LUT_FP16, 2), (128, 2),
                          (L.FLAG_TRANSVERSE_X | L.FLAG_TRANSVERSE_Z, 2), (0, 9)):
        p = L.Params(degree, 4, 64, 64, 1e-3, 0.0, 0.0, 0.0, 0.0, None, flags)
        h = ctypes.c_void_p()
        st = lib.sph_hoa_build_index(buf, buf, buf, 4, 0, ctypes.byref(p), None, ctypes.byref(h))
        assert L.STATUS[st] == "E_INVALID_ARG", (flags, degree)
        assert not h.value


@pytest.mark.parametrize("spec", [t for t in TABLES if t[3] <= 256 or t[:3] == ("cubic", 4, 2)])
def test_library_knot_tables_match_oracle(spec):
    """The library's own knot optimisation reproduces the oracle's tables (Sec. 3.4).

    Flat minima (E^2 below 1e-12 of the kernel norm, where the knots are not determined
    to more than a few digits) are compared on their error instead of their position.
    """
    kind, K, D, n = spec
    th, e2 = L.sph_hoa_knot_table(KIND_ID[kind], K, D, n)
    ref = load(*spec)
    d = np.abs(th / ref - 1).max(axis=1)
    flat = e2 < 1e-12 * 0.1
    assert np.all(d[~flat] < 1e-6), (np.argmax(d), d.max())


@pytest.mark.parametrize("spec", [t for t in TABLES if t[3] <= 256] + [("wendland", 4, 3, 4096)])
def test_library_projection_matches_oracle(spec):
    """For the same knots, the library's projection jumps (Sec. 3.3) equal the oracle's to the
    conditioning of the normal equations (grows with D; 1e-9 of the row's largest jump at D <= 3)."""
    from oracle import lut

    kind, K, D, n = spec
    theta = load(*spec)
    shat, smid, e2 = L.sph_hoa_lut_coefficients(KIND_ID[kind], K, D, theta)
    lams = lut.lambda_midpoints(kind, n)
    rows = sorted(set(list(range(0, n, max(1, n // 24))) + [n - 1]))
    tol = 1e-9 if D <= 3 else 1e-7
    for i in rows:
        ref, ref_mid = lut.difference_coefficients(kind, float(lams[i]), theta[i], K, D)
        scale = max(np.abs(ref).max(), np.abs(ref_mid).max())
        assert np.max(np.abs(shat[i] - ref)) <= tol * scale, (i, np.max(np.abs(shat[i] - ref)) / scale)
        assert np.max(np.abs(smid[i] - ref_mid)) <= tol * scale, i
        assert abs(e2[i] - lut.project(kind, float(lams[i]), theta[i], K, D)["E2"]) <= 1e-6 * e2[i] + 1e-25


@pytest.mark.parametrize("kind", list(KIND_ID))
@pytest.mark.parametrize("D", [1, 2, 3, 4, 6])
def test_library_tau_matches_oracle(kind, D):
    """The length quantum depends on the kernel through kappa and kappa' (App. A.4, A.5)."""
    r = quanta.fig4_sigma_ratio(kind)
    got = L.sph_hoa_optimal_tau(KIND_ID[kind], D, r, 0.7, 3.0)
    assert abs(got / (0.7 * quanta.optimal_tau(kind, D, r / 3.0)) - 1) < 1e-12
