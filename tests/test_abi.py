"""The C-ABI library: it loads, exports every symbol include/furax.h declares,
and rejects invalid arguments before any launch (no compute without a GPU)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "furax.h")
LIB = os.path.join(ROOT, "paper_2603_19600_amd", "libfurax.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(furax_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2603_19600_amd import build
        build.build()
    from paper_2603_19600_amd import furax
    return furax


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("furax_ang2pix", "furax_pointing_apply", "furax_pointing_transpose",
              "furax_noise_apply", "furax_pcg_mapmake", "furax_pointing_vjp",
              "furax_chi2_grad"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (furax_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    assert set(lib.EXPORTS) == set(_declared())
    for n in _declared():
        getattr(lib.library(), n)


def test_validation_happens_before_any_launch(lib):
    L = lib.library()
    P = lib._Pointing(0, 1, 10, lib.F64, 1, 1, 1, None, None, 0, 0, 1, 0.0)   # nside 0
    assert L.furax_pointing_apply(C.byref(P), lib.F64, 1, lib.F64, 1, None) == lib.EINVAL
    assert b"nside" in L.furax_last_error()
    P.nside = 16
    P.theta = None                                                              # NULL plane
    assert L.furax_pointing_apply(C.byref(P), lib.F64, 1, lib.F64, 1, None) == lib.EINVAL
    P.theta = 1
    assert L.furax_pointing_apply(C.byref(P), lib.F32, 1, lib.F64, 1, None) == lib.EINVAL
    P.hwp, P.hwp_den = 1, 0                                                     # bad HWP law
    assert L.furax_pointing_transpose(C.byref(P), lib.F64, 1, 1, 0, None) == lib.EINVAL
    P.hwp, P.hwp_den = 0, 1
    N = lib._Noise(1, 1, 11, None, 4, 1, 0)                                     # n_samp mismatch
    assert L.furax_normal_apply(C.byref(P), C.byref(N), lib.F64, 1, 1, None, None, None) \
        == lib.EINVAL
    N.n_samp = 10
    N.bandwidth = 11                                                            # b > n_samp
    assert L.furax_noise_apply(C.byref(N), lib.F64, 1, 2, None) == lib.EINVAL
    N.bandwidth, N.n_samp = 8193, 100000                                        # band limit
    N2 = lib._Noise(1, 1, 100000, None, 8193, 1, 0)
    assert L.furax_noise_apply(C.byref(N2), lib.F64, 1, 2, None) == lib.EUNSUPPORTED
    assert L.furax_noise_apply(C.byref(N2), lib.F32, 1, 2, None) == lib.EUNSUPPORTED
    N3 = lib._Noise(1, 1, 100, None, 4, 1, 0)                                   # aliasing in/out
    assert L.furax_noise_apply(C.byref(N3), lib.F64, 16, 16, None) == lib.EINVAL
    opts = lib._PcgOpts(-1, 0.0, lib.F64, 1e-3, 3, None, 0)                    # max_iter < 0
    info = lib._PcgInfo()
    Nd = lib._Noise(0, 1, 10, 1, 0, None, 0)
    assert L.furax_pcg_mapmake(C.byref(P), C.byref(Nd), lib.F64, 1, 1, None, C.byref(opts),
                               C.byref(info), None) == lib.EINVAL
    assert L.furax_ang2pix(9000, lib.F64, 1, 1, 4, 1, None) == lib.EINVAL
    # chi2 gradient: NULL map, band noise, FP64 pointing with an FP32 map
    assert L.furax_chi2_grad(C.byref(P), C.byref(Nd), lib.F64, None, 1, None, 1, None, None,
                             None) == lib.EINVAL
    Nb = lib._Noise(1, 1, 10, None, 4, 1, 0)
    assert L.furax_chi2_grad(C.byref(P), C.byref(Nb), lib.F64, 1, 1, None, 1, None, None,
                             None) == lib.EUNSUPPORTED
    assert L.furax_chi2_grad(C.byref(P), C.byref(Nd), lib.F32, 1, 1, None, 1, None, None,
                             None) == lib.EINVAL
    assert L.furax_pcg_iterate(None, 1) == lib.EINVAL
    assert L.furax_version() >= 100
