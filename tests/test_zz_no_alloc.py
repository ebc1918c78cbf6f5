"""GPU: furax_chi2_grad_noalloc, the chi-square gradient that allocates nothing
(its partial sums live in the library's static device scratch), against
furax_chi2_grad on the same inputs, called through the C ABI: two calls in a
row, the second on a smaller problem, and a problem too large for the scratch
rejected before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2603_19600_amd import synth
from tests.gpu_util import case, dev, rel_err, to_pointing

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fx():
    from paper_2603_19600_amd import furax
    return furax


def _inputs(fx, nside, n_det, n_samp, dtype, seed):
    w, h, t = case(nside, n_det, n_samp, seed=seed, dtype=dtype, hwp=True, gains=True, dpsi=True)
    P = to_pointing(nside, t)
    iv = torch.linspace(0.5, 2.0, n_det, dtype=torch.float64, device=dev())
    N = fx.Noise("diag", n_det, n_samp, inv_var=iv)
    g = torch.Generator(device=dev()).manual_seed(seed)
    m = torch.randn(3, w.npix, dtype=torch.float64, device=dev(), generator=g)
    d = torch.randn(n_det, n_samp, dtype=P.dtype, device=dev(), generator=g)
    return P, N, m, d


def _call(fx, name, P, N, m, d):
    L = fx.library()
    gm = torch.zeros(3, P.npix, dtype=torch.float64, device=dev())
    gg = torch.empty(P.n_det, dtype=torch.float64, device=dev())
    gd = torch.empty(P.n_det, dtype=torch.float64, device=dev())
    c2 = torch.empty((), dtype=torch.float64, device=dev())
    cp, cn = P.c(), N.c()
    st = getattr(L, name)(C.byref(cp), C.byref(cn), fx.F64, m.data_ptr(), d.data_ptr(),
                          c2.data_ptr(), gm.data_ptr(), gg.data_ptr(), gd.data_ptr(),
                          torch.cuda.current_stream().cuda_stream)
    assert st == fx.OK, L.furax_last_error()
    torch.cuda.synchronize()
    return gm, gg, gd, c2


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_chi2_grad_on_two_calls(fx, dtype):
    for shape, seed in (((64, 8, 300000), 1), ((32, 3, 5001), 2)):   # the second is smaller
        P, N, m, d = _inputs(fx, *shape, dtype, seed)
        gm, gg, gd, c2 = _call(fx, "furax_chi2_grad_noalloc", P, N, m, d)
        rm, rg, rd, rc = _call(fx, "furax_chi2_grad", P, N, m, d)
        # the same kernels with fixed-order per-detector and chi-square sums: bitwise
        assert torch.equal(gg, rg) and torch.equal(gd, rd) and torch.equal(c2, rc)
        # the map gradient's tile flushes are FP64 atomics: equal up to summation order
        assert rel_err(gm.cpu().numpy(), rm.cpu().numpy()) <= 1e-12
        assert float(gm.abs().sum()) > 0


def test_noalloc_rejects_a_problem_beyond_its_scratch(fx):
    """1024 detectors x 65536 samples need 2^21 + 4096 partial sums."""
    P, N, m, d = _inputs(fx, 64, 1024, 65536, "f32", 3)
    L = fx.library()
    gm = torch.zeros(3, P.npix, dtype=torch.float64, device=dev())
    gg = torch.full((P.n_det,), 7.0, dtype=torch.float64, device=dev())
    cp, cn = P.c(), N.c()
    st = L.furax_chi2_grad_noalloc(C.byref(cp), C.byref(cn), fx.F64, m.data_ptr(), d.data_ptr(),
                                   None, gm.data_ptr(), gg.data_ptr(), None,
                                   torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert st == fx.EUNSUPPORTED
    assert b"static scratch" in L.furax_last_error()
    assert float(gm.abs().sum()) == 0.0 and bool((gg == 7.0).all())
