"""The sweep's own logarithms (log_fast and log1p_fast, evaluated on the
device by the probe library) against the host C library's log and log1p: at
most 3 ulp apart over the skip's whole domain, U in (0, 1] (the 53-bit
uniforms of the sampler, end points included) and t_q from 1e-300 to 1e300.
The skip length floor(-log U / log1p(t_q)) can only differ between host and
device where the quotient lies within a few ulp of an integer: far inside the
1e-12 margin of the oracle's near-tie trace.  The Chung-Lu chain's log1p of
negative arguments (-t_q, t_q in (0, 1)) is checked the same way."""
import ctypes
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MAX_ULP = 3


@pytest.fixture(scope="module")
def probe():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2509_13230_amd as mh

    path = os.path.join(os.path.dirname(mh.__file__), "libmh_probe.so")
    P = ctypes.CDLL(path)
    P.mhp_sweep_logs.restype = ctypes.c_int
    P.mhp_sweep_logs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p]
    return P


def device_logs(P, u, t):
    ud = torch.as_tensor(np.ascontiguousarray(u, np.float64)).cuda()
    td = torch.as_tensor(np.ascontiguousarray(t, np.float64)).cuda()
    a = torch.empty_like(ud)
    b = torch.empty_like(td)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert P.mhp_sweep_logs(ud.data_ptr(), td.data_ptr(), ud.numel(), a.data_ptr(), b.data_ptr(), stream) == 0
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def ulps(got, ref):
    ref = np.asarray(ref)
    sp = np.spacing(np.abs(ref))
    sp = np.where(ref == 0, np.spacing(0.0), sp)
    return np.abs(got - ref) / sp


def test_sweep_logs_within_3_ulp(probe):
    rng = np.random.default_rng(17)
    n = 1 << 20
    # the sampler's uniforms: (((a << 21) | (b >> 11)) + 1) 2^-53 from 32-bit words
    w = rng.integers(0, 1 << 53, n, dtype=np.int64)
    u = (w + 1).astype(np.float64) * 2.0**-53
    u[:8] = [2.0**-53, 2.0**-52, 0.5, np.nextafter(0.5, 1), np.sqrt(0.5), np.nextafter(np.sqrt(0.5), 0),
             1.0 - 2.0**-53, 1.0]
    t = 10.0 ** rng.uniform(-300, 300, n)
    t[:12] = [0.0, 1e-300, 2.0**-53, 2.0**-52, 1e-17, 1e-8, 0.5, 1.0, 2.0, 1e6, 1e300, np.finfo(np.float64).max / 2]
    # t from 1e-300 to 1e6, densely: the proposal's t_q of a sparse row
    t[n // 2:] = 10.0 ** rng.uniform(-300, 6, n - n // 2)
    lg, lp = device_logs(probe, u, t)
    ref_lg = np.array([math.log(v) for v in u])
    ref_lp = np.array([math.log1p(v) for v in t])
    e1, e2 = ulps(lg, ref_lg), ulps(lp, ref_lp)
    assert e1.max() <= MAX_ULP, (e1.max(), u[np.argmax(e1)])
    assert e2.max() <= MAX_ULP, (e2.max(), t[np.argmax(e2)])
    # exact where the result is exact: log 1 = 0; log1p(t) = t below 2^-53 relative
    assert lg[7] == 0.0
    assert lp[0] == 0.0 and lp[1] == 1e-300


def test_log1p_of_negative_arguments_within_3_ulp(probe):
    # the Chung-Lu skip takes -log1p(-t_q) for t_q in (0, 1)
    rng = np.random.default_rng(18)
    n = 1 << 18
    t = -(10.0 ** rng.uniform(-300, 0, n))
    t = np.maximum(t, -(1.0 - 2.0**-53))
    t[:6] = [-1e-300, -2.0**-53, -0.5, -0.9, -(1.0 - 2.0**-53), -0.29289321881345254]
    u = np.full(n, 0.5)
    _, lp = device_logs(probe, u, t)
    ref = np.array([math.log1p(v) for v in t])
    e = ulps(lp, ref)
    assert e.max() <= MAX_ULP, (e.max(), t[np.argmax(e)])
