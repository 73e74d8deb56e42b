"""The benchmark's assignment comparison (include/pairs_ab.h): the balanced
circular assignment and the straightforward triangular one (Section 5) must
both give the oracle's exact count."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads as w
from gpu_util import announce, dev
from paper_1901_11204_amd import build as B

pytestmark = pytest.mark.gpu


def ab_lib():
    L = ctypes.CDLL(B.AB_LIB)
    L.pairs_ab_count_i32.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 4 + [
        ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.pairs_ab_count_i32.restype = ctypes.c_int
    return L


def ab_count(variant, arrays, K):
    import torch
    x, y, z, r = dev(*arrays)
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    n = int(arrays[0].shape[0])
    rc = ab_lib().pairs_ab_count_i32(variant, x.data_ptr(), y.data_ptr(), z.data_ptr(),
                                     r.data_ptr(), n, K, out.data_ptr(),
                                     torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    return int(out.item())


@pytest.mark.parametrize("K", [1, 8])
@pytest.mark.parametrize("variant", [0, 1])
def test_ab_counts_match_oracle(variant, K):
    for n in [0, 1, 2, 3, 63, 64, 65, 511, 512, 513, 1000, 4097]:
        s = w.spheres_i32(n, 70 + n, 64, 6, radius_lo=0)
        announce("ab count", variant, K, n)
        assert ab_count(variant, s.arrays(), K) == oracle.count_i32(*s.arrays()), (variant, K, n)


def test_ab_variants_agree_on_spheres_4096():
    s = w.spheres_4096()
    want = oracle.count_i32(*s.arrays())
    for variant in (0, 1):
        for K in (1, 8):
            assert ab_count(variant, s.arrays(), K) == want


@pytest.mark.parametrize("K", [1, 8])
@pytest.mark.parametrize("variant", [0, 1])
def test_ab_timed_run_records_every_wave(variant, K):
    """The timed run gives the same count and a start no later than the end
    for every wave (row block) of the launch."""
    import torch
    L = ab_lib()
    L.pairs_ab_count_i32_timed.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 4 + [
        ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.pairs_ab_count_i32_timed.restype = ctypes.c_int
    L.pairs_ab_waves.argtypes = [ctypes.c_int64, ctypes.c_int]
    L.pairs_ab_waves.restype = ctypes.c_int64
    s = w.spheres_i32(5000, 77, 64, 6, radius_lo=0)
    n = 5000
    waves = L.pairs_ab_waves(n, K)
    assert waves == (n + 64 * K - 1) // (64 * K)
    x, y, zz, r = dev(*s.arrays())
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    times = torch.zeros(2 * waves, dtype=torch.int64, device="cuda")
    announce("ab timed", variant, K)
    rc = L.pairs_ab_count_i32_timed(variant, x.data_ptr(), y.data_ptr(), zz.data_ptr(),
                                    r.data_ptr(), n, K, out.data_ptr(), times.data_ptr(),
                                    torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    torch.cuda.synchronize()
    assert int(out.item()) == oracle.count_i32(*s.arrays())
    t = times.cpu().numpy().reshape(-1, 2)
    assert np.all(t[:, 0] > 0) and np.all(t[:, 1] >= t[:, 0])
    khz = ctypes.c_int64(0)
    assert L.pairs_ab_wall_clock_khz(ctypes.byref(khz)) == 0 and khz.value > 0
