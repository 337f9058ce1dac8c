"""The LDS increment probe behind the vote's measured ceilings: each pattern
(conflict-free, hashed, the vote's own) runs, keeps every increment and
reports a positive rate."""
import ctypes
import os

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def probe():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2212_09460_amd", "liblaneprobe.so"))
    f = lib.lane_probe_lds_add
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_uint64)]
    return f


@pytest.mark.parametrize("pattern", [0, 1, 2])
def test_probe_counts_every_increment(probe, pattern):
    print("[case] LDS probe pattern", pattern, flush=True)
    groups, steps = 512, 20
    rate, chk = ctypes.c_double(0.0), ctypes.c_uint64(0)
    assert probe(groups, steps, pattern, ctypes.byref(rate), ctypes.byref(chk)) == 0
    assert chk.value == groups * 1024 * 16 * steps
    assert rate.value > 0
