"""The matrix-core ceiling measurement (libmc3ceil.so) on the GPU: a short run reports
a positive rate no higher than the published dense BF16 peak at the clock it measured
(small tolerance for timer resolution), and a clock within the device's range."""
import pytest

from gpu_helpers import announce
from paper_2102_05613_amd import native

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.ceiling_lib()


def test_mfma_ceiling_bounds():
    announce("mfma ceiling")
    r = native.mfma_ceiling(iters=2500, blocks=256, repeats=2)
    assert 0.5 < r["clock_ghz"] < 2.6
    assert 0.0 < r["tflops"] <= 2500.0 * r["clock_ghz"] / 2.4 * 1.02


def test_mfma_mix_orders():
    """LDS traffic in the loop costs matrix-core rate: no traffic >= 16 reads >= 32
    reads per 64 MFMAs (2% slack for timing noise), and every rate is positive."""
    announce("mfma mix")
    r = {m: native.mfma_mix(m, iters=2500, repeats=2) for m in native.MFMA_MIXES}
    assert all(v > 0.0 for v in r.values())
    assert r[0] * 1.02 >= r[4] and r[4] * 1.02 >= r[3]


def test_mfma_ceiling_rejects_bad_arguments():
    import ctypes
    t, g = ctypes.c_double(), ctypes.c_double()
    L = native.ceiling_lib()
    assert L.mc3c_mfma_ceiling(0, 256, 1, ctypes.byref(t), ctypes.byref(g)) == -1
    assert L.mc3c_mfma_ceiling(10, 0, 1, ctypes.byref(t), ctypes.byref(g)) == -1
    assert L.mc3c_mfma_ceiling(10, 256, 0, ctypes.byref(t), ctypes.byref(g)) == -1
    assert L.mc3c_mfma_mix(5, 10, 1, ctypes.byref(t)) == -1
    assert L.mc3c_mfma_mix(0, 0, 1, ctypes.byref(t)) == -1
