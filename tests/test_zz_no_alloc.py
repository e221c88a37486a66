"""mc3_create_noalloc: a context whose workspace is the library's fixed device array
(for callers that cannot allocate) runs exactly as one made by mc3_create.

Bar: records, states, energies and counters equal those of an mc3_create context bit
for bit (the same kernels on the same inputs), on two contexts in a row on the same
array, the second one smaller; a configuration beyond the array is refused; a second
live context on the same device is refused."""
import numpy as np
import pytest

from gpu_helpers import announce
from paper_2102_05613_amd import inputs, native

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()


def _run(cfg, J, scale, steps, noalloc):
    ctx = native.Context(cfg, noalloc=noalloc)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    ctx.step_n(0, steps, 0.4, 1.6, steps)
    rec = ctx.read_records(0, steps)
    e, bits, summ = ctx.measure()
    return ctx, (rec, e, bits, summ)


def test_noalloc_context_equals_regular_twice_second_smaller():
    # the first configuration is large enough to fill much of the array, the second smaller
    cases = [((600, 24, 40, 1, 8), "split_bf16", 30), ((64, 4, 2, 1, 2), "fp64", 50)]
    for (N, M, chains, kmin, kmax), prec, steps in cases:
        announce(f"noalloc N={N} M={M} chains={chains} {prec}")
        J, scale = inputs.couplings_gauss(N, 4000 + N)
        cfg = native.make_config(N, M, chains, kmin, kmax, precision=prec, trace_steps=steps, seed=8,
                                 recompute_every=10)
        assert native.workspace_size(cfg) <= native.NOALLOC_BYTES
        ref_ctx, ref = _run(cfg, J, scale, steps, noalloc=False)
        ref_ctx.close()
        ctx, got = _run(cfg, J, scale, steps, noalloc=True)
        assert np.array_equal(got[0], ref[0])
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
        assert got[3] == ref[3]
        assert got[3]["moves"] > 0
        # one live context per device on the array
        with pytest.raises(native.MC3Error) as ei:
            native.Context(cfg, noalloc=True)
        assert ei.value.status == native.MC3_E_STATE
        ctx.close()


def test_noalloc_refuses_configs_beyond_the_array():
    cfg = native.make_config(1024, 128, 256, 1, 128, precision="split_bf16")
    assert native.workspace_size(cfg) > native.NOALLOC_BYTES
    with pytest.raises(native.MC3Error) as ei:
        native.Context(cfg, noalloc=True)
    assert ei.value.status == native.MC3_E_WORKSPACE
    # the refusal leaves the array free
    small = native.make_config(32, 4, 1, 1, 1, precision="fp64")
    native.Context(small, noalloc=True).close()
