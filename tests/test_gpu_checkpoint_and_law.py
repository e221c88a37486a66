"""Checkpoint/resume, and the sampled law of the GPU chains.

Bars: a run resumed from a checkpoint in a new context reproduces the original's
records and final state bit for bit (pair-sum and field-update scorers); after
burn-in, the states of many independent GPU chains at N = 10 follow the exact
Boltzmann law (chi-square over all 2^10 states, pooled below 5 expected)."""
import numpy as np
import pytest

from exact_tools import all_energies, boltzmann
from gpu_helpers import announce
from paper_2102_05613_amd import inputs, native
from test_oracle_chain import _chi2_pass

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()


def _make(N, M, chains, kmin, kmax, J, scale, steps, **kw):
    cfg = native.make_config(N, M, chains, kmin, kmax, trace_steps=steps, seed=12, **kw)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    return ctx


@pytest.mark.parametrize("kw", [dict(precision="split_bf16"), dict(precision="fp64", scorer="delta"),
                                dict(precision="fp64", arity=2)])
def test_checkpoint_resume_bit_exact(kw):
    N, M, chains, n1, n2 = 300, 14, 6, 40, 60
    announce(f"checkpoint {kw}")
    J, scale = inputs.couplings_gauss(N, 77)
    a = _make(N, M, chains, 1, 3, J, scale, n2, **kw)
    a.init_chains()
    a.step_n(0, n1, 0.2, 2.0, n1 + n2)
    blob = a.checkpoint_save()
    a.step_n(n1, n2, 0.2, 2.0, n1 + n2)
    ra = a.read_records(n1, n2)
    ea, ba, sa = a.measure()
    b = _make(N, M, chains, 1, 3, J, scale, n2, **kw)
    b.checkpoint_load(blob)
    b.step_n(n1, n2, 0.2, 2.0, n1 + n2)
    rb = b.read_records(n1, n2)
    eb, bb, sb = b.measure()
    assert np.array_equal(ra, rb)
    assert np.array_equal(ea, eb) and np.array_equal(ba, bb)
    assert sa["steps_done"] == sb["steps_done"] == n1 + n2
    assert sa["moves"] == sb["moves"]
    # a checkpoint of another shape is refused
    c = _make(N, M + 1, chains, 1, 3, J, scale, 0, **kw)
    with pytest.raises(native.MC3Error) as ei:
        c.checkpoint_load(blob)
    assert ei.value.status == native.MC3_E_ARG
    with pytest.raises(native.MC3Error):
        c.checkpoint_load(b"\0" * len(blob))


@pytest.mark.parametrize("name,kw,M,kmin,kmax", [
    ("star, pair sums FP64", dict(precision="fp64"), 4, 1, 2),
    ("binary tree, field update", dict(precision="fp64", scorer="delta", arity=2), 6, 1, 1),
    ("line process, split BF16", dict(precision="split_bf16", arity=1, law="line"), 5, 1, 1),
    ("Metropolis, field update", dict(precision="fp64", scorer="delta", rule="metropolis"), 1, 1, 1)])
def test_states_follow_boltzmann(name, kw, M, kmin, kmax):
    N, chains, steps, beta = 10, 32768, 300, 1.0
    announce(f"Boltzmann law: {name}")
    J, scale = inputs.couplings_gauss(N, 55)
    cfg = native.make_config(N, M, chains, kmin, kmax, seed=3, **kw)
    ctx = native.Context(cfg)
    ctx.init_couplings(J, scale)
    ctx.init_chains()
    ctx.step_n(0, steps, beta, beta, 1)
    _, bits, _ = ctx.measure()
    states = bits[:, 0].astype(np.int64)
    pi = boltzmann(all_energies(J, scale), beta)
    counts = np.bincount(states, minlength=2 ** N)
    stat, dof = _chi2_pass(counts, pi, chains)
    assert stat < dof + 6 * np.sqrt(2 * dof), (name, stat, dof)
    # the test can tell: the same samples against the law at another temperature fail
    stat_w, dof_w = _chi2_pass(counts, boltzmann(all_energies(J, scale), 1.3 * beta), chains)
    assert stat_w > dof_w + 6 * np.sqrt(2 * dof_w), (name, stat_w, dof_w)
