"""Seeded couplings generated on the device (mc3_generate_couplings) against the
oracle's generator of the same definition: +-1 instances give a trajectory equal to
the oracle's record for record (integer energies, no guidance); Gaussian instances
give candidate energies within the path's tolerance of the oracle's energies on the
oracle's couplings (the device's log and cos may differ from the host's by an ulp)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import announce, compare_trajectory, eps_energy, gpu_spins, oracle_candidates
from paper_2102_05613_amd import native

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    native.lib()


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_pm1_generated_trajectory_equals_oracle(prec):
    N, M, chains, steps, seed = 32, 4, 1, 3000, 0xC0FFEE
    announce(f"generated pm1 couplings trajectory {prec}")
    cfg = native.make_config(N, M, chains, 1, 1, precision=prec, trace_steps=steps, seed=4)
    ctx = native.Context(cfg)
    scale = ctx.generate_couplings(native.MC3_J_PM1, seed)
    ctx.init_chains()
    ctx.step_n(0, steps, 1.0, 1.0, 1)
    rec = ctx.read_records(0, steps)
    ctx.close()
    J, scale_o = oracle.couplings(N, oracle.COUPLINGS_PM1, seed)
    assert scale == scale_o
    compare_trajectory(rec, J, scale, N, M, chains, 1, 1, 4, np.ones(steps), "mcmcmc", 0.0, exact=True)


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
@pytest.mark.parametrize("N,M,chains,kmax", [(256, 16, 4, 4), (1000, 17, 3, 100)])
def test_gauss_generated_energies_match_oracle(prec, N, M, chains, kmax):
    import torch
    seed = 0xBEEF + N
    announce(f"generated gauss couplings N={N} {prec}")
    cfg = native.make_config(N, M, chains, 1, kmax, precision=prec, seed=6)
    ctx = native.Context(cfg)
    scale = ctx.generate_couplings(native.MC3_J_GAUSS, seed)
    ctx.init_chains()
    s = gpu_spins(ctx)
    ctx.propose(7)
    E = torch.zeros(chains * M, dtype=torch.float64, device="cuda")
    ctx.score_candidates(E)
    Eg = E.cpu().numpy().reshape(chains, M)
    ctx.close()
    J, scale_o = oracle.couplings(N, oracle.COUPLINGS_GAUSS, seed)
    assert scale == scale_o == 1.0
    for c in range(chains):
        _, cols = oracle_candidates(6, c, 7, N, M, 1, kmax, s[c])
        Eo = np.array([oracle.energy(J, scale, x) for x in cols])
        np.testing.assert_allclose(Eg[c], Eo, rtol=0, atol=eps_energy(prec, N))


def test_generated_couplings_reject_bad_arguments():
    cfg = native.make_config(64, 4, 2, 1, 2, precision="fp64", seed=1)
    ctx = native.Context(cfg)
    assert native.lib().mc3_generate_couplings(ctx.h, 0, 2, 1) == native.MC3_E_ARG
    assert native.lib().mc3_generate_couplings(ctx.h, 1, 0, 1) == native.MC3_E_ARG
    ctx.close()
