"""CPU-only checks of the C ABI: the library loads, exports every declared symbol,
its structs match the header, and configuration/workspace validation happens before
any HIP call (so these run on a host without a GPU)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2102_05613_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mc3.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(native.LIB_PATH):
        from paper_2102_05613_amd import build
        build.build()
    return native.lib()


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mc3_[a-z_0-9]+)\s*\(", txt)))


def test_ceiling_library_exports_its_declared_symbol():
    """libmc3ceil.so loads without a GPU and exports what include/mc3_ceiling.h declares."""
    if not os.path.exists(native.CEIL_PATH):
        from paper_2102_05613_amd import build
        build.build()
    txt = open(os.path.join(ROOT, "include", "mc3_ceiling.h")).read()
    names = sorted(set(re.findall(r"\b(mc3c_[a-z_0-9]+)\s*\(", txt)))
    assert names == sorted(native.CEIL_EXPORTS)
    L = native.ceiling_lib()
    for n in names:
        assert hasattr(L, n), n


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert names == sorted(native.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", native.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mc3_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_header():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "mc3.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(mc3_config), offsetof(mc3_config, seed),
         offsetof(mc3_config, near_tie_tol), sizeof(mc3_record), offsetof(mc3_record, margin), sizeof(mc3_summary));
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(mc3_instance_desc), sizeof(mc3_batch_config),
         offsetof(mc3_batch_config, chain_base), offsetof(mc3_batch_config, seed),
         offsetof(mc3_batch_config, instances), offsetof(mc3_batch_config, scorer), offsetof(mc3_config, scorer));
  printf("%zu %zu %zu %zu\n", offsetof(mc3_config, arity), offsetof(mc3_config, law),
         offsetof(mc3_batch_config, arity), offsetof(mc3_batch_config, law));
  printf("%zu %zu\n", offsetof(mc3_config, law_table), offsetof(mc3_batch_config, law_table));
  printf("%zu %zu\n", offsetof(mc3_config, tile_cols), offsetof(mc3_batch_config, tile_cols));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(mc3_config, recompute_every), offsetof(mc3_config, energy_update),
         offsetof(mc3_config, drift_tol), offsetof(mc3_batch_config, recompute_every),
         offsetof(mc3_batch_config, energy_update), offsetof(mc3_batch_config, drift_tol));
  printf("%zu %zu %zu\n", offsetof(mc3_summary, recomputes), offsetof(mc3_summary, drift_events),
         sizeof(mc3_schedule));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        vals = [int(x) for x in subprocess.check_output([exe]).split()]
    assert vals == [ctypes.sizeof(native.Config), native.Config.seed.offset, native.Config.near_tie_tol.offset,
                    native.RECORD_DTYPE.itemsize, native.RECORD_DTYPE.fields["margin"][1],
                    ctypes.sizeof(native.Summary),
                    ctypes.sizeof(native.InstanceDesc), ctypes.sizeof(native.BatchConfig),
                    native.BatchConfig.chain_base.offset, native.BatchConfig.seed.offset,
                    native.BatchConfig.instances.offset, native.BatchConfig.scorer.offset,
                    native.Config.scorer.offset, native.Config.arity.offset, native.Config.law.offset,
                    native.BatchConfig.arity.offset, native.BatchConfig.law.offset,
                    native.Config.law_table.offset, native.BatchConfig.law_table.offset,
                    native.Config.tile_cols.offset, native.BatchConfig.tile_cols.offset,
                    native.Config.recompute_every.offset, native.Config.energy_update.offset,
                    native.Config.drift_tol.offset, native.BatchConfig.recompute_every.offset,
                    native.BatchConfig.energy_update.offset, native.BatchConfig.drift_tol.offset,
                    native.Summary.recomputes.offset, native.Summary.drift_events.offset,
                    ctypes.sizeof(native.Schedule)]


def test_version(lib):
    assert b"gfx950" in lib.mc3_version()


@pytest.mark.parametrize("kw", [dict(N=1), dict(N=8193), dict(M=0), dict(chains=0), dict(kmin=0),
                                dict(kmin=3, kmax=2), dict(kmax=65), dict(M=2, rule="metropolis"),
                                dict(trace_steps=-1), dict(mean_steps=-1), dict(M=4001), dict(chains=70000, M=256)])
def test_invalid_configs_rejected(lib, kw):
    base = dict(N=64, M=4, chains=2, kmin=1, kmax=4)
    rule = kw.pop("rule", "mcmcmc")
    base.update(kw)
    cfg = native.make_config(rule=rule, **base)
    n = ctypes.c_size_t()
    assert lib.mc3_workspace_size(ctypes.byref(cfg), ctypes.byref(n)) == native.MC3_E_ARG
    h = ctypes.c_void_p()
    assert lib.mc3_create(ctypes.byref(cfg), None, 0, None, ctypes.byref(h)) == native.MC3_E_ARG


def test_workspace_size_and_missing_workspace(lib):
    cfg = native.make_config(1024, 128, 256, 1, 128, precision="split_bf16", trace_steps=10)
    n = native.workspace_size(cfg)
    # J64 (8 MiB) + split J (6 MiB) + a ring of 17 steps of flip sets (4 MiB each) + ...
    assert 18 * 2 ** 20 + 17 * 4 * 2 ** 20 < n < 128 * 2 ** 20
    cfg2 = native.make_config(1024, 128, 512, 1, 128, precision="split_bf16", trace_steps=10)
    assert native.workspace_size(cfg2) > n
    h = ctypes.c_void_p()
    assert lib.mc3_create(ctypes.byref(cfg), None, n, None, ctypes.byref(h)) == native.MC3_E_WORKSPACE
    assert lib.mc3_create(ctypes.byref(cfg), ctypes.c_void_p(256), n - 1, None, ctypes.byref(h)) == native.MC3_E_WORKSPACE
    assert lib.mc3_create(ctypes.byref(cfg), ctypes.c_void_p(4096 + 8), n, None, ctypes.byref(h)) == native.MC3_E_WORKSPACE


def test_null_context_calls(lib):
    assert lib.mc3_destroy(None) == native.MC3_E_ARG
    assert lib.mc3_propose(None, 0) == native.MC3_E_ARG
    assert lib.mc3_sync(None) == native.MC3_E_ARG
    assert lib.mc3_last_error(None) == b"context is NULL"


def test_bitset_helpers_roundtrip():
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(0))
    s = np.where(rng.random((3, 77)) < 0.5, -1, 1).astype(np.int8)
    assert np.array_equal(native.bits_to_spins(native.spins_to_bits(s), 77), s)


def _batch_ws(lib, cfg):
    n = ctypes.c_size_t()
    return lib.mc3_batch_workspace_size(ctypes.byref(cfg), ctypes.byref(n)), n.value


def test_batch_single_instance_matches_single_config(lib):
    for prec in ("fp64", "split_bf16"):
        for shape in [(64, 4, 2, 1, 4), (1024, 128, 256, 1, 128), (8192, 1024, 32, 256, 256)]:
            single = native.workspace_size(native.make_config(*shape, precision=prec, trace_steps=3, mean_steps=5))
            st, n = _batch_ws(lib, native.make_batch_config([shape], precision=prec, trace_steps=3, mean_steps=5))
            assert st == native.MC3_OK and n == single


def test_batch_workspace_grows_with_instances(lib):
    one = (64, 8, 4, 1, 8)
    sizes = []
    for k in (1, 2, 10, 2000):
        st, n = _batch_ws(lib, native.make_batch_config([one] * k, precision="split_bf16"))
        assert st == native.MC3_OK
        sizes.append(n)
    assert sizes == sorted(sizes) and sizes[-1] < 2000 * sizes[0] + 2 ** 20


@pytest.mark.parametrize("bad", [dict(N=1), dict(M=0), dict(kmax=65), dict(chains=0), dict(M=2, rule="metropolis")])
def test_batch_rejects_any_invalid_instance(lib, bad):
    good = dict(N=64, M=4, chains=2, kmin=1, kmax=4)
    b = dict(good)
    rule = bad.pop("rule", "mcmcmc")
    b.update(bad)
    if rule == "metropolis":
        good = dict(good, M=1)
    descs = [tuple(good.values()), tuple(b.values()), tuple(good.values())]
    cfg = native.make_batch_config(descs, rule=rule)
    assert _batch_ws(lib, cfg)[0] == native.MC3_E_ARG
    h = ctypes.c_void_p()
    assert lib.mc3_batch_create(ctypes.byref(cfg), None, 0, None, ctypes.byref(h)) == native.MC3_E_ARG


def test_batch_rejects_bad_header_fields(lib):
    descs = [(64, 4, 2, 1, 4)]
    cfg = native.make_batch_config(descs)
    cfg.n_instances = 0
    assert _batch_ws(lib, cfg)[0] == native.MC3_E_ARG
    cfg = native.make_batch_config(descs)
    cfg.instances = ctypes.POINTER(native.InstanceDesc)()
    assert _batch_ws(lib, cfg)[0] == native.MC3_E_ARG
    cfg = native.make_batch_config(descs, chain_base=2 ** 28 - 1)
    assert _batch_ws(lib, cfg)[0] == native.MC3_E_ARG
    cfg = native.make_batch_config(descs, trace_steps=-2)
    assert _batch_ws(lib, cfg)[0] == native.MC3_E_ARG
    assert lib.mc3_init_couplings_instance(None, 0, None, 0, 1.0) == native.MC3_E_ARG
    assert lib.mc3_step_n_per_instance(None, 0, 1, 1.0, 1.0, 1) == native.MC3_E_ARG


@pytest.mark.parametrize("shape,scorer,arity,expect", [
    ((64, 4, 2, 1, 16), "delta", 0, native.MC3_OK),
    # beyond the small-flip kernel: stars go to the kernel for flip sets of any size
    ((64, 4, 2, 1, 17), "delta", 0, native.MC3_OK), ((4097, 4, 2, 1, 2), "delta", 0, native.MC3_OK),
    ((3000, 4, 2, 1, 2), "delta", 0, native.MC3_OK), ((8192, 4, 2, 1, 2), "delta", 0, native.MC3_OK),
    ((64, 513, 2, 1, 2), "delta", 0, native.MC3_OK), ((1024, 128, 4, 1, 128), "delta", 0, native.MC3_OK),
    ((2048, 256, 4, 1, 128), "delta", 0, native.MC3_OK),              # the star kernel's state: 106 KiB
    ((8192, 64, 2, 1, 2), "delta", 0, native.MC3_E_UNSUPPORTED),      # 200 KiB: beyond 160 KiB
    ((4096, 512, 2, 1, 16), "delta", 0, native.MC3_E_UNSUPPORTED),   # LDS beyond either kernel's limit
    ((64, 14, 2, 1, 17), "delta", 2, native.MC3_E_UNSUPPORTED),      # a tree with large flip sets
    ((64, 4, 2, 1, 17), "auto", 0, native.MC3_OK), ((64, 4, 2, 1, 16), "gemm", 0, native.MC3_OK)])
def test_field_update_scorer_limits(lib, shape, scorer, arity, expect):
    cfg = native.make_config(*shape, precision="fp64", scorer=scorer, arity=arity)
    n = ctypes.c_size_t()
    assert lib.mc3_workspace_size(ctypes.byref(cfg), ctypes.byref(n)) == expect
    if expect == native.MC3_E_UNSUPPORTED:
        h = ctypes.c_void_p()
        assert lib.mc3_create(ctypes.byref(cfg), None, 0, None, ctypes.byref(h)) == expect


def test_unknown_scorer_rejected(lib):
    cfg = native.make_config(64, 4, 2, 1, 2)
    cfg.scorer = 7
    n = ctypes.c_size_t()
    assert lib.mc3_workspace_size(ctypes.byref(cfg), ctypes.byref(n)) == native.MC3_E_ARG


@pytest.mark.parametrize("kw,expect", [
    (dict(arity=2), native.MC3_OK), (dict(arity=1, law="line"), native.MC3_OK),
    (dict(arity=2, law="line"), native.MC3_E_ARG), (dict(arity=-1), native.MC3_E_ARG),
    (dict(arity=0, law="line"), native.MC3_E_ARG),
    # field update: a binary tree on 127 nodes has paths of 12 edges
    (dict(M=126, kmin=1, kmax=2, arity=2, scorer="delta"), native.MC3_OK),
    (dict(M=126, kmin=1, kmax=3, arity=2, scorer="delta"), native.MC3_E_UNSUPPORTED),
    (dict(M=127, kmin=1, kmax=1, arity=1, law="line", scorer="delta"), native.MC3_E_UNSUPPORTED),
    (dict(M=127, kmin=1, kmax=1, arity=1, law="line", scorer="auto"), native.MC3_OK),
    (dict(M=31, kmin=1, kmax=1, arity=1, law="line", scorer="delta"), native.MC3_OK)])
def test_graph_shape_validation(lib, kw, expect):
    base = dict(N=64, M=6, chains=2, kmin=1, kmax=1)
    for k in ("M", "kmin", "kmax"):
        if k in kw:
            base[k] = kw.pop(k)
    cfg = native.make_config(precision="fp64", **base, **kw)
    n = ctypes.c_size_t()
    assert lib.mc3_workspace_size(ctypes.byref(cfg), ctypes.byref(n)) == expect


@pytest.mark.parametrize("table,arity,expect", [
    ([0.2, 0.3, 0.1, 0.1, 0.1, 0.1, 0.1], 0, native.MC3_OK),
    ([0.2, 0.0, 0.1, 0.1, 0.1, 0.1, 0.1], 2, native.MC3_OK),
    ([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0], 1, native.MC3_OK),
    (None, 0, native.MC3_E_ARG),
    ([0.0] * 7, 0, native.MC3_E_ARG),
    ([0.2, -0.1, 0.1, 0.1, 0.1, 0.1, 0.1], 0, native.MC3_E_ARG),
    ([0.2, float("nan"), 0.1, 0.1, 0.1, 0.1, 0.1], 0, native.MC3_E_ARG),
    ([0.2, float("inf"), 0.1, 0.1, 0.1, 0.1, 0.1], 0, native.MC3_E_ARG)])
def test_table_law_validation(lib, table, arity, expect):
    cfg = native.make_config(64, 6, 2, 1, 1, precision="fp64", arity=arity, law="table", law_table=table)
    n = ctypes.c_size_t()
    assert lib.mc3_workspace_size(ctypes.byref(cfg), ctypes.byref(n)) == expect


def test_table_law_batch_validation(lib):
    """A batch's table holds every instance's M_i+1 weights in instance order; one bad
    instance rejects the batch."""
    descs = [(64, 3, 2, 1, 1), (128, 2, 1, 1, 2)]
    n = ctypes.c_size_t()
    good = native.make_batch_config(descs, precision="fp64", law="table",
                                    law_table=[1.0, 2.0, 3.0, 4.0, 0.5, 0.0, 0.5])
    assert lib.mc3_batch_workspace_size(ctypes.byref(good), ctypes.byref(n)) == native.MC3_OK
    bad = native.make_batch_config(descs, precision="fp64", law="table",
                                   law_table=[1.0, 2.0, 3.0, 4.0, 0.0, 0.0, 0.0])
    assert lib.mc3_batch_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == native.MC3_E_ARG


@pytest.mark.parametrize("kw,expect", [
    (dict(recompute_every=-1), native.MC3_E_ARG), (dict(drift_tol=float("nan")), native.MC3_E_ARG),
    (dict(recompute_every=100, drift_tol=1e-6), native.MC3_OK),
    (dict(law="biased", scorer="delta", bias=0.5), native.MC3_OK),
    (dict(law="biased", scorer="auto", bias=0.5), native.MC3_OK),
    (dict(law="biased", scorer="gemm", bias=0.5), native.MC3_E_ARG),
    (dict(law="biased", scorer="delta", bias=float("inf")), native.MC3_E_ARG),
    (dict(law="biased", scorer="delta", kmax=2), native.MC3_E_ARG),
    (dict(law="biased", scorer="delta", arity=2), native.MC3_E_ARG),
    (dict(law="biased", scorer="delta", rule="metropolis", M=1), native.MC3_E_ARG),
    (dict(law="biased", scorer="delta", N=1025), native.MC3_E_UNSUPPORTED),
    (dict(law="biased", scorer="delta", M=513), native.MC3_E_UNSUPPORTED)])
def test_energy_and_proposal_options_validated(lib, kw, expect):
    args = dict(N=64, M=4, chains=2, kmin=1, kmax=1, precision="fp64")
    args.update(kw)
    cfg = native.make_config(**args)
    n = ctypes.c_size_t()
    assert lib.mc3_workspace_size(ctypes.byref(cfg), ctypes.byref(n)) == expect


def test_energy_update_field_validated(lib):
    cfg = native.make_config(64, 4, 2, 1, 1)
    cfg.energy_update = 7
    n = ctypes.c_size_t()
    assert lib.mc3_workspace_size(ctypes.byref(cfg), ctypes.byref(n)) == native.MC3_E_ARG


def test_noalloc_and_schedule_calls_reject_null(lib):
    h = ctypes.c_void_p()
    assert lib.mc3_create_noalloc(None, None, ctypes.byref(h)) == native.MC3_E_ARG
    assert lib.mc3_select_betas(None, 0, None) == native.MC3_E_ARG
    assert lib.mc3_step_n_schedules(None, 0, 1, None) == native.MC3_E_ARG
