"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/she.h, and rejects invalid configurations before any
device work (no GPU needed)."""
import os
import re

import pytest

from paper_2406_12157_amd import she
from paper_2406_12157_amd import workloads as W
from helpers import gpu_instance

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "she.h")


def declared_functions():
    text = open(HEADER).read()
    decl = r"^(?:she_status|void|const char \*)\s*(she_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(she.EXPORTS)


def test_library_exports_every_symbol():
    lib = she.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def cfg_for(insts, **kw):
    return [gpu_instance(she, i) for i in insts], kw


@pytest.mark.parametrize("mutate,status", [
    (dict(r=0.6), she.EUNSTABLE),
    (dict(r=-0.1), she.EINVAL),
    (dict(eps=-1.0), she.EINVAL),
    (dict(u_left=1.0, u_right=2.0), she.EINVAL),        # gradient with periodic walls
    (dict(n=(1,)), she.EINVAL),
    (dict(scheme=7), she.EINVAL),
    (dict(noise=3), she.EINVAL),
])
def test_invalid_1d_configs(mutate, status):
    inst = W.instance((64,), r=0.2)
    inst.update(mutate)
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, inst)])
    assert e.value.status == status


def test_grids_too_small_for_the_marches_are_rejected():
    # 2D PC reads two rows beyond a march chunk, 3D one plane beyond the next
    for inst in (W.instance((64, 2), r=0.1, scheme=W.HEUN), W.instance((32, 8, 1), r=0.1)):
        with pytest.raises(she.SheError) as e:
            she.Handle.arena_bytes([gpu_instance(she, inst)])
        assert e.value.status == she.EUNSUPPORTED
    she.Handle.arena_bytes([gpu_instance(she, W.instance((64, 2), r=0.1))])       # 2D FE: one step per launch
    she.Handle.arena_bytes([gpu_instance(she, W.instance((64, 3), r=0.1, scheme=W.HEUN))])


def test_empty_batch_is_rejected():
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([])
    assert e.value.status == she.EINVAL


def test_invalid_nd_configs():
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, W.instance((48, 16), r=0.1))])
    assert e.value.status == she.EUNSUPPORTED            # n[0] not a power of two
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, W.instance((64, 64), r=0.3))])
    assert e.value.status == she.EUNSTABLE               # r > 1/4 in 2D
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, W.instance((64, 64), r=0.1, bc=W.DIRICHLET))])
    assert e.value.status == she.EINVAL
    a = W.instance((64, 64), r=0.1, realisation=0)
    b = W.instance((64, 32), r=0.1, realisation=1)            # another grid in the same batch
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, a), gpu_instance(she, b)])
    assert e.value.status == she.EUNSUPPORTED


def test_invalid_tuning_and_graph_settings():
    insts = [gpu_instance(she, W.instance((64, 64), r=0.1))]
    for kw in (dict(tuning_flags=8), dict(graph_steps=-1), dict(graph_steps=(1 << 16) + 1)):
        with pytest.raises(she.SheError) as e:
            she.Handle.arena_bytes(insts, **kw)
        assert e.value.status == she.EINVAL, kw
    base = she.Handle.arena_bytes(insts)
    assert she.Handle.arena_bytes(insts, graph_steps=64, tuning_flags=she.TUNE_XCD_ORDER) == base
    assert she.Handle.arena_bytes(insts, tuning_flags=she.TUNE_SEARCH) == base
    # the autotuner allocates trial handles, so it refuses a caller arena (checked
    # before any device work)
    import torch
    arena = torch.empty(base, dtype=torch.uint8)
    with pytest.raises(she.SheError) as e:
        she.Handle(insts, arena=arena, tuning_flags=she.TUNE_SEARCH, stream=0)
    assert e.value.status == she.EINVAL


def test_time_correlation_settings():
    one = [gpu_instance(she, W.instance((64,), r=0.2))]
    base = she.Handle.arena_bytes(one, stats=she.STAT_MOMENTS)
    with_tc = she.Handle.arena_bytes(one, stats=she.STAT_TCORR, tcorr_lags=32)
    assert with_tc >= base + 8 * 32 * 64            # FP64 lag sums at least
    bad = [dict(stats=she.STAT_TCORR), dict(stats=she.STAT_TCORR, tcorr_lags=1025),
           dict(stats=she.STAT_MOMENTS, tcorr_lags=8), dict(stats=32)]
    for kw in bad:
        with pytest.raises(she.SheError) as e:
            she.Handle.arena_bytes(one, **kw)
        assert e.value.status == she.EINVAL, kw
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, W.instance((64, 64), r=0.1))], stats=she.STAT_TCORR,
                               tcorr_lags=8)
    assert e.value.status == she.EUNSUPPORTED


def test_composite_rod_validation():
    def arena(**kw):
        return she.Handle.arena_bytes([gpu_instance(she, W.instance((16,), bc=W.DIRICHLET, r=0.1, **kw))])
    base = arena()
    assert arena(cond=[1.0] * 8 + [3.0] * 8, cap=[1.0] * 8 + [0.7] * 8) > base   # coefficient block
    cases = [(dict(cond=[1.0] * 15 + [0.0]), she.EINVAL),
             (dict(cap=[1.0] * 15 + [float("nan")]), she.EINVAL),
             (dict(cond=[20.0] * 16), she.EUNSTABLE),
             (dict(cap=[0.1] * 16), she.EUNSTABLE),
             (dict(cond=[2.0] * 16, noise=1, u_left=1.0, u_right=2.0), she.EUNSUPPORTED)]
    for kw, status in cases:
        with pytest.raises(she.SheError) as e:
            arena(**kw)
        assert e.value.status == status, kw
    arena(cond=[2.0] * 16, noise=1)                                 # equilibrium: allowed
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, W.instance((8, 8), r=0.1, cond=[1.0] * 64))])
    assert e.value.status == she.EUNSUPPORTED


def test_burgers_validation():
    ok = W.instance((64,), eq=W.BURGERS, r=0.25, eps=1e-4, u0=0.15, nu=0.6)
    she.Handle.arena_bytes([gpu_instance(she, ok)])
    cases = [(W.instance((64,), r=0.25, nu=0.3), she.EINVAL),                              # nu on the heat equation
             (W.instance((64,), eq=W.BURGERS, r=0.05, u0=0.2, nu=0.9), she.EUNSTABLE),      # nu^2 > 2 r
             (W.instance((16, 16), eq=W.BURGERS, r=0.1, u0=0.2, nu=0.1), she.EUNSUPPORTED),
             (W.instance((64,), eq=W.BURGERS, r=0.25, u0=0.2, nu=0.3, cond=[1.0] * 64), she.EUNSUPPORTED),
             (W.instance((64,), eq=3, r=0.1), she.EINVAL)]
    for inst, status in cases:
        with pytest.raises(she.SheError) as e:
            she.Handle.arena_bytes([gpu_instance(she, inst)])
        assert e.value.status == status, inst


def test_implicit_scheme_validation():
    for scheme in (W.BE, W.CN):
        she.Handle.arena_bytes([gpu_instance(she, W.instance((64,), scheme=scheme, r=25.0))])   # no r limit
        cases = [(W.instance((16, 16), scheme=scheme, r=0.1), she.EUNSUPPORTED),
                 (W.instance((64,), eq=W.BURGERS, scheme=scheme, r=0.2, u0=0.3, nu=0.1), she.EUNSUPPORTED),
                 (W.instance((2,), scheme=scheme, r=0.2), she.EINVAL)]
        for inst, status in cases:
            with pytest.raises(she.SheError) as e:
                she.Handle.arena_bytes([gpu_instance(she, inst)])
            assert e.value.status == status, inst
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, W.instance((64,), scheme=4, r=0.1))])
    assert e.value.status == she.EINVAL


def test_arena_bytes_scale_with_problem():
    small = she.Handle.arena_bytes([gpu_instance(she, W.instance((64, 64), r=0.1))])
    big = she.Handle.arena_bytes([gpu_instance(she, W.instance((512, 512), r=0.1))])
    assert big >= 2 * 4 * 512 * 512 > small
    c3 = W.c3()
    b = she.Handle.arena_bytes([gpu_instance(she, i) for i in c3["instances"]], stats=she.STAT_SPATIAL)
    assert b >= 2 * 4 * 512 * 512 * 256


def test_ragged_batch_plan_accepts_c4():
    c4 = W.c4()
    b = she.Handle.arena_bytes([gpu_instance(she, i) for i in c4["instances"]], stats=she.STAT_MOMENTS)
    total = sum(i["n"][0] for i in c4["instances"])
    assert b >= total * (4 + 16)


def test_second_moment_stability_check_at_create():
    """A periodic FE heat instance with instantaneous noise has a stationary
    variance only while eps * beta < 1 (beta: the face temperature's share of
    the FE spectrum, computed here by theory.gamma_beta over the full mode
    grid).  The literal c1 (eps = 100) is refused with SHE_EUNSTABLE unless
    SHE_ALLOW_UNSTABLE is set; eps on either side of 1/beta decides it, in
    1D, 2D and 3D.  PC, Dirichlet and species instances are not checked."""
    import theory
    lit = W.c1(eps=100.0)["instances"][0]
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, lit)])
    assert e.value.status == she.EUNSTABLE
    she.Handle.arena_bytes([gpu_instance(she, lit)], flags=she.ALLOW_UNSTABLE)
    she.Handle.arena_bytes([gpu_instance(she, W.c1()["instances"][0])])            # eps = 1e-2
    for n, r in (((64,), 0.2), ((32, 16), 0.1), ((16, 8, 8), 0.05)):
        _, beta = theory.gamma_beta(r, n)
        she.Handle.arena_bytes([gpu_instance(she, W.instance(n, r=r, eps=0.999 / beta))])
        with pytest.raises(she.SheError) as e:
            she.Handle.arena_bytes([gpu_instance(she, W.instance(n, r=r, eps=1.001 / beta))])
        assert e.value.status == she.EUNSTABLE, n
    for kw in (dict(scheme=W.HEUN), dict(eq=W.SPECIES, u0=100.0), dict(noise=1), dict(noise=2)):
        she.Handle.arena_bytes([gpu_instance(she, W.instance((64,), r=0.2, eps=100.0, **kw))])
    she.Handle.arena_bytes([gpu_instance(she, W.instance((64,), bc=W.DIRICHLET, r=0.2, eps=100.0))])
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, W.c1()["instances"][0])], flags=2)
    assert e.value.status == she.EINVAL


def test_nd_batches_may_differ_in_r_u0_eps_and_init_sd():
    a = W.instance((64, 32), r=0.1, eps=1e-2, init_sd=0.1, realisation=0)
    ok = [a, dict(a, eps=3e-2, realisation=1), dict(a, init_sd=0.0, realisation=2), dict(a, r=0.2, realisation=3),
          dict(a, u0=2.0, u_left=2.0, u_right=2.0, realisation=4)]
    she.Handle.arena_bytes([gpu_instance(she, i) for i in ok])
    # each instance is checked against its own stability limit
    with pytest.raises(she.SheError) as e:
        she.Handle.arena_bytes([gpu_instance(she, a), gpu_instance(she, dict(a, r=0.3))])
    assert e.value.status == she.EUNSTABLE
    for bad in (dict(a, seed=4), dict(a, noise=1), dict(a, scheme=W.HEUN), dict(a, eq=W.SPECIES, u0=100.0,
                                                                                 u_left=100.0, u_right=100.0)):
        with pytest.raises(she.SheError) as e:
            she.Handle.arena_bytes([gpu_instance(she, a), gpu_instance(she, bad)])
        assert e.value.status == she.EUNSUPPORTED, bad


def test_batch_samples_settings():
    one = [gpu_instance(she, W.instance((64,), r=0.2))]
    she.Handle.arena_bytes(one, stats=she.STAT_MOMENTS, batch_samples=100)
    for kw in (dict(stats=she.STAT_MOMENTS, batch_samples=-1), dict(batch_samples=10)):
        with pytest.raises(she.SheError) as e:
            she.Handle.arena_bytes(one, **kw)
        assert e.value.status == she.EINVAL, kw
