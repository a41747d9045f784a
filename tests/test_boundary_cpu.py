"""Host-side checks of the C-ABI library (no GPU needed): the library loads
and exports every declared entry point, argument errors are reported, and
the host planner builds the same trees as the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from hlu_inputs import icosphere

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1906_00874_amd as P
    return P


def test_library_exports_every_declared_symbol():
    P = _lib()
    hdr = open(os.path.join(ROOT, "include", "hlu.h")).read()
    names = set(re.findall(r"\b(hlu_[a-z_]+)\s*\(", hdr))
    names -= {"hlu_handle_s"}
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(P.lib, n), n


def test_plan_matches_oracle_trees():
    P = _lib()
    for level, leaf in [(2, 16), (3, 32), (4, 32)]:
        xyz, area = icosphere(level)
        h = P.HLU(xyz, area, assemble=False, leaf=leaf, eta=2.0, eps=1e-6, cap=32)
        root, perm, leaves = O.cluster_tree(xyz, leaf)
        assert np.array_equal(perm, h.perm())
        H = O.HMatrix(xyz, area, leaf, 2.0, O.Rule(eps=1e-2, cap=4))
        st = h.stats()
        ost = H.stats()
        assert st["leaves"] == ost["leaves"]
        assert st["dense_blocks"] == ost["dense"]
        assert st["lowrank_blocks"] == ost["lowrank"]
        assert st["ops_factor"] > 0 and st["waves_factor"] > 0


def test_plan_matches_oracle_trees_log_kernels():
    """d = 1 and d = 2 inputs (points on a segment / a circle): the planner's
    cluster and block trees equal the oracle's."""
    from hlu_inputs import circle, segment
    P = _lib()
    for geo, kernel, reading in [(segment, P.KERNEL_LOG1D, O.READING_LOG1D),
                                 (circle, P.KERNEL_LOG2D, O.READING_LOG2D)]:
        xyz, h = geo(2048)
        hl = P.HLU(xyz, h, assemble=False, kernel=kernel, leaf=32, eta=2.0, eps=1e-6, cap=32)
        H = O.HMatrix(xyz, h, 32, 2.0, O.Rule(eps=1e-2, cap=4), reading=reading)
        assert np.array_equal(H.perm, hl.perm())
        st, ost = hl.stats(), H.stats()
        assert (st["leaves"], st["dense_blocks"], st["lowrank_blocks"]) == \
            (ost["leaves"], ost["dense"], ost["lowrank"])
    with pytest.raises(P.HLUError) as e:
        xyz, h = segment(64)
        h[3] = 0.0
        P.HLU(xyz, h, assemble=False, kernel=P.KERNEL_LOG1D)
    assert e.value.status == 1


def test_plan_eta_zero_has_no_lowrank_blocks():
    P = _lib()
    xyz, area = icosphere(2)
    h = P.HLU(xyz, area, assemble=False, leaf=16, eta=0.0, eps=1e-6)
    assert h.stats()["lowrank_blocks"] == 0


@pytest.mark.parametrize("bad", [
    dict(leaf=0), dict(leaf=65), dict(eta=-1.0), dict(cap=0), dict(cap=33),
    dict(cap_mv=65), dict(eps=0.0), dict(eps=1.5), dict(max_nrhs=0), dict(max_nrhs=65),
    dict(fixed_rank=40), dict(eps_mv=0.0), dict(eps=1e-9), dict(eps=1e-10),
    dict(device_assembly=2), dict(device_assembly=1, cap_mv=64),
    dict(operation=3), dict(operation=1, cap_mv=64), dict(operation=2, cap_mv=0, refine_tol=1e-10),
    dict(operation=1, cap_mv=0, device_assembly=1), dict(operation=1, cap_mv=0, kernel_b=7),
])
def test_plan_argument_errors(bad):
    P = _lib()
    xyz, area = icosphere(1)
    with pytest.raises(P.HLUError) as e:
        P.HLU(xyz, area, assemble=False, **bad)
    assert e.value.status == 1


def test_plan_rejects_nan_and_null():
    P = _lib()
    xyz, area = icosphere(1)
    xyz = xyz.copy()
    xyz[3, 1] = np.nan
    with pytest.raises(P.HLUError) as e:
        P.HLU(xyz, area, assemble=False)
    assert e.value.status == 1
    h = C.c_void_p()
    prm = P.binding.make_params()
    assert P.lib.hlu_plan(None, None, 10, C.byref(prm), C.byref(h)) == 1
    assert "NULL" in P.lib.hlu_last_error().decode()


def test_state_errors_without_device():
    P = _lib()
    xyz, area = icosphere(1)
    h = P.HLU(xyz, area, assemble=False)
    dummy = C.c_void_p(256)
    # solve before factor, factor before assemble, bind with too few bytes
    assert P.lib.hlu_solve(h.h, dummy, dummy, 1, h.n, None) == 6
    assert P.lib.hlu_factor(h.h, None) == 6
    assert P.lib.hlu_assemble(h.h, None) == 6
    assert P.lib.hlu_bind(h.h, dummy, 16) == 2
    assert P.lib.hlu_required_bytes(None) == 0


def test_batch_arguments_without_device():
    """The batch is built on the host from planned handles: an empty list or
    a handle listed twice is refused; a valid batch needs a workspace, and
    factoring before binding is a state error."""
    P = _lib()
    xyz, area = icosphere(1)
    h1 = P.HLU(xyz, area, assemble=False)
    h2 = P.HLU(xyz, area, assemble=False)
    out = C.c_void_p()
    arr = (C.c_void_p * 2)(h1.h, h1.h)
    assert P.lib.hlu_batch_create(arr, 2, C.byref(out)) == 1
    assert P.lib.hlu_batch_create(arr, 0, C.byref(out)) == 1
    arr = (C.c_void_p * 2)(h1.h, h2.h)
    assert P.lib.hlu_batch_create(arr, 2, C.byref(out)) == 0
    nb = P.lib.hlu_batch_required_bytes(out)
    # queue over both schedules' ops at least
    assert nb >= 4 * 2 * h1.stats()["ops_factor"]
    assert P.lib.hlu_batch_factor(out, None) == 6
    assert P.lib.hlu_batch_bind(out, C.c_void_p(256), 16) == 1
    P.lib.hlu_batch_destroy(out)


def test_schedule_statistics_scale():
    P = _lib()
    xyz, area = icosphere(3)
    h = P.HLU(xyz, area, assemble=False, leaf=32)
    st = h.stats()
    # every op in a wave is independent; the wave count is at least the
    # number of diagonal leaves (one getrf each, strictly ordered)
    assert st["waves_factor"] >= st["leaves"]
    launches = h.batches()
    assert launches[0] == st["leaves"]          # one getrf launch per leaf


@pytest.mark.parametrize("level,leaf,prec,fixed", [(2, 16, 0, 0), (3, 32, 0, 8), (3, 32, 1, 0),
                                                   (4, 32, 1, 0), (3, 64, 0, 0)])
def test_schedule_validates(level, leaf, prec, fixed):
    """Every descriptor stays inside the buffer at full capacity and has
    consistent operand shapes (checked on the host before any launch)."""
    P = _lib()
    xyz, area = icosphere(level)
    h = P.HLU(xyz, area, assemble=False, leaf=leaf, precision=prec, fixed_rank=fixed)
    h.validate()


def test_plan_tight_eps_accepted_with_fixed_rank_and_at_limit():
    """eps_factor below 1e-8 is refused only for tolerance-driven
    truncation: a fixed-rank plan ignores it, and 1e-8 itself is accepted."""
    P = _lib()
    xyz, area = icosphere(1)
    P.HLU(xyz, area, assemble=False, eps=1e-8)
    P.HLU(xyz, area, assemble=False, eps=1e-12, fixed_rank=4)


def test_set_refinement_arguments():
    P = _lib()
    xyz, area = icosphere(1)
    h = P.HLU(xyz, area, assemble=False, cap_mv=64, refine_tol=1e-10)
    h.set_refinement(0.0, 0)
    h.set_refinement(1e-12, 15)
    for tol, it in [(-1.0, 3), (1e-10, 16), (1e-10, -1), (float("nan"), 2)]:
        with pytest.raises(P.HLUError) as e:
            h.set_refinement(tol, it)
        assert e.value.status == 1
    # without the operator copy the refinement residual is summed directly
    # over the exact entries, so a tolerance is accepted there too
    h0 = P.HLU(xyz, area, assemble=False, cap_mv=0, refine_tol=0.0)
    h0.set_refinement(1e-10, 3)


def test_import_blocks_checks_the_file_before_the_device(tmp_path):
    """hlu_import_blocks: a file that does not match the handle's trees is
    refused (HLU_ERR_ARG) before any device access; a matching file on an
    unbound handle is HLU_ERR_STATE."""
    from hblocks import write_blocks
    P = _lib()
    xyz, area = icosphere(3)
    h = P.HLU(xyz, area, assemble=False, leaf=32, eta=2.0, eps=1e-6, cap=32)
    H = O.HMatrix(xyz, area, 32, 2.0, O.Rule(eps=1e-6, cap=32))
    good = tmp_path / "good.bin"
    write_blocks(H, good)
    with pytest.raises(P.HLUError) as e:
        h.import_blocks(good)
    assert e.value.status == 6
    blocks = list(O.leaves_of(H.block))
    cases = {
        "magic": dict(magic=b"HLUBLK00"),
        "perm": dict(perm=H.perm[::-1]),
        "missing": dict(blocks=blocks[:-1]),
        "twice": dict(blocks=blocks[:-1] + blocks[:1]),
    }
    for name, kw in cases.items():
        f = tmp_path / f"{name}.bin"
        write_blocks(H, f, **kw)
        with pytest.raises(P.HLUError) as e:
            h.import_blocks(f)
        assert e.value.status == 1, name
    # ranks above the handle's capacity
    h8 = P.HLU(xyz, area, assemble=False, leaf=32, eta=2.0, eps=1e-6, cap=4)
    with pytest.raises(P.HLUError) as e:
        h8.import_blocks(good)
    assert e.value.status == 1 and "capacity" in str(e.value)
    # a handle on another tree (leaf 16)
    h16 = P.HLU(xyz, area, assemble=False, leaf=16, eta=2.0, eps=1e-6, cap=32)
    with pytest.raises(P.HLUError) as e:
        h16.import_blocks(good)
    assert e.value.status == 1
    with pytest.raises(P.HLUError) as e:
        h.import_blocks(tmp_path / "absent.bin")
    assert e.value.status == 1
