"""Host-side checks of the libemagpie C ABI (no GPU work is enqueued)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import emagpie_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
E = pytest.importorskip("paper_2511_01793_amd.emagpie")

if not os.path.exists(E.LIB_PATH):
    pytest.skip("libemagpie.so not built", allow_module_level=True)


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "emagpie.h")).read()
    return sorted(set(re.findall(r"\b(emagpie_\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = E.lib()
    syms = declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(E.EXPORTS)
    assert b"gfx950" in L.emagpie_version()


def cfg(**kw):
    base = dict(n=128, m=32, n_pos=100, minibatch=10, levels=1, alpha=0.01, alpha_z=1.0,
                update_probe=1, joint_step=1, path=0, seed=0)
    base.update(kw)
    n = base.pop("n")
    base.setdefault("n_rows", n)
    base.setdefault("n_cols", n)
    return E.Config(**base)


@pytest.mark.parametrize("bad, status", [
    (dict(m=48), "E_SHAPE"), (dict(m=16), "E_SHAPE"), (dict(m=512), "E_SHAPE"), (dict(n=16), "E_SHAPE"),
    (dict(levels=0), "E_SHAPE"), (dict(levels=4), "E_SHAPE"), (dict(minibatch=0), "E_SHAPE"),
    (dict(minibatch=2048), "E_SHAPE"), (dict(n_pos=0), "E_SHAPE"),
    (dict(alpha=float("nan")), "E_ARG"), (dict(alpha=-1.0), "E_ARG"), (dict(alpha_z=float("inf")), "E_ARG"),
    (dict(path=9), "E_ARG"), (dict(update_probe=2), "E_ARG"), (dict(joint_step=3), "E_ARG"),
])
def test_config_validation(bad, status):
    with pytest.raises(E.EmagpieError) as ei:
        E.workspace_size(cfg(**bad))
    assert ei.value.name == status


def test_workspace_size_scales_with_problem():
    small = E.workspace_size(cfg())
    big = E.workspace_size(cfg(n=512, m=64, n_pos=1600, minibatch=64, levels=2))
    assert small > 100 * 32 * 32 * 4
    # intensities copy alone: 1600 * 64^2 * 4 bytes
    assert big > 1600 * 64 * 64 * 4 > small


def _init(c, positions, ws_ptr, ws_bytes):
    ctx = ctypes.c_void_p(None)
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.int32))
    st = E.lib().emagpie_init(ctypes.byref(ctx), ctypes.byref(c), pos.ctypes.data, 0x1000,
                              ws_ptr, ws_bytes, None)
    return st, E.last_error()


def test_init_rejects_positions_outside_object():
    c = cfg(n_pos=3)
    ws = E.workspace_size(c)
    for bad in ([0, 0], [96, 96], [97, 0], [0, -1]):
        pos = [[0, 0], [10, 10], bad]
        st, msg = _init(c, pos, 0x100000, ws)
        if bad in ([0, 0], [96, 96]):
            continue
        assert E.STATUS[st] == "E_POSITION", msg
        assert "scan position 2" in msg


def test_init_rejects_bad_workspace():
    c = cfg(n_pos=2)
    ws = E.workspace_size(c)
    st, msg = _init(c, [[0, 0], [1, 1]], 0x100010, ws)  # misaligned
    assert E.STATUS[st] == "E_WORKSPACE"
    st, msg = _init(c, [[0, 0], [1, 1]], 0x100000, ws - 1)  # too small
    assert E.STATUS[st] == "E_WORKSPACE"
    assert "too small" in msg


def test_library_permutation_equals_oracle_bit_exactly():
    for seed, epoch, n in [(0, 0, 1), (1, 0, 2), (1234567, 3, 100), (2**63 + 5, 99, 1600), (42, 7, 10000)]:
        np.testing.assert_array_equal(E.permutation(seed, epoch, n), O.permutation(seed, epoch, n))


@pytest.mark.parametrize("m", [32, 64, 128])
def test_plan_descriptions_are_consistent(m):
    d0 = E.plan_describe(m, 0, 0)
    count = d0["fft_plans"]
    assert count >= 2
    splits = set()
    for v in range(count):
        for f in range(12):
            d = E.plan_describe(m, v, f)
            assert d["r1"] * d["r2"] == m and d["r1"] in (4, 8, 16) and d["r2"] in (4, 8, 16)
            assert d["threads"] in (256, 512, 1024) and (m * m) % (4 * d["threads"]) == 0
            assert d["fin_tile"] ** 2 % d["fin_threads"] == 0 and d["fin_threads"] % 256 == 0
            # shapes 4..7 and 8..11 are 0..3 with the banded and the rows-per-XCD tile orders
            b = E.plan_describe(m, v, f % 4)
            assert (d["fin_threads"], d["fin_tile"]) == (b["fin_threads"], b["fin_tile"])
            assert d["fin_order"] == f // 4
        splits.add((d["r1"], d["r2"]))
    assert len(splits) >= 2  # at least two radix splits to choose from
    for bad_v, bad_f in [(count, 0), (-1, 0), (0, 12), (0, -1)]:
        with pytest.raises(E.EmagpieError) as ei:
            E.plan_describe(m, bad_v, bad_f)
        assert ei.value.name == "E_ARG"


@pytest.mark.parametrize("bad", [dict(fft_plan=9), dict(fft_plan=-2), dict(finalize_shape=12),
                                 dict(finalize_shape=-3), dict(path=5), dict(m=32, fft_plan=2)])
def test_plan_config_validation(bad):
    with pytest.raises(E.EmagpieError) as ei:
        E.workspace_size(cfg(**bad))
    assert ei.value.name == "E_ARG"


def test_tuning_needs_scratch_state_in_the_workspace():
    plain = E.workspace_size(cfg(n=256))
    tuned = E.workspace_size(cfg(n=256, fft_plan=E.TUNE))
    auto = E.workspace_size(cfg(n=256, path=E.PATHS["auto"]))
    assert tuned == auto >= plain + 256 * 256 * 8


def test_sequential_mode_configuration():
    with pytest.raises(E.EmagpieError) as ei:
        E.workspace_size(cfg(path=E.PATHS["chain"]))  # minibatch 10
    assert ei.value.name == "E_ARG"
    assert E.workspace_size(cfg(path=E.PATHS["chain"], minibatch=1)) > 0
    with pytest.raises(E.EmagpieError) as ei:
        E.workspace_size(cfg(zero_phase_memory=2))
    assert ei.value.name == "E_ARG"
    # the phase memory holds one complex64 phasor per pattern pixel
    assert E.workspace_size(cfg(zero_phase_memory=1)) >= E.workspace_size(cfg()) + 100 * 32 * 32 * 8


def test_probe_side_256_configuration():
    d = E.plan_describe(256, 0, 0)
    assert (d["r1"], d["r2"], d["threads"], d["fft_plans"]) == (16, 16, 256, 1)
    for path in ("fused", "graph", "auto"):
        assert E.workspace_size(cfg(m=256, n=300, path=E.PATHS[path])) > 100 * 256 * 256 * 4
    for path in ("plain", "persistent"):
        with pytest.raises(E.EmagpieError) as ei:
            E.workspace_size(cfg(m=256, n=300, path=E.PATHS[path]))
        assert ei.value.name == "E_UNSUPPORTED"
    with pytest.raises(E.EmagpieError) as ei:
        E.workspace_size(cfg(m=256, n=200, path=1))
    assert ei.value.name == "E_SHAPE"


def test_rectangular_objects_validated_per_side():
    # rows and columns are checked on their own: 100 x 300 takes windows up to (68, 268)
    c = cfg(n_rows=100, n_cols=300, n_pos=3)
    ws = E.workspace_size(c)
    assert ws > 0
    st, msg = _init(c, [[0, 0], [10, 10], [0, 269]], 0x100000, ws)
    assert E.STATUS[st] == "E_POSITION" and "scan position 2" in msg
    st, msg = _init(c, [[0, 0], [10, 10], [69, 0]], 0x100000, ws)
    assert E.STATUS[st] == "E_POSITION"
    for bad in (dict(n_rows=16, n_cols=300), dict(n_rows=300, n_cols=31), dict(n_cols=70000)):
        with pytest.raises(E.EmagpieError) as ei:
            E.workspace_size(cfg(**bad))
        assert ei.value.name == "E_SHAPE"


def test_last_error_per_context_and_per_thread():
    # with no context the thread's last failure; a null context is an argument error
    with pytest.raises(E.EmagpieError):
        E.workspace_size(cfg(m=48))
    assert "probe side" in E.last_error()
    st = E.lib().emagpie_epoch(None, 0x1000, 0x1000, 0, None, None, None)
    assert E.STATUS[st] == "E_ARG" and "null context" in E.last_error()


def test_many_instance_configuration():
    one = E.workspace_size(cfg())
    two = (E.Config * 2)(cfg(), cfg(n=256, m=64, n_pos=400, minibatch=64, levels=2))
    out = ctypes.c_size_t(0)
    assert E.lib().emagpie_workspace_size_many(2, two, ctypes.byref(out)) == 0
    assert out.value > one + E.workspace_size(cfg(n=256, m=64, n_pos=400, minibatch=64, levels=2))
    # sizing with a finalize shape left to the autotuner is an upper bound over the shapes
    tuned = (E.Config * 2)(cfg(), cfg(n=256, m=64, n_pos=400, minibatch=64, levels=2,
                                      finalize_shape=E.TUNE))
    out2 = ctypes.c_size_t(0)
    assert E.lib().emagpie_workspace_size_many(2, tuned, ctypes.byref(out2)) == 0
    assert out2.value >= out.value
    bad = (E.Config * 2)(cfg(), cfg(m=256, n=300, path=1))
    assert E.STATUS[E.lib().emagpie_workspace_size_many(2, bad, ctypes.byref(out))] == "E_UNSUPPORTED"
    assert E.STATUS[E.lib().emagpie_workspace_size_many(0, two, ctypes.byref(out))] == "E_ARG"
    ctx = ctypes.c_void_p(None)
    st = E.lib().emagpie_init_many(ctypes.byref(ctx), 2, two, None, None, 0x100000, 1 << 40, None)
    assert E.STATUS[st] == "E_ARG" and not ctx.value


def test_peak_measurement_rejects_small_buffers():
    out = np.zeros(2)
    st = E.lib().emagpie_measure_peaks(0x100000, 1 << 20, 3, out.ctypes.data, None)
    assert E.STATUS[st] == "E_WORKSPACE"
    st = E.lib().emagpie_measure_peaks(0x100000, 1 << 30, 0, out.ctypes.data, None)
    assert E.STATUS[st] == "E_ARG"
