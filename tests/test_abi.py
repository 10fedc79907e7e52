"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/sw.h declares, and the binding knows them all;
plus the host-only workload recipes."""
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(sw_[a-z_]+)\s*\(", src))
    return names


def test_header_declares_core_calls():
    names = declared_functions()
    for n in ("sw_create", "sw_sweep", "sw_measure", "sw_destroy", "sw_batch_create",
              "sw_server_submit", "sw_server_poll"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import ctypes
    import paper_1403_7560_amd as sw
    lib = ctypes.CDLL(sw.LIB_PATH)
    names = declared_functions()
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert names == set(sw.SIGNATURES), sorted(names ^ set(sw.SIGNATURES))
    sw.lib()  # argtypes/restype setup succeeds for all of them


def test_footprint_is_host_logic():
    import paper_1403_7560_amd as sw
    f2 = sw.footprint(sw.ISING, 2, 4096)
    assert f2 >= 4096 * 4096 * 6
    assert sw.footprint(sw.XY, 3, 128, 0) > sw.footprint(sw.ISING, 3, 128)
    with pytest.raises(sw.SWError):
        sw.footprint(sw.POTTS, 2, 64, 1)


def test_job_mix_recipe():
    from paper_1403_7560_amd import inputs
    jobs = inputs.job_mix(4000, rate=200.0, seed=3)
    t = np.array([j["arrival"] for j in jobs])
    assert np.all(np.diff(t) > 0)
    assert abs(len(jobs) / t[-1] - 200.0) < 15.0
    cats = np.array([(j["model"], j["dim"]) for j in jobs])
    for c in [(0, 2), (1, 2), (0, 3), (2, 3)]:
        frac = np.mean(np.all(cats == c, axis=1))
        assert 0.2 < frac < 0.3
    for j in jobs:
        lo, hi = (32, 2048) if j["dim"] == 2 else (16, 192)
        assert lo <= j["L"] <= hi and 100 <= j["sweeps"] <= 5000
        if j["model"] == 1:
            assert j["q"] in (3, 4, 10)
    L2 = np.log([j["L"] for j in jobs if j["dim"] == 2])
    assert abs(L2.mean() - 0.5 * (math.log(32) + math.log(2048))) < 0.1


def test_workload_temperatures():
    from paper_1403_7560_amd import inputs
    lats, n = inputs.workload("C4")
    T = np.array([1 / j["beta"] for j in lats])
    assert len(lats) == 32 and n == 2000
    assert T[0] == pytest.approx(0.95 * 2.2019) and T[-1] == pytest.approx(1.05 * 2.2019)
    assert np.allclose(np.diff(T), np.diff(T)[0])
    lats, _ = inputs.workload("C2-potts")
    assert lats[0]["beta"] == pytest.approx(math.log(1 + math.sqrt(3)))
    for name in ("C2-potts", "C2-ising"):
        small, _ = inputs.workload(name)
        big, n = inputs.workload(name + "-8192")
        assert n == 2000 and big[0]["L"] == 8192
        assert {k: v for k, v in big[0].items() if k != "L"} == {k: v for k, v in small[0].items() if k != "L"}


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_tile_shapes_are_host_logic():
    import paper_1403_7560_amd as sw
    for model in (sw.ISING, sw.POTTS, sw.XY, sw.CLOCK):
        for dim in (2, 3):
            n = sw.tile_count(model, dim)
            assert n >= 1
            for t in range(n):
                tx, ty, tz = sw.tile_shape(model, dim, t)
                assert tx == 64 and ty % 4 == 0 and (tz == 1 if dim == 2 else tz >= 1)
                assert tx * ty * tz <= 16384
            with pytest.raises(sw.SWError):
                sw.tile_shape(model, dim, n)
    assert sw.tile_shape(sw.ISING, 2, 0) == (64, 64, 1)
    with pytest.raises(sw.SWError):
        sw.tile_count(4, 2)


def test_invalid_lattice_arguments_fail_before_the_device():
    """Argument checks (and the default tile rule) run before any HIP call:
    bad arguments raise SW_E_INVALID, with or without a GPU."""
    import paper_1403_7560_amd as sw
    for args in [(4, 2, 10, 2), (sw.ISING, 4, 10, 2), (sw.ISING, 2, 2, 2), (sw.POTTS, 2, 10, 1),
                 (sw.POTTS, 2, 10, 257), (sw.ISING, 3, 1291, 2)]:
        with pytest.raises(sw.SWError) as e:
            sw.Lattice(*args, beta=0.4, seed=1)
        assert e.value.code == -1, args
    for args in [(sw.CLOCK, 2, 10, 3), (sw.CLOCK, 2, 10, 514), (sw.CLOCK, 2, 10, 0)]:
        with pytest.raises(sw.SWError) as e:
            sw.Lattice(*args, beta=0.4, seed=1)
        assert e.value.code == -1, args
    for tile in (-2, 99):
        with pytest.raises(sw.SWError) as e:
            sw.Lattice(sw.ISING, 2, 10, 2, beta=0.4, seed=1, tile=tile)
        assert e.value.code == -1


def test_ordered_state_recipe():
    from paper_1403_7560_amd import inputs
    for model, q, dt in ((0, 2, np.int8), (1, 3, np.uint8), (2, 0, np.float32)):
        st = inputs.ordered_state(model, 2, 200, q, seed=4)
        assert st.dtype == dt and st.size == 40000
        assert np.array_equal(st, inputs.ordered_state(model, 2, 200, q, seed=4))
        if model == 0:
            assert set(np.unique(st)) <= {-1, 1} and 0.96 < np.mean(st == 1) < 0.99
        elif model == 1:
            assert st.max() < q and 0.95 < np.mean(st == 0) < 0.98
        else:
            assert st.min() >= 0 and st.max() < np.float32(2 * math.pi)
            c = np.mean(np.cos(st.astype(np.float64)))
            assert 0.85 < c < 0.95  # about (1 - 0.05) * exp(-0.3^2 / 2)
