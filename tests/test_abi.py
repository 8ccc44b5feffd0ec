"""The C-ABI library loads, exports every symbol its header declares, and
rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1807_10058_amd as fcc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fcc_dct.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fcc_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "fcc_dct_plan" in names and "fcc_dct_batched" in names
    lib = ctypes.CDLL(fcc.lib_path())
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    for s in range(7):
        assert fcc.fcc_status_string(s).startswith("FCC_")


@pytest.mark.parametrize("n", [0, 3, 6, 2048, -4])
def test_plan_rejects_non_power_of_two(n):
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_plan(n)
    assert e.value.status == 2


def test_plan_rejects_singular_skew_like_the_oracle():
    """(0.3, 0.1, 0.7) makes zeros coincide: the oracle's matrix is singular and
    the plan refuses it; the default and a generic skew are accepted by the check."""
    F = oracle.matrix(2, (0.3, 0.1, 0.7))
    assert np.linalg.cond(F) > 1e12
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_plan(4, rst=(0.3, 0.1, 0.7))
    assert e.value.status == 3
    assert np.linalg.cond(oracle.matrix(2, (0.31, 0.07, 0.23))) < 1e6


@pytest.mark.parametrize("n", [512, 1024])
def test_plan_rejects_table_levels_above_256_as_unsupported(n):
    """Per-row gather tables pack node-local coordinates in 8 bits, so node
    sizes above 256 are served only by orbit-block launches; a schedule that
    asks for tables there is refused before any device work (runs without a GPU)."""
    tuning = {"tail_levels": [1, 1], "tile": [[[0, 0, 0]] * 2] * 2, "map": [[0] * 10, [0] * 10]}
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_plan_tuned(n, tuning=tuning, stream=0)
    assert e.value.status == 6
    tuning["map"] = [[fcc.FCC_MAP_ORBIT] * 10, [0] * 10]
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_plan_tuned(n, tuning=tuning, stream=0)
    assert e.value.status == 6


def test_plan_rejects_bad_flags_and_precision():
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_plan(4, prec=9)
    assert e.value.status == 1
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_plan(4, flags=fcc.FCC_STAGES_FP32 | fcc.FCC_STAGES_FP64)
    assert e.value.status == 1
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_plan(4, flags=1 << 9)
    assert e.value.status == 1


def test_tables_reject_bad_sizes():
    for nl in (1, 3, 2048):
        with pytest.raises(fcc.FccError):
            fcc.fcc_asp_tables(nl)


def _tuning(**kw):
    t = {"tail_levels": [1, 1], "tile": [[[0, 0, 0], [0, 0, 0]], [[0, 0, 0], [0, 0, 0]]], "map": [[0, 0], [0, 0]]}
    t.update(kw)
    return t


@pytest.mark.parametrize("bad", [
    {"tail_levels": [0, 1]}, {"tail_levels": [1, 5]},
    {"tile": [[[0, 0, -1], [0, 0, 0]], [[0, 0, 0], [0, 0, 0]]]},
    {"tile": [[[0, 0, 0], [0, 0, 0]], [[0, 10, 0], [0, 0, 0]]]},
    {"map": [[512, 0], [0, 0]]},
    {"map": [[0, 0, 0], [0, 0, 12]]},
])
def test_plan_tuned_rejects_bad_schedules(bad):
    # validated before any device work, so this runs without a GPU
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_plan_tuned(8, tuning=_tuning(**bad), stream=0)
    assert e.value.status == 1


def test_tuning_entry_points_reject_bad_arguments():
    lib = ctypes.CDLL(fcc.lib_path())
    lib.fcc_dct_get_tuning.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    buf = ctypes.create_string_buffer(256)
    assert lib.fcc_dct_get_tuning(None, buf) == 1
    with pytest.raises(fcc.FccError) as e:
        fcc.fcc_dct_autotune(8, reps=0, stream=0)
    assert e.value.status == 1
