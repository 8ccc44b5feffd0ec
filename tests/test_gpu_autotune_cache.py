"""Persisted schedules (FCC_AUTOTUNE_CACHE): a search in one process is read
back by the plans of a later process.  Each step runs in its own Python
process, one after the other."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SEARCH = """
import json, paper_1807_10058_amd as fcc
t = fcc.fcc_dct_autotune(16, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT | fcc.FCC_FOLD_BASE, reps=1)
print(json.dumps(t))
"""
READ = """
import json, paper_1807_10058_amd as fcc
p = fcc.fcc_dct_plan(16, prec=fcc.FCC_PREC_FP32, flags=fcc.FCC_REAL_INPUT | fcc.FCC_FOLD_BASE)
print(json.dumps(fcc.fcc_dct_get_tuning(p)))
"""


def _py(code, env):
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_search_persists_across_processes(tmp_path):
    path = str(tmp_path / "schedules.txt")
    env = dict(os.environ, FCC_AUTOTUNE_CACHE=path)
    found = _py(SEARCH, env)
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("fccdct-schedule 1 gfx")
    assert _py(READ, env) == found
    # a malformed line and a line for another architecture are skipped
    with open(path, "a") as f:
        f.write("fccdct-schedule 1 gfx000 16 1 129 1 1" + " 0" * 32 + "\n")
        f.write("garbage\n")
    assert _py(READ, env) == found
