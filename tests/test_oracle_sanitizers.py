"""The oracle (C) under AddressSanitizer and UndefinedBehaviorSanitizer: a build of
the same source with -fsanitize=address,undefined (recovery off) is driven through
scene generation, evaluation at every level (window and all-pairs radius modes),
the one-shot costs, the overlap heuristic, local ICP and the three searches in a
child process that preloads the ASan runtime; any report fails the test.  CPU
only."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
import numpy as np
import oracle
from oracle import Oracle
from paper_1510_05613_amd import scenes
assert oracle.LIB_PATH.endswith("liboracle_san.so"), oracle.LIB_PATH
lib = scenes.make_library("c1")
sc = scenes.make_scene(1, 0, oracle.render_fn, lib)
for mode in (0, 1):
    o = Oracle.from_scene(sc, nthreads=2, radius_mode=mode)
    first, second = (int(k) for k in sc.gt_order)
    pm, pp = [int(sc.obj_mesh[first])], [int(sc.gt_pose[first])]
    ps = np.arange(0, sc.grid.P, 37)
    o.eval([], [], np.full(len(ps), pm[0]), ps)
    o.eval(pm, pp, np.full(len(ps), int(sc.obj_mesh[second])), ps)
    o.jtree(list(sc.obj_mesh), list(sc.gt_pose))
    o.overlap(pm, pp, np.full(len(ps), int(sc.obj_mesh[second])), ps)
    o.icp([], [], np.full(4, pm[0]), ps[:4], iters=3, radius=0.02)
sub = np.arange(0, sc.grid.P, 97).astype(np.int32)
o = Oracle.from_scene(sc, nthreads=2)
o.set_symmetric(int(sc.obj_mesh[0]), True) if hasattr(o, "set_symmetric") else None
print(o.search_exhaustive(sub)["cost"], o.search_ucs(sub)["cost"],
      o.bruteforce_joint(sub)["cost"])
print(oracle.icp_step(np.eye(3), np.eye(3) + 0.01, np.eye(3)))
print("sanitized oracle ok")
"""


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no ASan runtime")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run([gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-std=c11", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-shared",
                    "-fPIC", "-o", lib, os.path.join(ROOT, "oracle", "perch_oracle.c"), "-lm",
                    "-lpthread"], check=True)
    env = dict(os.environ, LD_PRELOAD=asan, PERCH_ORACLE_LIB=lib, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", DRIVER], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "sanitized oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
