"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's C source and a small driver (tests/sanitize/oracle_driver.c)
are built with gcc -fsanitize=address,undefined and run on seeded
scenarios (the small box without terrain, the paper-scale box with its
terrain heightmap): the run must be clean, and every plan, commit and
scored step must equal the uninstrumented oracle's, which the other CPU
tests pin to the paper.
"""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, TIE_REL, AMB_BAND  # noqa: E402
from paper_2008_03518_amd import scenario as S  # noqa: E402

DRIVER = os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")
ORACLE_C = os.path.join(ROOT, "oracle", "fastmdp_oracle.c")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-D_DEFAULT_SOURCE", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", ORACLE_C, DRIVER, "-o", exe, "-lm"]
    subprocess.run(cmd, check=True)
    return exe


def _write(path, sc, n_req):
    c, p, r, t = sc.cfg, sc.plans, sc.requests, sc.terrain
    nx, ny = (t.nx, t.ny) if t is not None else (0, 0)
    with open(path, "wb") as f:
        np.array([c.n_head, len(c.climb), len(c.speed), c.max_steps, p.n, n_req, nx, ny], np.int32).tofile(f)
        np.array(list(c.box_min) + list(c.box_max) + [c.dt, c.gamma, c.r_goal, c.r_intr, c.R_intr, c.gamma_intr,
                                                      c.R_sep, c.r_terr, c.R_terr, c.gamma_terr, TIE_REL, AMB_BAND],
                 np.float64).tofile(f)
        np.array(c.climb, np.float64).tofile(f)
        np.array(c.speed, np.float64).tofile(f)
        if t is not None:
            np.array([t.x0, t.y0, t.cell], np.float64).tofile(f)
        p.t0.astype(np.int32).tofile(f)
        p.length.astype(np.int32).tofile(f)
        p.xyz.astype(np.float32).tofile(f)
        r.origin[:n_req].astype(np.float64).tofile(f)
        r.goal[:n_req].astype(np.float64).tofile(f)
        r.t0[:n_req].astype(np.int32).tofile(f)
        if t is not None:
            t.h.astype(np.float32).tofile(f)


@pytest.mark.parametrize("name", ["small", "paper_scale"])
def test_oracle_clean_under_sanitizers(driver, tmp_path, name):
    if name == "small":
        sc, n_req = S.small(seed=3, n_plans=120, n_requests=4), 4
    else:
        sc, n_req = S.paper_scale(seed=1, n_plans=150, n_requests=2), 2
    inp = str(tmp_path / "in.bin")
    _write(inp, sc, n_req)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([driver, inp], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr, res.stderr[-4000:]
    lines = res.stdout.strip().splitlines()
    orc = Oracle(sc.cfg, sc.plans, sc.terrain)
    for q in range(n_req):
        p = orc.plan(sc.requests.origin[q], sc.requests.goal[q], int(sc.requests.t0[q]))
        com = orc.commit(p) if p.status == 0 else False
        f = lines[q].split()
        assert int(f[1]) == p.status and int(f[2]) == p.n_points and int(f[3]) == int(com), (q, f)
        assert np.array_equal(np.array([float(x) for x in f[4:7]]), p.xyz[-1])
    ev = lines[n_req].split()
    assert ev[0] == "eval"
    o = Oracle(sc.cfg, sc.plans, sc.terrain)
    for q in range(n_req):                     # the driver scored request 0 after committing every plan
        pq = o.plan(sc.requests.origin[q], sc.requests.goal[q], int(sc.requests.t0[q]))
        if pq.status == 0:
            o.commit(pq)
    e = o.eval_step(sc.requests.origin[0], sc.requests.goal[0], int(sc.requests.t0[0]))
    assert int(ev[1]) == e["best"]
    assert np.array_equal(np.array([float(x) for x in ev[2:]]), e["V"])
