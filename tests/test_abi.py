"""The C-ABI library loads and exports every entry point its header declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastmdp.h")


def _lib_path():
    from paper_2008_03518_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    return b.LIB


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fastmdp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("fastmdp_plan_request", "fastmdp_commit_plan", "fastmdp_eval_step", "fastmdp_create",
                 "fastmdp_destroy", "fastmdp_load_plans", "fastmdp_set_terrain", "fastmdp_plan_fcfs"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    _lib_path()
    from paper_2008_03518_amd import fastmdp as fm
    assert sorted(fm.EXPORTS) == declared_symbols()
    assert fm.strerror(fm.E_CONFLICT).startswith("commit refused")


def test_struct_layouts_match_header():
    """ctypes mirrors of the ABI structs have the C sizes (compiled probe)."""
    import subprocess
    import tempfile
    _lib_path()
    from paper_2008_03518_amd import fastmdp as fm
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "fastmdp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(fastmdp_config), sizeof(fastmdp_request), sizeof(fastmdp_plan),
         sizeof(fastmdp_state), offsetof(fastmdp_config, tie_rel), offsetof(fastmdp_config, lookahead));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "p")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    got = [ctypes.sizeof(fm._Config), ctypes.sizeof(fm._Request), ctypes.sizeof(fm._Plan),
           ctypes.sizeof(fm._State), fm._Config.tie_rel.offset, fm._Config.lookahead.offset]
    assert [int(x) for x in out] == got


def test_create_rejects_invalid_configs():
    """Configuration errors come back as E_INVAL before any device call."""
    import copy
    _lib_path()
    from paper_2008_03518_amd import fastmdp as fm
    from paper_2008_03518_amd import scenario as S
    base = S.cfg_small()
    out = ctypes.c_void_p()

    def create(**changes):
        cfg = copy.deepcopy(base)
        for k, v in changes.items():
            setattr(cfg, k, v)
        c = fm.make_config(cfg)
        return fm._lib.fastmdp_create(ctypes.byref(c), ctypes.byref(out))

    assert create(plan_capacity=254) == fm.E_INVAL       # rows are read four entries per lane
    assert create(plan_capacity=2) == fm.E_INVAL
    assert create(gamma=1.0) == fm.E_INVAL
    assert create(dt=0.0) == fm.E_INVAL
    assert create(max_steps=16383 + 1) == fm.E_INVAL
    assert create(max_rows=1) == fm.E_INVAL
    assert create(lookahead=17) == fm.E_INVAL           # windows of at most 16 steps
    assert create(lookahead=-1) == fm.E_INVAL
    assert fm._lib.fastmdp_create(None, ctypes.byref(out)) == fm.E_INVAL


def test_request_batch_layout_matches_struct():
    """The vectorised request marshalling writes the fastmdp_request bytes."""
    _lib_path()
    from paper_2008_03518_amd import fastmdp as fm
    from paper_2008_03518_amd import scenario as S
    assert ctypes.sizeof(fm._Request) == fm._REQUEST_DTYPE.itemsize
    sc = S.small(seed=0, n_requests=5)
    req = sc.requests
    a = fm._request_array(req, req.n)
    p = a.ctypes.data_as(ctypes.POINTER(fm._Request))
    for k in range(req.n):
        r = fm._request(req.origin[k], req.goal[k], int(req.t0[k]), int(req.ident[k]))
        assert bytes(p[k]) == bytes(r), k
