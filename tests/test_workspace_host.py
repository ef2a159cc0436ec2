"""The workspace contract on the host (no GPU): sizes reported by
apsp_workspace_size, argument errors of apsp_set_workspace, and
APSP_E_NOMEM from the calls that need a workspace, all checked before any
device call.  A context with no device resources (APSP_FAULT=hostctx, a
host-side test hook like APSP_FAULT=create) stands in for a real one.  The
source check confirms that no compute entry point allocates or frees device
memory."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
API = os.path.join(ROOT, "paper_2310_03983_amd", "csrc", "api.cpp")

SCRIPT = r"""
import ctypes, sys
sys.path.insert(0, %(root)r)
from paper_2310_03983_amd import apsp as a
L = a.lib()
c = ctypes.c_void_p()
assert L.apsp_create(ctypes.byref(c), 0) == 0, a.last_error()
ws = L.apsp_workspace_size
def al(x): return (x + 255) // 256 * 256
# solve: the planner's feature pass (one int32 union-find parent per vertex)
assert ws(c, 0, 0, 16384, 0) == 256 + al(16384 * 4)
assert ws(c, 0, 1, 1, 0) == 0
# predecessors: flag, counts (ranges x n int32), offsets (+ ranges + 1, int64),
# then up to n^2/4 edges of 8 bytes, each part 256-byte aligned
n = 4096; nr = 4
want = 256 + al(nr * n * 4) + al((nr * n + nr + 1) * 8) + al(n * n // 4 * 8)
assert ws(c, 2, 0, n, 0) == want, (ws(c, 2, 0, n, 0), want)
assert ws(c, 2, 1, n, 0) == want
assert ws(c, 2, 0, 70000, 0) == 0          # dense only beyond 65535
assert ws(c, 2, 0, 1, 0) == 0
# batched: grows with the count and with the largest n
b1, b2, b3 = ws(c, 1, 0, 512, 100), ws(c, 1, 0, 512, 200), ws(c, 1, 0, 128, 200)
assert 0 < b3 < b2 and b1 < b2
assert ws(c, 1, 0, 512, 0) > 0
# invalid requests
assert ws(c, 9, 0, 10, 0) == 0 and "op" in a.last_error()
assert ws(c, 1, 7, 10, 1) == 0 and "dtype" in a.last_error()
assert ws(c, 1, 0, -1, 1) == 0
assert ws(None, 1, 0, 10, 1) == 0
# set_workspace argument errors
assert L.apsp_set_workspace(c, None, 64) == a.APSP_E_ARG
assert L.apsp_set_workspace(c, ctypes.c_void_p(0x10010), 64) == a.APSP_E_ARG
assert "aligned" in a.last_error()
assert L.apsp_set_workspace(c, None, 0) == 0
# batched with no workspace, then with one too small: NOMEM before any device call
sizes = (ctypes.c_int32 * 3)(300, 40, 512)
fake = ctypes.c_void_p(0x100000)
o = a.make_opts()
rc = L.apsp_batched(c, 0, 3, fake, fake, fake, sizes, ctypes.byref(o), None)
assert rc == a.APSP_E_NOMEM and "workspace" in a.last_error(), (rc, a.last_error())
need = ws(c, 1, 0, 512, 3)
assert L.apsp_set_workspace(c, ctypes.c_void_p(0x200000), 512) == 0
assert L.apsp_batched(c, 0, 3, fake, fake, fake, sizes, ctypes.byref(o), None) == a.APSP_E_NOMEM
assert str(512) in a.last_error()
# sparse predecessors without room for the fixed part: NOMEM
P = ctypes.c_void_p(0x900000)
rc = L.apsp_predecessors_ex(c, 0, 1000, fake, 1000, ctypes.c_void_p(0x500000), 1000, P, 1000, 2, None)
assert rc == a.APSP_E_NOMEM and "workspace" in a.last_error(), (rc, a.last_error())
# features need the workspace too
out4 = (ctypes.c_float * 4)()
assert L.apsp_set_workspace(c, None, 0) == 0
assert L.apsp_features(c, 0, 100, fake, 100, None, out4) == a.APSP_E_NOMEM
assert L.apsp_features(c, 0, 100, fake, 100, None, None) == a.APSP_E_ARG
ch = ctypes.c_int32(5)
assert L.apsp_solve_choice(c, ctypes.byref(ch)) == 0 and ch.value == -1
# path queries: argument errors come first
assert L.apsp_path(c, 10, fake, 10, -1, fake, fake, fake, 10, fake, None) == a.APSP_E_ARG
assert L.apsp_path(c, 10, fake, 10, 1, fake, fake, fake, 0, fake, None) == a.APSP_E_ARG
assert L.apsp_path(c, 10, fake, 10, 1, None, fake, fake, 10, fake, None) == a.APSP_E_ARG
assert L.apsp_path(c, 10, fake, 9, 1, fake, fake, fake, 10, fake, None) == a.APSP_E_ARG
assert L.apsp_path(c, 10, fake, 10, 0, None, None, None, 10, None, None) == 0
# deterministic mode: copies of the aliased operands (about n^2 / 2 elements)
assert ws(c, 3, 1, 1000, 0) == al(max(2 * (1000 * 1000 // 4), 256 * 1000) * 4)
assert ws(c, 3, 0, 100, 0) == al(256 * 100 * 4)
assert ws(c, 3, 1, 1, 0) == 0
od = a.make_opts(deterministic=True)
assert L.apsp_set_workspace(c, None, 0) == 0
for fn in (L.apsp_rkleene, L.apsp_fw, L.apsp_solve):
    rc = fn(c, 1, 1000, fake, 1000, ctypes.byref(od), None)
    assert rc == a.APSP_E_NOMEM and "DETERMINISTIC" in a.last_error(), (rc, a.last_error())
assert L.apsp_square(c, 1, 1000, fake, 1000, ctypes.byref(od), None) == a.APSP_E_UNSUPPORTED
# squaring pass count: nothing to report before the first apsp_square
npass = ctypes.c_int32(7)
assert L.apsp_square_passes(c, None, ctypes.byref(npass)) == a.APSP_E_STATE
assert L.apsp_square_passes(c, None, None) == a.APSP_E_ARG
print("host workspace checks ok", need)
"""


def test_workspace_contract_on_host():
    env = dict(os.environ, APSP_FAULT="hostctx", HIP_VISIBLE_DEVICES="")
    out = subprocess.run([sys.executable, "-c", SCRIPT % {"root": ROOT}], env=env, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "host workspace checks ok" in out.stdout


# entry points allowed to allocate or free device memory: context set-up and
# tear-down and the cost model's parameter set-up (not compute calls)
ALLOCATING = {"apsp_create", "apsp_destroy", "apsp_costmodel_init", "free_costmodel"}


def test_no_compute_call_allocates():
    src = open(API).read()
    current = None
    offenders = []
    for line in src.splitlines():
        m = re.match(r"^[A-Za-z_][\w:<>\s\*]*?\b(\w+)\s*\(", line)
        if m and not line.startswith((" ", "\t", "#", "//")) and not line.rstrip().endswith(";"):
            current = m.group(1)
        if re.search(r"\bhip(Malloc|Free|MallocAsync|FreeAsync|ExtMallocWithFlags|HostMalloc)\w*\s*\(", line):
            if current not in ALLOCATING:
                offenders.append((current, line.strip()))
    assert not offenders, offenders
