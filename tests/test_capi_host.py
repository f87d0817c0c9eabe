"""Host-side checks of the C ABI (no GPU needed, no kernel is ever launched).

* libm3s.so loads and exports every function include/m3s.h declares;
* the ctypes mirrors of the structs have the C compiler's layout;
* invalid arguments return the documented status codes before any HIP call.
"""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2412_12392_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "m3s.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(m3s_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_header_symbols_exported(lib):
    names = header_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), "libm3s.so does not export %s" % n
    assert sorted(_lib.EXPORTS) == names, "binding EXPORTS list differs from the header"
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (m3s_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_c(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "m3s.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(m3s_params), sizeof(m3s_pair), sizeof(m3s_outputs), sizeof(m3s_edge));
  printf("%zu %zu %zu %zu\n", offsetof(m3s_pair, Xii), offsetof(m3s_pair, p_init), offsetof(m3s_edge, out), offsetof(m3s_edge, refine_radius));
  printf("%zu %zu %zu\n", offsetof(m3s_params, max_dist), offsetof(m3s_outputs, xhat), offsetof(m3s_params, refine_levels));
  return 0;
}''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(_lib.Params), ctypes.sizeof(_lib.Pair), ctypes.sizeof(_lib.Outputs),
                    ctypes.sizeof(_lib.Edge),
                    _lib.Pair.Xii.offset, _lib.Pair.p_init.offset, _lib.Edge.out.offset, _lib.Edge.refine_radius.offset,
                    _lib.Params.max_dist.offset, _lib.Outputs.xhat.offset, _lib.Params.refine_levels.offset]


def test_defaults_and_strings(lib):
    p = _lib.default_params(lib)
    assert (p.max_iter, p.refine_radius, p.refine_levels) == (10, 3, 1)
    assert abs(p.lambda_init - 1e-8) < 1e-15 and abs(p.conf_min - 1.5) < 1e-7 and abs(p.max_theta - 1e-4) < 1e-10
    assert p.max_dist == float("inf")
    assert lib.m3s_version() == 2
    for s in range(7):
        assert lib.m3s_status_string(s)
    assert lib.m3s_status_string(99) == b"unknown status"


# Host buffers stand in for device pointers: every call below must fail
# validation, which happens before any HIP call, so nothing is dereferenced.
_buf = (ctypes.c_float * 64)()
_addr = ctypes.addressof(_buf)
_ws = (ctypes.c_char * 1024)()


def _pair(H=4, W=4, D=24, **kw):
    args = dict(Xii=_addr, Xji=_addr, Dii=_addr, Dji=_addr, Qii=0, Qji=0, p_init=0)
    args.update(kw)
    return _lib.Pair(H, W, D, args["Xii"], args["Xji"], args["Dii"], args["Dji"], args["Qii"], args["Qji"],
                     args["p_init"])


def _outs(**kw):
    args = dict(p=_addr, idx=_addr, valid=_addr, theta=0, xhat=0)
    args.update(kw)
    return _lib.Outputs(args["p"], args["idx"], args["valid"], args["theta"], args["xhat"])


def _fwd(lib, pair, prm=None, outs=None, ws=0, ws_bytes=0):
    prm = prm if prm is not None else _lib.default_params(lib)
    outs = outs if outs is not None else _outs()
    return lib.m3s_match_fwd(ctypes.byref(pair) if pair is not None else None, ctypes.byref(prm),
                             ctypes.byref(outs) if outs is not None else None, ws, ws_bytes, None)


@pytest.mark.parametrize("case,expect", [
    (dict(pair=None), 1),
    (dict(pair=dict(H=1)), 2),
    (dict(pair=dict(W=1)), 2),
    (dict(pair=dict(D=0)), 2),
    (dict(pair=dict(D=65)), 2),
    (dict(pair=dict(H=70000, W=70000)), 2),
    (dict(pair=dict(Xii=0)), 1),
    (dict(pair=dict(Dji=0)), 1),
    (dict(pair=dict(Qii=_addr)), 1),
    (dict(pair=dict(Xii=_addr + 1)), 3),
    (dict(outs=dict(p=0)), 1),
    (dict(outs=dict(valid=0)), 1),
    (dict(outs=dict(p=_addr + 4)), 3),
    (dict(prm=dict(max_iter=-1)), 3),
    (dict(prm=dict(max_iter=1001)), 3),
    (dict(prm=dict(refine_radius=9)), 3),
    (dict(prm=dict(refine_levels=0)), 3),
    (dict(prm=dict(refine_levels=5)), 3),
    (dict(prm=dict(lambda_init=0.0)), 3),
    (dict(prm=dict(lambda_init=float("nan"))), 3),
    (dict(prm=dict(max_theta=-1.0)), 3),
    (dict(prm=dict(max_dist=float("nan"))), 3),
    (dict(prm=dict(max_dist=0.0)), 3),
    (dict(prm=dict(conf_min=float("inf"))), 3),
    (dict(ws=0), 4),
    (dict(ws="misaligned"), 4),
    (dict(ws="small"), 4),
])
def test_fwd_validation(lib, case, expect):
    pair = None if case.get("pair", {}) is None else _pair(**case.get("pair", {}))
    prm = _lib.default_params(lib, **case.get("prm", {}))
    outs = _outs(**case.get("outs", {}))
    need = lib.m3s_workspace_bytes(ctypes.byref(_pair()), ctypes.byref(prm))
    ws_mode = case.get("ws", "none")
    base = (ctypes.addressof(_ws) + 255) // 256 * 256
    ws, nbytes = {"none": (0, 0), 0: (0, 0), "misaligned": (base + 4, 1 << 20), "small": (base, need - 1)}[ws_mode]
    st = _fwd(lib, pair, prm, outs, ws, nbytes)
    assert st == expect, (st, lib.m3s_last_error())
    assert lib.m3s_last_error()


def test_workspace_bytes(lib):
    prm = _lib.default_params(lib)
    assert lib.m3s_workspace_bytes(ctypes.byref(_pair(384, 512)), ctypes.byref(prm)) >= 384 * 512 * 36
    assert lib.m3s_workspace_bytes(ctypes.byref(_pair(1, 512)), ctypes.byref(prm)) == 0
    assert lib.m3s_workspace_bytes(None, ctypes.byref(prm)) == 0


def test_bwd_validation(lib):
    fwd = _outs()
    st = lib.m3s_match_bwd(None, ctypes.byref(fwd), _addr, 0, _addr, _addr, None)
    assert st == 1
    st = lib.m3s_match_bwd(ctypes.byref(_pair(H=1)), ctypes.byref(fwd), _addr, 0, _addr, _addr, None)
    assert st == 2
    st = lib.m3s_match_bwd(ctypes.byref(_pair()), ctypes.byref(_outs(valid=0)), _addr, 0, _addr, _addr, None)
    assert st == 1
    st = lib.m3s_match_bwd(ctypes.byref(_pair()), ctypes.byref(fwd), 0, 0, _addr, _addr, None)
    assert st == 1
    st = lib.m3s_match_bwd(ctypes.byref(_pair()), ctypes.byref(fwd), _addr + 1, 0, _addr, _addr, None)
    assert st == 3


def test_stats_validation(lib):
    outs = _outs()
    base = (ctypes.addressof(_ws) + 255) // 256 * 256
    assert lib.m3s_stats_workspace_bytes(384, 512) >= 384 * 512 // 8
    assert lib.m3s_stats_workspace_bytes(1, 512) == 0
    assert lib.m3s_match_stats(None, 4, 4, _addr, base, 1024, None) == 1
    assert lib.m3s_match_stats(ctypes.byref(outs), 1, 4, _addr, base, 1024, None) == 2
    assert lib.m3s_match_stats(ctypes.byref(outs), 4, 4, 0, base, 1024, None) == 1
    assert lib.m3s_match_stats(ctypes.byref(outs), 4, 4, _addr, 0, 0, None) == 4
    assert lib.m3s_match_stats(ctypes.byref(outs), 4, 4, _addr, base + 4, 1024, None) == 4


def test_batched_validation(lib):
    prm = _lib.default_params(lib)
    edges = (_lib.Edge * 2)()
    for e in edges:
        e.in_ = _pair()
        e.out = _outs()
        e.max_iter = -1
        e.refine_radius = -1
    assert lib.m3s_batched_workspace_bytes(edges, 2, ctypes.byref(prm)) > 0
    assert lib.m3s_match_batched(edges, 0, ctypes.byref(prm), 0, 0, 0, None) == 2
    assert lib.m3s_match_batched(None, 2, ctypes.byref(prm), 0, 0, 0, None) == 1
    assert lib.m3s_match_batched(edges, 2, ctypes.byref(prm), 0x8, 0, 0, None) == 6
    assert lib.m3s_match_batched(edges, 2, ctypes.byref(prm), 0, 0, 0, None) == 4
    edges[1].refine_radius = 9
    assert lib.m3s_match_batched(edges, 2, ctypes.byref(prm), 0, 0, 0, None) == 3
    assert lib.m3s_batched_workspace_bytes(edges, 2, ctypes.byref(prm)) == 0
    edges[1].refine_radius = -1
    edges[1].in_ = _pair(W=1)
    assert lib.m3s_match_batched(edges, 2, ctypes.byref(prm), 0, 0, 0, None) == 2
    assert b"edge 1" in lib.m3s_last_error()


def test_track_struct_layout(tmp_path):
    prog = tmp_path / "tlayout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "m3s.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(m3s_track_params), sizeof(m3s_track_problem),
         offsetof(m3s_track_params, huber), offsetof(m3s_track_problem, Xk), offsetof(m3s_track_problem, Qk));
  return 0;
}''')
    exe = tmp_path / "tlayout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(_lib.TrackParams), ctypes.sizeof(_lib.TrackProblem), _lib.TrackParams.huber.offset,
                    _lib.TrackProblem.Xk.offset, _lib.TrackProblem.Qk.offset]


def test_track_defaults_and_workspace(lib):
    p = _lib.default_track_params(lib)
    assert p.iters == 10 and abs(p.q_min - 1.5) < 1e-7 and abs(p.sigma_ray - 0.003) < 1e-9
    assert abs(p.sigma_dist - 0.1) < 1e-8 and abs(p.huber - 1.345) < 1e-6
    assert lib.m3s_track_workspace_bytes(384, 512) >= 256 + 192 * 37 * 4
    assert lib.m3s_track_workspace_bytes(384, 512) % 256 == 0
    assert lib.m3s_track_workspace_bytes(1, 512) == 0


def _track_prob(H=4, W=4, **kw):
    args = dict(Xk=_addr, Xf=_addr, idx=_addr, valid=_addr, Qf=_addr, Qk=_addr)
    args.update(kw)
    return _lib.TrackProblem(H, W, args["Xk"], args["Xf"], args["idx"], args["valid"], args["Qf"], args["Qk"])


@pytest.mark.parametrize("case,expect", [
    (dict(prob=None), 1),
    (dict(prob=dict(H=1)), 2),
    (dict(prob=dict(W=70000, H=70000)), 2),
    (dict(prob=dict(Xk=0)), 1),
    (dict(prob=dict(valid=0)), 1),
    (dict(prob=dict(Qk=0)), 1),
    (dict(T=0), 1),
    (dict(prob=dict(Xf=_addr + 2)), 3),
    (dict(T=_addr + 1), 3),
    (dict(prm=dict(iters=-1)), 3),
    (dict(prm=dict(iters=1001)), 3),
    (dict(prm=dict(q_min=float("nan"))), 3),
    (dict(prm=dict(sigma_ray=0.0)), 3),
    (dict(prm=dict(sigma_dist=float("nan"))), 3),
    (dict(prm=dict(huber=-1.0)), 3),
    (dict(ws=0), 4),
    (dict(ws="misaligned"), 4),
    (dict(ws="small"), 4),
])
def test_track_validation(lib, case, expect):
    prob = None if case.get("prob", {}) is None else _track_prob(**case.get("prob", {}))
    prm = _lib.default_track_params(lib, **case.get("prm", {}))
    need = lib.m3s_track_workspace_bytes(4, 4)
    base = (ctypes.addressof(_ws) + 255) // 256 * 256
    ws, nbytes = {"none": (0, 0), 0: (0, 0), "misaligned": (base + 4, 1024), "small": (base, need - 1)}[
        case.get("ws", "none")]
    T = case.get("T", _addr)
    st = lib.m3s_track_pose(ctypes.byref(prob) if prob is not None else None, ctypes.byref(prm), T, 0, ws, nbytes,
                            None)
    assert st == expect, (st, lib.m3s_last_error())
    assert lib.m3s_last_error()


def test_fuse_validation(lib):
    ok = _lib.FuseProblem(4, 4, _addr, _addr, _addr, _addr)
    assert lib.m3s_fuse_pointmap(None, _addr, None) == 1
    assert lib.m3s_fuse_pointmap(ctypes.byref(ok), 0, None) == 1
    assert lib.m3s_fuse_pointmap(ctypes.byref(_lib.FuseProblem(1, 4, _addr, _addr, _addr, _addr)), _addr, None) == 2
    assert lib.m3s_fuse_pointmap(ctypes.byref(_lib.FuseProblem(4, 4, 0, _addr, _addr, _addr)), _addr, None) == 1
    assert lib.m3s_fuse_pointmap(ctypes.byref(_lib.FuseProblem(4, 4, _addr, _addr, _addr + 2, _addr)), _addr, None) == 3
    assert lib.m3s_fuse_pointmap(ctypes.byref(ok), _addr + 1, None) == 3
    assert lib.m3s_last_error()


def test_backend_struct_layout(tmp_path):
    prog = tmp_path / "blayout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "m3s.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(m3s_backend_params), sizeof(m3s_backend_problem),
         offsetof(m3s_backend_params, step_tol), offsetof(m3s_backend_problem, Xc), offsetof(m3s_backend_problem, valid));
  return 0;
}''')
    exe = tmp_path / "blayout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(_lib.BackendParams), ctypes.sizeof(_lib.BackendProblem),
                    _lib.BackendParams.step_tol.offset, _lib.BackendProblem.Xc.offset, _lib.BackendProblem.valid.offset]


def test_backend_workspace(lib):
    p = _lib.default_backend_params(lib)
    assert p.iters == 10 and p.step_tol == 0.0 and abs(p.sigma_ray - 0.003) < 1e-9
    n = 7 * 31
    # the solve's matrix (fp64) plus one 40-float partial per accumulation
    # workgroup: 16 matches per lane, 256 lanes, so ceil(HW / 4096) per edge
    bpe = -(-384 * 512 // 4096)
    assert lib.m3s_backend_workspace_bytes(32, 384, 512, 64) >= n * n * 8 + 64 * bpe * 40 * 4
    assert lib.m3s_backend_workspace_bytes(32, 384, 512, 64) % 256 == 0
    assert lib.m3s_backend_workspace_bytes(1, 384, 512, 64) == 0
    assert lib.m3s_backend_workspace_bytes(129, 384, 512, 64) == 0
    assert lib.m3s_backend_workspace_bytes(4, 384, 512, 0) == 0


def _backend_prob(N=3, H=4, W=4, E=2, **kw):
    args = dict(Xc=_addr, Q=_addr, edges=_addr, idx=_addr, valid=_addr)
    args.update(kw)
    return _lib.BackendProblem(N, H, W, E, args["Xc"], args["Q"], args["edges"], args["idx"], args["valid"])


@pytest.mark.parametrize("case,expect", [
    (dict(prob=None), 1),
    (dict(prob=dict(H=1)), 2),
    (dict(prob=dict(N=1)), 2),
    (dict(prob=dict(N=129)), 2),
    (dict(prob=dict(E=0)), 2),
    (dict(prob=dict(E=65536)), 2),
    (dict(prob=dict(edges=0)), 1),
    (dict(prob=dict(valid=0)), 1),
    (dict(T=0), 1),
    (dict(prob=dict(idx=_addr + 2)), 3),
    (dict(prm=dict(iters=-1)), 3),
    (dict(prm=dict(step_tol=-1.0)), 3),
    (dict(prm=dict(step_tol=float("nan"))), 3),
    (dict(prm=dict(sigma_dist=0.0)), 3),
    (dict(prm=dict(huber=float("nan"))), 3),
    (dict(ws=0), 4),
    (dict(ws="misaligned"), 4),
    (dict(ws="small"), 4),
])
def test_backend_validation(lib, case, expect):
    prob = None if case.get("prob", {}) is None else _backend_prob(**case.get("prob", {}))
    prm = _lib.default_backend_params(lib, **case.get("prm", {}))
    need = lib.m3s_backend_workspace_bytes(3, 4, 4, 2)
    big = (ctypes.c_char * (need + 512))()
    base = (ctypes.addressof(big) + 255) // 256 * 256
    ws, nbytes = {"none": (0, 0), 0: (0, 0), "misaligned": (base + 4, need), "small": (base, need - 1)}[
        case.get("ws", "none")]
    T = case.get("T", _addr)
    st = lib.m3s_backend_gn(ctypes.byref(prob) if prob is not None else None, ctypes.byref(prm), T, 0, ws, nbytes,
                            None)
    assert st == expect, (st, lib.m3s_last_error())
    assert lib.m3s_last_error()


@pytest.mark.parametrize("case,expect", [
    (dict(pair=None), 1),
    (dict(pair=dict(H=1)), 2),
    (dict(pair=dict(H=513, W=512)), 2),          # above M3S_NOALLOC_MAX_PIXELS
    (dict(pair=dict(Dji=0)), 1),
    (dict(outs=dict(idx=0)), 1),
    (dict(prm=dict(refine_radius=9)), 3),
])
def test_noalloc_validation(lib, case, expect):
    """m3s_match_fwd_noalloc validates like m3s_match_fwd and rejects frames above
    its scratch limit, all before any HIP call."""
    pair = None if case.get("pair", {}) is None else _pair(**case.get("pair", {}))
    prm = _lib.default_params(lib, **case.get("prm", {}))
    outs = _outs(**case.get("outs", {}))
    st = lib.m3s_match_fwd_noalloc(ctypes.byref(pair) if pair is not None else None, ctypes.byref(prm),
                                   ctypes.byref(outs), None)
    assert st == expect, (st, lib.m3s_last_error())
    if expect == 2 and pair is not None and pair.H == 513:
        assert b"M3S_NOALLOC_MAX_PIXELS" in lib.m3s_last_error()
    assert _lib.M3S_NOALLOC_MAX_PIXELS == 1 << 18


def test_launch_override_struct_and_counters_null(tmp_path, lib):
    prog = tmp_path / "launch.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "m3s.h"
int main(void) {
  printf("%zu %zu %zu %zu %d\n", sizeof(m3s_launch_config), offsetof(m3s_launch_config, grid),
         offsetof(m3s_launch_config, xcd_remap), offsetof(m3s_launch_config, lm_unroll), M3S_PATH_COUNTERS);
  return 0;
}''')
    exe = tmp_path / "launch"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(_lib.LaunchConfig), _lib.LaunchConfig.grid.offset,
                    _lib.LaunchConfig.xcd_remap.offset, _lib.LaunchConfig.lm_unroll.offset, _lib.M3S_PATH_COUNTERS]
    cfg = _lib.LaunchConfig(3, 64, 0, 1, 2)
    lib.m3s_debug_set_launch(ctypes.byref(cfg))
    lib.m3s_debug_set_launch(None)
    assert lib.m3s_path_counters(None, 0) == 1


def test_bwd_batched_validation(tmp_path, lib):
    """m3s_match_bwd_batched: struct layout, workspace size and argument errors before any HIP call."""
    prog = tmp_path / "bwdb.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "m3s.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(m3s_bwd_edge), offsetof(m3s_bwd_edge, grad_xhat), offsetof(m3s_bwd_edge, grad_Xji));
  return 0;
}''')
    exe = tmp_path / "bwdb"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(_lib.BwdEdge), _lib.BwdEdge.grad_xhat.offset, _lib.BwdEdge.grad_Xji.offset]
    assert lib.m3s_bwd_batched_workspace_bytes(0) == 0
    need = lib.m3s_bwd_batched_workspace_bytes(3)
    assert need >= 256 + 3 * 80
    base = (ctypes.addressof(_ws) + 255) // 256 * 256
    good = _lib.BwdEdge(4, 4, _addr, _addr, _addr, _addr, _addr, 0, _addr, _addr)
    cases = [
        (None, 1, 0, (base, 1024), 1),
        ([good], 0, 0, (base, 1024), 2),
        ([good], 1, 0x8, (base, 1024), 6),
        ([good], 1, 0x2, (base, 1024), 6),
        ([_lib.BwdEdge(1, 4, _addr, _addr, _addr, _addr, _addr, 0, _addr, _addr)], 1, 0, (base, 1024), 2),
        ([_lib.BwdEdge(4, 4, 0, _addr, _addr, _addr, _addr, 0, _addr, _addr)], 1, 0, (base, 1024), 1),
        ([_lib.BwdEdge(4, 4, _addr, _addr, _addr, _addr, 0, 0, _addr, _addr)], 1, 0, (base, 1024), 1),
        ([_lib.BwdEdge(4, 4, _addr, _addr, _addr, _addr, _addr, 0, _addr + 2, _addr)], 1, 0, (base, 1024), 3),
        ([good], 1, 0, (0, 0), 4),
        ([good], 1, 0, (base + 4, 1024), 4),
    ]
    for edges, n, flags, (ws, nb), expect in cases:
        arr = None if edges is None else (_lib.BwdEdge * len(edges))(*edges)
        st = lib.m3s_match_bwd_batched(arr, n, flags, ws, nb, None)
        assert st == expect, (edges, n, flags, st, lib.m3s_last_error())


def test_tune_cache_file_validation(lib, tmp_path):
    """m3s_set_tune_cache: a missing file is accepted (created on the first
    tuning), a file of this format loads, anything else is refused."""
    missing = tmp_path / "none.json"
    assert lib.m3s_set_tune_cache(str(missing).encode()) == 0
    good = tmp_path / "good.json"
    good.write_text('{"format": "m3s-autotune", "version": 1, "entries": {"gfx950|256cu|0,384,512,24,10,3,5;RL1": '
                    '[5, 1024, 2, 1]}}')
    assert lib.m3s_set_tune_cache(str(good).encode()) == 0
    for text in ['{}', '{"format": "m3s-autotune", "version": 2, "entries": {}}',
                 '{"format": "m3s-autotune", "version": 1, "entries": {"k": [9, 1, 2, 1]}}',
                 '{"format": "m3s-autotune", "version": 1, "entries": {"k": [5, 1, 4, 1]}}',
                 '{"format": "m3s-autotune", "version": 1, "entries": {"k": [5, 1, 2]}}']:
        bad = tmp_path / "bad.json"
        bad.write_text(text)
        assert lib.m3s_set_tune_cache(str(bad).encode()) == 3, text
    assert lib.m3s_set_tune_cache(None) == 0
    lib.m3s_clear_caches()
