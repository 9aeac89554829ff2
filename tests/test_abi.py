"""The C-ABI library builds, loads and exports every symbol that
include/shapegrad.h declares; the ctypes layouts match the C structs.
No compute calls (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shapegrad.h")


def _lib_path():
    from paper_2311_05646_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2311_05646_amd import build
        build.build()
    return _lib.LIB_PATH


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:sg_status|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("eps_build", "eps_grad_vjp", "eps_grad_vjp_sparse", "eps_grad_vjp_geps", "eps_grad_fd",
              "eps_grad_fd_sparse", "sg_scene_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    path = _lib_path()
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2311_05646_amd import _lib
    _lib_path()
    assert sorted(_lib.SIGNATURES) == _declared()
    L = _lib.lib()
    for n in _declared():
        assert getattr(L, n) is not None


def test_struct_layouts():
    from paper_2311_05646_amd import _lib
    assert C.sizeof(_lib.sg_field) == 24
    assert C.sizeof(_lib.sg_sigma) == 16
    assert C.sizeof(_lib.sg_prim_desc) == 88
    assert C.sizeof(_lib.sg_node_desc) == 16
    assert C.sizeof(_lib.sg_scene_desc) == 160


def test_marshal_scene_tree_postfix():
    from paper_2311_05646_amd import _lib, workloads as W
    cfg = W.make_zoo(dim=3, root="difference")
    s, keep = _lib.marshal_scene(cfg["scene"])
    assert s.nnode == 3 and s.nprim == 8
    root = s.nodes_op[s.nnode - 1]
    assert root.op == _lib.OP["difference"] and root.nchild == 2
    assert [s.children[root.child_off + i] for i in range(2)] == [-1, -2]


def test_null_arguments_are_rejected_without_a_device():
    from paper_2311_05646_amd import _lib
    L = _lib.lib()
    assert L.sg_ctx_create(0, None) == -1
    assert L.sg_scene_create(None, None, None) == -1
    assert b"NULL" in L.sg_last_error()
    assert L.eps_build(None, None, None, 0, None, None) == -1
    assert L.sg_scene_set_deterministic(None, 1) == -1


def test_server_binding_makes_no_scene_level_calls():
    # a server handle is not a scene: the Server class must never pass its
    # handle to a call that takes an sg_scene*
    import inspect
    from paper_2311_05646_amd import api
    src = inspect.getsource(api.Server)
    assert "sg_scene_" not in src and "eps_" not in src
