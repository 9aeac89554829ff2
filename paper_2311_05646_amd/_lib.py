"""ctypes declarations of include/shapegrad.h and marshalling of scene
descriptions (see ``workloads`` for the dict format) into sg_scene_desc.

Loading fails loudly when libshapegrad.so is missing: there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SG_LIB_PATH selects another build of the same library (the host-only
# sanitizer builds of build.build_host_sanitized)
LIB_PATH = os.environ.get("SG_LIB_PATH") or os.path.join(HERE, "libshapegrad.so")

SG_OK, SG_EAGAIN = 0, 1
STATUS = {0: "SG_OK", 1: "SG_EAGAIN", -1: "SG_E_INVALID", -2: "SG_E_NOMEM", -3: "SG_E_TOO_LARGE",
          -4: "SG_E_DEVICE", -5: "SG_E_CANCELLED", -6: "SG_E_TIMEOUT", -7: "SG_E_UNSUPPORTED"}
PRIM = {"box": 0, "ellipse": 1, "poly": 2, "gcart": 3, "polar": 4, "series": 5, "polar2d": 6}
SIGMA = {"sigmoid": 0, "erf": 1, "sin": 2, "linear": 3, "quadratic": 4}
KMODE = {"local": 0, "fixed": 1}
OP = {"union": 0, "intersection": 1, "difference": 2, "levels": 3}
AXIS = {"x": 0, "y": 1, "z": 2}
FD_SCHEME = {"central": 0, "forward": 1}
MODE = {"eps": 0, "vjp": 1, "geps": 2, "fd": 3, "sparse": 4, "fd_sparse": 5}


class sg_field(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("idx", C.c_int64)]


class sg_sigma(C.Structure):
    _fields_ = [("kind", C.c_int32), ("kmode", C.c_int32), ("k", C.c_double)]


class sg_prim_desc(C.Structure):
    _fields_ = [("type", C.c_int32), ("nvert", C.c_int32), ("field_off", C.c_int32), ("nfield", C.c_int32),
                ("const_off", C.c_int32), ("nconst", C.c_int32), ("bounded", C.c_int32 * 3), ("pad", C.c_int32),
                ("sigma", sg_sigma * 3)]


class sg_node_desc(C.Structure):
    _fields_ = [("op", C.c_int32), ("nchild", C.c_int32), ("child_off", C.c_int32), ("aux", C.c_int32)]


class sg_scene_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("ncomp", C.c_int32), ("comp_axis", C.c_int32 * 3), ("pad0", C.c_int32),
                ("n", C.c_int64 * 3), ("nodes", C.POINTER(C.c_double) * 3), ("eps_bg", C.c_double),
                ("eps_fg", C.c_double), ("n_params", C.c_int64), ("nprim", C.c_int32), ("nfield", C.c_int32),
                ("nconst", C.c_int32), ("nnode", C.c_int32), ("nchild", C.c_int32), ("pad1", C.c_int32),
                ("prims", C.POINTER(sg_prim_desc)), ("fields", C.POINTER(sg_field)),
                ("consts", C.POINTER(C.c_double)), ("nodes_op", C.POINTER(sg_node_desc)),
                ("children", C.POINTER(C.c_int32))]


class sg_server_opts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_slots", C.c_int32), ("max_batch", C.c_int32),
                ("n_streams", C.c_int32), ("fake_executor", C.c_int32), ("fake_us", C.c_int64),
                ("max_launch_us", C.c_int64)]


class sg_req_stats(C.Structure):
    _fields_ = [("submit_ns", C.c_int64), ("admit_ns", C.c_int64), ("launch_ns", C.c_int64), ("done_ns", C.c_int64),
                ("batch_size", C.c_int32), ("pad", C.c_int32)]


_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_S = C.c_int32

# name -> (restype, argtypes); every symbol include/shapegrad.h declares
SIGNATURES = {
    "sg_ctx_create": (_S, [_I, C.POINTER(_P)]),
    "sg_ctx_destroy": (None, [_P]),
    "sg_last_error": (C.c_char_p, []),
    "sg_scene_create": (_S, [_P, C.POINTER(sg_scene_desc), C.POINTER(_P)]),
    "sg_scene_destroy": (None, [_P]),
    "sg_scene_info": (_S, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "sg_scene_set_launch": (_S, [_P, C.c_int32, C.c_int32]),
    "sg_scene_set_deterministic": (_S, [_P, _I]),
    "eps_build": (_S, [_P, _P, _P, _I, _P, _P]),
    "eps_grad_vjp": (_S, [_P, _P, _P, _I, _P, _P, _D, _P, _I, _P]),
    "eps_grad_vjp_noalloc": (_S, [_P, _P, _P, _I, _P, _P, _D, _P, _I, _P]),
    "eps_grad_vjp_geps": (_S, [_P, _P, _P, _I, _P, _P, _I, _P]),
    "eps_grad_vjp_sparse": (_S, [_P, _P, _P, _I, _P, _P, _D, _P, _I, _P]),
    "sg_scene_sparse_reads": (_S, [_P, C.POINTER(C.c_int64)]),
    "eps_grad_fd": (_S, [_P, _P, _P, _I, _P, _P, _D, _D, _I, _P, _I, _P]),
    "eps_grad_fd_sparse": (_S, [_P, _P, _P, _I, _P, _P, _D, _D, _I, _P, _I, _P]),
    "sg_scene_set_timing": (_S, [_P, _I]),
    "sg_scene_kernel_time": (_S, [_P, _I, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "sg_util_copy": (_S, [_P, _P, C.c_int64, _P]),
    "sg_fieldgen": (_S, [_P, _P, C.c_int64, C.c_uint64, _P]),
    "sg_server_create": (_S, [_P, C.POINTER(sg_server_opts), C.POINTER(_P)]),
    "sg_server_destroy": (_S, [_P]),
    "serve_open_session": (_S, [_P, _P, C.POINTER(C.c_uint32)]),
    "serve_open_fake_session": (_S, [_P, C.c_int64, C.c_int64, C.POINTER(C.c_uint32)]),
    "serve_submit": (_S, [_P, C.c_uint32, _P, C.c_uint64, _D, C.POINTER(C.c_uint64)]),
    "serve_submit_fields": (_S, [_P, C.c_uint32, _P, _P, _P, _D, C.POINTER(C.c_uint64)]),
    "serve_poll": (_S, [_P, C.c_uint64, _P, C.c_int64, C.POINTER(sg_req_stats)]),
    "serve_cancel": (_S, [_P, C.c_uint64]),
    "serve_counters": (_S, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                            C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
}

_lib = None


def lib():
    """The loaded C-ABI library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_05646_amd.build` "
                               "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class SGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def check(code):
    if code < 0:
        raise SGError(code, lib().sg_last_error().decode())
    return code


def marshal_scene(desc):
    """Build an sg_scene_desc from a scene dict.  Returns (struct, keepalive)."""
    X, Y, Z = [np.ascontiguousarray(a, dtype=np.float64) for a in desc["nodes"]]
    keep = [X, Y, Z]
    prims = desc["prims"]
    fields, consts, pd = [], [], (sg_prim_desc * len(prims))()
    for i, pr in enumerate(prims):
        d = pd[i]
        d.type = PRIM[pr["type"]]
        d.nvert = int(pr.get("nvert", 0))
        d.field_off = len(fields)
        d.nfield = len(pr["fields"])
        fields += list(pr["fields"])
        d.const_off = len(consts)
        d.nconst = len(pr.get("consts", []))
        consts += list(pr.get("consts", []))
        for a in range(3):
            d.bounded[a] = int(bool(pr["bounded"][a]))
            kind, kmode, k = pr["sigma"][a]
            d.sigma[a].kind = SIGMA[kind]
            d.sigma[a].kmode = KMODE[kmode]
            d.sigma[a].k = float(k)
    fa = (sg_field * max(1, len(fields)))()
    for i, (a, b, idx) in enumerate(fields):
        fa[i].a, fa[i].b, fa[i].idx = float(a), float(b), int(idx)
    # op tree -> postfix node list
    nodes, children = [], []

    def walk(node):
        if isinstance(node, (int, np.integer)):
            return int(node)
        ch = [walk(c) for c in node["children"]]
        aux = 0
        if node["op"] == "levels":      # level values go after the primitives' constants
            aux = len(consts)
            consts.extend(float(x) for x in node["levels"])
        nodes.append((OP[node["op"]], ch, aux))
        return -len(nodes)          # node k is referenced as -(k + 1)

    walk(desc["tree"])
    ca = (C.c_double * max(1, len(consts)))(*[float(c) for c in consts])
    na = (sg_node_desc * len(nodes))()
    for k, (op, ch, aux) in enumerate(nodes):
        na[k].op = op
        na[k].nchild = len(ch)
        na[k].child_off = len(children)
        na[k].aux = aux
        children += ch
    cha = (C.c_int32 * len(children))(*children)
    s = sg_scene_desc()
    s.dim = int(desc["dim"])
    s.ncomp = len(desc["components"])
    for c, ax in enumerate(desc["components"]):
        s.comp_axis[c] = AXIS[ax]
    for a, arr in enumerate((X, Y, Z)):
        s.n[a] = len(arr) - 1
        s.nodes[a] = arr.ctypes.data_as(C.POINTER(C.c_double))
    s.eps_bg = float(desc["eps_bg"])
    s.eps_fg = float(desc["eps_fg"])
    s.n_params = int(desc["n_params"])
    s.nprim, s.nfield, s.nconst = len(prims), len(fields), len(consts)
    s.nnode, s.nchild = len(nodes), len(children)
    s.prims = C.cast(pd, C.POINTER(sg_prim_desc))
    s.fields = C.cast(fa, C.POINTER(sg_field))
    s.consts = C.cast(ca, C.POINTER(C.c_double))
    s.nodes_op = C.cast(na, C.POINTER(sg_node_desc))
    s.children = C.cast(cha, C.POINTER(C.c_int32))
    keep += [pd, fa, ca, na, cha]
    return s, keep
