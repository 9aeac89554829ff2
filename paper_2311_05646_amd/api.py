"""Python binding of the C-ABI (argument marshalling only; every step of the
path runs in the HIP kernels of libshapegrad.so).  PyTorch supplies device
memory and the current HIP stream.

    scene = Scene(desc)                     # desc: see paper_2311_05646_amd.workloads
    eps = eps_build(scene, p)               # (C, Nz, Ny, Nx) float32 on the GPU
    g = eps_grad_vjp(scene, p, E, A, omega) # eq:1 / eq:AD fused adjoint gradient
    g = eps_grad_vjp_geps(scene, p, dFdeps) # reverse mode with an upstream dF/deps
    g = eps_grad_fd(scene, p, E, A, omega, h)  # finite-difference baseline
    eps = EpsBuild.apply(p_tensor, scene)   # autograd; backward = eps_grad_vjp_geps
"""
import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

_CTX = {}


def context(device=0):
    if device not in _CTX:
        h = C.c_void_p()
        check(lib().sg_ctx_create(int(device), C.byref(h)))
        _CTX[device] = h
    return _CTX[device]


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Scene:
    """A compiled scene (device tables) on one GPU."""

    def __init__(self, desc, device=0):
        self.desc = desc
        self.device = device
        self.ctx = context(device)
        sd, keep = _lib.marshal_scene(desc)
        h = C.c_void_p()
        check(lib().sg_scene_create(self.ctx, C.byref(sd), C.byref(h)))
        self.handle = h
        n = C.c_int64()
        nc = C.c_int32()
        dims = (C.c_int64 * 3)()
        check(lib().sg_scene_info(h, C.byref(n), C.byref(nc), dims))
        self.n_params = n.value
        self.ncomp = nc.value
        self.dims = tuple(dims)                       # (Nx, Ny, Nz)
        self.shape = (self.ncomp, dims[2], dims[1], dims[0])

    def set_launch(self, block_x=0, col_segments=0):
        check(lib().sg_scene_set_launch(self.handle, int(block_x), int(col_segments)))

    def set_deterministic(self, enable=True):
        """Two-pass (atomic-free) gradient reduction: bitwise-repeatable."""
        check(lib().sg_scene_set_deterministic(self.handle, int(bool(enable))))

    def set_timing(self, enable=True, every=1):
        """Trace the column kernel of later calls (HIP events on the call's
        stream): every `every`-th launch of each kind; enabling clears
        earlier records."""
        check(lib().sg_scene_set_timing(self.handle, int(every) if enable else 0))

    def kernel_time(self, mode):
        """(summed ms, launches) of the traced column kernels of one kind:
        'eps', 'vjp', 'geps', 'fd', 'sparse' or 'fd_sparse'."""
        t = C.c_double()
        n = C.c_int64()
        check(lib().sg_scene_kernel_time(self.handle, _lib.MODE[mode], C.byref(t), C.byref(n)))
        return t.value, n.value

    def sparse_reads(self):
        """(sample, column step) pairs whose fields the last eps_grad_vjp_sparse
        call read."""
        n = C.c_int64()
        check(lib().sg_scene_sparse_reads(self.handle, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "handle", None):
            lib().sg_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _p_arg(scene, p):
    """(pointer, on_device, keepalive) for p (numpy/list on host, or a CUDA
    float64 tensor)."""
    if isinstance(p, torch.Tensor) and p.is_cuda:
        if p.dtype != torch.float64 or not p.is_contiguous() or p.numel() != scene.n_params:
            raise ValueError("device p must be a contiguous float64 tensor of n_params")
        return C.c_void_p(p.data_ptr()), 1, p
    a = np.ascontiguousarray(np.asarray(p.detach().cpu() if isinstance(p, torch.Tensor) else p, dtype=np.float64))
    if a.size != scene.n_params:
        raise ValueError(f"p has {a.size} values, the scene has {scene.n_params} parameters")
    return C.c_void_p(a.ctypes.data), 0, a


def _plane_ptrs(scene, F):
    if not (isinstance(F, torch.Tensor) and F.is_cuda and F.dtype == torch.complex64 and F.is_contiguous()):
        raise ValueError("fields must be contiguous complex64 CUDA tensors")
    if tuple(F.shape) != scene.shape:
        raise ValueError(f"field shape {tuple(F.shape)} != {scene.shape}")
    step = F[0].numel() * 8
    base = F.data_ptr()
    return (C.c_void_p * 3)(*[base + c * step for c in range(scene.ncomp)] + [0] * (3 - scene.ncomp))


def _grad_out(scene, p_dev, grad, device):
    if grad is not None:
        if not (grad.is_cuda and grad.dtype == torch.float64 and grad.numel() == scene.n_params):
            raise ValueError("grad must be a float64 CUDA tensor of n_params")
        return grad, C.c_void_p(grad.data_ptr()), 1
    if p_dev:
        g = torch.empty(scene.n_params, dtype=torch.float64, device=device)
        return g, C.c_void_p(g.data_ptr()), 1
    g = np.empty(scene.n_params, dtype=np.float64)
    return g, C.c_void_p(g.ctypes.data), 0


def eps_build(scene, p, out=None, stream=None):
    dev = torch.device("cuda", scene.device)
    if out is None:
        out = torch.empty(scene.shape, dtype=torch.float32, device=dev)
    elif not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous() and tuple(out.shape) == scene.shape):
        raise ValueError("out must be a contiguous float32 CUDA tensor of the scene's plane shape")
    pp, pdev, keep = _p_arg(scene, p)
    check(lib().eps_build(scene.ctx, scene.handle, pp, pdev, C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def eps_grad_vjp(scene, p, E, A, omega, grad=None, stream=None):
    dev = torch.device("cuda", scene.device)
    pp, pdev, keep = _p_arg(scene, p)
    fe, fa = _plane_ptrs(scene, E), _plane_ptrs(scene, A)
    g, gp, gdev = _grad_out(scene, pdev, grad, dev)
    check(lib().eps_grad_vjp(scene.ctx, scene.handle, pp, pdev, fe, fa, float(omega), gp, gdev, _stream(stream)))
    return g


def eps_grad_vjp_noalloc(scene, p, E, A, omega, grad=None, stream=None):
    """eps_grad_vjp whose call allocates no device memory (its staging lives in
    the library's per-device scratch array; overlapping calls on one device race)."""
    dev = torch.device("cuda", scene.device)
    pp, pdev, keep = _p_arg(scene, p)
    fe, fa = _plane_ptrs(scene, E), _plane_ptrs(scene, A)
    g, gp, gdev = _grad_out(scene, pdev, grad, dev)
    check(lib().eps_grad_vjp_noalloc(scene.ctx, scene.handle, pp, pdev, fe, fa, float(omega), gp, gdev,
                                     _stream(stream)))
    return g


def eps_grad_vjp_sparse(scene, p, E, A, omega, grad=None, stream=None):
    """eps_grad_vjp that reads the fields only where d eps / d p can be nonzero."""
    dev = torch.device("cuda", scene.device)
    pp, pdev, keep = _p_arg(scene, p)
    fe, fa = _plane_ptrs(scene, E), _plane_ptrs(scene, A)
    g, gp, gdev = _grad_out(scene, pdev, grad, dev)
    check(lib().eps_grad_vjp_sparse(scene.ctx, scene.handle, pp, pdev, fe, fa, float(omega), gp, gdev,
                                    _stream(stream)))
    return g


def eps_grad_vjp_geps(scene, p, geps, grad=None, stream=None):
    dev = torch.device("cuda", scene.device)
    if not (geps.is_cuda and geps.dtype == torch.float32 and geps.is_contiguous() and tuple(geps.shape) == scene.shape):
        raise ValueError("grad_eps must be a contiguous float32 CUDA tensor of the scene's plane shape")
    pp, pdev, keep = _p_arg(scene, p)
    g, gp, gdev = _grad_out(scene, pdev, grad, dev)
    check(lib().eps_grad_vjp_geps(scene.ctx, scene.handle, pp, pdev, C.c_void_p(geps.data_ptr()), gp, gdev,
                                  _stream(stream)))
    return g


def eps_grad_fd(scene, p, E, A, omega, h, scheme="central", grad=None, stream=None):
    dev = torch.device("cuda", scene.device)
    pp, pdev, keep = _p_arg(scene, p)
    fe, fa = _plane_ptrs(scene, E), _plane_ptrs(scene, A)
    g, gp, gdev = _grad_out(scene, pdev, grad, dev)
    check(lib().eps_grad_fd(scene.ctx, scene.handle, pp, pdev, fe, fa, float(omega), float(h),
                            _lib.FD_SCHEME[scheme], gp, gdev, _stream(stream)))
    return g


def eps_grad_fd_sparse(scene, p, E, A, omega, h, scheme="central", grad=None, stream=None):
    """eps_grad_fd re-rasterizing, per parameter, only the tiles and steps its
    primitives reach, fused with the reduction."""
    dev = torch.device("cuda", scene.device)
    pp, pdev, keep = _p_arg(scene, p)
    fe, fa = _plane_ptrs(scene, E), _plane_ptrs(scene, A)
    g, gp, gdev = _grad_out(scene, pdev, grad, dev)
    check(lib().eps_grad_fd_sparse(scene.ctx, scene.handle, pp, pdev, fe, fa, float(omega), float(h),
                                   _lib.FD_SCHEME[scheme], gp, gdev, _stream(stream)))
    return g


def util_copy(dst, src, stream=None):
    n = src.numel() * src.element_size()
    check(lib().sg_util_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), n, _stream(stream)))


def fieldgen(scene_or_shape, seed, stream=None):
    """E_fwd, E_adj complex64 CUDA tensors drawn by the library's Philox
    generator from `seed` (the fields a serving request with that seed uses)."""
    shape = scene_or_shape.shape if isinstance(scene_or_shape, Scene) else tuple(scene_or_shape)
    E = torch.empty(shape, dtype=torch.complex64, device="cuda")
    A = torch.empty(shape, dtype=torch.complex64, device="cuda")
    check(lib().sg_fieldgen(C.c_void_p(E.data_ptr()), C.c_void_p(A.data_ptr()), E.numel(), int(seed),
                            _stream(stream)))
    return E, A


class Server:
    """Continuous-batching gradient server (C++ scheduler thread in the
    library).  submit() queues a request and returns a ticket; poll() waits for
    its gradient."""

    def __init__(self, hbm_budget_bytes=0, max_slots=64, max_batch=16, n_streams=2, device=0,
                 fake_executor=False, fake_us=0, max_launch_us=0):
        o = _lib.sg_server_opts(int(hbm_budget_bytes), int(max_slots), int(max_batch), int(n_streams),
                                int(bool(fake_executor)), int(fake_us), int(max_launch_us))
        h = C.c_void_p()
        ctx = None if fake_executor else context(device)
        check(lib().sg_server_create(ctx, C.byref(o), C.byref(h)))
        self.handle = h
        self.n_params = {}
        self._scenes = []
        self._scene_of = {}
        self._keep = {}          # caller planes of requests not yet polled

    def open_session(self, scene):
        sid = C.c_uint32()
        check(lib().serve_open_session(self.handle, scene.handle, C.byref(sid)))
        self.n_params[sid.value] = scene.n_params
        self._scenes.append(scene)
        self._scene_of[sid.value] = scene
        return sid.value

    def open_fake_session(self, n_params, request_bytes):
        sid = C.c_uint32()
        check(lib().serve_open_fake_session(self.handle, int(n_params), int(request_bytes), C.byref(sid)))
        self.n_params[sid.value] = int(n_params)
        return sid.value

    def submit(self, session, p, seed, omega):
        a = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
        n = self.n_params.get(session)
        if n is not None and a.size != n:
            raise ValueError("p has the wrong size for this session")
        t = C.c_uint64()
        check(lib().serve_submit(self.handle, int(session), C.c_void_p(a.ctypes.data), int(seed), float(omega),
                                 C.byref(t)))
        return t.value

    def submit_fields(self, session, p, E, A, omega):
        """A request on the caller's complex64 planes E, A (C, Nz, Ny, Nx CUDA
        tensors); they must stay alive and unchanged until the ticket is
        polled."""
        a = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
        n = self.n_params.get(session)
        if n is not None and a.size != n:
            raise ValueError("p has the wrong size for this session")
        sc = self._scene_of[session]
        fe, fa = _plane_ptrs(sc, E), _plane_ptrs(sc, A)
        t = C.c_uint64()
        check(lib().serve_submit_fields(self.handle, int(session), C.c_void_p(a.ctypes.data), fe, fa, float(omega),
                                        C.byref(t)))
        self._keep[t.value] = (E, A)
        return t.value

    def poll(self, ticket, n_params, timeout_us=-1):
        """(status, grad or None, stats dict).  status 'ok' | 'pending' (raises
        on cancelled / failed)."""
        g = np.empty(max(1, n_params), dtype=np.float64)
        st = _lib.sg_req_stats()
        r = lib().serve_poll(self.handle, int(ticket), C.c_void_p(g.ctypes.data), int(timeout_us), C.byref(st))
        if r == _lib.SG_EAGAIN:
            return "pending", None, None
        self._keep.pop(int(ticket), None)        # the ticket is retired: its planes are free
        check(r)
        stats = {k: getattr(st, k) for k in ("submit_ns", "admit_ns", "launch_ns", "done_ns", "batch_size")}
        return "ok", g[:n_params], stats

    def cancel(self, ticket):
        check(lib().serve_cancel(self.handle, int(ticket)))

    def counters(self):
        v = [C.c_int64() for _ in range(5)]
        check(lib().serve_counters(self.handle, *[C.byref(x) for x in v]))
        return dict(zip(("completed", "batches", "max_batch", "bytes_in_use", "bytes_held"), [x.value for x in v]))

    def close(self):
        if getattr(self, "handle", None):
            check(lib().sg_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EpsBuild(torch.autograd.Function):
    """eps(p) as a differentiable op: forward = eps_build, backward = the
    fused reverse-mode kernel (eps_grad_vjp_geps) that recomputes
    d eps / d p in registers instead of forming the Jacobian (eq:AD)."""

    @staticmethod
    def forward(ctx, p, scene):
        pd = p.detach()
        if not pd.is_cuda:
            pd = pd.to(device=torch.device("cuda", scene.device))
        pd = pd.to(torch.float64).contiguous()
        ctx.scene = scene
        ctx.save_for_backward(pd)
        ctx.p_device = p.device
        return eps_build(scene, pd)

    @staticmethod
    def backward(ctx, grad_eps):
        (pd,) = ctx.saved_tensors
        g = eps_grad_vjp_geps(ctx.scene, pd, grad_eps.to(torch.float32).contiguous())
        return g.to(ctx.p_device), None
