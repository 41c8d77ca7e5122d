"""Thin-disk self-gravity on MI355X: Python binding of libgravity.so.

The binding only marshals arguments into the C ABI declared in
``include/gravity.h``; every step of a solve runs in the library's HIP
kernels.  Arrays are torch tensors on the GPU (torch provides device memory
and streams).  There is no CPU path: importing this package fails if the
built library is missing.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgravity.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libgravity.so is not built (run paper_2001_02765_amd/build.py or "
                      "__graft_entry__.build()); there is no fallback path")

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EBUSY = range(6)
F32, F64 = 0, 1
SLOPES_NONE, SLOPES_GIVEN = 0, 1
AMR_EXACT, AMR_NESTED = 0, 1
NOALLOC_SCRATCH_BYTES = 64 << 20  # GRAVITY_NOALLOC_SCRATCH_BYTES
_STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EUNSUPPORTED", 5: "EBUSY"}

# exported symbols of include/gravity.h
SYMBOLS = ("gravity_plan", "gravity_plan_workspace_bytes", "gravity_plan_get_info",
           "gravity_solve", "gravity_solve_noalloc", "gravity_solve_xyz", "gravity_batch_workspace_bytes", "gravity_solve_batch",
           "gravity_solve_batch_persistent", "gravity_batch_persistent_abandoned",
           "gravity_solve_batch_xyz", "gravity_solve_profiled", "gravity_stage_name",
           "gravity_server_create", "gravity_server_submit", "gravity_server_submit_xyz",
           "gravity_server_poll", "gravity_server_wait",
           "gravity_server_drain", "gravity_server_get_stats", "gravity_server_reset_stats",
           "gravity_server_destroy", "gravity_plan_destroy", "gravity_cache_bytes",
           "gravity_last_error")


class PatchT(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("i0", ctypes.c_int32), ("j0", ctypes.c_int32),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


class DescT(ctypes.Structure):
    _fields_ = [("n0x", ctypes.c_int32), ("n0y", ctypes.c_int32), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("h0", ctypes.c_double), ("nlevels", ctypes.c_int32),
                ("npatches", ctypes.c_int32), ("patches", ctypes.POINTER(PatchT)),
                ("prec", ctypes.c_int), ("slopes", ctypes.c_int), ("G", ctypes.c_double),
                ("z", ctypes.c_double), ("amr_method", ctypes.c_int32)]


class InfoT(ctypes.Structure):
    _fields_ = [("n_finest", ctypes.c_int32), ("fft_size", ctypes.c_int32),
                ("n_cells", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_size_t), ("resident_bytes", ctypes.c_size_t),
                ("variants", ctypes.c_int32 * 3), ("ncomp", ctypes.c_int32)]


_vp = ctypes.c_void_p
_lib.gravity_plan.argtypes = [ctypes.POINTER(DescT), ctypes.POINTER(_vp)]
_lib.gravity_plan.restype = ctypes.c_int
_lib.gravity_plan_workspace_bytes.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
_lib.gravity_plan_workspace_bytes.restype = ctypes.c_int
_lib.gravity_plan_get_info.argtypes = [_vp, ctypes.POINTER(InfoT)]
_lib.gravity_plan_get_info.restype = ctypes.c_int
_lib.gravity_solve.argtypes = [_vp] * 8
_lib.gravity_solve.restype = ctypes.c_int
_lib.gravity_solve_noalloc.argtypes = [_vp] * 7
_lib.gravity_solve_noalloc.restype = ctypes.c_int
_lib.gravity_solve_xyz.argtypes = [_vp] * 9
_lib.gravity_solve_xyz.restype = ctypes.c_int
_lib.gravity_batch_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.POINTER(_vp),
                                               ctypes.POINTER(ctypes.c_size_t)]
_lib.gravity_batch_workspace_bytes.restype = ctypes.c_int
_lib.gravity_solve_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(_vp)] + [ctypes.POINTER(_vp)] * 5 + [_vp, _vp]
_lib.gravity_solve_batch.restype = ctypes.c_int
_lib.gravity_solve_batch_persistent.argtypes = [ctypes.c_int32, ctypes.POINTER(_vp)] + [ctypes.POINTER(_vp)] * 5 + [_vp, _vp]
_lib.gravity_solve_batch_persistent.restype = ctypes.c_int
_lib.gravity_batch_persistent_abandoned.argtypes = [ctypes.c_int32, ctypes.POINTER(_vp), _vp, _vp,
                                                    ctypes.POINTER(ctypes.c_uint32)]
_lib.gravity_batch_persistent_abandoned.restype = ctypes.c_int
_lib.gravity_solve_batch_xyz.argtypes = [ctypes.c_int32, ctypes.POINTER(_vp)] + [ctypes.POINTER(_vp)] * 6 + [_vp, _vp]
_lib.gravity_solve_batch_xyz.restype = ctypes.c_int
_lib.gravity_solve_profiled.argtypes = [_vp] * 8 + [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                                    ctypes.POINTER(ctypes.c_int32)]
_lib.gravity_solve_profiled.restype = ctypes.c_int
_lib.gravity_stage_name.argtypes = [_vp, ctypes.c_int32]
_lib.gravity_stage_name.restype = ctypes.c_char_p
_lib.gravity_plan_destroy.argtypes = [_vp]
_lib.gravity_plan_destroy.restype = None
_lib.gravity_cache_bytes.argtypes = []
_lib.gravity_cache_bytes.restype = ctypes.c_size_t
_lib.gravity_last_error.argtypes = []
_lib.gravity_last_error.restype = ctypes.c_char_p


class ServerStatsT(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("in_flight", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double), ("budget_bytes", ctypes.c_size_t),
                ("bytes_in_use", ctypes.c_size_t), ("peak_bytes_in_use", ctypes.c_size_t),
                ("batches", ctypes.c_int64), ("leaves_completed", ctypes.c_int64)]


_lib.gravity_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_vp)]
_lib.gravity_server_create.restype = ctypes.c_int
_lib.gravity_server_submit.argtypes = [_vp] * 8 + [ctypes.POINTER(ctypes.c_int64)]
_lib.gravity_server_submit.restype = ctypes.c_int
_lib.gravity_server_submit_xyz.argtypes = [_vp] * 9 + [ctypes.POINTER(ctypes.c_int64)]
_lib.gravity_server_submit_xyz.restype = ctypes.c_int
_lib.gravity_server_poll.argtypes = [_vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]
_lib.gravity_server_poll.restype = ctypes.c_int
_lib.gravity_server_wait.argtypes = [_vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
_lib.gravity_server_wait.restype = ctypes.c_int
_lib.gravity_server_drain.argtypes = [_vp]
_lib.gravity_server_drain.restype = ctypes.c_int
_lib.gravity_server_get_stats.argtypes = [_vp, ctypes.POINTER(ServerStatsT)]
_lib.gravity_server_get_stats.restype = ctypes.c_int
_lib.gravity_server_reset_stats.argtypes = [_vp]
_lib.gravity_server_reset_stats.restype = ctypes.c_int
_lib.gravity_server_destroy.argtypes = [_vp]
_lib.gravity_server_destroy.restype = None


class GravityError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status


def _check(st):
    if st != OK:
        raise GravityError(st, _lib.gravity_last_error().decode(errors="replace"))


def cache_bytes():
    """Device bytes held by the resident kernel-spectrum cache."""
    return int(_lib.gravity_cache_bytes())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_cells(t, dtype, n, what, required=True):
    """The C ABI takes plain device pointers and cannot see sizes: every
    array handed to it is checked here (dtype, device, contiguity, length)."""
    if t is None:
        if required:
            raise ValueError("%s is required" % what)
        return
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s CUDA tensor" % (what, dtype))
    if t.numel() != n:
        raise ValueError("%s must hold %d composite-packed cells, not %d" % (what, n, t.numel()))


def _check_workspace(ws, nbytes):
    if ws is None or not ws.is_cuda or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous CUDA tensor")
    if ws.numel() * ws.element_size() < nbytes:
        raise ValueError("workspace holds %d bytes, the solve needs %d"
                         % (ws.numel() * ws.element_size(), nbytes))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A solve plan: geometry, refinement layout, precision and resident spectra.

    n0: base cells per side; nlevels: 1 for a uniform grid; patches: sequence
    of (level, i0, j0, nx, ny) with level >= 1 (base is level 0).  The domain
    is [x0, x0 + n0 h0] x [y0, y0 + n0 h0] (default [-1, 1]^2).  z: height of
    the target plane above the disk (0: midplane, solved with ``solve``;
    otherwise the three components at that height, with ``solve_xyz``).
    amr: "exact" (the leaf sum to rounding, finest lattice <= 4096^2) or
    "nested" (the nested-correction approximation, cost ~ refined area).
    """

    def __init__(self, n0, prec=F32, slopes=True, G=1.0, x0=-1.0, y0=-1.0, h0=None,
                 nlevels=1, patches=(), z=0.0, amr="exact"):
        if h0 is None:
            h0 = 2.0 / n0
        pl = list(patches)
        self._patch_arr = (PatchT * max(1, len(pl)))()
        for k, p in enumerate(pl):
            if hasattr(p, "level"):
                p = (p.level, p.i0, p.j0, p.nx, p.ny)
            self._patch_arr[k] = PatchT(*[int(v) for v in p])
        d = DescT(int(n0), int(n0), float(x0), float(y0), float(h0), int(nlevels), len(pl),
                  ctypes.cast(self._patch_arr, ctypes.POINTER(PatchT)), int(prec),
                  SLOPES_GIVEN if slopes else SLOPES_NONE, float(G), float(z),
                  {"exact": AMR_EXACT, "nested": AMR_NESTED}[amr])
        h = _vp()
        _check(_lib.gravity_plan(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.prec = int(prec)
        self.slopes = bool(slopes)
        info = InfoT()
        _check(_lib.gravity_plan_get_info(h, ctypes.byref(info)))
        self.n_finest = info.n_finest
        self.fft_size = info.fft_size
        self.n_cells = info.n_cells
        self.n_leaves = info.n_leaves
        self.workspace_bytes = info.workspace_bytes
        self.resident_bytes = info.resident_bytes
        self.variants = tuple(info.variants)
        self.ncomp = info.ncomp
        self.z = float(z)
        self.amr = amr if nlevels > 1 else "exact"

    @property
    def handle(self):
        return self._h

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.prec == F64 else torch.float32

    def close(self):
        if getattr(self, "_h", None):
            _lib.gravity_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_inputs(self, sigma, dsx, dsy):
        _check_cells(sigma, self.torch_dtype, self.n_cells, "sigma")
        _check_cells(dsx, self.torch_dtype, self.n_cells, "dsx", required=False)
        _check_cells(dsy, self.torch_dtype, self.n_cells, "dsy", required=False)

    def _check_outputs(self, outs, workspace):
        for name, o in zip(("fx", "fy", "fz"), outs):
            _check_cells(o, self.torch_dtype, self.n_cells, name)
        _check_workspace(workspace, self.workspace_bytes)

    def workspace(self):
        """A fresh device workspace tensor of the required size."""
        import torch
        return torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8, device="cuda")

    def solve(self, sigma, dsx=None, dsy=None, fx=None, fy=None, workspace=None, stream=None):
        """Queue a solve on ``stream`` (default: torch's current stream).

        Inputs are composite-packed device tensors of the plan's dtype; returns
        (fx, fy), allocated if not given."""
        import torch
        dt = self.torch_dtype
        self._check_inputs(sigma, dsx, dsy)
        if fx is None:
            fx = torch.empty(self.n_cells, dtype=dt, device=sigma.device)
        if fy is None:
            fy = torch.empty(self.n_cells, dtype=dt, device=sigma.device)
        if workspace is None:
            workspace = self.workspace()
        self._check_outputs((fx, fy), workspace)
        _check(_lib.gravity_solve(self._h, _ptr(sigma), _ptr(dsx), _ptr(dsy), _ptr(fx), _ptr(fy),
                                  _ptr(workspace), _stream_handle(stream)))
        return fx, fy

    def solve_noalloc(self, sigma, dsx=None, dsy=None, fx=None, fy=None, stream=None):
        """As ``solve``, through gravity_solve_noalloc: the library's static
        per-device scratch array serves as workspace (nothing is allocated;
        NOALLOC_SCRATCH_BYTES bounds the plan's workspace).  Allocation-free
        solves whose work overlaps on one device race on that array."""
        import torch
        dt = self.torch_dtype
        self._check_inputs(sigma, dsx, dsy)
        if fx is None:
            fx = torch.empty(self.n_cells, dtype=dt, device=sigma.device)
        if fy is None:
            fy = torch.empty(self.n_cells, dtype=dt, device=sigma.device)
        for name, o in (("fx", fx), ("fy", fy)):
            _check_cells(o, dt, self.n_cells, name)
        _check(_lib.gravity_solve_noalloc(self._h, _ptr(sigma), _ptr(dsx), _ptr(dsy), _ptr(fx),
                                          _ptr(fy), _stream_handle(stream)))
        return fx, fy

    def solve_xyz(self, sigma, dsx=None, dsy=None, fx=None, fy=None, fz=None, workspace=None,
                  stream=None):
        """Off-plane plans: queue a solve of (Fx, Fy, Fz) at height z above
        every leaf centre; returns (fx, fy, fz), allocated if not given."""
        import torch
        dt = self.torch_dtype
        self._check_inputs(sigma, dsx, dsy)
        out = [o if o is not None else torch.empty(self.n_cells, dtype=dt, device=sigma.device)
               for o in (fx, fy, fz)]
        if workspace is None:
            workspace = self.workspace()
        self._check_outputs(out, workspace)
        _check(_lib.gravity_solve_xyz(self._h, _ptr(sigma), _ptr(dsx), _ptr(dsy), _ptr(out[0]),
                                      _ptr(out[1]), _ptr(out[2]), _ptr(workspace),
                                      _stream_handle(stream)))
        return tuple(out)

    def profile(self, sigma, dsx, dsy, fx, fy, workspace, reps=20, stream=None):
        """Mean device milliseconds of one launch of each pipeline stage, each
        stage launched ``reps`` times back to back between HIP events on the
        solve stream: {stage name: ms}."""
        self._check_inputs(sigma, dsx, dsy)
        self._check_outputs((fx, fy), workspace)
        ms = (ctypes.c_double * 8)()
        ns = ctypes.c_int32()
        _check(_lib.gravity_solve_profiled(self._h, _ptr(sigma), _ptr(dsx), _ptr(dsy), _ptr(fx),
                                           _ptr(fy), _ptr(workspace), _stream_handle(stream),
                                           int(reps), ms, ctypes.byref(ns)))
        return {_lib.gravity_stage_name(self._h, k).decode(): ms[k] for k in range(ns.value)}


def batch_workspace_bytes(plans):
    n = len(plans)
    arr = (_vp * max(1, n))(*[p.handle for p in plans])
    b = ctypes.c_size_t()
    _check(_lib.gravity_batch_workspace_bytes(n, arr, ctypes.byref(b)))
    return int(b.value)


def solve_batch(plans, sigma, dsx, dsy, fx, fy, workspace, stream=None, fz=None, persistent=False):
    """Queue independent solves as one batch (see gravity_solve_batch); fz:
    third outputs, needed when the batch holds off-plane plans.
    persistent: gravity_solve_batch_persistent (one persistent launch per
    precision for the uniform solves of FFT sizes 128..2048)."""
    n = len(plans)

    def arr(ts):
        if ts is None:
            return None
        return (_vp * max(1, n))(*[None if t is None else t.data_ptr() for t in ts])

    for k, p in enumerate(plans):
        p._check_inputs(sigma[k], None if dsx is None else dsx[k], None if dsy is None else dsy[k])
        for name, o in (("fx", fx), ("fy", fy), ("fz", fz)):
            # a missing fz is the library's to reject (off-plane plan in a midplane call)
            if o is not None or name != "fz":
                _check_cells(None if o is None else o[k], p.torch_dtype, p.n_cells,
                             "%s[%d]" % (name, k), required=(name != "fz"))
    _check_workspace(workspace, batch_workspace_bytes(plans))
    ph = (_vp * max(1, n))(*[p.handle for p in plans])
    if persistent:
        if fz is not None:
            raise ValueError("the persistent batch takes midplane plans only")
        _check(_lib.gravity_solve_batch_persistent(n, ph, arr(sigma), arr(dsx), arr(dsy), arr(fx),
                                                   arr(fy), _ptr(workspace), _stream_handle(stream)))
    elif fz is None:
        _check(_lib.gravity_solve_batch(n, ph, arr(sigma), arr(dsx), arr(dsy), arr(fx), arr(fy),
                                        _ptr(workspace), _stream_handle(stream)))
    else:
        _check(_lib.gravity_solve_batch_xyz(n, ph, arr(sigma), arr(dsx), arr(dsy), arr(fx), arr(fy),
                                            arr(fz), _ptr(workspace), _stream_handle(stream)))


def batch_persistent_abandoned(plans, workspace, stream=None):
    """Work units the last persistent batch over these plans and this
    workspace abandoned at a wait's bound (0 unless the device or the
    library is at fault); waits for the stream."""
    n = len(plans)
    ph = (_vp * max(1, n))(*[p.handle for p in plans])
    out = ctypes.c_uint32(0)
    _check(_lib.gravity_batch_persistent_abandoned(n, ph, _ptr(workspace), _stream_handle(stream),
                                                   ctypes.byref(out)))
    return int(out.value)


class Server:
    """Continuous-batching request server (see gravity_server_create).

    budget_bytes: device arena for request workspaces (the HBM admission
    budget); nstreams: HIP streams the dispatcher spreads batches over."""

    def __init__(self, budget_bytes, nstreams=4, max_batch=8):
        h = _vp()
        _check(_lib.gravity_server_create(int(budget_bytes), int(nstreams), int(max_batch),
                                          ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, plan, sigma, dsx, dsy, fx, fy, fz=None, stream=None):
        """Queue a solve (fz: third output of an off-plane plan); tensors must
        stay alive until it completes (the server keeps references until
        wait()).  The server's work waits for what is already queued on
        ``stream`` (default: torch's current stream), which wrote the inputs.
        Returns a ticket."""
        plan._check_inputs(sigma, dsx, dsy)
        for name, o in (("fx", fx), ("fy", fy)):
            _check_cells(o, plan.torch_dtype, plan.n_cells, name)
        _check_cells(fz, plan.torch_dtype, plan.n_cells, "fz", required=False)
        tk = ctypes.c_int64()
        if fz is None:
            _check(_lib.gravity_server_submit(self._h, plan.handle, _ptr(sigma), _ptr(dsx), _ptr(dsy),
                                              _ptr(fx), _ptr(fy), _stream_handle(stream),
                                              ctypes.byref(tk)))
        else:
            _check(_lib.gravity_server_submit_xyz(self._h, plan.handle, _ptr(sigma), _ptr(dsx),
                                                  _ptr(dsy), _ptr(fx), _ptr(fy), _ptr(fz),
                                                  _stream_handle(stream), ctypes.byref(tk)))
        self._keep[tk.value] = (plan, sigma, dsx, dsy, fx, fy, fz)
        return tk.value

    def poll(self, ticket):
        d = ctypes.c_int32()
        _check(_lib.gravity_server_poll(self._h, int(ticket), ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket):
        """Block until the ticket completes; returns its latency in ms."""
        lat = ctypes.c_double()
        try:
            _check(_lib.gravity_server_wait(self._h, int(ticket), ctypes.byref(lat)))
        finally:
            self._keep.pop(int(ticket), None)
        return lat.value

    def drain(self):
        _check(_lib.gravity_server_drain(self._h))
        self._keep.clear()

    def stats(self):
        s = ServerStatsT()
        _check(_lib.gravity_server_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStatsT._fields_}

    def reset_stats(self):
        _check(_lib.gravity_server_reset_stats(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.gravity_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
