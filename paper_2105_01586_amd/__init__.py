"""Python binding of the MI355X FEM harmonic-inpainting library (``libfi.so``).

Thin ctypes layer over the C ABI in ``include/fi.h``: it checks tensor
shapes, dtypes and devices and passes raw pointers. Every step of the
computation runs in the library's HIP kernels; there is no fallback. Device
memory comes from PyTorch tensors on the GPU, and calls run on PyTorch's
current stream of that device unless another stream is given.

Names follow the paper (Chizhov and Weickert, arXiv 2105.01586): f is the
image, the mask K is a sorted array of linear pixel indices, g holds the
grey values stored at the mask pixels, u = B g is the inpainted image
(Sections 2 and 4).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

__all__ = [
    "FIError", "NoConvergence", "library", "Context", "Mesh", "SolveOpts", "TonalOpts",
    "PREC_FP32_IR", "PREC_FP64", "lib_path", "EXPORTED_SYMBOLS", "host_mesh", "grow_mask",
    "Server", "ServerOpts", "footprint_bound", "densify", "DENSIFY_TOPK", "DENSIFY_TRIANGLES",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libfi.so")

OK, E_INVALID, E_EMPTY_MASK, E_NO_CONVERGENCE, E_NOMEM, E_HIP = range(6)
PREC_FP32_IR, PREC_FP64 = 0, 1
DENSIFY_TOPK, DENSIFY_TRIANGLES = 0, 1

EXPORTED_SYMBOLS = (
    "fi_solve_opts_default", "fi_tonal_opts_default", "fi_last_error", "fi_version",
    "fi_ctx_create", "fi_ctx_set_stream", "fi_ctx_destroy", "fi_mesh_build", "fi_mesh_destroy",
    "fi_mesh_get_info", "fi_assemble", "fi_inpaint", "fi_vertex_values", "fi_error",
    "fi_adjoint", "fi_solve", "fi_error_dev", "fi_tonal_opt", "fi_mesh_export_geometry", "fi_mesh_export_csr",
    "fi_mesh_export_ss_plan",
    "fi_owner_map", "fi_topk_new_pixels", "fi_time_cg_kernel", "fi_cg_kernel_bytes",
    "fi_host_mesh_build", "fi_host_mesh_info", "fi_host_mesh_export", "fi_host_mesh_destroy",
    "fi_mesh_upload", "fi_grow_mask", "fi_server_opts_default", "fi_server_create",
    "fi_server_submit", "fi_server_poll", "fi_server_stats_get", "fi_server_clock",
    "fi_server_destroy", "fi_server_footprint", "fi_paper_densify_step", "fi_densify",
    "fi_inpaint_rgb", "fi_error_rgb", "fi_tonal_opt_rgb", "fi_time_cg_multi_kernel",
    "fi_cg_multi_kernel_bytes", "fi_mesh_build_delaunay", "fi_host_mesh_build_delaunay",
    "fi_densify_delaunay", "fi_l1_opts_default", "fi_tonal_opt_l1", "fi_inpaint_image",
    "fi_mse_dev", "fi_mse_backward", "fi_topk_new_pixels_noalloc",
)


class FIError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[fi status {code}] {msg}")
        self.code = code


class NoConvergence(FIError):
    pass


class _SolveOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("rtol", ctypes.c_double),
                ("inner_rtol", ctypes.c_double), ("max_inner", ctypes.c_int),
                ("max_refine", ctypes.c_int), ("check_every", ctypes.c_int),
                ("atol", ctypes.c_double)]


class _SolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("refinements", ctypes.c_int32),
                ("status", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("residual", ctypes.c_double), ("rhs_norm", ctypes.c_double),
                ("launches", ctypes.c_int64)]


class _TonalOpts(ctypes.Structure):
    _fields_ = [("inner", _SolveOpts), ("rtol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("start_from_g", ctypes.c_int), ("cold_adjoint", ctypes.c_int)]


class _TonalStats(ctypes.Structure):
    _fields_ = [("outer_iterations", ctypes.c_int32), ("status", ctypes.c_int32),
                ("inner_iterations", ctypes.c_int64), ("rel_normal_residual", ctypes.c_double),
                ("mse_initial", ctypes.c_double), ("mse_final", ctypes.c_double)]


class _L1Opts(ctypes.Structure):
    _fields_ = [("inner", _SolveOpts), ("eps", ctypes.c_double), ("irls_iters", ctypes.c_int),
                ("cgls_iters", ctypes.c_int), ("start_from_g", ctypes.c_int)]


class _L1Stats(ctypes.Structure):
    _fields_ = [("irls_iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("inner_iterations", ctypes.c_int64), ("mae_initial", ctypes.c_double),
                ("mae_final", ctypes.c_double), ("mse_final", ctypes.c_double)]


class _MeshInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("N", "P", "V", "T", "L", "n", "m", "nnz_ff", "nnz_fd", "device_bytes",
                 "cg_blocks", "cg_block_size", "large_mode", "cg_iters_per_launch",
                 "cg_max_region", "cg_region_rows", "cg_lmat_rows")]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int), ("precision", ctypes.c_int),
                ("hbm_budget", ctypes.c_size_t), ("build_threads", ctypes.c_int),
                ("chunk", ctypes.c_int)]


class _JobDesc(ctypes.Structure):
    _fields_ = [("side", ctypes.c_int), ("f", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("m", ctypes.c_int64), ("tonal_iters", ctypes.c_int), ("g_out", ctypes.c_void_p),
                ("inner", _SolveOpts)]


class _JobResult(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32),
                ("mse_inpaint", ctypes.c_double), ("mse_tonal", ctypes.c_double),
                ("inner_iterations", ctypes.c_int64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("footprint_bound", ctypes.c_int64), ("error", ctypes.c_char * 128)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("jobs_submitted", "jobs_done", "jobs_failed", "peak_resident", "step_rounds",
                 "slot_steps", "arena_bytes", "arena_used_bytes", "arena_peak_bytes")] + \
               [("clock", ctypes.c_double)]


_lib = None
_live_servers: "weakref.WeakSet" = weakref.WeakSet()
_live_meshes: "weakref.WeakSet" = weakref.WeakSet()
_live_contexts: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_all() -> None:
    # Meshes first (they borrow their context), before the HIP runtime's own
    # exit handlers run.
    for obj in list(_live_servers) + list(_live_meshes) + list(_live_contexts):
        try:
            obj.close()
        except Exception:
            pass


def library() -> ctypes.CDLL:
    """Loads libfi.so (raises if it was not built: there is no other path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(lib_path):
        raise ImportError(f"{lib_path} is missing; build it with __graft_entry__.build() "
                          "or python paper_2105_01586_amd/build.py")
    L = ctypes.CDLL(lib_path)
    vp, i32p, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), \
        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
    sig = {
        "fi_solve_opts_default": (None, [ctypes.POINTER(_SolveOpts)]),
        "fi_tonal_opts_default": (None, [ctypes.POINTER(_TonalOpts)]),
        "fi_last_error": (ctypes.c_char_p, []),
        "fi_version": (ctypes.c_char_p, []),
        "fi_ctx_create": (ctypes.c_int, [ctypes.c_int, vp, ctypes.POINTER(vp)]),
        "fi_ctx_set_stream": (ctypes.c_int, [vp, vp]),
        "fi_ctx_destroy": (ctypes.c_int, [vp]),
        "fi_mesh_build": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64,
                                         ctypes.POINTER(vp)]),
        "fi_mesh_destroy": (ctypes.c_int, [vp]),
        "fi_mesh_get_info": (ctypes.c_int, [vp, ctypes.POINTER(_MeshInfo)]),
        "fi_assemble": (ctypes.c_int, [vp]),
        "fi_inpaint": (ctypes.c_int, [vp, vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                      ctypes.POINTER(_SolveStats)]),
        "fi_vertex_values": (ctypes.c_int, [vp, vp]),
        "fi_error": (ctypes.c_int, [vp, vp, vp, dp, vp, vp]),
        "fi_error_dev": (ctypes.c_int, [vp, vp, vp, vp]),
        "fi_mse_dev": (ctypes.c_int, [vp, vp, vp, vp]),
        "fi_mse_backward": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                           ctypes.POINTER(_SolveStats)]),
        "fi_solve": (ctypes.c_int, [vp, vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                    ctypes.POINTER(_SolveStats)]),
        "fi_adjoint": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                      ctypes.POINTER(_SolveStats)]),
        "fi_tonal_opt": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(_TonalOpts),
                                        ctypes.POINTER(_TonalStats)]),
        "fi_mesh_export_geometry": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
        "fi_mesh_export_csr": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "fi_mesh_export_ss_plan": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "fi_owner_map": (ctypes.c_int, [vp, vp]),
        "fi_topk_new_pixels": (ctypes.c_int, [vp, vp, ctypes.c_int64, vp]),
        "fi_topk_new_pixels_noalloc": (ctypes.c_int, [vp, vp, ctypes.c_int64, vp]),
        "fi_time_cg_kernel": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, dp]),
        "fi_cg_kernel_bytes": (ctypes.c_int, [vp, ctypes.c_int, i64p]),
        "fi_host_mesh_build": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, vp, ctypes.c_int64,
                                              ctypes.POINTER(vp)]),
        "fi_host_mesh_info": (ctypes.c_int, [vp, ctypes.POINTER(_MeshInfo)]),
        "fi_host_mesh_export": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
        "fi_host_mesh_destroy": (ctypes.c_int, [vp]),
        "fi_mesh_upload": (ctypes.c_int, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "fi_grow_mask": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int, ctypes.POINTER(_SolveOpts), vp, vp, vp]),
        "fi_paper_densify_step": (ctypes.c_int, [vp, vp, ctypes.c_int64, vp, i64p]),
        "fi_densify": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int, ctypes.c_int, ctypes.POINTER(_SolveOpts), vp,
                                      vp, vp, i64p]),
        "fi_inpaint_rgb": (ctypes.c_int, [vp, vp, vp, vp, ctypes.POINTER(_SolveOpts),
                                          ctypes.POINTER(_SolveStats)]),
        "fi_error_rgb": (ctypes.c_int, [vp, vp, vp, dp, dp]),
        "fi_tonal_opt_rgb": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(_TonalOpts),
                                            ctypes.POINTER(_TonalStats)]),
        "fi_time_cg_multi_kernel": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                   dp]),
        "fi_cg_multi_kernel_bytes": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, i64p]),
        "fi_mesh_build_delaunay": (ctypes.c_int, [vp, ctypes.c_int, vp, ctypes.c_int64, vp,
                                                  ctypes.c_int64, ctypes.POINTER(vp)]),
        "fi_host_mesh_build_delaunay": (ctypes.c_int, [ctypes.c_int, vp, ctypes.c_int64, vp,
                                                       ctypes.c_int64, ctypes.POINTER(vp)]),
        "fi_densify_delaunay": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, ctypes.c_int64, vp,
                                               ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                               ctypes.POINTER(_SolveOpts), vp, vp, vp, i64p]),
        "fi_inpaint_image": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp,
                                            ctypes.POINTER(_SolveOpts),
                                            ctypes.POINTER(_SolveStats)]),
        "fi_l1_opts_default": (None, [ctypes.POINTER(_L1Opts)]),
        "fi_tonal_opt_l1": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(_L1Opts),
                                           ctypes.POINTER(_L1Stats), vp]),
        "fi_server_opts_default": (None, [ctypes.POINTER(_ServerOpts)]),
        "fi_server_create": (ctypes.c_int, [vp, ctypes.POINTER(_ServerOpts), ctypes.POINTER(vp)]),
        "fi_server_submit": (ctypes.c_int, [vp, ctypes.POINTER(_JobDesc),
                                            ctypes.POINTER(ctypes.c_uint64)]),
        "fi_server_poll": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.c_int,
                                          ctypes.POINTER(_JobResult)]),
        "fi_server_stats_get": (ctypes.c_int, [vp, ctypes.POINTER(_ServerStats)]),
        "fi_server_clock": (ctypes.c_double, [vp]),
        "fi_server_destroy": (ctypes.c_int, [vp]),
        "fi_server_footprint": (ctypes.c_int, [ctypes.c_int, vp, ctypes.c_int64, ctypes.c_int,
                                               i64p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    del i32p
    _lib = L
    return L


def _check(rc: int, what: str) -> None:
    if rc == OK:
        return
    msg = library().fi_last_error().decode(errors="replace")
    cls = NoConvergence if rc == E_NO_CONVERGENCE else FIError
    raise cls(rc, f"{what}: {msg}")


@dataclass
class SolveOpts:
    """Options of one harmonic-extension solve (defaults as in the C library)."""
    precision: int = PREC_FP32_IR
    rtol: float = 1e-10
    inner_rtol: float = 1e-5
    max_inner: int = 20000
    max_refine: int = 40
    check_every: int = 32
    atol: float = 0.0  # 0: the library's default absolute bound; < 0: none

    def c(self) -> _SolveOpts:
        return _SolveOpts(self.precision, self.rtol, self.inner_rtol, self.max_inner,
                          self.max_refine, self.check_every, self.atol)


@dataclass
class TonalOpts:
    inner: SolveOpts = None
    rtol: float = 1e-8
    max_outer: int = 500
    start_from_g: bool = False
    cold_adjoint: bool = False

    def c(self) -> _TonalOpts:
        inner = (self.inner or SolveOpts()).c()
        return _TonalOpts(inner, self.rtol, self.max_outer, int(self.start_from_g),
                          int(self.cold_adjoint))


def _stats(s) -> dict:
    return {k: getattr(s, k) for k, _ in s._fields_}


def _torch():
    import torch
    return torch


def host_mesh(side: int, mask_idx, unknowns=None) -> dict:
    """Builds the mesh on the host only (no GPU) and exports it: the quadtree
    mesh, or with ``unknowns`` (pixel indices) the paper's Delaunay mesh.

    Returns numpy arrays: vxy (V, 2), tri (T, 3), leaves (L, 3), free_vids,
    mask_vids, plus the counts.
    """
    L = library()
    mask = np.ascontiguousarray(np.asarray(mask_idx, dtype=np.int32).ravel())
    h = ctypes.c_void_p()
    if unknowns is None:
        _check(L.fi_host_mesh_build(int(side), int(side), mask.ctypes.data_as(ctypes.c_void_p),
                                    mask.size, ctypes.byref(h)), "fi_host_mesh_build")
    else:
        unk = np.ascontiguousarray(np.asarray(unknowns, dtype=np.int32).ravel())
        _check(L.fi_host_mesh_build_delaunay(int(side), mask.ctypes.data_as(ctypes.c_void_p),
                                             mask.size, unk.ctypes.data_as(ctypes.c_void_p),
                                             unk.size, ctypes.byref(h)),
               "fi_host_mesh_build_delaunay")
    try:
        info = _MeshInfo()
        _check(L.fi_host_mesh_info(h, ctypes.byref(info)), "fi_host_mesh_info")
        d = _stats(info)
        out = {"vxy": np.empty((d["V"], 2), np.int32), "tri": np.empty((d["T"], 3), np.int32),
               "leaves": np.empty((d["L"], 3), np.int32), "free_vids": np.empty(d["n"], np.int32),
               "mask_vids": np.empty(d["m"], np.int32)}
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(L.fi_host_mesh_export(h, c(out["vxy"]), c(out["tri"]), c(out["leaves"]),
                                     c(out["free_vids"]), c(out["mask_vids"])),
               "fi_host_mesh_export")
        out.update({k: int(v) for k, v in d.items()})
        return out
    finally:
        L.fi_host_mesh_destroy(h)


class Context:
    """Device and HIP stream binding. ``stream`` defaults to torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(library().fi_ctx_create(self.device, ctypes.c_void_p(stream.cuda_stream),
                                       ctypes.byref(h)), "fi_ctx_create")
        self._h = h
        self._meshes = weakref.WeakSet()
        _live_contexts.add(self)

    def set_stream(self, stream) -> None:
        self.stream = stream
        _check(library().fi_ctx_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)),
               "fi_ctx_set_stream")

    def close(self) -> None:
        """Destroys the context after every mesh built on it."""
        for m in list(getattr(self, "_meshes", ())):
            m.close()
        if getattr(self, "_h", None):
            library().fi_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(t, dtype, numel, name, device):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name} must live on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Mesh:
    """Quadtree FEM mesh for one (image side, mask) pair, with its device matrices."""

    def __init__(self, ctx: Context, side: int, mask_idx, unknowns=None):
        """``unknowns``: None for the quadtree mesh; else the unknown vertices
        (pixel indices) of the paper's Delaunay mesh."""
        self.ctx = ctx
        mask = np.ascontiguousarray(np.asarray(mask_idx, dtype=np.int32).ravel())
        self._mask = mask
        h = ctypes.c_void_p()
        if unknowns is None:
            _check(library().fi_mesh_build(ctx._h, int(side), int(side),
                                           mask.ctypes.data_as(ctypes.c_void_p), mask.size,
                                           ctypes.byref(h)), "fi_mesh_build")
        else:
            unk = np.ascontiguousarray(np.asarray(unknowns, dtype=np.int32).ravel())
            _check(library().fi_mesh_build_delaunay(ctx._h, int(side),
                                                    mask.ctypes.data_as(ctypes.c_void_p),
                                                    mask.size, unk.ctypes.data_as(ctypes.c_void_p),
                                                    unk.size, ctypes.byref(h)),
                   "fi_mesh_build_delaunay")
        self._h = h
        ctx._meshes.add(self)
        _live_meshes.add(self)
        info = _MeshInfo()
        _check(library().fi_mesh_get_info(h, ctypes.byref(info)), "fi_mesh_get_info")
        self.info = _stats(info)
        for k in ("N", "P", "V", "T", "L", "n", "m"):
            setattr(self, k, int(self.info[k]))

    @property
    def mask(self) -> np.ndarray:
        return self._mask

    def large_mode(self) -> bool:
        """True when a separate launch sums each CG step's partial sums."""
        return bool(self.info["large_mode"])

    def close(self) -> None:
        if getattr(self, "_h", None):
            library().fi_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self):
        return self.ctx.device

    def _empty(self, n, dtype):
        torch = _torch()
        return torch.empty(n, dtype=dtype, device=f"cuda:{self._dev()}")

    # -- the hot path ------------------------------------------------------
    def assemble(self) -> None:
        _check(library().fi_assemble(self._h), "fi_assemble")

    def inpaint(self, f=None, g=None, u=None, opts: SolveOpts | None = None):
        """u = B g (g defaults to f on the mask). Returns (u, stats)."""
        torch = _torch()
        d = self._dev()
        if u is None:
            u = self._empty(self.P, torch.float64)
        st = _SolveStats()
        o = (opts or SolveOpts()).c()
        rc = library().fi_inpaint(self._h, _ptr(f, torch.uint8, self.P, "f", d),
                                  _ptr(g, torch.float64, self.m, "g", d),
                                  _ptr(u, torch.float64, self.P, "u", d), ctypes.byref(o),
                                  ctypes.byref(st))
        _check(rc, "fi_inpaint")
        return u, _stats(st)

    def vertex_values(self):
        torch = _torch()
        out = self._empty(self.V, torch.float64)
        _check(library().fi_vertex_values(self._h, ctypes.c_void_p(out.data_ptr())),
               "fi_vertex_values")
        return out

    def error(self, u, f, pixel: bool = False, triangle: bool = False):
        """Returns (mse, e or None, E_T or None)."""
        torch = _torch()
        d = self._dev()
        e = self._empty(self.P, torch.float64) if pixel else None
        E = self._empty(self.T, torch.float64) if triangle else None
        mse = ctypes.c_double()
        rc = library().fi_error(self._h, _ptr(u, torch.float64, self.P, "u", d),
                                _ptr(f, torch.uint8, self.P, "f", d), ctypes.byref(mse),
                                _ptr(e, torch.float64, self.P, "e", d),
                                _ptr(E, torch.float64, self.T, "E", d))
        _check(rc, "fi_error")
        return mse.value, e, E

    def adjoint(self, r, s=None, opts: SolveOpts | None = None):
        """s = B^T r. Returns (s, stats)."""
        torch = _torch()
        d = self._dev()
        if s is None:
            s = self._empty(self.m, torch.float64)
        st = _SolveStats()
        o = (opts or SolveOpts()).c()
        rc = library().fi_adjoint(self._h, _ptr(r, torch.float64, self.P, "r", d),
                                  _ptr(s, torch.float64, self.m, "s", d), ctypes.byref(o),
                                  ctypes.byref(st))
        _check(rc, "fi_adjoint")
        return s, _stats(st)

    def solve(self, b, x0=None, x=None, opts: SolveOpts | None = None):
        """x = K_FF^{-1} b (free unknowns in free-vertex order), started from
        x0 (None: 0). Returns (x, stats)."""
        torch = _torch()
        d = self._dev()
        if x is None:
            x = self._empty(self.n, torch.float64)
        st = _SolveStats()
        o = (opts or SolveOpts()).c()
        x0p = None if x0 is None else _ptr(x0, torch.float64, self.n, "x0", d)
        rc = library().fi_solve(self._h, _ptr(b, torch.float64, self.n, "b", d), x0p,
                                _ptr(x, torch.float64, self.n, "x", d), ctypes.byref(o),
                                ctypes.byref(st))
        _check(rc, "fi_solve")
        return x, _stats(st)

    def tonal_opt(self, f, g=None, opts: TonalOpts | None = None):
        """g* = argmin ||B g - f||^2 by CGLS. Returns (g, stats)."""
        torch = _torch()
        d = self._dev()
        o = opts or TonalOpts()
        if g is None:
            g = self._empty(self.m, torch.float64)
            o = TonalOpts(o.inner, o.rtol, o.max_outer, False, o.cold_adjoint)
        co = o.c()
        st = _TonalStats()
        rc = library().fi_tonal_opt(self._h, _ptr(f, torch.uint8, self.P, "f", d),
                                    _ptr(g, torch.float64, self.m, "g", d), ctypes.byref(co),
                                    ctypes.byref(st))
        _check(rc, "fi_tonal_opt")
        return g, _stats(st)

    def tonal_opt_l1(self, f, g=None, eps: float = 0.5, irls_iters: int = 8,
                     cgls_iters: int = 20, inner: SolveOpts | None = None):
        """L1 tonal optimisation by IRLS (fi_tonal_opt_l1). Returns (g, stats,
        MAE at the start and after each step)."""
        torch = _torch()
        d = self._dev()
        start = g is not None
        if g is None:
            g = self._empty(self.m, torch.float64)
        o = _L1Opts((inner or SolveOpts()).c(), float(eps), int(irls_iters), int(cgls_iters),
                    int(start))
        st = _L1Stats()
        hist = np.empty(int(irls_iters) + 1, np.float64)
        rc = library().fi_tonal_opt_l1(self._h, _ptr(f, torch.uint8, self.P, "f", d),
                                       _ptr(g, torch.float64, self.m, "g", d), ctypes.byref(o),
                                       ctypes.byref(st), hist.ctypes.data_as(ctypes.c_void_p))
        _check(rc, "fi_tonal_opt_l1")
        return g, _stats(st), hist

    # -- colour (planar: channel c at [c * P, (c + 1) * P)) ------------------
    def inpaint_rgb(self, f=None, g=None, u=None, opts: SolveOpts | None = None):
        """u_c = B g_c for the three channels (g defaults to f on the mask).
        f: uint8[3P], g: float64[3m], u: float64[3P]. Returns (u, [stats] * 3)."""
        torch = _torch()
        d = self._dev()
        if u is None:
            u = self._empty(3 * self.P, torch.float64)
        st = (_SolveStats * 3)()
        o = (opts or SolveOpts()).c()
        rc = library().fi_inpaint_rgb(self._h, _ptr(f, torch.uint8, 3 * self.P, "f", d),
                                      _ptr(g, torch.float64, 3 * self.m, "g", d),
                                      _ptr(u, torch.float64, 3 * self.P, "u", d), ctypes.byref(o),
                                      st)
        _check(rc, "fi_inpaint_rgb")
        return u, [_stats(x) for x in st]

    def error_dev(self, u, f, sse=None):
        """Sum of squared errors of u against f into a one-element float64
        device tensor, without waiting for it (MSE = sum / P). Returns it."""
        torch = _torch()
        d = self._dev()
        if sse is None:
            sse = self._empty(1, torch.float64)
        rc = library().fi_error_dev(self._h, _ptr(u, torch.float64, self.P, "u", d),
                                    _ptr(f, torch.uint8, self.P, "f", d),
                                    _ptr(sse, torch.float64, 1, "sse", d))
        _check(rc, "fi_error_dev")
        return sse

    def mse_dev(self, u, f, mse=None):
        """MSE of u against f into a one-element float64 device tensor,
        without waiting for it. Returns it."""
        torch = _torch()
        d = self._dev()
        if mse is None:
            mse = self._empty(1, torch.float64)
        rc = library().fi_mse_dev(self._h, _ptr(u, torch.float64, self.P, "u", d),
                                  _ptr(f, torch.uint8, self.P, "f", d),
                                  _ptr(mse, torch.float64, 1, "mse", d))
        _check(rc, "fi_mse_dev")
        return mse

    def mse_backward(self, u, f, scale=None, grad=None, opts: SolveOpts | None = None):
        """grad = s (2 / P) B^T (u - f) with s the one-element device tensor
        `scale` (None: 1) and u = B g. Returns (grad, stats)."""
        torch = _torch()
        d = self._dev()
        if grad is None:
            grad = self._empty(self.m, torch.float64)
        st = _SolveStats()
        o = (opts or SolveOpts()).c()
        sp = None if scale is None else _ptr(scale, torch.float64, 1, "scale", d)
        rc = library().fi_mse_backward(self._h, _ptr(u, torch.float64, self.P, "u", d),
                                       _ptr(f, torch.uint8, self.P, "f", d), sp,
                                       _ptr(grad, torch.float64, self.m, "grad", d),
                                       ctypes.byref(o), ctypes.byref(st))
        _check(rc, "fi_mse_backward")
        return grad, _stats(st)

    def error_rgb(self, u, f):
        """Returns (colour MSE over all 3P values, [MSE of each channel])."""
        torch = _torch()
        d = self._dev()
        mse = ctypes.c_double()
        ch = (ctypes.c_double * 3)()
        rc = library().fi_error_rgb(self._h, _ptr(u, torch.float64, 3 * self.P, "u", d),
                                    _ptr(f, torch.uint8, 3 * self.P, "f", d), ctypes.byref(mse),
                                    ch)
        _check(rc, "fi_error_rgb")
        return mse.value, list(ch)

    def tonal_opt_rgb(self, f, g=None, opts: TonalOpts | None = None):
        """Per-channel CGLS with shared solve launches. Returns (g[3m], [stats] * 3)."""
        torch = _torch()
        d = self._dev()
        o = opts or TonalOpts()
        if g is None:
            g = self._empty(3 * self.m, torch.float64)
            o = TonalOpts(o.inner, o.rtol, o.max_outer, False, o.cold_adjoint)
        co = o.c()
        st = (_TonalStats * 3)()
        rc = library().fi_tonal_opt_rgb(self._h, _ptr(f, torch.uint8, 3 * self.P, "f", d),
                                        _ptr(g, torch.float64, 3 * self.m, "g", d),
                                        ctypes.byref(co), st)
        _check(rc, "fi_tonal_opt_rgb")
        return g, [_stats(x) for x in st]

    def device_bytes(self) -> int:
        """Device memory the mesh holds now (channel state included once created)."""
        info = _MeshInfo()
        _check(library().fi_mesh_get_info(self._h, ctypes.byref(info)), "fi_mesh_get_info")
        return int(info.device_bytes)

    # -- exports for checking --------------------------------------------
    def export_geometry(self) -> dict:
        vxy = np.empty((self.V, 2), np.int32)
        tri = np.empty((self.T, 3), np.int32)
        leaves = np.empty((self.L, 3), np.int32)
        fv = np.empty(self.n, np.int32)
        mv = np.empty(self.m, np.int32)
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(library().fi_mesh_export_geometry(self._h, c(vxy), c(tri), c(leaves), c(fv), c(mv)),
               "fi_mesh_export_geometry")
        return {"vxy": vxy, "tri": tri, "leaves": leaves, "free_vids": fv, "mask_vids": mv}

    def export_csr(self) -> dict:
        n = self.n
        nff, nfd = int(self.info["nnz_ff"]), int(self.info["nnz_fd"])
        a = {"ff_rowptr": np.empty(n + 1, np.int32), "ff_col": np.empty(nff, np.int32),
             "ff_val": np.empty(nff, np.float64), "fd_rowptr": np.empty(n + 1, np.int32),
             "fd_col": np.empty(nfd, np.int32), "fd_val": np.empty(nfd, np.float64)}
        c = lambda x: x.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(library().fi_mesh_export_csr(self._h, c(a["ff_rowptr"]), c(a["ff_col"]),
                                            c(a["ff_val"]), c(a["fd_rowptr"]), c(a["fd_col"]),
                                            c(a["fd_val"])), "fi_mesh_export_csr")
        return a

    def export_ss_plan(self) -> dict:
        """The S-iteration launch's plan (fi_mesh_export_ss_plan) as numpy arrays."""
        i = self.info
        a = {"perm": np.empty(self.n, np.int32),
             "blocks": np.empty((int(i["cg_blocks"]), 8), np.int32),
             "region": np.empty(int(i["cg_region_rows"]), np.int32),
             "lmat": np.empty((int(i["cg_lmat_rows"]), 6), np.uint16)}
        c = lambda x: x.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(library().fi_mesh_export_ss_plan(self._h, c(a["perm"]), c(a["blocks"]),
                                                c(a["region"]), c(a["lmat"])),
               "fi_mesh_export_ss_plan")
        return a

    def owner_map(self):
        torch = _torch()
        out = self._empty(self.P, torch.int32)
        _check(library().fi_owner_map(self._h, ctypes.c_void_p(out.data_ptr())), "fi_owner_map")
        return out

    def topk_new_pixels(self, e, k: int):
        torch = _torch()
        out = self._empty(max(int(k), 1), torch.int32)
        rc = library().fi_topk_new_pixels(self._h, _ptr(e, torch.float64, self.P, "e", self._dev()),
                                          int(k), ctypes.c_void_p(out.data_ptr()))
        _check(rc, "fi_topk_new_pixels")
        return out[:int(k)]

    def topk_new_pixels_noalloc(self, e, out):
        """fi_topk_new_pixels into the caller's int32 tensor ``out`` (its
        length is k), with the library's fixed workspace: no allocation."""
        torch = _torch()
        d = self._dev()
        k = int(out.numel())
        rc = library().fi_topk_new_pixels_noalloc(
            self._h, _ptr(e, torch.float64, self.P, "e", d), k,
            _ptr(out, torch.int32, k, "out", d) if k > 0 else None)
        _check(rc, "fi_topk_new_pixels_noalloc")
        return out

    def paper_densify_step(self, e, k: int):
        """Section 3's per-triangle step: up to k new pixels (ascending)."""
        torch = _torch()
        out = self._empty(max(int(k), 1), torch.int32)
        added = ctypes.c_int64()
        rc = library().fi_paper_densify_step(self._h, _ptr(e, torch.float64, self.P, "e",
                                                           self._dev()),
                                             int(k), ctypes.c_void_p(out.data_ptr()),
                                             ctypes.byref(added))
        _check(rc, "fi_paper_densify_step")
        return out[:added.value]

    # -- measurement ---------------------------------------------------------
    def time_cg_kernel(self, precision: int = PREC_FP32_IR, reps: int = 200) -> float:
        ms = ctypes.c_double()
        _check(library().fi_time_cg_kernel(self._h, int(precision), int(reps), ctypes.byref(ms)),
               "fi_time_cg_kernel")
        return ms.value

    def cg_kernel_bytes(self, precision: int = PREC_FP32_IR) -> int:
        b = ctypes.c_int64()
        _check(library().fi_cg_kernel_bytes(self._h, int(precision), ctypes.byref(b)),
               "fi_cg_kernel_bytes")
        return b.value

    def time_cg_multi_kernel(self, nrhs: int = 3, precision: int = PREC_FP32_IR,
                             reps: int = 200) -> float:
        ms = ctypes.c_double()
        _check(library().fi_time_cg_multi_kernel(self._h, int(nrhs), int(precision), int(reps),
                                                 ctypes.byref(ms)), "fi_time_cg_multi_kernel")
        return ms.value

    def cg_multi_kernel_bytes(self, nrhs: int = 3, precision: int = PREC_FP32_IR) -> int:
        b = ctypes.c_int64()
        _check(library().fi_cg_multi_kernel_bytes(self._h, int(nrhs), int(precision),
                                                  ctypes.byref(b)), "fi_cg_multi_kernel_bytes")
        return b.value


def inpaint_image(ctx: Context, f, mask_u8, g=None, opts: SolveOpts | None = None):
    """One-shot inpainting (fi_inpaint_image): f uint8 device tensor of
    side * side pixels, mask_u8 a host array of the same size (nonzero =
    mask pixel), g optional device values at the mask pixels in ascending
    order. Returns (u, stats)."""
    torch = _torch()
    mask_u8 = np.ascontiguousarray(np.asarray(mask_u8, dtype=np.uint8).ravel())
    side = int(round(mask_u8.size ** 0.5))
    if side * side != mask_u8.size:
        raise ValueError("square images only")
    d = ctx.device
    m = int(np.count_nonzero(mask_u8))
    u = torch.empty(side * side, dtype=torch.float64, device=f"cuda:{d}")
    st = _SolveStats()
    o = (opts or SolveOpts()).c()
    rc = library().fi_inpaint_image(ctx._h, side, side, _ptr(f, torch.uint8, side * side, "f", d),
                                    mask_u8.ctypes.data_as(ctypes.c_void_p),
                                    _ptr(g, torch.float64, m, "g", d),
                                    ctypes.c_void_p(u.data_ptr()), ctypes.byref(o),
                                    ctypes.byref(st))
    _check(rc, "fi_inpaint_image")
    return u, _stats(st)


def grow_mask(ctx: Context, side: int, f, mask0, k_add: int, rounds: int,
              opts: SolveOpts | None = None):
    """Error-driven mask growth (fi_grow_mask).

    Returns (mask_order, mse, gpu_ms): the int32 pixel indices in order of
    addition (mask0 first, then each round's additions), the MSE after each
    of the rounds + 1 inpaintings, and the device milliseconds of each
    round's solve, interpolation and error.
    """
    torch = _torch()
    mask0 = np.ascontiguousarray(np.asarray(mask0, dtype=np.int32).ravel())
    P = int(side) * int(side)
    out = np.empty(mask0.size + int(rounds) * int(k_add), np.int32)
    mse = np.empty(int(rounds) + 1, np.float64)
    ms = np.empty(int(rounds) + 1, np.float64)
    o = (opts or SolveOpts()).c()
    c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    rc = library().fi_grow_mask(ctx._h, int(side), _ptr(f, torch.uint8, P, "f", ctx.device),
                                c(mask0), mask0.size, int(k_add), int(rounds), ctypes.byref(o),
                                c(out), c(mse), c(ms))
    _check(rc, "fi_grow_mask")
    return out, mse, ms


def densify(ctx: Context, side: int, f, mask0, k_add: int, rounds: int,
            rule: int = DENSIFY_TRIANGLES, opts: SolveOpts | None = None, unknowns=None):
    """Mask growth by a chosen rule (fi_densify); returns (mask_order, mse,
    gpu_ms) like grow_mask, mask_order holding mask0 then the pixels added.
    With ``unknowns`` the rounds run on the paper's Delaunay mesh with those
    unknown vertices (fi_densify_delaunay, per-triangle rule)."""
    torch = _torch()
    mask0 = np.ascontiguousarray(np.asarray(mask0, dtype=np.int32).ravel())
    P = int(side) * int(side)
    out = np.empty(mask0.size + int(rounds) * int(k_add), np.int32)
    mse = np.empty(int(rounds) + 1, np.float64)
    ms = np.empty(int(rounds) + 1, np.float64)
    total = ctypes.c_int64()
    o = (opts or SolveOpts()).c()
    c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    fp = _ptr(f, torch.uint8, P, "f", ctx.device)
    if unknowns is None:
        rc = library().fi_densify(ctx._h, int(side), fp, c(mask0), mask0.size, int(k_add),
                                  int(rounds), int(rule), ctypes.byref(o), c(out), c(mse), c(ms),
                                  ctypes.byref(total))
        _check(rc, "fi_densify")
    else:
        if rule != DENSIFY_TRIANGLES:
            raise ValueError("the Delaunay loop uses the per-triangle rule")
        unk = np.ascontiguousarray(np.asarray(unknowns, dtype=np.int32).ravel())
        rc = library().fi_densify_delaunay(ctx._h, int(side), fp, c(mask0), mask0.size, c(unk),
                                           unk.size, int(k_add), int(rounds), ctypes.byref(o),
                                           c(out), c(mse), c(ms), ctypes.byref(total))
        _check(rc, "fi_densify_delaunay")
    return out[:total.value], mse, ms


# ------------------------------------------------------------------ serving --
def footprint_bound(side: int, mask_idx, tonal_iters: int = 30) -> int:
    """Device bytes the server reserves before it admits a request (host only)."""
    m = np.ascontiguousarray(mask_idx, dtype=np.int32)
    out = ctypes.c_int64()
    _check(library().fi_server_footprint(int(side), m.ctypes.data_as(ctypes.c_void_p), m.size,
                                         int(tonal_iters), ctypes.byref(out)),
           "fi_server_footprint")
    return out.value


@dataclass
class ServerOpts:
    """Options of a serving engine (defaults as in the C library)."""
    max_slots: int = 16
    precision: int = PREC_FP32_IR
    hbm_budget: int = 32 << 30
    build_threads: int = 4
    chunk: int = 8

    def c(self) -> _ServerOpts:
        return _ServerOpts(self.max_slots, self.precision, self.hbm_budget, self.build_threads,
                           self.chunk)


class Server:
    """Continuous-batching server: submit (image, mask) requests, collect g
    and the MSEs. Requests run ``inpaint`` then ``tonal_iters`` CGLS
    iterations; see ``fi_server_*`` in include/fi.h."""

    def __init__(self, ctx: Context, opts: ServerOpts | None = None):
        self.opts = opts or ServerOpts()
        h = ctypes.c_void_p()
        _check(library().fi_server_create(ctx._h, ctypes.byref(self.opts.c()), ctypes.byref(h)),
               "fi_server_create")
        self._h = h
        self._g = {}
        _live_servers.add(self)

    def submit(self, f, mask_idx, tonal_iters: int = 30, inner: SolveOpts | None = None) -> int:
        f = np.ascontiguousarray(f, dtype=np.uint8)
        side = int(round(f.size ** 0.5))
        if side * side != f.size:
            raise FIError(E_INVALID, "image must be square")
        m = np.ascontiguousarray(mask_idx, dtype=np.int32)
        g = np.empty(max(m.size, 1), np.float64)
        d = _JobDesc(side, f.ctypes.data_as(ctypes.c_void_p), m.ctypes.data_as(ctypes.c_void_p),
                     m.size, int(tonal_iters), g.ctypes.data_as(ctypes.c_void_p),
                     (inner or SolveOpts()).c())
        t = ctypes.c_uint64()
        _check(library().fi_server_submit(self._h, ctypes.byref(d), ctypes.byref(t)),
               "fi_server_submit")
        self._g[t.value] = g[:m.size]
        return t.value

    def poll(self, ticket: int, wait: bool = True) -> dict | None:
        """None while running; else a dict with g, the MSEs, timings, status."""
        r = _JobResult()
        _check(library().fi_server_poll(self._h, ticket, int(wait), ctypes.byref(r)),
               "fi_server_poll")
        if not r.done:
            return None
        out = {k: getattr(r, k) for k, _ in r._fields_ if k != "error"}
        out["error"] = r.error.decode(errors="replace")
        out["g"] = self._g.pop(ticket)
        return out

    def stats(self) -> dict:
        s = _ServerStats()
        _check(library().fi_server_stats_get(self._h, ctypes.byref(s)), "fi_server_stats_get")
        return {k: getattr(s, k) for k, _ in s._fields_}

    def clock(self) -> float:
        return library().fi_server_clock(self._h)

    def close(self) -> None:
        if self._h:
            library().fi_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
