"""Python binding of libwsp (ctypes).  Argument marshalling only.

Every step of the operator runs in the HIP library; PyTorch supplies device
memory and streams.  Module-level functions mirror the C ABI in
``include/wsp.h`` one to one (``wsp_create``, ``wsp_set_uvw``, ...);
:class:`Operator` strings them together for the common case.

Beyond the Stokes operator (``Operator.degrid`` / ``Operator.grid``):

- ``make_params(kernels="planes")`` interpolates every tap on the fly from
  pre-sampled 1-D w-planes instead of storing per-visibility taps;
- ``make_params(dde_support=J_D)`` with ``Operator.set_dde(d_u, d_v)``
  convolves each kernel with a separable per-visibility DDE kernel;
- ``Operator.degrid_pol`` / ``Operator.grid_pol`` apply the linear
  polarisation operator y_P = Phi Q + i Phi U and its adjoint, each Stokes
  image folded on its own.

There is no fallback: if ``libwsp.so`` is missing or cannot be loaded the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
import warnings

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwsp.so")

WSP_OK = 0
WSP_WARN_QUAD_MAXEVAL = 1
WSP_EINVAL = -1
WSP_ENOMEM_BINDING = -2
WSP_ESUPPORT = -3
WSP_EHIP = -4
WSP_ESTATE = -5

WSP_FP32_FP64PHASE = 0
WSP_FP64 = 1

PRECISIONS = {"fp32_fp64phase": WSP_FP32_FP64PHASE, "fp64": WSP_FP64}
WSP_KERNELS_EXACT = 0
WSP_KERNELS_PLANES = 1
KERNEL_MODES = {"exact": WSP_KERNELS_EXACT, "planes": WSP_KERNELS_PLANES}
WSP_LAYOUT_AUTO = 0
WSP_LAYOUT_RUNS = 1
WSP_LAYOUT_INTERLEAVED = 2
TAP_LAYOUTS = {"auto": WSP_LAYOUT_AUTO, "runs": WSP_LAYOUT_RUNS, "interleaved": WSP_LAYOUT_INTERLEAVED}

EXPORTED = ("wsp_default_params", "wsp_create", "wsp_set_uvw", "wsp_set_stacks",
            "wsp_set_dde", "wsp_get_stacks", "wsp_get_support", "wsp_plan_stats", "wsp_footprint",
            "wsp_bind_memory",
            "wsp_build_kernels", "wsp_build_kernels_part", "wsp_build_kernels_noalloc", "wsp_quad_stats", "wsp_degrid", "wsp_grid",
            "wsp_degrid_ws", "wsp_grid_ws",
            "wsp_degrid_pol", "wsp_grid_pol", "wsp_kernel_values", "wsp_set_timing", "wsp_stage_times", "wsp_destroy",
            "wsp_last_error")

STAGES = ("taper_pad", "fft_forward", "degrid", "zero", "grid", "fft_inverse", "crop_untaper")


class wsp_params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("oversample", ctypes.c_double),
        ("fov_rad", ctypes.c_double),
        ("kb_support", ctypes.c_int32),
        ("kb_beta", ctypes.c_double),
        ("support_scale", ctypes.c_double),
        ("n_stacks", ctypes.c_int32),
        ("fold_conjugate", ctypes.c_int32),
        ("quad_rel_tol", ctypes.c_double),
        ("quad_abs_tol", ctypes.c_double),
        ("quad_max_panels", ctypes.c_int32),
        ("max_support", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("kmeans_tol", ctypes.c_double),
        ("kmeans_max_iter", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("kernel_mode", ctypes.c_int32),
        ("plane_dq", ctypes.c_double),
        ("plane_dw", ctypes.c_double),
        ("dde_support", ctypes.c_int32),
        ("item_taps", ctypes.c_int32),
        ("band_rows", ctypes.c_int32),
        ("tap_layout", ctypes.c_int32),
    ]


class wsp_plan_info(ctypes.Structure):
    _fields_ = [
        ("visibilities", ctypes.c_int64),
        ("taps", ctypes.c_int64),
        ("entries", ctypes.c_int64),
        ("runs", ctypes.c_int64),
        ("items", ctypes.c_int64),
        ("tiles", ctypes.c_int64),
        ("split_tiles", ctypes.c_int64),
        ("touched_cells", ctypes.c_int64),
        ("plan_bytes", ctypes.c_int64),
        ("plan_peak_bytes", ctypes.c_int64),
        ("build_temp_bytes", ctypes.c_int64),
        ("last_build_temp_bytes", ctypes.c_int64),
        ("max_support", ctypes.c_int32),
        ("kmeans_iterations", ctypes.c_int32),
        ("band_rows", ctypes.c_int32),
        ("tap_layout", ctypes.c_int32),
        ("group_steps", ctypes.c_int64),
        ("classes", ctypes.c_int64),
        ("long_taps", ctypes.c_int64),
        ("fft_lds", ctypes.c_int32),
        ("fft_rows", ctypes.c_int32),
    ]


class WspError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"wsp status {status}: {message}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libwsp.so (once) and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "wsp_default_params": (None, [ctypes.POINTER(wsp_params)]),
        "wsp_create": (i32, [ctypes.POINTER(wsp_params), ctypes.POINTER(P)]),
        "wsp_set_uvw": (i32, [P, P, i64, P, P]),
        "wsp_set_stacks": (i32, [P, P, P, P]),
        "wsp_set_dde": (i32, [P, P, P, P]),
        "wsp_get_stacks": (i32, [P, P, P, P]),
        "wsp_get_support": (i32, [P, P, P]),
        "wsp_plan_stats": (i32, [P, ctypes.POINTER(wsp_plan_info)]),
        "wsp_footprint": (i32, [P, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]),
        "wsp_bind_memory": (i32, [P, P, sz, P, sz, P, sz]),
        "wsp_build_kernels": (i32, [P, P]),
        "wsp_build_kernels_part": (i32, [P, i64, i64, P]),
        "wsp_build_kernels_noalloc": (i32, [P, P]),
        "wsp_quad_stats": (i32, [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "wsp_degrid": (i32, [P, P, P, P]),
        "wsp_grid": (i32, [P, P, P, P]),
        "wsp_degrid_ws": (i32, [P, P, P, P, sz, P, sz, P]),
        "wsp_grid_ws": (i32, [P, P, P, P, sz, P, sz, P]),
        "wsp_degrid_pol": (i32, [P, P, P, P, P]),
        "wsp_grid_pol": (i32, [P, P, P, P, P]),
        "wsp_kernel_values": (i32, [P, i64, P, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32)]),
        "wsp_set_timing": (i32, [P, i32]),
        "wsp_stage_times": (i32, [P, P, P]),
        "wsp_destroy": (None, [P]),
        "wsp_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int) -> int:
    if status < 0:
        raise WspError(status, load_library().wsp_last_error().decode())
    if status > 0:
        warnings.warn(f"wsp warning {status}: {load_library().wsp_last_error().decode()}")
    return status


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return t.data_ptr()
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    raise TypeError(type(t))


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


# ---- one-to-one wrappers of the C ABI ---------------------------------------

def wsp_default_params() -> wsp_params:
    p = wsp_params()
    load_library().wsp_default_params(ctypes.byref(p))
    return p


def wsp_create(params: wsp_params) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(load_library().wsp_create(ctypes.byref(params), ctypes.byref(ctx)))
    return ctx


def wsp_set_uvw(ctx, uvw: torch.Tensor, weights: torch.Tensor | None = None, stream=None):
    _check(load_library().wsp_set_uvw(ctx, _ptr(uvw), uvw.shape[0], _ptr(weights), _stream(stream)))


def wsp_set_stacks(ctx, labels: np.ndarray, centres: np.ndarray, stream=None):
    _check(load_library().wsp_set_stacks(ctx, _ptr(labels), _ptr(centres), _stream(stream)))


def wsp_set_dde(ctx, d_u: torch.Tensor, d_v: torch.Tensor, stream=None):
    _check(load_library().wsp_set_dde(ctx, _ptr(d_u), _ptr(d_v), _stream(stream)))


def wsp_get_stacks(ctx, labels: np.ndarray | None, centres: np.ndarray):
    it = ctypes.c_int32()
    _check(load_library().wsp_get_stacks(ctx, _ptr(labels), _ptr(centres), ctypes.byref(it)))
    return it.value


def wsp_get_support(ctx, jp: np.ndarray, folded: np.ndarray | None = None):
    _check(load_library().wsp_get_support(ctx, _ptr(jp), _ptr(folded)))


def wsp_plan_stats(ctx) -> dict:
    info = wsp_plan_info()
    _check(load_library().wsp_plan_stats(ctx, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in info._fields_}


def wsp_footprint(ctx):
    k, g, s = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().wsp_footprint(ctx, ctypes.byref(k), ctypes.byref(g), ctypes.byref(s)))
    return k.value, g.value, s.value


def wsp_bind_memory(ctx, kernels: torch.Tensor, grids: torch.Tensor, scratch: torch.Tensor):
    nb = lambda t: t.numel() * t.element_size()
    _check(load_library().wsp_bind_memory(ctx, _ptr(kernels), nb(kernels), _ptr(grids), nb(grids),
                                          _ptr(scratch), nb(scratch)))


def wsp_build_kernels(ctx, stream=None) -> int:
    return _check(load_library().wsp_build_kernels(ctx, _stream(stream)))


def wsp_build_kernels_part(ctx, first: int, count: int, stream=None) -> int:
    return _check(load_library().wsp_build_kernels_part(ctx, first, count, _stream(stream)))


def wsp_build_kernels_noalloc(ctx, stream=None) -> int:
    return _check(load_library().wsp_build_kernels_noalloc(ctx, _stream(stream)))


def wsp_quad_stats(ctx):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().wsp_quad_stats(ctx, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def wsp_degrid(ctx, image: torch.Tensor, vis: torch.Tensor, stream=None):
    _check(load_library().wsp_degrid(ctx, _ptr(image), _ptr(vis), _stream(stream)))


def wsp_grid(ctx, vis: torch.Tensor, image: torch.Tensor, stream=None):
    _check(load_library().wsp_grid(ctx, _ptr(vis), _ptr(image), _stream(stream)))


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def wsp_degrid_ws(ctx, image: torch.Tensor, vis: torch.Tensor, grids: torch.Tensor, scratch: torch.Tensor,
                  stream=None):
    _check(load_library().wsp_degrid_ws(ctx, _ptr(image), _ptr(vis), _ptr(grids), _nbytes(grids), _ptr(scratch),
                                        _nbytes(scratch), _stream(stream)))


def wsp_grid_ws(ctx, vis: torch.Tensor, image: torch.Tensor, grids: torch.Tensor, scratch: torch.Tensor,
                stream=None):
    _check(load_library().wsp_grid_ws(ctx, _ptr(vis), _ptr(image), _ptr(grids), _nbytes(grids), _ptr(scratch),
                                      _nbytes(scratch), _stream(stream)))


def wsp_degrid_pol(ctx, q_image: torch.Tensor, u_image: torch.Tensor, vis: torch.Tensor, stream=None):
    _check(load_library().wsp_degrid_pol(ctx, _ptr(q_image), _ptr(u_image), _ptr(vis), _stream(stream)))


def wsp_grid_pol(ctx, vis: torch.Tensor, q_image: torch.Tensor, u_image: torch.Tensor, stream=None):
    _check(load_library().wsp_grid_pol(ctx, _ptr(vis), _ptr(q_image), _ptr(u_image), _stream(stream)))


def wsp_kernel_values(ctx, p: int, complex_dtype=np.complex64):
    L = load_library()
    jp, u0, v0 = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(L.wsp_kernel_values(ctx, p, None, ctypes.byref(jp), ctypes.byref(u0), ctypes.byref(v0)))
    out = np.empty((jp.value, jp.value), dtype=complex_dtype)
    _check(L.wsp_kernel_values(ctx, p, _ptr(out), ctypes.byref(jp), ctypes.byref(u0),
                               ctypes.byref(v0)))
    return out, u0.value, v0.value


def wsp_set_timing(ctx, enable: bool):
    _check(load_library().wsp_set_timing(ctx, int(bool(enable))))


def wsp_stage_times(ctx):
    """{stage: (total ms, launches)} since the last wsp_set_timing."""
    ms = np.zeros(len(STAGES))
    cnt = np.zeros(len(STAGES), dtype=np.int64)
    _check(load_library().wsp_stage_times(ctx, _ptr(ms), _ptr(cnt)))
    return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(STAGES)}


def wsp_destroy(ctx):
    load_library().wsp_destroy(ctx)


def wsp_last_error() -> str:
    return load_library().wsp_last_error().decode()


# ---- convenience ----------------------------------------------------------------

def make_params(n: int, fov_rad: float, *, oversample: float = 2.0, kb_support: int = 4,
                kb_beta: float = 0.0, support_scale: float = 1.0, n_stacks: int = 1,
                fold: bool = False, quad_tol: float = 1e-6, quad_max_panels: int = 1024,
                max_support: int = 1024, precision: str = "fp32_fp64phase",
                kmeans_tol: float = 1e-3, kmeans_max_iter: int = 100, device: int = 0,
                kernels: str = "exact", plane_dq: float = 0.0, plane_dw: float = 0.0,
                dde_support: int = 0, item_taps: int = 0, band_rows: int = 0,
                tap_layout: str = "auto") -> wsp_params:
    """Parameters with the library defaults; ``kernels="planes"`` selects taps
    interpolated on the fly from pre-sampled 1-D w-planes (steps plane_dq in
    cells, plane_dw in wavelengths; 0 = the library's defaults 1/64, 1/16)."""
    p = wsp_default_params()
    p.n = n
    p.fov_rad = fov_rad
    p.oversample = oversample
    p.kb_support = kb_support
    p.kb_beta = kb_beta
    p.support_scale = support_scale
    p.n_stacks = n_stacks
    p.fold_conjugate = int(bool(fold))
    p.quad_rel_tol = quad_tol
    p.quad_abs_tol = quad_tol
    p.quad_max_panels = quad_max_panels
    p.max_support = max_support
    p.precision = PRECISIONS[precision]
    p.kmeans_tol = kmeans_tol
    p.kmeans_max_iter = kmeans_max_iter
    p.device = device
    p.kernel_mode = KERNEL_MODES[kernels]
    p.plane_dq = plane_dq
    p.plane_dw = plane_dw
    p.dde_support = dde_support
    p.item_taps = item_taps
    p.band_rows = band_rows
    p.tap_layout = TAP_LAYOUTS[tap_layout]
    return p


class Operator:
    """Phi and Re Phi^dagger for one set of visibilities, kernels resident on the GPU."""

    def __init__(self, params: wsp_params, uvw, weights=None, labels=None, centres=None,
                 build: bool = True, stream=None):
        self.params = params
        self.fp64 = params.precision == WSP_FP64
        self.real_dtype = torch.float64 if self.fp64 else torch.float32
        self.complex_dtype = torch.complex128 if self.fp64 else torch.complex64
        self.device = torch.device("cuda", params.device)
        self.n = params.n
        self.ctx = wsp_create(params)
        self.uvw = torch.as_tensor(np.asarray(uvw, dtype=np.float64)).to(self.device).contiguous()
        self.m = self.uvw.shape[0]
        self.weights = (None if weights is None else
                        torch.as_tensor(np.asarray(weights, dtype=np.float64)).to(self.device).contiguous())
        wsp_set_uvw(self.ctx, self.uvw, self.weights, stream)
        if labels is not None:
            self.set_stacks(labels, centres, stream)
        self._bind()
        self.build_status = None
        if build:
            self.build(stream)

    def _bind(self):
        kb, gb, sb = wsp_footprint(self.ctx)
        self.footprint = {"kernel_bytes": kb, "grid_bytes": gb, "scratch_bytes": sb}
        self.kernels = torch.empty(max(kb, 256), dtype=torch.uint8, device=self.device)
        self.grids = torch.empty(max(gb, 256), dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(max(sb, 256), dtype=torch.uint8, device=self.device)
        wsp_bind_memory(self.ctx, self.kernels, self.grids, self.scratch)

    def set_stacks(self, labels, centres, stream=None):
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        centres = np.ascontiguousarray(centres, dtype=np.float64)
        wsp_set_stacks(self.ctx, labels, centres, stream)
        self._bind()

    def set_dde(self, d_u, d_v, stream=None):
        """Per-visibility separable DDE kernels, complex [M, J_D] each (Eq. (11)); rebuild after."""
        d_u = torch.as_tensor(np.asarray(d_u)).to(self.device, self.complex_dtype).contiguous()
        d_v = torch.as_tensor(np.asarray(d_v)).to(self.device, self.complex_dtype).contiguous()
        jd = self.params.dde_support
        if d_u.shape != (self.m, jd) or d_v.shape != (self.m, jd):
            raise ValueError(f"DDE kernels must be [{self.m}, {jd}]")
        wsp_set_dde(self.ctx, d_u, d_v, stream)

    def build(self, stream=None, part: int | None = None, progress=None) -> int:
        """Build all kernels; with ``part``, in slices of that many visibilities,
        calling ``progress(done, total)`` after each."""
        if part is None:
            self.build_status = wsp_build_kernels(self.ctx, stream)
            return self.build_status
        status = 0
        for first in range(0, self.m, part):
            cnt = min(part, self.m - first)
            status = max(status, wsp_build_kernels_part(self.ctx, first, cnt, stream))
            if progress is not None:
                progress(first + cnt, self.m)
        self.build_status = status
        return status

    def stacks(self):
        K = self.params.n_stacks
        labels = np.empty(self.m, dtype=np.int32)
        centres = np.empty(K, dtype=np.float64)
        it = wsp_get_stacks(self.ctx, labels, centres)
        return labels, centres, it

    def support(self):
        jp = np.empty(self.m, dtype=np.int32)
        folded = np.empty(self.m, dtype=np.uint8)
        wsp_get_support(self.ctx, jp, folded)
        return jp, folded.astype(bool)

    def quad_stats(self):
        return wsp_quad_stats(self.ctx)

    def plan_stats(self) -> dict:
        return wsp_plan_stats(self.ctx)

    def kernel(self, p: int):
        return wsp_kernel_values(self.ctx, p, np.complex128 if self.fp64 else np.complex64)

    def new_workspace(self):
        """A (grids, scratch) pair of this operator's footprint sizes: with one per
        concurrent request, requests on this operator can run at once on
        different streams (``workspace=`` of degrid / grid)."""
        fp = self.footprint
        return (torch.empty(max(fp["grid_bytes"], 256), dtype=torch.uint8, device=self.device),
                torch.empty(max(fp["scratch_bytes"], 256), dtype=torch.uint8, device=self.device))

    def degrid(self, image: torch.Tensor, out: torch.Tensor | None = None, stream=None, workspace=None):
        image = image.to(self.device, self.real_dtype).contiguous()
        if image.shape != (self.n, self.n):
            raise ValueError(f"image must be {self.n}x{self.n}")
        if out is None:
            out = torch.empty(self.m, dtype=self.complex_dtype, device=self.device)
        if workspace is None:
            wsp_degrid(self.ctx, image, out, stream)
        else:
            wsp_degrid_ws(self.ctx, image, out, workspace[0], workspace[1], stream)
        return out

    def grid(self, vis: torch.Tensor, out: torch.Tensor | None = None, stream=None, workspace=None):
        vis = vis.to(self.device, self.complex_dtype).contiguous()
        if vis.shape != (self.m,):
            raise ValueError(f"vis must have {self.m} entries")
        if out is None:
            out = torch.empty((self.n, self.n), dtype=self.real_dtype, device=self.device)
        if workspace is None:
            wsp_grid(self.ctx, vis, out, stream)
        else:
            wsp_grid_ws(self.ctx, vis, out, workspace[0], workspace[1], stream)
        return out

    def degrid_pol(self, q_image: torch.Tensor, u_image: torch.Tensor, out: torch.Tensor | None = None,
                   stream=None):
        """Linear-polarisation visibilities y_Q + i y_U, each Stokes image folded on its own (Eq. (9))."""
        q_image = q_image.to(self.device, self.real_dtype).contiguous()
        u_image = u_image.to(self.device, self.real_dtype).contiguous()
        if q_image.shape != (self.n, self.n) or u_image.shape != (self.n, self.n):
            raise ValueError(f"images must be {self.n}x{self.n}")
        if out is None:
            out = torch.empty(self.m, dtype=self.complex_dtype, device=self.device)
        wsp_degrid_pol(self.ctx, q_image, u_image, out, stream)
        return out

    def grid_pol(self, vis: torch.Tensor, stream=None):
        """(Re Phi^dagger vis, Re Phi^dagger (-i vis)): the adjoint of degrid_pol."""
        vis = vis.to(self.device, self.complex_dtype).contiguous()
        if vis.shape != (self.m,):
            raise ValueError(f"vis must have {self.m} entries")
        q = torch.empty((self.n, self.n), dtype=self.real_dtype, device=self.device)
        u = torch.empty((self.n, self.n), dtype=self.real_dtype, device=self.device)
        wsp_grid_pol(self.ctx, vis, q, u, stream)
        return q, u

    def close(self):
        if getattr(self, "ctx", None) is not None:
            wsp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
