"""Python binding of libzm (Zernike moments on MI355X / gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/zm.h``.  PyTorch supplies
device memory and the HIP stream.  There is no CPU fallback: if the built
library is missing, importing this package raises.

Typical use::

    import torch, paper_2304_14492_amd as zm
    plan = zm.Plan(200, 2160, 3840, dtype="f32")
    frames = torch.rand(8, 2160, 3840, device="cuda")
    Z = plan.moments(frames)            # [8, num_moments, 2] float32 (re, im)
    Zc = zm.as_complex(Z)               # complex view, canonical (n, m) order

Also here: ``Batch`` / ``moments_batch`` (frames of mixed sizes and orders in
one persistent launch), ``reconstruct`` / ``recon_error`` (eq. (9), (10),
(12), (13), min-max), ``embed`` / ``pad_size`` (Sec. 3), ``moment_cartesian``
(one moment by the Cartesian pixel sum of eq. (6) / (14) with 8-point
symmetry); ``serve`` (continuous batching) and ``dedup`` (moment hashes,
Sec. 2.7) are submodules.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libzm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libzm.so is not built ({LIB_PATH}); run `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python paper_2304_14492_amd/_build.py` first")

# torch first: its HIP runtime is then the one libzm binds to, so the
# library, torch's allocator and torch's streams share one runtime in the
# process (loading libzm first pulls in the system runtime instead).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

ZM_OK, ZM_EINVAL, ZM_ENOMEM, ZM_EDEVICE, ZM_EUNSUPPORTED, ZM_EBUSY = 0, -1, -2, -3, -4, -5
DTYPES = {"f64": 0, "f32": 1, "bf16x2": 2, "f16x2": 3}
RULES = {"midpoint": 0, "gauss_legendre": 1}


class zm_plan_desc(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int), ("H", ctypes.c_int), ("W", ctypes.c_int), ("dtype", ctypes.c_int),
                ("neumann", ctypes.c_int), ("rings", ctypes.c_int), ("angles", ctypes.c_int),
                ("rule", ctypes.c_int), ("device", ctypes.c_int)]


class zm_plan_info_t(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int), ("H", ctypes.c_int), ("W", ctypes.c_int), ("rings", ctypes.c_int),
                ("angles", ctypes.c_int), ("num_moments", ctypes.c_int), ("rings_padded", ctypes.c_int),
                ("dtype", ctypes.c_int), ("neumann", ctypes.c_int), ("rule", ctypes.c_int),
                ("device", ctypes.c_int), ("resident_bytes", ctypes.c_size_t),
                ("workspace_bytes_per_image", ctypes.c_size_t), ("workspace_bytes_fixed", ctypes.c_size_t)]


class zm_job(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("d_image", ctypes.c_void_p), ("d_Z", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_SIGS = {
    "zm_num_moments": (ctypes.c_int, [ctypes.c_int]),
    "zm_index": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "zm_plan": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(_vp)]),
    "zm_plan_ex": (ctypes.c_int, [ctypes.POINTER(zm_plan_desc), ctypes.POINTER(_vp)]),
    "zm_plan_info": (ctypes.c_int, [_vp, ctypes.POINTER(zm_plan_info_t)]),
    "zm_radial_table": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), _sz]),
    "zm_ring_nodes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _sz]),
    "zm_operand_table": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double), _sz]),
    "zm_workspace_size": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_sz)]),
    "zm_moments": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_longlong, _vp, _vp, _sz, _vp]),
    "zm_moments_polar": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _sz, _vp]),
    "zm_resample_polar": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_longlong, _vp, _vp]),
    "zm_moments_static": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_longlong, _vp, _vp]),
    "zm_static_scratch_bytes": (_sz, []),
    "zm_count_nonfinite": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp]),
    "zm_spectra": (ctypes.c_int, [_vp, _vp, ctypes.c_int, ctypes.c_longlong, _vp, _sz, _vp]),
    "zm_project": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _sz, _vp]),
    "zm_reconstruct": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _sz, _vp]),
    "zm_recon_workspace_size": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_sz)]),
    "zm_recon_error": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _vp, _sz, _vp]),
    "zm_pad_size": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "zm_embed": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp]),
    "zm_batch_create": (ctypes.c_int, [ctypes.POINTER(zm_job), ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
    "zm_batch_run": (ctypes.c_int, [_vp, _vp]),
    "zm_batch_update": (ctypes.c_int, [_vp, ctypes.POINTER(zm_job), ctypes.c_int]),
    "zm_batch_check": (ctypes.c_int, [_vp]),
    "zm_batch_config": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_sz)]),
    "zm_batch_destroy": (ctypes.c_int, [_vp]),
    "zm_moments_batch": (ctypes.c_int, [ctypes.POINTER(zm_job), ctypes.c_int, _vp]),
    "zm_batch_workspace_size": (ctypes.c_int, [ctypes.POINTER(zm_job), ctypes.c_int, ctypes.POINTER(_sz)]),
    "zm_moments_batch_ws": (ctypes.c_int, [ctypes.POINTER(zm_job), ctypes.c_int, _vp, _sz, _vp]),
    "zm_batch_stage_size": (ctypes.c_int, [ctypes.POINTER(zm_job), ctypes.c_int, ctypes.POINTER(_sz)]),
    "zm_moments_batch_async": (ctypes.c_int, [ctypes.POINTER(zm_job), ctypes.c_int, _vp, _sz, _vp, _sz, _vp]),
    "zm_batch_stage_status": (ctypes.c_int, [_vp]),
    "zm_cartesian_workspace_size": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_sz)]),
    "zm_moment_cartesian": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_longlong, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, _vp, _vp, _sz, _vp]),
    "zm_destroy": (ctypes.c_int, [_vp]),
    "zm_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "zm_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class ZmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.zm_status_str(status).decode() + ": " + _lib.zm_last_error().decode()
        super().__init__(f"{where}: {msg}")


def _check(st: int, where: str):
    if st != ZM_OK:
        raise ZmError(st, where)


def num_moments(n_max: int) -> int:
    return _lib.zm_num_moments(n_max)


def index(n: int, m: int) -> int:
    return _lib.zm_index(n, m)


RECON_POLAR, RECON_CARTESIAN = 0, 1
RECON_ONESIDED, RECON_MINMAX = 1, 2


def pad_size(n: int):
    """(size, offset) of the Sec. 3 embedding of an n x n image."""
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(_lib.zm_pad_size(n, ctypes.byref(a), ctypes.byref(b)), "zm_pad_size")
    return a.value, b.value


def embed(frames, stream=None):
    """Embed [B, n, n] frames (float32/float64 CUDA) into [B, size, size] zero grids (Sec. 3)."""
    import torch
    B, n, n2 = frames.shape
    if n != n2:
        raise ValueError("embed expects square frames")
    if frames.dtype not in (torch.float32, torch.float64):
        raise ValueError(f"embed expects float32 or float64 frames, got {frames.dtype}")
    frames = frames.contiguous()
    _need(frames, "frames")
    size, _ = pad_size(n)
    out = torch.empty(B, size, size, dtype=frames.dtype, device=frames.device)
    _keep_alive(stream, out)
    _check(_lib.zm_embed(_vp(frames.data_ptr()), n, B, _vp(out.data_ptr()), int(frames.dtype == torch.float64),
                         _stream_handle(stream)), "zm_embed")
    return out


def moment_cartesian(frames, n: int, m: int, neumann: bool = False, workspace=None, stream=None):
    """One moment Z_nm of each of [B, N, N] (or [N, N]) float32 CUDA frames by
    the Cartesian pixel sum of eq. (6) (eq. (14) with ``neumann``), using the
    8-point symmetry of the square grid.  Returns a complex128 tensor [B]
    (a 0-d tensor for one frame) on the frames' device."""
    import torch
    squeeze = frames.dim() == 2
    if squeeze:
        frames = frames.unsqueeze(0)
    B, N, N2 = frames.shape
    if N != N2:
        raise ValueError("moment_cartesian expects square frames")
    if frames.dtype != torch.float32 or not frames.is_cuda:
        raise ValueError("moment_cartesian expects float32 CUDA frames")
    frames = frames.contiguous()
    need = _sz()
    _check(_lib.zm_cartesian_workspace_size(N, B, ctypes.byref(need)), "zm_cartesian_workspace_size")
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=frames.device)
        _keep_alive(stream, workspace)
    _need(workspace, "workspace", dtype=torch.uint8, device=frames.device.index)
    out = torch.empty(B, 2, dtype=torch.float64, device=frames.device)
    _keep_alive(stream, out)
    _check(_lib.zm_moment_cartesian(_vp(frames.data_ptr()), N, B, N * N, int(n), int(m), int(bool(neumann)),
                                    _vp(out.data_ptr()), _vp(workspace.data_ptr()), workspace.numel(),
                                    _stream_handle(stream)), "zm_moment_cartesian")
    z = torch.view_as_complex(out)
    return z[0] if squeeze else z


def exported_symbols():
    return list(_SIGS)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t, name, shape=None, dtype=None, min_numel=None, device=None, contiguous=True, on_device=True):
    """Check a buffer before its pointer crosses the ABI: the kernels trust
    shape, element type, layout and device, so a mismatch would become an
    out-of-bounds device access.  Raises ValueError naming the problem."""
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name}: expected dtype {dtype}, got {t.dtype}")
    if contiguous and not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name}: needs at least {min_numel} elements, has {t.numel()}")
    if not on_device:
        return
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a CUDA (HIP) tensor")
    if device is not None and device >= 0 and t.device.index != device:
        raise ValueError(f"{name}: on device {t.device.index}, the plan is on device {device}")


def _keep_alive(stream, *tensors):
    """Tensors allocated here but used by work on a caller-given stream stay
    reserved until that stream has passed this point (the caching allocator
    otherwise hands their memory out again once they are freed)."""
    if stream is None:
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


class Plan:
    """A resident plan: polar grid, FP64 radial table (eq. (7)) and the
    projection operand, for frames of one size and one n_max."""

    def __init__(self, n_max: int, H: int, W: int, dtype: str = "f32", neumann: bool = False,
                 rings: int = 0, angles: int = 0, rule: str = "midpoint", device: int = -1):
        d = zm_plan_desc(n_max, H, W, DTYPES[dtype], int(bool(neumann)), rings, angles, RULES[rule], device)
        h = _vp()
        _check(_lib.zm_plan_ex(ctypes.byref(d), ctypes.byref(h)), "zm_plan_ex")
        self._h = h
        self.dtype = dtype
        info = zm_plan_info_t()
        _check(_lib.zm_plan_info(h, ctypes.byref(info)), "zm_plan_info")
        self.info = info
        self.n_max, self.H, self.W = info.n_max, info.H, info.W
        self.rings, self.angles, self.num_moments = info.rings, info.angles, info.num_moments
        self.rings_padded = info.rings_padded
        self.neumann = bool(info.neumann)
        self.device = info.device

    def close(self):
        """Free the plan.  Work still in flight on it is waited for first
        (the library refuses to free a plan that is in use)."""
        if getattr(self, "_h", None):
            st = _lib.zm_destroy(self._h)
            if st == ZM_EBUSY and torch.cuda.is_available():
                torch.cuda.synchronize(self.device if self.device >= 0 else None)
                st = _lib.zm_destroy(self._h)
            if st == ZM_EBUSY:
                raise ZmError(st, "zm_destroy")  # a Batch built on the plan still exists
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def radial_table(self):
        import numpy as np
        out = np.empty((self.num_moments, self.rings), dtype=np.float64)
        _check(_lib.zm_radial_table(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size),
               "zm_radial_table")
        return out

    def ring_nodes(self):
        import numpy as np
        rho = np.empty(self.rings, dtype=np.float64)
        w = np.empty(self.rings, dtype=np.float64)
        _check(_lib.zm_ring_nodes(self._h, rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self.rings), "zm_ring_nodes")
        return rho, w

    def workspace_size(self, batch: int) -> int:
        n = _sz()
        _check(_lib.zm_workspace_size(self._h, batch, ctypes.byref(n)), "zm_workspace_size")
        return n.value

    def _real_dtype(self):
        import torch
        return torch.float64 if self.dtype == "f64" else torch.float32

    def workspace(self, batch: int, device=None):
        import torch
        return torch.empty(self.workspace_size(batch), dtype=torch.uint8, device=device or "cuda")

    def _check_out(self, out, B):
        _need(out, "out", shape=(B, self.num_moments, 2), dtype=self._real_dtype(), device=self.device)

    def _check_workspace(self, workspace, B):
        import torch
        _need(workspace, "workspace", dtype=torch.uint8, min_numel=self.workspace_size(B), device=self.device)

    def moments(self, frames, out=None, workspace=None, stream=None):
        """frames: CUDA tensor [B, H, W] (or [H, W]) of float32 (float64 for
        dtype "f64"), rows contiguous.  Returns [B, num_moments, 2] (re, im)."""
        import torch
        squeeze = frames.dim() == 2
        if squeeze:
            frames = frames.unsqueeze(0)
        self._check_frames(frames)
        B = frames.shape[0]
        if out is None:
            out = torch.empty(B, self.num_moments, 2, dtype=self._real_dtype(), device=frames.device)
            _keep_alive(stream, out)
        if workspace is None:
            workspace = self.workspace(B, frames.device)
            _keep_alive(stream, workspace)
        self._check_out(out, B)
        self._check_workspace(workspace, B)
        st = _lib.zm_moments(self._h, _vp(frames.data_ptr()), B, frames.stride(0) if B > 1 else self.H * self.W,
                             _vp(out.data_ptr()), _vp(workspace.data_ptr()), workspace.numel(),
                             _stream_handle(stream))
        _check(st, "zm_moments")
        return out[0] if squeeze else out

    def moments_static(self, frames, out=None, stream=None):
        """zm_moments_static: as moments(), with the library's static device
        scratch as the workspace (no allocation in the library; calls that
        overlap on one device race).  ``out`` must be given by callers that
        cannot allocate."""
        import torch
        squeeze = frames.dim() == 2
        if squeeze:
            frames = frames.unsqueeze(0)
        self._check_frames(frames)
        B = frames.shape[0]
        if out is None:
            out = torch.empty(B, self.num_moments, 2, dtype=self._real_dtype(), device=frames.device)
            _keep_alive(stream, out)
        self._check_out(out, B)
        _check(_lib.zm_moments_static(self._h, _vp(frames.data_ptr()), B,
                                      frames.stride(0) if B > 1 else self.H * self.W, _vp(out.data_ptr()),
                                      _stream_handle(stream)), "zm_moments_static")
        return out[0] if squeeze else out

    def count_nonfinite(self, Z, counts=None, stream=None):
        """zm_count_nonfinite: per frame, how many of the moment values in Z
        ([B, num_moments, 2] or [num_moments, 2], as moments() returns) are
        NaN or +-Inf.  Returns an int32 CUDA tensor [B] (asynchronous)."""
        import torch
        if Z.dim() == 2:
            Z = Z.unsqueeze(0)
        B = Z.shape[0]
        _need(Z, "Z", shape=(B, self.num_moments, 2), dtype=self._real_dtype(), device=self.device)
        if counts is None:
            counts = torch.empty(B, dtype=torch.int32, device=Z.device)
            _keep_alive(stream, counts)
        _need(counts, "counts", shape=(B,), dtype=torch.int32, device=self.device)
        _check(_lib.zm_count_nonfinite(self._h, _vp(Z.data_ptr()), B, _vp(counts.data_ptr()), _stream_handle(stream)),
               "zm_count_nonfinite")
        return counts

    def _check_frames(self, frames):
        if frames.dim() != 3 or frames.shape[1] != self.H or frames.shape[2] != self.W:
            raise ValueError(f"expected frames of shape [B, {self.H}, {self.W}], got {tuple(frames.shape)}")
        if frames.dtype != self._real_dtype():
            raise ValueError(f"frames must be a CUDA {self._real_dtype()} tensor, got {frames.dtype}")
        if frames.stride(2) != 1 or frames.stride(1) != self.W:
            raise ValueError("frame rows must be contiguous")
        if frames.shape[0] > 1 and frames.stride(0) < self.H * self.W:
            raise ValueError("frames must not overlap (frame stride < H * W)")
        _need(frames, "frames", contiguous=False, device=self.device)

    def spectra(self, frames, workspace, stream=None):
        """Stage 1 only: ring spectra of frames [B, H, W] into `workspace`."""
        self._check_frames(frames)
        B = frames.shape[0]
        self._check_workspace(workspace, B)
        _check(_lib.zm_spectra(self._h, _vp(frames.data_ptr()), B,
                               frames.stride(0) if B > 1 else self.H * self.W, _vp(workspace.data_ptr()),
                               workspace.numel(), _stream_handle(stream)), "zm_spectra")

    def project(self, batch, out, workspace, stream=None):
        """Stage 2 only: moments of the spectra left in `workspace` by spectra()."""
        self._check_out(out, batch)
        self._check_workspace(workspace, batch)
        _check(_lib.zm_project(self._h, batch, _vp(out.data_ptr()), _vp(workspace.data_ptr()),
                               workspace.numel(), _stream_handle(stream)), "zm_project")
        return out

    def resample_polar(self, frames, out=None, stream=None):
        """The resampler alone: frames [B, H, W] -> polar image [B, rings, angles] (Sec. 2.5)."""
        import torch
        squeeze = frames.dim() == 2
        if squeeze:
            frames = frames.unsqueeze(0)
        self._check_frames(frames)
        B = frames.shape[0]
        if out is None:
            out = torch.empty(B, self.rings, self.angles, dtype=self._real_dtype(), device=frames.device)
            _keep_alive(stream, out)
        _need(out, "out", shape=(B, self.rings, self.angles), dtype=self._real_dtype(), device=self.device)
        _check(_lib.zm_resample_polar(self._h, _vp(frames.data_ptr()), B,
                                      frames.stride(0) if B > 1 else self.H * self.W, _vp(out.data_ptr()),
                                      _stream_handle(stream)), "zm_resample_polar")
        return out[0] if squeeze else out

    def moments_polar(self, polar, out=None, workspace=None, stream=None):
        """polar: CUDA tensor [B, rings, angles], contiguous."""
        import torch
        squeeze = polar.dim() == 2
        if squeeze:
            polar = polar.unsqueeze(0)
        polar = polar.contiguous()
        if polar.shape[1:] != (self.rings, self.angles) or polar.dtype != self._real_dtype():
            raise ValueError("polar must be [B, rings, angles] of the plan's real dtype")
        _need(polar, "polar", device=self.device)
        B = polar.shape[0]
        if out is None:
            out = torch.empty(B, self.num_moments, 2, dtype=self._real_dtype(), device=polar.device)
            _keep_alive(stream, out)
        if workspace is None:
            workspace = self.workspace(B, polar.device)
            _keep_alive(stream, workspace)
        self._check_out(out, B)
        self._check_workspace(workspace, B)
        _check(_lib.zm_moments_polar(self._h, _vp(polar.data_ptr()), B, _vp(out.data_ptr()),
                                     _vp(workspace.data_ptr()), workspace.numel(), _stream_handle(stream)),
               "zm_moments_polar")
        return out[0] if squeeze else out


def _recon_ws(plan, batch, device):
    import torch
    n = _sz()
    _check(_lib.zm_recon_workspace_size(plan._h, batch, ctypes.byref(n)), "zm_recon_workspace_size")
    return torch.empty(max(n.value, 1), dtype=torch.uint8, device=device)


def reconstruct(plan, Z, kind="cartesian", one_sided=False, minmax_ref=None, stream=None):
    """eq. (9) from moments Z [B, num_moments, 2] (plan's real dtype, CUDA).
    kind "polar" -> [B, R, A]; "cartesian" -> [B, H, W] (0 outside the disk).
    minmax_ref: frames [B, H, W] to renormalise onto (Cartesian only)."""
    import torch
    squeeze = Z.dim() == 2
    if squeeze:
        Z = Z.unsqueeze(0)
    if kind not in ("polar", "cartesian"):
        raise ValueError(f"kind must be 'polar' or 'cartesian', got {kind!r}")
    Z = Z.contiguous()
    B = Z.shape[0]
    _need(Z, "Z", shape=(B, plan.num_moments, 2), dtype=plan._real_dtype(), device=plan.device)
    k = RECON_POLAR if kind == "polar" else RECON_CARTESIAN
    shape = (B, plan.rings, plan.angles) if k == RECON_POLAR else (B, plan.H, plan.W)
    out = torch.empty(shape, dtype=plan._real_dtype(), device=Z.device)
    flags = (RECON_ONESIDED if one_sided else 0) | (RECON_MINMAX if minmax_ref is not None else 0)
    ws = _recon_ws(plan, B, Z.device)
    _keep_alive(stream, out, ws)
    ref = None
    if minmax_ref is not None:
        ref = minmax_ref.unsqueeze(0) if minmax_ref.dim() == 2 else minmax_ref
        ref = ref.contiguous()
        _need(ref, "minmax_ref", shape=(B, plan.H, plan.W), dtype=plan._real_dtype(), device=plan.device)
    _check(_lib.zm_reconstruct(plan._h, _vp(Z.data_ptr()), B, _vp(out.data_ptr()), k, flags,
                               _vp(ref.data_ptr()) if ref is not None else None, _vp(ws.data_ptr()), ws.numel(),
                               _stream_handle(stream)), "zm_reconstruct")
    return out[0] if squeeze else out


def recon_error(plan, ref, recon, stream=None):
    """eq. (13), eq. (10) and eq. (12) per frame over the disk: list of dicts
    (eps12 covers the pixels with f != 0; zeros counts those left out)."""
    import numpy as np
    if ref.dim() == 2:
        ref, recon = ref.unsqueeze(0), recon.unsqueeze(0)
    ref, recon = ref.contiguous(), recon.contiguous()
    B = ref.shape[0]
    for t, name in ((ref, "ref"), (recon, "recon")):
        _need(t, name, shape=(B, plan.H, plan.W), dtype=plan._real_dtype(), on_device=False)
    _need(ref, "ref", device=plan.device)
    _need(recon, "recon", device=plan.device)
    ws = _recon_ws(plan, B, ref.device)
    _keep_alive(stream, ws)
    out = np.empty((B, 7), dtype=np.float64)
    _check(_lib.zm_recon_error(plan._h, _vp(ref.data_ptr()), _vp(recon.data_ptr()), B,
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _vp(ws.data_ptr()), ws.numel(),
                               _stream_handle(stream)), "zm_recon_error")
    return [dict(eps13=r[0], eps10=r[1], sse=r[2], fmax=r[3], count=int(r[4]), eps12=r[5], zeros=int(r[6]))
            for r in out]


BATCH_AUTOTUNE, BATCH_NO_GRAPH, BATCH_PER_PLAN = 1, 2, 4


def _jobs(plans, frames, outs):
    n = len(plans)
    if not (len(frames) == n and len(outs) == n):
        raise ValueError("plans, frames and outputs must have the same length")
    import torch
    arr = (zm_job * n)()
    for i, (p, f, z) in enumerate(zip(plans, frames, outs)):
        # FP64 plans are refused by the library (ZM_EUNSUPPORTED) before any device access
        real = torch.float64 if p.dtype == "f64" else torch.float32
        _need(f, f"job {i} frame", shape=(p.H, p.W), dtype=real, on_device=False)
        _need(z, f"job {i} output", shape=(p.num_moments, 2), dtype=real, on_device=False)
        _need(f, f"job {i} frame", device=p.device)
        _need(z, f"job {i} output", device=p.device)
        arr[i].plan = p.handle
        arr[i].d_image = f.data_ptr()
        arr[i].d_Z = z.data_ptr()
    return arr


class Batch:
    """Mixed batch (frames of different sizes / orders) in one persistent
    launch, replayed from a captured HIP graph.  frames[i] is a [H, W] float32
    CUDA tensor matching plans[i]; outs[i] is [num_moments, 2] float32."""

    def __init__(self, plans, frames, outs=None, autotune=False, graph=True, per_plan=False):
        import torch
        if outs is None:
            outs = [torch.empty(p.num_moments, 2, dtype=p._real_dtype(), device=f.device) for p, f in zip(plans, frames)]
        self.plans, self.frames, self.outs = list(plans), list(frames), list(outs)
        jobs = _jobs(self.plans, self.frames, self.outs)
        flags = (BATCH_AUTOTUNE if autotune else 0) | (0 if graph else BATCH_NO_GRAPH) | \
            (BATCH_PER_PLAN if per_plan else 0)
        h = _vp()
        _check(_lib.zm_batch_create(jobs, len(jobs), flags, ctypes.byref(h)), "zm_batch_create")
        self._h = h

    def run(self, stream=None):
        _check(_lib.zm_batch_run(self._h, _stream_handle(stream)), "zm_batch_run")
        return self.outs

    def update(self, frames, outs=None):
        if outs is not None:
            self.outs = list(outs)
        self.frames = list(frames)
        jobs = _jobs(self.plans, self.frames, self.outs)
        _check(_lib.zm_batch_update(self._h, jobs, len(jobs)), "zm_batch_update")

    def check(self):
        _check(_lib.zm_batch_check(self._h), "zm_batch_check")

    def config(self):
        g, o, n, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), _sz()
        _check(_lib.zm_batch_config(self._h, ctypes.byref(g), ctypes.byref(o), ctypes.byref(n), ctypes.byref(b)),
               "zm_batch_config")
        return dict(grid=g.value, order=o.value, n_items=n.value, device_bytes=b.value,
                    route="per_plan" if g.value == 0 else "persistent")

    def close(self):
        if getattr(self, "_h", None):
            _lib.zm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_workspace_size(plans, frames, outs) -> int:
    """Device bytes zm_moments_batch_ws needs for these jobs."""
    jobs = _jobs(plans, frames, outs)
    n = _sz()
    _check(_lib.zm_batch_workspace_size(jobs, len(jobs), ctypes.byref(n)), "zm_batch_workspace_size")
    return n.value


def moments_batch(plans, frames, outs=None, workspace=None, stream=None):
    """One-shot mixed batch (no graph); returns the list of [num_moments, 2]
    outputs.  With ``workspace`` (a uint8 CUDA tensor of at least
    batch_workspace_size bytes) the library allocates no device memory."""
    import torch
    if outs is None:
        outs = [torch.empty(p.num_moments, 2, dtype=p._real_dtype(), device=f.device) for p, f in zip(plans, frames)]
        _keep_alive(stream, *outs)
    jobs = _jobs(plans, frames, outs)
    if workspace is None:
        _check(_lib.zm_moments_batch(jobs, len(jobs), _stream_handle(stream)), "zm_moments_batch")
        return outs
    n = _sz()
    _check(_lib.zm_batch_workspace_size(jobs, len(jobs), ctypes.byref(n)), "zm_batch_workspace_size")
    _need(workspace, "workspace", dtype=torch.uint8, min_numel=n.value, device=plans[0].device)
    _check(_lib.zm_moments_batch_ws(jobs, len(jobs), _vp(workspace.data_ptr()), workspace.numel(),
                                    _stream_handle(stream)), "zm_moments_batch_ws")
    return outs


class BatchLaunch:
    """zm_moments_batch_async: one persistent launch of a mixed batch,
    enqueued on ``stream`` without waiting.  Allocates (unless given) the
    device workspace and a pinned staging buffer and keeps them, the frames
    and the outputs referenced until ``check`` has run after the stream
    passed the launch (e.g. after ``done.synchronize()`` or ``done.query()``
    of an event recorded after it)."""

    def __init__(self, plans, frames, outs=None, workspace=None, stage=None, stream=None):
        import torch
        if outs is None:
            outs = [torch.empty(p.num_moments, 2, dtype=p._real_dtype(), device=f.device)
                    for p, f in zip(plans, frames)]
        jobs = _jobs(plans, frames, outs)
        n, m = _sz(), _sz()
        _check(_lib.zm_batch_workspace_size(jobs, len(jobs), ctypes.byref(n)), "zm_batch_workspace_size")
        _check(_lib.zm_batch_stage_size(jobs, len(jobs), ctypes.byref(m)), "zm_batch_stage_size")
        if workspace is None:
            workspace = torch.empty(n.value, dtype=torch.uint8, device=frames[0].device)
        if stage is None:
            stage = torch.empty(m.value, dtype=torch.uint8, pin_memory=True)
        _need(workspace, "workspace", dtype=torch.uint8, min_numel=n.value, device=plans[0].device)
        _need(stage, "stage", dtype=torch.uint8, min_numel=m.value, on_device=False)
        if stage.is_cuda or not stage.is_pinned():
            raise ValueError("stage: must be pinned host memory")
        _keep_alive(stream, workspace, *frames, *outs)
        self.plans, self.frames, self.outs, self.workspace, self.stage = plans, frames, outs, workspace, stage
        _check(_lib.zm_moments_batch_async(jobs, len(jobs), _vp(workspace.data_ptr()), workspace.numel(),
                                           _vp(stage.data_ptr()), stage.numel(), _stream_handle(stream)),
               "zm_moments_batch_async")

    def check(self):
        """The run's status from the staging buffer (call after the stream passed it)."""
        _check(_lib.zm_batch_stage_status(_vp(self.stage.data_ptr())), "zm_batch_stage_status")


def as_complex(Z):
    """[..., num_moments, 2] real tensor -> complex tensor [..., num_moments]."""
    import torch
    return torch.view_as_complex(Z.contiguous())
