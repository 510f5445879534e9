"""Thin Python binding of libhologen's C ABI (include/hologen.h).

Argument marshalling only: every step of the hologram path runs in the HIP
kernels behind the C ABI.  PyTorch supplies device memory (tensor
``data_ptr()``) and streams (``torch.cuda.current_stream().cuda_stream``).
If the shared library has not been built this module raises on first use;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

HG_OK = 0
HG_ERR_INVALID_ARGUMENT = 1
HG_ERR_UNSUPPORTED_SIZE = 2
HG_ERR_OUT_OF_MEMORY = 3
HG_ERR_DEVICE = 4
HG_ERR_INTERNAL = 5

HG_FOURIER = 0
HG_FRESNEL = 1
HG_ANGULAR = 2
HG_PHASE = 0
HG_PHASE_QUANTISED = 1
HG_BINARY_PHASE = 2
HG_AMPLITUDE = 3
HG_FORWARD = 1
HG_INVERSE = -1

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhologen.so")

HG_KERNEL_GS_REPLAY = 1
HG_KERNEL_GS_SLM = 2
HG_KERNEL_OSPR_A = 3
HG_KERNEL_OSPR_B = 4
HG_KERNEL_OSPR_C = 5
HG_KERNEL_PROP_ROW = 6
HG_KERNEL_PROP_COL = 7

EXPORTED = ("hg_plan_create", "hg_plan_destroy", "hg_workspace_bytes", "hg_length_supported",
            "hg_propagate", "hg_gs_iterate", "hg_gs_iterate_window", "hg_gs_iterate_noalloc", "hg_workspace_bytes_batched", "hg_gs_iterate_batched",
            "hg_multiplane_workspace_bytes", "hg_gs_multiplane",
            "hg_multiplane_workspace_bytes_batched", "hg_gs_multiplane_batched",
            "hg_ospr", "hg_ospr_pairs", "hg_search_workspace_bytes", "hg_pixel_search",
            "hg_grad_workspace_bytes", "hg_grad", "hg_grad_adam",
            "hg_grad_workspace_bytes_batched", "hg_grad_batched", "hg_grad_adam_batched",
            "hg_timing_begin", "hg_timing_end", "hg_error")


class hg_plan_desc(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("propagation", ctypes.c_int32),
                ("wavelength", ctypes.c_double), ("pixel_pitch", ctypes.c_double),
                ("distance", ctypes.c_double),
                ("modulation", ctypes.c_int32), ("levels", ctypes.c_int32)]


class HologenError(RuntimeError):
    def __init__(self, status: int, text: str):
        super().__init__(f"hologen status {status}: {text}")
        self.status = status


_lib = None


def library() -> ctypes.CDLL:
    """Load libhologen.so (once) and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2006_10509_amd.build`")
    # Load torch's HIP runtime first: libhologen.so then binds to the same
    # libamdhip64 (both carry the SONAME libamdhip64.so.7), so torch's device
    # pointers and streams are valid in library calls.  A second runtime in the
    # process would give the library its own device context and streams.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    _check_single_hip_runtime()
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.hg_plan_create.argtypes = [ctypes.POINTER(hg_plan_desc), ctypes.POINTER(vp)]
    lib.hg_plan_create.restype = i32
    lib.hg_plan_destroy.argtypes = [vp]
    lib.hg_plan_destroy.restype = i32
    lib.hg_workspace_bytes.argtypes = [vp]
    lib.hg_workspace_bytes.restype = sz
    lib.hg_length_supported.argtypes = [i32]
    lib.hg_length_supported.restype = i32
    lib.hg_propagate.argtypes = [vp, vp, vp, i32, vp, vp]
    lib.hg_propagate.restype = i32
    lib.hg_gs_iterate.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, vp]
    lib.hg_gs_iterate.restype = i32
    lib.hg_gs_iterate_window.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, vp, vp]
    lib.hg_gs_iterate_window.restype = i32
    lib.hg_gs_iterate_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp]
    lib.hg_gs_iterate_noalloc.restype = i32
    lib.hg_workspace_bytes_batched.argtypes = [vp, i32]
    lib.hg_workspace_bytes_batched.restype = sz
    lib.hg_gs_iterate_batched.argtypes = [vp, i32, vp, vp, vp, vp, vp, i32, vp, vp]
    lib.hg_gs_iterate_batched.restype = i32
    lib.hg_ospr.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.hg_ospr.restype = i32
    lib.hg_ospr_pairs.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.hg_ospr_pairs.restype = i32
    lib.hg_multiplane_workspace_bytes.argtypes = [vp, i32]
    lib.hg_multiplane_workspace_bytes.restype = sz
    lib.hg_gs_multiplane.argtypes = [ctypes.POINTER(vp), i32, vp, vp, vp, vp, vp, i32, vp, vp]
    lib.hg_gs_multiplane.restype = i32
    lib.hg_multiplane_workspace_bytes_batched.argtypes = [vp, i32, i32]
    lib.hg_multiplane_workspace_bytes_batched.restype = sz
    lib.hg_gs_multiplane_batched.argtypes = [ctypes.POINTER(vp), i32, i32, vp, vp, vp, vp, vp, i32, vp, vp]
    lib.hg_gs_multiplane_batched.restype = i32
    lib.hg_search_workspace_bytes.argtypes = [vp]
    lib.hg_search_workspace_bytes.restype = sz
    lib.hg_pixel_search.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]
    lib.hg_pixel_search.restype = i32
    lib.hg_grad_workspace_bytes.argtypes = [vp, i32]
    lib.hg_grad_workspace_bytes.restype = sz
    lib.hg_grad.argtypes = [ctypes.POINTER(vp), i32, vp, vp, vp, vp, vp, vp]
    lib.hg_grad.restype = i32
    f32 = ctypes.c_float
    lib.hg_grad_adam.argtypes = [ctypes.POINTER(vp), i32, vp, vp, vp, vp, i32, i32, f32, f32, f32, f32,
                                 vp, vp, vp]
    lib.hg_grad_adam.restype = i32
    lib.hg_grad_workspace_bytes_batched.argtypes = [vp, i32, i32]
    lib.hg_grad_workspace_bytes_batched.restype = sz
    lib.hg_grad_batched.argtypes = [ctypes.POINTER(vp), i32, i32, vp, vp, vp, vp, vp, vp]
    lib.hg_grad_batched.restype = i32
    lib.hg_grad_adam_batched.argtypes = [ctypes.POINTER(vp), i32, i32, vp, vp, vp, vp, i32, i32, f32, f32, f32,
                                         f32, vp, vp, vp]
    lib.hg_grad_adam_batched.restype = i32
    lib.hg_timing_begin.argtypes = [vp, i32, i32]
    lib.hg_timing_begin.restype = i32
    lib.hg_timing_end.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.hg_timing_end.restype = i32
    lib.hg_error.argtypes = [i32]
    lib.hg_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check_single_hip_runtime() -> None:
    try:
        with open("/proc/self/maps") as f:
            paths = {line.split()[-1] for line in f if "libamdhip64" in line}
    except OSError:
        return
    real = {os.path.realpath(p) for p in paths}
    if len(real) > 1:
        raise RuntimeError(f"two HIP runtimes are loaded in this process: {sorted(real)}")


def hg_error(status: int) -> str:
    return library().hg_error(status).decode()


def _check(status: int) -> None:
    if status != HG_OK:
        raise HologenError(status, hg_error(status))


def hg_length_supported(n: int) -> bool:
    return bool(library().hg_length_supported(n))


# ---------------------------------------------------------------------------
# tensor marshalling
# ---------------------------------------------------------------------------

def _ptr(t, dtype=None, shape=None, name="tensor", optional=False) -> Optional[int]:
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


@dataclass
class Plan:
    """Owns an hg_plan; mirrors hg_plan_desc."""
    width: int
    height: int
    propagation: int = HG_FOURIER
    wavelength: float = 0.0
    pixel_pitch: float = 0.0
    distance: float = 0.0
    modulation: int = HG_PHASE
    levels: int = 0

    def __post_init__(self):
        self._handle = hg_plan_create(self)

    @property
    def handle(self) -> int:
        if self._handle is None:
            raise RuntimeError("plan destroyed")
        return self._handle

    def desc(self) -> hg_plan_desc:
        return hg_plan_desc(self.width, self.height, self.propagation, self.wavelength,
                            self.pixel_pitch, self.distance, self.modulation, self.levels)

    def workspace_bytes(self) -> int:
        return int(library().hg_workspace_bytes(self.handle))

    def workspace(self, device="cuda"):
        import torch
        return torch.empty(self.workspace_bytes(), dtype=torch.uint8, device=device)

    def destroy(self) -> None:
        if getattr(self, "_handle", None) is not None:
            library().hg_plan_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def hg_plan_create(spec) -> int:
    """Create a plan from a Plan (or anything with the hg_plan_desc fields)."""
    desc = hg_plan_desc(spec.width, spec.height, spec.propagation, spec.wavelength,
                        spec.pixel_pitch, spec.distance, spec.modulation, spec.levels)
    out = ctypes.c_void_p()
    _check(library().hg_plan_create(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def hg_propagate(plan: Plan, x, out, direction: int, workspace=None, stream=None) -> None:
    import torch
    shape = (plan.height, plan.width)
    _check(library().hg_propagate(plan.handle, _ptr(x, torch.complex64, shape, "in"),
                                  _ptr(out, torch.complex64, shape, "out"), direction,
                                  _ptr(workspace, torch.uint8, None, "workspace", optional=True),
                                  _stream(stream)))


def hg_gs_iterate(plan: Plan, target_amp, phase, iterations: int, workspace,
                  illumination=None, levels=None, nmse=None, stream=None) -> None:
    """In-place GS: ``phase`` holds the starting phase on entry, the result on exit."""
    import torch
    shape = (plan.height, plan.width)
    _check(library().hg_gs_iterate(
        plan.handle, _ptr(target_amp, torch.float32, shape, "target_amp"),
        _ptr(illumination, torch.float32, shape, "illumination", optional=True),
        _ptr(phase, torch.float32, shape, "phase"),
        _ptr(levels, torch.uint8, shape, "levels", optional=True),
        _ptr(nmse, torch.float32, (iterations + 1,), "nmse", optional=True),
        int(iterations), _workspace(workspace, plan.workspace_bytes()), _stream(stream)))


def hg_gs_iterate_window(plan: Plan, target_amp, window, phase, iterations: int, workspace,
                         illumination=None, levels=None, nmse=None, stream=None) -> None:
    """Signal-window GS: ``window`` [H, W] uint8, centred like the target,
    nonzero inside; ``phase`` in place as in hg_gs_iterate."""
    import torch
    shape = (plan.height, plan.width)
    _check(library().hg_gs_iterate_window(
        plan.handle, _ptr(target_amp, torch.float32, shape, "target_amp"),
        _ptr(window, torch.uint8, shape, "window"),
        _ptr(illumination, torch.float32, shape, "illumination", optional=True),
        _ptr(phase, torch.float32, shape, "phase"),
        _ptr(levels, torch.uint8, shape, "levels", optional=True),
        _ptr(nmse, torch.float32, (iterations + 1,), "nmse", optional=True),
        int(iterations), _workspace(workspace, plan.workspace_bytes()), _stream(stream)))


# bytes of the static device workspace hg_gs_iterate_noalloc uses (hologen.h)
HG_NOALLOC_WORKSPACE_MAX = 64 << 20


def hg_gs_iterate_noalloc(plan: Plan, target_amp, phase, iterations: int,
                          illumination=None, levels=None, nmse=None, stream=None) -> None:
    """hg_gs_iterate with the library's static per-device workspace: no
    allocation in the call.  Calls on one device share that workspace, so
    overlapping calls race."""
    import torch
    shape = (plan.height, plan.width)
    _check(library().hg_gs_iterate_noalloc(
        plan.handle, _ptr(target_amp, torch.float32, shape, "target_amp"),
        _ptr(illumination, torch.float32, shape, "illumination", optional=True),
        _ptr(phase, torch.float32, shape, "phase"),
        _ptr(levels, torch.uint8, shape, "levels", optional=True),
        _ptr(nmse, torch.float32, (iterations + 1,), "nmse", optional=True),
        int(iterations), _stream(stream)))


def hg_ospr_pairs(plan: Plan, target_amp, sub_phase, intensity, workspace, holograms=None,
                  nmse=None, stream=None) -> None:
    """OSPR with two subframes (Re and Im) per inverse transform; holograms is
    [2 n_pairs, H, W] or None."""
    import torch
    shape = (plan.height, plan.width)
    n_pairs = int(sub_phase.shape[0])
    _check(library().hg_ospr_pairs(
        plan.handle, _ptr(target_amp, torch.float32, shape, "target_amp"),
        _ptr(sub_phase, torch.float32, (n_pairs,) + shape, "sub_phase"), n_pairs,
        _ptr(holograms, torch.uint8, (2 * n_pairs,) + shape, "holograms", optional=True),
        _ptr(intensity, torch.float32, shape, "intensity"),
        _ptr(nmse, torch.float32, (1,), "nmse", optional=True),
        _workspace(workspace, plan.workspace_bytes()), _stream(stream)))


def multiplane_workspace(planes, device="cuda"):
    import torch
    planes, _ = _plans(planes)
    n = int(library().hg_multiplane_workspace_bytes(planes[0].handle, len(planes)))
    return torch.empty(n, dtype=torch.uint8, device=device)


def hg_gs_multiplane(planes, target_amp, phase, iterations: int, workspace, illumination=None, levels=None,
                     nmse=None, stream=None) -> None:
    """Multi-plane GS, one plane after another; target_amp is [n_planes, H, W]."""
    import torch
    planes, arr = _plans(planes)
    P = len(planes)
    shape = (planes[0].height, planes[0].width)
    need = int(library().hg_multiplane_workspace_bytes(planes[0].handle, P))
    _check(library().hg_gs_multiplane(
        arr, P, _ptr(target_amp, torch.float32, (P,) + shape, "target_amp"),
        _ptr(illumination, torch.float32, shape, "illumination", optional=True),
        _ptr(phase, torch.float32, shape, "phase"), _ptr(levels, torch.uint8, shape, "levels", optional=True),
        _ptr(nmse, torch.float32, (iterations * P + P,), "nmse", optional=True), int(iterations),
        _workspace(workspace, need), _stream(stream)))


def multiplane_workspace_batched(planes, batch: int, device="cuda"):
    import torch
    planes, _ = _plans(planes)
    n = int(library().hg_multiplane_workspace_bytes_batched(planes[0].handle, len(planes), int(batch)))
    return torch.empty(n, dtype=torch.uint8, device=device)


def hg_gs_multiplane_batched(planes, target_amp, phase, iterations: int, workspace, illumination=None,
                             levels=None, nmse=None, stream=None) -> None:
    """Multi-plane GS on a batch of problems: target_amp [batch, n_planes, H, W],
    phase and levels [batch, H, W], nmse [batch, iterations * n_planes + n_planes]."""
    import torch
    planes, arr = _plans(planes)
    P = len(planes)
    batch = int(phase.shape[0])
    shape = (planes[0].height, planes[0].width)
    need = int(library().hg_multiplane_workspace_bytes_batched(planes[0].handle, P, batch))
    _check(library().hg_gs_multiplane_batched(
        arr, P, batch, _ptr(target_amp, torch.float32, (batch, P) + shape, "target_amp"),
        _ptr(illumination, torch.float32, shape, "illumination", optional=True),
        _ptr(phase, torch.float32, (batch,) + shape, "phase"),
        _ptr(levels, torch.uint8, (batch,) + shape, "levels", optional=True),
        _ptr(nmse, torch.float32, (batch, iterations * P + P), "nmse", optional=True), int(iterations),
        _workspace(workspace, need), _stream(stream)))


def search_workspace(plan: Plan, device="cuda"):
    import torch
    return torch.empty(int(library().hg_search_workspace_bytes(plan.handle)), dtype=torch.uint8, device=device)


def hg_pixel_search(plan: Plan, target_amp, levels, trials, workspace, temperature=None, uniform=None,
                    accepted=None, nmse=None, stream=None) -> None:
    """Direct binary search (temperature None) or simulated annealing over the
    [n, 2] int32 trial list (pixel index, candidate level); ``levels`` is
    updated in place."""
    import torch
    shape = (plan.height, plan.width)
    n = int(trials.shape[0])
    _check(library().hg_pixel_search(
        plan.handle, _ptr(target_amp, torch.float32, shape, "target_amp"),
        _ptr(levels, torch.uint8, shape, "levels"), _ptr(trials, torch.int32, (n, 2), "trials"), n,
        _ptr(temperature, torch.float32, (n,), "temperature", optional=True),
        _ptr(uniform, torch.float32, (n,), "uniform", optional=True),
        _ptr(accepted, torch.uint8, (n,), "accepted", optional=True),
        _ptr(nmse, torch.float32, (n + 1,), "nmse", optional=True),
        _workspace(workspace, int(library().hg_search_workspace_bytes(plan.handle))), _stream(stream)))


def workspace_bytes_batched(plan: Plan, batch: int) -> int:
    return int(library().hg_workspace_bytes_batched(plan.handle, batch))


def hg_gs_iterate_batched(plan: Plan, target_amp, phase, iterations: int, workspace,
                          illumination=None, levels=None, nmse=None, stream=None) -> None:
    """GS on a [batch, H, W] stack of same-shape holograms, one launch per pass."""
    import torch
    batch = int(phase.shape[0])
    shape = (batch, plan.height, plan.width)
    _check(library().hg_gs_iterate_batched(
        plan.handle, batch, _ptr(target_amp, torch.float32, shape, "target_amp"),
        _ptr(illumination, torch.float32, shape[1:], "illumination", optional=True),
        _ptr(phase, torch.float32, shape, "phase"),
        _ptr(levels, torch.uint8, shape, "levels", optional=True),
        _ptr(nmse, torch.float32, (batch, iterations + 1), "nmse", optional=True),
        int(iterations), _workspace(workspace, workspace_bytes_batched(plan, batch)), _stream(stream)))


def hg_ospr(plan: Plan, target_amp, sub_phase, intensity, workspace, holograms=None,
            nmse=None, stream=None) -> None:
    import torch
    shape = (plan.height, plan.width)
    n_sub = int(sub_phase.shape[0])
    _check(library().hg_ospr(
        plan.handle, _ptr(target_amp, torch.float32, shape, "target_amp"),
        _ptr(sub_phase, torch.float32, (n_sub,) + shape, "sub_phase"), n_sub,
        _ptr(holograms, torch.uint8, (n_sub,) + shape, "holograms", optional=True),
        _ptr(intensity, torch.float32, shape, "intensity"),
        _ptr(nmse, torch.float32, (1,), "nmse", optional=True),
        _workspace(workspace, plan.workspace_bytes()), _stream(stream)))


def _workspace(ws, need: int, name: str = "workspace") -> int:
    import torch
    ptr = _ptr(ws, torch.uint8, None, name)
    if ws.numel() < need:
        raise ValueError(f"{name} has {ws.numel()} bytes, the call needs {need}")
    return ptr


def _plans(planes):
    planes = list(planes)
    if not planes:
        raise ValueError("at least one plane is required")
    return planes, (ctypes.c_void_p * len(planes))(*[p.handle for p in planes])


def grad_workspace_bytes(planes) -> int:
    planes, _ = _plans(planes)
    return int(library().hg_grad_workspace_bytes(planes[0].handle, len(planes)))


def grad_workspace(planes, device="cuda"):
    import torch
    return torch.empty(grad_workspace_bytes(planes), dtype=torch.uint8, device=device)


def hg_grad(planes, target_amp, phase, workspace, grad=None, loss=None, stream=None) -> None:
    """Loss and/or dL/dphi of the multi-plane NMSE at ``phase`` (read only).
    ``target_amp`` is [n_planes, H, W] (centred amplitudes), one per plan."""
    import torch
    planes, arr = _plans(planes)
    shape = (planes[0].height, planes[0].width)
    _check(library().hg_grad(
        arr, len(planes), _ptr(target_amp, torch.float32, (len(planes),) + shape, "target_amp"),
        _ptr(phase, torch.float32, shape, "phase"), _ptr(grad, torch.float32, shape, "grad", optional=True),
        _ptr(loss, torch.float32, (1,), "loss", optional=True),
        _workspace(workspace, grad_workspace_bytes(planes)), _stream(stream)))


def hg_grad_adam(planes, target_amp, phase, adam_m, adam_v, steps: int, workspace, first_step: int = 1,
                 lr: float = 0.05, betas=(0.9, 0.999), eps: float = 1e-8, loss=None, stream=None) -> None:
    """``steps`` Adam steps on ``phase`` in place; ``loss`` [steps + 1] or None."""
    import torch
    planes, arr = _plans(planes)
    shape = (planes[0].height, planes[0].width)
    _check(library().hg_grad_adam(
        arr, len(planes), _ptr(target_amp, torch.float32, (len(planes),) + shape, "target_amp"),
        _ptr(phase, torch.float32, shape, "phase"), _ptr(adam_m, torch.float32, shape, "adam_m"),
        _ptr(adam_v, torch.float32, shape, "adam_v"), int(steps), int(first_step), float(lr),
        float(betas[0]), float(betas[1]), float(eps),
        _ptr(loss, torch.float32, (int(steps) + 1,), "loss", optional=True),
        _workspace(workspace, grad_workspace_bytes(planes)), _stream(stream)))


def grad_workspace_bytes_batched(planes, batch: int) -> int:
    planes, _ = _plans(planes)
    return int(library().hg_grad_workspace_bytes_batched(planes[0].handle, len(planes), int(batch)))


def grad_workspace_batched(planes, batch: int, device="cuda"):
    import torch
    return torch.empty(grad_workspace_bytes_batched(planes, batch), dtype=torch.uint8, device=device)


def hg_grad_batched(planes, target_amp, phase, workspace, grad=None, loss=None, stream=None) -> None:
    """hg_grad on a batch: ``target_amp`` [B, n_planes, H, W], ``phase`` and
    ``grad`` [B, H, W], ``loss`` [B]."""
    import torch
    planes, arr = _plans(planes)
    shape = (planes[0].height, planes[0].width)
    b = int(phase.shape[0]) if phase is not None and phase.dim() == 3 else -1
    _check(library().hg_grad_batched(
        arr, len(planes), b, _ptr(target_amp, torch.float32, (b, len(planes)) + shape, "target_amp"),
        _ptr(phase, torch.float32, (b,) + shape, "phase"),
        _ptr(grad, torch.float32, (b,) + shape, "grad", optional=True),
        _ptr(loss, torch.float32, (b,), "loss", optional=True),
        _workspace(workspace, grad_workspace_bytes_batched(planes, max(b, 1))), _stream(stream)))


def hg_grad_adam_batched(planes, target_amp, phase, adam_m, adam_v, steps: int, workspace, first_step: int = 1,
                         lr: float = 0.05, betas=(0.9, 0.999), eps: float = 1e-8, loss=None, stream=None) -> None:
    """hg_grad_adam on a batch: ``target_amp`` [B, n_planes, H, W], ``phase``,
    ``adam_m``, ``adam_v`` [B, H, W], ``loss`` [B, steps + 1] or None."""
    import torch
    planes, arr = _plans(planes)
    shape = (planes[0].height, planes[0].width)
    b = int(phase.shape[0]) if phase is not None and phase.dim() == 3 else -1
    _check(library().hg_grad_adam_batched(
        arr, len(planes), b, _ptr(target_amp, torch.float32, (b, len(planes)) + shape, "target_amp"),
        _ptr(phase, torch.float32, (b,) + shape, "phase"), _ptr(adam_m, torch.float32, (b,) + shape, "adam_m"),
        _ptr(adam_v, torch.float32, (b,) + shape, "adam_v"), int(steps), int(first_step), float(lr),
        float(betas[0]), float(betas[1]), float(eps),
        _ptr(loss, torch.float32, (b, int(steps) + 1), "loss", optional=True),
        _workspace(workspace, grad_workspace_bytes_batched(planes, max(b, 1))), _stream(stream)))


_LOSS_FN = None


def hologram_loss(phase, target_amp, planes, workspace=None):
    """Differentiable multi-plane NMSE loss L(phase) as a 0-dim tensor.

    A torch.autograd.Function over hg_grad: when ``phase`` requires a gradient
    the forward call also runs the adjoint passes (the field is recomputed
    from the phase inside them, never stored) and keeps only dL/dphase for
    the backward call."""
    global _LOSS_FN
    import torch
    if _LOSS_FN is None:
        class _HologramLoss(torch.autograd.Function):
            @staticmethod
            def forward(ctx, phi, target, plane_list, ws):
                loss = torch.empty(1, dtype=torch.float32, device=phi.device)
                if ctx.needs_input_grad[0]:
                    grad = torch.empty_like(phi)
                    hg_grad(plane_list, target, phi.detach().contiguous(), ws, grad=grad, loss=loss)
                    ctx.save_for_backward(grad)
                else:
                    hg_grad(plane_list, target, phi.detach().contiguous(), ws, loss=loss)
                return loss[0]

            @staticmethod
            def backward(ctx, g):
                (grad,) = ctx.saved_tensors
                return g * grad, None, None, None

        _LOSS_FN = _HologramLoss
    if workspace is None:
        workspace = grad_workspace(planes, device=phase.device)
    return _LOSS_FN.apply(phase, target_amp, list(planes), workspace)


def hg_timing_begin(plan: Plan, kernel: int, repeats: int = 1) -> None:
    _check(library().hg_timing_begin(plan.handle, kernel, repeats))


def hg_timing_end(plan: Plan):
    """(summed kernel milliseconds, number of kernel executions timed)."""
    total = ctypes.c_double()
    count = ctypes.c_int64()
    _check(library().hg_timing_end(plan.handle, ctypes.byref(total), ctypes.byref(count)))
    return total.value, count.value
