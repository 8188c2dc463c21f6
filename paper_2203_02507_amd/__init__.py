"""Python binding of libfpm (include/fpm.h): argument marshalling only.

Every step of the reconstruction runs in the HIP library; this module turns
torch tensors (device memory, streams) or numpy arrays (host memory) into
plain pointers and sizes.  Importing it loads ``libfpm.so`` built in-tree by
``paper_2203_02507_amd/build.py``; if the library is missing the import
fails -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

try:  # torch first: libfpm then binds to the HIP runtime torch already loaded
    import torch
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfpm.so")

FPM_OK, FPM_PENDING = 0, 1
FPM_E_ARG, FPM_E_GEOMETRY, FPM_E_NOMEM, FPM_E_DEVICE = -1, -2, -3, -4
FPM_E_DIVERGED, FPM_E_CANCELLED, FPM_E_UNSUPPORTED, FPM_E_STATE = -5, -6, -7, -8
FPM_MEM_HOST, FPM_MEM_DEVICE = 0, 1
FPM_SCHED_SEQUENTIAL, FPM_SCHED_LED_GROUPS, FPM_SCHED_GROUP_ORDER, FPM_SCHED_PIPELINED = 0, 1, 2, 3
FPM_PREC_FP32_FFT, FPM_PREC_MFMA_BF16X3, FPM_PREC_MFMA_FP16 = 0, 1, 2

STATUS_NAMES = {0: "FPM_OK", 1: "FPM_PENDING", -1: "FPM_E_ARG", -2: "FPM_E_GEOMETRY",
                -3: "FPM_E_NOMEM", -4: "FPM_E_DEVICE", -5: "FPM_E_DIVERGED",
                -6: "FPM_E_CANCELLED", -7: "FPM_E_UNSUPPORTED", -8: "FPM_E_STATE"}

# every entry point declared in include/fpm.h
EXPORTS = ("fpm_plan", "fpm_plan_destroy", "fpm_plan_tile_info", "fpm_plan_tables",
           "fpm_plan_device_bytes", "fpm_forward", "fpm_reconstruct", "fpm_server_create",
           "fpm_server_destroy", "fpm_submit", "fpm_poll", "fpm_wait", "fpm_cancel",
           "fpm_last_error", "fpm_version", "fpm_profile_reconstruct", "fpm_stitch",
           "fpm_stitch_noalloc", "fpm_estimate_defocus", "fpm_plan_status",
           "fpm_online_begin", "fpm_online_push", "fpm_online_finish", "fpm_online_abort")


class FpmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class TileDescC(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("upsample", C.c_int32),
        ("led_rows", C.c_int32), ("led_cols", C.c_int32),
        ("led_pitch_um", C.c_double), ("led_height_um", C.c_double),
        ("led_origin_x_um", C.c_double), ("led_origin_y_um", C.c_double),
        ("wavelength_um", C.c_double), ("na_obj", C.c_double), ("pixel_um", C.c_double),
        ("tile_x_um", C.c_double), ("tile_y_um", C.c_double), ("defocus_um", C.c_double),
        ("iterations", C.c_int32), ("pupil_update", C.c_int32),
        ("precision", C.c_int32), ("schedule", C.c_int32),
    ]


class TileInfoC(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("N", C.c_int32), ("L", C.c_int32),
        ("support_count", C.c_int32), ("ngroups", C.c_int32), ("max_group", C.c_int32),
        ("steps", C.c_int32), ("iterations", C.c_int32),
        ("min_tie_distance", C.c_double),
        ("intensity_offset", C.c_int64), ("object_offset", C.c_int64),
        ("pupil_offset", C.c_int64), ("residual_offset", C.c_int64),
        ("levels", C.c_int32), ("reserved", C.c_int32),
    ]


class KernelTimeC(C.Structure):
    _fields_ = [("launches", C.c_int32), ("pad", C.c_int32), ("items", C.c_int64),
                ("total_ms", C.c_double), ("busy_ms", C.c_double)]


KERNEL_KINDS = ("update", "pupil_mean", "iter_end", "spec_max", "init")


class RequestStatsC(C.Structure):
    _fields_ = [("submit_s", C.c_double), ("admit_s", C.c_double), ("finish_s", C.c_double),
                ("updates", C.c_int64), ("status", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2203_02507_amd/build.py "
                          "(or __graft_entry__.build()) first")
    L = C.CDLL(LIB_PATH)
    vp, ip, dp = C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)
    L.fpm_plan.argtypes = [C.POINTER(TileDescC), C.c_int32, C.POINTER(vp)]
    L.fpm_plan.restype = C.c_int
    L.fpm_plan_destroy.argtypes = [vp]
    L.fpm_plan_destroy.restype = None
    L.fpm_plan_tile_info.argtypes = [vp, C.c_int32, C.POINTER(TileInfoC)]
    L.fpm_plan_tile_info.restype = C.c_int
    L.fpm_plan_tables.argtypes = [vp, C.c_int32, ip, ip, ip, ip]
    L.fpm_plan_tables.restype = C.c_int
    L.fpm_plan_device_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.fpm_plan_device_bytes.restype = C.c_int
    L.fpm_forward.argtypes = [vp, vp, vp, vp, C.c_int, vp]
    L.fpm_forward.restype = C.c_int
    L.fpm_reconstruct.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp]
    L.fpm_reconstruct.restype = C.c_int
    L.fpm_server_create.argtypes = [C.c_size_t, C.c_int32, C.POINTER(vp)]
    L.fpm_server_create.restype = C.c_int
    L.fpm_server_destroy.argtypes = [vp]
    L.fpm_server_destroy.restype = None
    L.fpm_submit.argtypes = [vp, C.POINTER(TileDescC), vp, C.c_int, C.POINTER(C.c_uint64)]
    L.fpm_submit.restype = C.c_int
    L.fpm_poll.argtypes = [vp, C.c_uint64, vp, vp, vp, C.POINTER(RequestStatsC)]
    L.fpm_poll.restype = C.c_int
    L.fpm_wait.argtypes = [vp, C.c_uint64, C.c_double, vp, vp, vp, C.POINTER(RequestStatsC)]
    L.fpm_wait.restype = C.c_int
    L.fpm_cancel.argtypes = [vp, C.c_uint64]
    L.fpm_cancel.restype = C.c_int
    L.fpm_profile_reconstruct.argtypes = [vp, vp, C.POINTER(KernelTimeC), vp]
    L.fpm_profile_reconstruct.restype = C.c_int
    L.fpm_stitch.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, C.c_int, vp]
    L.fpm_stitch.restype = C.c_int
    L.fpm_stitch_noalloc.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp]
    L.fpm_stitch_noalloc.restype = C.c_int
    L.fpm_estimate_defocus.argtypes = [C.POINTER(TileDescC), C.c_int32, vp, C.c_int, C.c_double,
                                       C.c_double, C.c_double, C.c_int32, vp, vp, C.c_int32, vp]
    L.fpm_estimate_defocus.restype = C.c_int
    L.fpm_plan_status.argtypes = [vp, C.POINTER(C.c_int)]
    L.fpm_plan_status.restype = C.c_int
    L.fpm_online_begin.argtypes = [vp, vp]
    L.fpm_online_begin.restype = C.c_int
    L.fpm_online_push.argtypes = [vp, C.c_int32, vp, C.c_int, vp]
    L.fpm_online_push.restype = C.c_int
    L.fpm_online_finish.argtypes = [vp, C.c_int, vp, vp, vp, vp]
    L.fpm_online_finish.restype = C.c_int
    L.fpm_online_abort.argtypes = [vp]
    L.fpm_online_abort.restype = C.c_int
    L.fpm_last_error.argtypes = []
    L.fpm_last_error.restype = C.c_char_p
    L.fpm_version.argtypes = []
    L.fpm_version.restype = C.c_char_p
    return L


lib = _load()


def last_error() -> str:
    return lib.fpm_last_error().decode(errors="replace")


def check(status: int) -> int:
    if status not in (FPM_OK, FPM_PENDING):
        raise FpmError(status, last_error())
    return status


def to_c_desc(d) -> TileDescC:
    """Fill the C descriptor from any object with TileDesc's field names."""
    c = TileDescC()
    for name, _ in TileDescC._fields_:
        setattr(c, name, getattr(d, name))
    return c


# ------------------------------------------------------------ marshalling

def _ptr(x, where: int):
    """Pointer of a torch tensor (device) or numpy array (host); None -> NULL."""
    if x is None:
        return None
    if torch is not None and isinstance(x, torch.Tensor):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if (where == FPM_MEM_DEVICE) != x.is_cuda:
            raise ValueError("tensor placement does not match `where`")
        return C.c_void_p(x.data_ptr())
    if isinstance(x, np.ndarray):
        if where != FPM_MEM_HOST:
            raise ValueError("numpy arrays are host memory; use where=FPM_MEM_HOST")
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return C.c_void_p(x.ctypes.data)
    raise TypeError(f"unsupported buffer type {type(x)}")


# element size and accepted dtypes of the C buffer kinds; a complex64 buffer
# may also be a float32 array of interleaved (re, im) pairs
_KIND_BYTES = {"f32": 4, "c64": 8, "f64": 8}
_KIND_NP = {"f32": ("float32",), "c64": ("complex64", "float32"), "f64": ("float64",)}


def _buf(x, where: int, kind: str, count: int, what: str):
    """_ptr, after checking that `x` holds at least `count` elements of the
    C type `kind`: the library writes and reads exactly that many, so a
    short or mistyped buffer is refused here, before any call is made."""
    p = _ptr(x, where)
    if p is None:
        return None
    if torch is not None and isinstance(x, torch.Tensor):
        dt, nbytes = str(x.dtype).replace("torch.", ""), x.numel() * x.element_size()
    else:
        dt, nbytes = str(x.dtype), x.nbytes
    if dt not in _KIND_NP[kind]:
        raise TypeError(f"{what}: dtype {dt}, expected {' or '.join(_KIND_NP[kind])}")
    need = int(count) * _KIND_BYTES[kind]
    if nbytes < need:
        raise ValueError(f"{what}: {nbytes} bytes, needs at least {need}")
    return p


def _stream(stream):
    if stream is None:
        if torch is not None and torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        return None
    if torch is not None and isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


# ---------------------------------------------------------- entry points

@dataclass
class TileInfo:
    n: int
    N: int
    L: int
    support_count: int
    ngroups: int
    max_group: int
    steps: int
    iterations: int
    min_tie_distance: float
    intensity_offset: int
    object_offset: int
    pupil_offset: int
    residual_offset: int
    levels: int


class Plan:
    """Owner of an ``fpm_plan_t``; destroyed with the object."""

    def __init__(self, descs: Sequence):
        arr = (TileDescC * len(descs))(*[to_c_desc(d) for d in descs])
        h = C.c_void_p()
        check(lib.fpm_plan(arr, len(descs), C.byref(h)))
        self._h = h
        self.ntiles = len(descs)
        self.infos = [self.tile_info(t) for t in range(self.ntiles)]
        self.total_intensity = sum(i.L * i.n * i.n for i in self.infos)
        self.total_object = sum(i.N * i.N for i in self.infos)
        self.total_pupil = sum(i.n * i.n for i in self.infos)
        self.total_residual = sum(i.iterations for i in self.infos)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.fpm_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass

    def tile_info(self, t: int) -> TileInfo:
        info = TileInfoC()
        check(lib.fpm_plan_tile_info(self._h, t, C.byref(info)))
        return TileInfo(**{k: getattr(info, k) for k, _ in TileInfoC._fields_
                           if k != "reserved"})

    def tables(self, t: int):
        L = self.infos[t].L
        off = np.zeros((L, 2), np.int32)
        order = np.zeros(L, np.int32)
        gof = np.zeros(L, np.int32)
        sweep = np.zeros(L, np.int32)
        ip = C.POINTER(C.c_int32)
        check(lib.fpm_plan_tables(self._h, t, off.ctypes.data_as(ip), order.ctypes.data_as(ip),
                                  gof.ctypes.data_as(ip), sweep.ctypes.data_as(ip)))
        return off, order, gof, sweep

    def device_bytes(self) -> int:
        b = C.c_size_t()
        check(lib.fpm_plan_device_bytes(self._h, C.byref(b)))
        return b.value


def fpm_plan(descs: Sequence) -> Plan:
    return Plan(descs)


def fpm_forward(plan: Plan, obj, pupil, intensity, where: int, stream=None) -> int:
    return check(lib.fpm_forward(plan.handle, _buf(obj, where, "c64", plan.total_object, "object"),
                                 _buf(pupil, where, "c64", plan.total_pupil, "pupil"),
                                 _buf(intensity, where, "f32", plan.total_intensity, "intensity"),
                                 where, _stream(stream)))


def fpm_reconstruct(plan: Plan, intensity, where: int, object_out=None, pupil_out=None,
                    residual_out=None, stream=None) -> int:
    return check(lib.fpm_reconstruct(
        plan.handle, _buf(intensity, where, "f32", plan.total_intensity, "intensity"), where,
        _buf(object_out, where, "c64", plan.total_object, "object_out"),
        _buf(pupil_out, where, "c64", plan.total_pupil, "pupil_out"),
        _buf(residual_out, where, "f64", plan.total_residual, "residual_out"), _stream(stream)))


def fpm_online_begin(plan: Plan, stream=None) -> int:
    """Sec. 3.4 Fig. 7a: open an online session on `plan`."""
    return check(lib.fpm_online_begin(plan.handle, _stream(stream)))


def fpm_online_push(plan: Plan, led: int, intensity, where: int, stream=None) -> int:
    """The tiles' images of LED `led`, float [tile][n][n]; runs that LED's
    update on every tile."""
    return check(lib.fpm_online_push(plan.handle, led,
                                     _buf(intensity, where, "f32", plan.total_pupil, "intensity"),
                                     where, _stream(stream)))


def fpm_online_finish(plan: Plan, where: int, object_out=None, pupil_out=None,
                      residual_out=None, stream=None) -> int:
    return check(lib.fpm_online_finish(
        plan.handle, where, _buf(object_out, where, "c64", plan.total_object, "object_out"),
        _buf(pupil_out, where, "c64", plan.total_pupil, "pupil_out"),
        _buf(residual_out, where, "f64", plan.total_residual, "residual_out"), _stream(stream)))


def fpm_online_abort(plan: Plan) -> int:
    return check(lib.fpm_online_abort(plan.handle))


def fpm_profile_reconstruct(plan: Plan, intensity, stream=None) -> dict:
    """Per-kind kernel time of one eager reconstruction sweep (HIP events
    around every launch, chains concurrent): launches, items, summed launch
    durations and the union of the launch intervals."""
    out = (KernelTimeC * len(KERNEL_KINDS))()
    check(lib.fpm_profile_reconstruct(
        plan.handle, _buf(intensity, FPM_MEM_DEVICE, "f32", plan.total_intensity, "intensity"),
        out, _stream(stream)))
    return {name: {"launches": out[i].launches, "items": out[i].items,
                   "total_ms": out[i].total_ms, "busy_ms": out[i].busy_ms}
            for i, name in enumerate(KERNEL_KINDS)}


def fpm_plan_status(plan: "Plan") -> int:
    """Outcome of the plan's last device-mode call (FPM_OK, FPM_E_ARG or
    FPM_E_DIVERGED), once its work has run."""
    st = C.c_int(0)
    check(lib.fpm_plan_status(plan.handle, C.byref(st)))
    return st.value


def fpm_stitch(tiles, rows: int, cols: int, side: int, overlap: int, out, where: int,
               stream=None) -> int:
    """Sec. 3.1 Eq. (1): tiles complex64 [rows][cols][side][side] -> out
    complex64 [H][W] (see include/fpm.h)."""
    # sizes are checked for a geometry the library accepts; it rejects the rest itself
    ok = rows > 0 and cols > 0 and side > 0 and 0 <= overlap < side
    H, W = stitched_shape(rows, cols, side, overlap) if ok else (0, 0)
    count = rows * cols * side * side if ok else 0
    return check(lib.fpm_stitch(_buf(tiles, where, "c64", count, "tiles"), rows, cols, side,
                                overlap, _buf(out, where, "c64", H * W, "out"),
                                where, _stream(stream)))


def fpm_stitch_noalloc(tiles, rows: int, cols: int, side: int, overlap: int, out,
                       stream=None) -> int:
    """fpm_stitch on device buffers with the library's fixed scratch (no
    allocation; at most 4096 tiles; returns once enqueued on `stream`)."""
    ok = rows > 0 and cols > 0 and side > 0 and 0 <= overlap < side
    H, W = stitched_shape(rows, cols, side, overlap) if ok else (0, 0)
    count = rows * cols * side * side if ok else 0
    return check(lib.fpm_stitch_noalloc(
        _buf(tiles, FPM_MEM_DEVICE, "c64", count, "tiles"), rows, cols, side, overlap,
        _buf(out, FPM_MEM_DEVICE, "c64", H * W, "out"), _stream(stream)))


def defocus_candidates(z_lo: float, z_hi: float, z_step: float) -> int:
    """Number of candidate z values fpm_estimate_defocus scores."""
    return int(np.floor((z_hi - z_lo) / z_step + 1e-6)) + 1 if z_step > 0 and z_hi >= z_lo else 0


def fpm_estimate_defocus(descs, intensity, where: int, z_lo: float = -40.0, z_hi: float = 40.0,
                         z_step: float = 5.0, iterations: int = 10, stream=None):
    """Sec. 3.4 Fig. 7b: defocus distance of each tile from its bright-field
    images (see include/fpm.h).  Returns (z [ntiles], scores [ntiles][K])."""
    descs = list(descs)
    arr = (TileDescC * len(descs))(*[to_c_desc(d) for d in descs])
    count = sum(d.led_rows * d.led_cols * d.n * d.n for d in descs)
    K = max(defocus_candidates(z_lo, z_hi, z_step), 1)
    z = np.zeros(len(descs), np.float64)
    scores = np.zeros((len(descs), K), np.float64)
    check(lib.fpm_estimate_defocus(arr, len(descs), _buf(intensity, where, "f32", count, "intensity"),
                                   where, float(z_lo), float(z_hi), float(z_step), int(iterations),
                                   C.c_void_p(z.ctypes.data), C.c_void_p(scores.ctypes.data), K,
                                   _stream(stream)))
    return z, scores


def stitched_shape(rows: int, cols: int, side: int, overlap: int):
    return rows * (side - overlap) + overlap, cols * (side - overlap) + overlap


def version() -> str:
    return lib.fpm_version().decode()


# ------------------------------------------------------ device helpers

def device_buffers(plan: Plan, device="cuda"):
    """Allocate torch device outputs shaped like the plan's concatenated arrays."""
    obj = torch.empty(plan.total_object * 2, dtype=torch.float32, device=device)
    pup = torch.empty(plan.total_pupil * 2, dtype=torch.float32, device=device)
    res = torch.empty(max(plan.total_residual, 1), dtype=torch.float64, device=device)
    return obj, pup, res


def split_tiles(plan: Plan, obj: np.ndarray, pup: np.ndarray, res: np.ndarray):
    """Per-tile views (complex object [N][N], complex pupil [n][n], residual)."""
    out = []
    oc = obj.view(np.complex64) if obj.dtype == np.float32 else obj
    pc = pup.view(np.complex64) if pup.dtype == np.float32 else pup
    for i in plan.infos:
        o = oc[i.object_offset:i.object_offset + i.N * i.N].reshape(i.N, i.N)
        p = pc[i.pupil_offset:i.pupil_offset + i.n * i.n].reshape(i.n, i.n)
        r = res[i.residual_offset:i.residual_offset + i.iterations]
        out.append((o, p, r))
    return out


# --------------------------------------------------------------- serving

@dataclass
class RequestStats:
    submit_s: float
    admit_s: float
    finish_s: float
    updates: int
    status: int


class Server:
    """Owner of an ``fpm_server_t`` (continuous-batching request loop)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64):
        h = C.c_void_p()
        check(lib.fpm_server_create(int(hbm_budget_bytes), int(max_slots), C.byref(h)))
        self._h = h
        self._keep = {}   # request id -> (desc, buffer) kept alive until collected

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.fpm_server_destroy(self._h)
            self._h = C.c_void_p()
        self._keep = {}

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def submit(self, desc, intensity, where: int) -> int:
        rid = C.c_uint64()
        cd = to_c_desc(desc)
        count = desc.led_rows * desc.led_cols * desc.n * desc.n
        check(lib.fpm_submit(self._h, C.byref(cd), _buf(intensity, where, "f32", count, "intensity"),
                             where, C.byref(rid)))
        self._keep[rid.value] = (cd, intensity)
        return rid.value

    def _collect(self, fn, rid, desc, *extra):
        N = desc.n * desc.upsample
        obj = np.zeros((N, N), np.complex64)
        pup = np.zeros((desc.n, desc.n), np.complex64)
        res = np.zeros(max(desc.iterations, 1), np.float64)
        st = RequestStatsC()
        status = fn(self._h, rid, *extra, C.c_void_p(obj.ctypes.data), C.c_void_p(pup.ctypes.data),
                    C.c_void_p(res.ctypes.data), C.byref(st))
        stats = RequestStats(st.submit_s, st.admit_s, st.finish_s, st.updates, st.status)
        if status == FPM_PENDING:
            return None, stats
        self._keep.pop(rid, None)
        check(status)
        return (obj, pup, res[:desc.iterations]), stats

    def poll(self, rid: int, desc):
        """(outputs, stats) once finished; (None, stats) while pending."""
        return self._collect(lib.fpm_poll, rid, desc)

    def wait(self, rid: int, desc, timeout_s: float = 600.0):
        return self._collect(lib.fpm_wait, rid, desc, C.c_double(timeout_s))

    def cancel(self, rid: int) -> None:
        check(lib.fpm_cancel(self._h, rid))
