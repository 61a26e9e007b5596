"""Python binding of libvof.so, the MI355X geometric PLIC VoF flux library.

Argument marshalling only: every step of the flux path runs in the HIP
kernels behind the C ABI declared in include/vof.h.  The functions carry the
same names as the C entry points.  Arrays may be NumPy arrays (host memory)
or torch CUDA tensors (device memory, passed by pointer); the HIP stream is
torch's current stream unless one is given.  The library must have been
built (``python -m paper_1305_3417_amd.build``); importing works without it,
but the first call raises if libvof.so is missing.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvof.so")

VOF_OK = 0
VOF_EINVAL = -1
VOF_EBADMESH = -2
VOF_ENOMEM = -3
VOF_EDEVICE = -4
VOF_ENUMERIC = -5
VOF_ESTENCIL = -6
VOF_ECAPACITY = -8
VOF_HOST = 0
VOF_DEVICE = 1
VOF_FACE_LAMBDA = 0
VOF_FACE_VPHASE = 1
VOF_FACE_ITERS = 2
VOF_FACE_KIND = 3
VOF_FACE_STATUS = 4
VOF_MAX_FACE_POINTS = 8
VOF_GRADIENT_NAG = 0
VOF_GRADIENT_LSQ = 1

EXPORTED = [
    "vof_context_create", "vof_context_destroy", "vof_last_error", "vof_version",
    "vof_mesh_upload", "vof_mesh_destroy", "vof_mesh_get_info", "vof_get_params",
    "vof_set_params", "vof_set_alpha", "vof_read_alpha", "vof_map_alpha", "vof_set_velocity",
    "vof_reconstruct", "vof_advect", "vof_advect_noalloc", "vof_read_face", "vof_read_planes",
    "vof_read_point_velocity", "vof_get_stats", "vof_reset_stats", "vof_synchronize",
    "vof_selftest_tet_clip", "vof_selftest_tet_clip_closed", "vof_profile_enable", "vof_profile_kernel_name", "vof_read_profile",
    "vof_batch_create", "vof_batch_destroy", "vof_batch_advect", "vof_batch_synchronize",
    "vof_batch_get_config", "vof_batch_set_config", "vof_autotune",
    "vof_server_create", "vof_server_submit", "vof_server_wait", "vof_server_get_stats",
    "vof_server_destroy",
]
VOF_EBUSY = -7
VOF_MAX_BATCH = 256


class VofError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


class vof_mesh_desc(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("n_cells", C.c_int64), ("n_faces", C.c_int64),
                ("n_internal", C.c_int64), ("points", C.c_void_p), ("face_offsets", C.c_void_p),
                ("face_points", C.c_void_p), ("owner", C.c_void_p), ("neighbour", C.c_void_p),
                ("memory", C.c_int32)]


class vof_mesh_info(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("n_cells", C.c_int64), ("n_faces", C.c_int64),
                ("n_internal", C.c_int64), ("stencil_entries", C.c_int64),
                ("max_face_points", C.c_int32), ("max_cell_faces", C.c_int32),
                ("device_bytes", C.c_int64)]


class vof_params(C.Structure):
    _fields_ = [("eps", C.c_double), ("correction_rtol", C.c_double),
                ("correction_max_iter", C.c_int32), ("position_tol", C.c_double),
                ("position_max_iter", C.c_int32), ("gradient_zero", C.c_double),
                ("check_stencil", C.c_int32), ("gradient", C.c_int32),
                ("narrow_band", C.c_int32), ("wisps", C.c_int32)]


class vof_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("face_fluxes", C.c_int64),
                ("geometric_faces", C.c_int64), ("interface_cells", C.c_int64),
                ("fallback_cells", C.c_int64), ("unreached_faces", C.c_int64),
                ("capacity_overflows", C.c_int64), ("stencil_leaks", C.c_int64),
                ("correction_iters", C.c_int64), ("clip_pairs", C.c_int64),
                ("general_tets", C.c_int64),
                ("ledger", C.c_double), ("mass", C.c_double),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double),
                ("wisps", C.c_int64), ("wisps_left", C.c_int64),
                ("chunk_rescans", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vof_batch_config(C.Structure):
    _fields_ = [("grid_flux", C.c_int32), ("grid_clip", C.c_int32), ("clip_claim", C.c_int32),
                ("grid_plane", C.c_int32), ("grid_cells", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vof_server_stats_t(C.Structure):
    _fields_ = [("jobs_done", C.c_int64), ("jobs_waiting", C.c_int64),
                ("face_fluxes", C.c_int64), ("ticks", C.c_int64),
                ("latency_p50_s", C.c_double), ("latency_p99_s", C.c_double),
                ("latency_max_s", C.c_double), ("face_fluxes_per_s", C.c_double),
                ("max_resident", C.c_int32), ("budget_bytes", C.c_int64),
                ("peak_bytes", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libvof.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1305_3417_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "vof_context_create": (i32, [i32, vp, C.POINTER(vp)]),
            "vof_context_destroy": (i32, [vp]),
            "vof_last_error": (C.c_char_p, []),
            "vof_version": (C.c_char_p, []),
            "vof_mesh_upload": (i32, [vp, C.POINTER(vof_mesh_desc), C.POINTER(vp)]),
            "vof_mesh_destroy": (i32, [vp]),
            "vof_mesh_get_info": (i32, [vp, C.POINTER(vof_mesh_info)]),
            "vof_get_params": (i32, [vp, C.POINTER(vof_params)]),
            "vof_set_params": (i32, [vp, C.POINTER(vof_params)]),
            "vof_set_alpha": (i32, [vp, vp, i32]),
            "vof_read_alpha": (i32, [vp, vp, i32]),
            "vof_map_alpha": (i32, [vp, vp, vp, vp, i32]),
            "vof_set_velocity": (i32, [vp, vp, vp, i32]),
            "vof_reconstruct": (i32, [vp]),
            "vof_advect": (i32, [vp, i32, vp, vp]),
            "vof_advect_noalloc": (i32, [vp, i32, vp, vp]),
            "vof_read_face": (i32, [vp, i32, vp, i32]),
            "vof_read_planes": (i32, [vp, vp, vp, vp, i32]),
            "vof_read_point_velocity": (i32, [vp, vp, i32]),
            "vof_get_stats": (i32, [vp, C.POINTER(vof_stats)]),
            "vof_reset_stats": (i32, [vp]),
            "vof_synchronize": (i32, [vp]),
            "vof_selftest_tet_clip": (d, [vp, i32, vp]),
            "vof_selftest_tet_clip_closed": (d, [vp, i32, vp]),
            "vof_profile_enable": (i32, [vp, i32]),
            "vof_profile_kernel_name": (C.c_char_p, [i32]),
            "vof_read_profile": (i32, [vp, vp, vp, i32]),
            "vof_batch_create": (i32, [vp, vp, i32, C.POINTER(vp)]),
            "vof_batch_destroy": (i32, [vp]),
            "vof_batch_advect": (i32, [vp, i32, vp, vp]),
            "vof_batch_synchronize": (i32, [vp]),
            "vof_batch_get_config": (i32, [vp, C.POINTER(vof_batch_config)]),
            "vof_batch_set_config": (i32, [vp, C.POINTER(vof_batch_config)]),
            "vof_autotune": (i32, [vp, i32, vp, vp, C.c_char_p, C.POINTER(vof_batch_config)]),
            "vof_server_create": (i32, [vp, i64, C.POINTER(vp)]),
            "vof_server_submit": (i32, [vp, vp, vp, vp, vp, i32, vp, vp, C.POINTER(vp)]),
            "vof_server_wait": (i32, [vp, vp, C.POINTER(d)]),
            "vof_server_get_stats": (i32, [vp, C.POINTER(vof_server_stats_t)]),
            "vof_server_destroy": (i32, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int, where: str, ok=(VOF_OK,)):
    if code not in ok:
        raise VofError(code, where, (lib().vof_last_error() or b"").decode())
    return code


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch") and hasattr(a, "data_ptr")


def _arg(a, dtype):
    """(pointer, memory, keepalive) of an input array."""
    if _is_torch(a):
        import torch
        tdt = {np.float64: torch.float64, np.int64: torch.int64, np.int32: torch.int32,
               np.int8: torch.int8, np.uint8: torch.uint8}[dtype]
        if a.dtype != tdt or not a.is_contiguous():
            raise TypeError(f"expected a contiguous {tdt} tensor")
        return C.c_void_p(a.data_ptr()), (VOF_DEVICE if a.is_cuda else VOF_HOST), a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data_as(C.c_void_p), VOF_HOST, arr


def _out(out, n, dtype):
    if out is None:
        out = np.empty(n, dtype=dtype)
    p, mem, keep = _arg(out, dtype)
    if not _is_torch(out) and keep is not out:
        raise TypeError("output arrays must be contiguous and of the right dtype")
    return out, p, mem


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover - torch is optional for the binding
        pass
    return C.c_void_p(0)


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def vof_version() -> str:
    return lib().vof_version().decode()


def vof_last_error() -> str:
    return (lib().vof_last_error() or b"").decode()


def vof_context_create(device: int = 0, stream=None):
    h = C.c_void_p()
    s = _current_stream() if stream is None else C.c_void_p(int(stream))
    _check(lib().vof_context_create(int(device), s, C.byref(h)), "vof_context_create")
    return h


def vof_context_destroy(ctx):
    _check(lib().vof_context_destroy(ctx), "vof_context_destroy")


_live_meshes: "weakref.WeakSet" = weakref.WeakSet()


class MeshHandle:
    """Owns a vof_mesh* and the host arrays it was uploaded from."""

    def __init__(self, h, info, keep):
        self.h = h
        self.info = info
        self._keep = keep
        _live_meshes.add(self)

    def close(self):
        if self.h:
            lib().vof_mesh_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # never call into the HIP runtime while the interpreter is shutting down
        # (module globals may already be gone then, hence the bound default)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_cells(self):
        return self.info.n_cells

    @property
    def n_faces(self):
        return self.info.n_faces

    @property
    def n_points(self):
        return self.info.n_points


@atexit.register
def _close_live_meshes():
    for m in list(_live_meshes):
        try:
            m.close()
        except Exception:
            pass


def vof_mesh_upload(ctx, points, face_offsets, face_points, owner, neighbour, n_cells):
    """Upload an owner/neighbour mesh (internal faces first)."""
    pp, pm, k1 = _arg(points, np.float64)
    op, om, k2 = _arg(face_offsets, np.int64)
    fp, fm, k3 = _arg(face_points, np.int32)
    wp, wm, k4 = _arg(owner, np.int32)
    npn, nm, k5 = _arg(neighbour, np.int32)
    mems = {pm, om, fm, wm, nm}
    if len(mems) != 1:
        raise TypeError("all mesh arrays must live in the same memory")
    d = vof_mesh_desc(n_points=int(k1.shape[0] if k1.ndim == 2 else k1.shape[0] // 3),
                      n_cells=int(n_cells), n_faces=int(k4.shape[0]),
                      n_internal=int(k5.shape[0]), points=pp, face_offsets=op, face_points=fp,
                      owner=wp, neighbour=npn, memory=mems.pop())
    h = C.c_void_p()
    _check(lib().vof_mesh_upload(ctx, C.byref(d), C.byref(h)), "vof_mesh_upload")
    info = vof_mesh_info()
    _check(lib().vof_mesh_get_info(h, C.byref(info)), "vof_mesh_get_info")
    return MeshHandle(h, info, (k1, k2, k3, k4, k5))


def vof_mesh_destroy(mesh: MeshHandle):
    mesh.close()


def vof_mesh_get_info(mesh: MeshHandle):
    info = vof_mesh_info()
    _check(lib().vof_mesh_get_info(mesh.h, C.byref(info)), "vof_mesh_get_info")
    return info


def vof_get_params(mesh: MeshHandle) -> vof_params:
    p = vof_params()
    _check(lib().vof_get_params(mesh.h, C.byref(p)), "vof_get_params")
    return p


def vof_set_params(mesh: MeshHandle, params: vof_params):
    _check(lib().vof_set_params(mesh.h, C.byref(params)), "vof_set_params")


def vof_set_alpha(mesh: MeshHandle, alpha):
    p, mem, keep = _arg(alpha, np.float64)
    if keep.shape[0] != mesh.n_cells:
        raise ValueError("alpha must have n_cells entries")
    _check(lib().vof_set_alpha(mesh.h, p, mem), "vof_set_alpha")


def vof_map_alpha(dst: MeshHandle, src: MeshHandle, map_offsets, map_cells):
    """alpha of dst from src's alpha by the geometric mapping (int32 CSR over
    dst's cells of src cells: one containing cell, or the cells of a union)."""
    po, mo, ko = _arg(map_offsets, np.int32)
    pc, mc, kc = _arg(map_cells, np.int32)
    if mo != mc:
        raise TypeError("map_offsets and map_cells must both be host or both device arrays")
    if ko.shape[0] != dst.n_cells + 1:
        raise ValueError("map_offsets must have n_cells(dst) + 1 entries")
    _check(lib().vof_map_alpha(dst.h, src.h, po, pc, mo), "vof_map_alpha")


def vof_read_alpha(mesh: MeshHandle, out=None, ok=(VOF_OK,)):
    out, p, mem = _out(out, mesh.n_cells, np.float64)
    _check(lib().vof_read_alpha(mesh.h, p, mem), "vof_read_alpha", ok)
    return out


def vof_set_velocity(mesh: MeshHandle, U0c, F0):
    up, um, k1 = _arg(U0c, np.float64)
    fp, fm, k2 = _arg(F0, np.float64)
    if um != fm:
        raise TypeError("U0c and F0 must live in the same memory")
    if k1.size != 3 * mesh.n_cells or k2.shape[0] != mesh.n_faces:
        raise ValueError("U0c must be (n_cells, 3) and F0 (n_faces,)")
    _check(lib().vof_set_velocity(mesh.h, up, fp, um), "vof_set_velocity")


def vof_reconstruct(mesh: MeshHandle):
    _check(lib().vof_reconstruct(mesh.h), "vof_reconstruct")


def vof_advect(mesh: MeshHandle, dt, scale):
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    scale = np.ascontiguousarray(scale, dtype=np.float64)
    if dt.shape != scale.shape or dt.ndim != 1:
        raise ValueError("dt and scale must be 1-D arrays of equal length")
    _check(lib().vof_advect(mesh.h, int(dt.shape[0]), dt.ctypes.data_as(C.c_void_p),
                            scale.ctypes.data_as(C.c_void_p)), "vof_advect")


VOF_NOALLOC_MAX_STEPS = 65536


def vof_advect_noalloc(mesh: MeshHandle, dt, scale):
    """vof_advect with no device allocation (schedule staged in the library's
    fixed per-device buffer; at most VOF_NOALLOC_MAX_STEPS steps)."""
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    scale = np.ascontiguousarray(scale, dtype=np.float64)
    if dt.shape != scale.shape or dt.ndim != 1:
        raise ValueError("dt and scale must be 1-D arrays of equal length")
    _check(lib().vof_advect_noalloc(mesh.h, int(dt.shape[0]), dt.ctypes.data_as(C.c_void_p),
                                    scale.ctypes.data_as(C.c_void_p)), "vof_advect_noalloc")


def vof_read_face(mesh: MeshHandle, what: int, out=None, ok=(VOF_OK,)):
    dtype = np.float64 if what in (VOF_FACE_LAMBDA, VOF_FACE_VPHASE) else np.uint8
    out, p, mem = _out(out, mesh.n_faces, dtype)
    _check(lib().vof_read_face(mesh.h, int(what), p, mem), "vof_read_face", ok)
    return out


def vof_read_planes(mesh: MeshHandle, ok=(VOF_OK,)):
    """(cls int8 [C], normal [C,3], s [C]) of the last reconstruction (host)."""
    n = mesh.n_cells
    cls = np.empty(n, dtype=np.int8)
    nrm = np.empty((n, 3), dtype=np.float64)
    s = np.empty(n, dtype=np.float64)
    _check(lib().vof_read_planes(mesh.h, cls.ctypes.data_as(C.c_void_p),
                                 nrm.ctypes.data_as(C.c_void_p), s.ctypes.data_as(C.c_void_p),
                                 VOF_HOST), "vof_read_planes", ok)
    return cls, nrm, s


def vof_read_point_velocity(mesh: MeshHandle):
    out = np.empty((mesh.n_points, 3), dtype=np.float64)
    _check(lib().vof_read_point_velocity(mesh.h, out.ctypes.data_as(C.c_void_p), VOF_HOST),
           "vof_read_point_velocity")
    return out


def vof_get_stats(mesh: MeshHandle, ok=(VOF_OK,)) -> dict:
    st = vof_stats()
    _check(lib().vof_get_stats(mesh.h, C.byref(st)), "vof_get_stats", ok)
    return st.as_dict()


def vof_reset_stats(mesh: MeshHandle):
    _check(lib().vof_reset_stats(mesh.h), "vof_reset_stats")


def vof_synchronize(mesh: MeshHandle, ok=(VOF_OK,)):
    return _check(lib().vof_synchronize(mesh.h), "vof_synchronize", ok)


def _selftest(fn, tet, planes) -> float:
    tet = np.ascontiguousarray(tet, dtype=np.float64).reshape(12)
    planes = np.ascontiguousarray(np.atleast_2d(planes), dtype=np.float64)
    if planes.size == 0:
        planes = np.zeros((0, 4))
    return fn(tet.ctypes.data_as(C.c_void_p), int(planes.shape[0]),
              planes.ctypes.data_as(C.c_void_p))


def vof_selftest_tet_clip(tet, planes) -> float:
    return _selftest(lib().vof_selftest_tet_clip, tet, planes)


def vof_selftest_tet_clip_closed(tet, planes) -> float:
    return _selftest(lib().vof_selftest_tet_clip_closed, tet, planes)


def vof_profile_enable(mesh: MeshHandle, enable: bool = True):
    _check(lib().vof_profile_enable(mesh.h, int(bool(enable))), "vof_profile_enable")


def vof_profile_kernel_name(i: int):
    r = lib().vof_profile_kernel_name(int(i))
    return None if r is None else r.decode()


def vof_read_profile(mesh: MeshHandle) -> dict:
    """{kernel name: (total ms, launches)} since the last read."""
    names = []
    while vof_profile_kernel_name(len(names)) is not None:
        names.append(vof_profile_kernel_name(len(names)))
    ms = np.zeros(len(names))
    cnt = np.zeros(len(names), dtype=np.int64)
    _check(lib().vof_read_profile(mesh.h, ms.ctypes.data_as(C.c_void_p),
                                  cnt.ctypes.data_as(C.c_void_p), len(names)), "vof_read_profile")
    return {n: (float(ms[i]), int(cnt[i])) for i, n in enumerate(names)}


def upload_mesh(ctx, mesh) -> MeshHandle:
    """vof_mesh_upload of a workloads.Mesh-like object (host arrays)."""
    return vof_mesh_upload(ctx, mesh.points, mesh.face_offsets, mesh.face_points, mesh.owner,
                           mesh.neighbour, mesh.n_cells)


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------

class BatchHandle:
    """Owns a vof_batch* (the meshes stay owned by their handles)."""

    def __init__(self, h, meshes):
        self.h = h
        self.meshes = list(meshes)

    def close(self):
        if self.h:
            lib().vof_batch_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def vof_batch_create(ctx, meshes) -> BatchHandle:
    arr = (C.c_void_p * len(meshes))(*[m.h for m in meshes])
    h = C.c_void_p()
    _check(lib().vof_batch_create(ctx, arr, len(meshes), C.byref(h)), "vof_batch_create")
    return BatchHandle(h, meshes)


def vof_batch_destroy(batch: BatchHandle):
    batch.close()


def vof_batch_advect(batch: BatchHandle, dt, scale):
    """dt, scale: (n_meshes, n_steps) arrays (row i: mesh i's schedule)."""
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    scale = np.ascontiguousarray(scale, dtype=np.float64)
    if dt.shape != scale.shape or dt.ndim != 2 or dt.shape[0] != len(batch.meshes):
        raise ValueError("dt and scale must be (n_meshes, n_steps) arrays")
    _check(lib().vof_batch_advect(batch.h, int(dt.shape[1]), dt.ctypes.data_as(C.c_void_p),
                                  scale.ctypes.data_as(C.c_void_p)), "vof_batch_advect")


def vof_batch_synchronize(batch: BatchHandle, ok=(VOF_OK,)):
    return _check(lib().vof_batch_synchronize(batch.h), "vof_batch_synchronize", ok)


def vof_batch_get_config(batch: BatchHandle) -> vof_batch_config:
    c = vof_batch_config()
    _check(lib().vof_batch_get_config(batch.h, C.byref(c)), "vof_batch_get_config")
    return c


def vof_batch_set_config(batch: BatchHandle, config: vof_batch_config):
    _check(lib().vof_batch_set_config(batch.h, C.byref(config)), "vof_batch_set_config")


def vof_autotune(batch: BatchHandle, dt, scale, cache_path=None) -> dict:
    """Advance the batch by dt.shape[1] steps while timing candidate launch
    configurations; the fastest becomes the batch's configuration (returned)."""
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    scale = np.ascontiguousarray(scale, dtype=np.float64)
    if dt.shape != scale.shape or dt.ndim != 2 or dt.shape[0] != len(batch.meshes):
        raise ValueError("dt and scale must be (n_meshes, n_steps) arrays")
    c = vof_batch_config()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().vof_autotune(batch.h, int(dt.shape[1]), dt.ctypes.data_as(C.c_void_p),
                              scale.ctypes.data_as(C.c_void_p), path, C.byref(c)),
           "vof_autotune")
    return c.as_dict()


# ---------------------------------------------------------------------------
# served form
# ---------------------------------------------------------------------------

class ServerHandle:
    def __init__(self, h):
        self.h = h

    def close(self):
        if self.h:
            lib().vof_server_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class JobHandle:
    def __init__(self, h, n_cells, keep):
        self.h = h
        self.n_cells = n_cells
        self._keep = keep


def vof_server_create(ctx, hbm_budget_bytes: int) -> ServerHandle:
    h = C.c_void_p()
    _check(lib().vof_server_create(ctx, int(hbm_budget_bytes), C.byref(h)), "vof_server_create")
    return ServerHandle(h)


def vof_server_destroy(server: ServerHandle):
    server.close()


def vof_server_submit(server: ServerHandle, mesh: MeshHandle, alpha0, U0c, F0, dt, scale,
                      ok=(VOF_OK,)):
    """Queue a job; returns a JobHandle (or None when the call returns a code
    listed in `ok` other than VOF_OK, e.g. VOF_EBUSY)."""
    a = np.ascontiguousarray(alpha0, dtype=np.float64)
    u = np.ascontiguousarray(U0c, dtype=np.float64)
    f = np.ascontiguousarray(F0, dtype=np.float64)
    dt = np.ascontiguousarray(dt, dtype=np.float64)
    sc = np.ascontiguousarray(scale, dtype=np.float64)
    if a.shape[0] != mesh.n_cells or u.size != 3 * mesh.n_cells or f.shape[0] != mesh.n_faces:
        raise ValueError("alpha0 (n_cells), U0c (n_cells, 3), F0 (n_faces)")
    if dt.shape != sc.shape or dt.ndim != 1:
        raise ValueError("dt and scale must be 1-D arrays of equal length")
    h = C.c_void_p()
    p = lambda x: x.ctypes.data_as(C.c_void_p)  # noqa: E731
    rc = _check(lib().vof_server_submit(server.h, mesh.h, p(a), p(u), p(f), int(dt.shape[0]),
                                        p(dt), p(sc), C.byref(h)), "vof_server_submit", ok)
    return JobHandle(h, mesh.n_cells, mesh) if rc == VOF_OK else None


def vof_server_wait(job: JobHandle, alpha_out=None):
    """Block until the job has finished; returns (alpha, latency in seconds)."""
    out = np.empty(job.n_cells) if alpha_out is None else alpha_out
    lat = C.c_double()
    h, job.h = job.h, None
    _check(lib().vof_server_wait(h, out.ctypes.data_as(C.c_void_p), C.byref(lat)),
           "vof_server_wait")
    return out, lat.value


def vof_server_get_stats(server: ServerHandle) -> dict:
    st = vof_server_stats_t()
    _check(lib().vof_server_get_stats(server.h, C.byref(st)), "vof_server_get_stats")
    return st.as_dict()
