"""Python binding of libitm.so, the gfx950 voxel-block-hashing TSDF fusion library.

Argument marshalling only: every step of allocation, compaction, integration and
raycasting runs in the library's HIP kernels.  Device buffers are torch tensors on
the current HIP device; the library runs on torch's current stream.  The names
mirror the C ABI in include/itm.h.  There is no fallback: if libitm.so is missing
or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libitm.so")

ITM_OK, ITM_ERR_ARG, ITM_ERR_OOM, ITM_ERR_HIP, ITM_ERR_STATE = 0, -1, -2, -3, -4
ITM_VOX_F32, ITM_VOX_F16, ITM_VOX_S16U8 = 0, 1, 2
FORMATS = {"f32": ITM_VOX_F32, "f16": ITM_VOX_F16, "s16u8": ITM_VOX_S16U8}
KERNELS = ("alloc", "integrate", "raycast", "refine", "icp_fine", "icp_coarse")
ITM_KERNEL_COUNT = len(KERNELS)


class ItmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"itm status {status}: {msg}")
        self.status = status


class itm_intrinsics(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]


class itm_track_params(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("iters", C.c_int32 * 4), ("dist_thresh", C.c_float * 4),
                ("min_inliers", C.c_int32)]


class itm_track_info(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("rms", C.c_double), ("steps", C.c_int32)]


class itm_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_allocated", "n_visible_last", "n_excess_used",
                                        "n_dropped_total", "vba_capacity", "n_updated_last",
                                        "n_entries", "bytes_per_voxel", "n_visible_total",
                                        "n_updated_total")]


_lib = None
_P = C.c_void_p
EXPORTED = ("itm_scene_create", "itm_scene_create_ex", "itm_scene_destroy", "itm_set_stream",
            "itm_integrate", "itm_raycast", "itm_export_blocks", "itm_import_blocks", "itm_get_stats",
            "itm_profile_enable", "itm_profile_read", "itm_last_error", "itm_last_status",
            "itm_refiner_create", "itm_refiner_destroy", "itm_refiner_set_stream",
            "itm_refiner_get_params", "itm_refiner_forward", "itm_refiner_gradient",
            "itm_refiner_train_step", "itm_gather_blocks", "itm_scene_set_refiner",
            "itm_export_blocks_refined", "itm_refine_visible", "itm_scene_set_search_range", "itm_expected_depths",
            "itm_track_default_params", "itm_track", "itm_icp_system", "itm_track_noalloc",
            "itm_scene_enable_colour", "itm_scene_enable_swapping", "itm_swap_stats", "itm_integrate_colour", "itm_raycast_colour", "itm_export_colour")
ITM_REFINE_PARAMS = 27712


def lib():
    """Load libitm.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1410_0925_amd.build`")
        L = C.CDLL(LIB_PATH)
        sig = {
            "itm_scene_create": (_P, [C.c_float, C.c_float, C.c_int32, C.c_int64, C.c_int64]),
            "itm_scene_create_ex": (_P, [C.c_float, C.c_float, C.c_int32, C.c_int64, C.c_int64,
                                         C.c_int32, _P, C.c_float, C.c_float]),
            "itm_scene_destroy": (None, [_P]),
            "itm_set_stream": (C.c_int, [_P, _P]),
            "itm_integrate": (C.c_int, [_P, _P, C.POINTER(itm_intrinsics), _P]),
            "itm_raycast": (C.c_int, [_P, C.POINTER(itm_intrinsics), _P, _P, _P]),
            "itm_export_blocks": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.POINTER(C.c_int64)]),
            "itm_import_blocks": (C.c_int, [_P, _P, _P, _P, C.c_int64]),
            "itm_get_stats": (C.c_int, [_P, C.POINTER(itm_stats)]),
            "itm_profile_enable": (C.c_int, [_P, C.c_int]),
            "itm_profile_read": (C.c_int, [_P, _P, _P]),
            "itm_last_error": (C.c_char_p, []),
            "itm_last_status": (C.c_int, []),
            "itm_refiner_create": (_P, [_P, _P]),
            "itm_refiner_destroy": (None, [_P]),
            "itm_refiner_set_stream": (C.c_int, [_P, _P]),
            "itm_refiner_get_params": (C.c_int, [_P, _P]),
            "itm_refiner_forward": (C.c_int, [_P, _P, C.c_int64, _P]),
            "itm_refiner_gradient": (C.c_int, [_P, _P, _P, _P, C.c_int64, _P, _P]),
            "itm_refiner_train_step": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_float, _P]),
            "itm_gather_blocks": (C.c_int, [_P, _P, C.c_int64, _P]),
            "itm_scene_set_refiner": (C.c_int, [_P, _P, C.c_float]),
            "itm_refine_visible": (C.c_int, [_P]),
            "itm_export_blocks_refined": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.POINTER(C.c_int64)]),
            "itm_scene_set_search_range": (C.c_int, [_P, C.c_int32, C.c_int32]),
            "itm_expected_depths": (C.c_int, [_P, C.POINTER(itm_intrinsics), _P, _P]),
            "itm_track_default_params": (None, [C.POINTER(itm_track_params)]),
            "itm_track": (C.c_int, [_P, _P, C.POINTER(itm_intrinsics), _P, _P, _P, _P,
                                    C.POINTER(itm_track_params), _P, C.POINTER(itm_track_info)]),
            "itm_track_noalloc": (C.c_int, [_P, _P, C.POINTER(itm_intrinsics), _P, _P, _P, _P,
                                            C.POINTER(itm_track_params), _P, C.POINTER(itm_track_info)]),
            "itm_icp_system": (C.c_int, [_P, _P, C.POINTER(itm_intrinsics), C.c_int32, _P, _P, _P, _P,
                                         C.c_float, _P]),
            "itm_scene_enable_colour": (C.c_int, [_P]),
            "itm_scene_enable_swapping": (C.c_int, [_P, C.c_int64, C.c_int32, C.c_int32]),
            "itm_swap_stats": (C.c_int, [_P, _P]),
            "itm_integrate_colour": (C.c_int, [_P, _P, _P, C.POINTER(itm_intrinsics), _P]),
            "itm_raycast_colour": (C.c_int, [_P, C.POINTER(itm_intrinsics), _P, _P, _P, _P]),
            "itm_export_colour": (C.c_int, [_P, _P, C.c_int64, C.POINTER(C.c_int64)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != ITM_OK:
        raise ItmError(status, lib().itm_last_error().decode())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _intr(K, width=None, height=None):
    if isinstance(K, itm_intrinsics):
        return K
    fx, fy, cx, cy = K[:4]
    w = width if width is not None else K[4]
    h = height if height is not None else K[5]
    return itm_intrinsics(float(fx), float(fy), float(cx), float(cy), int(w), int(h))


def _pose(T):
    T = np.ascontiguousarray(T, np.float64).reshape(16)
    return T, T.ctypes.data_as(C.c_void_p)


def _dev(t, dtype_name, numel):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on the GPU")
    if str(t.dtype) != dtype_name or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"expected a contiguous {dtype_name} tensor of {numel} elements")
    return C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# C ABI mirrors
# ---------------------------------------------------------------------------
def itm_scene_create(voxel_size, mu, max_w, n_buckets, n_excess):
    h = lib().itm_scene_create(voxel_size, mu, max_w, n_buckets, n_excess)
    if not h:
        raise ItmError(lib().itm_last_status(), lib().itm_last_error().decode())
    return h


def itm_scene_create_ex(voxel_size, mu, max_w, n_buckets, n_excess, fmt=ITM_VOX_F32, stream=None,
                        z_near=0.2, z_far=5.0):
    h = lib().itm_scene_create_ex(voxel_size, mu, max_w, n_buckets, n_excess, fmt, stream,
                                  z_near, z_far)
    if not h:
        raise ItmError(lib().itm_last_status(), lib().itm_last_error().decode())
    return h


def itm_scene_destroy(h):
    lib().itm_scene_destroy(h)


def itm_set_stream(h, stream):
    _check(lib().itm_set_stream(h, stream))


def itm_integrate(h, depth, K, T_wc):
    Ki = _intr(K)
    ptr = _dev(depth, "torch.float32", Ki.width * Ki.height)
    T, Tp = _pose(T_wc)
    _check(lib().itm_integrate(h, ptr, C.byref(Ki), Tp))


def itm_raycast(h, K, T_wc, out_pts, out_normals):
    Ki = _intr(K)
    n = Ki.width * Ki.height * 4
    p = _dev(out_pts, "torch.float32", n)
    q = _dev(out_normals, "torch.float32", n)
    T, Tp = _pose(T_wc)
    _check(lib().itm_raycast(h, C.byref(Ki), Tp, p, q))


def itm_scene_enable_colour(h):
    _check(lib().itm_scene_enable_colour(h))


def itm_integrate_colour(h, depth, rgbx, K, T_wc):
    Ki = _intr(K)
    ptr = _dev(depth, "torch.float32", Ki.width * Ki.height)
    c = _dev(rgbx, "torch.uint8", 4 * Ki.width * Ki.height)
    T, Tp = _pose(T_wc)
    _check(lib().itm_integrate_colour(h, ptr, c, C.byref(Ki), Tp))


def itm_raycast_colour(h, K, T_wc, out_pts, out_normals, out_rgbx):
    Ki = _intr(K)
    n = Ki.width * Ki.height * 4
    p = _dev(out_pts, "torch.float32", n)
    q = _dev(out_normals, "torch.float32", n)
    c = _dev(out_rgbx, "torch.uint8", n)
    T, Tp = _pose(T_wc)
    _check(lib().itm_raycast_colour(h, C.byref(Ki), Tp, p, q, c))


def itm_export_colour(h):
    n = C.c_int64(0)
    _check(lib().itm_export_colour(h, None, 0, C.byref(n)))
    m = n.value
    rgbw = np.empty((m, 512, 4), np.uint8)
    _check(lib().itm_export_colour(h, rgbw.ctypes.data_as(_P), m, C.byref(n)))
    return rgbw


def itm_scene_set_search_range(h, enable, tile_capacity=0):
    _check(lib().itm_scene_set_search_range(h, 1 if enable else 0, int(tile_capacity)))


def itm_expected_depths(h, K, T_wc, out):
    Ki = _intr(K)
    z = _dev(out, "torch.float32", Ki.width * Ki.height * 2)
    T, Tp = _pose(T_wc)
    _check(lib().itm_expected_depths(h, C.byref(Ki), Tp, z))


def itm_track_default_params():
    p = itm_track_params()
    lib().itm_track_default_params(C.byref(p))
    return p


def track_params(iters=None, dist=None, min_inliers=None):
    """itm_track_params from per-level lists (finest first); unset fields keep
    the library's defaults."""
    p = itm_track_default_params()
    if iters is not None:
        if not 1 <= len(iters) <= 4:
            raise ValueError("1 to 4 levels")
        p.n_levels = len(iters)
        for i, v in enumerate(iters):
            p.iters[i] = int(v)
    if dist is not None:
        for i, v in enumerate(dist):
            p.dist_thresh[i] = float(v)
    if min_inliers is not None:
        p.min_inliers = int(min_inliers)
    return p


def itm_track(h, depth, K, ref_pts, ref_normals, T_ref, T_init, params=None, noalloc=False):
    Ki = _intr(K)
    n = Ki.width * Ki.height
    d = _dev(depth, "torch.float32", n)
    v = _dev(ref_pts, "torch.float32", 4 * n)
    q = _dev(ref_normals, "torch.float32", 4 * n)
    Tr, Trp = _pose(T_ref)
    Ti, Tip = _pose(T_init)
    out = np.empty(16, np.float64)
    info = itm_track_info()
    fn = lib().itm_track_noalloc if noalloc else lib().itm_track
    _check(fn(h, d, C.byref(Ki), v, q, Trp, Tip, C.byref(params) if params is not None else None,
              out.ctypes.data_as(_P), C.byref(info)))
    return out.reshape(4, 4), {"pairs": int(info.n_pairs), "rms": float(info.rms), "steps": int(info.steps)}


def itm_icp_system(h, depth, K, level, ref_pts, ref_normals, T_ref, T, dist_thresh):
    Ki = _intr(K)
    n = Ki.width * Ki.height
    d = _dev(depth, "torch.float32", n)
    v = _dev(ref_pts, "torch.float32", 4 * n)
    q = _dev(ref_normals, "torch.float32", 4 * n)
    Tr, Trp = _pose(T_ref)
    T2, Tp = _pose(T)
    sys_ = np.empty(29, np.float64)
    _check(lib().itm_icp_system(h, d, C.byref(Ki), int(level), v, q, Trp, Tp, float(dist_thresh),
                                sys_.ctypes.data_as(_P)))
    return sys_


def itm_export_blocks(h, values=True):
    n = C.c_int64(0)
    _check(lib().itm_export_blocks(h, None, None, None, 0, C.byref(n)))
    m = n.value
    coords = np.empty((m, 3), np.int32)
    sdf = np.empty((m, 512), np.float32) if values else None
    w = np.empty((m, 512), np.float32) if values else None
    _check(lib().itm_export_blocks(h, coords.ctypes.data_as(_P),
                                   sdf.ctypes.data_as(_P) if values else None,
                                   w.ctypes.data_as(_P) if values else None, m, C.byref(n)))
    return coords, sdf, w


def itm_import_blocks(h, coords, sdf, w):
    c = np.ascontiguousarray(coords, np.int32).reshape(-1, 3)
    f = np.ascontiguousarray(sdf, np.float32).reshape(-1, 512)
    q = np.ascontiguousarray(w, np.float32).reshape(-1, 512)
    if not (len(c) == len(f) == len(q)):
        raise ValueError("coords, sdf and w must hold the same number of blocks")
    _check(lib().itm_import_blocks(h, c.ctypes.data_as(_P), f.ctypes.data_as(_P), q.ctypes.data_as(_P), len(c)))


def itm_get_stats(h):
    st = itm_stats()
    _check(lib().itm_get_stats(h, C.byref(st)))
    return {name: getattr(st, name) for name, _ in itm_stats._fields_}


def itm_profile_enable(h, enable=True):
    _check(lib().itm_profile_enable(h, 1 if enable else 0))


def itm_profile_read(h):
    ms = np.zeros(ITM_KERNEL_COUNT, np.float64)
    n = np.zeros(ITM_KERNEL_COUNT, np.int64)
    _check(lib().itm_profile_read(h, ms.ctypes.data_as(_P), n.ctypes.data_as(_P)))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS)}


def itm_last_error():
    return lib().itm_last_error().decode()


def itm_refiner_create(params, stream=None):
    p = np.ascontiguousarray(params, np.float32)
    if p.size != ITM_REFINE_PARAMS:
        raise ValueError(f"expected {ITM_REFINE_PARAMS} parameters")
    h = lib().itm_refiner_create(p.ctypes.data_as(_P), stream)
    if not h:
        raise ItmError(ITM_ERR_ARG, lib().itm_last_error().decode())
    return h


def itm_refiner_destroy(h):
    lib().itm_refiner_destroy(h)


def itm_refiner_get_params(h):
    out = np.empty(ITM_REFINE_PARAMS, np.float32)
    _check(lib().itm_refiner_get_params(h, out.ctypes.data_as(_P)))
    return out


def itm_refiner_forward(h, inputs, out):
    n = inputs.shape[0]
    _check(lib().itm_refiner_forward(h, _dev(inputs, "torch.float32", n * 2000), n,
                                     _dev(out, "torch.float32", n * 512)))


def itm_refiner_gradient(h, inputs, target, mask, grad=None, loss=None):
    n = inputs.shape[0]
    _check(lib().itm_refiner_gradient(
        h, _dev(inputs, "torch.float32", n * 2000), _dev(target, "torch.float32", n * 512),
        _dev(mask, "torch.uint8", n * 512), n,
        None if grad is None else _dev(grad, "torch.float32", ITM_REFINE_PARAMS),
        None if loss is None else _dev(loss, "torch.float32", 1)))


def itm_refiner_train_step(h, inputs, target, mask, lr, loss=None):
    n = inputs.shape[0]
    _check(lib().itm_refiner_train_step(
        h, _dev(inputs, "torch.float32", n * 2000), _dev(target, "torch.float32", n * 512),
        _dev(mask, "torch.uint8", n * 512), n, float(lr),
        None if loss is None else _dev(loss, "torch.float32", 1)))


def itm_gather_blocks(h, coords, out):
    n = coords.shape[0]
    _check(lib().itm_gather_blocks(h, _dev(coords, "torch.int32", n * 3), n,
                                   _dev(out, "torch.float32", n * 2000)))


def itm_scene_set_refiner(h, refiner, w_threshold):
    _check(lib().itm_scene_set_refiner(h, refiner, float(w_threshold)))


def itm_export_blocks_refined(h):
    n = C.c_int64(0)
    _check(lib().itm_export_blocks_refined(h, None, None, None, 0, C.byref(n)))
    m = n.value
    coords = np.empty((m, 3), np.int32)
    sdf = np.empty((m, 512), np.float32)
    flags = np.empty(m, np.uint8)
    _check(lib().itm_export_blocks_refined(h, coords.ctypes.data_as(_P), sdf.ctypes.data_as(_P),
                                           flags.ctypes.data_as(_P), m, C.byref(n)))
    return coords, sdf, flags.astype(bool)


class Refiner:
    """The learned block refiner on the current GPU (owns the library object)."""

    def __init__(self, params):
        self.h = itm_refiner_create(params, _stream())

    def close(self):
        if getattr(self, "h", None):
            itm_refiner_destroy(self.h)
            self.h = None

    def __del__(self):
        # at interpreter exit this module's names may already be None: the
        # process's end then releases the device memory
        if itm_refiner_destroy is not None and _lib is not None:
            self.close()

    def _sync_stream(self):
        _check(lib().itm_refiner_set_stream(self.h, _stream()))

    def params(self):
        self._sync_stream()
        return itm_refiner_get_params(self.h)

    def forward(self, inputs, out=None):
        import torch
        if out is None:
            out = torch.empty((inputs.shape[0], 512), dtype=torch.float32, device="cuda")
        self._sync_stream()
        itm_refiner_forward(self.h, inputs, out)
        return out

    def gradient(self, inputs, target, mask):
        import torch
        g = torch.empty(ITM_REFINE_PARAMS, dtype=torch.float32, device="cuda")
        l = torch.empty(1, dtype=torch.float32, device="cuda")
        self._sync_stream()
        itm_refiner_gradient(self.h, inputs, target, mask, g, l)
        return g, l

    def train_step(self, inputs, target, mask, lr, loss=None):
        self._sync_stream()
        itm_refiner_train_step(self.h, inputs, target, mask, lr, loss)


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------
class Scene:
    """A fused volume on the current GPU (owns the library scene)."""

    def __init__(self, voxel_size, mu, max_w, n_buckets, n_excess, fmt="f32", z_near=0.2,
                 z_far=5.0):
        self.fmt = FORMATS[fmt] if isinstance(fmt, str) else int(fmt)
        self.h = itm_scene_create_ex(voxel_size, mu, max_w, n_buckets, n_excess, self.fmt,
                                     _stream(), z_near, z_far)
        self.voxel_size, self.mu, self.max_w = voxel_size, mu, max_w

    @classmethod
    def from_params(cls, p, fmt="f32"):
        return cls(p["voxel_size"], p["mu"], p["max_w"], p["n_buckets"], p["n_excess"], fmt=fmt)

    def close(self):
        if getattr(self, "h", None):
            itm_scene_destroy(self.h)
            self.h = None

    def __del__(self):
        # at interpreter exit this module's names may already be None: the
        # process's end then releases the device memory
        if itm_scene_destroy is not None and _lib is not None:
            self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _sync_stream(self):
        _check(lib().itm_set_stream(self.h, _stream()))

    def integrate(self, depth, K, T_wc):
        self._sync_stream()
        itm_integrate(self.h, depth, K, T_wc)

    def raycast(self, K, T_wc, out_pts=None, out_normals=None):
        import torch
        Ki = _intr(K)
        if out_pts is None:
            out_pts = torch.empty((Ki.height, Ki.width, 4), dtype=torch.float32, device="cuda")
        if out_normals is None:
            out_normals = torch.empty((Ki.height, Ki.width, 4), dtype=torch.float32, device="cuda")
        self._sync_stream()
        itm_raycast(self.h, Ki, T_wc, out_pts, out_normals)
        return out_pts, out_normals

    def enable_colour(self):
        """Give every voxel a colour (r, g, b) and a colour weight."""
        self._sync_stream()
        itm_scene_enable_colour(self.h)

    def integrate_colour(self, depth, rgbx, K, T_wc):
        """Fuse a depth frame and its registered colour image (uint8 [H, W, 4])."""
        self._sync_stream()
        itm_integrate_colour(self.h, depth, rgbx, K, T_wc)

    def raycast_colour(self, K, T_wc, pts=None, nrm=None, rgb=None):
        """Points, normals and colours (uint8 [H, W, 4]) rendered at T_wc."""
        import torch
        Ki = _intr(K)
        if pts is None:
            pts = torch.empty((Ki.height, Ki.width, 4), dtype=torch.float32, device="cuda")
        if nrm is None:
            nrm = torch.empty((Ki.height, Ki.width, 4), dtype=torch.float32, device="cuda")
        if rgb is None:
            rgb = torch.empty((Ki.height, Ki.width, 4), dtype=torch.uint8, device="cuda")
        self._sync_stream()
        itm_raycast_colour(self.h, Ki, T_wc, pts, nrm, rgb)
        return pts, nrm, rgb

    def export_colour(self):
        """Colour voxels [n, 512, 4] (r, g, b, colour weight) in export order."""
        self._sync_stream()
        return itm_export_colour(self.h)

    def set_search_range(self, enable=True, tile_capacity=0):
        """Raycast inside each pixel's expected depth range (on) or over
        [z_near, z_far] (off, the default)."""
        self._sync_stream()
        itm_scene_set_search_range(self.h, enable, tile_capacity)

    def expected_depths(self, K, T_wc, out=None):
        """[H, W, 2] float32 (z_min, z_max) per pixel from the last frame's visible
        blocks at pose T_wc; (+inf, 0) where none projects."""
        import torch
        Ki = _intr(K)
        if out is None:
            out = torch.empty((Ki.height, Ki.width, 2), dtype=torch.float32, device="cuda")
        self._sync_stream()
        itm_expected_depths(self.h, Ki, T_wc, out)
        return out

    def track(self, depth, K, ref_pts, ref_normals, T_ref, T_init=None, iters=None, dist=None,
              min_inliers=None, noalloc=False):
        """Pose of `depth` (camera -> world, [4, 4]) by point-to-plane alignment to
        the reference maps a raycast wrote at T_ref, and {pairs, rms, steps}.
        iters / dist: per level, finest first (default (4, 6, 10) / (0.02, 0.05,
        0.1) m).  noalloc: use itm_track_noalloc (the library's static scratch)."""
        self._sync_stream()
        p = track_params(iters, dist, min_inliers)
        return itm_track(self.h, depth, K, ref_pts, ref_normals, T_ref, T_ref if T_init is None else T_init, p,
                         noalloc=noalloc)

    def icp_system(self, depth, K, level, ref_pts, ref_normals, T_ref, T, dist_thresh):
        """The 29 sums of one Gauss-Newton step at pose T on hierarchy level
        `level` (upper triangle of A, g, sum d^2, pairs)."""
        self._sync_stream()
        return itm_icp_system(self.h, depth, K, level, ref_pts, ref_normals, T_ref, T, dist_thresh)

    def export(self, values=True):
        self._sync_stream()
        return itm_export_blocks(self.h, values)

    def enable_swapping(self, device_blocks, swap_in, swap_out):
        """Swapping (section "Swapping"): a device pool of device_blocks voxel
        blocks; per frame at most swap_in host copies merged back and swap_out
        blocks that left the view moved to the host.  Before the first frame."""
        self._sync_stream()
        _check(lib().itm_scene_enable_swapping(self.h, int(device_blocks), int(swap_in), int(swap_out)))

    def swap_stats(self):
        self._sync_stream()
        out = np.zeros(8, np.int64)
        _check(lib().itm_swap_stats(self.h, out.ctypes.data_as(_P)))
        keys = ["n_device", "n_host_only", "n_pending", "swapped_in_last", "swapped_out_last",
                "swapped_in_total", "swapped_out_total", "no_block_total"]
        return {k: int(v) for k, v in zip(keys, out)}

    def import_blocks(self, coords, sdf, w):
        """Load blocks (int32 [n, 3], F and W float [n, 512]); they become the
        visible set."""
        self._sync_stream()
        itm_import_blocks(self.h, coords, sdf, w)

    def stats(self):
        self._sync_stream()
        return itm_get_stats(self.h)

    def gather(self, coords):
        """Network inputs [n, 2, 1000] of the blocks at coords (int32 [n, 3])."""
        import torch
        c = torch.as_tensor(np.ascontiguousarray(coords, np.int32)).cuda()
        out = torch.empty((c.shape[0], 2000), dtype=torch.float32, device="cuda")
        self._sync_stream()
        itm_gather_blocks(self.h, c, out)
        return out

    def set_refiner(self, refiner, w_threshold=10.0):
        self._sync_stream()
        itm_scene_set_refiner(self.h, None if refiner is None else refiner.h, w_threshold)
        self._refiner = refiner   # keep it alive while attached

    def export_refined(self):
        self._sync_stream()
        return itm_export_blocks_refined(self.h)

    def refine_visible(self):
        """Run the attached refiner over the current visible set now."""
        self._sync_stream()
        _check(lib().itm_refine_visible(self.h))

    def profile(self, enable=True):
        itm_profile_enable(self.h, enable)

    def profile_read(self):
        self._sync_stream()
        return itm_profile_read(self.h)
