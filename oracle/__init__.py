"""CPU oracle of the per-frame fusion path (binary64, plain loops).

TEST INFRASTRUCTURE ONLY: imported by `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py`, never by the product package.  The C source,
`itm_oracle.c`, shares nothing with the GPU library; see its header for which
section of the paper each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "itm_oracle.c")
_LIB_DEFAULT = os.path.join(_HERE, "liboracle.so")
_LIB = _LIB_DEFAULT   # the build lib() loads

# binary64 everywhere, no contraction of a*b+c, no fast-math: decisions taken in
# binary32 must round exactly as written
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared"]


# the CPU-baseline build: the same source and semantics (no contraction, no
# fast-math), optimised for the host it runs on; built on that host when first used
def _host_tag() -> str:
    """a tag of this host's CPU (model and feature flags): a -march=native build
    is only loaded on the kind of CPU it was built for"""
    import hashlib
    info = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith(("model name", "flags")):
                    info += line
                if line.strip() == "":
                    break
    except OSError:
        pass
    return hashlib.sha1(info.encode()).hexdigest()[:12]


_LIB_NATIVE = os.path.join(_HERE, f"liboracle_native_{_host_tag()}.so")
CFLAGS_NATIVE = ["-O3", "-march=native"] + [f for f in CFLAGS if f != "-O2"]


def _stale(path: str) -> bool:
    """whether a build is missing or older than the source"""
    return not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC)


def _compile(path: str, flags) -> None:
    tmp = path + f".tmp{os.getpid()}"   # concurrent test workers each write their own
    subprocess.check_call(["gcc", *flags, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, path)


def use_native_build() -> str:
    """Load the -O3 -march=native build (compiled here if missing or older than
    the source) instead of the default one; must be called before any other
    oracle call."""
    global _LIB
    if _lib is not None and _LIB != _LIB_NATIVE:
        raise RuntimeError("the oracle library is already loaded")
    if _stale(_LIB_NATIVE):
        _compile(_LIB_NATIVE, CFLAGS_NATIVE)
    _LIB = _LIB_NATIVE
    return _LIB


def build(force: bool = True) -> str:
    for f in os.listdir(_HERE):   # host builds: rebuilt from the current source when next used
        if f.startswith("liboracle_native_") and f.endswith(".so"):
            os.remove(os.path.join(_HERE, f))
    if force or _stale(_LIB_DEFAULT):
        _compile(_LIB_DEFAULT, CFLAGS)
    return _LIB_DEFAULT


_lib = None
_P = C.c_void_p
_i64, _i32, _u32, _f32 = C.c_int64, C.c_int32, C.c_uint32, C.c_float


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        if _stale(_LIB):   # missing, or the source changed since it was built
            _compile(_LIB, CFLAGS_NATIVE if _LIB == _LIB_NATIVE else CFLAGS)
        L = C.CDLL(_LIB)
        sig = {
            "orc_hash_index": (_u32, [_i32, _i32, _i32, _u32]),
            "orc_scene_create": (_P, [_f32, _f32, _i32, _i64, _i64]),
            "orc_scene_destroy": (None, [_P]),
            "orc_set_range": (C.c_int, [_P, _f32, _f32]),
            "orc_set_pixel_order": (None, [_P, _P]),
            "orc_raycast_touched": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P]),
            "orc_find": (_i64, [_P, _i32, _i32, _i32]),
            "orc_insert": (_i64, [_P, _i32, _i32, _i32]),
            "orc_dda_blocks": (_i64, [_P, _P, _P, _i64]),
            "orc_segment": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, C.c_int, C.c_int, _f32, _P, _P]),
            "orc_allocate": (_i64, [_P, _P, C.c_int, C.c_int, _P, _P]),
            "orc_integrate": (_i64, [_P, _P, C.c_int, C.c_int, _P, _P]),
            "orc_visible_keys": (_i64, [_P, _P, _i64]),
            "orc_stats": (None, [_P, _P]),
            "orc_entries": (None, [_P, _P, _P, _P]),
            "orc_export": (_i64, [_P, _P, _P, _P, _i64]),
            "orc_update_voxels": (_i64, [_P, _P, C.c_int, C.c_int, _P, _P, _P, _P, _i64, _P, _P]),
            "orc_voxel_outcomes": (C.c_int, [_P, _P, C.c_int, C.c_int, _P, _P, _P, _P, _P]),
            "orc_export_candidates": (_i64, [_P, _P, _P, _P, _P, _P, _i64]),
            "orc_import": (_i64, [_P, _P, _P, _P, _i64]),
            "orc_enable_swapping": (C.c_int, [_P, _i64, _i64, _i64]),
            "orc_swap_stats": (None, [_P, _P]),
            "orc_dense_create": (_P, [_i64, _i64, _i64, _i64, _i64, _i64, _f32, _f32, _i32]),
            "orc_dense_destroy": (None, [_P]),
            "orc_dense_integrate": (_i64, [_P, _P, C.c_int, C.c_int, _P, _P, _P, _i64]),
            "orc_dense_read": (None, [_P, _P, _P, _P]),
            "orc_raycast": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P, _P, _P, _P]),
            "orc_raycast_range": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P, _P, _P, _P, _P]),
            "orc_raycast_alt": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
            "orc_raycast_crossing": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P]),
            "orc_expected_depths": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P]),
            "orc_num_threads": (C.c_int, []),
            "orc_set_threads": (None, [C.c_int]),
            "orc_enable_colour": (C.c_int, [_P]),
            "orc_integrate_colour": (_i64, [_P, _P, _P, C.c_int, C.c_int, _P, _P]),
            "orc_export_colour": (_i64, [_P, _P, _i64]),
            "orc_colour_at": (C.c_int, [_P, _P, _i64, _P]),
            "orc_depth_level": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P, _P]),
            "orc_icp_system": (C.c_int, [_P, C.c_int, C.c_int, _P, C.c_int, _P, _P, _P, _P, C.c_double, _P]),
            "orc_solve6": (C.c_int, [_P, _P, _P]),
            "orc_pose_step": (None, [_P, _P]),
            "orc_track": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P, _P, C.c_int, _P, _P, C.c_int, _P, _P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def hash_index(x: int, y: int, z: int, mask: int) -> int:
    return int(lib().orc_hash_index(x, y, z, mask))


def dda_blocks(P0, P1) -> np.ndarray:
    """Blocks crossed by the segment P0 -> P1 (binary32 block units), in visit order."""
    a = np.ascontiguousarray(P0, np.float32)
    b = np.ascontiguousarray(P1, np.float32)
    n = lib().orc_dda_blocks(_ptr(a), _ptr(b), None, 0)
    out = np.empty((n, 3), np.int32)
    lib().orc_dda_blocks(_ptr(a), _ptr(b), _ptr(out), n)
    return out


def _K(intr):
    return np.ascontiguousarray(intr, np.float64)


class Scene:
    """Hashed TSDF volume on the CPU (the paper's voxel block hashing)."""

    def __init__(self, voxel_size, mu, max_w, n_buckets, n_excess):
        self.h = lib().orc_scene_create(voxel_size, mu, max_w, n_buckets, n_excess)
        if not self.h:
            raise ValueError("invalid oracle scene parameters")
        self.voxel_size, self.mu, self.max_w = voxel_size, mu, max_w
        self.n_buckets, self.n_excess = n_buckets, n_excess
        self.n_entries = 2 * n_buckets + n_excess

    @classmethod
    def from_params(cls, p):
        return cls(p["voxel_size"], p["mu"], p["max_w"], p["n_buckets"], p["n_excess"])

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_scene_destroy(self.h)
            self.h = None

    def set_range(self, z_near, z_far):
        if lib().orc_set_range(self.h, z_near, z_far) != 0:
            raise ValueError("bad range")

    def find(self, x, y, z) -> int:
        return int(lib().orc_find(self.h, x, y, z))

    def insert(self, x, y, z) -> int:
        return int(lib().orc_insert(self.h, x, y, z))

    def segment(self, depth_value, u, v, W, H, intr, T_wc):
        P0 = np.zeros(3, np.float32)
        P1 = np.zeros(3, np.float32)
        ok = lib().orc_segment(self.h, W, H, _ptr(_K(intr)), _ptr(np.ascontiguousarray(T_wc, np.float64)),
                               u, v, depth_value, _ptr(P0), _ptr(P1))
        return (P0, P1) if ok else None

    def allocate(self, depth, intr, T_wc) -> int:
        d = np.ascontiguousarray(depth, np.float32)
        H, W = d.shape
        return int(lib().orc_allocate(self.h, _ptr(d), W, H, _ptr(_K(intr)),
                                      _ptr(np.ascontiguousarray(T_wc, np.float64))))

    def integrate(self, depth, intr, T_wc) -> int:
        """Allocation then integration of one frame; returns updated voxel count."""
        d = np.ascontiguousarray(depth, np.float32)
        H, W = d.shape
        r = int(lib().orc_integrate(self.h, _ptr(d), W, H, _ptr(_K(intr)),
                                    _ptr(np.ascontiguousarray(T_wc, np.float64))))
        if r < 0:
            raise MemoryError("oracle integrate failed")
        return r

    def visible_keys(self) -> np.ndarray:
        n = lib().orc_visible_keys(self.h, None, 0)
        out = np.empty((n, 3), np.int32)
        lib().orc_visible_keys(self.h, _ptr(out), n)
        return out

    def stats(self) -> dict:
        out = np.zeros(8, np.int64)
        lib().orc_stats(self.h, _ptr(out))
        keys = ["n_allocated", "n_visible", "n_excess_used", "n_dropped_total", "excess_demand",
                "n_updated_last", "n_ambiguous_last"]
        return {k: int(v) for k, v in zip(keys, out)}

    def entries(self):
        n = self.n_entries
        pos = np.empty((n, 3), np.int16)
        off = np.empty(n, np.int32)
        ptr = np.empty(n, np.int32)
        lib().orc_entries(self.h, _ptr(pos), _ptr(off), _ptr(ptr))
        return pos, off, ptr

    def export(self, with_values=True):
        n = lib().orc_export(self.h, None, None, None, 0)
        coords = np.empty((n, 3), np.int32)
        F = np.empty((n, 512), np.float64) if with_values else None
        Wt = np.empty((n, 512), np.int32) if with_values else None
        lib().orc_export(self.h, _ptr(coords), _ptr(F), _ptr(Wt), n)
        return coords, F, Wt

    def enable_swapping(self, device_blocks, swap_in, swap_out):
        """Swapping (section "Swapping"): a device pool of device_blocks voxel
        blocks; per frame at most swap_in host copies merged back and swap_out
        device blocks that left the view moved to the host."""
        if lib().orc_enable_swapping(self.h, int(device_blocks), int(swap_in), int(swap_out)):
            raise ValueError("swapping: bad sizes, already on, colour on, or more blocks than the pool")

    def swap_stats(self) -> dict:
        out = np.zeros(8, np.int64)
        lib().orc_swap_stats(self.h, _ptr(out))
        keys = ["n_device", "n_host_only", "n_pending", "swapped_in_last", "swapped_out_last",
                "swapped_in_total", "swapped_out_total", "no_block_total"]
        return {k: int(v) for k, v in zip(keys, out)}

    def import_blocks(self, coords, F, Wt) -> int:
        """Load blocks (coords int [n, 3], F [n, 512], W [n, 512] integer-valued, the
        layout of export()); they become the visible set.  Returns the number loaded."""
        c = np.ascontiguousarray(coords, np.int32).reshape(-1, 3)
        f = np.ascontiguousarray(F, np.float64).reshape(-1, 512)
        w = np.ascontiguousarray(np.asarray(Wt).astype(np.int32)).reshape(-1, 512)
        assert len(c) == len(f) == len(w)
        return int(lib().orc_import(self.h, _ptr(c), _ptr(f), _ptr(w), len(c)))

    def set_pixel_order(self, order):
        """Visit the pixels of the following frames' allocation in this order (a
        permutation of range(W * H)), or row-major with None."""
        self._order = None if order is None else np.ascontiguousarray(order, np.int32)
        lib().orc_set_pixel_order(self.h, _ptr(self._order))

    def export_candidates(self):
        """Voxels with more than one correct state (a decision within its binary32
        error bound of a threshold, see the oracle's integration): per extra
        state a row.  Returns dict(key int32 [n, 4] = block x, y, z, in-block
        index; F float64 [n]; W int32 [n]; rgbw uint8 [n, 4]; unresolved bool [n])."""
        n = lib().orc_export_candidates(self.h, None, None, None, None, None, 0)
        key = np.empty((n, 4), np.int32)
        F = np.empty(n, np.float64)
        Wt = np.empty(n, np.int32)
        rgbw = np.empty((n, 4), np.uint8)
        unr = np.empty(n, np.uint8)
        lib().orc_export_candidates(self.h, _ptr(key), _ptr(F), _ptr(Wt), _ptr(rgbw), _ptr(unr), n)
        return dict(key=key, F=F, W=Wt, rgbw=rgbw, unresolved=unr.astype(bool))

    def voxel_outcomes(self, depth, intr, T_wc, vox):
        """Step one of the update for one voxel: [(updated, f), ...], the binary64
        decision first, then the other outcomes within the decision margins;
        and whether a case stayed unresolved."""
        d = np.ascontiguousarray(depth, np.float32)
        H, W = d.shape
        upd = np.zeros(16, np.int32)
        f = np.zeros(16, np.float64)
        n = int(lib().orc_voxel_outcomes(self.h, _ptr(d), W, H, _ptr(_K(intr)),
                                         _ptr(np.ascontiguousarray(T_wc, np.float64)),
                                         _ptr(np.ascontiguousarray(vox, np.int32)), _ptr(upd), _ptr(f)))
        return [(bool(upd[i]), float(f[i])) for i in range(abs(n))], n < 0

    def enable_colour(self):
        """Colour (r, g, b, colour weight) per voxel from now on."""
        if lib().orc_enable_colour(self.h):
            raise MemoryError

    def integrate_colour(self, depth, rgbx, intr, T_wc) -> int:
        """A frame with its registered colour image (uint8 [H, W, 4])."""
        d = np.ascontiguousarray(depth, np.float32)
        H, W = d.shape
        c = np.ascontiguousarray(rgbx, np.uint8)
        assert c.shape == (H, W, 4)
        r = int(lib().orc_integrate_colour(self.h, _ptr(d), _ptr(c), W, H, _ptr(_K(intr)),
                                           _ptr(np.ascontiguousarray(T_wc, np.float64))))
        if r < 0:
            raise RuntimeError("colour not enabled or allocation failed")
        return r

    def export_colour(self):
        """uint8 [n, 512, 4] (r, g, b, colour weight) in the order of export()."""
        n = lib().orc_export_colour(self.h, None, 0)
        if n < 0:
            raise RuntimeError("colour not enabled")
        out = np.empty((n, 512, 4), np.uint8)
        lib().orc_export_colour(self.h, _ptr(out), n)
        return out

    def colour_at(self, pts):
        """Colour of the nearest voxel of each hit point (float32 [..., 4], world
        metres, w > 0 = hit): uint8 [..., 4] = (r, g, b, 255), zeros elsewhere."""
        p = np.ascontiguousarray(pts, np.float32)
        out = np.empty(p.shape[:-1] + (4,), np.uint8)
        if lib().orc_colour_at(self.h, _ptr(p), p.size // 4, _ptr(out)):
            raise RuntimeError("colour not enabled")
        return out

    def update_voxels(self, depth, intr, T_wc, vox, active, F, Wt) -> int:
        """Apply one frame's update to individual voxels (absolute voxel coords)."""
        d = np.ascontiguousarray(depth, np.float32)
        H, W = d.shape
        vox = np.ascontiguousarray(vox, np.int32)
        act = np.ascontiguousarray(active, np.uint8)
        assert F.dtype == np.float64 and Wt.dtype == np.int32 and F.flags.c_contiguous
        return int(lib().orc_update_voxels(self.h, _ptr(d), W, H, _ptr(_K(intr)),
                                           _ptr(np.ascontiguousarray(T_wc, np.float64)),
                                           _ptr(vox), _ptr(act), len(vox), _ptr(F), _ptr(Wt)))

    def raycast(self, W, H, intr, T_wc, zrange=None, alternatives=False):
        """Returns (pts [H,W,4], normals [H,W,4], camera depth [H,W], flags, steps)
        of the march that takes the binary64 reads.  zrange: [H,W,2] binary32
        expected depth ranges (expected_depths), or None for the fixed range
        [z_near, z_far].  alternatives: also follow every read within the binary32
        decision margin and append alt [H,W,8,6] = the ray's other correct
        outcomes (hit (-1 = unused row), camera depth, normal xyz, normal valid).
        flags: bit 0 a sign decision with |F_n| < 1e-4, bit 1 iteration cap, bit 2
        other outcomes exist, bit 3 more branches than followed."""
        pts = np.empty((H, W, 4), np.float64)
        nrm = np.empty((H, W, 4), np.float64)
        zc = np.empty((H, W), np.float64)
        fl = np.empty((H, W), np.uint8)
        st = np.empty((H, W), np.int32)
        zr = None if zrange is None else np.ascontiguousarray(zrange, np.float32)
        assert zr is None or zr.shape == (H, W, 2)
        alt = np.empty((H, W, 8, 6), np.float64) if alternatives else None
        lib().orc_raycast_alt(self.h, W, H, _ptr(_K(intr)), _ptr(np.ascontiguousarray(T_wc, np.float64)),
                              _ptr(zr), _ptr(pts), _ptr(nrm), _ptr(zc), _ptr(fl), _ptr(st), _ptr(alt))
        if alternatives:
            return pts, nrm, zc, fl, st, alt
        return pts, nrm, zc, fl, st

    def raycast_touched(self, W, H, intr, T_wc, zrange=None):
        """(distinct blocks whose voxels a raycast reads, distinct buckets it probes)"""
        out = np.zeros(2, np.int64)
        zr = None if zrange is None else np.ascontiguousarray(zrange, np.float32)
        if lib().orc_raycast_touched(self.h, W, H, _ptr(_K(intr)), _ptr(np.ascontiguousarray(T_wc, np.float64)),
                                     _ptr(zr), _ptr(out)):
            raise MemoryError
        return int(out[0]), int(out[1])

    def expected_depths(self, W, H, intr, T_wc):
        """[H,W,2] binary32 (z_min, z_max) per pixel from the last frame's visible
        blocks; (+inf, 0) where no block projects."""
        zr = np.empty((H, W, 2), np.float32)
        lib().orc_expected_depths(self.h, W, H, _ptr(_K(intr)), _ptr(np.ascontiguousarray(T_wc, np.float64)),
                                  _ptr(zr))
        return zr

    def raycast_crossing(self, W, H, intr, T_wc):
        zc = np.empty((H, W), np.float64)
        lib().orc_raycast_crossing(self.h, W, H, _ptr(_K(intr)),
                                   _ptr(np.ascontiguousarray(T_wc, np.float64)), _ptr(zc))
        return zc


class Dense:
    """Dense TSDF grid on the CPU (the paper's plain voxel array)."""

    def __init__(self, origin, size, voxel_size, mu, max_w):
        self.size = tuple(int(s) for s in size)
        self.origin = tuple(int(o) for o in origin)
        self.h = lib().orc_dense_create(*self.origin, *self.size, voxel_size, mu, max_w)
        if not self.h:
            raise ValueError("invalid dense grid")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_dense_destroy(self.h)
            self.h = None

    def integrate(self, depth, intr, T_wc, mask_keys=None) -> int:
        d = np.ascontiguousarray(depth, np.float32)
        H, W = d.shape
        mk = None if mask_keys is None else np.ascontiguousarray(mask_keys, np.int32)
        return int(lib().orc_dense_integrate(self.h, _ptr(d), W, H, _ptr(_K(intr)),
                                             _ptr(np.ascontiguousarray(T_wc, np.float64)),
                                             _ptr(mk), 0 if mk is None else len(mk)))

    def read(self):
        nx, ny, nz = self.size
        F = np.empty((nz, ny, nx), np.float64)
        Wt = np.empty((nz, ny, nx), np.int32)
        fr = np.empty((nz, ny, nx), np.uint64)
        lib().orc_dense_read(self.h, _ptr(F), _ptr(Wt), _ptr(fr))
        return F, Wt, fr


# -- depth tracker (section "Tracking") --------------------------------------

def depth_level(depth, level):
    """Level `level` of the depth hierarchy (binary64; 0 where no valid depth)."""
    d = np.ascontiguousarray(depth, np.float32)
    H, W = d.shape
    out = np.empty(W * H, np.float64)
    wl, hl = C.c_int(), C.c_int()
    if lib().orc_depth_level(_ptr(d), W, H, level, _ptr(out), C.byref(wl), C.byref(hl)):
        raise MemoryError
    return out[: wl.value * hl.value].reshape(hl.value, wl.value)


def _maps(V, N, H, W):
    V = np.ascontiguousarray(V, np.float32)
    N = np.ascontiguousarray(N, np.float32)
    assert V.shape == (H, W, 4) and N.shape == (H, W, 4)
    return V, N


def icp_system(depth, intr, level, V, N, T_ref, T, dist_thresh):
    """The 29 sums of one Gauss-Newton step: upper triangle of A (21), g (6),
    sum of squared distances, number of pairs."""
    d = np.ascontiguousarray(depth, np.float32)
    H, W = d.shape
    V, N = _maps(V, N, H, W)
    sys_ = np.empty(29, np.float64)
    lib().orc_icp_system(_ptr(d), W, H, _ptr(_K(intr)), level, _ptr(V), _ptr(N),
                         _ptr(np.ascontiguousarray(T_ref, np.float64)),
                         _ptr(np.ascontiguousarray(T, np.float64)), float(dist_thresh), _ptr(sys_))
    return sys_


def solve6(A_up, b):
    x = np.empty(6, np.float64)
    if lib().orc_solve6(_ptr(np.ascontiguousarray(A_up, np.float64)), _ptr(np.ascontiguousarray(b, np.float64)),
                        _ptr(x)):
        raise np.linalg.LinAlgError("not positive definite")
    return x


def pose_step(xi, T):
    T = np.array(T, np.float64, copy=True, order="C")
    lib().orc_pose_step(_ptr(np.ascontiguousarray(xi, np.float64)), _ptr(T))
    return T


def track(depth, intr, V, N, T_ref, T_init, iters=(4, 6, 10), dist=(0.02, 0.05, 0.1), min_inliers=100):
    """Point-to-plane tracking over len(iters) levels (finest first).  Returns
    (T [4,4], info {pairs, rms, steps})."""
    d = np.ascontiguousarray(depth, np.float32)
    H, W = d.shape
    V, N = _maps(V, N, H, W)
    it = np.ascontiguousarray(iters, np.int32)
    ds = np.ascontiguousarray(dist, np.float64)
    T = np.empty((4, 4), np.float64)
    info = np.empty(3, np.float64)
    lib().orc_track(_ptr(d), W, H, _ptr(_K(intr)), _ptr(V), _ptr(N), _ptr(np.ascontiguousarray(T_ref, np.float64)),
                    _ptr(np.ascontiguousarray(T_init, np.float64)), len(it), _ptr(it), _ptr(ds), int(min_inliers),
                    _ptr(T), _ptr(info))
    return T, {"pairs": int(info[0]), "rms": float(info[1]), "steps": int(info[2])}


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def fuse_stream(stream, n_frames=None, scene=None):
    """Run allocation + integration over the first n_frames of a synth.Stream."""
    sc = scene or Scene.from_params(stream.params)
    n = stream.n_frames if n_frames is None else n_frames
    for f in range(n):
        sc.integrate(stream.depth[f], stream.intrinsics, stream.T_wc[f])
    return sc
