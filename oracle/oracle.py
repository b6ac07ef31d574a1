"""ctypes wrapper of the C++ oracle (oracle.cpp). Test infrastructure only.

Every function takes numpy arrays laid out as in the C-ABI (structure of
arrays, float32) and returns numpy arrays; continuous outputs are float64.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.cpp with g++ (OpenMP, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int
F32 = ctypes.c_float
F64 = ctypes.c_double


def _declare(lib):
    lib.or_project.argtypes = [I64, P, P, P, P, P, P, I32, I32, F32, F32, F32, F32, F32,
                               P, P, P, P, P, P, I32]
    lib.or_project.restype = I32
    lib.or_pinned_log2.argtypes = [F64]
    lib.or_pinned_log2.restype = F64
    lib.or_tile_lists.argtypes = [I64, P, P, P, I32, I32, I32, P, P]
    lib.or_tile_lists.restype = I64
    lib.or_forward.argtypes = [I64, P, P, P, P, P, P, I32, I32, F32, F32, F32, F32, F32,
                               P, P, P, P, P, P, P, I32]
    lib.or_forward.restype = I32
    lib.or_backward.argtypes = [I64, P, P, P, P, P, P, I32, I32, F32, F32, F32, F32, F32,
                                P, P, P, P, P, P, P, P, P, P, P, I32]
    lib.or_backward.restype = I32
    lib.or_record.argtypes = [I64, P, P, P, P, P, P, I32, I32, F32, F32, F32, F32, F32,
                              P, P, P, P, I32]
    lib.or_record.restype = I64
    lib.or_frozen_loss.argtypes = [I64, P, P, P, P, P, P, I32, I32, F64, F64, F64, F64,
                                   P, P, P, P, P, P, P, I32]
    lib.or_frozen_loss.restype = F64


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _scene_args(scene):
    arrs = [_f32(scene.means), _f32(scene.scales), _f32(scene.quats), _f32(scene.opacity),
            _f32(scene.colors)]
    return arrs


def _cam_args(scene):
    i = scene.intr
    return [int(i.width), int(i.height), float(i.fx), float(i.fy), float(i.cx), float(i.cy)]


NEAR_Z = 0.2


def pinned_log2(x: float) -> float:
    return load().or_pinned_log2(float(x))


def project(scene, near_z: float = NEAR_Z, nthreads: int = 0) -> dict:
    """Pinned projection: visible, zkey, bbox[4,n], ctr[2,n], rec[6,n], z32."""
    lib = load()
    n = scene.n
    means, scales, quats, opac, colors = _scene_args(scene)
    vm = _f32(scene.viewmat)
    out = dict(visible=np.zeros(n, np.uint8), zkey=np.zeros(n, np.uint32),
               bbox=np.zeros((4, n), np.int32), ctr=np.zeros((2, n), np.int32),
               rec=np.zeros((6, n), np.float32), z32=np.zeros(n, np.float32))
    lib.or_project(n, _ptr(means), _ptr(scales), _ptr(quats), _ptr(opac), _ptr(colors), _ptr(vm),
                   *_cam_args(scene), float(near_z),
                   _ptr(out["visible"]), _ptr(out["zkey"]), _ptr(out["bbox"]), _ptr(out["ctr"]),
                   _ptr(out["rec"]), _ptr(out["z32"]), int(nthreads))
    return out


def tile_lists(proj: dict, width: int, height: int, tile: int):
    """Per-tile lists (CSR): offsets [T+1] int64, ids [K] uint32 (Gaussian index)."""
    lib = load()
    n = proj["visible"].shape[0]
    vis, zk, bb = proj["visible"], proj["zkey"], np.ascontiguousarray(proj["bbox"])
    K = lib.or_tile_lists(n, _ptr(vis), _ptr(zk), _ptr(bb), width, height, tile, None, None)
    T = ((width + tile - 1) // tile) * ((height + tile - 1) // tile)
    offsets = np.zeros(T + 1, np.int64)
    ids = np.zeros(max(K, 1), np.uint32)
    lib.or_tile_lists(n, _ptr(vis), _ptr(zk), _ptr(bb), width, height, tile, _ptr(offsets), _ptr(ids))
    return offsets, ids[:K]


def forward(scene, near_z: float = NEAR_Z, nthreads: int = 0) -> dict:
    lib = load()
    i = scene.intr
    H, W = i.height, i.width
    arrs = _scene_args(scene)
    vm = _f32(scene.viewmat)
    out = dict(rgb=np.zeros((3, H, W)), depth=np.zeros((H, W)), sil=np.zeros((H, W)),
               tfinal=np.zeros((H, W)), ncomp=np.zeros((H, W), np.int32),
               flags=np.zeros((H, W), np.uint8), counters=np.zeros(4, np.int64))
    lib.or_forward(scene.n, *[_ptr(a) for a in arrs], _ptr(vm), *_cam_args(scene), float(near_z),
                   _ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["sil"]), _ptr(out["tfinal"]),
                   _ptr(out["ncomp"]), _ptr(out["flags"]), _ptr(out["counters"]), int(nthreads))
    return out


def backward(scene, g_rgb, g_depth, g_sil, near_z: float = NEAR_Z, nthreads: int = 0) -> dict:
    lib = load()
    n = scene.n
    arrs = _scene_args(scene)
    vm = _f32(scene.viewmat)
    gr, gd, gs = _f32(g_rgb), _f32(g_depth), _f32(g_sil)
    out = dict(means=np.zeros((3, n)), scales=np.zeros((3, n)), quats=np.zeros((4, n)),
               opacity=np.zeros(n), colors=np.zeros((3, n)), viewmat=np.zeros(12),
               twist=np.zeros(6), gflags=np.zeros(n, np.uint8))
    lib.or_backward(n, *[_ptr(a) for a in arrs], _ptr(vm), *_cam_args(scene), float(near_z),
                    _ptr(gr), _ptr(gd), _ptr(gs),
                    _ptr(out["means"]), _ptr(out["scales"]), _ptr(out["quats"]), _ptr(out["opacity"]),
                    _ptr(out["colors"]), _ptr(out["viewmat"]), _ptr(out["twist"]), _ptr(out["gflags"]),
                    int(nthreads))
    return out


def record(scene, near_z: float = NEAR_Z, nthreads: int = 0) -> dict:
    """Frozen decisions at the scene's parameters (see or_record)."""
    lib = load()
    n = scene.n
    arrs = _scene_args(scene)
    vm = _f32(scene.viewmat)
    P = scene.intr.pixels
    args = [n, *[_ptr(a) for a in arrs], _ptr(vm), *_cam_args(scene), float(near_z)]
    total = lib.or_record(*args, None, None, None, None, int(nthreads))
    offsets = np.zeros(P + 1, np.int64)
    ids = np.zeros(max(total, 1), np.int32)
    clamped = np.zeros(max(total, 1), np.uint8)
    fov = np.zeros(2 * n, np.int8)
    lib.or_record(*args, _ptr(offsets), _ptr(ids), _ptr(clamped), _ptr(fov), int(nthreads))
    return dict(offsets=offsets, ids=ids, clamped=clamped, fov=fov)


def frozen_loss(params: dict, viewmat, intr, rec: dict, g_rgb, g_depth, g_sil, nthreads: int = 0) -> float:
    """L = sum G_C.C + G_D D + G_S S at double-precision parameters with all
    decisions frozen to `rec`."""
    lib = load()
    m, s, q, o, c = (_f64(params[k]) for k in ("means", "scales", "quats", "opacity", "colors"))
    vm = _f64(viewmat)
    gr, gd, gs = _f32(g_rgb), _f32(g_depth), _f32(g_sil)
    return lib.or_frozen_loss(m.shape[1], _ptr(m), _ptr(s), _ptr(q), _ptr(o), _ptr(c), _ptr(vm),
                              int(intr.width), int(intr.height), float(np.float32(intr.fx)),
                              float(np.float32(intr.fy)), float(np.float32(intr.cx)),
                              float(np.float32(intr.cy)),
                              _ptr(rec["offsets"]), _ptr(rec["ids"]), _ptr(rec["clamped"]), _ptr(rec["fov"]),
                              _ptr(gr), _ptr(gd), _ptr(gs), int(nthreads))


def apply_twist(viewmat, xi) -> np.ndarray:
    """exp(xi^) [R|t] in double precision (left perturbation), xi = (rho, phi).
    Uses the closed-form SE(3) exponential (Rodrigues with the V matrix)."""
    V = np.asarray(viewmat, np.float64).reshape(3, 4)
    rho = np.asarray(xi[:3], np.float64)
    phi = np.asarray(xi[3:], np.float64)
    th = float(np.linalg.norm(phi))
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th < 1e-12:
        Rx = np.eye(3) + K
        Vm = np.eye(3) + 0.5 * K
    else:
        Rx = np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * (K @ K)
        Vm = np.eye(3) + (1 - math.cos(th)) / th ** 2 * K + (th - math.sin(th)) / th ** 3 * (K @ K)
    tx = Vm @ rho
    R = Rx @ V[:, :3]
    t = Rx @ V[:, 3] + tx
    return np.concatenate([R, t.reshape(3, 1)], axis=1).reshape(12)
