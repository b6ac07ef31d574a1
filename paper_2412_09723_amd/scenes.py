"""Seeded synthetic inputs for the RGB-D Gaussian rasterizer.

This module only draws random numbers and lays them out; it contains none of
the rasterizer's arithmetic (no projection, compositing or gradients), so both
the GPU path and the CPU oracle can take their inputs from it.

The Gaussian map of the paper (Sec. 3.3) is a set of Gaussians, each with a
mean, a covariance (stored here as per-axis scales plus a rotation
quaternion, App. C.1 names the per-axis scales), an opacity and a colour.
The camera pose (Sec. 3.1) is a world-to-camera rigid transform [R|t].

The datasets the paper evaluates on (Multi-agent Replica, 7-Scenes) are not
available; these generators stand in for them with indoor-room-shaped scenes.

Layout (matches the C-ABI): structure-of-arrays float32,
  means [3][N], scales [3][N] (std-dev in metres), quats [4][N] (w,x,y,z),
  opacity [N] (already in (0,1)), colors [3][N] (RGB, degree-0),
  viewmat [12] = row-major 3x4 [R|t] mapping world to camera
  (camera x right, y down, z forward).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Intrinsics", "Scene", "rng_for", "frustum_scene", "room_scene",
    "room_center_pose", "look_outward_pose", "perturb_pose", "upstream_grads",
    "small_frustum", "room_view", "keyframe_ring", "four_agent_rooms", "serving_agents",
    "poisson_trace",
]


@dataclasses.dataclass(frozen=True)
class Intrinsics:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    @property
    def pixels(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Scene:
    """One render job's inputs: a Gaussian map, a pose and pinhole intrinsics."""
    means: np.ndarray      # float32 [3, N]
    scales: np.ndarray     # float32 [3, N]
    quats: np.ndarray      # float32 [4, N]
    opacity: np.ndarray    # float32 [N]
    colors: np.ndarray     # float32 [3, N]
    viewmat: np.ndarray    # float32 [12]
    intr: Intrinsics

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def map_arrays(self):
        return dict(means=self.means, scales=self.scales, quats=self.quats,
                    opacity=self.opacity, colors=self.colors)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.means[:, idx]),
                     np.ascontiguousarray(self.scales[:, idx]),
                     np.ascontiguousarray(self.quats[:, idx]),
                     np.ascontiguousarray(self.opacity[idx]),
                     np.ascontiguousarray(self.colors[:, idx]),
                     self.viewmat.copy(), self.intr)


def rng_for(stream: int, agent: int = 0, salt: int = 0) -> np.random.Generator:
    """PCG64 stream with seed = 1000*stream + agent (+ salt for auxiliary draws);
    each workload below draws from its own stream number."""
    return np.random.Generator(np.random.PCG64(1000 * stream + agent + 7919 * salt))


def _attributes(rng: np.random.Generator, n: int):
    """Per-Gaussian attributes shared by every configuration:
    scales log-uniform in [0.01, 0.1] m per axis, quaternions N(0, I4)
    normalised, opacity sigmoid(N(0,1)), RGB uniform in [0,1]."""
    scales = np.exp(rng.uniform(math.log(0.01), math.log(0.1), size=(3, n)))
    q = rng.standard_normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opacity = 1.0 / (1.0 + np.exp(-rng.standard_normal(size=n)))
    colors = rng.uniform(0.0, 1.0, size=(3, n))
    return (scales.astype(np.float32), q.astype(np.float32),
            opacity.astype(np.float32), colors.astype(np.float32))


def _identity_viewmat() -> np.ndarray:
    return np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], dtype=np.float32)


def _viewmat_from_rt(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    return np.concatenate([R, t.reshape(3, 1)], axis=1).reshape(12).astype(np.float32)


def _viewmat_rt(viewmat: np.ndarray):
    v = np.asarray(viewmat, dtype=np.float64).reshape(3, 4)
    return v[:, :3].copy(), v[:, 3].copy()


def frustum_scene(n: int, intr: Intrinsics, rng: np.random.Generator,
                  zmin: float = 1.0, zmax: float = 5.0,
                  viewmat: np.ndarray | None = None) -> Scene:
    """Means uniform in (pixel x depth) of the camera frustum, depth in
    [zmin, zmax] m, expressed in world coordinates for the given pose."""
    z = rng.uniform(zmin, zmax, size=n)
    u = rng.uniform(0.0, intr.width, size=n)
    v = rng.uniform(0.0, intr.height, size=n)
    pc = np.stack([(u - intr.cx) * z / intr.fx, (v - intr.cy) * z / intr.fy, z])
    vm = _identity_viewmat() if viewmat is None else np.asarray(viewmat, np.float32)
    R, t = _viewmat_rt(vm)
    pw = R.T @ (pc - t.reshape(3, 1))           # camera -> world
    scales, quats, opacity, colors = _attributes(rng, n)
    return Scene(pw.astype(np.float32), scales, quats, opacity, colors, vm.copy(), intr)


def room_scene(n: int, rng: np.random.Generator, room=(6.0, 4.0, 3.0),
               planar_frac: float = 0.7, noise: float = 0.02) -> np.ndarray:
    """Means for a box-shaped room [0,Lx]x[0,Ly]x[0,Lz]: `planar_frac` of them
    on the six faces (area-weighted, N(0, noise) along the face normal), the
    rest uniform in the volume. Returns float64 [3, n]."""
    Lx, Ly, Lz = room
    n_pl = int(round(planar_frac * n))
    n_vol = n - n_pl
    faces = [  # (axis fixed, value, other axes)
        (0, 0.0), (0, Lx), (1, 0.0), (1, Ly), (2, 0.0), (2, Lz)]
    dims = np.array([Lx, Ly, Lz])
    areas = np.array([np.prod(np.delete(dims, a)) for a, _ in faces])
    which = rng.choice(6, size=n_pl, p=areas / areas.sum())
    pts = rng.uniform(0.0, 1.0, size=(3, n_pl)) * dims.reshape(3, 1)
    for f, (axis, val) in enumerate(faces):
        sel = which == f
        pts[axis, sel] = val + noise * rng.standard_normal(size=int(sel.sum()))
    vol = rng.uniform(0.0, 1.0, size=(3, n_vol)) * dims.reshape(3, 1)
    out = np.concatenate([pts, vol], axis=1)
    perm = rng.permutation(n)
    return out[:, perm]


def room_center_pose(room=(6.0, 4.0, 3.0)) -> np.ndarray:
    """Camera at the room centre looking along +x with world z up:
    camera x = -world y, camera y = -world z, camera z = +world x."""
    R = np.array([[0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]])
    c = 0.5 * np.asarray(room, dtype=np.float64)
    return _viewmat_from_rt(R, -R @ c)


def look_outward_pose(center: np.ndarray, yaw: float) -> np.ndarray:
    """Camera at `center` looking horizontally along (cos yaw, sin yaw, 0),
    world z up."""
    f = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(f, up)
    R = np.stack([right, -up, f])
    return _viewmat_from_rt(R, -R @ np.asarray(center, np.float64))


def _axis_angle(axis: np.ndarray, angle: float) -> np.ndarray:
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def perturb_pose(viewmat: np.ndarray, rng: np.random.Generator,
                 trans: float = 0.02, rot_deg: float = 1.0) -> np.ndarray:
    """Left-perturb a world-to-camera pose by `trans` metres along a random unit
    direction and `rot_deg` degrees about a random unit axis."""
    R, t = _viewmat_rt(viewmat)
    d = rng.standard_normal(3)
    a = rng.standard_normal(3)
    dR = _axis_angle(a, math.radians(rot_deg))
    return _viewmat_from_rt(dR @ R, dR @ t + trans * d / np.linalg.norm(d))


def upstream_grads(intr: Intrinsics, rng: np.random.Generator, w_depth: float = 1.0,
                   w_sil: float = 0.0):
    """Upstream gradients shaped like those of a mean-L1 loss: each RGB entry
    is +-1/(3HW), each depth entry +-w_depth/(HW), silhouette +-w_sil/(HW).
    Signs are random (independent of any render) so that both sides of a
    comparison see exactly the same upstream values."""
    H, W = intr.height, intr.width
    gc = rng.choice([-1.0, 1.0], size=(3, H, W)) / (3.0 * H * W)
    gd = rng.choice([-1.0, 1.0], size=(H, W)) * (w_depth / (H * W))
    gs = rng.choice([-1.0, 1.0], size=(H, W)) * (w_sil / (H * W))
    return gc.astype(np.float32), gd.astype(np.float32), gs.astype(np.float32)


# ---------------------------------------------------------------- workloads

SMALL_INTR = Intrinsics(160, 120, 150.0, 150.0, 80.0, 60.0)
ROOM_INTR = Intrinsics(1200, 680, 600.0, 600.0, 600.0, 340.0)
VGA_INTR = Intrinsics(640, 480, 500.0, 500.0, 320.0, 240.0)


def small_frustum(seed_agent: int = 0, n: int = 4096) -> Scene:
    """160x120, fx=fy=150, identity pose, 4,096 Gaussians in the frustum at 1-5 m."""
    return frustum_scene(n, SMALL_INTR, rng_for(0, seed_agent))


def _room_map(n: int, rng: np.random.Generator, room) -> tuple:
    means = room_scene(n, rng, room)
    scales, quats, opacity, colors = _attributes(rng, n)
    return means.astype(np.float32), scales, quats, opacity, colors


def room_view(n: int = 1_000_000, agent: int = 0, intr: Intrinsics = ROOM_INTR,
            room=(6.0, 4.0, 3.0), stream: int = 1) -> Scene:
    """1200x680, fx=fy=600, 1M Gaussians in a 6x4x3 m room (70% planar with
    2 cm noise, 30% volumetric), camera at the room centre."""
    rng = rng_for(stream, agent)
    m = _room_map(n, rng, room)
    return Scene(*m, room_center_pose(room), intr)


def keyframe_ring(n: int = 500_000, views: int = 8, intr: Intrinsics = VGA_INTR):
    """Mapping step: `views` keyframes on a horizontal 1 m circle (45 degree
    spacing), each facing radially outward; n/views Gaussians drawn in each
    keyframe's frustum at 1-5 m. Returns (map Scene for view 0, [viewmats])."""
    rng = rng_for(2, 0)
    center = np.array([0.0, 0.0, 1.5])
    poses = []
    parts = []
    per = n // views
    for k in range(views):
        yaw = 2.0 * math.pi * k / views
        vm = look_outward_pose(center + np.array([math.cos(yaw), math.sin(yaw), 0.0]), yaw)
        poses.append(vm)
        cnt = per if k < views - 1 else n - per * (views - 1)
        parts.append(frustum_scene(cnt, intr, rng, viewmat=vm))
    cat = lambda f: np.ascontiguousarray(np.concatenate([getattr(p, f) for p in parts], axis=-1))
    scene = Scene(cat("means"), cat("scales"), cat("quats"), cat("opacity"), cat("colors"),
                  poses[0].copy(), intr)
    return scene, poses


FOUR_AGENT_SIZES = (200_000, 600_000, 1_200_000, 2_000_000)
FOUR_AGENT_ROOM_SCALE = (1.0, 1.2, 1.4, 1.6)


def four_agent_rooms(sizes=FOUR_AGENT_SIZES, intr: Intrinsics = ROOM_INTR):
    """Batching: one room map per agent with its own seed and room size scaled
    by (1, 1.2, 1.4, 1.6), each rendered at 1200x680 from its room centre."""
    scenes = []
    for a, n in enumerate(sizes):
        s = FOUR_AGENT_ROOM_SCALE[a % len(FOUR_AGENT_ROOM_SCALE)]
        scenes.append(room_view(n=n, agent=a, intr=intr, room=(6.0 * s, 4.0 * s, 3.0 * s), stream=3))
    return scenes


def serving_agents(n_agents: int = 8, nmin: float = 1e5, nmax: float = 3e6, scale: float = 1.0):
    """Serving: agent k keeps a resident room map of exp(U(ln nmin, ln nmax))
    Gaussians (times `scale`); agents 0-3 render 640x480, 4-7 1200x680."""
    rng = rng_for(4, 0, salt=1)
    sizes = np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=n_agents))
    out = []
    for a in range(n_agents):
        n = max(1, int(sizes[a] * scale))
        intr = VGA_INTR if a < n_agents // 2 else ROOM_INTR
        out.append(room_view(n=n, agent=a, intr=intr, stream=4))
    return out


def poisson_trace(n_agents: int, rate_per_agent: float, duration_s: float, seed: int = 4):
    """Arrival times (s) and agent ids of Poisson job streams, one per agent,
    merged in time order; each job is tracking (pose-only gradients) or mapping
    (all gradients) with probability 1/2, and carries a random-walk step index."""
    rng = rng_for(4, 0, salt=seed)
    events = []
    for a in range(n_agents):
        t = 0.0
        k = 0
        while True:
            t += rng.exponential(1.0 / rate_per_agent)
            if t >= duration_s:
                break
            events.append((t, a, k, bool(rng.integers(0, 2))))
            k += 1
    events.sort()
    return events


def gicp_scene(n_src: int = 200_000, seed: int = 0, noise: float = 0.003, deg: float = 0.3, metres: float = 0.005,
               max_dist: float = 4.0):
    """Inputs of the alignment workload: the room map of `room_view`, and
    n_src observed points -- means of the map's visible surface Gaussians
    (in front of the camera, within max_dist) with N(0, noise) jitter,
    expressed in the camera frame and listed in the raster order of the
    pixels they project to, as a depth camera delivers them. Returns (scene,
    src_means [3, n_src] float32 camera frame, T_true [12] camera-to-world
    float32, T0 [12]: T_true moved by `metres` along a random direction and
    `deg` degrees about a random axis, as an initial estimate)."""
    sc = room_view()
    rng = np.random.default_rng(7000 + seed)
    V = sc.viewmat.astype(np.float64).reshape(3, 4)
    R, t = V[:, :3], V[:, 3]
    n_surf = int(0.7 * sc.n)                              # the planar part of the room generator
    p = R @ sc.means[:, :n_surf].astype(np.float64) + t[:, None]
    ok = np.flatnonzero((p[2] > 0.3) & (np.linalg.norm(p, axis=0) < max_dist) &
                        (np.abs(p[0] / p[2]) < 1.0) & (np.abs(p[1] / p[2]) < 0.6))
    pick = rng.choice(ok, size=min(n_src, ok.size), replace=False)
    src = p[:, pick] + rng.normal(0.0, noise, (3, pick.size))
    it = sc.intr                                          # raster order: pixel row, then column
    u = it.fx * src[0] / src[2] + it.cx
    v = it.fy * src[1] / src[2] + it.cy
    src = src[:, np.lexsort((u, np.floor(v)))]
    Tw = np.concatenate([R.T, (-R.T @ t)[:, None]], axis=1)   # camera to world
    ax = rng.standard_normal(3)
    ax /= np.linalg.norm(ax)
    dr = rng.standard_normal(3)
    dr /= np.linalg.norm(dr)
    th = np.deg2rad(deg)
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    Rd = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * (K @ K)
    T0 = np.concatenate([Rd @ Tw[:, :3], (Rd @ Tw[:, 3] + metres * dr)[:, None]], axis=1)
    return (sc, src.astype(np.float32), Tw.reshape(12).astype(np.float32), T0.reshape(12).astype(np.float32))
