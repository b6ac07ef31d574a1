"""Brute-force numpy re-derivation of the rasterizer forward pass.

TEST INFRASTRUCTURE ONLY. Written independently of `oracle.cpp` so that the
two can pin each other on tiny scenes (<= 64 Gaussians, <= 32x32 pixels):

  * every pixel is tested against every Gaussian (no buckets, no tiles);
  * the quaternion-to-rotation map is scipy's (an independent library
    routine, with its (x, y, z, w) component order);
  * the conic is numpy's matrix inverse of the 2x2 screen covariance;
  * the pinned decision values (pixel box, depth key, binary32 Mahalanobis
    test) are re-implemented here in numpy with an exact emulation of the
    binary32 fused multiply-add;
  * render(acceptance="plain") drops that recipe altogether: candidates,
    order and per-pixel acceptance come from the plain binary64 definition
    (d^2 <= 9 and o exp(-d^2/2) >= 1/255 from numpy's inverse of the screen
    covariance), so comparing it with the oracle tests the recipe instead of
    restating it.

Compositing follows Eq. 2 of the paper (front-to-back "over"), with the
readings stated in oracle.cpp (alpha clamp 0.99, 3-sigma footprint, 1/255
alpha floor, stop before transmittance falls below 1e-4).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial.transform import Rotation

KAPPA = float.fromhex("0x1.b2da4e9808a53p-1")
Q9 = float.fromhex("0x1.9f7f051d0f35ep+2")
LOG2E = float.fromhex("0x1.71547652b82fep+0")
BOX_SIGMAS = 3.01171875


def fmaf(a, b, c):
    """Correctly rounded binary32 a*b+c for float32 arrays (exact emulation).

    a*b of two binary32 values is exact in binary64. s = fl64(ab + c) with its
    exact error e (TwoSum). Rounding s to binary32 is correct unless s lies
    exactly half-way between two binary32 values and e != 0; then the result
    is the neighbour on the side of e."""
    a = np.asarray(a, np.float32).astype(np.float64)
    b = np.asarray(b, np.float32).astype(np.float64)
    c = np.asarray(c, np.float32).astype(np.float64)
    p = a * b
    s = p + c
    bp = s - c
    e = (p - bp) + (c - (s - bp))
    r = s.astype(np.float32)
    rd = r.astype(np.float64)
    toward = np.where(s > rd, np.inf, -np.inf).astype(np.float32)
    nb = np.nextafter(r, toward)
    mid = (rd + nb.astype(np.float64)) * 0.5
    is_mid = (s == mid) & (s != rd) & (e != 0)
    # at a midpoint, go to the neighbour that lies on the side of e
    up = e > 0
    lo_hi = np.where(rd < nb.astype(np.float64), 1, -1)   # +1 if nb above r
    choose_nb = np.where(up, lo_hi > 0, lo_hi < 0)
    out = np.where(is_mid & choose_nb, nb, r)
    # also: r could sit on the wrong side when s itself is a midpoint and
    # e points back toward r; then r is correct (already handled).
    return out.astype(np.float32)


def pinned_log2(x: float) -> float:
    m, e = math.frexp(x)
    m = m * 2.0
    e = e - 1
    if m > 1.4142135623730951:
        m = m * 0.5
        e = e + 1
    y = (m - 1.0) / (m + 1.0)
    y2 = y * y
    p = 1.0 / 23.0
    for k in range(10, -1, -1):
        p = p * y2 + 1.0 / float(2 * k + 1)
    return float(e) + (2.0 * y * p) * LOG2E


def pinned(scene, near_z=0.2):
    """Pinned recipe, one Gaussian at a time, plain Python floats (binary64,
    no fused operations)."""
    n = scene.n
    V = [float(v) for v in np.asarray(scene.viewmat, np.float32)]
    R = [[V[0], V[1], V[2]], [V[4], V[5], V[6]], [V[8], V[9], V[10]]]
    t = [V[3], V[7], V[11]]
    intr = scene.intr
    fx, fy = float(np.float32(intr.fx)), float(np.float32(intr.fy))
    cx, cy = float(np.float32(intr.cx)), float(np.float32(intr.cy))
    W, H = intr.width, intr.height
    near = float(np.float32(near_z))
    out = []
    for i in range(n):
        mu = [float(scene.means[k, i]) for k in range(3)]
        s = [float(scene.scales[k, i]) for k in range(3)]
        q = [float(scene.quats[k, i]) for k in range(4)]
        o = float(scene.opacity[i])
        rec = dict(visible=False)
        out.append(rec)
        p = [((R[j][0] * mu[0] + R[j][1] * mu[1]) + R[j][2] * mu[2]) + t[j] for j in range(3)]
        if not (p[2] > near) or not all(math.isfinite(v) for v in p):
            continue
        if not math.isfinite(o) or not all(math.isfinite(v) for v in s):
            continue
        if not all(math.isfinite(float(scene.colors[k, i])) for k in range(3)):
            continue
        n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]
        if not (n2 > 0.0) or not math.isfinite(n2):
            continue
        rn = 1.0 / math.sqrt(n2)
        w, x, y, z = q[0] * rn, q[1] * rn, q[2] * rn, q[3] * rn
        xx, yy, zz, xy, xz, yz = x * x, y * y, z * z, x * y, x * z, y * z
        wx, wy, wz = w * x, w * y, w * z
        Rq = [[1.0 - 2.0 * (yy + zz), 2.0 * (xy - wz), 2.0 * (xz + wy)],
              [2.0 * (xy + wz), 1.0 - 2.0 * (xx + zz), 2.0 * (yz - wx)],
              [2.0 * (xz - wy), 2.0 * (yz + wx), 1.0 - 2.0 * (xx + yy)]]
        M = [[Rq[a][b] * s[b] for b in range(3)] for a in range(3)]
        Wm = [[(R[a][0] * M[0][b] + R[a][1] * M[1][b]) + R[a][2] * M[2][b] for b in range(3)] for a in range(3)]
        rz = 1.0 / p[2]
        xn, yn = p[0] * rz, p[1] * rz
        limx = (0.65 * float(W)) / fx
        limy = (0.65 * float(H)) / fy
        xc = min(max(xn, -limx), limx)
        yc = min(max(yn, -limy), limy)
        j00, j02 = fx * rz, -((fx * xc) * rz)
        j11, j12 = fy * rz, -((fy * yc) * rz)
        V0 = [j00 * Wm[0][k] + j02 * Wm[2][k] for k in range(3)]
        V1 = [j11 * Wm[1][k] + j12 * Wm[2][k] for k in range(3)]
        S00 = ((V0[0] * V0[0] + V0[1] * V0[1]) + V0[2] * V0[2]) + 0.3
        S01 = (V0[0] * V1[0] + V0[1] * V1[1]) + V0[2] * V1[2]
        S11 = ((V1[0] * V1[0] + V1[1] * V1[1]) + V1[2] * V1[2]) + 0.3
        if not (S00 <= 4194304.0) or not (S11 <= 4194304.0) or not math.isfinite(S01):
            continue
        u = fx * xn + cx
        v = fy * yn + cy
        if not (abs(u) <= 4194304.0) or not (abs(v) <= 4194304.0):
            continue
        rx = math.ceil(BOX_SIGMAS * math.sqrt(S00))
        ry = math.ceil(BOX_SIGMAS * math.sqrt(S11))
        xlo, xhi = math.ceil(u - rx), math.floor(u + rx)
        ylo, yhi = math.ceil(v - ry), math.floor(v + ry)
        if not (xlo <= W - 1 and xhi >= 0 and ylo <= H - 1 and yhi >= 0):
            continue
        det = S00 * S11 - S01 * S01
        if not (det > 0.0):
            continue
        z32 = np.float32(p[2])
        if not np.isfinite(z32):
            continue
        sd, s11 = math.sqrt(det), math.sqrt(S11)
        l11, l12, l22 = s11 / sd, -S01 / (sd * s11), 1.0 / s11
        uf0, vf0 = math.floor(u), math.floor(v)
        lo255 = 255.0 * o
        qc = min(Q9, pinned_log2(lo255)) if lo255 > 0.0 else -math.inf
        rec.update(visible=True, zkey=int(z32.view(np.uint32)), z32=z32,
                   xlo=max(xlo, 0), xhi=min(xhi, W - 1), ylo=max(ylo, 0), yhi=min(yhi, H - 1),
                   ui=int(uf0), vi=int(vf0), uf=np.float32(u - uf0), vf=np.float32(v - vf0),
                   a=np.float32(KAPPA * l11), b=np.float32(KAPPA * l12), c=np.float32(KAPPA * l22),
                   qcut=np.float32(qc), xlo_raw=xlo, xhi_raw=xhi, ylo_raw=ylo, yhi_raw=yhi)
    return out


def pinned_q(rec, x, y):
    """Binary32 Mahalanobis test value at integer pixels x, y (arrays)."""
    dx = (np.asarray(x - rec["ui"]).astype(np.float32) - rec["uf"]).astype(np.float32)
    dy = (np.asarray(y - rec["vi"]).astype(np.float32) - rec["vf"]).astype(np.float32)
    t1 = fmaf(rec["a"], dx, (rec["b"] * dy).astype(np.float32))
    t2 = (rec["c"] * dy).astype(np.float32)
    return fmaf(t1, t1, (t2 * t2).astype(np.float32))


def continuous(scene):
    """Continuous projection from the definition: scipy rotation, numpy
    matrix products and inverse. Returns per-Gaussian dicts."""
    V = np.asarray(scene.viewmat, np.float64).reshape(3, 4)
    R, t = V[:, :3], V[:, 3]
    intr = scene.intr
    fx, fy = float(np.float32(intr.fx)), float(np.float32(intr.fy))
    cx, cy = float(np.float32(intr.cx)), float(np.float32(intr.cy))
    q = scene.quats.astype(np.float64)
    rot = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], axis=1)).as_matrix()
    out = []
    for i in range(scene.n):
        mu = scene.means[:, i].astype(np.float64)
        s = scene.scales[:, i].astype(np.float64)
        Rq = rot[i]
        Sigma = Rq @ np.diag(s * s) @ Rq.T
        p = R @ mu + t
        X, Y, Z = p
        limx = 0.65 * intr.width / fx
        limy = 0.65 * intr.height / fy
        xt = Z * min(max(X / Z, -limx), limx)
        yt = Z * min(max(Y / Z, -limy), limy)
        J = np.array([[fx / Z, 0.0, -fx * xt / Z ** 2], [0.0, fy / Z, -fy * yt / Z ** 2]])
        Sp = J @ (R @ Sigma @ R.T) @ J.T + 0.3 * np.eye(2)
        out.append(dict(p=p, Sp=Sp, conic=np.linalg.inv(Sp), u=fx * X / Z + cx, v=fy * Y / Z + cy))
    return out


PLAIN_MARGIN = 1e-5   # relative closeness to a threshold that makes a plain decision ambiguous


def plain_accept(c, opacity, x, y):
    """The plain definition of "Gaussian counts at pixel (x, y)", in binary64
    from the continuous projection: d^2 <= 9 and o exp(-d^2 / 2) >= 1/255,
    d^2 = (p - mu')^T Sigma'^-1 (p - mu'). Returns (accepted, ambiguous):
    ambiguous when d^2 lies within PLAIN_MARGIN (relative) of 9, or
    o exp(-d^2 / 2) within PLAIN_MARGIN of 1/255."""
    dx, dy = np.asarray(x, np.float64) - c["u"], np.asarray(y, np.float64) - c["v"]
    Q = c["conic"]
    d2 = Q[0, 0] * dx * dx + 2.0 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
    at = opacity * np.exp(-0.5 * d2)
    acc = (d2 <= 9.0) & (at >= 1.0 / 255.0)
    amb = (np.abs(d2 - 9.0) <= PLAIN_MARGIN * 9.0) | (np.abs(at * 255.0 - 1.0) <= PLAIN_MARGIN)
    return acc, amb


def render(scene, near_z=0.2, acceptance="recipe"):
    """Per-pixel brute force: every pixel against every Gaussian. Returns
    rgb [3,H,W], depth, sil, tfinal, ncomp.

    acceptance="recipe": visibility, order and the per-pixel test follow the
    pinned binary32 recipe (depth key, then index; q <= qcut inside the pixel
    box). acceptance="plain": they follow the definition alone, in binary64:
    a Gaussian is a candidate when its mean lies beyond the near plane with
    finite attributes and a non-zero quaternion, candidates are visited by
    (binary64 camera depth, index), and one counts at a pixel by
    plain_accept. The result then also holds `ambiguous`, the pixels where
    some candidate's decision lies within PLAIN_MARGIN of its threshold."""
    if acceptance not in ("recipe", "plain"):
        raise ValueError(acceptance)
    plain = acceptance == "plain"
    pins = pinned(scene, near_z)
    cont = continuous(scene)
    W, H = scene.intr.width, scene.intr.height
    if plain:
        near = float(np.float32(near_z))
        cand = []
        for i in range(scene.n):
            p = cont[i]["p"]
            attrs = np.concatenate([scene.scales[:, i], scene.colors[:, i], [scene.opacity[i]]])
            if (p[2] > near and np.all(np.isfinite(p)) and np.all(np.isfinite(attrs))
                    and np.any(scene.quats[:, i] != 0) and np.all(np.isfinite(cont[i]["conic"]))):
                cand.append(i)
        order = sorted(cand, key=lambda i: (cont[i]["p"][2], i))
        ys, xs = np.mgrid[0:H, 0:W]
        dec = {i: plain_accept(cont[i], float(scene.opacity[i]), xs, ys) for i in order}
        ambiguous = np.zeros((H, W), bool)
        for i in order:
            ambiguous |= dec[i][1]
    else:
        order = sorted([i for i in range(scene.n) if pins[i]["visible"]], key=lambda i: (pins[i]["zkey"], i))
    rgb = np.zeros((3, H, W))
    depth = np.zeros((H, W))
    tfin = np.ones((H, W))
    ncomp = np.zeros((H, W), np.int32)
    for y in range(H):
        for x in range(W):
            T = 1.0
            C = np.zeros(3)
            D = 0.0
            k = 0
            for i in order:
                if plain:
                    if not dec[i][0][y, x]:
                        continue
                else:
                    r = pins[i]
                    if not (r["xlo"] <= x <= r["xhi"] and r["ylo"] <= y <= r["yhi"]):
                        continue
                    if not (pinned_q(r, x, y) <= r["qcut"]):
                        continue
                c = cont[i]
                d = np.array([x - c["u"], y - c["v"]])
                pw = -0.5 * float(d @ c["conic"] @ d)
                alpha = min(0.99, float(scene.opacity[i]) * math.exp(pw))
                Tn = T * (1.0 - alpha)
                if Tn < 1e-4:
                    break
                C += scene.colors[:, i].astype(np.float64) * alpha * T
                D += c["p"][2] * alpha * T
                T = Tn
                k += 1
            rgb[:, y, x] = C
            depth[y, x] = D
            tfin[y, x] = T
            ncomp[y, x] = k
    out = dict(rgb=rgb, depth=depth, sil=1.0 - tfin, tfinal=tfin, ncomp=ncomp, pinned=pins, cont=cont)
    if plain:
        out["ambiguous"] = ambiguous
    return out
