"""Candidate selection of the intra-agent consensus (Sec. 3.4, "1) Selection"),
in numpy.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
path. Shares no code with the GPU implementation.

The agent keeps, from its local map, the Gaussians within its current field
of view and within a given distance of its estimated pose. Readings (the
paper names the two criteria and no formula):
  - "within a distance of the pose": the Euclidean distance from the mean to
    the camera centre, which is the norm of the mean in camera coordinates
    p = R mu + t for the world-to-camera pose [R|t]; at most max_dist
    (inclusive);
  - "within the field of view": the mean lies beyond the near plane
    (p_z > near, strict, as the renderer culls) and its pinhole projection
    (u, v) = (fx p_x / p_z + cx, fy p_y / p_z + cy) falls on the image, whose
    pixels are sampled at integer coordinates 0..W-1, 0..H-1, widened by a
    margin of m pixels: -m <= u <= W - 1 + m, likewise v (inclusive);
  - a mean with a non-finite coordinate is never selected;
  - the selected Gaussians keep their map order (an index list);
  - the decisions are integers taken in binary64 from the binary32 inputs
    widened exactly, in one fixed order with no fused operations:
      p_k = ((R_k0 mu_0 + R_k1 mu_1) + R_k2 mu_2) + t_k,
      d2 = (p_0 p_0 + p_1 p_1) + p_2 p_2,  selected needs d2 <= max_dist^2,
      rz = 1 / p_z,  u = fx (p_x rz) + cx,  v = fy (p_y rz) + cy.
"""
import numpy as np


def select_mask(means, viewmat, intr, near_z=0.2, max_dist=3.0, margin=0.0) -> np.ndarray:
    """Boolean [n]: True where the Gaussian is a candidate."""
    mu = np.asarray(means, np.float32).astype(np.float64)
    V = np.asarray(viewmat, np.float32).astype(np.float64).reshape(3, 4)
    p = [((V[k, 0] * mu[0] + V[k, 1] * mu[1]) + V[k, 2] * mu[2]) + V[k, 3] for k in range(3)]
    fx, fy = float(np.float32(intr.fx)), float(np.float32(intr.fy))
    cx, cy = float(np.float32(intr.cx)), float(np.float32(intr.cy))
    near = float(np.float32(near_z))
    dmax = float(np.float32(max_dist))
    m = float(np.float32(margin))
    with np.errstate(all="ignore"):
        finite = np.isfinite(p[0]) & np.isfinite(p[1]) & np.isfinite(p[2])
        d2 = (p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]
        front = p[2] > near
        rz = 1.0 / p[2]
        u = fx * (p[0] * rz) + cx
        v = fy * (p[1] * rz) + cy
        inside = (u >= -m) & (u <= (intr.width - 1) + m) & (v >= -m) & (v <= (intr.height - 1) + m)
    return finite & front & (d2 <= dmax * dmax) & inside


def select(means, viewmat, intr, near_z=0.2, max_dist=3.0, margin=0.0) -> np.ndarray:
    """Indices of the candidates, ascending (map order), int32."""
    return np.flatnonzero(select_mask(means, viewmat, intr, near_z, max_dist, margin)).astype(np.int32)
