"""Pinhole camera: pixel-centre unprojection and perspective projection.

Oracle code (test infrastructure only).

The paper un-projects a pixel's world position from the depth buffer and
projects marched points back to the screen (Sec. 3.3; Appendix D,
Algorithm 1) without fixing conventions.  Reading taken: view coordinates
X = (x-c).right, Y = (x-c).up, Z = (x-c).forward with Z the stored linear
depth; px = cx + fx*X/Z, py = cy - fy*Y/Z with row 0 on top; pixel (i, j)
covers [i, i+1) x [j, j+1) and is un-projected at its centre.
"""

import numpy as np


def unpack(cam):
    """Camera dict -> float64 pieces."""
    rot = np.asarray(cam["rot"], np.float64).reshape(3, 3)
    return dict(W=int(cam["width"]), H=int(cam["height"]),
                pos=np.asarray(cam["pos"], np.float64), right=rot[0], up=rot[1], fwd=rot[2],
                fx=float(cam["fx"]), fy=float(cam["fy"]), cx=float(cam["cx"]),
                cy=float(cam["cy"]), z_near=float(cam["z_near"]))


def pixel_view_point(c, i, j, depth):
    """View-space point of pixel centre (i+1/2, j+1/2) at linear depth ``depth``."""
    X = (i + 0.5 - c["cx"]) * depth / c["fx"]
    Y = -(j + 0.5 - c["cy"]) * depth / c["fy"]
    return np.stack([X, Y, depth], axis=-1)


def view_to_world_dir(c, v):
    return v[..., 0:1] * c["right"] + v[..., 1:2] * c["up"] + v[..., 2:3] * c["fwd"]


def world_to_view_dir(c, d):
    return np.stack([d @ c["right"], d @ c["up"], d @ c["fwd"]], axis=-1)


def project(c, v):
    """Screen coordinates (px, py) of view-space points ``v[..., 3]``."""
    return (c["cx"] + c["fx"] * v[..., 0] / v[..., 2],
            c["cy"] - c["fy"] * v[..., 1] / v[..., 2])


def view_ray_dir(c, i, j):
    """Unit world direction from the camera through pixel centre (i, j)."""
    v = np.stack([(i + 0.5 - c["cx"]) / c["fx"], -(j + 0.5 - c["cy"]) / c["fy"],
                  np.ones(np.shape(i))], axis=-1)
    d = view_to_world_dir(c, v)
    return d / np.linalg.norm(d, axis=-1, keepdims=True)
