"""Closed-form test scenes shared by the oracle pins and the GPU tests.

G-buffers are built here by exact ray casting of one or two planes, so the
expected answers (hit pixels, furnace values) follow from geometry alone.
"""

import numpy as np

def floor_wall_scene(w=64, h=64, wall_z=-6.0, cam_h=1.0):
    """Camera at height cam_h looking along -z at a mirror floor y=0 and a
    fronto-parallel wall z=wall_z.  G-buffers by exact ray casting here."""
    cam = dict(width=w, height=h, pos=np.array([0.0, cam_h, 0.0]),
               rot=np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, -1.0]]),
               fx=w * 0.8, fy=w * 0.8, cx=w / 2, cy=h / 2, z_near=0.01)
    fx = fy = w * 0.8
    cx, cy = w / 2, h / 2
    jj, ii = np.meshgrid(np.arange(h, dtype=float), np.arange(w, dtype=float), indexing="ij")
    x = (ii + 0.5 - cx) / fx
    y = -(jj + 0.5 - cy) / fy
    t_floor = np.where(y < 0, -cam_h / np.where(y < 0, y, -1), np.inf)
    t_wall = -wall_z
    is_floor = t_floor < t_wall
    depth = np.where(is_floor, t_floor, t_wall)
    nr = np.zeros((h, w, 4))
    am = np.zeros((h, w, 4))
    nr[is_floor] = [0, 1, 0, 0.0]            # mirror floor
    am[is_floor] = [1, 1, 1, 1.0]
    nr[~is_floor] = [0, 0, 1, 0.7]           # rough dielectric wall
    am[~is_floor] = [0.5, 0.5, 0.5, 0.0]
    rad = np.zeros((h, w, 4))
    rad[..., 0] = np.arange(h * w).reshape(h, w) + 1.0   # identifies the pixel
    rad[..., 1] = 1.0
    rad[..., 2] = 2.0
    return cam, dict(depth=depth, normal_rough=nr, albedo_metal=am, radiance=rad), is_floor


def open_floor(w=48, h=32, rough=0.0, metal=1.0, albedo=1.0):
    """Camera looking down at an unbounded floor and nothing else."""
    cam = dict(width=w, height=h, pos=np.array([0.0, 3.0, 0.0]),
               rot=np.array([[1.0, 0, 0], [0, 0, -1.0], [0, -1.0, 0]]),
               fx=w * 0.6, fy=w * 0.6, cx=w / 2, cy=h / 2, z_near=0.01)
    depth = np.full((h, w), 3.0)
    nr = np.tile([0, 1.0, 0, rough], (h, w, 1))
    am = np.tile([albedo, albedo, albedo, metal], (h, w, 1))
    rad = np.tile([5.0, 6.0, 7.0, 0], (h, w, 1))
    return cam, dict(depth=depth, normal_rough=nr, albedo_metal=am, radiance=rad)


