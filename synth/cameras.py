"""Camera builders (inputs only).

A camera is (type, eye, U, V, W, width, height): type 0 = parallel projection, 1 =
perspective (Appendix A of the paper).  Pixel (px, py) maps to u = 2(px+0.5)/width - 1,
v = 2(py+0.5)/height - 1; how rays follow from (eye, U, V, W) is the renderer's job.
Builders here only place the camera relative to a cube of shape (nx, ny, nz), whose
voxel centres sit at integer coordinates 0..n-1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Camera:
    type: int
    eye: tuple
    U: tuple
    V: tuple
    W: tuple
    width: int
    height: int

    def as_f32(self):
        """Same camera with every vector rounded to float32 (what both sides consume)."""
        f = lambda v: tuple(float(np.float32(c)) for c in v)  # noqa: E731
        return Camera(self.type, f(self.eye), f(self.U), f(self.V), f(self.W),
                      self.width, self.height)


def ortho_axis(nx, ny, nz, width, height, axis="+z", distance=10.0):
    """Parallel projection looking along a cube axis, the image covering that face exactly.

    For a 64^3 cube, axis '+z' gives eye = (31.5, 31.5, -10), U = (32,0,0), V = (0,32,0),
    W = (0,0,1).
    """
    c = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    n = (nx, ny, nz)
    sign = 1.0 if axis[0] == "+" else -1.0
    a = "xyz".index(axis[1])
    b, d = [i for i in range(3) if i != a]  # image u along b, v along d
    eye = list(c)
    eye[a] = (-0.5 - distance) if sign > 0 else (n[a] - 0.5 + distance)
    U = [0.0, 0.0, 0.0]
    V = [0.0, 0.0, 0.0]
    W = [0.0, 0.0, 0.0]
    U[b] = n[b] / 2.0
    V[d] = n[d] / 2.0
    W[a] = sign
    return Camera(0, tuple(eye), tuple(U), tuple(V), tuple(W), width, height)


def _basis(forward, up_hint=(0.0, 1.0, 0.0)):
    w = np.asarray(forward, dtype=np.float64)
    w = w / np.linalg.norm(w)
    up = np.asarray(up_hint, dtype=np.float64)
    if abs(float(np.dot(up, w))) > 0.999:
        up = np.array([1.0, 0.0, 0.0])
    u = np.cross(up, w)
    u = u / np.linalg.norm(u)
    v = np.cross(w, u)
    return u, v, w


def perspective_direction(centre, view_dir, distance, fov_y_deg, width, height):
    """Perspective camera at ``centre - distance * view_dir`` looking along ``view_dir``.

    W is the unit forward vector; |V| = tan(fov_y/2), |U| = |V| * width/height, so rays
    through the image edges span the vertical field of view.
    """
    u, v, w = _basis(view_dir)
    t = math.tan(math.radians(fov_y_deg) / 2.0)
    eye = np.asarray(centre, dtype=np.float64) - distance * w
    U = u * t * (width / height)
    V = v * t
    return Camera(1, tuple(eye), tuple(U), tuple(V), tuple(w), width, height)


def perspective_lookat(nx, ny, nz, azimuth_deg, elevation_deg, distance, fov_y_deg,
                       width, height):
    """Orbit camera about the cube centre.  Azimuth 0 / elevation 0 looks along +z (the
    sky-plane view); azimuth turns about the y (Dec) axis; positive elevation raises
    the eye towards +y."""
    c = np.array([(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
    az, el = math.radians(azimuth_deg), math.radians(elevation_deg)
    e = np.array([math.sin(az) * math.cos(el), math.sin(el), -math.cos(az) * math.cos(el)])
    return perspective_direction(c, -e, distance, fov_y_deg, width, height)


def rotation_views(nx, ny, nz, width=1920, height=1080, step_deg=10.0, elevation_deg=20.0,
                   fov_y_deg=40.0, distance=None):
    """Full-rotation protocol: azimuth 0..360 (exclusive) at a fixed elevation; distance
    defaults to twice the half-diagonal of the cube."""
    if distance is None:
        distance = 2.0 * 0.5 * math.sqrt(nx * nx + ny * ny + nz * nz)
    n = int(round(360.0 / step_deg))
    return [perspective_lookat(nx, ny, nz, i * step_deg, elevation_deg, distance, fov_y_deg,
                               width, height) for i in range(n)]
