"""Hand-built test configurations (inputs only): a big floor triangle,
walls, ceilings, plates, and receiver grids lying on the floor."""
import numpy as np

import workloads as w

FLOOR = (np.array([[-100.0, 0.0, -100.0], [300.0, 0.0, -100.0], [-100.0, 0.0, 300.0]]),
         np.array([[0, 1, 2]], dtype=np.int64))


def build(parts):
    V, F = w._merge(parts)
    return w.Scene(V, F)


def wall_x(x, y0=0.0, y1=50.0, z0=-50.0, z1=50.0):
    """Vertical quad in the plane X = x."""
    return w.quad((x, y0, z0), (0.0, y1 - y0, 0.0), (0.0, 0.0, z1 - z0))


def plate_y(y, x0, x1, z0, z1):
    """Horizontal quad at height y over [x0,x1] x [z0,z1]."""
    return w.quad((x0, y, z0), (x1 - x0, 0.0, 0.0), (0.0, 0.0, z1 - z0))


def floor_grid(nx, nz, spacing, x0=0.0, z0=0.0):
    """Receivers on the floor (prim 0 = the floor triangle), normal up."""
    return w.plane_gbuffer(nx, nz, spacing, origin=(x0, 0.0, z0), prim=0)


def lambert_polygon_ff(p, n, verts):
    """Lambert's point-to-polygon form factor (Lambertian receiver at p with
    normal n, polygon vertices in order): (1/2pi) sum theta_i n.unit(a_i x b_i)."""
    p = np.asarray(p, np.float64)
    n = np.asarray(n, np.float64)
    total = 0.0
    m = len(verts)
    for i in range(m):
        a = np.asarray(verts[i], np.float64) - p
        b = np.asarray(verts[(i + 1) % m], np.float64) - p
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        c = np.cross(a, b)
        theta = np.arctan2(np.linalg.norm(c), np.dot(a, b))
        total += theta * np.dot(n, c / np.linalg.norm(c))
    return abs(total) / (2.0 * np.pi)


def polygon_fan(center, verts):
    """Triangle fan of a convex polygon around its centre."""
    c = np.asarray(center, np.float64)
    V = np.vstack([c[None, :], np.asarray(verts, np.float64)])
    m = len(verts)
    F = np.array([[0, 1 + i, 1 + (i + 1) % m] for i in range(m)], dtype=np.int64)
    return V, F
