"""Shape measurements on phase fields, shared by the oracle pins and the GPU
tests (NumPy only)."""
import math

import numpy as np


def contact_angle(phi, yw=-0.5, ycut=3.0):
    """Contact angle (degrees, through the phi = 1 phase) of a 2D sessile
    droplet on the wall y = yw: circle fit to the phi = 1/2 contour above
    y = ycut, cos(theta) = -(y_centre - yw) / radius."""
    ny, nx = phi.shape
    pts = []
    for j in range(nx):
        for i in range(ny - 1):
            a, b = phi[i, j] - 0.5, phi[i + 1, j] - 0.5
            if a * b < 0:
                pts.append((j, i + a / (a - b)))
    for i in range(ny):
        for j in range(nx - 1):
            a, b = phi[i, j] - 0.5, phi[i, j + 1] - 0.5
            if a * b < 0:
                pts.append((j + a / (a - b), i))
    pts = np.array(pts)
    pts = pts[pts[:, 1] > ycut]
    A = np.c_[2 * pts[:, 0], 2 * pts[:, 1], np.ones(len(pts))]
    cx, cy, c = np.linalg.lstsq(A, (pts ** 2).sum(1), rcond=None)[0]
    r = math.sqrt(c + cx * cx + cy * cy)
    return math.degrees(math.acos(max(-1.0, min(1.0, -(cy - yw) / r))))
