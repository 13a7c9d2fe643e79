"""Design parameters mapped to porosity (the optimisation routine of Sec. 4).

``BoxDesign`` moves and raises buildings and sets the trees' porosity:
parameter 3b is the height change of building b, 3b + 1 and 3b + 2 its
shift along x and y; the last parameter is the porosity shared by all
trees.  The porosity field comes from ``uf_smooth_porosity`` (logistic
steps of a given width across object faces), so the objective varies
continuously with every parameter, on the GPU.
"""
import numpy as np

from .voxelize import smooth_porosity


class BoxDesign:
    def __init__(self, n, h, boxes, cylinders, width, dtype="f32", device="cuda:0"):
        """boxes: rows (x0, x1, y0, y1, z0, z1, phi); cylinders: rows
        (cx, cy, R, z0, z1, phi) -- the design at zero parameters (the tree
        porosity parameter starts at the trees' first porosity)."""
        self.n, self.h, self.width = tuple(n), tuple(h), float(width)
        self.boxes = np.asarray(boxes, np.float64).reshape(-1, 7)
        self.cylinders = np.asarray(cylinders, np.float64).reshape(-1, 6)
        self.dtype, self.device = dtype, device

    @property
    def nparams(self):
        return 3 * len(self.boxes) + 1

    def initial(self):
        t = np.zeros(self.nparams)
        t[-1] = self.cylinders[0, 5] if len(self.cylinders) else 0.5
        return t

    def objects(self, theta):
        theta = np.asarray(theta, np.float64)
        b = self.boxes.copy()
        d = theta[:3 * len(b)].reshape(-1, 3)
        b[:, 5] += d[:, 0]
        b[:, 0:2] += d[:, 1:2]
        b[:, 2:4] += d[:, 2:3]
        c = self.cylinders.copy()
        if len(c):
            c[:, 5] = min(max(theta[-1], 0.0), 1.0)
        return b, c

    def porosity(self, theta):
        b, c = self.objects(theta)
        return smooth_porosity(self.n, self.h, b, c, self.width, self.dtype, self.device)
