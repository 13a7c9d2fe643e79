"""Design parameters mapped to porosity (the optimisation routine of Sec. 4).

``BoxDesign`` moves and raises buildings and sets the trees' porosity:
parameter 3b is the height change of building b, 3b + 1 and 3b + 2 its
shift along x and y; the last parameter is the porosity shared by all
trees.  The porosity field comes from ``uf_smooth_porosity`` (logistic
steps of a given width across object faces), so the objective varies
continuously with every parameter, on the GPU; ``gradient`` chains a
porosity gradient back to the parameters through its reverse.
"""
import numpy as np

from .voxelize import smooth_porosity, smooth_porosity_grad


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

    def gradient(self, theta, phibar):
        """dJ/dtheta from phibar = dJ/dphi (float64 [nx, ny, nz] on the GPU):
        the reverse of the smoothed map (uf_smooth_porosity_grad), then of
        the parameter shifts in ``objects``."""
        theta = np.asarray(theta, np.float64)
        b, c = self.objects(theta)
        gb, gc = smooth_porosity_grad(self.n, self.h, b, c, self.width, phibar)
        g = np.zeros(self.nparams)
        nb = len(b)
        g[0:3 * nb:3] = gb[:, 5]
        g[1:3 * nb:3] = gb[:, 0] + gb[:, 1]
        g[2:3 * nb:3] = gb[:, 2] + gb[:, 3]
        if len(c) and 0.0 <= theta[-1] <= 1.0:
            g[-1] = gc[:, 5].sum()
        return g
