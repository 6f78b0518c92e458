"""Workload descriptions (shapes, boundary data, partition, seeds).

Each workload is a plain record of arrays and parameters.  Sides of the domain
are numbered 0..2d-1 as (-x, +x, -y, +y, -z, +z); boundary values are given per
boundary face, in the x-fastest order of the cells adjacent to that side.

Recipes (synthetic stand-ins for the paper's fields, Section 5):

* ``c1``: 64x64 unit square, 4x4 subdomains of 16x16 cells, overlap 2,
  piecewise-constant interface spaces, constant Robin parameter 1, Gaussian
  log K (sigma^2 = 1, correlation 0.1, seed 1), p = 1 on x = 0, p = 0 on x = 1,
  no flow on y = 0, 1, 2 smoothing steps.
* ``c2``: 256x256, subdomains of 16x16, overlap 0, 2 or 4, piecewise-linear
  spaces, Gaussian log K (sigma^2 = 4, correlation 0.05, seed 2), no flow on
  all sides with a unit injector in the first cell and a unit producer in the
  last cell (quarter five-spot), alpha = 1, 5 smoothing steps.
* ``c3``: 1024x1024, subdomains of 16x16, overlap 4, piecewise-constant,
  binary channels (contrast 1e4, widths 4-12 cells, seed 3), p = 1 / 0 on the
  x faces, alpha = 1, 10 smoothing steps.
* ``c4``: 64x224x80 cubic cells (h = 1/64), subdomains of 4^3, overlap 2,
  piecewise-constant, layered Gaussian log K (sigma^2 = 5, correlations
  (0.2, 0.2, 0.02), clipped to contrast 1e6, seed 4), p = 1 / 0 on the x faces,
  alpha = 1, 3 smoothing steps.
* ``c5``: one member of a batch of 256x256 fields (sigma^2 = 2, correlation
  0.05, seed 100 + member), subdomains of 16x16, overlap 2, piecewise-constant,
  p = 1 / 0 on the x faces, alpha = 1, 5 smoothing steps.

Every recipe accepts a ``scale`` divisor for the number of subdomains per axis
so that tests can run the same recipe on a smaller grid.
"""
from dataclasses import dataclass, field, replace
import numpy as np

from .fields import gaussian_logk, channel_logk, layered_logk


@dataclass
class Workload:
    name: str
    dim: int
    ncell: tuple            # cells per axis, axis 0 = x
    h: float                # cell size (cubic cells)
    logk: np.ndarray        # numpy shape ncell[::-1]
    source: np.ndarray      # source density f per cell, same shape
    bc_type: tuple          # per side: "D" (pressure) or "N" (normal velocity)
    bc_value: list          # per side: 1-D array over that side's faces
    sub: tuple              # cells per subdomain per axis
    overlap: int            # oversampling width l (cells)
    space: str              # "const" | "linear" | "fine"
    beta_mode: str          # "alpha" (beta = alpha H / K_H) or "const"
    beta_mbf: float         # alpha (or beta) for the basis functions
    beta_smooth: float      # alpha (or beta) for the smoothing steps
    nsmooth: int            # number of smoothing steps
    meta: dict = field(default_factory=dict)
    # diagonal permeability tensor: log K per axis, shape (dim, *ncell[::-1])
    # (row a: the entry of axis a); None for scalar K (logk)
    logk_axes: np.ndarray = None

    @property
    def ncells(self):
        return int(np.prod(self.ncell))

    @property
    def perm(self):
        """K per cell, or (dim, cells) per axis for a diagonal tensor."""
        if self.logk_axes is not None:
            return np.exp(np.asarray(self.logk_axes)).reshape(self.dim, -1)
        return np.exp(self.logk)

    def with_tensor(self, log_ratio):
        """The same workload with a diagonal tensor: axis a's log K is logk
        plus log_ratio[a] (an array of the grid's shape, or a number)."""
        ax = np.stack([np.asarray(self.logk) + np.broadcast_to(np.asarray(r, dtype=np.float64),
                                                                np.shape(self.logk))
                       for r in log_ratio])
        return replace(self, logk_axes=ax)

    def with_(self, **kw):
        return replace(self, **kw)


def side_shape(ncell, side):
    a = side // 2
    return tuple(n for b, n in enumerate(ncell) if b != a)


def _bc(ncell, types, values):
    out = []
    for s, (t, v) in enumerate(zip(types, values)):
        n = int(np.prod(side_shape(ncell, s)))
        out.append(np.full(n, float(v)))
    return list(types), out


def _dirichlet_x(ncell):
    d = len(ncell)
    types = ["D", "D"] + ["N"] * (2 * d - 2)
    values = [1.0, 0.0] + [0.0] * (2 * d - 2)
    return _bc(ncell, types, values)


def make_workload(name, scale=1, overlap=None, space=None, seed=None,
                  nsmooth=None, member=0):
    """Build a workload by recipe name ("c1".."c5", "homog", "linear")."""
    if name == "c1":
        m = max(1, 4 // scale)
        ncell = (16 * m, 16 * m)
        h = 1.0 / ncell[0]
        y = gaussian_logk(ncell, h, 1.0, 0.1, 1 if seed is None else seed)
        types, vals = _dirichlet_x(ncell)
        w = Workload("c1", 2, ncell, h, y, np.zeros_like(y), tuple(types), vals,
                     (16, 16), 2, "const", "const", 1.0, 1.0, 2)
    elif name == "c2":
        m = max(1, 16 // scale)
        ncell = (16 * m, 16 * m)
        h = 1.0 / ncell[0]
        y = gaussian_logk(ncell, h, 4.0, 0.05, 2 if seed is None else seed)
        f = np.zeros_like(y)
        f[0, 0] = 1.0 / h ** 2
        f[-1, -1] = -1.0 / h ** 2
        types, vals = _bc(ncell, ["N"] * 4, [0.0] * 4)
        w = Workload("c2", 2, ncell, h, y, f, tuple(types), vals,
                     (16, 16), 4, "linear", "alpha", 1.0, 1.0, 5)
    elif name == "c3":
        m = max(1, 64 // scale)
        ncell = (16 * m, 16 * m)
        h = 1.0 / ncell[0]
        nch = max(1, int(round(30 * m / 64)))
        y = channel_logk(ncell[0], ncell[1], 3 if seed is None else seed,
                         n_channels=nch)
        types, vals = _dirichlet_x(ncell)
        w = Workload("c3", 2, ncell, h, y, np.zeros_like(y), tuple(types), vals,
                     (16, 16), 4, "const", "alpha", 1.0, 1.0, 10)
    elif name == "c4":
        mx, my, mz = max(1, 16 // scale), max(1, 56 // scale), max(1, 20 // scale)
        ncell = (4 * mx, 4 * my, 4 * mz)
        h = 1.0 / 64
        y = layered_logk(ncell, h, 5.0, (0.2, 0.2, 0.02),
                         4 if seed is None else seed, 1e6)
        types, vals = _dirichlet_x(ncell)
        w = Workload("c4", 3, ncell, h, y, np.zeros_like(y), tuple(types), vals,
                     (4, 4, 4), 2, "const", "alpha", 1.0, 1.0, 3)
    elif name == "c5":
        m = max(1, 16 // scale)
        ncell = (16 * m, 16 * m)
        h = 1.0 / ncell[0]
        y = gaussian_logk(ncell, h, 2.0, 0.05,
                          (100 + member) if seed is None else seed)
        types, vals = _dirichlet_x(ncell)
        w = Workload("c5", 2, ncell, h, y, np.zeros_like(y), tuple(types), vals,
                     (16, 16), 2, "const", "alpha", 1.0, 1.0, 5)
    elif name == "homog":
        # constant K, f = 8 pi^2 cos(2 pi x) cos(2 pi y), no flow (Section 5)
        m = max(1, 4 // scale)
        ncell = (20 * m, 20 * m)
        h = 1.0 / ncell[0]
        xc = (np.arange(ncell[0]) + 0.5) * h
        f = 8 * np.pi ** 2 * np.cos(2 * np.pi * xc)[None, :] * np.cos(2 * np.pi * xc)[:, None]
        y = np.zeros((ncell[1], ncell[0]))
        types, vals = _bc(ncell, ["N"] * 4, [0.0] * 4)
        w = Workload("homog", 2, ncell, h, y, f, tuple(types), vals,
                     (20, 20), 2, "linear", "alpha", 1.0, 1.0, 2)
    else:
        raise KeyError(name)
    kw = {}
    if overlap is not None:
        kw["overlap"] = overlap
    if space is not None:
        kw["space"] = space
    if nsmooth is not None:
        kw["nsmooth"] = nsmooth
    return w.with_(**kw) if kw else w


WORKLOADS = ("c1", "c2", "c3", "c4", "c5", "homog")
