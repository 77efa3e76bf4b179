"""Staggered (MAC) grid of the paper (Sec. 2.2; wall-normal stretching along z, the
solver's non-uniform direction, which the paper calls y).  Test infrastructure only.

Indices: cells i = 0..nx-1, j = 0..ny-1 (periodic), k = 1..nz with ghost planes
k = 0 and k = nz + 1.  With walls in y as well (the square duct of Sec. 4.4) the arrays
carry two ghost rows, stored after the interior ones: row ny is the ghost above y = ly and
row ny + 1 the ghost below y = 0.  Row ny + 1 is where the periodic index j - 1 of row 0
lands, so the periodic difference operators give the wall-bounded ones on every interior
row once the ghost rows hold the boundary values; nys = ny + 2 is the stored row count.
The y spacing is uniform; v at row j sits at (j + 1) dy, so row ny - 1 of v is the wall
face y = ly and the ghost row ny + 1 is the wall face y = 0.  zf[k] is the top face of cell k (zf[0] = 0, zf[nz] = lz),
zc[k] the centre, dzf[k] = zf[k] - zf[k-1] the cell height, dzc[k] = zc[k+1] - zc[k]
the distance between centres k and k+1 (k = 0..nz).
"""
import numpy as np


def tanh_faces(nz, lz, beta):
    """R1 (the paper names tanh clustering only through its tables): faces
    zf(k) = (lz/2) [1 + tanh(beta (2k/nz - 1)) / tanh(beta)], made exactly
    mirror-symmetric: for k < nz/2 the upper face is b = fl(lz - zf(k)) and the lower face
    is reset to lz - b, which is exact (Sterbenz, since lz/2 <= b <= lz), so that
    zf(nz - k) = lz - zf(k) and zf(k) = lz - zf(nz - k) both hold bitwise."""
    zf = np.empty(nz + 1)
    for k in range(nz + 1):
        zf[k] = 0.5 * lz * (1.0 + np.tanh(beta * (2.0 * k / nz - 1.0)) / np.tanh(beta))
    for k in range((nz + 1) // 2):
        b = lz - zf[k]
        zf[nz - k] = b
        zf[k] = lz - b
    zf[0] = 0.0
    zf[nz] = lz
    if nz % 2 == 0:
        zf[nz // 2] = 0.5 * lz
    return zf


class Grid:
    """Metric arrays in float64; all plain loops so each value can be read off."""

    def __init__(self, case):
        nx, ny, nz = case.nx, case.ny, case.nz
        self.nx, self.ny, self.nz = nx, ny, nz
        self.lx, self.ly, self.lz = case.lx, case.ly, case.lz
        self.dx = case.lx / nx
        self.dy = case.ly / ny
        self.periodic_z = case.zperiodic
        self.ywalls = case.ywalls
        self.nys = ny + 2 if self.ywalls else ny
        self.yc = np.array([(j + 0.5) * self.dy for j in range(ny)])
        if case.beta > 0.0 and not case.zperiodic:
            zf = tanh_faces(nz, case.lz, case.beta)
        else:
            zf = np.array([case.lz * k / nz for k in range(nz + 1)])
        self.zf = zf
        zc = np.zeros(nz + 2)
        dzf = np.zeros(nz + 2)
        for k in range(1, nz + 1):
            zc[k] = 0.5 * (zf[k - 1] + zf[k])
            dzf[k] = zf[k] - zf[k - 1]
        if self.periodic_z:
            zc[0] = zc[nz] - case.lz
            zc[nz + 1] = zc[1] + case.lz
            dzf[0] = dzf[nz]
            dzf[nz + 1] = dzf[1]
        else:
            zc[0] = -zc[1]                      # ghost centre mirrored about the wall
            zc[nz + 1] = 2.0 * case.lz - zc[nz]
            dzf[0] = dzf[1]
            dzf[nz + 1] = dzf[nz]
        dzc = np.zeros(nz + 1)
        for k in range(nz + 1):
            dzc[k] = zc[k + 1] - zc[k]
        self.zc, self.dzf, self.dzc = zc, dzf, dzc

    def wall_distance(self):
        """Distance of each interior cell centre (k = 1..nz) to the nearer wall."""
        zc = self.zc[1:self.nz + 1]
        return np.minimum(zc, self.lz - zc)

    def delta(self):
        """R5: filter width (dx dy dzf_k)^(1/3) per interior plane (not defined in the paper)."""
        return (self.dx * self.dy * self.dzf[1:self.nz + 1]) ** (1.0 / 3.0)
