"""Seeded initial fields (see the package docstring for the array convention).

Random draws use numpy's PCG64 generator seeded by the caller, so the CPU
oracle and the GPU path always start from bit-identical inputs.
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _empty(nx, ny, nz):
    return np.zeros((nz + 2, ny, nx))


def isotropic_field(n, seed, k0=4.0, urms=1.0, length=2 * np.pi):
    """Triply periodic random velocity with energy spectrum E(k) ~ k^4 exp(-2 (k/k0)^2).

    Gaussian complex amplitudes on integer wavevectors with 1 <= |k| and
    every |k_i| < n/2 (Nyquist excluded), |u_hat|^2 ~ E(|k|)/(4 pi |k|^2),
    made solenoidal in the continuous sense (u_hat . k = 0), evaluated at
    each component's own face positions, then scaled so that
    sqrt(<u^2 + v^2 + w^2>/3) = urms.  No discrete projection is applied.
    Returns (u, v, w) in the ghosted layout with zero ghost planes.
    """
    rng = _rng(seed)
    kint = np.fft.fftfreq(n, 1.0 / n)                 # integer wavenumbers
    kz, ky, kx = np.meshgrid(kint, kint, kint, indexing="ij")
    kk = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    keep = (kk >= 1.0) & (np.abs(kx) < n / 2) & (np.abs(ky) < n / 2) & (np.abs(kz) < n / 2)
    amp = np.zeros_like(kk)
    e = kk[keep] ** 4 * np.exp(-2.0 * (kk[keep] / k0) ** 2)
    amp[keep] = np.sqrt(e / (4.0 * np.pi * kk[keep] ** 2))
    hat = []
    for _ in range(3):
        re = rng.standard_normal(kk.shape)
        im = rng.standard_normal(kk.shape)
        hat.append(amp * (re + 1j * im))
    ux, uy, uz = hat
    kk2 = np.where(kk > 0, kk ** 2, 1.0)
    kdotu = (kx * ux + ky * uy + kz * uz) / kk2
    ux, uy, uz = ux - kx * kdotu, uy - ky * kdotu, uz - kz * kdotu
    h = length / n
    kscale = 2 * np.pi / length

    def at(hatc, sx, sy, sz):
        ph = np.exp(1j * kscale * (kx * sx + ky * sy + kz * sz))
        return np.real(np.fft.ifftn(hatc * ph)) * n ** 3

    # positions relative to (i dx, j dy, k dz): u face (1, 1/2, 1/2) etc.
    u = at(ux, 1.0 * h, 0.5 * h, 0.5 * h)
    v = at(uy, 0.5 * h, 1.0 * h, 0.5 * h)
    w = at(uz, 0.5 * h, 0.5 * h, 1.0 * h)
    s = urms / np.sqrt((np.mean(u ** 2) + np.mean(v ** 2) + np.mean(w ** 2)) / 3.0)
    out = []
    for f in (u, v, w):
        g = _empty(n, n, n)
        g[1:n + 1] = s * f
        out.append(g)
    return tuple(out)


def channel_field(nx, ny, nz, zc, seed, ubulk=1.0, noise=0.1, half_height=1.0):
    """Laminar Poiseuille profile plus seeded uniform noise.

    u = 1.5 U_b (1 - (z/h - 1)^2) + noise U_b (2 xi - 1), v = w = noise U_b (2 xi - 1)
    with xi ~ U[0, 1).  zc holds the cell-centre heights of planes 0..nz+1;
    w at the two wall faces (planes 0 and nz) is zero.
    """
    rng = _rng(seed)
    u, v, w = _empty(nx, ny, nz), _empty(nx, ny, nz), _empty(nx, ny, nz)
    z = np.asarray(zc, dtype=np.float64)[1:nz + 1] / half_height
    prof = 1.5 * ubulk * (1.0 - (z - 1.0) ** 2)
    u[1:nz + 1] = prof[:, None, None] + noise * ubulk * (2.0 * rng.random((nz, ny, nx)) - 1.0)
    v[1:nz + 1] = noise * ubulk * (2.0 * rng.random((nz, ny, nx)) - 1.0)
    w[1:nz + 1] = noise * ubulk * (2.0 * rng.random((nz, ny, nx)) - 1.0)
    w[nz] = 0.0
    return u, v, w


def duct_field(nx, ny, nz, zc, ly, lz, seed, ubulk=1.0, noise=0.1):
    """Square-duct start: u = 2.25 U_b (1 - (2y/ly - 1)^2)(1 - (2z/lz - 1)^2) plus seeded
    uniform noise, v = w = noise, on the duct layout with two ghost rows in y (rows ny, ny+1,
    left zero); v on the wall face row ny - 1 and w on the wall face plane nz are zero.
    zc holds the cell-centre heights of planes 0..nz+1."""
    rng = _rng(seed)
    shape = (nz + 2, ny + 2, nx)
    u, v, w = np.zeros(shape), np.zeros(shape), np.zeros(shape)
    y = (np.arange(ny) + 0.5) * (ly / ny)
    z = np.asarray(zc, dtype=np.float64)[1:nz + 1]
    prof = 2.25 * ubulk * (1.0 - (2.0 * z / lz - 1.0) ** 2)[:, None] * (1.0 - (2.0 * y / ly - 1.0) ** 2)[None, :]
    u[1:nz + 1, :ny] = prof[:, :, None] + noise * ubulk * (2.0 * rng.random((nz, ny, nx)) - 1.0)
    v[1:nz + 1, :ny] = noise * ubulk * (2.0 * rng.random((nz, ny, nx)) - 1.0)
    w[1:nz + 1, :ny] = noise * ubulk * (2.0 * rng.random((nz, ny, nx)) - 1.0)
    v[:, ny - 1] = 0.0
    w[nz] = 0.0
    return u, v, w


def uniform_shear_field(nx, ny, nz, zc, shear, z0=0.0):
    """u = shear (z - z0) at the u positions, v = w = 0."""
    u, v, w = _empty(nx, ny, nz), _empty(nx, ny, nz), _empty(nx, ny, nz)
    z = np.asarray(zc, dtype=np.float64)[1:nz + 1]
    u[1:nz + 1] = (shear * (z - z0))[:, None, None]
    return u, v, w


def taylor_green_field(n, nz, eps, length=2 * np.pi):
    """u = eps sin x cos y, v = -eps cos x sin y, w = 0 on an n x n x nz periodic box."""
    h = length / n
    x_face = (np.arange(n) + 1.0) * h
    x_cent = (np.arange(n) + 0.5) * h
    u, v, w = _empty(n, n, nz), _empty(n, n, nz), _empty(n, n, nz)
    uu = eps * np.sin(x_face)[None, :] * np.cos(x_cent)[:, None]      # [j, i]
    vv = -eps * np.cos(x_cent)[None, :] * np.sin(x_face)[:, None]
    u[1:nz + 1] = uu[None]
    v[1:nz + 1] = vv[None]
    return u, v, w


def random_state(nx, ny, nz, seed, scale=1.0):
    """Independent uniform(-scale, scale) values for u, v, w, p (interior planes only)."""
    rng = _rng(seed)
    out = []
    for _ in range(4):
        g = _empty(nx, ny, nz)
        g[1:nz + 1] = scale * (2.0 * rng.random((nz, ny, nx)) - 1.0)
        out.append(g)
    return tuple(out)


def box_ensemble(nbox, seed, sizes=(32, 48, 64, 96), k0s=(3.0, 4.0, 6.0), nu_range=(5e-4, 2e-3)):
    """Descriptors of an ensemble of periodic boxes: equal counts of each size,
    shuffled order, k0 uniform over k0s, nu log-uniform over nu_range, one seed per box."""
    rng = _rng(seed)
    per = nbox // len(sizes)
    ns = []
    for s in sizes:
        ns += [s] * per
    ns += [sizes[-1]] * (nbox - len(ns))
    ns = [int(x) for x in rng.permutation(np.array(ns))]
    k0 = rng.choice(np.array(k0s), size=nbox)
    lognu = rng.uniform(np.log(nu_range[0]), np.log(nu_range[1]), size=nbox)
    seeds = rng.integers(1, 2 ** 31 - 1, size=nbox)
    return [dict(n=ns[b], k0=float(k0[b]), nu=float(np.exp(lognu[b])), seed=int(seeds[b]))
            for b in range(nbox)]
