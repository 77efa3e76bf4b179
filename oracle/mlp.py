"""Learned Smagorinsky-coefficient closure: a 7 -> 64 -> 64 -> 1 multilayer perceptron with
SiLU activations mapping local strain/rotation invariants, y+ and Delta/delta to the
dynamic model's coefficient c_s (the C_s^2 of Eq. dsmag).  Test infrastructure only.

The paper only motivates such closures (Sec. 1: SGS models trained on data produced by
the LES solver itself); the network, its inputs (R24), target (R25), output clip (R26)
and out-of-range fallback (R27) are this project's readings.

Parameters are a dict of float64 arrays: W1 (64, 7), b1 (64,), W2 (64, 64), b2 (64,),
W3 (1, 64), b3 (1,).  Flattened order (for Adam and the device buffers):
W1 row-major, b1, W2 row-major, b2, W3, b3  -> 4737 values.
"""
import numpy as np

from .ops import xm, xp, ym, yp
from . import bc

SHAPES = (("W1", (64, 7)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
          ("W3", (1, 64)), ("b3", (1,)))
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def flatten(params):
    return np.concatenate([params[k].ravel() for k, _ in SHAPES])


def unflatten(vec):
    out, o = {}, 0
    for k, s in SHAPES:
        n = int(np.prod(s))
        out[k] = np.asarray(vec[o:o + n], dtype=np.float64).reshape(s)
        o += n
    return out


def init_params(seed):
    """He-uniform style initialisation from a seeded PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for k, s in SHAPES:
        if k.startswith("W"):
            fan_in = s[1]
            lim = np.sqrt(6.0 / fan_in) * 0.5
            p[k] = rng.uniform(-lim, lim, size=s)
        else:
            p[k] = np.zeros(s)
    return p


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.  The value is
    first rounded to float32 (the kernel holds it in float32 before the conversion)."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, emulate_bf16=False):
    """x: (N, 7) normalised features.  Returns (y (N,), cache).  With emulate_bf16 the
    operands of the two 64-wide products (x, W1, h1, W2) are rounded to bfloat16 as the
    kernels round them; biases, layer 3 and every accumulation stay in full precision."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2 = r(params["W1"]), r(params["W2"])
    xb = r(x)
    z1 = xb @ W1.T + params["b1"]
    h1 = silu(z1)
    h1b = r(h1)
    z2 = h1b @ W2.T + params["b2"]
    h2 = silu(z2)
    y = h2 @ params["W3"][0] + params["b3"][0]
    return y, dict(xb=xb, z1=z1, h1b=h1b, z2=z2, h2=h2, W1=W1, W2=W2)


def loss_and_grad(params, x, t, emulate_bf16=False):
    """Mean-squared error L = mean((y - t)^2) and its gradient by backpropagation.
    With emulate_bf16 the backward products round dz2 and dz1 to bfloat16 as well."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    n = x.shape[0]
    y, c = forward(params, x, emulate_bf16)
    e = y - t
    loss = np.mean(e * e)
    dy = 2.0 * e / n
    g = {}
    g["W3"] = (dy @ c["h2"])[None, :]
    g["b3"] = np.array([dy.sum()])
    dz2 = (dy[:, None] * params["W3"][0][None, :]) * dsilu(c["z2"])
    dz2b = r(dz2)
    g["W2"] = dz2b.T @ c["h1b"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2b @ c["W2"]
    dz1 = dh1 * dsilu(c["z1"])
    dz1b = r(dz1)
    g["W1"] = dz1b.T @ c["xb"]
    g["b1"] = dz1.sum(axis=0)
    return loss, g


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) on flattened float64 vectors; t is the 1-based step."""
    gvec = flatten(grads)
    m = b1 * m + (1.0 - b1) * gvec
    v = b2 * v + (1.0 - b2) * gvec * gvec
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    p = flatten(params) - lr * mh / (np.sqrt(vh) + eps)
    return unflatten(p), m, v


# ---------------------------------------------------------------- features
def rotation_centre(g, u, v, w):
    """Rotation tensor Omega_ij = (du_i/dx_j - du_j/dx_i)/2 at cell centres, built like the
    off-diagonal strain (edges, then the four-edge mean).  Returns (O12, O13, O23)."""
    n = g.nz
    I = slice(1, n + 1)
    K0, K1 = slice(0, n + 1), slice(1, n + 2)
    dzc = g.dzc[0:n + 1][:, None, None]
    r12 = 0.5 * ((yp(u[I]) - u[I]) / g.dy - (xp(v[I]) - v[I]) / g.dx)
    r13 = 0.5 * ((u[K1] - u[K0]) / dzc - (xp(w[K0]) - w[K0]) / g.dx)
    r23 = 0.5 * ((v[K1] - v[K0]) / dzc - (yp(w[K0]) - w[K0]) / g.dy)
    o12 = 0.25 * (r12 + xm(r12) + ym(r12) + xm(ym(r12)))
    o13 = 0.25 * (r13[1:n + 1] + xm(r13[1:n + 1]) + r13[0:n] + xm(r13[0:n]))
    o23 = 0.25 * (r23[1:n + 1] + ym(r23[1:n + 1]) + r23[0:n] + ym(r23[0:n]))
    return o12, o13, o23


def raw_features(case, g, u, v, w, s, utau_walls):
    """R24: the seven unnormalised inputs per cell, shape (nz, ny, nx, 7):
    tr(S^2), tr(O^2), tr(S^3), tr(O^2 S), tr(O^2 S^2) of S^ = S/n and O^ = Omega/n with
    n = sqrt(S_ij S_ij + O_ij O_ij) (zero where n = 0), then y+ = d u_tau/nu (d the distance
    to the nearer wall, u_tau that wall's friction velocity; 0 with periodic z) and
    Delta/delta with delta = 1.  s: centre strain (S11, S22, S33, S12, S13, S23) with the
    SGS-strain ghosts; the rotation uses the same ghosts.
    R40 (square duct): y+ is the smallest d_w u_tau,w / nu over the four walls, the rule of
    the van Driest factor (R36), with utau_walls = (z bottom, z top, y = 0, y = ly); the
    features of the interior rows are returned, shape (nz, ny, nx, 7)."""
    us, vs, ws = bc.strain_ghosts(case, g, u, v, w)
    o12, o13, o23 = rotation_centre(g, us, vs, ws)
    s11, s22, s33, s12, s13, s23 = s
    S = np.stack([np.stack([s11, s12, s13], -1), np.stack([s12, s22, s23], -1),
                  np.stack([s13, s23, s33], -1)], -2)
    z = np.zeros_like(o12)
    O = np.stack([np.stack([z, o12, o13], -1), np.stack([-o12, z, o23], -1),
                  np.stack([-o13, -o23, z], -1)], -2)
    nrm = np.sqrt(np.sum(S * S, axis=(-1, -2)) + np.sum(O * O, axis=(-1, -2)))
    inv = np.where(nrm > 0.0, 1.0 / np.where(nrm > 0.0, nrm, 1.0), 0.0)[..., None, None]
    Sh, Oh = S * inv, O * inv
    S2 = Sh @ Sh
    O2 = Oh @ Oh
    tr = lambda a: np.trace(a, axis1=-2, axis2=-1)
    f = np.zeros(o12.shape + (7,))
    f[..., 0] = tr(S2)
    f[..., 1] = tr(O2)
    f[..., 2] = tr(S2 @ Sh)
    f[..., 3] = tr(O2 @ Sh)
    f[..., 4] = tr(O2 @ S2)
    f[..., 6] = g.delta()[:, None, None]
    if g.ywalls:
        f = f[:, :g.ny]
        zc = g.zc[1:g.nz + 1][:, None]
        yc = g.yc[None, :]
        ut = utau_walls
        dz_plus = np.minimum(zc * ut[0], (g.lz - zc) * ut[1])
        dy_plus = np.minimum(yc * ut[2], (g.ly - yc) * ut[3])
        f[..., 5] = (np.minimum(dz_plus, dy_plus) / case.nu)[:, :, None]
        return f
    if case.zperiodic:
        yplus = np.zeros(g.nz)
    else:
        zc = g.zc[1:g.nz + 1]
        lower = zc <= 0.5 * g.lz
        dist = np.where(lower, zc, g.lz - zc)
        yplus = dist * np.where(lower, utau_walls[0], utau_walls[1]) / case.nu
    f[..., 5] = yplus[:, None, None]
    return f


def normalise(f, lo, hi):
    """Min-max scaling to [0, 1] with the training ranges lo, hi (7 each)."""
    return (f - lo) / (hi - lo)


def out_of_range(fn, margin=0.05):
    """R27: a point is flagged when any normalised input leaves [-margin, 1 + margin]."""
    return np.any((fn < -margin) | (fn > 1.0 + margin), axis=-1)


def mlp_eddy_viscosity(case, g, u, v, w, params, lo, hi, cs_fallback, utau_walls,
                       emulate_bf16=True):
    """Learned closure: nu_t = max(0, MLP(x)) Delta^2 |S| (R26 clip), with flagged points
    taking the fallback coefficient of their plane (R27), or of their x line in a duct
    (cs_fallback (nz, ny) or wider, R38).  Returns (nu_t, flags) on the interior rows."""
    from .sgs import model_strain
    from .ops import strain_magnitude
    s = model_strain(case, g, u, v, w)
    smag = strain_magnitude(s)[:, :g.ny]
    fn = normalise(raw_features(case, g, u, v, w, s, utau_walls), lo, hi)
    flags = out_of_range(fn)
    y, _ = forward(params, fn.reshape(-1, 7), emulate_bf16)
    c = np.maximum(y.reshape(smag.shape), 0.0)
    cf = np.asarray(cs_fallback)
    cf = cf[:, :g.ny, None] if g.ywalls else cf[:, None, None]
    c = np.where(flags, cf, c)
    return c * (g.delta() ** 2)[:, None, None] * smag, flags
