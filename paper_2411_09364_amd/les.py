"""ctypes binding of the C ABI in include/les.h (argument marshalling only).

Every step of the substep runs in the HIP library liblesmi.so; this module only loads
it, converts arguments, and lets torch own the device buffers and the stream.  If the
library is missing the import fails: there is no CPU fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liblesmi.so")

LES_OK, LES_EINVAL, LES_ENOMEM, LES_EDEVICE, LES_ENOTSUP, LES_ENONFINITE, LES_ESTATE = 0, -1, -2, -3, -4, -5, -6
ZBC_PERIODIC, ZBC_NOSLIP, ZBC_WALLMODEL = 0, 1, 2
SGS_NONE, SGS_SMAG, SGS_SMAG_VD, SGS_DSM, SGS_MLP = 0, 1, 2, 3, 4
FP64, MIXED = 0, 1
VISC_EXPLICIT, VISC_CN_Z, VISC_CN_3D = 0, 1, 2
FIELD_U, FIELD_V, FIELD_W, FIELD_P, FIELD_WORKSPACE, FIELD_NUT, FIELD_CS, FIELD_TAUW, FIELD_ZGRID, FIELD_TAUWY = range(10)
YBC_PERIODIC, YBC_WALL = 0, 1
ABI_VERSION = 2


class LesConfig(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("lz", ctypes.c_double), ("zbc", ctypes.c_int32), ("beta", ctypes.c_double),
                ("nu", ctypes.c_double), ("sgs", ctypes.c_int32), ("cs", ctypes.c_double),
                ("implicit_z", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ubulk", ctypes.c_double), ("h_wm", ctypes.c_double), ("kappa", ctypes.c_double),
                ("bconst", ctypes.c_double), ("ybc", ctypes.c_int32)]


class LesLayout(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("dims", ctypes.c_int64 * 3), ("elem_bytes", ctypes.c_int64), ("bytes", ctypes.c_int64)]


class LesDiag(ctypes.Structure):
    _fields_ = [("max_div", ctypes.c_double), ("ubulk", ctypes.c_double), ("max_vel", ctypes.c_double),
                ("tauw_mean", ctypes.c_double * 2), ("dt", ctypes.c_double),
                ("nonfinite", ctypes.c_int64), ("mlp_flagged", ctypes.c_int64)]


class LesStats(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int64), ("series_len", ctypes.c_int64), ("tau_w", ctypes.c_double),
                ("u_tau", ctypes.c_double), ("re_tau", ctypes.c_double), ("u_b", ctypes.c_double),
                ("c_f", ctypes.c_double), ("c_f_sigma", ctypes.c_double)]


STATS_NPROF = 11
STATS_SERIES_MAX = 65536
STAT_NAMES = ("U", "V", "W", "P", "NUT", "uu", "vv", "ww", "uv", "uw", "vw")


class LesError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _load():
    if not os.path.exists(LIBPATH):
        raise ImportError(f"HIP library not built: {LIBPATH} (run python paper_2411_09364_amd/build.py)")
    # torch brings its own HIP runtime; loading it first lets the library resolve to that same
    # runtime, so that the two share devices, streams and memory
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIBPATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "les_init": [ctypes.POINTER(LesConfig), vp, ctypes.POINTER(vp)],
        "les_layout": [vp, i32, ctypes.POINTER(LesLayout)],
        "les_bind": [vp, i32, vp],
        "les_nut": [vp],
        "les_dt": [vp, dbl, ctypes.POINTER(dbl)],
        "les_set_dt": [vp, dbl],
        "les_substep": [vp, i32],
        "les_step": [vp, i32],
        "les_poisson": [vp, vp],
        "les_project": [vp],
        "les_read": [vp, i32, vp],
        "les_diag": [vp, ctypes.POINTER(LesDiag)],
        "les_mlp_bind": [vp, vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl)],
        "les_mlp_sample": [vp, ctypes.c_uint64, ctypes.c_int64, vp, vp],
        "les_mlp_normalize": [vp, vp, ctypes.c_int64, ctypes.POINTER(dbl), ctypes.POINTER(dbl), vp],
        "les_mlp_forward": [vp, vp, vp, ctypes.c_int64, vp],
        "les_mlp_grad": [vp, vp, vp, vp, ctypes.c_int64, vp, vp, vp],
        "les_mlp_grad_noalloc": [vp, vp, vp, vp, ctypes.c_int64, vp, vp],
        "les_mlp_adam": [vp, vp, vp, vp, vp, i32, ctypes.c_float],
        "les_mlp_train_step": [vp, vp, vp, vp, ctypes.c_int64, vp, vp, vp, vp, i32, ctypes.c_float, vp],
        "les_free": [vp],
        "les_timing": [vp, i32],
        "les_batch_init": [ctypes.POINTER(LesConfig), i32, vp, ctypes.POINTER(vp)],
        "les_batch_layout": [vp, i32, ctypes.POINTER(LesLayout)],
        "les_batch_offset": [vp, i32, i32, ctypes.POINTER(ctypes.c_int64)],
        "les_batch_bind": [vp, i32, vp],
        "les_batch_nut": [vp],
        "les_batch_dt": [vp, dbl],
        "les_batch_set_dt": [vp, dbl],
        "les_batch_substep": [vp, i32],
        "les_batch_step": [vp, dbl, i32],
        "les_batch_autotune": [vp, i32, ctypes.c_char_p, ctypes.c_size_t],
        "les_batch_read": [vp, i32, i32, vp],
        "les_batch_diag": [vp, i32, ctypes.POINTER(LesDiag)],
        "les_batch_mlp_sample": [vp, ctypes.c_uint64, ctypes.c_int64, vp, vp],
        "les_batch_free": [vp],
        "les_timing_report": [vp, ctypes.c_char_p, ctypes.c_size_t],
        "les_stats_reset": [vp],
        "les_stats_sample": [vp],
        "les_stats_read": [vp, i32, ctypes.POINTER(LesStats), vp],
        "les_profile_error": [ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl), i32, dbl, dbl,
                              ctypes.POINTER(dbl)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.les_mlp_workspace_bytes.argtypes = [ctypes.c_int64]
    lib.les_mlp_workspace_bytes.restype = ctypes.c_int64
    lib.les_batch_last_error.argtypes = [vp]
    lib.les_batch_last_error.restype = ctypes.c_char_p
    lib.les_strerror.argtypes = [ctypes.c_int]
    lib.les_strerror.restype = ctypes.c_char_p
    lib.les_last_error.argtypes = [vp]
    lib.les_last_error.restype = ctypes.c_char_p
    return lib


LIB = _load()


def exported_symbols():
    """Names of the ABI functions the binding resolves (all must exist in the library)."""
    return ["les_init", "les_layout", "les_bind", "les_nut", "les_dt", "les_set_dt", "les_substep",
            "les_step", "les_poisson", "les_project", "les_read", "les_diag", "les_mlp_bind", "les_mlp_sample",
            "les_mlp_normalize", "les_mlp_forward", "les_mlp_workspace_bytes", "les_mlp_grad",
            "les_mlp_grad_noalloc", "les_mlp_adam", "les_mlp_train_step", "les_free", "les_strerror", "les_last_error",
            "les_timing", "les_timing_report", "les_batch_init", "les_batch_layout", "les_batch_offset",
            "les_batch_bind", "les_batch_nut", "les_batch_dt", "les_batch_set_dt", "les_batch_substep",
            "les_batch_step", "les_batch_autotune", "les_batch_read", "les_batch_diag", "les_batch_mlp_sample",
            "les_batch_last_error", "les_batch_free", "les_stats_reset", "les_stats_sample", "les_stats_read",
            "les_profile_error"]


def make_config(nx, ny, nz, lx, ly, lz, zbc=ZBC_PERIODIC, beta=0.0, nu=1e-3, sgs=SGS_NONE, cs=0.17,
                implicit_z=0, precision=FP64, ubulk=0.0, h_wm=0.0, kappa=0.41, bconst=5.2, ybc=YBC_PERIODIC):
    return LesConfig(ABI_VERSION, nx, ny, nz, lx, ly, lz, zbc, beta, nu, sgs, cs, int(implicit_z),
                     precision, ubulk, h_wm, kappa, bconst, int(ybc))


def _check(ctx, st, what):
    if st != LES_OK:
        detail = LIB.les_last_error(ctx).decode() if ctx else LIB.les_strerror(st).decode()
        raise LesError(st, f"{what}: {detail or LIB.les_strerror(st).decode()}")


# ---------------------------------------------------------------- thin wrappers (same names)
def les_init(cfg, stream_handle=0):
    out = ctypes.c_void_p()
    st = LIB.les_init(ctypes.byref(cfg), ctypes.c_void_p(stream_handle), ctypes.byref(out))
    if st != LES_OK:
        raise LesError(st, f"les_init: {LIB.les_strerror(st).decode()}")
    return out


def les_layout(ctx, field):
    lay = LesLayout()
    _check(ctx, LIB.les_layout(ctx, field, ctypes.byref(lay)), "les_layout")
    return lay


def les_bind(ctx, field, ptr):
    _check(ctx, LIB.les_bind(ctx, field, ctypes.c_void_p(ptr)), "les_bind")


def les_nut(ctx):
    _check(ctx, LIB.les_nut(ctx), "les_nut")


def les_dt(ctx, cfl, sync=True):
    out = ctypes.c_double(0.0)
    _check(ctx, LIB.les_dt(ctx, cfl, ctypes.byref(out) if sync else None), "les_dt")
    return out.value if sync else None


def les_set_dt(ctx, dt):
    _check(ctx, LIB.les_set_dt(ctx, dt), "les_set_dt")


def les_substep(ctx, stage):
    _check(ctx, LIB.les_substep(ctx, stage), "les_substep")


def les_step(ctx, use_graph=False):
    _check(ctx, LIB.les_step(ctx, 1 if use_graph else 0), "les_step")


def les_poisson(ctx, ptr):
    _check(ctx, LIB.les_poisson(ctx, ctypes.c_void_p(ptr)), "les_poisson")


def les_project(ctx):
    _check(ctx, LIB.les_project(ctx), "les_project")


def les_read(ctx, field, ptr):
    _check(ctx, LIB.les_read(ctx, field, ctypes.c_void_p(ptr)), "les_read")


def les_diag(ctx):
    d = LesDiag()
    st = LIB.les_diag(ctx, ctypes.byref(d))
    if st not in (LES_OK, LES_ENONFINITE):
        _check(ctx, st, "les_diag")
    return d, st


def _d7(a):
    return (ctypes.c_double * 7)(*[float(x) for x in a])


def les_mlp_bind(ctx, params_ptr, lo, hi):
    _check(ctx, LIB.les_mlp_bind(ctx, ctypes.c_void_p(params_ptr), _d7(lo), _d7(hi)), "les_mlp_bind")


def les_mlp_sample(ctx, seed, n, x_ptr, y_ptr):
    _check(ctx, LIB.les_mlp_sample(ctx, seed, n, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr)), "les_mlp_sample")


def les_mlp_normalize(stream, xraw_ptr, n, lo, hi, x_ptr):
    _check(None, LIB.les_mlp_normalize(ctypes.c_void_p(stream), ctypes.c_void_p(xraw_ptr), n, _d7(lo), _d7(hi),
                                       ctypes.c_void_p(x_ptr)), "les_mlp_normalize")


def les_mlp_forward(stream, params_ptr, x_ptr, n, y_ptr):
    _check(None, LIB.les_mlp_forward(ctypes.c_void_p(stream), ctypes.c_void_p(params_ptr), ctypes.c_void_p(x_ptr), n,
                                     ctypes.c_void_p(y_ptr)), "les_mlp_forward")


def les_mlp_workspace_bytes(n):
    return int(LIB.les_mlp_workspace_bytes(n))


def les_mlp_grad(stream, params_ptr, x_ptr, y_ptr, n, ws_ptr, grad_ptr, loss_ptr):
    vp = ctypes.c_void_p
    _check(None, LIB.les_mlp_grad(vp(stream), vp(params_ptr), vp(x_ptr), vp(y_ptr), n, vp(ws_ptr), vp(grad_ptr),
                                  vp(loss_ptr)), "les_mlp_grad")


MLP_NOALLOC_MAX_SAMPLES = 65536


def les_mlp_grad_noalloc(stream, params_ptr, x_ptr, y_ptr, n, grad_ptr, loss_ptr):
    vp = ctypes.c_void_p
    st = LIB.les_mlp_grad_noalloc(vp(stream), vp(params_ptr), vp(x_ptr), vp(y_ptr), n, vp(grad_ptr), vp(loss_ptr))
    if st != LES_OK:
        raise LesError(st, f"les_mlp_grad_noalloc: {LIB.les_last_error(None).decode()}")


def les_mlp_adam(stream, params_ptr, grad_ptr, m_ptr, v_ptr, step, lr):
    vp = ctypes.c_void_p
    _check(None, LIB.les_mlp_adam(vp(stream), vp(params_ptr), vp(grad_ptr), vp(m_ptr), vp(v_ptr), step, lr),
           "les_mlp_adam")


def les_mlp_train_step(stream, params_ptr, x_ptr, y_ptr, n, ws_ptr, grad_ptr, m_ptr, v_ptr, step, lr, loss_ptr):
    vp = ctypes.c_void_p
    _check(None, LIB.les_mlp_train_step(vp(stream), vp(params_ptr), vp(x_ptr), vp(y_ptr), n, vp(ws_ptr),
                                        vp(grad_ptr), vp(m_ptr), vp(v_ptr), step, lr, vp(loss_ptr)),
           "les_mlp_train_step")


class Mlp:
    """Torch-owned parameters, Adam moments and gradient workspace of the learned closure;
    every operation runs in the library's kernels on the given stream."""

    NPARAM = 4737

    def __init__(self, params_host, stream=None, device="cuda"):
        import torch
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.params = torch.as_tensor(params_host, dtype=torch.float32).to(device).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.step_count = 0
        self._ws = None
        torch.cuda.synchronize()   # the copies above ran on torch's current stream

    def _workspace(self, n):
        torch = self.torch
        need = les_mlp_workspace_bytes(n)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.params.device)
        return self._ws

    def forward(self, x):
        torch = self.torch
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        les_mlp_forward(self.stream.cuda_stream, self.params.data_ptr(), x.data_ptr(), x.shape[0], y.data_ptr())
        return y

    def gradient(self, x, y):
        ws = self._workspace(x.shape[0])
        les_mlp_grad(self.stream.cuda_stream, self.params.data_ptr(), x.data_ptr(), y.data_ptr(), x.shape[0],
                     ws.data_ptr(), self.grad.data_ptr(), self.loss.data_ptr())
        return self.grad, self.loss

    def train_step(self, x, y, lr):
        ws = self._workspace(x.shape[0])
        self.step_count += 1
        les_mlp_train_step(self.stream.cuda_stream, self.params.data_ptr(), x.data_ptr(), y.data_ptr(),
                           x.shape[0], ws.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                           self.step_count, lr, self.loss.data_ptr())
        return self.loss


def les_stats_reset(ctx):
    _check(ctx, LIB.les_stats_reset(ctx), "les_stats_reset")


def les_stats_sample(ctx):
    _check(ctx, LIB.les_stats_sample(ctx), "les_stats_sample")


def les_stats_read(ctx, nbatch, profiles_ptr=None):
    out = LesStats()
    _check(ctx, LIB.les_stats_read(ctx, nbatch, ctypes.byref(out), ctypes.c_void_p(profiles_ptr)), "les_stats_read")
    return out


def les_profile_error(z, phi, ref, z0, z1):
    import numpy as np
    z, phi, ref = (np.ascontiguousarray(a, dtype=np.float64) for a in (z, phi, ref))
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    eps = ctypes.c_double(0.0)
    _check(None, LIB.les_profile_error(p(z), p(phi), p(ref), len(z), z0, z1, ctypes.byref(eps)), "les_profile_error")
    return eps.value


def les_timing(ctx, enable):
    _check(ctx, LIB.les_timing(ctx, 1 if enable else 0), "les_timing")


def les_timing_report(ctx):
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(ctx, LIB.les_timing_report(ctx, buf, len(buf)), "les_timing_report")
    return json.loads(buf.value.decode())


def les_free(ctx):
    _check(None, LIB.les_free(ctx), "les_free")


# ---------------------------------------------------------------- torch-owned solver
class Solver:
    """One context with torch-allocated fields and workspace on its own stream.

    Fields are torch tensors of shape (nz + 2, ny, nx) in the context's storage type
    ((nz + 2, ny + 2, nx) for ducts: two ghost rows after the interior rows).
    """

    def __init__(self, cfg, device="cuda"):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = les_init(cfg, self.stream.cuda_stream)
        lay = les_layout(self.ctx, FIELD_U)
        self.dtype = torch.float64 if lay.elem_bytes == 8 else torch.float32
        self.shape = tuple(int(d) for d in lay.dims)   # (nz + 2, ny [+ 2 ghost rows for ducts], nx)
        with torch.cuda.stream(self.stream):
            self.u, self.v, self.w, self.p = (torch.zeros(self.shape, dtype=self.dtype, device=device)
                                              for _ in range(4))
            wsb = les_layout(self.ctx, FIELD_WORKSPACE).bytes
            self.workspace = torch.empty(wsb + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        for f, t in ((FIELD_U, self.u), (FIELD_V, self.v), (FIELD_W, self.w), (FIELD_P, self.p)):
            les_bind(self.ctx, f, t.data_ptr())
        self.stream.synchronize()
        les_bind(self.ctx, FIELD_WORKSPACE, base + off)
        self.workspace_bytes = wsb

    def set_state(self, u, v, w, p=None):
        """Copy host arrays (numpy, field shape) into the device fields."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            for dst, src in ((self.u, u), (self.v, v), (self.w, w), (self.p, p)):
                if src is None:
                    dst.zero_()
                else:
                    dst.copy_(torch.as_tensor(src, dtype=self.dtype))
        self.stream.synchronize()

    def project(self):
        """Initial projection of the bound velocity (les_project); call nut() afterwards."""
        les_project(self.ctx)

    def nut(self):
        les_nut(self.ctx)

    def set_dt(self, dt):
        les_set_dt(self.ctx, dt)

    def dt(self, cfl=0.5):
        return les_dt(self.ctx, cfl)

    def substep(self, stage):
        les_substep(self.ctx, stage)

    def step(self, use_graph=False):
        les_step(self.ctx, use_graph)

    def synchronize(self):
        self.stream.synchronize()

    def fields(self):
        """Host float64 copies of u, v, w, p."""
        self.synchronize()
        return tuple(t.double().cpu().numpy() for t in (self.u, self.v, self.w, self.p))

    def eddy_viscosity(self):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            out = torch.empty(self.shape, dtype=self.dtype, device=self.u.device)
        les_read(self.ctx, FIELD_NUT, out.data_ptr())
        self.synchronize()
        return out.double().cpu().numpy()

    def coefficient(self):
        """Dynamic coefficient per plane (nz,), or per x line (nz, ny) for ducts."""
        torch = self.torch
        shape = (self.cfg.nz, self.cfg.ny) if self.cfg.ybc == YBC_WALL else (self.cfg.nz,)
        out = torch.empty(shape, dtype=torch.float64, device=self.u.device)
        les_read(self.ctx, FIELD_CS, out.data_ptr())
        self.synchronize()
        return out.cpu().numpy()

    def wall_stress(self):
        torch = self.torch
        out = torch.empty((4, self.shape[1], self.cfg.nx), dtype=torch.float64, device=self.u.device)
        les_read(self.ctx, FIELD_TAUW, out.data_ptr())
        self.synchronize()
        return out.cpu().numpy()

    def wall_stress_y(self):
        """Ducts with the wall model: (4, nz + 2, nx) stresses of the y walls."""
        torch = self.torch
        out = torch.empty((4, self.cfg.nz + 2, self.cfg.nx), dtype=torch.float64, device=self.u.device)
        les_read(self.ctx, FIELD_TAUWY, out.data_ptr())
        self.synchronize()
        return out.cpu().numpy()

    def zgrid(self):
        import numpy as np
        buf = np.zeros(2 * self.cfg.nz + 3)
        les_read(self.ctx, FIELD_ZGRID, buf.ctypes.data)
        return buf[:self.cfg.nz + 1], buf[self.cfg.nz + 1:]

    def poisson(self, f):
        """Solve D G phi = f for a host array f (field shape); returns phi (host)."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            t = torch.as_tensor(f, dtype=self.dtype).to(self.u.device)
        self.stream.synchronize()
        les_poisson(self.ctx, t.data_ptr())
        self.synchronize()
        return t.double().cpu().numpy()

    def diag(self):
        return les_diag(self.ctx)

    def stats_reset(self):
        les_stats_reset(self.ctx)

    def stats_sample(self):
        les_stats_sample(self.ctx)

    def stats(self, nbatch=8):
        """(scalars dict, profiles dict of host arrays [nz], or [nz][ny] cross-sections for
        ducts) of the accumulated statistics."""
        import numpy as np
        shape = (STATS_NPROF, self.cfg.nz, self.cfg.ny) if self.cfg.ybc == YBC_WALL else (STATS_NPROF, self.cfg.nz)
        prof = np.zeros(shape)
        out = les_stats_read(self.ctx, nbatch, prof.ctypes.data)
        sc = {f: getattr(out, f) for f, _ in LesStats._fields_}
        return sc, {name: prof[q] for q, name in enumerate(STAT_NAMES)}

    def mlp_bind(self, mlp, lo, hi):
        les_mlp_bind(self.ctx, mlp.params.data_ptr(), lo, hi)
        self._mlp = mlp   # keep the parameters alive while bound

    def mlp_sample(self, seed, n):
        torch = self.torch
        x = torch.empty((n, 7), dtype=torch.float32, device=self.u.device)
        y = torch.empty(n, dtype=torch.float32, device=self.u.device)
        les_mlp_sample(self.ctx, seed, n, x.data_ptr(), y.data_ptr())
        self.synchronize()
        return x, y

    def close(self):
        if self.ctx:
            self.synchronize()
            les_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- batched ensembles
def _bcheck(b, st, what):
    if st != LES_OK:
        msg = LIB.les_batch_last_error(b).decode() if b else ""
        raise LesError(st, f"{what}: {msg or LIB.les_strerror(st).decode()}")


class Batch:
    """Many periodic boxes advanced together (one launch per kernel kind for all boxes).
    Fields of box b are views into the concatenated torch buffers."""

    def __init__(self, cfgs, device="cuda"):
        import torch
        self.torch = torch
        self.cfgs = list(cfgs)
        self.stream = torch.cuda.Stream(device=device)
        arr = (LesConfig * len(self.cfgs))(*self.cfgs)
        h = ctypes.c_void_p()
        st = LIB.les_batch_init(arr, len(self.cfgs), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != LES_OK:
            raise LesError(st, f"les_batch_init: {LIB.les_strerror(st).decode()}")
        self.h = h
        lay = LesLayout()
        _bcheck(h, LIB.les_batch_layout(h, FIELD_U, ctypes.byref(lay)), "les_batch_layout")
        self.dtype = torch.float64 if lay.elem_bytes == 8 else torch.float32
        fbytes = lay.bytes
        _bcheck(h, LIB.les_batch_layout(h, FIELD_WORKSPACE, ctypes.byref(lay)), "les_batch_layout")
        wbytes = lay.bytes
        esz = 8 if self.dtype == torch.float64 else 4
        with torch.cuda.stream(self.stream):
            self.buf = [torch.zeros(fbytes // esz + 64, dtype=self.dtype, device=device) for _ in range(4)]
            self.workspace = torch.empty(wbytes + 256, dtype=torch.uint8, device=device)
        self.stream.synchronize()
        self.ptrs = []
        for q in range(4):
            base = self.buf[q].data_ptr()
            off = (-base) % 256
            self.ptrs.append(base + off)
            _bcheck(h, LIB.les_batch_bind(h, q, ctypes.c_void_p(base + off)), "les_batch_bind")
        wb = self.workspace.data_ptr()
        _bcheck(h, LIB.les_batch_bind(h, FIELD_WORKSPACE, ctypes.c_void_p(wb + ((-wb) % 256))), "les_batch_bind")
        self.offsets = []
        for b in range(len(self.cfgs)):
            o = ctypes.c_int64()
            _bcheck(h, LIB.les_batch_offset(h, b, FIELD_U, ctypes.byref(o)), "les_batch_offset")
            self.offsets.append(o.value)

    def field(self, q, b):
        """Torch view of field q (0 u, 1 v, 2 w, 3 p) of box b."""
        c = self.cfgs[b]
        n = (c.nz + 2) * c.ny * c.nx
        esz = 8 if self.dtype == self.torch.float64 else 4
        start = (self.ptrs[q] - self.buf[q].data_ptr() + self.offsets[b]) // esz
        return self.buf[q][start:start + n].view(c.nz + 2, c.ny, c.nx)

    def set_state(self, b, u, v, w, p=None):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            for q, src in enumerate((u, v, w, p)):
                dst = self.field(q, b)
                if src is None:
                    dst.zero_()
                else:
                    dst.copy_(torch.as_tensor(src, dtype=self.dtype))
        self.stream.synchronize()

    def fields(self, b):
        self.stream.synchronize()
        return tuple(self.field(q, b).double().cpu().numpy() for q in range(4))

    def nut(self):
        _bcheck(self.h, LIB.les_batch_nut(self.h), "les_batch_nut")

    def set_dt(self, dt):
        _bcheck(self.h, LIB.les_batch_set_dt(self.h, dt), "les_batch_set_dt")

    def dt(self, cfl):
        _bcheck(self.h, LIB.les_batch_dt(self.h, cfl), "les_batch_dt")

    def substep(self, stage):
        _bcheck(self.h, LIB.les_batch_substep(self.h, stage), "les_batch_substep")

    def step(self, cfl=0.5, use_graph=False):
        _bcheck(self.h, LIB.les_batch_step(self.h, cfl, 1 if use_graph else 0), "les_batch_step")

    def autotune(self, substeps=6):
        import json
        buf = ctypes.create_string_buffer(4096)
        _bcheck(self.h, LIB.les_batch_autotune(self.h, substeps, buf, len(buf)), "les_batch_autotune")
        return json.loads(buf.value.decode())

    def eddy_viscosity(self, b):
        torch = self.torch
        c = self.cfgs[b]
        out = torch.empty((c.nz + 2, c.ny, c.nx), dtype=self.dtype, device=self.buf[0].device)
        _bcheck(self.h, LIB.les_batch_read(self.h, b, FIELD_NUT, ctypes.c_void_p(out.data_ptr())), "les_batch_read")
        self.stream.synchronize()
        return out.double().cpu().numpy()

    def mlp_sample(self, seed, n_per_box):
        """Training pairs of every box (les_batch_mlp_sample): box b's rows are
        [b n_per_box, (b + 1) n_per_box) of x (raw inputs) and y."""
        torch = self.torch
        nb = len(self.cfgs)
        with torch.cuda.stream(self.stream):
            x = torch.empty((nb * n_per_box, 7), dtype=torch.float32, device=self.buf[0].device)
            y = torch.empty(nb * n_per_box, dtype=torch.float32, device=self.buf[0].device)
        _bcheck(self.h, LIB.les_batch_mlp_sample(self.h, ctypes.c_uint64(seed), ctypes.c_int64(n_per_box),
                                                 ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())),
                "les_batch_mlp_sample")
        self.stream.synchronize()
        return x, y

    def box_dt(self, b):
        d = LesDiag()
        st = LIB.les_batch_diag(self.h, b, ctypes.byref(d))
        if st not in (LES_OK, LES_ENONFINITE):
            _bcheck(self.h, st, "les_batch_diag")
        return d

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.h:
            self.stream.synchronize()
            LIB.les_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
