"""The C ABI library loads on the host and exports every function include/les.h declares;
argument validation runs before any device work (no GPU needed)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "les.h")).read()
    return sorted(set(re.findall(r"^(?:les_status|const char\*|int64_t)\s+(les_\w+)\(", src, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("les_init", "les_substep", "les_poisson", "les_nut", "les_free"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2411_09364_amd import les
    import ctypes
    lib = ctypes.CDLL(les.LIBPATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) <= set(les.exported_symbols())


def _init(**kw):
    from paper_2411_09364_amd import les
    base = dict(nx=32, ny=32, nz=32, lx=1.0, ly=1.0, lz=1.0)
    base.update(kw)
    return les.les_init(les.make_config(**base), 0)


@pytest.mark.parametrize("kw,status", [
    (dict(nx=14), -4), (dict(nx=50), -4), (dict(ny=1022), -4), (dict(nx=2048), -4), (dict(nz=22), -4),
    (dict(lx=-1.0), -1), (dict(nu=0.0), -1), (dict(zbc=7), -1), (dict(sgs=9), -1),
    (dict(implicit_z=1), -4), (dict(implicit_z=3), -1), (dict(implicit_z=-1), -1),
    (dict(precision=3), -1), (dict(zbc=1, nz=3), -1),
    (dict(zbc=2, nz=16, beta=1.0, h_wm=5.0), -1), (dict(cs=-0.1), -1), (dict(beta=float("nan")), -1),
])
def test_invalid_configurations_rejected(kw, status):
    from paper_2411_09364_amd import les
    with pytest.raises(les.LesError) as e:
        _init(**kw)
    assert e.value.status == status


def test_valid_configurations_and_layout():
    from paper_2411_09364_amd import les
    ctx = _init(nx=48, ny=24, nz=20, zbc=les.ZBC_WALLMODEL, beta=1.5, sgs=les.SGS_DSM, implicit_z=1,
                precision=les.MIXED)
    lay = les.les_layout(ctx, les.FIELD_U)
    assert (lay.dims[0], lay.dims[1], lay.dims[2]) == (22, 24, 48)
    assert lay.elem_bytes == 4 and lay.bytes == 22 * 24 * 48 * 4
    assert les.les_layout(ctx, les.FIELD_WORKSPACE).bytes > 8 * lay.bytes
    # calls that need bound memory fail cleanly with a status, not a crash
    with pytest.raises(les.LesError) as e:
        les.les_substep(ctx, 0)
    assert e.value.status == les.LES_ESTATE
    with pytest.raises(les.LesError) as e:
        les.les_bind(ctx, les.FIELD_U, 8)          # misaligned pointer, checked on the host
    assert e.value.status == les.LES_EINVAL
    les.les_free(ctx)


@pytest.mark.parametrize("zbc", [0, 1, 2])
def test_cn_in_all_directions_accepted_for_every_z_condition(zbc):
    from paper_2411_09364_amd import les
    kw = dict(zbc=zbc, nz=16) if zbc else {}
    ctx = _init(implicit_z=les.VISC_CN_3D, sgs=les.SGS_DSM, **kw)
    assert les.les_layout(ctx, les.FIELD_WORKSPACE).bytes > 0
    les.les_free(ctx)


@pytest.mark.parametrize("kw,status", [
    (dict(ybc=1), -4),                                              # y walls need z walls
    (dict(ybc=1, zbc=1, nz=16, implicit_z=2), -4),                  # no CN in y
    (dict(ybc=1, zbc=2, nz=16, h_wm=0.9), -1),                      # h_wm beyond the duct's middle row
    (dict(ybc=2, zbc=1, nz=16), -1),
])
def test_duct_configurations_rejected(kw, status):
    from paper_2411_09364_amd import les
    with pytest.raises(les.LesError) as e:
        _init(**kw)
    assert e.value.status == status


def test_duct_learned_closure_accepted():
    from paper_2411_09364_amd import les
    ctx = _init(ybc=1, zbc=2, nz=16, sgs=les.SGS_MLP)
    assert les.les_layout(ctx, les.FIELD_CS).bytes == 8 * 16 * 32   # per x line (nz, ny)
    les.les_free(ctx)


def test_duct_layout_has_two_ghost_rows():
    from paper_2411_09364_amd import les
    ctx = _init(nx=16, ny=12, nz=10, zbc=les.ZBC_WALLMODEL, ybc=les.YBC_WALL, sgs=les.SGS_SMAG_VD,
                h_wm=0.2, implicit_z=1)
    lay = les.les_layout(ctx, les.FIELD_U)
    assert (lay.dims[0], lay.dims[1], lay.dims[2]) == (12, 14, 16)
    assert lay.bytes == 12 * 14 * 16 * 8
    assert les.les_layout(ctx, les.FIELD_TAUW).bytes == 4 * 14 * 16 * 8
    assert les.les_layout(ctx, les.FIELD_TAUWY).bytes == 4 * 12 * 16 * 8
    les.les_free(ctx)
    ctx = _init()
    with pytest.raises(les.LesError) as e:
        les.les_layout(ctx, les.FIELD_TAUWY)
    assert e.value.status == les.LES_EINVAL
    les.les_free(ctx)


def test_library_grid_matches_oracle_grid():
    """Host-side metrics of the library (read back through the ABI, no GPU) equal the
    oracle's to roundoff."""
    import numpy as np
    from paper_2411_09364_amd import les
    import oracle
    ctx = _init(nx=16, ny=8, nz=24, lz=2.0, zbc=les.ZBC_NOSLIP, beta=1.5)
    buf = np.zeros(2 * 24 + 3)
    les.les_read(ctx, les.FIELD_ZGRID, buf.ctypes.data)
    g = oracle.Grid(oracle.Case(16, 8, 24, 1.0, 1.0, 2.0, zbc=1, beta=1.5))
    assert np.allclose(buf[:25], g.zf, rtol=0, atol=1e-15)
    assert np.allclose(buf[25:], g.zc, rtol=0, atol=1e-15)
    les.les_free(ctx)


def test_profile_error_host_function_matches_oracle():
    """les_profile_error is host code (no GPU): Eq. error against the oracle's reading on a
    stretched point set, and its argument checks."""
    import numpy as np
    from paper_2411_09364_amd import les
    from oracle import stats as ST
    rng = np.random.default_rng(9)
    z = np.sort(rng.uniform(0.0, 1.2, 33))
    ref = 1.0 + np.sin(2.0 * z)
    phi = ref + 0.03 * rng.standard_normal(z.size)
    e = les.les_profile_error(z, phi, ref, 0.1, 1.0)
    assert abs(e - ST.eps_phi(z, phi, ref, 0.1, 1.0)) < 1e-15
    with pytest.raises(les.LesError):
        les.les_profile_error(z[::-1], phi, ref, 0.1, 1.0)
    with pytest.raises(les.LesError):
        les.les_profile_error(z, phi, ref, 1.0, 0.1)
