"""The C-ABI library on the CPU: it loads, exports every entry point that
include/lbe.h declares, agrees with the oracle on the velocity set, and
rejects bad input with the documented codes before touching a device."""
import os
import re

import numpy as np
import pytest

import paper_1907_04732_amd as lbe
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "lbe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbe_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lbe.load()
    names = header_functions()
    assert "lbe_init" in names and "lbe_step" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(lbe.ENTRY_POINTS) <= set(names)


def test_library_is_built_from_these_sources():
    """lbe_build_id is the hash of the sources beside the library (the
    binding refuses a stale build), and a changed hash is refused."""
    from paper_1907_04732_amd.build import source_hash
    lib = lbe.load()
    assert lib.lbe_build_id().decode() == source_hash()
    import ctypes
    raw = ctypes.CDLL(lbe.LIB_PATH)
    raw.lbe_build_id.restype = ctypes.c_char_p
    assert raw.lbe_build_id().decode() == source_hash()


def test_stale_library_is_refused(tmp_path, monkeypatch):
    """A library whose build id differs from the sources is not loaded."""
    import shutil
    import paper_1907_04732_amd.build as B
    stale = tmp_path / "liblbe.so"
    shutil.copy(lbe.LIB_PATH, stale)
    monkeypatch.setattr(lbe, "_lib", None)
    monkeypatch.setattr(B, "source_hash", lambda: "0000000000000000")
    with pytest.raises(OSError, match="other sources"):
        lbe.load(str(stale))


def test_velocity_set_matches_oracle_order():
    import oracle
    c, w = lbe.velocities()
    co, wo = oracle.velocities()
    assert (c == co).all()
    assert np.array_equal(w, wo)


def test_error_strings():
    lib = lbe.load()
    for code in (lbe.OK, lbe.EINVAL, lbe.EGEOM, lbe.ENOMEM, lbe.EDEVICE, lbe.ENOCONV, lbe.ENONFINITE):
        assert lib.lbe_strerror(code)
    assert lbe.kernel_names()[0] == "fluid"


def _slab_params(**kw):
    shape, t, ps = W.slab(2, 2, 8, 1)
    base = dict(shape=shape, z=(1, -1), D=(0.05, 0.05), lB=0.4)
    base.update(kw)
    return lbe.make_params(**base), t, ps


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(omega=2.0), dict(omega=-0.1),
                                dict(check_every=0), dict(lB=-1.0), dict(rho0=0.0),
                                dict(D=(0.05, -1.0)), dict(Eapp=(np.nan, 0, 0)),
                                dict(precision=7), dict(poisson=9), dict(flags=16),
                                dict(flags=8),  # Krylov acceleration needs multigrid
                                dict(poisson=1, mg_levels=1), dict(poisson=1, mg_nu1=0, mg_nu2=0),
                                dict(poisson=1, mg_nu1_coarse=-1)])
def test_invalid_parameters_rejected(kw):
    p, t, ps = _slab_params(**kw)
    with pytest.raises(lbe.LbeError) as e:
        lbe.Lbe(p, t, ps, None, (1e-3, 1e-3))
    assert e.value.code == lbe.EINVAL


def test_invalid_dimensions_and_inputs():
    p = lbe.make_params((0, 2, 10), (1, -1), (0.05, 0.05), 0.4)
    with pytest.raises(lbe.LbeError) as e:
        lbe.Lbe(p, np.zeros(0, np.uint8), np.zeros(0), None, (1e-3, 1e-3))
    assert e.value.code == lbe.EINVAL
    p, t, ps = _slab_params()
    n0 = np.full((2, t.size), 1e-3)
    n0[1, 9] = np.inf
    with pytest.raises(lbe.LbeError) as e:
        lbe.Lbe(p, t, ps, n0)
    assert e.value.code == lbe.EINVAL
    ps2 = ps.copy()
    ps2[0] = np.nan
    with pytest.raises(lbe.LbeError) as e:
        lbe.Lbe(p, t, ps2, None, (1e-3, 1e-3))
    assert e.value.code == lbe.EINVAL


def test_geometry_rejected():
    shape = (4, 4, 4)
    p = lbe.make_params(shape, (1, -1), (0.05, 0.05), 0.4)
    with pytest.raises(lbe.LbeError) as e:  # fluid touching no electrode
        lbe.Lbe(p, np.zeros(64, np.uint8), np.zeros(64), None, (1e-3, 1e-3))
    assert e.value.code == lbe.EGEOM
    shape, t, ps = W.slab(3, 2, 8, 1)  # odd periodic extent > 2
    p = lbe.make_params(shape, (1, -1), (0.05, 0.05), 0.4)
    with pytest.raises(lbe.LbeError) as e:
        lbe.Lbe(p, t, ps, None, (1e-3, 1e-3))
    assert e.value.code == lbe.EGEOM



def test_batched_systems_rejected():
    """lbe_init_batch validates the system map before touching a device."""
    shape, t, ps = W.slab(2, 2, 8, 1)
    p = lbe.make_params(shape, (1, -1), (0.05, 0.05), 0.4)
    sy = np.zeros(t.size, np.uint16)
    nref = np.full((2, 2), 1e-3)
    with pytest.raises(lbe.LbeError) as e:  # index >= nsys
        lbe.Lbe(p, t, ps, None, nref, system=sy + 2, nsys=2)
    assert e.value.code == lbe.EINVAL
    with pytest.raises(lbe.LbeError) as e:  # nsys out of range
        lbe.Lbe(p, t, ps, None, nref, system=sy, nsys=0)
    assert e.value.code == lbe.EINVAL
    half = sy.copy()
    half[t.size // 2:] = 1  # one fluid column split between two systems
    with pytest.raises(lbe.LbeError) as e:
        lbe.Lbe(p, t, ps, None, nref, system=half, nsys=2)
    assert e.value.code == lbe.EGEOM
