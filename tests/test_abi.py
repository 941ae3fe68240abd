"""CPU-side checks of the C ABI: the library loads, exports every function the
header declares, and rejects invalid parameters before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_1905_05524_amd import adg
from paper_1905_05524_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(adg3?_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = adg.lib()
    names = header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(adg.EXPORTED)


def test_binding_constants_match_header_enums():
    """Every enumerator of include/*.h has the binding's value (inputs.py for
    the bubble shapes), so a constant dropped from the binding fails here."""
    found = {}
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", h)).read(), flags=re.S)
            for body in re.findall(r"enum\s*\{(.*?)\}", src, flags=re.S):
                for name, val in re.findall(r"(ADG\w+)\s*=\s*(-?\d+)", body):
                    found[name] = int(val)
    assert len(found) >= 13
    for name, val in found.items():
        src = I if name.startswith("ADG_SHAPE_") else adg
        attr = name[len("ADG_"):] if src is I else name
        assert getattr(src, attr) == val, name


def _init(phys, mesh):
    p = adg.make_params(phys)
    d = adg.adg_mesh_desc()
    d.x0, d.z0, d.Lx, d.Lz = 0.0, 0.0, float(mesh["Lx"]), float(mesh["Lz"])
    d.nx, d.nz, d.max_level = mesh["nx"], mesh["nz"], mesh.get("max_level", 0)
    for k, b in enumerate(mesh["bc"]):
        d.bc[k] = b
    h = ctypes.c_void_p()
    rc = adg.lib().adg_init_mesh(ctypes.byref(p), ctypes.byref(d), ctypes.byref(h))
    return rc, adg.lib().adg_last_error().decode()


@pytest.mark.parametrize("change,msg", [
    (dict(N=0), "order"), (dict(N=8), "order"), (dict(gamma=1.0), "gas"), (dict(cfl=0.0), "cfl"),
    (dict(mu=-1.0), "gas"), (dict(picard_iters=-2), "picard"),
])
def test_invalid_params_rejected(change, msg):
    w = I.bubble81()
    phys = dict(w["phys"], **change)
    rc, err = _init(phys, w["mesh"])
    assert rc == adg.ADG_EINVAL and msg in err


@pytest.mark.parametrize("change,msg", [
    (dict(nx=0), "domain"), (dict(Lz=500.0), "square"), (dict(bc=[0, 1, 1, 1]), "pairs"),
    (dict(bc=[1, 1, 7, 1]), "bc"), (dict(max_level=1), "max_level"),
])
def test_invalid_mesh_rejected(change, msg):
    w = I.bubble81()
    mesh = dict(w["mesh"], **change)
    rc, err = _init(w["phys"], mesh)
    assert rc == adg.ADG_EINVAL and msg in err


def _init_leaves(nx, nz, max_level, n_leaves=1):
    """adg_init_mesh with a leaf-list mesh of the given coarse grid (the leaf
    arrays are never read: validation fails first)."""
    w = I.bubble81()
    p = adg.make_params(w["phys"])
    d = adg.adg_mesh_desc()
    d.Lx, d.Lz, d.nx, d.nz, d.max_level = 1.0 * nx, 1.0 * nz, nx, nz, max_level
    for k in range(4):
        d.bc[k] = adg.ADG_BC_WALL
    one = (ctypes.c_int32 * 1)(0)
    d.n_leaves = n_leaves
    d.leaf_level = d.leaf_i = d.leaf_j = ctypes.cast(one, ctypes.POINTER(ctypes.c_int32))
    h = ctypes.c_void_p()
    rc = adg.lib().adg_init_mesh(ctypes.byref(p), ctypes.byref(d), ctypes.byref(h))
    return rc, adg.lib().adg_last_error().decode()


def test_meshes_beyond_32_bit_indices_rejected():
    """A wide coarse grid at a deep level would overflow 32-bit leaf and box
    indices: nx * 3^max_level and nz * 3^max_level must stay below 2^31, and
    a leaf-list mesh's coarse grid below 2^26 cells."""
    rc, err = _init_leaves(1 << 26, 1, 8)
    assert rc == adg.ADG_EINVAL and "coarse" not in err and "32-bit" in err
    rc, err = _init_leaves(1, 400000, 8)          # 400000 * 6561 > 2^31
    assert rc == adg.ADG_EINVAL and "32-bit" in err
    rc, err = _init_leaves(1 << 14, 1 << 13, 1)   # 2^27 coarse cells
    assert rc == adg.ADG_EINVAL and "coarse" in err


def test_null_arguments_rejected():
    L = adg.lib()
    assert L.adg_step(None, None) == adg.ADG_EINVAL
    assert L.adg_destroy(None) == adg.ADG_EINVAL
    assert L.adg_set_state(None, None, None, None) == adg.ADG_EINVAL
    assert L.adg_step_static(None, None, None, None) == adg.ADG_EINVAL
    assert L.adg_batch_set_mode(None, 1) == adg.ADG_EINVAL
    assert L.adg_step_to(None, None, None, None, None) == adg.ADG_EINVAL


def _init3(phys, mesh):
    p = adg.make_params(phys)
    d = adg.make_mesh3_desc(mesh)
    h = ctypes.c_void_p()
    rc = adg.lib().adg3_init_mesh(ctypes.byref(p), ctypes.byref(d), ctypes.byref(h))
    return rc, adg.lib().adg_last_error().decode()


@pytest.mark.parametrize("change,msg", [
    (dict(N=0), "order"), (dict(N=6), "order"), (dict(gamma=1.0), "gas"), (dict(cfl=0.0), "cfl"),
])
def test_invalid_params_rejected_3d(change, msg):
    w = I.bubble3d()
    rc, err = _init3(dict(w["phys"], **change), w["mesh"])
    assert rc == adg.ADG_EINVAL and msg in err


def test_manufactured_source_unsupported_in_3d():
    w = I.bubble3d()
    rc, err = _init3(dict(w["phys"], mms=1), w["mesh"])
    assert rc == adg.ADG_EUNSUPPORTED and "two-dimensional" in err


@pytest.mark.parametrize("change,msg", [
    (dict(nx=0), "domain"), (dict(h=0.0), "domain"), (dict(h=float("nan")), "domain"),
    (dict(bc=[0, 1, 1, 1, 1, 1]), "pairs"), (dict(bc=[1, 1, 1, 1, 1, 7]), "bc"),
    (dict(nx=1024, ny=1024, nz=64), "too many"),
])
def test_invalid_mesh_rejected_3d(change, msg):
    w = I.bubble3d()
    rc, err = _init3(w["phys"], dict(w["mesh"], **change))
    assert rc == adg.ADG_EINVAL and msg in err


def test_null_arguments_rejected_3d():
    L = adg.lib()
    assert L.adg3_step(None, None) == adg.ADG_EINVAL
    assert L.adg3_destroy(None) == adg.ADG_EINVAL
    assert L.adg3_set_state(None, None, None, None) == adg.ADG_EINVAL
    assert L.adg3_init_mesh(None, None, None) == adg.ADG_EINVAL


def _init_fv(phys, mesh):
    p = adg.make_params(dict(phys, N=phys.get("N", 0)))
    d = adg.make_fv_desc(mesh)
    h = ctypes.c_void_p()
    rc = adg.lib().adg_fv_init(ctypes.byref(p), ctypes.byref(d), ctypes.byref(h))
    return rc, adg.lib().adg_last_error().decode()


@pytest.mark.parametrize("change,code,msg", [
    (dict(N=1), adg.ADG_EINVAL, "order"), (dict(gamma=0.9), adg.ADG_EINVAL, "gas"),
    (dict(cfl=0.0), adg.ADG_EINVAL, "cfl"), (dict(mu=1e-3), adg.ADG_EUNSUPPORTED, "inviscid"),
    (dict(mms=1), adg.ADG_EUNSUPPORTED, "manufactured"),
])
def test_invalid_params_rejected_fv(change, code, msg):
    w = I.fv_bubbles()
    rc, err = _init_fv(dict(w["phys"], **change), w["mesh"])
    assert rc == code and msg in err


@pytest.mark.parametrize("change,msg", [
    (dict(nx=0), "domain"), (dict(bc=[0, 1, 1, 1]), "pairs"), (dict(bc=[1, 1, 1, 9]), "bc"),
])
def test_invalid_mesh_rejected_fv(change, msg):
    w = I.fv_bubbles()
    rc, err = _init_fv(w["phys"], dict(w["mesh"], **change))
    assert rc == adg.ADG_EINVAL and msg in err


def test_null_arguments_rejected_fv():
    L = adg.lib()
    assert L.adg_fv_step(None, None) == adg.ADG_EINVAL
    assert L.adg_fv_destroy(None) == adg.ADG_EINVAL
    assert L.adg_fv_init(None, None, None) == adg.ADG_EINVAL


def test_peaks_arguments_checked_before_any_device_work():
    L = adg.lib()
    nb = ctypes.c_size_t()
    assert L.adg_peaks_sink_bytes(ctypes.byref(nb)) == adg.ADG_OK and nb.value > 0
    assert L.adg_peaks_sink_bytes(None) == adg.ADG_EINVAL
    out = (ctypes.c_double * 3)()
    assert L.adg_measure_peaks(None, None, None, 0, out, None) == adg.ADG_EINVAL
    assert L.adg_measure_peaks(ctypes.c_void_p(16), None, None, 0, None, None) == adg.ADG_EINVAL
    # a copy size with null buffers, and a size that is not a multiple of 16
    assert L.adg_measure_peaks(ctypes.c_void_p(16), None, None, 64, out, None) == adg.ADG_EINVAL
    assert L.adg_measure_peaks(ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(32), 40, out,
                               None) == adg.ADG_EINVAL
