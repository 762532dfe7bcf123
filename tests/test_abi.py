"""Host-side checks of the C ABI: the library loads and exports what the header declares."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1411_0278_amd import mbstokes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbstokes.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mbs_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_bound_entry_points():
    assert set(declared_functions()) == set(mbstokes.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(mbstokes.LIB_PATH):
        pytest.skip("libmbstokes.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(mbstokes.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", mbstokes.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (mbs_[a-z_0-9]+)", out))
    assert set(declared_functions()) <= exported


def test_default_params_and_struct_layout():
    if not os.path.exists(mbstokes.LIB_PATH):
        pytest.skip("libmbstokes.so not built")
    p = mbstokes.default_params()
    assert p.lmax == 2 and p.restart == 30 and abs(p.tol - 1e-10) < 1e-25
    assert abs(p.eta * 6 * 3.141592653589793 - 1) < 1e-15 and p.a == 1.0
    assert p.plane == 0 and p.plane_z == 0.0 and p.box == 0.0 and p.ewald_xi == 0.0 and p.ewald_mesh == 0
    assert ctypes.sizeof(mbstokes.Params) == 9 * 8 + 14 * 4
    assert ctypes.sizeof(mbstokes.Stats) == 4 * 4 + 8 * 8 + 2 * 4
    assert ctypes.sizeof(mbstokes.SlipEx) == 3 * 8


def _struct_fields(name):
    """Field names of `typedef struct name { ... } name;` in the header, in order."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), txt, flags=re.S).group(1)
    return re.findall(r"\b(?:const\s+)?(?:int32_t|int64_t|double|float|uint32_t)\s*\*?\s*([a-z_0-9]+)\s*;", body)


def test_binding_structs_match_the_header_field_by_field():
    """The ctypes mirrors of the parameter, statistics and slip structs name the header's fields in the
    header's order (a field added, renamed or moved on one side only would shift the others)."""
    for cname, py in (("mbs_params", mbstokes.Params), ("mbs_stats", mbstokes.Stats),
                      ("mbs_slip_ex", mbstokes.SlipEx)):
        assert _struct_fields(cname) == [f[0] for f in py._fields_], cname


def test_create_without_gpu_fails_cleanly():
    """Without a visible device mbs_create returns an error code, never a context."""
    if not os.path.exists(mbstokes.LIB_PATH):
        pytest.skip("libmbstokes.so not built")
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = mbstokes.load()
    h = ctypes.c_void_p()
    p = mbstokes.default_params()
    rc = lib.mbs_create(ctypes.byref(h), 0, ctypes.byref(p))
    assert rc != 0 and not h.value
    assert len(lib.mbs_last_error(None)) > 0


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1411_0278_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, flags=re.M), f
                assert "oracle/" not in txt, f


def test_trap_checkpoint_roundtrip(tmp_path):
    """The checkpoint format: plain arrays in a .npz, read back without pickling."""
    import numpy as np

    from paper_1411_0278_amd import trap
    rng = np.random.default_rng(0)
    R, p, hist = rng.standard_normal((7, 3)), rng.standard_normal((7, 3)), rng.standard_normal(77)
    path = str(tmp_path / "ck.npz")
    trap.save_checkpoint(path, 12, R, p, hist, 0.5, (1.0, 0.5, 0.0), 0.01, 2)
    ck = trap.load_checkpoint(path)
    assert int(ck["step"]) == 12 and int(ck["order"]) == 2 and float(ck["dt"]) == 0.01
    assert np.array_equal(ck["R"], R) and np.array_equal(ck["p"], p) and np.array_equal(ck["hist"], hist)
    assert tuple(ck["slip_coef"]) == (1.0, 0.5, 0.0) and float(ck["k_trap"]) == 0.5
