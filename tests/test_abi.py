"""CPU checks of the boundary: the HIP library builds for gfx950, loads, and
exports every function include/vlbm.h declares (no compute call without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2401_17183_amd", "libvlbm.so")


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(?:int|const char\s*\*)\s*(vlbm_\w+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_paper_calls():
    names = declared_functions()
    for n in ["vlbm_mesh_create", "vlbm_geometry_precompute", "vlbm_init", "vlbm_step", "vlbm_moments"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvlbm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvlbm.so not built")
def test_binding_signatures_cover_the_header():
    from paper_2401_17183_amd import vlbm
    assert set(declared_functions()) <= set(vlbm._SIGS), set(declared_functions()) - set(vlbm._SIGS)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvlbm.so not built")
def test_lattice_tables_match_the_oracle():
    """Host-only call: the library's velocity tables equal the oracle's."""
    import numpy as np
    from oracle import lattice
    from paper_2401_17183_amd import vlbm
    for name, code in (("D2Q9", vlbm.D2Q9), ("D3Q19", vlbm.D3Q19), ("D2Q21", vlbm.D2Q21), ("D3Q39", vlbm.D3Q39)):
        c, w = vlbm.lattice_info(code)
        lat = lattice.by_name(name)
        assert np.array_equal(c, lat.c), name
        # each side writes its weights as its own fractions: equal to rounding
        assert np.allclose(w, lat.w, rtol=2e-16, atol=0), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvlbm.so not built")
def test_argument_errors_without_a_device():
    """Validation happens before any device call."""
    import numpy as np
    from paper_2401_17183_amd import vlbm
    topo = vlbm.vlbm_topology()
    h = ctypes.c_void_p()
    n = (ctypes.c_int64 * 3)(4, 4, 2)    # D2Q9 with n[2] != 1
    X = np.zeros(16 * 2)
    with pytest.raises(vlbm.VlbmError) as e:
        vlbm.vlbm_mesh_create(vlbm.D2Q9, n, X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(topo),
                              1.0, ctypes.byref(h))
    assert e.value.code == vlbm.ERR_ARG
    n = (ctypes.c_int64 * 3)(4, 4, 1)
    topo.face[1][0] = vlbm.PERIODIC
    topo.face[1][1] = vlbm.WALL
    with pytest.raises(vlbm.VlbmError) as e:
        vlbm.vlbm_mesh_create(vlbm.D2Q9, n, X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(topo),
                              1.0, ctypes.byref(h))
    assert e.value.code == vlbm.ERR_ARG and "periodic" in str(e.value)


@pytest.mark.parametrize("case", ["empty", "huge", "lattice", "dx", "face", "null"])
def test_mesh_arguments_rejected_without_a_device(case):
    """Empty and oversized index boxes, unknown lattices and face kinds, a
    non-positive dx and null pointers fail with VLBM_ERR_ARG on the host."""
    import numpy as np
    from paper_2401_17183_amd import vlbm
    topo = vlbm.vlbm_topology()
    h = ctypes.c_void_p()
    lattice, n, dx = vlbm.D2Q9, [4, 4, 1], 1.0
    if case == "empty":
        n = [0, 4, 1]
    elif case == "huge":
        n = [1 << 21, 4, 1]
    elif case == "lattice":
        lattice = 7
    elif case == "dx":
        dx = -1.0
    elif case == "face":
        topo.face[0][0] = 5
    nn = (ctypes.c_int64 * 3)(*n)
    X = np.zeros(16 * 2)
    ptr = None if case == "null" else X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    with pytest.raises(vlbm.VlbmError) as e:
        vlbm.vlbm_mesh_create(lattice, nn, ptr, ctypes.byref(topo), dx, ctypes.byref(h))
    assert e.value.code == vlbm.ERR_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvlbm.so not built")
@pytest.mark.parametrize("lattice,n,faces,code", [
    ("D3Q39", (4, 4, 4), "two walls", "UNSUPPORTED"),  # three-cell links: walls on one axis at most
    ("D3Q39", (4, 4, 4), "far field", "UNSUPPORTED"),  # and no far field
    ("D2Q21", (4, 2, 1), "periodic", "ARG"),           # an axis shorter than the longest link
    ("D2Q21", (4, 4, 2), "periodic", "ARG")])           # a 2-D lattice with n[2] != 1
def test_long_link_lattices_rejected_where_unsupported(lattice, n, faces, code):
    """Lattices with links up to three cells long take axes of at least three
    cells, walls on one axis at most and no far field; the checks run on the
    host."""
    import numpy as np
    from paper_2401_17183_amd import vlbm
    topo = vlbm.vlbm_topology()
    if faces == "two walls":
        topo.face[1][0] = topo.face[1][1] = vlbm.WALL
        topo.face[2][0] = topo.face[2][1] = vlbm.WALL
    elif faces == "far field":
        topo.face[1][0] = vlbm.WALL
        topo.face[1][1] = vlbm.FARFIELD
    h = ctypes.c_void_p()
    X = np.zeros(4096)
    with pytest.raises(vlbm.VlbmError) as e:
        vlbm.vlbm_mesh_create(vlbm.LATTICES[lattice], (ctypes.c_int64 * 3)(*n),
                              X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(topo), 1.0,
                              ctypes.byref(h))
    assert e.value.code == getattr(vlbm, "ERR_" + code)


def test_conv_descriptor_rejected_without_a_device():
    """Channel counts off the multiple of 8, bad strides and upsampling with a
    stride fail before any device call."""
    from paper_2401_17183_amd import vlbm
    for d in (vlbm.conv_desc(1, 8, 8, 12, 16), vlbm.conv_desc(1, 8, 8, 16, 16, stride=3),
              vlbm.conv_desc(1, 8, 8, 16, 16, upsample=True, stride=2), vlbm.conv_desc(0, 8, 8, 16, 16)):
        with pytest.raises(vlbm.VlbmError) as e:
            vlbm.vlbm_conv2d_forward(ctypes.byref(d), ctypes.c_void_p(16), None, ctypes.c_void_p(16), None,
                                     ctypes.c_void_p(16), None, None)
        assert e.value.code == vlbm.ERR_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvlbm.so not built")
def test_batch_calls_reject_a_null_batch():
    """Batch entry points check their handle on the host."""
    from paper_2401_17183_amd import vlbm
    for call, args in ((vlbm.vlbm_batch_set_active, (None, None)), (vlbm.vlbm_batch_step, (None, 1)),
                       (vlbm.vlbm_batch_residuals, (None, None))):
        with pytest.raises(vlbm.VlbmError) as e:
            call(*args)
        assert e.value.code == vlbm.ERR_ARG
