"""The C-ABI library loads and exports every function include/md.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")
LIB = os.path.join(ROOT, "paper_2405_07898_amd", "libmdeam.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:md_status|void|size_t|const char\*)\s+(md_\w+)\s*\(", text,
                       flags=re.M)
    return sorted(set(names))


def test_header_declares_the_api():
    names = declared_functions()
    for required in ("md_init", "md_init_batch", "md_workspace_bytes", "md_create",
                     "md_build_neighbors", "md_step", "md_energy", "md_fm_forward",
                     "md_fm_backward", "md_autotune"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
def test_binding_matches_header():
    from paper_2405_07898_amd import md

    assert sorted(md.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
def test_status_strings_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.md_status_string.restype = ctypes.c_char_p
    assert lib.md_status_string(0) == b"ok"
    assert b"capacity" in lib.md_status_string(-4)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
@pytest.mark.parametrize("box,ok", [
    ((20.0, 20.0, 20.0), True),
    ((10.0, 20.0, 20.0), False),    # periodic edge below 2 (r_cut + skin) = 10.6
    ((-3.0, -3.0, -3.0), True),     # open edges: any positive extent, one cell
    ((-3.0, -3.0, 10.0), False),    # the periodic edge is still checked
    ((-40.0, -40.0, 16.5), True),   # a slab: open x, y, periodic z with 3 cells
    ((0.0, 20.0, 20.0), False),
    ((-0.0, 20.0, 20.0), False),
    ((float("inf"), 20.0, 20.0), False),
    ((-float("nan"), 20.0, 20.0), False),
])
def test_box_validation_without_gpu(box, ok):
    """md_workspace_size validates the box on the host: a positive length is a
    periodic edge, a negative one an open edge of that extent."""
    import numpy as np

    from paper_2405_07898_amd import md

    lib = md.lib()
    p = md.make_params(mass=183.84, dt=1.0, r_cut=5.0, skin=0.3, ftm2v=1.0)
    n = (ctypes.c_int64 * 1)(1000)
    b = np.array(box, dtype=np.float64)
    out = ctypes.c_size_t(0)
    rc = lib.md_workspace_size(ctypes.byref(p), 1, n, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(out))
    assert (rc == 0) == ok, rc
    if not ok:
        assert rc == -2
    else:
        assert out.value > 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
@pytest.mark.parametrize("prec,mode,ok", [(0, 0, True), (1, 0, True), (0, 1, True), (1, 1, False),
                                          (0, 2, False)])
def test_list_mode_validation_without_gpu(prec, mode, ok):
    """The half-list form exists in float64 only; unknown list forms are rejected."""
    import numpy as np

    from paper_2405_07898_amd import md

    lib = md.lib()
    p = md.make_params(mass=183.84, dt=1.0, r_cut=5.0, skin=0.3, ftm2v=1.0, precision=prec,
                       list_mode=mode)
    n = (ctypes.c_int64 * 1)(1000)
    b = np.array([20.0, 20.0, 20.0])
    full = ctypes.c_size_t(0)
    out = ctypes.c_size_t(0)
    rc = lib.md_workspace_size(ctypes.byref(p), 1, n, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(out))
    assert (rc == 0) == ok
    if not ok:
        assert rc == -1
    elif mode == 1:
        # the half form's pair slots: 52 + 52 cap bytes per atom more than the full list
        p0 = md.make_params(mass=183.84, dt=1.0, r_cut=5.0, skin=0.3, ftm2v=1.0)
        lib.md_workspace_size(ctypes.byref(p0), 1, n, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              ctypes.byref(full))
        extra = out.value - full.value
        per_atom = 52 + 52 * 128
        assert per_atom * 1000 <= extra <= per_atom * 1000 + 11 * 256


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
@pytest.mark.parametrize("nt,prec,mode,ok", [(0, 0, 0, True), (1, 0, 0, True), (2, 0, 0, True),
                                             (4, 0, 0, True), (5, 0, 0, False), (-1, 0, 0, False),
                                             (2, 1, 0, False), (2, 0, 1, False)])
def test_type_count_validation_without_gpu(nt, prec, mode, ok):
    """Several atom types: up to MD_MAX_TYPES, float64 and the full list only;
    the workspace grows with the type count."""
    import numpy as np

    from paper_2405_07898_amd import md

    lib = md.lib()
    n = (ctypes.c_int64 * 1)(1000)
    b = np.array([20.0, 20.0, 20.0])

    def size(**kw):
        p = md.make_params(mass=183.84, dt=1.0, r_cut=5.0, skin=0.3, ftm2v=1.0, **kw)
        out = ctypes.c_size_t(0)
        rc = lib.md_workspace_size(ctypes.byref(p), 1, n,
                                   b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(out))
        return rc, out.value

    rc, sz = size(n_types=nt, precision=prec, list_mode=mode)
    assert (rc == 0) == ok, rc
    if ok and nt > 1:
        assert sz > size()[1]


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
@pytest.mark.parametrize("launch,mode,nt,ok", [(0, 0, 0, True), (1, 0, 0, True), (2, 0, 0, False),
                                               (1, 1, 0, False), (1, 0, 2, False)])
def test_launch_mode_validation_without_gpu(launch, mode, nt, ok):
    """The persistent launch runs the one-species full-list passes only."""
    import numpy as np

    from paper_2405_07898_amd import md

    lib = md.lib()
    p = md.make_params(mass=183.84, dt=1.0, r_cut=5.0, skin=0.3, ftm2v=1.0, launch_mode=launch,
                       list_mode=mode, n_types=nt)
    n = (ctypes.c_int64 * 1)(1000)
    b = np.array([20.0, 20.0, 20.0])
    out = ctypes.c_size_t(0)
    rc = lib.md_workspace_size(ctypes.byref(p), 1, n, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(out))
    assert (rc == 0) == ok


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
@pytest.mark.parametrize("knots,ok", [((64, 64, 64), True), ((600, 600, 600), True),
                                      ((700, 700, 700), False)])
def test_fm_table_size_limit_without_gpu(knots, ok):
    """The force-matching coefficient histogram (4 bins per segment, 8 bytes
    each, all three tables) must fit 64 KB of LDS."""
    import numpy as np

    from paper_2405_07898_amd import md

    lib = md.lib()
    lib.md_fm_workspace_size.restype = ctypes.c_int32
    n = (ctypes.c_int64 * 1)(2000)
    b = np.array([33.04, 33.04, 33.04])
    nk = (ctypes.c_int32 * 3)(*knots)
    out = ctypes.c_size_t(0)
    rc = lib.md_fm_workspace_size(1, n, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.c_double(5.0), 128, nk, ctypes.byref(out))
    assert (rc == 0) == ok, rc
    if not ok:
        assert rc == -3


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
@pytest.mark.parametrize("atoms,cap,ok", [
    ((1,), 128, True),                      # the smallest system
    ((0,), 128, False),                     # an empty replica
    ((500, 0, 500), 128, False),            # an empty replica inside a batch
    ((-3,), 128, False),
    ((8_388_607,), 128, True),              # the largest list at capacity 128
    ((8_388_608,), 128, False),             # 2^32 bytes of list
    ((4_194_304, 4_194_304), 128, False),   # the same, over two replicas
    ((67_108_863,), 16, True),              # the largest atom index
    ((67_108_864,), 8, False),              # 2^26 atoms
])
def test_size_limits_without_gpu(atoms, cap, ok):
    """md_workspace_size checks the sizes on the host: at least one atom per
    replica, fewer than 2^26 atoms (26-bit list index) and below 2^32 bytes of
    list."""
    import numpy as np

    from paper_2405_07898_amd import md

    lib = md.lib()
    p = md.make_params(mass=183.84, dt=1.0, r_cut=5.0, skin=0.3, ftm2v=1.0, nbr_capacity=cap)
    n = (ctypes.c_int64 * len(atoms))(*atoms)
    b = np.tile(np.array([400.0, 400.0, 400.0]), len(atoms))
    out = ctypes.c_size_t(0)
    rc = lib.md_workspace_size(ctypes.byref(p), len(atoms), n,
                               b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(out))
    assert (rc == 0) == ok, rc
    if not ok:
        assert rc == -1
    else:
        assert out.value >= 4 * cap * sum(atoms)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
def test_no_replicas_without_gpu():
    import numpy as np

    from paper_2405_07898_amd import md

    lib = md.lib()
    p = md.make_params(mass=183.84, dt=1.0, r_cut=5.0, skin=0.3, ftm2v=1.0)
    n = (ctypes.c_int64 * 1)(100)
    b = np.array([20.0, 20.0, 20.0])
    out = ctypes.c_size_t(0)
    rc = lib.md_workspace_size(ctypes.byref(p), 0, n, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(out))
    assert rc == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
def test_workspace_bytes_matches_workspace_size_without_gpu():
    """md_workspace_bytes returns md_workspace_size's count, and 0 for sizes
    that md_workspace_size rejects."""
    import numpy as np

    from paper_2405_07898_amd import md

    lib = md.lib()
    p = md.make_params(mass=183.84, dt=1.0, r_cut=5.0, skin=0.3, ftm2v=1.0)
    n = (ctypes.c_int64 * 2)(1000, 250)
    b = np.array([[20.0, 20.0, 20.0], [-30.0, -30.0, 16.0]], dtype=np.float64)
    bp = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    out = ctypes.c_size_t(0)
    assert lib.md_workspace_size(ctypes.byref(p), 2, n, bp, ctypes.byref(out)) == 0
    assert lib.md_workspace_bytes(ctypes.byref(p), 2, n, bp) == out.value > 0
    bad = np.array([[10.0, 20.0, 20.0]], dtype=np.float64)
    assert lib.md_workspace_bytes(ctypes.byref(p), 1, n,
                                  bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
    assert lib.md_workspace_bytes(None, 1, n, bp) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmdeam.so not built")
def test_init_rejects_bad_arguments_without_gpu():
    """md_init / md_init_batch validate parameters, sizes and the box on the
    host before any device call, and leave *out NULL."""
    import numpy as np

    from paper_2405_07898_amd import md

    lib = md.lib()
    p = md.make_params(mass=183.84, dt=1.0, r_cut=5.0, skin=0.3, ftm2v=1.0)
    ctx = ctypes.c_void_p(1234)
    box = np.array([10.0, 20.0, 20.0])  # below 2 (r_cut + skin)
    rc = lib.md_init(ctypes.byref(ctx), ctypes.byref(p), 100,
                     box.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, None, None,
                     ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256), 1 << 20,
                     None)
    assert rc in (md.MD_E_BOX, md.MD_E_TABLE) and ctx.value is None
    ctx = ctypes.c_void_p(1234)
    rc = lib.md_init_batch(ctypes.byref(ctx), ctypes.byref(p), 1, None, None, None, None, None,
                           None, None, None, 0, None)
    assert rc == md.MD_E_ARG and ctx.value is None
