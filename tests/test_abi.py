"""C ABI checks that need no GPU: the library loads, exports every function
include/helm.h declares, fills the default options, sizes the workspace and
rejects invalid arguments on the host before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2608_22946_amd import helm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(helm._LIB_PATH):
        from paper_2608_22946_amd import build
        build.build()
    return helm.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "helm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(helm_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(helm.EXPORTED)


def test_default_options_match_paper_protocol(L):
    o = helm.default_options()
    assert o.struct_size == ctypes.sizeof(helm.HelmOptions)
    assert (o.sigma, o.omega_h, o.omega_2h, o.omega_4h, o.gamma_max) == (0.9, 0.8, 0.8, 0.2, 1.119058)
    assert (o.nJ_h, o.nJ_2h, o.nJ_4h, o.m_h, o.c_2h, o.m_2h, o.m_4h, o.m_out) == (2, 2, 2, 2, 2, 10, 4, 5)


def _opts(**kw):
    o = helm.default_options()
    o.iofd_K = 40
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ws(L, dims, n_pml, o):
    b = ctypes.c_size_t(0)
    rc = L.helm_workspace_size(*dims, n_pml, ctypes.byref(o), ctypes.byref(b))
    return rc, b.value


def test_workspace_size_scales_with_grid_and_precision(L):
    rc, b32 = _ws(L, (56, 56, 56), 4, _opts(precision=helm.FP32))
    assert rc == 0
    rc, b64 = _ws(L, (56, 56, 56), 4, _opts(precision=helm.FP64))
    assert rc == 0
    n0 = 65 ** 3
    # at least the outer basis (11), smoother (5) and FP64 x, b at the fine level
    assert b32 >= n0 * (16 * 8 + 2 * 16)
    assert b64 > b32
    rc, big = _ws(L, (112, 112, 112), 8, _opts(precision=helm.FP32))
    assert 7.0 < big / b32 < 9.0


@pytest.mark.parametrize("dims,n_pml", [((10, 12, 12), 0), ((12, 12, 12), -1), ((0, 12, 12), 2), ((2, 2, 2), 1),
                                        ((4094, 8, 8), 2)])
def test_bad_dims_rejected(L, dims, n_pml):
    rc, _ = _ws(L, dims, n_pml, _opts())
    assert rc == helm.HELM_OK - 1   # HELM_EINVAL
    assert L.helm_last_error(None)


def test_mixed_workspace_is_smaller_and_needs_two_sweeps(L):
    """HELM_MIXED keeps the 2h-4h cycle's vectors and K_2h's Z in half precision
    (4 bytes per complex node) and runs only the fused two-sweep Jacobi there."""
    rc, b32 = _ws(L, (56, 56, 56), 4, _opts(precision=helm.FP32))
    rc2, bmx = _ws(L, (56, 56, 56), 4, _opts(precision=helm.MIXED))
    assert rc == 0 and rc2 == 0
    n1, n2 = 33 ** 3, 17 ** 3
    # Z2 (10) + y, r at 2h and P (5) + Z (4) + e at 4h drop from 8 to 4 bytes per node
    saved = 4 * (12 * n1 + 10 * n2)
    assert abs((b32 - bmx) - saved) <= 256 * 40, (b32 - bmx, saved)
    for field in ("nJ_2h", "nJ_4h"):
        for nj in (1, 3):
            rc, _ = _ws(L, (56, 56, 56), 4, _opts(precision=helm.MIXED, **{field: nj}))
            assert rc == -1
            assert b"nJ_2h and nJ_4h must be 2" in L.helm_last_error(None)


def test_workspace_grows_by_one_solver_copy_per_lane(L):
    sizes = [_ws(L, (56, 56, 56), 4, _opts(lanes=k))[1] for k in (1, 2, 3)]
    assert sizes[1] > sizes[0] and sizes[2] - sizes[1] == sizes[1] - sizes[0]
    assert _ws(L, (56, 56, 56), 4, _opts(lanes=0))[1] == sizes[0]


def test_workspace_grows_linearly_with_batch(L):
    """Each batched slot holds one more copy of the lane's vectors, states and partials."""
    sizes = [_ws(L, (56, 56, 56), 4, _opts(batch=k))[1] for k in (1, 2, 3)]
    # equal steps up to the 256-byte alignment of the workspace slices
    assert sizes[1] > sizes[0] and abs((sizes[2] - sizes[1]) - (sizes[1] - sizes[0])) <= 256 * 64
    assert _ws(L, (56, 56, 56), 4, _opts(batch=0))[1] == sizes[0]
    # one slot's copy is at least the lane's fine-level vectors (outer 11, smoother 5, x, b, temporary)
    assert sizes[1] - sizes[0] >= 65 ** 3 * (17 * 8 + 2 * 16)


def test_good_tile_options_accepted(L):
    for tz in (0, 2, 3, 6, 8, 12, 16, 24, 32, 64):
        for split in (-1, 0, 1):
            rc, _ = _ws(L, (24, 24, 24), 4, _opts(tile_tz=tz, tile_split=split))
            assert rc == 0, (tz, split)


@pytest.mark.parametrize("field,value", [("m_out", 0), ("m_2h", 13), ("m_4h", 9), ("nJ_h", 0), ("c_2h", 0),
                                         ("iofd_K", 0), ("omega_2h", -0.1), ("struct_size", 8), ("precision", 7),
                                         ("tile_tz", 1), ("tile_tz", 65), ("tile_tz", -1), ("tile_split", 2), ("tile_split", -2),
                                         ("lanes", 9), ("lanes", -1), ("pml_variant", 3), ("pml_variant", -1),
                                         ("batch", 9), ("batch", -1)])
def test_bad_options_rejected(L, field, value):
    rc, _ = _ws(L, (24, 24, 24), 4, _opts(**{field: value}))
    assert rc == -1


def test_setup_validates_before_device_work(L):
    """Every failure below is decided on the host; none touches the GPU."""
    tab = helm.table_flat(helm.load_table())
    o = _opts()
    o.iofd_table = tab.ctypes.data
    out = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)
    # NULL velocity
    assert L.helm_setup(None, 24, 24, 24, 10.0, 1.0, 4, ctypes.byref(o), dummy, 1 << 30, ctypes.byref(out)) == -1
    # bad h / omega
    assert L.helm_setup(dummy, 24, 24, 24, -1.0, 1.0, 4, ctypes.byref(o), dummy, 1 << 30, ctypes.byref(out)) == -1
    assert L.helm_setup(dummy, 24, 24, 24, 10.0, float("nan"), 4, ctypes.byref(o), dummy, 1 << 30,
                        ctypes.byref(out)) == -1
    # missing table
    o2 = _opts()
    assert L.helm_setup(dummy, 24, 24, 24, 10.0, 1.0, 4, ctypes.byref(o2), dummy, 1 << 30, ctypes.byref(out)) == -1
    # non-finite table entry
    bad = tab.copy()
    bad[5] = np.nan
    o3 = _opts()
    o3.iofd_table = bad.ctypes.data
    assert L.helm_setup(dummy, 24, 24, 24, 10.0, 1.0, 4, ctypes.byref(o3), dummy, 1 << 30, ctypes.byref(out)) == -1
    # pml_variant 2 needs at least two PML cells
    o4 = _opts(pml_variant=2)
    o4.iofd_table = tab.ctypes.data
    assert L.helm_setup(dummy, 24, 24, 24, 10.0, 1.0, 0, ctypes.byref(o4), dummy, 1 << 30, ctypes.byref(out)) == -1
    assert b"pml_variant 2" in L.helm_last_error(None)
    # workspace too small, and misaligned
    assert L.helm_setup(dummy, 24, 24, 24, 10.0, 1.0, 4, ctypes.byref(o), dummy, 100, ctypes.byref(out)) == -2
    assert L.helm_setup(ctypes.c_void_p(0x1001), 24, 24, 24, 10.0, 1.0, 4, ctypes.byref(o), ctypes.c_void_p(0x1008),
                        1 << 40, ctypes.byref(out)) == -2
    assert b"workspace" in L.helm_last_error(None)


def test_calls_on_null_hierarchy(L):
    its = np.zeros(1, np.int32)
    rel = np.zeros(1)
    assert L.helm_solve(None, ctypes.c_void_p(8), 1, 1e-6, ctypes.c_void_p(16), its.ctypes.data, rel.ctypes.data) == -1
    assert L.helm_apply(None, 0, 0, ctypes.c_void_p(8), ctypes.c_void_p(16)) == -1
    assert L.helm_residual_restrict(None, 0, 0, ctypes.c_void_p(8), ctypes.c_void_p(16), ctypes.c_void_p(24)) == -1
    assert L.helm_grad(None, None, None, None, 1, 1e-6, None, None, 0, None, None) == -1
    assert L.helm_solve_checkpoint(None, None, 1, 1e-6, None, None, None, None) == -1
    nb = ctypes.c_size_t(0)
    assert L.helm_grad_workspace_size(None, ctypes.byref(nb)) == -1
    L.helm_destroy(None)


def test_static_dots_rejects_arguments_on_host(L):
    """helm_vec_dots_static validates before touching the device (no GPU here)."""
    w = ctypes.c_void_p(16)
    assert L.helm_vec_dots_static(7, 10, 0, None, w, w, None) == -1           # precision
    assert L.helm_vec_dots_static(helm.FP32, 0, 0, None, w, w, None) == -1    # n
    assert L.helm_vec_dots_static(helm.FP32, 10, 13, None, w, w, None) == -1  # k > 12
    assert L.helm_vec_dots_static(helm.FP32, 10, 2, None, w, w, None) == -1   # V missing
    assert L.helm_vec_dots_static(helm.FP64, 10, 0, None, w, None, None) == -1  # out missing


def test_tile_file_checked_on_the_cpu(L, tmp_path):
    """helm_tiles_load reads and checks a tile-choice file without a GPU (nothing matches an
    architecture then); bad paths, foreign files and malformed lines are rejected."""
    n = ctypes.c_int(-1)
    good = tmp_path / "tiles.txt"
    good.write_text("# helm tile choices v2\n"
                    "gfx950 1 0 0 -1 1 352 352 352 24 0\n"
                    "gfx950 1 1 0 -1 8 176 176 176 12 1\n")
    assert L.helm_tiles_load(str(good).encode(), ctypes.addressof(n)) == 0 and n.value == 0
    assert L.helm_tiles_load(None, None) == -1
    assert L.helm_tiles_save(None) == -1
    assert L.helm_tiles_load(str(tmp_path / "missing.txt").encode(), None) == -1
    assert L.helm_tiles_save(str(tmp_path / "no" / "such" / "dir.txt").encode()) == -1
    for bad in ["gfx950 1 0 0 -1 1 352 352 352 24 0\n",                                 # no header
                "# helm tile choices v1\ngfx950 1 0 0 -1 352 352 352 24 0\n",            # older format
                "# helm tile choices v2\ngfx950 1 0 0 -1 1 352 352 352 24\n",            # field missing
                "# helm tile choices v2\ngfx950 1 0 0 -1 1 352 352 352 65 0\n",          # depth > 64
                "# helm tile choices v2\ngfx950 3 0 0 -1 1 352 352 352 24 0\n",          # precision
                "# helm tile choices v2\ngfx950 1 0 0 -1 9 352 352 352 24 0\n",          # slots > 8
                "# helm tile choices v2\ngfx950 1 0 0 -1 1 352 352 352 24 0 7\n",        # trailing field
                ""]:
        f = tmp_path / "bad.txt"
        f.write_text(bad)
        assert L.helm_tiles_load(str(f).encode(), None) == -1, bad
        assert L.helm_last_error(None)
    # saving an empty table writes the header alone, which loads again
    out = tmp_path / "saved.txt"
    assert L.helm_tiles_save(str(out).encode()) == 0
    assert out.read_text().splitlines()[0] == "# helm tile choices v2"
    assert L.helm_tiles_load(str(out).encode(), ctypes.addressof(n)) == 0 and n.value == 0
