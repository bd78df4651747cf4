"""CPU checks of the C ABI: the library loads and exports every entry point
include/*.h declares, and the binding covers each of them (no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(sw[bs]?_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sw_create", "sw_destroy", "sw_set_bed", "sw_set_soil", "sw_set_state",
                 "sw_set_inflow", "sw_set_sed_sources", "sw_advance", "sw_advance_fixed_dt",
                 "sw_get_fields", "sw_get_sums", "sw_last_error", "sw_replace_state",
                 "swb_create", "swb_advance", "sws_create", "sws_forward", "sws_train_step",
                 "sws_advance"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2103_15196_amd import csph
    lib = ctypes.CDLL(csph.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2103_15196_amd import csph
    bound = {n for n, _, _ in csph.SIGNATURES}
    assert set(declared_functions()) <= bound


def test_struct_layouts_match_header():
    from paper_2103_15196_amd import csph
    assert ctypes.sizeof(csph.sw_grid) == 4 + 4 + 8 + 16
    assert ctypes.sizeof(csph.sw_params) == 11 * 8 + 4 + 4 + 4 + 4
    assert ctypes.sizeof(csph.sws_stats) == 5 * 4 + 4 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(csph.sw_step_record) == 8 + 6 * 8 + 4 + 4
    p = csph.default_params()
    assert p.cfl == 0.3 and p.eps_dry == 1e-5 and p.sed_law == csph.SW_SED_EQ4
    assert p.limiter == csph.SW_LIM_MINMOD and p.hll_speeds == csph.SW_HLL_DAVIS


def test_product_path_does_not_touch_the_oracle():
    """The HIP binding and kernels never import, link or call the oracle."""
    pkg = os.path.join(ROOT, "paper_2103_15196_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f"{f} mentions the oracle"


def test_create_rejects_grids_beyond_the_32_bit_plane_offsets():
    """sw_create checks the size limit of include/csph.h before any HIP call:
    a pitched plane of 2^30 cells or more (the strip kernels' 32-bit byte
    offsets) is SW_ERR_ARG, as are empty grids and a non-positive dx."""
    from paper_2103_15196_amd import csph
    p = csph.default_params()
    h = ctypes.c_void_p()
    for nx, ny, dx in ((32768, 32768, 1.0), (65536, 16384, 1.0), (32769, 32767, 1.0),
                       (0, 10, 1.0), (10, 0, 1.0), (10, 10, 0.0), (10, 10, -1.0)):
        g = csph.make_grid(nx, ny, dx)
        rc = csph.lib.sw_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h))
        assert rc == csph.SW_ERR_ARG, (nx, ny, dx, rc)
        assert not h.value


def test_create_refuses_the_second_order_force_on_the_unfused_path():
    """The second-order force is built into the strip kernels only: sw_create
    refuses it with the unfused sequence before any HIP call."""
    from paper_2103_15196_amd import csph
    p = csph.default_params()
    p.flags = csph.SW_FLAG_FORCE2 | csph.SW_FLAG_UNFUSED
    h = ctypes.c_void_p()
    g = csph.make_grid(64, 32, 1.0)
    assert csph.lib.sw_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == csph.SW_ERR_ARG
    assert not h.value


def test_noalloc_rejects_grids_beyond_its_scratch_array():
    """sw_advance_noalloc checks its arguments and the size of the grid against
    its fixed scratch array before any HIP call: SW_ERR_ARG and a message."""
    from paper_2103_15196_amd import csph
    p = csph.default_params()
    buf = ctypes.create_string_buffer(256)
    dummy = ctypes.c_void_p(16)  # never dereferenced: rejected before any device work
    for nx, ny in ((2048, 1024), (1024, 1100), (4096, 4096), (0, 8)):
        g = csph.make_grid(nx, ny, 1.0)
        rc = csph.lib.sw_advance_noalloc(ctypes.byref(g), ctypes.byref(p), 0.02, 5e-4, 0.4,
                                         dummy, dummy, dummy, dummy, 10, 0.0, 0.0, None, None,
                                         None, buf, 256)
        assert rc == csph.SW_ERR_ARG, (nx, ny, rc)
        assert buf.value, (nx, ny)
    assert b"scratch" in buf.value or b"nx, ny" in buf.value
    g = csph.make_grid(1024, 1024, 1.0)
    rc = csph.lib.sw_advance_noalloc(ctypes.byref(g), ctypes.byref(p), 0.02, 5e-4, 1.0,
                                     dummy, dummy, dummy, dummy, 10, 0.0, 0.0, None, None, None,
                                     buf, 256)
    assert rc == csph.SW_ERR_ARG and b"psi" in buf.value
