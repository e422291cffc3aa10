"""The C ABI: the library loads, exports every entry point the header declares, and
rejects invalid arguments on the host (no GPU work is started by these calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oit.h")
LIB = os.path.join(ROOT, "paper_2605_13855_amd", "liboit.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(oit_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_host_validation_rejects_bad_arguments(lib):
    from paper_2605_13855_amd import oit
    from paper_2605_13855_amd import scenes
    cam = scenes.look_at_camera((0, 0, -3), 64, 48)
    cams = oit.camera_array([cam])
    cap = oit.Capacity(100, 100, 0)
    tu = oit.Tuning(16, 64, 1000)
    assert oit.workspace_bytes(cap, cams, 1, tu) > 0
    assert oit.workspace_bytes(cap, cams, 1, oit.Tuning(12, 64, 1000)) == 0
    assert b"tile" in oit.lib.oit_last_error()
    assert oit.workspace_bytes(cap, cams, 0, tu) == 0
    assert oit.workspace_bytes(oit.Capacity(100, 200, 0), cams, 1, tu) == 0
    assert oit.workspace_bytes(cap, cams, 1, oit.Tuning(16, 48, 1000)) == 0
    bad = scenes.look_at_camera((0, 0, -3), 0, 48)
    assert oit.workspace_bytes(cap, oit.camera_array([bad]), 1, tu) == 0
    # render_fwd with NULL splats fails before any device work
    rc = oit.lib.oit_render_fwd(None, None, None, cams, 1, ctypes.byref(cap), None, None, None, None, None,
                                None, None, None, None, None, 0, ctypes.byref(tu), None)
    assert rc == -1
    rc = oit.lib.oit_update_active_set(None, 10, 0, 5, 0.0, None, None, 0, None, None, None, 0, None, None, 0, None)
    assert rc == -1
    assert oit.lib.oit_select_workspace_bytes(0) == 0
    assert oit.lib.oit_select_workspace_bytes(5000) > 5000
    # the no-allocation selection refuses sizes beyond its static scratch on the host
    rc = oit.lib.oit_update_active_set_noalloc(None, oit.NOALLOC_SELECT_MAX_N + 1, 0, 5, 0.0, None, None, 0, None,
                                               None, None, 0, None, None, None)
    assert rc == -1 and b"scratch" in oit.lib.oit_last_error()
    rc = oit.lib.oit_update_active_set_noalloc(None, 10, 0, 5, 0.0, None, None, 0, None, None, None, 0, None, None,
                                               None)
    assert rc == -1


def test_workspace_grows_with_views_and_capacity(lib):
    from paper_2605_13855_amd import oit
    from paper_2605_13855_amd import scenes
    cams1 = oit.camera_array([scenes.look_at_camera((0, 0, -3), 64, 48)])
    cams2 = oit.camera_array([scenes.look_at_camera((0, 0, -3), 64, 48)] * 2)
    tu = oit.Tuning(16, 64, 1000)
    a = oit.workspace_bytes(oit.Capacity(100, 100, 0), cams1, 1, tu)
    b = oit.workspace_bytes(oit.Capacity(100, 100, 0), cams2, 2, tu)
    c = oit.workspace_bytes(oit.Capacity(100, 50, 50), cams1, 1, tu)
    assert b > a and c < a + 100 * 100


def test_host_api_compiles_without_warnings():
    """The host layer compiles warning-free with -Wall (an infinitely recursive helper, for
    one, is only visible as a warning and once sent garbage pointers to the GPU)."""
    import subprocess
    import sys
    sys.path.insert(0, ROOT)
    from paper_2605_13855_amd import build as B
    src = os.path.join(ROOT, "paper_2605_13855_amd", "csrc", "oit_api.hip")
    cmd = [B.hipcc(), *B.FLAGS, "-c", src, "-o", os.devnull]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    bad = [ln for ln in (r.stdout + r.stderr).splitlines() if "warning:" in ln and not B._benign(ln)]
    assert not bad, bad


def test_density_entry_points_validate_on_host(lib):
    """The densification calls reject bad arguments before any device work."""
    from paper_2605_13855_amd import oit
    from paper_2605_13855_amd import scenes
    assert oit.densify_workspace_bytes(0) == 0
    assert oit.densify_workspace_bytes(1000) >= 6 * 4000
    cam = scenes.look_at_camera((0, 0, -3), 64, 48)
    cams = oit.camera_array([cam])
    cap = oit.Capacity(100, 100, 0)
    tu = oit.Tuning(16, 64, 1000)
    fake = ctypes.c_void_p(4096)
    # no accumulators
    assert oit.lib.oit_densify_stats(cams, 1, ctypes.byref(cap), None, None, None, None, None, None, fake, 1 << 30,
                                     ctypes.byref(tu), None) == -1
    # dense mode with a device count
    assert oit.lib.oit_densify_stats(cams, 1, ctypes.byref(cap), None, fake, None, fake, fake, fake, fake, 1 << 30,
                                     ctypes.byref(tu), None) == -1
    assert oit.lib.oit_densify_plan(None, None, None, None, None, None, None, None, 0, None) == -1
    sp = oit.Splats(100, *([4096] * 6))
    bad = oit.DensityRules(2e-4, 0.01, 0.0, 0.005, 0.0, 0.0, 1.0, 0)       # extent 0
    assert oit.lib.oit_densify_plan(ctypes.byref(sp), fake, fake, fake, fake, ctypes.byref(bad), fake, fake,
                                    1 << 30, None) == -1
    assert b"rules" in oit.lib.oit_last_error()
    ok_rules = oit.DensityRules(2e-4, 0.01, 1.0, 0.005, 0.0, 0.0, 1.0, 0)
    assert oit.lib.oit_densify_plan(ctypes.byref(sp), fake, fake, fake, fake, ctypes.byref(ok_rules), fake, fake,
                                    16, None) == -4                              # workspace too small
    P6 = ctypes.c_void_p * 6
    six = P6(*([4096] * 6))
    assert oit.lib.oit_densify_apply(ctypes.byref(sp), six, six, None, six, six, six, 10, fake, 1 << 30, None) == -1
    assert oit.lib.oit_reset_opacity(None, None, None, 10, 0.01, None) == -1
    assert oit.lib.oit_reset_opacity(fake, fake, fake, 10, 1.5, None) == -1


def test_l1_loss_workspace_is_the_render_workspace_head(lib):
    """oit_l1_loss needs a fixed head (status, camera table, its block shares); every
    render workspace starts with that head, and a smaller buffer is refused on the host."""
    from paper_2605_13855_amd import oit
    from paper_2605_13855_amd import scenes
    need = oit.l1_loss_workspace_bytes()
    assert need >= 2048 * 8 and need % 256 == 0
    for w, h, views in ((64, 48, 1), (1600, 1200, 16), (1960, 1090, 8)):
        cams = oit.camera_array([scenes.look_at_camera((0, 0, -3), w, h)] * views)
        for tile in (8, 16, 32):
            assert oit.workspace_bytes(oit.Capacity(100, 100, 0), cams, views, oit.Tuning(tile, 64, 1)) >= need
    cams = oit.camera_array([scenes.look_at_camera((0, 0, -3), 64, 48)])
    fake = ctypes.c_void_p(4096)
    rc = oit.lib.oit_l1_loss(fake, fake, cams, 1, fake, fake, fake, need - 1, None)
    assert rc == -4 and b"needs" in oit.lib.oit_last_error()


def test_pair_capacity_bound_on_the_host(lib):
    """Tile-entry offsets are 32-bit: the host refuses a pair capacity of 2^32 - 1 or more,
    so every offset at or past the capacity (the device scan saturates there) is dropped
    and reported as an overflow instead of wrapping round."""
    from paper_2605_13855_amd import oit
    from paper_2605_13855_amd import scenes
    cams = oit.camera_array([scenes.look_at_camera((0, 0, -3), 64, 48)])
    cap = oit.Capacity(100, 100, 0)
    assert oit.workspace_bytes(cap, cams, 1, oit.Tuning(16, 64, 2 ** 32 - 2)) > 4 * (2 ** 32 - 2)
    assert oit.workspace_bytes(cap, cams, 1, oit.Tuning(16, 64, 2 ** 32 - 1)) == 0
    assert b"pair_capacity" in oit.lib.oit_last_error()
    assert oit.workspace_bytes(cap, cams, 1, oit.Tuning(16, 64, 0)) == 0
