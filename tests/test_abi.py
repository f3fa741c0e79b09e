"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/tetsplat.h declares, sizes workspaces, and rejects bad
arguments before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2406_01579_amd import _lib
    return _lib


def _declared():
    src = open(os.path.join(ROOT, "include", "tetsplat.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(render_\w+)\s*\(", src, flags=re.M)))


def test_header_functions_exported(L):
    names = _declared()
    assert len(names) >= 9
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_struct_layout_matches_header(L, tmp_path):
    """ctypes mirrors of the ABI structs have the C compiler's size and offsets."""
    import subprocess
    structs = {"render_scene": L.render_scene, "render_view": L.render_view, "render_params": L.render_params,
               "render_grads": L.render_grads, "render_status": L.render_status,
               "render_debug_view": L.render_debug_view}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tetsplat.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


class _Fake:
    def __init__(self, p):
        self.p = p

    def data_ptr(self):
        return self.p


def _args(L, w, tile=(16, 16), ptr=4096):
    from paper_2406_01579_amd import frontend
    sc = w.scenes[0]
    scenes = (L.render_scene * 1)(L.render_scene(ptr, ptr, ptr, ptr, sc.V, sc.K, sc.s))
    views = frontend.make_views(w.cams, [0] * w.cams.shape[0], [_Fake(ptr)] * w.cams.shape[0])
    p = frontend.Params(tile_w=tile[0], tile_h=tile[1]).c()
    return scenes, views, p


def _size(L, scenes, views, p, kept=0, ent=0):
    n = C.c_size_t(0)
    rc = L.lib().render_workspace_size(C.byref(scenes), len(scenes), C.byref(views), len(views), C.byref(p),
                                       kept, ent, C.byref(n))
    return rc, n.value


def test_workspace_size_scales(L):
    w = synth.tiny()
    scenes, views, p = _args(L, w)
    rc, a = _size(L, scenes, views, p)
    assert rc == 0 and a > 0
    rc, b = _size(L, scenes, views, p, kept=2000, ent=100000)
    assert rc == 0 and b != a
    rc, c = _size(L, scenes, views, p, kept=2000, ent=200000)
    assert rc == 0 and c > b
    for tile in [(8, 8), (16, 8), (8, 16), (16, 16), (32, 8)]:
        s2, v2, p2 = _args(L, w, tile)
        assert _size(L, s2, v2, p2)[0] == 0


@pytest.mark.parametrize("tile", [(12, 16), (4, 4), (32, 32), (0, 8)])
def test_bad_tile_rejected(L, tile):
    scenes, views, p = _args(L, synth.tiny(), tile)
    rc, _ = _size(L, scenes, views, p)
    assert rc == L.RENDER_EINVAL
    assert b"tile" in L.lib().render_last_error()


def test_bad_arguments_rejected_before_device_work(L):
    lib = L.lib()
    w = synth.tiny()
    scenes, views, p = _args(L, w)
    ws = 1 << 20
    # null scenes
    assert lib.render_forward(None, 1, C.byref(views), 1, C.byref(p), 0, 0, ws, 1 << 30, None) == L.RENDER_EINVAL
    # scene index out of range
    views[0].scene = 3
    assert lib.render_forward(C.byref(scenes), 1, C.byref(views), 1, C.byref(p), 0, 0, ws, 1 << 30,
                              None) == L.RENDER_EINVAL
    assert b"scene index" in lib.render_last_error()
    views[0].scene = 0
    # null output image
    views[0].out = None
    assert lib.render_forward(C.byref(scenes), 1, C.byref(views), 1, C.byref(p), 0, 0, ws, 1 << 30,
                              None) == L.RENDER_EINVAL
    views[0].out = 4096
    # unaligned tet pointer
    scenes[0].tets = 4100
    assert lib.render_forward(C.byref(scenes), 1, C.byref(views), 1, C.byref(p), 0, 0, ws, 1 << 30,
                              None) == L.RENDER_EINVAL
    scenes[0].tets = 4096
    # unknown flag, bad clamp
    p.flags = 64
    assert lib.render_forward(C.byref(scenes), 1, C.byref(views), 1, C.byref(p), 0, 0, ws, 1 << 30,
                              None) == L.RENDER_EINVAL
    p.flags = 0
    p.alpha_clamp = 1.5
    assert lib.render_forward(C.byref(scenes), 1, C.byref(views), 1, C.byref(p), 0, 0, ws, 1 << 30,
                              None) == L.RENDER_EINVAL
    p.alpha_clamp = 0.99
    p.waves = 3
    assert lib.render_forward(C.byref(scenes), 1, C.byref(views), 1, C.byref(p), 0, 0, ws, 1 << 30,
                              None) == L.RENDER_EINVAL
    assert b"waves" in lib.render_last_error()
    p.waves = 4
    # misaligned workspace
    assert lib.render_forward(C.byref(scenes), 1, C.byref(views), 1, C.byref(p), 0, 0, ws + 4, 1 << 30,
                              None) == L.RENDER_EINVAL
    # too small a workspace
    rc, need = _size(L, scenes, views, p)
    assert lib.render_forward(C.byref(scenes), 1, C.byref(views), 1, C.byref(p), 0, 0, ws, need - 256,
                              None) == L.RENDER_ENOSPC
    assert b"needs" in lib.render_last_error()
    # backward needs gradient buffers and upstream gradients
    assert lib.render_backward(C.byref(scenes), 1, C.byref(views), 1, C.byref(p), 0, 0, ws, need, None, None,
                               None) == L.RENDER_EINVAL


def test_static_forward_rejects_a_problem_past_its_workspace(L):
    """The no-allocation forward checks its size on the host, before any
    device work: a problem whose workspace exceeds the static array is
    refused with RENDER_ENOSPC; bad arguments as render_forward."""
    lib = L.lib()
    w = synth.training(s=320.0, R=8, size=64, views=1)
    scenes, views, p = _args(L, w)
    assert lib.render_forward_static(None, 1, C.byref(views), 1, C.byref(p), 0, 0, None, None) == L.RENDER_EINVAL
    # 8 views at 4096^2 of the same scene: far past 64 MiB
    big = (L.render_view * 8)()
    for v in range(8):
        C.memmove(C.byref(big[v]), C.byref(views[0]), C.sizeof(L.render_view))
        big[v].width = big[v].height = 4096
    rc, need = _size(L, scenes, big, p)
    assert rc == 0 and need > L.STATIC_WORKSPACE_BYTES
    assert lib.render_forward_static(C.byref(scenes), 1, C.byref(big), 8, C.byref(p), 0, 0, None,
                                     None) == L.RENDER_ENOSPC
    assert b"static workspace" in lib.render_last_error()


def test_decode_status_roundtrip(L):
    hdr = np.zeros(64, np.uint32)
    hdr[0], hdr[1], hdr[2], hdr[3], hdr[4] = 11, 22, 33, 2, 0
    h8 = hdr.view(np.uint8).copy()
    h8[32:40] = np.frombuffer(np.int64(1000).tobytes(), np.uint8)
    h8[40:48] = np.frombuffer(np.int64(500).tobytes(), np.uint8)
    h8[48:56] = np.frombuffer(np.uint64(44).tobytes(), np.uint8)
    s = L.render_status()
    assert L.lib().render_decode_status(h8.ctypes.data, C.byref(s)) == 0
    assert (s.kept, s.records, s.entries, s.overflow) == (11, 22, 33, 2)
    assert (s.entry_capacity, s.kept_capacity, s.entries_needed) == (1000, 500, 44)


def test_profile_api_without_work(L):
    L.profile(True)
    d = L.profile_read()
    assert all(v == (0.0, 0) for v in d.values())
    L.profile(False)


def test_product_path_has_no_cpu_fallback():
    """The package never imports the oracle and fails loudly without the library."""
    import paper_2406_01579_amd
    pkg = os.path.dirname(paper_2406_01579_amd.__file__)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(root, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
    from paper_2406_01579_amd import _lib
    saved = _lib.LIB_PATH, _lib._lib
    try:
        _lib.LIB_PATH, _lib._lib = "/nonexistent/libtetsplat.so", None
        with pytest.raises(RuntimeError, match="missing"):
            _lib.lib()
    finally:
        _lib.LIB_PATH, _lib._lib = saved


def test_regularizer_entry_points_validate_on_the_host(L):
    lib = L.lib()
    n = C.c_size_t(0)
    assert lib.render_mesh_edges_workspace_size(1000, C.byref(n)) == L.RENDER_OK and n.value > 4 * 4 * 6000
    assert lib.render_mesh_edges_workspace_size(-1, C.byref(n)) == L.RENDER_EINVAL
    assert lib.render_regularizers_workspace_size(100, 300, C.byref(n)) == L.RENDER_OK
    need = n.value
    assert need >= 2 * 4 * 3 * 100
    ws = 1 << 20
    # unaligned tets, null count, too small a workspace
    assert lib.render_mesh_edges(4100, 10, 20, 8192, 4096, ws, 1 << 20, None) == L.RENDER_EINVAL
    assert lib.render_mesh_edges(4096, 10, 20, 8192, None, ws, 1 << 20, None) == L.RENDER_EINVAL
    assert lib.render_mesh_edges(4096, 10, 20, 8192, 4096, ws, 16, None) == L.RENDER_ENOSPC
    # gradients: both buffers or neither, and weights with them
    args = [4096, 8192, 12288, 100, 300, 16384, 20480, 1800]
    assert lib.render_regularizers(*args, None, None, 24576, None, ws, need, None) == L.RENDER_EINVAL
    assert lib.render_regularizers(*args, None, None, 24576, 28672, ws, need, None) == L.RENDER_EINVAL
    assert lib.render_regularizers(*args, 32768, None, 24576, 28672, ws, need - 256, None) == L.RENDER_ENOSPC
    assert lib.render_regularizers(*args[:5], 16388, 20480, 1800, None, None, None, None, ws, need,
                                   None) == L.RENDER_EINVAL


def test_resort_window_arguments(L):
    """The resort window is 0..RENDER_WINDOW_MAX on 8x8 tiles; with it on, the
    workspace holds 44 bytes per entry for its backward's blend records,
    blend masks and pair places, and not the per-tile order's 8-byte blend
    mask per entry: 36 bytes per entry more."""
    w = synth.tiny()
    scenes, views, p = _args(L, w, (8, 8))
    rc, base = _size(L, scenes, views, p, ent=10000)
    assert rc == 0
    p.window = 5
    rc, with_win = _size(L, scenes, views, p, ent=10000)
    assert rc == 0 and 36 * 10000 <= with_win - base <= 36 * 10000 + 3 * 256
    for bad in (-1, L.RENDER_WINDOW_MAX + 1):
        p.window = bad
        assert _size(L, scenes, views, p)[0] == L.RENDER_EINVAL
        assert b"window" in L.lib().render_last_error()
    s2, v2, p2 = _args(L, w, (16, 16))
    p2.window = 3
    assert _size(L, s2, v2, p2)[0] == L.RENDER_EINVAL
    assert b"8x8" in L.lib().render_last_error()


def test_chunk_length_arguments(L):
    """LDS chunk lengths: forward 32/64, backward 16/32 (0: the defaults), on
    the multi-wave 8x8 path only; they do not change the workspace."""
    w = synth.tiny()
    scenes, views, p = _args(L, w, (8, 8))
    rc, base = _size(L, scenes, views, p)
    assert rc == 0
    for cf, cb in ((32, 16), (64, 32), (32, 0), (0, 16)):
        p.chunk_fwd, p.chunk_bwd = cf, cb
        rc, n = _size(L, scenes, views, p)
        assert rc == 0 and n == base
    for cf, cb in ((16, 0), (128, 0), (0, 8), (0, 64), (-32, 0)):
        p.chunk_fwd, p.chunk_bwd = cf, cb
        assert _size(L, scenes, views, p)[0] == L.RENDER_EINVAL
        assert b"chunk" in L.lib().render_last_error()
    p.chunk_fwd, p.chunk_bwd = 32, 16
    for waves, window in ((1, 0), (4, 3)):
        p.waves, p.window = waves, window
        assert _size(L, scenes, views, p)[0] == L.RENDER_EINVAL
    p.waves, p.window = 4, 0
    s2, v2, p2 = _args(L, w, (16, 16))
    p2.chunk_fwd = 32
    assert _size(L, s2, v2, p2)[0] == L.RENDER_EINVAL


def test_coarse_grid_entry_points_validate_on_the_host(L):
    """Bad resolutions, null and misaligned pointers are rejected before any
    device work (the pointers below are never dereferenced)."""
    lib = L.lib()
    assert lib.render_cube_grid(0, 4096, 8192, 16384, None) == L.RENDER_EINVAL
    assert lib.render_cube_grid(1025, 4096, 8192, 16384, None) == L.RENDER_EINVAL
    assert lib.render_cube_grid(8, None, 8192, 16384, None) == L.RENDER_EINVAL
    assert lib.render_cube_grid(8, 4096, None, 16384, None) == L.RENDER_EINVAL
    assert lib.render_cube_grid(8, 4096, 8192, 16388, None) == L.RENDER_EINVAL
    assert lib.render_refit_cube(4096, 8192, 0, 16384, None) == L.RENDER_EINVAL
    assert lib.render_refit_cube(None, 8192, 8, 16384, None) == L.RENDER_EINVAL
    assert lib.render_refit_cube(4096, 8192, 8, 16386, None) == L.RENDER_EINVAL
    assert b"misaligned" in lib.render_last_error()


def test_memory_flags_shrink_or_grow_the_workspace(L):
    """RENDER_RECOMPUTE_STATE drops the 8 B per pixel of compositing state;
    RENDER_RECORD_GRADS replaces 96 B per entry by 96 B per record;
    RENDER_DETERMINISTIC adds its corner sort (4 x 48 B per kept tet); the
    last two exclude each other."""
    w = synth.training(s=320.0, R=16, size=128, views=2)
    scenes, views, p = _args(L, w, (8, 8))
    kept, ent = 3000, 40000
    rc, base = _size(L, scenes, views, p, kept, ent)
    assert rc == 0
    pixels = 2 * 128 * 128
    rec = 2 * kept
    p.flags = L.RENDER_RECOMPUTE_STATE
    rc, a = _size(L, scenes, views, p, kept, ent)
    assert rc == 0 and abs((base - a) - 8 * pixels) <= 512
    p.flags = L.RENDER_RECORD_GRADS
    rc, b = _size(L, scenes, views, p, kept, ent)
    assert rc == 0 and abs((base - b) - 96 * (ent - rec)) <= 512
    p.flags = L.RENDER_RECOMPUTE_STATE | L.RENDER_RECORD_GRADS
    rc, c = _size(L, scenes, views, p, kept, ent)
    assert rc == 0 and abs((base - c) - 8 * pixels - 96 * (ent - rec)) <= 1024
    p.flags = L.RENDER_DETERMINISTIC
    rc, d = _size(L, scenes, views, p, kept, ent)
    assert rc == 0 and d - base >= 4 * kept * 48
    p.flags = L.RENDER_DETERMINISTIC | L.RENDER_RECORD_GRADS
    rc, _ = _size(L, scenes, views, p, kept, ent)
    assert rc == L.RENDER_EINVAL and b"exclude" in L.lib().render_last_error()
