"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, the ctypes structures match the C layouts, and the host-side
argument checks reject bad calls before anything is enqueued."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2606_30436_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kgs.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:kgs_status|void|const char\*)\s+(kgs_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED)


STRUCTS = {
    "kgs_camera": L.KgsCamera, "kgs_config": L.KgsConfig, "kgs_gaussians": L.KgsGaussians,
    "kgs_image": L.KgsImage, "kgs_grads": L.KgsGrads, "kgs_view_stats": L.KgsViewStats,
    "kgs_lifecycle_state": L.KgsLifecycleState, "kgs_buffers": L.KgsBuffers, "kgs_chunk_desc": L.KgsChunkDesc,
    "kgs_spawn_list": L.KgsSpawnList, "kgs_gaussians_out": L.KgsGaussiansOut, "kgs_anchors": L.KgsAnchors,
}


def test_struct_layouts_match_the_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "kgs.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    for line in out:
        if not line:
            continue
        cname, field, val = line.split()
        cls = STRUCTS[cname]
        if field == "size":
            assert ctypes.sizeof(cls) == int(val), cname
        else:
            assert getattr(cls, field).offset == int(val), (cname, field)


def _cfg(**kw):
    c = L.kgs_config_default(320, 240)
    c.max_views, c.max_gaussians, c.slot_capacity, c.pair_capacity = 2, 1000, 2000, 16000
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("bad", [dict(tile_w=12), dict(batch=100), dict(tile_w=32, tile_h=16, batch=128), dict(batch=256),
                                 dict(sh_degree=4), dict(max_views=0),
                                 dict(max_views=65), dict(width=0), dict(pair_capacity=2 ** 32), dict(alpha_min=0.0)])
def test_invalid_configs_are_rejected(bad):
    with pytest.raises(L.KgsError) as e:
        L.kgs_workspace_size(_cfg(**bad))
    assert e.value.code == L.KGS_ERR_INVALID_ARG


def test_host_argument_checks_and_call_order():
    lib = L.load()
    cfg = _cfg()
    n = L.kgs_workspace_size(cfg)
    assert n > 0
    # the context only carves the workspace: a host buffer stands in for device
    # memory here, and every call below fails its host check before any launch
    raw = ctypes.create_string_buffer(n + 512)
    base = (ctypes.addressof(raw) + 255) & ~255
    h = ctypes.c_void_p()
    assert lib.kgs_create(ctypes.byref(cfg), ctypes.c_void_p(base + 1), n, ctypes.byref(h)) == L.KGS_ERR_INVALID_ARG
    assert lib.kgs_create(ctypes.byref(cfg), ctypes.c_void_p(base), n - 1, ctypes.byref(h)) == L.KGS_ERR_INVALID_ARG
    assert lib.kgs_create(ctypes.byref(cfg), ctypes.c_void_p(base), n, ctypes.byref(h)) == L.KGS_OK
    ctx = h
    try:
        assert lib.kgs_bin_sort(ctx, None) == L.KGS_ERR_STATE
        img = L.KgsImage()
        assert lib.kgs_render_fwd(ctx, ctypes.byref(img), None) == L.KGS_ERR_INVALID_ARG
        assert lib.kgs_project(ctx, None, None, 1, None, None) == L.KGS_ERR_INVALID_ARG
        g = L.KgsGaussians()
        g.n = 5000  # above max_gaussians
        assert lib.kgs_project(ctx, ctypes.byref(g), ctypes.c_void_p(8), 1, None, None) == L.KGS_ERR_INVALID_ARG
        g.n = 10
        assert lib.kgs_project(ctx, ctypes.byref(g), ctypes.c_void_p(8), 1, None, None) == L.KGS_ERR_INVALID_ARG
        assert lib.kgs_set_tiling(ctx, 8, 32, 64) == L.KGS_OK
        assert lib.kgs_set_tiling(ctx, 8, 8, 64) == L.KGS_ERR_INVALID_ARG
        assert lib.kgs_set_tiling(ctx, 32, 16, 64) == L.KGS_OK
        assert lib.kgs_set_tiling(ctx, 16, 32, 128) == L.KGS_ERR_INVALID_ARG
        assert lib.kgs_chunk_launch(None, None) == L.KGS_ERR_INVALID_ARG
        assert lib.kgs_status_string(3) == b"device capacity exceeded"
    finally:
        lib.kgs_destroy(ctx)


def test_library_refuses_to_run_without_its_build(tmp_path, monkeypatch):
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        L.load(str(tmp_path / "missing.so"))


def test_static_chunk_close_host_checks():
    """The allocation-free chunk close rejects bad arguments on the host (no
    device address is looked up, nothing is launched)."""
    lib = L.load()
    st, s = L.KgsViewStats(), L.KgsLifecycleState()
    assert lib.kgs_accumulate_stats_static(ctypes.byref(st), 10, 2, ctypes.byref(s), 5.0, 0, None) == L.KGS_ERR_INVALID_ARG
    st.kappa_sum = st.omega_sum = st.gamma_sum = 8
    s.densify = s.prune_score = 8
    for n, V in ((L.ACCUMULATE_STATIC_MAX_N + 1, 2), (-1, 2), (10, 0)):
        assert lib.kgs_accumulate_stats_static(ctypes.byref(st), n, V, ctypes.byref(s), 5.0, 0, None) == L.KGS_ERR_INVALID_ARG
    assert lib.kgs_accumulate_stats_static(None, 10, 2, ctypes.byref(s), 5.0, 0, None) == L.KGS_ERR_INVALID_ARG
