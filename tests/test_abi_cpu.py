"""The C-ABI library without a GPU: it loads, exports every function that
include/ssr.h declares, its structures have the layout the binding assumes,
and the host-only paths (sizes, status strings, argument checks that return
before touching a device) behave as documented."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssr.h")
LIB = os.path.join(ROOT, "paper_2504_01358_amd", "libssr.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "_b", os.path.join(ROOT, "paper_2504_01358_amd", "build.py"))
        m = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(m)
        m.build()
    from paper_2504_01358_amd import ssr
    return ssr


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssr_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) == 25, names
    raw = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(raw, n), n
    assert set(names) == set(lib.SYMBOLS)


def test_struct_layout_matches_header(lib, tmp_path):
    src = tmp_path / "layout.c"
    fields = {
        "ssr_camera": ["width", "height", "pos", "rot", "fx", "fy", "cx", "cy", "z_near"],
        "ssr_gbuffer": ["depth", "normal_rough", "albedo_metal", "radiance", "dtype", "hiz"],
        "ssr_env": ["rgb", "width", "height", "mips"],
        "ssr_params": ["spp", "march", "max_steps", "step_len", "max_dist", "thickness", "seed",
                       "frame", "flags"],
        "ssr_session_cfg": ["hbm_budget_bytes", "max_slots", "max_bypass", "flags"],
        "ssr_request": ["scene_id", "params", "out_rgb"],
        "ssr_result": ["status", "t_submit", "t_admit", "t_done", "workspace_bytes"],
        "ssr_session_stats": ["scene_bytes", "arena_bytes", "arena_used", "running", "waiting",
                              "completed"],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ssr.h"', "int main(void){"]
    for s, fs in fields.items():
        lines.append(f'printf("{s} size %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n"):
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    py = {"ssr_camera": lib.Camera, "ssr_gbuffer": lib.GBuffer, "ssr_env": lib.Env,
          "ssr_params": lib.Params, "ssr_session_cfg": lib.SessionCfg, "ssr_request": lib.Request,
          "ssr_result": lib.Result, "ssr_session_stats": lib.SessionStats}
    for s, cls in py.items():
        assert got[(s, "size")] == ctypes.sizeof(cls), s
        for f in fields[s]:
            assert got[(s, f)] == getattr(cls, f).offset, (s, f)


def test_sizes_and_status_strings(lib):
    # env mip chain: levels He x 2He down to 1 x 2, four floats per texel
    assert lib.env_mips_floats(512, 256) == 4 * sum((512 >> k) * (256 >> k) for k in range(9))
    assert lib.env_mips_floats(2, 1) == 8
    for bad in ((512, 255), (500, 250), (256, 256), (0, 0), (2 * 16384, 16384)):
        assert lib.env_mips_floats(*bad) == 0
    # depth pyramid, levels 0..top with ceil halving, four floats per texel
    # (own pair, parent's pair), rows stored in pairs (an odd row count padded
    # by one), at most 4 GiB
    def hiz(w, h):
        n = w * (h + h % 2)
        while w > 1 or h > 1:
            w, h = (w + 1) // 2, (h + 1) // 2
            n += w * (h + h % 2)
        return 4 * n if 16 * n <= 2 ** 32 - 16 else 0
    for w, h in ((1920, 1080), (1, 1), (7, 3), (3840, 2160), (16384, 1), (16384, 12000),
                 (16384, 16384)):
        assert lib.hiz_floats(w, h) == hiz(w, h)
    assert lib.hiz_floats(16384, 16384) == 0
    assert lib.hiz_floats(0, 5) == 0 and lib.hiz_floats(16385, 2) == 0
    for s in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9, 1):
        assert lib.status_string(s) and lib.status_string(s) != "unknown status"
    assert lib.status_string(-99) == "unknown status"


def test_codes_count(lib):
    raw = lib.lib
    assert raw.ssr_codes_count(1920, 1080, 16, 0) == 1920 * 1080 * 16
    assert raw.ssr_codes_count(1920, 1080, 16, lib.CODES_TILED) == 240 * 135 * 64 * 16
    assert raw.ssr_codes_count(203, 117, 4, lib.CODES_TILED) == 26 * 15 * 64 * 4
    assert raw.ssr_codes_count(0, 5, 4, lib.CODES_TILED) == 0
    assert raw.ssr_codes_count(-1, 5, 4, 0) == 0
    assert lib.codes_shape(203, 117, 4, lib.CODES_TILED) == (26 * 15, 4, 64)
    assert lib.codes_shape(203, 117, 4) == (117, 203, 4)


def test_host_side_argument_checks(lib):
    raw = lib.lib
    cam = lib.Camera()
    g = lib.GBuffer()
    e = lib.Env()
    p = lib.Params()
    byref = ctypes.byref
    # null context / structures: rejected before any device work
    assert raw.ssr_shade(None, byref(cam), byref(g), byref(e), byref(p), None, None, None, None) == -1
    assert raw.ssr_trace(None, byref(cam), byref(g), byref(p), None, None, None) == -1
    assert raw.ssr_resolve(None, byref(cam), byref(g), byref(e), byref(p), None, None, None) == -1
    assert raw.ssr_env_build_mips(None, 512, 256, None, None) == -1
    assert raw.ssr_hiz_build(None, 16, 16, 0.0, None, None) == -1
    assert raw.ssr_philox4x32_10(None, None, 0, None, None) == 0
    assert raw.ssr_philox4x32_10(None, None, 5, None, None) == -1
    assert raw.ssr_philox4x32_10(None, None, -1, None, None) == -1
    assert raw.ssr_ctx_create(0, None) == -1
    cfg = lib.SessionCfg(1 << 30, 4, 4, 0)
    assert raw.ssr_session_create(0, byref(cfg), None) == -1
    h = ctypes.c_void_p()
    for bad in (lib.SessionCfg(0, 4, 4, 0), lib.SessionCfg(1 << 30, 0, 4, 0),
                lib.SessionCfg(1 << 30, 65, 4, 0), lib.SessionCfg(1 << 30, 4, -1, 0),
                lib.SessionCfg(1 << 30, 4, 4, 2)):
        assert raw.ssr_session_create(0, byref(bad), byref(h)) == -1
    assert raw.ssr_session_submit(None, None, None) == -1
    assert raw.ssr_session_poll(None, 1, None) == -1
    assert raw.ssr_session_wait(None, 1, None) == -1
    assert raw.ssr_session_request_bytes(None, None) == -1
    assert raw.ssr_session_get_stats(None, None) == -1
    # first pass: null context, bad table sizes, bad camera or storage type
    assert raw.ssr_first_pass(None, byref(cam), byref(g), byref(e), None, None) == -1
    for n in (-1, 0, 1, 1025):
        assert raw.ssr_brdf_lut(n, ctypes.c_void_p(16), None) == -1
    assert raw.ssr_brdf_lut(128, None, None) == -1
    assert raw.ssr_depth_normals(byref(cam), None, 0, None, None) == -1   # fx = 0
    ok = lib.Camera()
    ok.fx = ok.fy = 100.0
    ok.z_near = 0.01
    ok.rot[0] = ok.rot[4] = ok.rot[8] = 1.0
    assert raw.ssr_depth_normals(byref(ok), None, 0, None, None) == 0     # empty image
    assert raw.ssr_depth_normals(byref(ok), None, 3, None, None) == -2
    ok.width, ok.height = 4, 4
    assert raw.ssr_depth_normals(byref(ok), None, 0, None, None) == -1    # null buffers
    # the allocation-free entry point: its argument checks come before it
    # looks at any device (null structures, a bad camera, an empty image)
    assert raw.ssr_shade_static(None, byref(g), byref(e), byref(p), None, None, None, None) == -1
    assert raw.ssr_shade_static(byref(cam), None, byref(e), byref(p), None, None, None, None) == -1
    ok.width, ok.height = 0, 0
    p0 = lib.Params(1, 1, 64, 0.1, 10.0, 0.05, 0, 0, 0)
    g0 = lib.GBuffer(None, None, None, None, 0, None)
    e0 = lib.Env(ctypes.c_void_p(16), 8, 4, None)
    assert raw.ssr_shade_static(byref(ok), byref(g0), byref(e0), byref(p0), None, None, None, None) == 0
    raw.ssr_session_destroy(None)
    raw.ssr_ctx_destroy(None)


def test_static_scratch_size_matches_header(lib):
    text = open(HEADER).read()
    m = re.search(r"#define SSR_STATIC_SCRATCH_BYTES \((\d+)ll << (\d+)\)", text)
    assert m, "SSR_STATIC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == lib.STATIC_SCRATCH_BYTES
    # the headline frame (1920 x 1080, 16 samples) fits with every part in
    # scratch: counter, pyramid, tile-major codes, the 512 x 256 mip chain
    al = lambda n: (n + 255) // 256 * 256
    need = (256 + al(lib.hiz_floats(1920, 1080) * 4)
            + al(lib.lib.ssr_codes_count(1920, 1080, 16, lib.CODES_TILED) * 4)
            + al(lib.env_mips_floats(512, 256) * 4))
    assert need <= lib.STATIC_SCRATCH_BYTES
