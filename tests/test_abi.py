"""C-ABI checks that need no GPU: the library loads, exports every function
include/gs.h declares, and host-side validation rejects bad arguments with
the documented status before anything is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2604_12626_amd import binding
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    from paper_2604_12626_amd import binding
    assert set(binding.EXPORTS) == set(names)


def test_struct_layouts_match_header(lib):
    from paper_2604_12626_amd import binding as B
    assert ctypes.sizeof(B.Camera) == 64
    assert ctypes.sizeof(B.Params) == 4 * 12
    assert ctypes.sizeof(B.Gaussians) == 8 + 4 + 4 + 6 * 8
    assert ctypes.sizeof(B.Projected) == 24


def test_status_strings_and_defaults(lib):
    from paper_2604_12626_amd import binding as B
    assert lib.gs_version() == 2
    assert lib.gs_status_string(0) == b"GS_OK"
    assert lib.gs_status_string(3) == b"GS_ERR_WORKSPACE_TOO_SMALL"
    p = B.make_params(640, 480)
    assert (p.width, p.height) == (640, 480)
    assert p.alpha_max == pytest.approx(0.99) and p.alpha_min == pytest.approx(1 / 255) and p.t_min == pytest.approx(1e-4)
    assert p.near_plane == pytest.approx(0.2) and p.lowpass == pytest.approx(0.3) and p.sigma_cut == 3.0


def _err(lib):
    return lib.gs_last_error().decode()


def test_validation_rejects_bad_arguments_without_a_gpu(lib):
    from paper_2604_12626_amd import binding as B
    p = B.make_params(64, 64)
    seg = B.Gaussians()
    seg.n, seg.sh_degree = 10, 0
    seg.means = seg.opacity = seg.sh = ctypes.c_void_p(0x1000)
    seg.log_scales = ctypes.c_void_p(0x2000)
    seg.quats = ctypes.c_void_p(0x3000)
    cams = ctypes.c_void_p(0x4000)
    mask = (ctypes.c_uint32 * 1)(1)
    out = B.Projected(10, ctypes.c_void_p(0x5000), ctypes.c_void_p(0x6000))
    # no segments
    assert lib.gs_project(None, 0, cams, 1, mask, ctypes.byref(p), ctypes.byref(out), None) == B.GS_ERR_INVALID_ARGUMENT
    # SH degree 4
    seg.sh_degree = 4
    assert lib.gs_project(ctypes.byref(seg), 1, cams, 1, mask, ctypes.byref(p), ctypes.byref(out), None) == \
        B.GS_ERR_INVALID_ARGUMENT
    assert "sh_degree" in _err(lib)
    seg.sh_degree = 0
    # mask bit beyond n_segs
    bad = (ctypes.c_uint32 * 1)(2)
    assert lib.gs_project(ctypes.byref(seg), 1, cams, 1, bad, ctypes.byref(p), ctypes.byref(out), None) == \
        B.GS_ERR_INVALID_ARGUMENT
    # instance count mismatch
    out.n_instances = 11
    assert lib.gs_project(ctypes.byref(seg), 1, cams, 1, mask, ctypes.byref(p), ctypes.byref(out), None) == \
        B.GS_ERR_INVALID_ARGUMENT
    assert "n_instances" in _err(lib)
    # misaligned quaternions
    out.n_instances = 10
    seg.quats = ctypes.c_void_p(0x3004)
    assert lib.gs_project(ctypes.byref(seg), 1, cams, 1, mask, ctypes.byref(p), ctypes.byref(out), None) == \
        B.GS_ERR_INVALID_ARGUMENT
    # bad image size
    p2 = B.make_params(0, 64)
    assert lib.gs_project(ctypes.byref(seg), 1, cams, 1, mask, ctypes.byref(p2), ctypes.byref(out), None) == \
        B.GS_ERR_INVALID_ARGUMENT
    # an unknown layout
    seg.layout = 2
    assert lib.gs_project(ctypes.byref(seg), 1, cams, 1, mask, ctypes.byref(p), ctypes.byref(out), None) == \
        B.GS_ERR_INVALID_ARGUMENT
    assert "layout" in _err(lib)


def test_render_backward_validation(lib):
    """The backward's argument list as the header declares it (the work
    order after the ranges), and its host validation, without a GPU."""
    from paper_2604_12626_amd import binding as B
    p = B.make_params(64, 64)
    out = B.Projected(10, ctypes.c_void_p(0x5000), ctypes.c_void_p(0x6000))
    mask = (ctypes.c_uint32 * 1)(1)
    args = [None, 0, ctypes.c_void_p(0x4000), 1, mask, ctypes.byref(p), ctypes.byref(out), None, None, None, None,
            None, None, 0, None, None, None, None, 0, None, None]
    assert lib.gs_render_backward(*args) == B.GS_ERR_INVALID_ARGUMENT
    with pytest.raises(TypeError):
        lib.gs_render_backward(*args[:-1])


def test_bin_sort_capacity_and_workspace_errors(lib):
    from paper_2604_12626_amd import binding as B
    p = B.make_params(640, 480)
    proj = B.Projected(100, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000))
    a = ctypes.c_void_p(0x10000)
    ws_need = lib.gs_bin_sort_workspace(100, 1000, 1, ctypes.byref(p))
    assert ws_need > 0
    st = lib.gs_bin_sort(ctypes.byref(proj), 1, ctypes.byref(p), a, ws_need - 1, a, a, 1000, a, None, a, a, None)
    assert st == B.GS_ERR_WORKSPACE_TOO_SMALL
    st = lib.gs_bin_sort(ctypes.byref(proj), 1, ctypes.byref(p), a, ws_need, a, a, 1 << 30, a, None, a, a, None)
    assert st == B.GS_ERR_UNSUPPORTED
    st = lib.gs_bin_sort(ctypes.byref(proj), 1, ctypes.byref(p), a, ws_need, a, a, 0, a, None, a, a, None)
    assert st == B.GS_ERR_INVALID_ARGUMENT
    # workspace grows with capacity (ping-pong key/value buffers)
    assert lib.gs_bin_sort_workspace(100, 2000, 1, ctypes.byref(p)) >= ws_need + 1000 * 12


def test_lbs_and_composite_validation(lib):
    from paper_2604_12626_amd import binding as B
    a = ctypes.c_void_p(0x10000)
    assert lib.gs_deform_lbs(-1, a, a, a, a, a, a, a, 1, 24, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_deform_lbs(10, a, a, a, a, a, a, a, 1, 0, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_deform_lbs(10, None, a, a, a, a, a, a, 1, 24, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_deform_lbs(0, None, None, None, None, None, None, None, 1, 24, None, None, None) == B.GS_OK
    p = B.make_params(64, 64)
    proj = B.Projected(10, None, a)
    st = lib.gs_composite(ctypes.byref(proj), a, a, None, 1, ctypes.byref(p), a, 8, a, a, a, None, None, None, 0,
                          None)
    assert st == B.GS_ERR_WORKSPACE_TOO_SMALL
    st = lib.gs_composite(ctypes.byref(proj), None, a, None, 1, ctypes.byref(p), a, 256, a, a, a, None, None, None,
                          0, None)
    assert st == B.GS_ERR_INVALID_ARGUMENT
    ws = lib.gs_composite_workspace(1, ctypes.byref(p))
    st = lib.gs_composite(ctypes.byref(proj), a, a, ctypes.c_void_p(0x10002), 1, ctypes.byref(p), a, ws, a, a, a,
                          None, None, None, 0, None)
    assert st == B.GS_ERR_INVALID_ARGUMENT  # misaligned work order
    st = lib.gs_composite(ctypes.byref(proj), a, a, None, 1, ctypes.byref(p), a, ws, a, a, a, None, None,
                          ctypes.c_void_p(0x10002), 100, None)
    assert st == B.GS_ERR_INVALID_ARGUMENT  # misaligned checkpoints


def test_lbs_joint_gradient_validation(lib):
    from paper_2604_12626_amd import binding as B
    a = ctypes.c_void_p(0x10000)
    f = lib.gs_deform_lbs_backward_joints
    assert f(-1, a, a, a, a, a, a, a, 1, 24, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(10, a, a, a, a, a, a, a, 1, 24, a, a, None, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(10, a, a, a, a, a, a, None, 1, 24, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(10, a, a, a, a, a, a, a, 1, 300, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(10, a, a, a, a, a, a, ctypes.c_void_p(0x10008), 1, 24, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT


def test_forward_kinematics_validation(lib):
    from paper_2604_12626_amd import binding as B
    a = ctypes.c_void_p(0x10000)
    f = lib.gs_forward_kinematics
    par = lambda *p: (ctypes.c_int32 * len(p))(*p)
    assert f(0, 3, par(-1, 0, 1), None, None, None, None, None) == B.GS_OK
    assert f(2, 0, par(-1), a, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(2, 257, None, a, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(2, 3, None, a, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(2, 3, par(-1, 2, 0), a, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT  # child before parent
    assert "before" in _err(lib)
    assert f(2, 3, par(-1, 0, -2), a, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(2, 3, par(-1, 0, 1), a, None, a, a, None) == B.GS_ERR_INVALID_ARGUMENT


def test_lbs_clip_validation(lib):
    from paper_2604_12626_amd import binding as B
    a = ctypes.c_void_p(0x10000)
    f = lib.gs_deform_lbs_clip
    assert f(0, None, None, None, None, None, None, None, 0, None, None, None, 1, 24, None, None, None) == B.GS_OK
    assert f(10, a, a, a, a, a, a, a, 0, a, a, a, 1, 24, a, a, None) == B.GS_ERR_INVALID_ARGUMENT  # no frames
    assert f(10, a, a, a, a, a, a, None, 5, a, a, a, 1, 24, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(10, a, a, a, a, a, a, a, 5, a, None, a, 1, 24, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(10, a, a, a, a, a, a, ctypes.c_void_p(0x10004), 5, a, a, a, 1, 24, a, a, None) == \
        B.GS_ERR_INVALID_ARGUMENT  # misaligned clip
    assert f(10, a, a, a, a, a, a, a, 5, a, a, a, 0, 24, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    g = lib.gs_deform_lbs_clip_backward
    assert g(10, a, a, a, a, a, a, a, 5, a, a, None, 1, 24, a, a, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert g(10, a, a, a, a, a, a, a, 5, a, a, a, 1, 24, a, a, a, a, None, None) == B.GS_ERR_INVALID_ARGUMENT


def test_capsule_queries_validation(lib):
    from paper_2604_12626_amd import binding as B
    a = ctypes.c_void_p(0x10000)
    f = lib.gs_capsule_queries
    ok = [a, a, a, 0.1, 1.5, a, 4, 23, a, a, a, 2, a, a, a, a, None]
    assert f(0, *([None] * 3), 0.1, 1.5, None, 0, 0, None, None, None, 0, None, None, None, None, None) == B.GS_OK
    assert f(-1, *ok) == B.GS_ERR_INVALID_ARGUMENT
    for k, bad in ((3, -0.1), (3, float("nan")), (4, float("inf")), (6, 0), (7, 0), (11, 0)):
        args = list(ok)
        args[k] = bad
        assert f(5, *args) == B.GS_ERR_INVALID_ARGUMENT, k
    for k in (0, 2, 5, 8, 9, 10, 12):  # required arrays
        args = list(ok)
        args[k] = None
        assert f(5, *args) == B.GS_ERR_INVALID_ARGUMENT, k
    args = list(ok)
    args[1] = None  # no step but step outputs given
    assert f(5, *args) == B.GS_ERR_INVALID_ARGUMENT and "all" in _err(lib)
    args = list(ok)
    args[5] = ctypes.c_void_p(0x10004)  # misaligned capsules
    assert f(5, *args) == B.GS_ERR_INVALID_ARGUMENT


def test_sensor_compose_validation(lib):
    from paper_2604_12626_amd import binding as B
    a = ctypes.c_void_p(0x10000)
    bad = ctypes.c_void_p(0x10002)
    f = lib.gs_sensor_compose
    assert f(0, 4, 4, None, None, None, None, None, None, None, None) == B.GS_OK  # no views: no-op
    assert f(-1, 4, 4, a, a, a, None, None, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(1, 0, 4, a, a, a, None, None, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(1, 4, (1 << 16) + 1, a, a, a, None, None, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(100000, 1 << 16, 1 << 16, a, a, a, None, None, a, a, None) == B.GS_ERR_INVALID_ARGUMENT  # > 2^38 px
    assert f(1, 4, 4, None, a, a, None, None, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(1, 4, 4, a, a, a, None, None, a, None, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(1, 4, 4, a, a, a, a, None, a, a, None) == B.GS_ERR_INVALID_ARGUMENT  # mesh colour without depth
    assert "both" in _err(lib)
    assert f(1, 4, 4, a, a, a, None, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT
    assert f(1, 4, 4, a, a, bad, None, None, a, a, None) == B.GS_ERR_INVALID_ARGUMENT  # misaligned
    assert f(1, 4, 4, a, a, a, bad, a, a, a, None) == B.GS_ERR_INVALID_ARGUMENT


def test_tile_order_sizes(lib):
    # 8 queues of ceil(n_views * T / 8) words; the compositing workspace holds
    # 2048 bytes of counters and room for one order
    from paper_2604_12626_amd import binding as B
    for (w, h, v, T) in ((64, 64, 1, 16), (640, 480, 1, 1200), (100, 70, 3, 35), (256, 256, 64, 256)):
        p = B.make_params(w, h)
        words = lib.gs_tile_order_words(v, ctypes.byref(p))
        assert words == 8 * ((v * T + 7) // 8)
        assert lib.gs_composite_workspace(v, ctypes.byref(p)) == 2048 + 4 * words
    p = B.make_params(64, 64)
    assert lib.gs_tile_order_words(0, ctypes.byref(p)) == 0
    assert lib.gs_tile_order_words(1, None) == 0
    # segment checkpoints: one slot per GS_SEGMENT key slots (+1), 4 quadrants x 5 values x 64
    # pixels, and GS_SEGMENT + 2 words of the backward's work list per slot, plus its count
    for cap in (1, 63, 64, 1 << 20):
        assert lib.gs_checkpoint_floats(cap) == (cap // 64 + 1) * (4 * 5 * 64 + 66) + 1
    assert lib.gs_checkpoint_floats(0) == 0


def test_tuning_validation():
    from paper_2604_12626_amd import binding as B
    prev = B.get_tuning()
    try:
        for bad in ({"composite_groups_per_cu": 0}, {"composite_groups_per_cu": 33},
                    {"sort_partition_keys": 2048}, {"sort_lookback": 8}, {"sort_algorithm": 2},
                    {"composite_pairs": 3}, {"composite_pairs": -1}):
            before = B.get_tuning()
            with pytest.raises(B.GSError):
                B.set_tuning(**bad)
            assert B.get_tuning() == before
        B.set_tuning(5, sort_partition_keys=8192, sort_lookback=64, sort_algorithm=1, composite_pairs=2)
        assert B.get_tuning() == {"composite_groups_per_cu": 5, "sort_partition_keys": 8192, "sort_lookback": 64,
                                  "sort_algorithm": 1, "composite_pairs": 2}
        B.set_tuning()
        assert B.get_tuning() == {"composite_groups_per_cu": 3, "sort_partition_keys": 4096, "sort_lookback": 16,
                                  "sort_algorithm": 0, "composite_pairs": 0}
    finally:
        B.set_tuning(**prev)


def test_renderer_checkpoint_modes():
    # True / False / "auto" only; "auto" records checkpoints up to the item limit
    from paper_2604_12626_amd import render
    import pytest as _pt
    with _pt.raises(ValueError):
        render.Renderer(64, 64, device="cpu", checkpoints="sometimes")
    r = render.Renderer(64, 64, device="cpu", checkpoints="auto")
    assert r.checkpoints == "auto" and r.T * 1 <= render.Renderer.AUTO_CHECKPOINT_ITEMS


def test_bench_refuses_more_than_one_gpu():
    # the benchmark measures one GPU; --gpus N > 1 exits with a message before touching a device
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_composite_noalloc_rejects_launches_beyond_its_scratch(lib):
    """gs_composite_noalloc holds its queue counters and work order in a
    library-owned per-GPU array sized for GS_NOALLOC_MAX_ITEMS (view, tile)
    items: a larger launch is refused before anything touches a device."""
    import ctypes as C
    from paper_2604_12626_amd import binding as B
    hdr = open(os.path.join(ROOT, "include", "gs.h")).read()
    max_items = int(re.search(r"#define GS_NOALLOC_MAX_ITEMS (\d+)", hdr).group(1))
    assert max_items == 65536
    p = B.make_params(256, 256)  # 256 tiles per view
    proj = B.Projected(0, None, None)
    dummy = C.c_void_p(256)  # never dereferenced: validation fails first
    n_views = max_items // 256 + 1
    st = lib.gs_composite_noalloc(C.byref(proj), dummy, dummy, None, n_views, C.byref(p), dummy, dummy, dummy,
                                  None, None, None, 0, None)
    assert st == 2 and "scratch" in _err(lib)  # GS_ERR_UNSUPPORTED
    st = lib.gs_composite_noalloc(C.byref(proj), None, dummy, None, 1, C.byref(p), dummy, dummy, dummy,
                                  None, None, None, 0, None)
    assert st == 1  # GS_ERR_INVALID_ARGUMENT: NULL list values
