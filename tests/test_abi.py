"""The C-ABI library loads and exports every entry point its header declares;
host-side validation rejects bad calls before touching the device.  CPU only:
no kernel is launched."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2309_04581_amd import meshrf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "meshrf.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mr_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_documented_entry_points():
    names = declared()
    for must in ("mr_field_create", "mr_mesh_build_bvh", "mr_mesh_refit", "mr_render"):
        assert must in names
    assert sorted(meshrf.EXPORTED) == names


def test_library_exports_every_declared_symbol():
    L = meshrf.lib()
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    assert "gfx950" in meshrf.mr_version()


def test_render_validation_before_any_launch():
    opts = meshrf.RenderOpts()
    opts.t_near, opts.t_far, opts.n_samples = 0.05, 4.0, 64
    out = meshrf.RenderOut()
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_render(None, None, -1, None, None, 4, None, [], opts, out, None, 0, stream=_Null())
    assert e.value.status == meshrf.MR_ERR_INVALID_ARG and "n < 0" in str(e.value)
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_render(None, None, 4, None, None, 4, None, [], opts, out, None, 0, stream=_Null())
    assert e.value.status == meshrf.MR_ERR_INVALID_ARG
    bad = meshrf.RenderOpts()
    bad.t_near, bad.t_far, bad.n_samples = 1.0, 0.5, 64
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_render(None, None, 0, None, None, 4, None, [], bad, out, None, 0, stream=_Null())
    assert "t_near" in str(e.value)
    with pytest.raises(meshrf.MrError):
        meshrf.mr_render(None, None, 0, None, None, 99, None, [], opts, out, None, 0, stream=_Null())
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_render(None, None, 0, None, None, 4, None, [[0, 0, 0, -1, 0, 0]], opts, out, None, 0,
                         stream=_Null())
    assert "intensity" in str(e.value)
    assert meshrf.mr_render_workspace_size(1000) >= 2 * 16 * 4 * 1000


def test_mesh_and_field_validation_before_any_upload():
    v = np.zeros((3, 3), np.float32)
    f = np.array([[0, 1, 5]], np.int32)
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_mesh_build_bvh(v, f, [0], [[meshrf.MR_MIRROR, 1, 1, 1, 1]], stream=_Null())
    assert "index out of range" in str(e.value)
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_mesh_build_bvh(v, np.array([[0, 1, 2]], np.int32), [0],
                                 [[meshrf.MR_GLASS, 0.9, 1, 1, 1]], stream=_Null())
    assert "ior" in str(e.value)
    from paper_2309_04581_amd import scenegen as sg
    fld = sg.tiny_field()
    d = meshrf.FieldDesc()
    res = np.array(fld.resolutions, np.int32)
    d.n_levels, d.feats_per_level, d.log2_table_size = 8, 2, 14
    d.host_resolutions = res.ctypes.data
    d.density_in, d.density_hidden, d.density_out = 32, 64, 16
    d.color_in, d.color_hidden, d.color_hidden_layers, d.sh_components = 32, 48, 1, 4
    d.aabb_min = (C.c_float * 3)(-1, -1, -1)
    d.aabb_max = (C.c_float * 3)(1, 1, 1)
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_field_create(d, fld.table, fld.mlp, stream=_Null())
    assert e.value.status == meshrf.MR_ERR_UNSUPPORTED
    d.color_hidden = 64
    bad_mlp = fld.mlp.copy()
    bad_mlp[5] = np.nan
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_field_create(d, fld.table, bad_mlp, stream=_Null())
    assert "non-finite" in str(e.value)


def test_noalloc_render_refuses_more_rays_than_its_array_holds():
    """mr_render_noalloc checks n against its fixed array before anything else
    (no device call, so no GPU is needed to see it); n = 0 returns at once."""
    opts = meshrf.RenderOpts()
    opts.t_near, opts.t_far, opts.n_samples = 0.05, 4.0, 64
    out = meshrf.RenderOut()
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_render_noalloc(None, None, meshrf.MR_NOALLOC_MAX_RAYS + 1, None, None, 4, None, [], opts, out,
                                 stream=_Null())
    assert e.value.status == meshrf.MR_ERR_INVALID_ARG and "262144" in str(e.value)
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_render_noalloc(None, None, 4, None, None, 4, None, [], opts, out, stream=_Null())
    assert e.value.status == meshrf.MR_ERR_INVALID_ARG and "null rays" in str(e.value)
    meshrf.mr_render_noalloc(None, None, 0, None, None, 4, None, [], opts, out, stream=_Null())
    hdr = open(HEADER).read()
    assert f"#define MR_NOALLOC_MAX_RAYS {meshrf.MR_NOALLOC_MAX_RAYS}" in hdr


def test_autotune_candidates_are_valid_launch_shapes():
    """The autotuner's candidates (generated from the device's compute units,
    256 without a GPU, and the queue length) are shapes mr_render accepts, and
    the stage tiles follow the queue length."""
    small = meshrf.mr_autotune_candidates(4096)
    big = meshrf.mr_autotune_candidates(12_000_000)
    for c in (small, big):
        assert len(c) == 6 and all(1 <= len(v) <= 6 for v in c)
        assert all(0 <= v <= 64 for v in c[0] + c[1])
        assert all(v % 128 == 0 and 128 <= v <= 4096 for v in c[2])
        assert all(v >= 0 for v in c[3]) and all(1 <= v <= 64 for v in c[4]) and all(v >= -1 for v in c[5])
    assert small[2] == [128] and max(big[2]) > 128
    with pytest.raises(meshrf.MrError):
        meshrf.mr_autotune_candidates(-1)


def test_autotune_search_validates_before_any_launch():
    """The launch-shape search refuses bad repetition and sweep counts and a
    bad render before it renders anything (no GPU is needed to see it)."""
    opts = meshrf.RenderOpts()
    opts.t_near, opts.t_far, opts.n_samples = 0.05, 4.0, 64
    out = meshrf.RenderOut()
    for reps, passes, what in ((0, 1, "reps"), (1, 0, "passes"), (101, 1, "reps")):
        with pytest.raises(meshrf.MrError) as e:
            meshrf.mr_autotune_search(None, None, 4, None, None, 4, None, [], opts, out, None, 0, reps=reps,
                                      passes=passes, stream=_Null())
        assert e.value.status == meshrf.MR_ERR_INVALID_ARG and what in str(e.value)
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_autotune_search(None, None, 4, None, None, 4, None, [], opts, out, None, 0, stream=_Null())
    assert "null rays" in str(e.value)


@pytest.mark.parametrize("levels,sh,layers", [(8, 4, 2), (8, 16, 1), (16, 4, 2), (16, 16, 1)])
def test_field_layouts_without_kernels_are_refused_before_upload(levels, sh, layers):
    """Only layouts with march kernels are accepted: the others are refused
    by mr_field_create before any device allocation (no GPU is needed to see
    the refusal)."""
    from paper_2309_04581_amd import scenegen as sg
    fld = sg.tiny_field() if levels == 8 else sg.mid_field()
    d = meshrf.FieldDesc()
    res = np.array(fld.resolutions, np.int32)
    d.n_levels, d.feats_per_level, d.log2_table_size = levels, 2, int(fld.log2_table)
    d.host_resolutions = res.ctypes.data
    d.density_in, d.density_hidden, d.density_out = 32, 64, 16
    d.color_in, d.color_hidden, d.color_hidden_layers, d.sh_components = 32, 64, layers, sh
    d.aabb_min = (C.c_float * 3)(-1, -1, -1)
    d.aabb_max = (C.c_float * 3)(1, 1, 1)
    n_mlp = 64 * 32 + 16 * 64 + 64 * 32 + (layers - 1) * 64 * 64 + 3 * 64
    mlp = np.zeros(n_mlp, np.float32)
    with pytest.raises(meshrf.MrError) as e:
        meshrf.mr_field_create(d, fld.table, mlp, stream=_Null())
    assert e.value.status == meshrf.MR_ERR_UNSUPPORTED and "layouts" in str(e.value)


class _Null:
    cuda_stream = 0
