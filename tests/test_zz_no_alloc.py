"""mr_render_noalloc, the render for callers that cannot allocate, through the
C ABI: its outputs equal mr_render's on the same inputs, call after call on
the library's one array per device, the second call smaller than the first
(what the first left in the array must not leak into the second)."""
import numpy as np
import pytest

from paper_2309_04581_amd import scenegen as sg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from test_gpu_parity import dev, host, mr, oracle_camera_rays  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(M, sc, F, G, o, d, opts):
    """The same render through mr_render and mr_render_noalloc (outputs of
    the second pre-filled with a sentinel)."""
    R = M.Renderer(len(o), sc.max_bounces)
    R.render(F, G, dev(o), dev(d), sc.lights, opts)
    torch.cuda.synchronize()
    assert R.status() == 0
    ref = {k: host(getattr(R, k)) for k in ("radiance", "throughput", "bounces", "hit_ids", "counters")}
    N = M.Renderer(len(o), sc.max_bounces)
    for t in (N.radiance, N.throughput):
        t.fill_(-7.0)
    for t in (N.bounces, N.hit_ids, N.counters):
        t.fill_(-7)
    gave_up = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    N.render_noalloc(F, G, dev(o), dev(d), sc.lights, opts, gave_up=gave_up)
    torch.cuda.synchronize()
    got = {k: host(getattr(N, k)) for k in ref}
    assert int(gave_up.item()) == 0
    return ref, got


def _equal(ref, got, what):
    for k in ("hit_ids", "bounces", "counters"):
        np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{what}: {k}")
    for k in ("radiance", "throughput"):
        # the two calls run the same kernels on the same inputs: identical bits
        np.testing.assert_array_equal(got[k].view(np.uint32), ref[k].view(np.uint32), err_msg=f"{what}: {k}")


def test_noalloc_render_equals_render_on_two_calls_in_a_row():
    """First the mid scene (glass sphere, mirror cube, lit floor, 16-level
    field, 8 bounces) at 512x512, the largest size the array holds; then the
    64x64 tiny scene (8-level field, mirror cube), a smaller call."""
    M = mr()
    mid = sg.mid_scene(width=512, height=512)
    o, d = oracle_camera_rays(mid)
    assert len(o) == M.MR_NOALLOC_MAX_RAYS
    F, G = M.Field(mid.field), M.Mesh(mid.mesh)
    F.build_occupancy(mid.occupancy_res, mid.occupancy_thresh)
    ref, got = _both(M, mid, F, G, o, d, M.make_opts(mid, use_occupancy=True))
    _equal(ref, got, "mid 512x512")
    assert ref["bounces"].max() >= 3 and (ref["hit_ids"][:, 0] >= 0).sum() > 10000

    tiny = sg.tiny_scene()
    o, d = oracle_camera_rays(tiny)
    assert len(o) < M.MR_NOALLOC_MAX_RAYS
    F, G = M.Field(tiny.field), M.Mesh(tiny.mesh)
    ref, got = _both(M, tiny, F, G, o, d, M.make_opts(tiny))
    _equal(ref, got, "tiny 64x64")
    assert (ref["hit_ids"][:, 0] >= 0).sum() > 100


def test_noalloc_render_refuses_before_launch():
    """Too many rays, or a layout refusal, leaves the outputs untouched."""
    M = mr()
    sc = sg.tiny_scene(width=16, height=16)
    F, G = M.Field(sc.field), M.Mesh(sc.mesh)
    o, d = oracle_camera_rays(sc)
    N = M.Renderer(len(o), sc.max_bounces)
    N.radiance.fill_(-7.0)
    torch.cuda.synchronize()
    with pytest.raises(M.MrError) as e:
        N.render_noalloc(F, G, dev(o), dev(d), sc.lights, M.make_opts(sc, use_occupancy=True))
    assert e.value.status == M.MR_ERR_STATE
    torch.cuda.synchronize()
    assert bool((N.radiance == -7.0).all())
