"""The entry point that allocates nothing, sfm_guided_match_noalloc, against
sfm_guided_match through the C ABI: identical outputs on calls in a row (each
smaller than the one before, so anything a call left in the shared scratch
array would show), no device memory taken by its calls, and its limits."""
import numpy as np
import pytest

import scenes
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

SFM_ECAPACITY = -4


@pytest.fixture(scope="module")
def sfm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1512_06235_amd as sfm
    sfm.lib()   # raises when the library is not built
    return sfm


@pytest.fixture(scope="module")
def arc():
    scene, pairs = scenes.make_arc_batch()
    images = [(scene.image(k).xy, scene.image(k).desc) for k in range(scene.n_images)]
    return scene, pairs, images


def _pick(scene, pairs, n, seed):
    rng = np.random.default_rng(seed)
    sel = sorted(rng.choice(len(pairs), size=n, replace=False))
    sub = [pairs[k] for k in sel]
    return sub, np.stack([scene.F(a, b) for a, b, _ in sub])


def _assert_same(ref, got, what):
    for k in ("offset", "n_comparisons", "n_borderline"):
        a, b = getattr(ref, k).cpu().numpy(), getattr(got, k).cpu().numpy()
        assert np.array_equal(a, b), f"{what}: {k} differs"
    n = int(ref.offset[-1])
    for k in ("query", "match", "d1", "d2"):
        a, b = getattr(ref, k)[:n].cpu().numpy(), getattr(got, k)[:n].cpu().numpy()
        assert np.array_equal(a, b), f"{what}: {k} differs"
    if ref.emit_all:
        for k in ("all_match", "all_d1", "all_d2", "all_count"):
            a, b = getattr(ref, k).cpu().numpy(), getattr(got, k).cpu().numpy()
            assert np.array_equal(a, b), f"{what}: {k} differs"
    return n


def test_noalloc_equals_batched_on_calls_in_a_row(sfm, arc):
    import torch
    scene, pairs, images = arc
    ref = sfm.Matcher().register(images)
    na = sfm.Matcher().register(images)
    calls = [(_pick(scene, pairs, 40, 11), True, 4), (_pick(scene, pairs, 12, 12), True, 4),
             (_pick(scene, pairs, 5, 13), False, 8)]
    sizes = [sfm.sfm_workspace_size(ref.ctx, p) for (p, _), _, _ in calls]
    say(f"  no-alloc calls: {[len(p) for (p, _), _, _ in calls]} pairs, scratch {sizes} bytes")
    assert sizes[0] > sizes[1] > sizes[2] and sizes[0] <= sfm.NOALLOC_SCRATCH_BYTES
    # Reference results and every output buffer first: the window below then
    # holds only the entry point's own calls.
    expect, bufs = [], []
    for (p, F), emit_all, gt in calls:
        sfm.sfm_set_tuning(ref.ctx, gt, 8)
        expect.append(ref.match(p, F, form="batched", emit_all=emit_all))
        bufs.append(na.buffers(p, emit_all))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    for k, ((p, F), emit_all, gt) in enumerate(calls):
        say(f"  no-alloc call {k}: {len(p)} pairs, emit_all={emit_all}, group_tiles={gt}")
        sfm.sfm_set_tuning(na.ctx, gt, 8)
        na.match(p, F, form="noalloc", emit_all=emit_all, out=bufs[k])
        n = _assert_same(expect[k], bufs[k], f"call {k}")
        say(f"  no-alloc call {k}: {n} matches identical")
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info(0)[0] == free0, "device memory changed during the calls"
    ref.close()
    na.close()


def test_noalloc_two_contexts_two_streams(sfm, arc):
    """Two contexts share the GPU's scratch; calls on different streams,
    issued back to back, are ordered on the device and both stay exact."""
    import torch
    scene, pairs, images = arc
    ref = sfm.Matcher().register(images)
    a = sfm.Matcher().register(images)
    b = sfm.Matcher().register(images)
    (pa, Fa), (pb, Fb) = _pick(scene, pairs, 20, 21), _pick(scene, pairs, 9, 22)
    ea, eb = ref.match(pa, Fa, emit_all=True), ref.match(pb, Fb, emit_all=True)
    oa, ob = a.buffers(pa, True), b.buffers(pb, True)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    say("  no-alloc: two contexts on two streams")
    for _ in range(2):
        a.match(pa, Fa, form="noalloc", emit_all=True, out=oa, stream=sa, sync=False)
        b.match(pb, Fb, form="noalloc", emit_all=True, out=ob, stream=sb, sync=False)
    sfm.sfm_sync(a.ctx, sa)
    sfm.sfm_sync(b.ctx, sb)
    _assert_same(ea, oa, "context a")
    _assert_same(eb, ob, "context b")
    for m in (ref, a, b):
        m.close()


def test_noalloc_limits_and_empty(sfm, arc):
    scene, pairs, images = arc
    m = sfm.Matcher().register(images)
    ref = sfm.Matcher().register(images)
    # Too many pairs: rejected before anything is enqueued.
    many = [(0, 1, 4.0)] * (sfm.NOALLOC_MAX_PAIRS + 1)
    F01 = np.stack([scene.F(0, 1)] * len(many))
    with pytest.raises(sfm.SfmError) as e:
        sfm.sfm_guided_match_noalloc(m.ctx, many, F01, m.buffers(many[:1]), sfm.options())
    assert e.value.status == SFM_ECAPACITY and "at most" in str(e.value)
    # More scratch than the array holds: rejected with the size it needs.
    big = max(pairs, key=lambda p: len(images[p[0]][0]) + len(images[p[1]][0]))
    per = sfm.sfm_workspace_size(m.ctx, [big])
    reps = sfm.NOALLOC_SCRATCH_BYTES // per + 2
    over = [big] * reps
    assert sfm.sfm_workspace_size(m.ctx, over) > sfm.NOALLOC_SCRATCH_BYTES
    Fo = np.stack([scene.F(big[0], big[1])] * reps)
    say(f"  no-alloc: {reps} copies of the largest pair need "
        f"{sfm.sfm_workspace_size(m.ctx, over)} bytes")
    with pytest.raises(sfm.SfmError) as e:
        m.match(over, Fo, form="noalloc", out=m.buffers(over, False))
    assert e.value.status == SFM_ECAPACITY and "scratch" in str(e.value)
    # No pairs: offset[0] is written, nothing else.
    out = m.buffers([], False)
    out.offset.fill_(7)
    m.match([], np.zeros((0, 3, 3)), form="noalloc", out=out)
    assert int(out.offset.cpu()[0]) == 0
    # The context still matches exactly after the rejected calls.
    p, F = _pick(scene, pairs, 6, 31)
    _assert_same(ref.match(p, F, emit_all=True), m.match(p, F, form="noalloc", emit_all=True),
                 "after rejections")
    m.close()
    ref.close()
