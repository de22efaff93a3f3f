"""GPU parity of the hue image pipeline (include/ot_hue.h) against the
oracle: bin counts, target counts, shift, output bins and the rendered 8-bit
frames must match bit for bit (integer and byte work; every FP32 step on both
sides is the same single rounded operation)."""
import numpy as np
import pytest

from oracle import hue as ref
from synth import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def othue():
    import torch
    from paper_1501_04840_amd import othue as o
    assert torch.cuda.is_available()
    o.lib()
    return o


def _say(msg):
    print(msg, flush=True)


def _renderer(o, img, n):
    import torch
    N = img.shape[0] * img.shape[1]
    r = o.HueRenderer(N, n)
    r.set_source(torch.from_numpy(np.ascontiguousarray(img).reshape(-1)).cuda())
    return r


def _frame_check(r, src, target):
    import torch
    out, bins = r.render(torch.from_numpy(np.asarray(target, np.float32)).cuda(), with_bins=True)
    ct, s = r.plan_info()
    rgb_ref, k_ref, ct_ref, s_ref = src.render(np.asarray(target, np.float32))
    assert s == s_ref
    assert np.array_equal(ct, ct_ref)
    assert np.array_equal(bins.cpu().numpy(), k_ref)
    assert np.array_equal(out.cpu().numpy(), rgb_ref)


@pytest.mark.parametrize("H,W,n", [(96, 80, 64), (97, 83, 180), (64, 64, 360), (1, 1, 2),
                                   (33, 7, 4096)])
def test_source_histogram(othue, H, W, n):
    _say(f"hue histogram {H}x{W} n={n}")
    img = inputs.hue_image(H * 1000 + W, H, W)
    r = _renderer(othue, img, n)
    src = ref.Source(img, n)
    c, d = r.histogram()
    assert np.array_equal(c.cpu().numpy(), src.counts)
    assert np.array_equal(d.cpu().numpy(), src.density().astype(np.float32))
    r.close()


@pytest.mark.parametrize("H,W,n", [(96, 80, 64), (97, 83, 180), (64, 64, 360), (1, 1, 2),
                                   (33, 7, 4096)])
def test_frames_match_oracle(othue, H, W, n):
    _say(f"hue frames {H}x{W} n={n}")
    img = inputs.hue_image(7 + H + W, H, W)
    r = _renderer(othue, img, n)
    src = ref.Source(img, n)
    rng = np.random.default_rng(n)
    targets = [
        np.roll(src.density(), n // 3),                    # rotated own histogram
        inputs.von_mises_hist(55 + n, n),                  # a smooth periodic density
        src.counts.astype(np.float32),                     # own counts: identity
        np.zeros(n, np.float32),                           # no mass: identity
        rng.uniform(-0.2, 1.0, n),                         # negative entries count as 0
    ]
    t = rng.uniform(0, 1, n).astype(np.float32)
    t[:: 5] = np.nan
    t[1:: 7] = np.inf
    targets.append(t)
    for tg in targets:
        _frame_check(r, src, tg)
    r.close()


def test_identity_frame_is_the_source(othue):
    import torch
    _say("hue identity frame")
    img = inputs.hue_image(3, 120, 100)
    r = _renderer(othue, img, 180)
    c, d = r.histogram()
    out = r.render(d)
    assert np.array_equal(out.cpu().numpy(), img.reshape(-1, 3))
    assert r.plan_info()[1] == 0
    r.close()


def test_calls_before_a_source_are_refused(othue):
    import torch
    _say("hue state errors")
    r = othue.HueRenderer(64, 16)
    tg = torch.ones(16, device="cuda")
    out = torch.empty(64, 3, dtype=torch.uint8, device="cuda")
    for call in (lambda: othue.ot_hue_histogram(r.h, None, tg),
                 lambda: othue.ot_hue_plan(r.h, tg, 1),
                 lambda: othue.ot_hue_apply(r.h, out),
                 lambda: othue.ot_hue_plan_info(r.h, 0)):
        with pytest.raises(othue.OtDynError) as e:
            call()
        assert e.value.status == -7
    with pytest.raises(othue.OtDynError) as e:
        othue.ot_hue_render(r.h, tg, 0, out)
    assert e.value.status == -1
    r.close()


def test_plan_then_apply_equals_render(othue):
    """The frame split in its two calls: one plan serves several applies, and
    apply before a plan for the current source is refused."""
    import torch
    _say("hue plan/apply")
    n = 180
    img = inputs.hue_image(41, 70, 90)
    r = _renderer(othue, img, n)
    N = 70 * 90
    tg = torch.from_numpy(inputs.von_mises_hist(9, n)).cuda()
    ref_out = r.render(tg)
    othue.ot_hue_plan(r.h, tg)
    a = torch.empty(N, 3, dtype=torch.uint8, device="cuda")
    b = torch.empty(N, 3, dtype=torch.uint8, device="cuda")
    othue.ot_hue_apply(r.h, a)
    othue.ot_hue_apply(r.h, b)
    assert torch.equal(a, ref_out) and torch.equal(b, ref_out)
    r.set_source(torch.from_numpy(img.reshape(-1).copy()).cuda())
    with pytest.raises(othue.OtDynError) as e:
        othue.ot_hue_apply(r.h, a)
    assert e.value.status == -7
    r.close()


def test_unaligned_images_take_the_pixel_path(othue):
    """Source and frame at odd byte offsets and bins at a 4-byte offset: the
    pixel-by-pixel form of the frame kernel, same results."""
    import torch
    _say("hue unaligned")
    n, H, W = 180, 61, 47
    N = H * W
    img = inputs.hue_image(51, H, W)
    big = torch.zeros(3 * N + 16, dtype=torch.uint8, device="cuda")
    big[1:1 + 3 * N] = torch.from_numpy(img.reshape(-1).copy()).cuda()
    r = othue.HueRenderer(N, n)
    r.set_source(big[1:1 + 3 * N])
    assert r.src.data_ptr() % 4 == 1
    src = ref.Source(img, n)
    tg = inputs.von_mises_hist(13, n)
    rgb_ref, k_ref, _, _ = src.render(tg)
    ob = torch.zeros(3 * N + 16, dtype=torch.uint8, device="cuda")
    bb = torch.zeros(N + 8, dtype=torch.int32, device="cuda")
    othue.ot_hue_render(r.h, torch.from_numpy(tg).cuda(), 1, ob[3:3 + 3 * N], bb[1:1 + N])
    torch.cuda.synchronize()
    assert np.array_equal(ob[3:3 + 3 * N].cpu().numpy().reshape(-1, 3), rgb_ref)
    assert np.array_equal(bb[1:1 + N].cpu().numpy(), k_ref)
    assert int(ob[:3].sum()) == 0 and int(ob[3 + 3 * N:].sum()) == 0
    assert int(bb[0]) == 0 and int(bb[1 + N:].sum()) == 0
    r.close()


@pytest.mark.parametrize("H,W,n", [(40, 36, 128), (37, 29, 180)])
def test_frames_in_one_call(othue, H, W, n):
    """Several frames per call (one plan block per frame, frames along the
    grid's y): each frame as the oracle gives it, the plan arrays growing and
    shrinking between calls; with N not a multiple of 4 the frames take the
    pixel path."""
    import torch
    _say(f"hue frames per call {H}x{W} n={n}")
    img = inputs.hue_image(61 + n, H, W)
    N = H * W
    r = _renderer(othue, img, n)
    src = ref.Source(img, n)
    rng = np.random.default_rng(n)
    pool = [np.roll(src.density(), 5 * i) for i in range(3)] + \
           [inputs.von_mises_hist(70 + i, n) for i in range(3)] + \
           [src.counts.astype(np.float64), np.zeros(n), rng.uniform(-0.5, 1, n)]
    for F in (3, 7, 2):
        tg = np.stack([pool[(F + i) % len(pool)] for i in range(F)]).astype(np.float32)
        out, bins = r.render_frames(torch.from_numpy(tg).cuda(), with_bins=True)
        out, bins = out.cpu().numpy(), bins.cpu().numpy()
        for f in range(F):
            rgb_ref, k_ref, ct_ref, s_ref = src.render(tg[f])
            ct, s = r.plan_info(f)
            assert s == s_ref and np.array_equal(ct, ct_ref)
            assert np.array_equal(bins[f], k_ref)
            assert np.array_equal(out[f], rgb_ref)
    with pytest.raises(othue.OtDynError):
        othue.ot_hue_plan_info(r.h, 2)                 # the last plan had 2 frames
    r.close()


def test_new_source_on_one_renderer(othue):
    import torch
    _say("hue two sources")
    n = 128
    a = inputs.hue_image(11, 50, 60)
    b = inputs.hue_image(12, 50, 60)
    r = _renderer(othue, a, n)
    _frame_check(r, ref.Source(a, n), inputs.von_mises_hist(5, n))
    r.set_source(torch.from_numpy(b.reshape(-1).copy()).cuda())
    _frame_check(r, ref.Source(b, n), inputs.von_mises_hist(6, n))
    r.close()


def test_pipeline_frames_along_the_geodesic(othue):
    """Sec. 5 end to end: the two images' hue densities, the periodic 1D
    transport between them, and the frames for time levels of f."""
    import torch
    from paper_1501_04840_amd import otdyn
    _say("hue pipeline")
    n, P = 180, 16
    a = inputs.hue_image(21, 128, 96)
    b = inputs.hue_image(22, 128, 96)
    ra = _renderer(othue, a, n)
    rb = _renderer(othue, b, n)
    _, da = ra.histogram()
    _, db = rb.histogram()
    f0 = (da + 0.05) / (da + 0.05).mean()              # positive densities of mean one
    f1 = (db + 0.05) / (db + 0.05).mean()
    d = otdyn.ot_dyn_default_desc(n, 1, 1, P)
    d.bc[0] = otdyn.OT_BC_PERIODIC
    prob = otdyn.Problem(d, "cuda:0")
    prob.set_boundary(f0.reshape(1, 1, n), f1.reshape(1, 1, n))
    prob.init(otdyn.OT_INIT_COLD)
    prob.step(400)
    torch.cuda.synchronize()
    src = ref.Source(a, n)
    for t in (0, P // 4, P // 2, P):
        row = prob.F[0, t, 0, 0].contiguous()
        _frame_check(ra, src, row.cpu().numpy())
    prob.close()
    ra.close()
    rb.close()


def test_one_megapixel_frame(othue):
    _say("hue 1024x1024 n=360")
    img = inputs.hue_image(31, 1024, 1024, sigma=24.0)
    n = 360
    r = _renderer(othue, img, n)
    src = ref.Source(img, n)
    _frame_check(r, src, inputs.von_mises_hist(77, n))
    r.close()


def test_rgb_hsv_conversions_match_oracle(othue):
    """RGB -> HSV bit for bit on every 8-bit colour; HSV -> RGB bit for bit on
    random, edge and out-of-range values; the round trip exact."""
    import torch
    _say("hue rgb<->hsv")
    v = torch.arange(256, dtype=torch.int32)
    r, g, b = torch.meshgrid(v, v, v, indexing="ij")
    px = torch.stack([r.reshape(-1), g.reshape(-1), b.reshape(-1)], dim=1).to(torch.uint8)
    N = px.shape[0]
    dpx = px.cuda()
    hsv = torch.empty(N, 3, dtype=torch.float32, device="cuda")
    othue.ot_hue_rgb_to_hsv(dpx, N, hsv)
    back = torch.empty(N, 3, dtype=torch.uint8, device="cuda")
    othue.ot_hue_hsv_to_rgb(hsv, N, back)
    torch.cuda.synchronize()
    ref_hsv = ref.hsv_of_rgb(px.numpy())
    assert np.array_equal(hsv.cpu().numpy(), ref_hsv)
    assert torch.equal(back.cpu(), px)
    rng = np.random.default_rng(12)
    x = rng.uniform(-0.5, 1.5, (100003, 3)).astype(np.float32)
    x[::97, 0] = np.nan
    x[1::89, 1] = np.inf
    x[2::83, 2] = -np.inf
    dx = torch.from_numpy(x).cuda()
    out = torch.empty(x.shape[0], 3, dtype=torch.uint8, device="cuda")
    othue.ot_hue_hsv_to_rgb(dx, x.shape[0], out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref.rgb_of_hsv(x))


def test_bench_configuration_frames(othue):
    """The configuration bench.py times: the 3840 x 2160 image, 360 bins, 33
    frames in one launch; frames 0, 16 and 32 compared in full with the
    oracle, and every frame's output bins with its target counts."""
    import torch
    _say("hue 3840x2160, 33 frames per call")
    H, W, n, F = 2160, 3840, 360, 33
    img = inputs.hue_image(501, H, W, sigma=24.0)
    dens = np.stack([inputs.von_mises_hist(600 + i, n) for i in range(F)]).astype(np.float32)
    r = _renderer(othue, img, n)
    out, bins = r.render_frames(torch.from_numpy(dens).cuda(), with_bins=True)
    torch.cuda.synchronize()
    counts = torch.stack([torch.bincount(bins[f].long(), minlength=n) for f in range(F)]).cpu()
    src = ref.Source(img, n)
    for f in range(F):
        ct, _ = r.plan_info(f)
        assert np.array_equal(counts[f].numpy(), ct)
        assert np.array_equal(ct, ref.target_counts(dens[f], H * W, src.counts))
    for f in (0, F // 2, F - 1):
        rgb_ref, k_ref, _, s_ref = src.render(dens[f])
        assert r.plan_info(f)[1] == s_ref
        assert np.array_equal(bins[f].cpu().numpy(), k_ref)
        assert np.array_equal(out[f].cpu().numpy(), rgb_ref)
    r.close()


def test_random_pixel_image_order(othue):
    """Uniformly random pixels: many distinct, close hues, so the output bins
    depend on the exact strict order of the source's hues."""
    import torch
    _say("hue random pixels")
    rng = np.random.default_rng(77)
    img = rng.integers(0, 256, size=(300, 301, 3), dtype=np.uint8)
    for n in (7, 360, 4096):
        r = _renderer(othue, img, n)
        src = ref.Source(img, n)
        _frame_check(r, src, inputs.von_mises_hist(90 + n, n))
        _frame_check(r, src, np.roll(src.density(), n // 5))
        r.close()


def test_frames_beyond_the_workspace_capacity(othue):
    """The renderer's workspace plans for max_frames frames per call: a plan
    for more is refused (OT_ERR_SHAPE) before any launch, and the binding's
    renderer makes room for them (a new renderer over a larger workspace,
    the source prepared again), with frames equal to those of a renderer
    that had the room from the start."""
    import torch
    from paper_1501_04840_amd import otdyn
    _say("hue frames beyond the workspace capacity")
    H, W, n, F = 37, 53, 90, 5
    img = inputs.hue_image(77, H, W)
    src = torch.from_numpy(img.reshape(-1).copy()).cuda()
    tg = torch.from_numpy(np.stack([inputs.von_mises_hist(800 + i, n) for i in range(F)])
                          .astype(np.float32)).cuda()
    small = othue.HueRenderer(H * W, n, max_frames=2)
    small.set_source(src)
    with pytest.raises(otdyn.OtDynError) as e:
        othue.ot_hue_plan(small.h, tg, F)
    assert e.value.status == otdyn.OT_ERR_SHAPE
    a = small.render_frames(tg)
    assert small.max_frames == F
    big = othue.HueRenderer(H * W, n, max_frames=F)
    big.set_source(src)
    b = big.render_frames(tg)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    small.close()
    big.close()
