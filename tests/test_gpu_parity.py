"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs.  Images within 1e-5 (normwise, per view, pixels touched by a
float-ambiguous alpha = 1/255 pair excluded and counted), gradients within 1e-4
(normwise per parameter group), sigma within 1e-4, integer outputs bit-exact."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2605_13855_amd import scenes
from tests.gpu_common import (IMAGE_RTOL, NEAR_MARGIN, compare_grads, compare_image, image_views, oracle_grads,
                              sigma_ok, to_np)

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2605_13855_amd import oit
    from paper_2605_13855_amd.render import (ActiveSetTrainer, Renderer, new_grads, params_to_device, render)

DEV = "cuda"


def log(msg):
    print(msg, flush=True)


def mask_near(g_views, nears):
    """Zero dL/dC at the pixels that a float-ambiguous pair (alpha within NEAR_MARGIN of
    1/255) touches: there float32 and FP64 may take different contribution decisions,
    and the flipped pair's own term (about alpha dL/dalpha / 255) would show in the
    per-row gradient check of its splat.  Both sides get the masked dL/dC."""
    for g, near in zip(g_views, nears):
        g[:, near] = 0.0


def dense_case(sc, tile=16, batch=64, near_margin=NEAR_MARGIN, check_grads=True, windows=None, seed=0,
               sigma_atol=0.0, bwd_mode=0):
    """Render sc densely on the GPU and in the oracle; compare image, state and grads."""
    params = params_to_device(sc.params)
    sigma = torch.tensor([sc.sigma], device=DEV)
    r = Renderer(sc.cameras, sc.n, tile=tile, batch=batch)
    if bwd_mode:
        r.set_tuning(bwd_mode=bwd_mode)
    r.fit_pair_capacity(params, sigma, sc.background)
    r.forward(params, sigma, sc.background)
    torch.cuda.synchronize()
    assert r.status() == 0
    imgs = image_views(r, r.image, 3)
    states = image_views(r, r.pixstate, oit.PIXSTATE_PLANES)
    worst = 0.0
    masked = 0
    nears = []
    for k, cam in enumerate(sc.cameras):
        ref = O.render(sc.params, sc.sigma, sc.background, cam, near_margin=near_margin)
        nears.append(ref["near"])
        err = compare_image(imgs[k], ref["image"], ref["near"])
        masked += int(ref["near"].sum())
        worst = max(worst, err)
        log(f"  view {k} {cam.width}x{cam.height}: image err {err:.2e}, near-masked px {int(ref['near'].sum())}, "
            f"pairs {ref['pairs']}")
        assert err <= IMAGE_RTOL, (k, err)
        # per-pixel totals T and Q on unmasked pixels
        ok = ~ref["near"]
        np.testing.assert_allclose(states[k][0][ok], ref["state"][0][ok], rtol=1e-4, atol=1e-6)
    if not check_grads:
        return r
    rng = np.random.default_rng(seed)
    g_views = [rng.normal(size=(3, c.height, c.width)) for c in sc.cameras]
    mask_near(g_views, nears)
    if windows:
        for k, w in enumerate(windows):
            m = np.zeros_like(g_views[k])
            x0, y0, x1, y1 = w
            m[:, y0:y1, x0:x1] = 1.0
            g_views[k] *= m
    gimg = r.pack([g.astype(np.float32) for g in g_views])
    g_gpu = new_grads(sc.n, DEV)
    gsig = torch.zeros(1, dtype=torch.float64, device=DEV)
    r.backward(params, sigma, sc.background, gimg, g_gpu, gsig)
    torch.cuda.synchronize()
    # the oracle gets exactly the float32 gradient image the GPU got
    g_ref, s_ref, s_abs = oracle_grads(sc.params, sc.sigma, sc.background, sc.cameras,
                                       [g.astype(np.float32).astype(np.float64) for g in g_views], windows,
                                       with_abs=True)
    compare_grads({g: to_np(g_gpu[g]) for g, _ in O.GROUPS}, g_ref, log)
    ok, srel = sigma_ok(float(gsig.item()), s_ref, s_abs)
    log(f"  grad sigma: gpu {float(gsig.item()):.6e} oracle {s_ref:.6e} (sum |terms| {s_abs:.3e}) rel {srel:.2e}")
    assert ok or abs(float(gsig.item()) - s_ref) <= sigma_atol
    return r


def backward_walk_counts(sc, tile=16):
    params = params_to_device(sc.params)
    sigma = torch.tensor([sc.sigma], device=DEV)
    r = Renderer(sc.cameras, sc.n, tile=tile, batch=64)
    r.fit_pair_capacity(params, sigma, sc.background)
    r.forward(params, sigma, sc.background)
    gimg = torch.ones(3 * r.total_px, device=DEV)
    r.backward(params, sigma, sc.background, gimg, new_grads(sc.n, DEV),
               torch.zeros(1, dtype=torch.float64, device=DEV))
    torch.cuda.synchronize()
    c = r.counters()
    return c[3], c[4], c[5]


def test_backward_walks_three_ways():
    """The backward walks the smallest footprints box by box; of the other work items,
    those whose splats nearly all reach all the item's pixel groups are walked group by
    group by the whole wave, and the rest by (entry, group) pairs dealt to the lanes.  The
    config-1 scenes of the parity cases (sub-pixel, default and large splats) take all
    three walks between them, the sub-pixel one mostly the box walk."""
    counts = {}
    for name, mu in (("sub-pixel", -6.0), ("default", -3.5), ("large", -2.5)):
        items, boxed, waved = backward_walk_counts(scenes.make_scene(1, log_scale_mu=mu))
        log(f"  config 1, {name} splats: {items} backward work items, {boxed} walked box by box, "
            f"{waved} group by group by the whole wave, {items - boxed - waved} by dealt pairs")
        assert 0 <= boxed and 0 <= waved and boxed + waved <= items
        counts[name] = (items, boxed, waved)
    items, boxed, _ = counts["sub-pixel"]
    assert boxed > items // 2
    assert any(w > 0 for _, _, w in counts.values())
    assert any(i - b - w > 0 for i, b, w in counts.values())


def test_large_splat_parity():
    """Splats large against the tile (log-scale ~ N(-2.5, 0.3)): most backward work items
    have nearly every splat reach every pixel group, the case walked group by group by the
    whole wave."""
    for tile in (16, 32):
        log(f"large splats, tile {tile}")
        dense_case(scenes.make_scene(1, log_scale_mu=-2.5), tile=tile, batch=64)


def test_subpixel_scene_parity():
    """Sub-pixel splats (log-scale ~ N(-6, 0.3)): images and gradients against the
    oracle, with the backward walking footprint boxes."""
    for tile in (8, 16, 32):
        log(f"sub-pixel scene, tile {tile}")
        dense_case(scenes.make_scene(1, log_scale_mu=-6.0), tile=tile, batch=64)


@pytest.mark.parametrize("tile,batch", [(16, 64), (8, 32), (32, 256), (16, 128)])
def test_tiny_dense_parity(tile, batch):
    log(f"tiny dense parity tile={tile} batch={batch}")
    sc = scenes.make_scene(1)
    dense_case(sc, tile, batch)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_per_pixel_backward_matches_oracle(tile):
    """The per-pixel backward (atomics per pair, the 3DGS baseline of the paper's
    ablation) gives the same gradients as the oracle."""
    log(f"per-pixel backward, tile={tile}")
    sc = scenes.random_scene(25, 2500, 72, 56, n_views=2, mean_range=1.0)
    dense_case(sc, tile, 64, bwd_mode=1)


def test_ragged_image_and_tiles():
    log("ragged 100x75 image, 3000 splats")
    sc = scenes.random_scene(21, 3000, 100, 75, mean_range=1.0)
    dense_case(sc, 16, 64)
    dense_case(sc, 32, 64)


def test_multiview_uneven_batch():
    log("multi-view batch of uneven sizes in one launch")
    sc = scenes.random_scene(22, 1500, 64, 48, n_views=1, mean_range=1.0)
    cams = [scenes.orbit_camera(3.5, 0.3 * k, 0.1 * k - 0.2, 48 + 24 * k, 40 + 10 * k) for k in range(4)]
    rng = np.random.default_rng(5)
    sc.cameras = cams
    sc.targets = [rng.uniform(size=(3, c.height, c.width)).astype(np.float32) for c in cams]
    dense_case(sc, 16, 64)


def test_edge_cases():
    log("edge cases: one splat; everything behind the camera")
    sc = scenes.random_scene(23, 1, 32, 32, mean_range=0.0, log_scale_mu=-2.0)
    # a lone splat has F = c on every pixel, so dL/dw and dL/dsigma vanish exactly; float32
    # round-off of (c - F) leaves ~1e-10, far below any real sigma gradient (~1e-2 here)
    dense_case(sc, 8, 32, sigma_atol=1e-8)
    sc2 = scenes.random_scene(24, 50, 40, 30, mean_range=0.5)
    sc2.params["mean"][2, :] -= 10.0     # all behind the camera
    params = params_to_device(sc2.params)
    sigma = torch.tensor([sc2.sigma], device=DEV)
    r = Renderer(sc2.cameras, sc2.n, tile=16)
    r.forward(params, sigma, (0.25, 0.5, 0.75))
    img = image_views(r, r.image, 3)[0]
    np.testing.assert_allclose(img[0], 0.25, atol=0)
    np.testing.assert_allclose(img[2], 0.75, atol=0)


def test_dense_config2_full_frame_and_crop_grads():
    log("config 2: 100k splats, 800x800; full-frame image, 64x64 centre-crop gradients")
    sc = scenes.make_scene(2)
    dense_case(sc, 16, 64, windows=[(368, 368, 432, 432)])


def test_l1_loss_matches_oracle():
    sc = scenes.make_scene(1)
    params = params_to_device(sc.params)
    sigma = torch.tensor([sc.sigma], device=DEV)
    r = Renderer(sc.cameras, sc.n)
    r.forward(params, sigma, sc.background)
    tgt = r.pack(sc.targets)
    gi = torch.zeros_like(r.image)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    oit.l1_loss(r.image, tgt, r.cams_arr, r.n_views, gi, loss, r.ws)
    torch.cuda.synchronize()
    L, g = O.l1_loss(to_np(r.image).reshape(3, 128, 128), sc.targets[0])
    # |C - I| is formed in float32 on the GPU and accumulated in float64
    assert float(loss.item()) == pytest.approx(L, rel=1e-7)
    np.testing.assert_array_equal(to_np(gi).reshape(3, 128, 128), g.astype(np.float32).astype(np.float64))


def test_l1_loss_writes_only_its_workspace_head():
    """The L1 loss given a workspace of exactly oit_l1_loss_workspace_bytes() inside a
    larger sentinel-filled buffer leaves every byte past that size untouched."""
    sc = scenes.make_scene(2)
    cams = oit.camera_array(sc.cameras)
    need = oit.l1_loss_workspace_bytes()
    buf = torch.full((need + 256 + 65536,), 0xA5, dtype=torch.uint8, device=DEV)
    off = (-buf.data_ptr()) % 256
    ws = buf[off:off + need]
    rng = np.random.default_rng(2)
    img = torch.tensor(rng.random(3 * 800 * 800).astype(np.float32), device=DEV)
    tgt = torch.tensor(rng.random(3 * 800 * 800).astype(np.float32), device=DEV)
    gi = torch.zeros_like(img)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    oit.l1_loss(img, tgt, cams, 1, gi, loss, ws)
    torch.cuda.synchronize()
    tail = buf[off + need:]
    assert bool((tail == 0xA5).all())
    L, _ = O.l1_loss(to_np(img).reshape(3, 800, 800), to_np(tgt).reshape(3, 800, 800))
    assert float(loss.item()) == pytest.approx(L, rel=1e-7)


def test_l1_loss_on_the_render_workspace_keeps_the_backward_exact():
    """forward, L1 loss on the renderer's own workspace, backward: the gradients equal
    the oracle's for the same loss gradient (the loss must not disturb the tile lists
    and records the backward reads), dense at tile 16 and 5% active at tile 32."""
    sc = scenes.random_scene(27, 6000, 160, 120, n_views=2, mean_range=1.0)
    params = params_to_device(sc.params)
    sigma = torch.tensor([sc.sigma], device=DEV)
    for tile, frac in ((16, None), (32, 0.05)):
        n = sc.n
        act = pre = None
        if frac is None:
            r = Renderer(sc.cameras, n, tile=tile)
            r.fit_pair_capacity(params, sigma, sc.background)
            rows = np.arange(n)
        else:
            k = int(np.ceil(frac * n))
            idx, didx, dsg, _ = run_select(torch.rand(n, device=DEV), torch.ones(n, dtype=torch.uint8, device=DEV),
                                           k)
            act = {"idx": torch.tensor(idx, dtype=torch.int32, device=DEV),
                   "n": torch.tensor([len(idx)], dtype=torch.int32, device=DEV),
                   "delta_idx": torch.tensor(didx, dtype=torch.int32, device=DEV),
                   "delta_sign": torch.tensor(dsg, dtype=torch.int8, device=DEV),
                   "n_delta": torch.tensor([len(didx)], dtype=torch.int32, device=DEV)}
            pre = torch.zeros(9 * r_total_px(sc), device=DEV)
            r = Renderer(sc.cameras, n, active_capacity=k, delta_capacity=len(didx), tile=tile)
            r.fit_pair_capacity(params, sigma, sc.background, act, pre)
            rows = idx
        r.forward(params, sigma, sc.background, act, pre)
        tgt = r.pack(sc.targets)
        gi = torch.zeros_like(r.image)
        loss = torch.zeros(1, dtype=torch.float64, device=DEV)
        oit.l1_loss(r.image, tgt, r.cams_arr, r.n_views, gi, loss, r.ws)
        for v, cam in zip(r.views(gi, 3), sc.cameras):
            near = O.render(sc.params, sc.sigma, sc.background, cam, near_margin=NEAR_MARGIN)["near"]
            v[:, torch.tensor(near, device=DEV)] = 0.0
        g_gpu = new_grads(r.cap.active_capacity, DEV)
        gsig = torch.zeros(1, dtype=torch.float64, device=DEV)
        r.backward(params, sigma, sc.background, gi, g_gpu, gsig, act, pre)
        torch.cuda.synchronize()
        assert r.status() == 0
        g_views = [to_np(v) for v in r.views(gi, 3)]
        g_ref, _ = oracle_grads(sc.params, sc.sigma, sc.background, sc.cameras, g_views)
        ref = {kk: v[:, rows] for kk, v in g_ref.items()}
        compare_grads({g: to_np(g_gpu[g])[:, :len(rows)] for g, _ in O.GROUPS}, ref, log,
                      f"tile {tile} active {frac}: ")


def pre_sums(planes):
    """The stored pre-rendered accumulators [9][H][W] as the plain sums the oracle
    gives: the buffer keeps its colour sums centred on the colour offset 1/2, so
    P0 = P0' + Q0 / 2 and P1 = P1' + Q1 / 2."""
    out = np.array(planes, dtype=np.float64, copy=True)
    out[0:3] += 0.5 * out[6]
    out[3:6] += 0.5 * out[7]
    return out


def r_total_px(sc):
    return sum(c.width * c.height for c in sc.cameras)


def test_odd_pixel_counts_take_the_scalar_pixel_kernels():
    """A batch whose first view has an odd pixel count (101 x 77), so that the second
    view's planes start off any 16-byte boundary: L1 loss and gradient, images and
    parameter gradients against the oracle."""
    sc = scenes.random_scene(26, 1500, 64, 48, n_views=1, mean_range=1.0)
    sc.cameras = [scenes.orbit_camera(3.5, 0.2, 0.0, 101, 77), scenes.orbit_camera(3.5, -0.3, 0.1, 64, 48)]
    rng = np.random.default_rng(26)
    sc.targets = [rng.uniform(size=(3, c.height, c.width)).astype(np.float32) for c in sc.cameras]
    dense_case(sc, 16, 64)
    params = params_to_device(sc.params)
    sigma = torch.tensor([sc.sigma], device=DEV)
    r = Renderer(sc.cameras, sc.n)
    r.fit_pair_capacity(params, sigma, sc.background)
    r.forward(params, sigma, sc.background)
    tgt = r.pack(sc.targets)
    gi = torch.zeros_like(r.image)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    oit.l1_loss(r.image, tgt, r.cams_arr, r.n_views, gi, loss, r.ws)
    torch.cuda.synchronize()
    L_tot = 0.0
    for k, cam in enumerate(sc.cameras):
        img = to_np(r.views(r.image, 3)[k])
        L, g = O.l1_loss(img, sc.targets[k])
        L_tot += L
        np.testing.assert_array_equal(to_np(r.views(gi, 3)[k]), g.astype(np.float32).astype(np.float64))
    assert float(loss.item()) == pytest.approx(L_tot, rel=1e-7)


# ---------------------------------------------------------------------------------
# active set
# ---------------------------------------------------------------------------------

def run_select(score, label, k, mode=0, thresh=0.0, dcap=None):
    n = score.numel()
    acap = max(k, 1) if mode == 0 else n
    dcap = dcap or n
    idx = torch.zeros(acap, dtype=torch.int32, device=DEV)
    na = torch.zeros(1, dtype=torch.int32, device=DEV)
    didx = torch.zeros(dcap, dtype=torch.int32, device=DEV)
    dsg = torch.zeros(dcap, dtype=torch.int8, device=DEV)
    nd = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = torch.zeros(oit.select_workspace_bytes(n) + 256, dtype=torch.uint8, device=DEV)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + oit.select_workspace_bytes(n)]
    oit.update_active_set(score, n, mode, k, thresh, label, idx, na, didx, dsg, nd, ws)
    torch.cuda.synchronize()
    a = int(na.item())
    d = int(nd.item())
    return idx[:a].cpu().numpy(), didx[:d].cpu().numpy(), dsg[:d].cpu().numpy(), oit.read_status(ws)


@pytest.mark.parametrize("n,k", [(1, 1), (1000, 37), (5000, 250), (70001, 3500), (300000, 15000), (4096, 4096)])
def test_topk_selection_bit_exact(n, k):
    rng = np.random.default_rng(n + k)
    s = (rng.integers(0, 50, size=n) / 7.0).astype(np.float32)     # heavy ties
    s[rng.random(n) < 0.2] = 0.0
    old = (rng.random(n) < 0.3).astype(np.uint8)
    score = torch.tensor(s, device=DEV)
    label = torch.tensor(old, device=DEV)
    idx, didx, dsg, st = run_select(score, label, k)
    want = O.select_topk(s, k)
    np.testing.assert_array_equal(idx, want)
    lab, widx, wsign = O.label_delta(old, want, n)
    np.testing.assert_array_equal(label.cpu().numpy(), lab)
    np.testing.assert_array_equal(didx, widx)
    np.testing.assert_array_equal(dsg, wsign)
    assert st == 0


def test_threshold_selection_bit_exact():
    rng = np.random.default_rng(3)
    n = 20000
    s = rng.exponential(size=n).astype(np.float32)
    old = (rng.random(n) < 0.5).astype(np.uint8)
    label = torch.tensor(old, device=DEV)
    idx, didx, dsg, st = run_select(torch.tensor(s, device=DEV), label, 0, mode=1, thresh=1.0)
    want = O.select_threshold(s.astype(np.float64), 1.0)
    np.testing.assert_array_equal(idx, want)
    _, widx, wsign = O.label_delta(old, want, n)
    np.testing.assert_array_equal(didx, widx)
    np.testing.assert_array_equal(dsg, wsign)


def test_selection_overflow_sets_status():
    n = 1000
    s = np.linspace(0, 1, n).astype(np.float32)
    label = torch.zeros(n, dtype=torch.uint8, device=DEV)
    idx, didx, dsg, st = run_select(torch.tensor(s, device=DEV), label, 500, dcap=100)
    assert st & oit.STATUS_DELTA_OVERFLOW
    assert len(didx) == 100
    np.testing.assert_array_equal(didx, np.arange(500, 600))


def test_sparse_adam_matches_oracle():
    rng = np.random.default_rng(9)
    n = 5000
    rows = np.sort(rng.choice(n, size=700, replace=False))
    host = {"p": {g: rng.normal(size=(c, n)) for g, c in O.GROUPS},
            "m": {g: rng.normal(size=(c, n)) * 0.01 for g, c in O.GROUPS},
            "v": {g: rng.random(size=(c, n)) * 0.01 for g, c in O.GROUPS}}
    params, m, v = (params_to_device(host[k]) for k in ("p", "m", "v"))
    ref = {g: tuple(host[k][g].astype(np.float32).astype(np.float64) for k in ("p", "m", "v")) for g, _ in O.GROUPS}
    acap = 1024
    grads = {g: torch.zeros((c, acap), device=DEV) for g, c in O.GROUPS}
    gv = {g: rng.normal(size=(c, len(rows))).astype(np.float32) for g, c in O.GROUPS}
    for g, _ in O.GROUPS:
        grads[g][:, :len(rows)] = torch.tensor(gv[g], device=DEV)
    idx = torch.zeros(acap, dtype=torch.int32, device=DEV)
    idx[:len(rows)] = torch.tensor(rows, dtype=torch.int32, device=DEV)
    na = torch.tensor([len(rows)], dtype=torch.int32, device=DEV)
    step = torch.tensor([4], dtype=torch.int32, device=DEV)
    lr = [1e-3, 2e-3, 3e-3, 1e-2, 5e-3, 5e-3]
    oit.sparse_adam_step(params, oit.grads_struct(grads, acap), m, v, idx, na, n, lr, 0.9, 0.999, 1e-15, step)
    torch.cuda.synchronize()
    assert int(step.item()) == 5
    f32 = lambda x: float(np.float32(x))    # the kernel receives float32 hyper-parameters
    for k, (g, _) in enumerate(O.GROUPS):
        p0, m0, v0 = ref[g]
        O.adam_rows(p0, gv[g].astype(np.float64), m0, v0, rows, f32(lr[k]), f32(0.9), f32(0.999), f32(1e-15), 5)
        np.testing.assert_allclose(to_np(params[g]).T, p0, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(to_np(m[g]).T, m0, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(to_np(v[g]).T, v0, rtol=1e-5, atol=1e-9)


def test_sparse_adam_leaves_inactive_rows_bitwise():
    rng = np.random.default_rng(10)
    n = 3000
    rows = np.sort(rng.choice(n, size=300, replace=False))
    params = params_to_device({g: rng.normal(size=(c, n)) for g, c in O.GROUPS})
    m = {g: torch.zeros((n, c), device=DEV) for g, c in O.GROUPS}
    v = {g: torch.zeros((n, c), device=DEV) for g, c in O.GROUPS}
    before = {g: params[g].clone() for g, _ in O.GROUPS}
    grads = {g: torch.ones((c, 300), device=DEV) for g, c in O.GROUPS}
    idx = torch.tensor(rows, dtype=torch.int32, device=DEV)
    na = torch.tensor([300], dtype=torch.int32, device=DEV)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    oit.sparse_adam_step(params, oit.grads_struct(grads, 300), m, v, idx, na, n, [1e-3] * 6, 0.9, 0.999, 1e-15,
                         step)
    torch.cuda.synchronize()
    keep = torch.tensor(np.setdiff1d(np.arange(n), rows), device=DEV)
    for g, _ in O.GROUPS:
        assert torch.equal(params[g][keep], before[g][keep])
        assert torch.equal(m[g][keep], torch.zeros_like(m[g][keep]))
        assert not torch.equal(params[g][idx.long()], before[g][idx.long()])


@pytest.mark.parametrize("tile,batch", [(16, 64), (32, 32), (32, 64), (32, 128), (32, 256)])
def test_active_set_render_equals_dense(tile, batch):
    """Active splats rendered against the pre-rendered inactive set give the dense image
    and, on the active rows, the dense gradients (Sec. 4.1) -- after a first selection
    (every label change leaves A: sign +1) and after a second one, whose label changes
    have both signs (splats leaving pre and joining it in the same pass: App. A, BAU).
    Tile 32 runs the forward variant with label changes at six waves per SIMD, the
    launch of the timed step, at every LDS batch."""
    log(f"active set vs dense, 2 views, tile {tile}, batch {batch}")
    active_set_case(scenes.random_scene(31, 4000, 96, 80, n_views=2, mean_range=1.0), tile, batch)


@pytest.mark.parametrize("tile", [16, 32])
def test_opacity_cap_parity(tile):
    """Splats whose opacity exceeds the 0.99 cap (Sec. 3, alpha = min(0.99, ...)): the
    forward takes its clamping variant only when a listed record can reach the cap, so a
    scene with a tenth of its splats at opacity 0.9975 is compared with the oracle dense
    and through the active-set path, the capped splats among the active rows and the
    label changes of both signs."""
    sc = scenes.random_scene(37, 3000, 96, 80, n_views=2, mean_range=1.0)
    sc.params["opacity_logit"][0, ::10] = 6.0
    log(f"opacity cap, dense, tile {tile}")
    dense_case(sc, tile, 64)
    log(f"opacity cap, active set, tile {tile}")
    active_set_case(sc, tile, 64)


def active_set_case(sc, tile, batch):
    n = sc.n
    params = params_to_device(sc.params)
    sigma = torch.tensor([sc.sigma], device=DEV)
    rng = np.random.default_rng(31)
    total_px = sum(c.width * c.height for c in sc.cameras)
    # step 1: every splat active (pre empty); step 2: top-k of random scores
    k = 900
    label = torch.ones(n, dtype=torch.uint8, device=DEV)
    score = torch.tensor(rng.random(n).astype(np.float32), device=DEV)
    idx, didx, dsg, st = run_select(score, label, k)
    act = {"idx": torch.tensor(idx, dtype=torch.int32, device=DEV),
           "n": torch.tensor([len(idx)], dtype=torch.int32, device=DEV),
           "delta_idx": torch.tensor(didx, dtype=torch.int32, device=DEV),
           "delta_sign": torch.tensor(dsg, dtype=torch.int8, device=DEV),
           "n_delta": torch.tensor([len(didx)], dtype=torch.int32, device=DEV)}
    pre = torch.zeros(9 * total_px, device=DEV)
    r = Renderer(sc.cameras, n, active_capacity=k, delta_capacity=len(didx), tile=tile, batch=batch)
    r.fit_pair_capacity(params, sigma, sc.background, act, pre)
    r.forward(params, sigma, sc.background, act, pre)
    torch.cuda.synchronize()
    assert r.status() == 0
    imgs = image_views(r, r.image, 3)
    pres = image_views(r, pre, 9)
    inactive = np.ones(n, bool)
    inactive[idx] = False
    nears = []
    for v, cam in enumerate(sc.cameras):
        dense = O.render(sc.params, sc.sigma, sc.background, cam, near_margin=NEAR_MARGIN)
        nears.append(dense["near"])
        err = compare_image(imgs[v], dense["image"], dense["near"])
        log(f"  view {v}: active-set image vs dense oracle err {err:.2e}")
        assert err <= IMAGE_RTOL
        ref_pre = O.render(sc.params, sc.sigma, sc.background, cam, include=inactive.astype(np.uint8))["pre"]
        ok = ~dense["near"]
        got = pre_sums(pres[v])
        for p in range(9):
            rel = np.abs(got[p][ok] - ref_pre[p][ok]).max() / max(np.abs(ref_pre[p]).max(), 1e-30)
            assert rel < 1e-4, (v, p, rel)
    # gradients on the active rows equal the dense gradients restricted to A
    g_views = [rng.normal(size=(3, c.height, c.width)).astype(np.float32) for c in sc.cameras]
    mask_near(g_views, nears)
    gimg = r.pack(g_views)
    g_gpu = new_grads(k, DEV)
    gsig = torch.zeros(1, dtype=torch.float64, device=DEV)
    r.backward(params, sigma, sc.background, gimg, g_gpu, gsig, act, pre)
    torch.cuda.synchronize()
    g_ref, s_ref, s_abs = oracle_grads(sc.params, sc.sigma, sc.background, sc.cameras,
                                       [g.astype(np.float64) for g in g_views], with_abs=True)
    compare_grads({g: to_np(g_gpu[g])[:, :len(idx)] for g, _ in O.GROUPS},
                  {g: v[:, idx] for g, v in g_ref.items()}, log, "active: ")
    ok, srel = sigma_ok(float(gsig.item()), s_ref, s_abs)
    log(f"  sigma (active + pre part) rel {srel:.2e}")
    assert ok

    # step 3: a new selection; the label changes move splats in and out of pre
    score2 = torch.tensor(rng.random(n).astype(np.float32), device=DEV)
    idx2, didx2, dsg2, _ = run_select(score2, label, k)
    act2 = {"idx": torch.tensor(idx2, dtype=torch.int32, device=DEV),
            "n": torch.tensor([len(idx2)], dtype=torch.int32, device=DEV),
            "delta_idx": torch.tensor(didx2, dtype=torch.int32, device=DEV),
            "delta_sign": torch.tensor(dsg2, dtype=torch.int8, device=DEV),
            "n_delta": torch.tensor([len(didx2)], dtype=torch.int32, device=DEV)}
    assert (dsg2 > 0).any() and (dsg2 < 0).any(), "the second selection changes labels both ways"
    pre_before = pre.clone()
    r2 = Renderer(sc.cameras, n, active_capacity=k, delta_capacity=max(len(didx2), 1), tile=tile, batch=batch)
    r2.fit_pair_capacity(params, sigma, sc.background, act2, pre)
    r2.forward(params, sigma, sc.background, act2, pre)
    torch.cuda.synchronize()
    assert r2.status() == 0
    imgs2 = image_views(r2, r2.image, 3)
    for v, cam in enumerate(sc.cameras):
        dense = O.render(sc.params, sc.sigma, sc.background, cam, near_margin=NEAR_MARGIN)
        err = compare_image(imgs2[v], dense["image"], dense["near"])
        log(f"  after label changes, view {v}: err {err:.2e}")
        assert err <= IMAGE_RTOL
    # gradients of the second step's active rows, sigma with its pre part
    g_gpu2 = new_grads(k, DEV)
    gsig2 = torch.zeros(1, dtype=torch.float64, device=DEV)
    r2.backward(params, sigma, sc.background, gimg, g_gpu2, gsig2, act2, pre)
    torch.cuda.synchronize()
    assert r2.status() == 0
    compare_grads({g: to_np(g_gpu2[g])[:, :len(idx2)] for g, _ in O.GROUPS},
                  {g: v[:, idx2] for g, v in g_ref.items()}, log, "second selection: ")
    ok, srel = sigma_ok(float(gsig2.item()), s_ref, s_abs)
    log(f"  second selection: sigma rel {srel:.2e}")
    assert ok
    # the same pass from a pair capacity far too small through forward_fitted: the lists
    # overflow, the capacity grows, the pre buffer gets its label changes exactly once
    r3 = Renderer(sc.cameras, n, active_capacity=k, delta_capacity=max(len(didx2), 1), tile=tile, batch=batch,
                  pair_capacity=100)
    r3.forward_fitted(params, sigma, sc.background, act2, pre_before)
    torch.cuda.synchronize()
    assert r3.tuning.pair_capacity > 100 and r3.status() == 0
    assert torch.equal(r3.image, r2.image)
    assert torch.equal(pre_before, pre)

    # step 4: pre is up to date; the same active list with no label-change list takes the
    # forward's variant without label changes: the same image bit for bit, pre untouched,
    # and at tile 32 the dense image within tolerance
    act4 = {"idx": act2["idx"], "n": act2["n"]}
    img2 = r2.image.clone()
    pre_now = pre.clone()
    r2.forward(params, sigma, sc.background, act4, pre)
    torch.cuda.synchronize()
    assert r2.status() == 0
    assert torch.equal(pre, pre_now)
    assert torch.equal(r2.image, img2)
    r4 = Renderer(sc.cameras, n, active_capacity=k, tile=32, batch=64)
    r4.fit_pair_capacity(params, sigma, sc.background, act4, pre)
    r4.forward(params, sigma, sc.background, act4, pre)
    torch.cuda.synchronize()
    assert r4.status() == 0
    assert torch.equal(pre, pre_now)
    imgs4 = image_views(r4, r4.image, 3)
    for v, cam in enumerate(sc.cameras):
        dense = O.render(sc.params, sc.sigma, sc.background, cam, near_margin=NEAR_MARGIN)
        err = compare_image(imgs4[v], dense["image"], dense["near"])
        log(f"  no label-change list, tile 32, view {v}: err {err:.2e}")
        assert err <= IMAGE_RTOL


def test_tile_entry_counts_add_up():
    """The per-tile entry counts (a diagnostic of the forward's work per workgroup) add up
    to the entries the binning produced, in the active and the label-change class; in
    dense mode no tile holds a label change."""
    sc = scenes.random_scene(41, 3000, 96, 72, n_views=3, mean_range=1.0)
    params = params_to_device(sc.params)
    sigma = torch.tensor([sc.sigma], device=DEV)
    r = Renderer(sc.cameras, sc.n, tile=16)
    r.fit_pair_capacity(params, sigma, sc.background)
    r.forward(params, sigma, sc.background)
    torch.cuda.synchronize()
    views = r.tile_entries()
    assert [v.shape[1:] for v in views] == [((c.height + 15) // 16, (c.width + 15) // 16) for c in sc.cameras]
    assert sum(int(v[0].sum()) for v in views) == r.pairs_needed()
    assert all(int(v[1].sum()) == 0 for v in views)
    k = 700
    idx, didx, dsg, _ = run_select(torch.rand(sc.n, device=DEV), torch.ones(sc.n, dtype=torch.uint8, device=DEV), k)
    act = {"idx": torch.tensor(idx, dtype=torch.int32, device=DEV),
           "n": torch.tensor([len(idx)], dtype=torch.int32, device=DEV),
           "delta_idx": torch.tensor(didx, dtype=torch.int32, device=DEV),
           "delta_sign": torch.tensor(dsg, dtype=torch.int8, device=DEV),
           "n_delta": torch.tensor([len(didx)], dtype=torch.int32, device=DEV)}
    pre = torch.zeros(9 * r_total_px(sc), device=DEV)
    ra = Renderer(sc.cameras, sc.n, active_capacity=k, delta_capacity=len(didx), tile=16)
    ra.fit_pair_capacity(params, sigma, sc.background, act, pre)
    ra.forward(params, sigma, sc.background, act, pre)
    torch.cuda.synchronize()
    views = ra.tile_entries()
    na, nd = sum(int(v[0].sum()) for v in views), sum(int(v[1].sum()) for v in views)
    assert na + nd == ra.pairs_needed() and na > 0 and nd > 0


def test_pair_overflow_is_reported_and_bounded():
    sc = scenes.make_scene(1)
    params = params_to_device(sc.params)
    sigma = torch.tensor([sc.sigma], device=DEV)
    r = Renderer(sc.cameras, sc.n, tile=16, pair_capacity=100)
    r.forward(params, sigma, sc.background)
    torch.cuda.synchronize()
    assert r.status() & oit.STATUS_PAIR_OVERFLOW
    need = r.pairs_needed()
    assert need > 100
    r.set_tuning(pair_capacity=need)
    r.forward(params, sigma, sc.background)
    assert r.status() == 0


def test_entry_count_past_32_bits_is_reported_not_wrapped():
    """20,000 splats that each cover a whole 4096 x 4096 view at tile 8 need 5.2e9 tile
    entries, more than 32-bit offsets hold: the count saturates at 2^32 - 1, the overflow
    bit is set and the call stays within its capacity."""
    n = 20000
    rng = np.random.default_rng(61)
    cam = scenes.look_at_camera((0.0, 0.0, -3.0), 4096, 4096)
    p = {g: np.zeros((c, n)) for g, c in O.GROUPS}
    p["mean"][:] = rng.uniform(-0.05, 0.05, size=(3, n))
    p["log_scale"][:] = 0.3
    p["quat"][0] = 1.0
    p["opacity_logit"][:] = 4.0
    p["vsh"][0] = 1.0
    params = params_to_device(p)
    sigma = torch.tensor([10.0], device=DEV)
    r = Renderer([cam], n, tile=8, batch=64, pair_capacity=1 << 20)
    r.forward(params, sigma, (0.0, 0.0, 0.0))
    torch.cuda.synchronize()
    st = r.status()
    need = r.pairs_needed()
    log(f"  status {st}, entries needed (saturated) {need}")
    assert st & oit.STATUS_PAIR_OVERFLOW
    assert need == 2 ** 32 - 1
    assert bool(torch.isfinite(r.image).all())


def test_forward_and_backward_are_run_to_run_reproducible():
    """The tile lists come from a stable sort, the backward has no atomics and dL/dsigma
    adds its block shares in a fixed order: two calls on the same inputs give bitwise
    equal images, states and gradients, sigma's included (dense, then active set)."""
    sc = scenes.make_scene(2)
    params = params_to_device(sc.params)
    sigma = torch.tensor([sc.sigma], device=DEV)
    r = Renderer(sc.cameras, sc.n, tile=32, batch=64)
    r.fit_pair_capacity(params, sigma, sc.background)
    rng = np.random.default_rng(3)
    gimg = r.pack([rng.normal(size=(3, c.height, c.width)).astype(np.float32) for c in sc.cameras])
    outs = []
    for _ in range(2):
        r.forward(params, sigma, sc.background)
        g = new_grads(sc.n, DEV)
        gsig = torch.zeros(1, dtype=torch.float64, device=DEV)
        r.backward(params, sigma, sc.background, gimg, g, gsig)
        torch.cuda.synchronize()
        outs.append((r.image.clone(), r.pixstate.clone(), {k: v.clone() for k, v in g.items()}, gsig.clone()))
    assert r.status() == 0
    (i0, s0, g0, q0), (i1, s1, g1, q1) = outs
    assert torch.equal(i0, i1) and torch.equal(s0, s1)
    for k in g0:
        assert torch.equal(g0[k], g1[k]), k
    assert torch.equal(q0, q1)

    # the active-set path at the same tiling: label changes folded into a pre-rendered
    # buffer by the one-launch forward, then the backward restricted to the active rows
    n = sc.n
    k = max(1, n // 20)
    idx, didx, dsg, _ = run_select(torch.rand(n, device=DEV), torch.ones(n, dtype=torch.uint8, device=DEV), k)
    act = {"idx": torch.tensor(idx, dtype=torch.int32, device=DEV),
           "n": torch.tensor([len(idx)], dtype=torch.int32, device=DEV),
           "delta_idx": torch.tensor(didx, dtype=torch.int32, device=DEV),
           "delta_sign": torch.tensor(dsg, dtype=torch.int8, device=DEV),
           "n_delta": torch.tensor([len(didx)], dtype=torch.int32, device=DEV)}
    total_px = sum(c.width * c.height for c in sc.cameras)
    ra = Renderer(sc.cameras, n, active_capacity=k, delta_capacity=max(len(didx), 1), tile=32, batch=64)
    ra.fit_pair_capacity(params, sigma, sc.background, act, torch.zeros(9 * total_px, device=DEV))
    outs = []
    for _ in range(2):
        pre = torch.zeros(9 * total_px, device=DEV)
        ra.forward(params, sigma, sc.background, act, pre)
        g = new_grads(k, DEV)
        gsig = torch.zeros(1, dtype=torch.float64, device=DEV)
        ra.backward(params, sigma, sc.background, gimg, g, gsig, act, pre)
        torch.cuda.synchronize()
        outs.append((ra.image.clone(), pre, {kk: v.clone() for kk, v in g.items()}, gsig.clone()))
    assert ra.status() == 0
    (i0, p0, g0, q0), (i1, p1, g1, q1) = outs
    assert torch.equal(i0, i1) and torch.equal(p0, p1)
    for kk in g0:
        assert torch.equal(g0[kk], g1[kk]), kk
    assert torch.equal(q0, q1)


def test_autograd_matches_oracle_finite_differences():
    """OITRender's backward against FP64 central differences of the oracle forward."""
    log("autograd vs oracle finite differences")
    sc = scenes.random_scene(41, 40, 40, 32, mean_range=0.4, log_scale_mu=-2.5)
    params = {g: t.requires_grad_(True) for g, t in params_to_device(sc.params).items()}
    sigma = torch.tensor([sc.sigma], device=DEV, requires_grad=True)
    r = Renderer(sc.cameras, sc.n, tile=8, batch=32)
    rng = np.random.default_rng(41)
    gw = rng.normal(size=(3, 32, 40))
    img = render(r, sigma, params, sc.background)
    loss = (img * torch.tensor(gw.reshape(-1), dtype=torch.float32, device=DEV)).sum()
    loss.backward()
    cam = sc.cameras[0]
    base = O.render(sc.params, sc.sigma, sc.background, cam)

    def L(p, s=sc.sigma):
        rr = O.render(p, s, sc.background, cam)
        return float((gw * rr["image"]).sum()), rr["signature"]

    checked = 0
    for name, ncomp in O.GROUPS:
        an = to_np(params[name].grad).T      # [n][C] -> [C][n]
        picks = [(c, i) for c in range(ncomp) for i in range(sc.n)]
        rng.shuffle(picks)
        num = den = 0.0
        for c, i in picks[:40]:
            p = {k: v.astype(np.float64).copy() for k, v in sc.params.items()}
            x0 = p[name][c, i]
            h = 1e-6 * max(1.0, abs(x0))
            p[name][c, i] = x0 + h
            lp, sp = L(p)
            p[name][c, i] = x0 - h
            lm, sm = L(p)
            if sp != base["signature"] or sm != base["signature"]:
                continue
            fd = (lp - lm) / (2 * h)
            num += (an[c, i] - fd) ** 2
            den += fd ** 2
            checked += 1
        rel = math.sqrt(num) / max(math.sqrt(den), 1e-30)
        log(f"  {name}: autograd vs FD rel {rel:.2e}")
        assert rel <= 1e-3
    h = 1e-6 * sc.sigma
    fd = (L(sc.params, sc.sigma + h)[0] - L(sc.params, sc.sigma - h)[0]) / (2 * h)
    assert float(sigma.grad.item()) == pytest.approx(fd, rel=1e-3, abs=1e-8)
    assert checked > 100


def test_graph_replays_match_eager():
    """A captured active-set iteration replayed several times gives the same state as
    the same iterations run eagerly."""
    log("hipGraph replay vs eager")
    sc = scenes.random_scene(51, 3000, 64, 48, n_views=2, mean_range=1.0)

    def make():
        t = ActiveSetTrainer(sc, fraction=0.2, tile=16)
        t.warmup_dense_scores()
        return t

    eager = make()
    graphed = make()
    for _ in range(1):
        eager.iteration()
    graphed.capture()          # runs one eager warm-up iteration, then captures
    for it in range(3):
        eager.iteration()
        graphed.replay()
        torch.cuda.synchronize()
        # some unrelated eager work between replays
        _ = (torch.randn(1000, device=DEV) * 2).sum().item()
        for g, _ in O.GROUPS:
            np.testing.assert_allclose(to_np(graphed.params[g]), to_np(eager.params[g]), rtol=1e-5, atol=1e-6)
        assert float(graphed.loss.item()) == pytest.approx(float(eager.loss.item()), rel=1e-5)
        log(f"  replay {it}: loss {float(graphed.loss.item()):.6f}")
