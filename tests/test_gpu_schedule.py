"""GPU parity of the paper's active-set schedule: FPS view subsampling, label changes
between label arrays, epsilon-threshold activeness on the subsampled views, and lazily
updated per-view pre-rendered buffers (Sec. 4.1, Alg. "Active Set Method")."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2605_13855_amd import scenes
from tests.gpu_common import IMAGE_RTOL, NEAR_MARGIN, compare_image, oracle_grads, to_np

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2605_13855_amd import oit
    from paper_2605_13855_amd.render import _aligned_workspace, params_to_host
    from paper_2605_13855_amd.schedule import PaperScheduleTrainer

DEV = "cuda"


def log(msg):
    print(msg, flush=True)


def test_fps_views_match_oracle():
    rng = np.random.default_rng(0)
    for n, s in [(1, 1), (7, 3), (64, 30), (300, 30)]:
        c = rng.normal(size=(n, 3)).astype(np.float32)
        start = int(rng.integers(n))
        assert oit.fps_views(c, s, start) == O.fps(c, s, start)


@pytest.mark.parametrize("n", [1, 999, 1024, 100003])
def test_label_delta_bit_exact(n):
    rng = np.random.default_rng(n)
    old = (rng.random(n) < 0.4).astype(np.uint8)
    new = (rng.random(n) < 0.3).astype(np.uint8)
    ws = _aligned_workspace(oit.select_workspace_bytes(n), DEV)
    idx = torch.zeros(n, dtype=torch.int32, device=DEV)
    na = torch.zeros(1, dtype=torch.int32, device=DEV)
    didx = torch.zeros(n, dtype=torch.int32, device=DEV)
    dsg = torch.zeros(n, dtype=torch.int8, device=DEV)
    nd = torch.zeros(1, dtype=torch.int32, device=DEV)
    oit.label_delta(torch.tensor(old, device=DEV), torch.tensor(new, device=DEV), n, idx, na, didx, dsg, nd, ws)
    torch.cuda.synchronize()
    want_idx = np.nonzero(new)[0]
    _, widx, wsign = O.label_delta(old, want_idx, n)
    np.testing.assert_array_equal(idx[:int(na.item())].cpu().numpy(), want_idx)
    np.testing.assert_array_equal(didx[:int(nd.item())].cpu().numpy(), widx)
    np.testing.assert_array_equal(dsg[:int(nd.item())].cpu().numpy(), wsign)


def small_scene(n_views=6):
    sc = scenes.random_scene(61, 3000, 64, 48, n_views=n_views, mean_range=1.0)
    return sc


def test_threshold_activeness_on_subsampled_views():
    """The active set after an update is {score > 1} with the score of the summed
    gradient over the FPS views; compared with the oracle away from the threshold."""
    sc = small_scene()
    probe = PaperScheduleTrainer(sc, eps=[1.0] * 6, interval=100, n_sub=3, seed=1, loss="l1")
    probe.update_active_set()
    s = to_np(probe.score)
    eps = [float(np.quantile(s, 0.7))] * 6          # about 30% active
    t = PaperScheduleTrainer(sc, eps=eps, interval=100, n_sub=3, seed=1, loss="l1")
    t.update_active_set()
    torch.cuda.synchronize()
    views = t.last_update_views
    cams = [sc.cameras[i] for i in views]
    # oracle: dense render of the subsampled views, L1 gradient, summed parameter gradients
    dldc = []
    for i in views:
        r = O.render(sc.params, sc.sigma, sc.background, sc.cameras[i])
        _, g = O.l1_loss(r["image"], sc.targets[i])
        dldc.append(g)
    g_ref, _ = oracle_grads(sc.params, sc.sigma, sc.background, cams, dldc)
    score_ref = O.activeness_score(g_ref, np.arange(sc.n), {g: e for (g, _), e in zip(O.GROUPS, eps)})
    s_gpu = to_np(t.score)
    rel = np.linalg.norm(s_gpu - score_ref) / np.linalg.norm(score_ref)
    log(f"  score rel err {rel:.2e}, active {t.active_fraction():.3f}")
    assert rel < 1e-3
    lab = t.labels[t.epoch].cpu().numpy().astype(bool)
    want = score_ref > 1.0
    clear = np.abs(score_ref - 1.0) > 1e-3
    assert np.array_equal(lab[clear], want[clear])


def test_schedule_lazy_pre_buffers_match_dense_oracle():
    """After several updates and iterations, rendering any view with the active set and
    its lazily updated pre-rendered buffer gives the dense image of the current splats."""
    sc = small_scene(6)
    probe = PaperScheduleTrainer(sc, eps=[1.0] * 6, interval=100, n_sub=3, seed=2)
    probe.update_active_set()
    eps = [float(np.quantile(to_np(probe.score), 0.6))] * 6
    del probe
    t = PaperScheduleTrainer(sc, eps=eps, interval=4, n_sub=3, seed=2, lr=5e-3)
    for _ in range(14):
        t.iteration()
    torch.cuda.synchronize()
    log(f"  epoch {t.epoch}, active {t.active_fraction():.3f}, rebuilds {t.rebuilds}, view epochs {t.view_epoch}")
    assert t.epoch >= 3
    params = params_to_host(t.params)
    sigma = float(t.sigma.item())
    for v, cam in enumerate(sc.cameras):
        t.render_view(v)
        img = to_np(t.r.image).reshape(3, cam.height, cam.width)
        ref = O.render(params, sigma, sc.background, cam, near_margin=NEAR_MARGIN)
        err = compare_image(img, ref["image"], ref["near"])
        log(f"  view {v}: image err {err:.2e}")
        assert err <= IMAGE_RTOL
