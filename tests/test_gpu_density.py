"""GPU parity of the first training phase's density control (3DGS's densification,
pruning and opacity reset, kept by the paper with a random keep probability: Sec. 5.1
"Implementation Details") and of checkpoint / resume."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2605_13855_amd import scenes
from tests.gpu_common import GRAD_RTOL, IMAGE_RTOL, NEAR_MARGIN, compare_image, to_np

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2605_13855_amd import checkpoint, oit
    from paper_2605_13855_amd.density import DensifyingTrainer, hand_over
    from paper_2605_13855_amd.render import Renderer, _aligned_workspace, new_grads, params_to_device, params_to_host
    from paper_2605_13855_amd.schedule import PaperScheduleTrainer

DEV = "cuda"
F = {f: k for k, f in enumerate(O.PROJECT_FIELDS)}


def log(msg):
    print(msg, flush=True)


def visibility_ambiguous(row, w, h):
    """Whether a small perturbation of the footprint box flips the visibility decision."""
    base = O.footprint_visible(row, w, h)
    for dt, dx, dy in ((2e-4, 0, 0), (-2e-4, 0, 0), (0, 1e-3, 0), (0, -1e-3, 0), (0, 0, 1e-3), (0, 0, -1e-3)):
        r = row.copy()
        r[F["tau"]] *= 1 + dt
        r[F["mx"]] += dx
        r[F["my"]] += dy
        if O.footprint_visible(r, w, h) != base:
            return True
    return False


def test_densify_stats_match_oracle():
    """Statistic after a dense three-view backward: visible-view counts equal (away
    from the box edge), gradient-norm sums and radii normwise to the gradient bar."""
    sc = scenes.random_scene(71, 3000, 64, 48, n_views=3, mean_range=1.2)
    params = params_to_device(sc.params)
    sigma = torch.tensor([sc.sigma], device=DEV)
    r = Renderer(sc.cameras, sc.n, tile=16)
    r.fit_pair_capacity(params, sigma, sc.background)
    r.forward(params, sigma, sc.background)
    rng = np.random.default_rng(71)
    g_views = [rng.normal(size=(3, c.height, c.width)).astype(np.float32) for c in sc.cameras]
    r.backward(params, sigma, sc.background, r.pack(g_views), new_grads(sc.n, DEV),
               torch.zeros(1, dtype=torch.float64, device=DEV))
    acc = torch.zeros(sc.n, device=DEV)
    den = torch.zeros(sc.n, device=DEV)
    rad = torch.zeros(sc.n, device=DEV)
    oit.densify_stats(r.cams_arr, r.n_views, r.cap, None, None, None, acc, den, rad, r.ws, r.tuning)
    torch.cuda.synchronize()
    assert r.status() == 0
    a_ref, d_ref, r_ref = O.densify_stats(sc.params, sc.sigma, sc.background, sc.cameras,
                                          [g.astype(np.float64) for g in g_views])
    amb = np.zeros(sc.n, bool)
    for cam in sc.cameras:
        pr = O.project(sc.params, sc.sigma, cam)
        amb |= np.array([visibility_ambiguous(pr[i], cam.width, cam.height) for i in range(sc.n)])
    a, d, rr = to_np(acc), to_np(den), to_np(rad)
    ok = ~amb
    log(f"  visible in some view: {(d_ref > 0).sum()}, ambiguous {amb.sum()}")
    np.testing.assert_array_equal(d[ok], d_ref[ok])
    same = ok & (d == d_ref)
    rel = np.linalg.norm(a[same] - a_ref[same]) / np.linalg.norm(a_ref[same])
    rrel = np.linalg.norm(rr[same] - r_ref[same]) / np.linalg.norm(r_ref[same])
    log(f"  accum rel {rel:.2e}, radius rel {rrel:.2e}")
    assert rel <= GRAD_RTOL and rrel <= 1e-5


def random_plan_inputs(seed, n):
    """Splats and statistics that reach every case, with every decision input at least
    1% away from its threshold."""
    sc = scenes.random_scene(seed, n, 32, 32)
    rng = np.random.default_rng(seed)
    p = {g: sc.params[g].astype(np.float32) for g, _ in O.GROUPS}
    p["log_scale"] += rng.normal(0, 0.7, size=p["log_scale"].shape).astype(np.float32)
    p["opacity_logit"] = rng.normal(-2.0, 2.5, size=(1, n)).astype(np.float32)
    den = rng.integers(0, 4, size=n).astype(np.float32)
    acc = (rng.exponential(1.0, size=n) * den).astype(np.float32)
    radius = rng.uniform(0, 40, size=n).astype(np.float32)
    uniform = rng.random(n).astype(np.float32)
    smax = np.exp(p["log_scale"].astype(np.float64)).max(axis=0)
    extent = 2.0
    rules = O.DensityRules(grad_threshold=1.0, percent_dense=float(np.median(smax)) / extent, scene_extent=extent,
                           min_opacity=0.05, max_screen_size=30.0, max_world_frac=float(np.quantile(smax, 0.9)) / extent,
                           keep_probability=0.7)
    avg = np.where(den > 0, acc / np.maximum(den, 1), 0)
    op = 1 / (1 + np.exp(-p["opacity_logit"][0].astype(np.float64)))
    near = (np.abs(avg / rules.grad_threshold - 1) < 0.01) | (np.abs(uniform / rules.keep_probability - 1) < 0.01)
    for lim in (rules.percent_dense * extent, rules.max_world_frac * extent, rules.max_world_frac * extent * 1.6):
        near |= np.abs(smax / lim - 1) < 0.01
    near |= np.abs(op / rules.min_opacity - 1) < 0.01
    near |= np.abs(radius / rules.max_screen_size - 1) < 0.01
    acc[near] = 0.0          # no longer a candidate ...
    p["opacity_logit"][0, near] = 3.0     # ... and well above the minimum opacity
    radius[near] = 1.0
    ls = p["log_scale"][:, near]
    p["log_scale"][:, near] = np.minimum(ls, np.float32(np.log(0.5 * rules.percent_dense * extent)))
    return p, acc, den, radius, uniform, rng.normal(size=(n, 2, 3)).astype(np.float32), rules


def rules_struct(r):
    return oit.DensityRules(r.grad_threshold, r.percent_dense, r.scene_extent, r.min_opacity, r.max_screen_size,
                            r.max_world_frac, r.keep_probability, 0)


@pytest.mark.parametrize("n", [1, 777, 5000])
def test_densify_plan_and_apply_match_oracle(n):
    p, acc, den, radius, uniform, normals, rules = random_plan_inputs(80 + n, n)
    rng = np.random.default_rng(n)
    m = {g: rng.normal(size=(c, n)).astype(np.float32) for g, c in O.GROUPS}
    v = {g: rng.random(size=(c, n)).astype(np.float32) for g, c in O.GROUPS}
    dp, dm, dv = params_to_device(p), params_to_device(m), params_to_device(v)
    t = lambda x: torch.tensor(x, device=DEV)
    ws = _aligned_workspace(oit.densify_workspace_bytes(n), DEV)
    n_new = torch.zeros(1, dtype=torch.int64, device=DEV)
    sp = oit.splats_struct(dp)
    oit.densify_plan(sp, t(acc), t(den), t(radius), t(uniform), rules_struct(rules), n_new, ws)
    nn = int(n_new.item())
    f64 = {g: p[g].astype(np.float64) for g, _ in O.GROUPS}
    q, qm, qv, src = O.densify(f64, {g: m[g].astype(np.float64) for g in m}, {g: v[g].astype(np.float64) for g in v},
                               acc, den, radius, uniform, normals.astype(np.float64), rules)
    clone, split, ko, kc, kch = O.densify_decisions(f64, acc, den, radius, uniform, rules)
    log(f"  n {n}: kept {ko.sum()}, clones {kc.sum()}, split {kch.sum()} -> {nn} (oracle {len(src)})")
    assert nn == len(src)
    if nn == 0:
        return
    p2 = {g: torch.full((nn, c), float("nan"), device=DEV) for g, c in O.GROUPS}
    m2 = {g: torch.full((nn, c), float("nan"), device=DEV) for g, c in O.GROUPS}
    v2 = {g: torch.full((nn, c), float("nan"), device=DEV) for g, c in O.GROUPS}
    oit.densify_apply(sp, dm, dv, t(normals), p2, m2, v2, nn, ws)
    torch.cuda.synchronize()
    got = params_to_host(p2)
    gm, gv = params_to_host(m2), params_to_host(v2)
    nchild = 2 * kch.sum()
    copies = nn - nchild
    for g, _ in O.GROUPS:
        exact = slice(0, copies) if g in ("mean", "log_scale") else slice(0, nn)
        np.testing.assert_array_equal(got[g][:, exact], q[g][:, exact].astype(np.float32), err_msg=g)
        np.testing.assert_array_equal(gm[g], qm[g].astype(np.float32), err_msg=g)
        np.testing.assert_array_equal(gv[g], qv[g].astype(np.float32), err_msg=g)
    if nchild:
        ch = slice(copies, nn)
        scale = np.abs(q["mean"][:, ch]).max() + np.exp(q["log_scale"][:, ch]).max()
        assert np.abs(got["mean"][:, ch] - q["mean"][:, ch]).max() <= 1e-6 * scale
        assert np.abs(got["log_scale"][:, ch] - q["log_scale"][:, ch]).max() <= 1e-6


def test_reset_opacity_matches_oracle():
    rng = np.random.default_rng(90)
    n = 3001
    logit = rng.normal(-3, 3, size=n).astype(np.float32)
    m = rng.normal(size=n).astype(np.float32)
    v = rng.random(n).astype(np.float32)
    tl, tm, tv = (torch.tensor(x, device=DEV) for x in (logit, m, v))
    oit.reset_opacity(tl, tm, tv, n, 0.01)
    torch.cuda.synchronize()
    p = {"opacity_logit": logit[None].astype(np.float64)}
    mm = {"opacity_logit": m[None].astype(np.float64)}
    vv = {"opacity_logit": v[None].astype(np.float64)}
    O.reset_opacity(p, mm, vv, 0.01)
    np.testing.assert_array_equal(to_np(tl), p["opacity_logit"][0].astype(np.float32).astype(np.float64))
    assert not tm.any() and not tv.any()


def small_training_scene():
    return scenes.random_scene(95, 2500, 64, 48, n_views=4, mean_range=1.0)


def test_densifying_trainer_renders_its_new_set_and_hands_over():
    """A first phase with two densifications: the densified set renders like the dense
    oracle on every view, and the active-set schedule continues from it."""
    sc = small_training_scene()
    t = DensifyingTrainer(sc, densify_from=0, densify_until=100, densify_interval=5, opacity_reset_interval=1000,
                          grad_threshold=2e-5, keep_probability=0.6, seed=3, loss="l1")
    for _ in range(11):
        t.iteration()
    torch.cuda.synchronize()
    log(f"  history {t.history}, splats {t.n}")
    assert len(t.history) == 2 and t.n != sc.n
    params = params_to_host(t.params)
    sigma = float(t.sigma.item())
    r = Renderer(sc.cameras, t.n, tile=16)
    r.fit_pair_capacity(t.params, t.sigma, sc.background)
    r.forward(t.params, t.sigma, sc.background)
    for k, cam in enumerate(sc.cameras):
        img = to_np(r.views(r.image, 3)[k])
        ref = O.render(params, sigma, sc.background, cam, near_margin=NEAR_MARGIN)
        err = compare_image(img, ref["image"], ref["near"])
        log(f"  view {k}: err {err:.2e}")
        assert err <= IMAGE_RTOL
    nxt = hand_over(t, sc, [1e-3] * 6, interval=4, n_sub=2, seed=4, loss="l1")
    for _ in range(5):
        nxt.iteration()
    torch.cuda.synchronize()
    assert nxt.n == t.n and np.isfinite(float(nxt.loss.item()))
    for g in t.params:
        assert torch.isfinite(nxt.params[g]).all()


def states_equal(a, b):
    for d1, d2 in ((a.params, b.params), (a.m, b.m), (a.v, b.v)):
        for g in d1:
            if not torch.equal(d1[g], d2[g]):
                return False, g
    for k in ("sigma", "sig_m", "sig_v", "step"):
        if not torch.equal(getattr(a, k), getattr(b, k)):
            return False, k
    return True, None


def test_checkpoint_resume_densifying_trainer_bitwise(tmp_path):
    """Save in the middle of a densification interval, resume in a trainer built with
    another seed: the next iterations (a densification and an opacity reset among them)
    repeat bit for bit, sigma included."""
    sc = small_training_scene()
    kw = dict(densify_from=0, densify_until=100, densify_interval=5, opacity_reset_interval=7,
              grad_threshold=2e-5, keep_probability=0.6, loss="l1")
    a = DensifyingTrainer(sc, seed=5, **kw)
    for _ in range(3):
        a.iteration()
    path = tmp_path / "first.safetensors"
    checkpoint.save(a, path)
    for _ in range(6):
        a.iteration()
    b = DensifyingTrainer(sc, seed=6, **kw)
    checkpoint.load(b, path)
    for _ in range(6):
        b.iteration()
    torch.cuda.synchronize()
    assert a.history == b.history and a.it == b.it
    eq, what = states_equal(a, b)
    assert eq, what


def test_checkpoint_resume_schedule_trainer_bitwise(tmp_path):
    """The schedule trainer resumed from a checkpoint taken between active-set updates
    repeats the uninterrupted run bit for bit (labels, pre-rendered buffers, splats)."""
    sc = small_training_scene()
    probe = PaperScheduleTrainer(sc, eps=[1.0] * 6, interval=100, n_sub=2, seed=1, loss="l1")
    probe.update_active_set()
    eps = [float(np.quantile(to_np(probe.score), 0.7))] * 6
    del probe
    kw = dict(interval=4, n_sub=2, lr=5e-3, loss="l1")
    a = PaperScheduleTrainer(sc, eps=eps, seed=2, **kw)
    for _ in range(6):
        a.iteration()
    path = tmp_path / "sched.safetensors"
    checkpoint.save(a, path)
    for _ in range(7):
        a.iteration()
    b = PaperScheduleTrainer(sc, eps=eps, seed=9, **kw)
    checkpoint.load(b, path)
    for _ in range(7):
        b.iteration()
    torch.cuda.synchronize()
    eq, what = states_equal(a, b)
    assert eq, what
    assert a.epoch == b.epoch and a.view_epoch == b.view_epoch
    assert torch.equal(a.labels[a.epoch], b.labels[b.epoch])
    for pa, pb in zip(a.pre, b.pre):
        assert torch.equal(pa, pb)


def test_checkpoint_resume_active_set_trainer_bitwise(tmp_path):
    """The top-k-every-step trainer resumed into a captured HIP graph: the state is
    restored in place, so the graph's replays continue the saved run bit for bit."""
    from paper_2605_13855_amd.render import ActiveSetTrainer
    sc = scenes.random_scene(97, 3000, 64, 48, n_views=2, mean_range=1.0)

    def make():
        t = ActiveSetTrainer(sc, fraction=0.2, tile=16)
        t.warmup_dense_scores()
        return t

    a = make()
    for _ in range(3):
        a.iteration()
    path = tmp_path / "active.safetensors"
    checkpoint.save(a, path)
    for _ in range(4):
        a.iteration()
    b = make()
    b.capture()                      # one eager warm-up iteration, then the graph
    checkpoint.load(b, path)
    for _ in range(4):
        b.replay()
    torch.cuda.synchronize()
    eq, what = states_equal(a, b)
    assert eq, what
    assert torch.equal(a.label, b.label) and torch.equal(a.pre, b.pre)
