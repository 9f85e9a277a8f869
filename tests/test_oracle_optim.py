"""Pins of the optimisation oracle (oracle/optim.py) against things other
than itself: PyTorch's Adam, closed forms of Adam's steps, pose identities,
invariants of the decoupled step, the projection of created Gaussians back
to their pixels by the C oracle, and convergence of the tracking loop."""
import numpy as np
import pytest
import torch

import oracle
from oracle import optim
from paper_2408_05635_amd import scenes


def _torch_adam(x0, grads, lr, b1, b2, eps):
    x = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([x], lr=lr, betas=(b1, b2), eps=eps)
    out = []
    for g in grads:
        opt.zero_grad()
        x.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        out.append(x.detach().numpy().copy())
    return out


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    x = rng.normal(size=11)
    grads = [rng.normal(size=11) * 10.0 ** rng.uniform(-6, 1, size=11) for _ in range(6)]
    ref = _torch_adam(x, grads, 3e-3, 0.9, 0.999, 1e-8)
    m = np.zeros(11)
    v = np.zeros(11)
    for k, g in enumerate(grads):
        x, m, v = optim.adam_step(x, g, m, v, k + 1, 3e-3, 0.9, 0.999, 1e-8)
        np.testing.assert_allclose(x, ref[k], rtol=1e-14, atol=1e-16)


def test_adam_closed_forms():
    # bias correction makes every step of a constant gradient lr * g / (|g| + eps)
    g = np.array([2.0, -0.5, 1e-3, -7.0])
    x0 = np.array([0.1, 0.2, 0.3, 0.4])
    lr, eps = 1e-2, 1e-8
    x, m, v = x0, np.zeros(4), np.zeros(4)
    for k in range(1, 6):
        x, m, v = optim.adam_step(x, g, m, v, k, lr, 0.9, 0.999, eps)
        np.testing.assert_allclose(x, x0 - k * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # a zero gradient on the first step leaves x where it is
    x1, _, _ = optim.adam_step(x0, np.zeros(4), np.zeros(4), np.zeros(4), 1, lr, 0.9, 0.999, eps)
    assert np.array_equal(x1, x0)


def test_map_step_matches_torch_per_group():
    rng = np.random.default_rng(8)
    n = 9
    hp = optim.MapAdam()
    params = {k: rng.normal(size=(n, d)) for k, d in (("means", 3), ("quats", 4), ("log_scales", 3), ("rgb", 3))}
    params["opacity_logits"] = rng.normal(size=n)
    m = {k: np.zeros_like(a) for k, a in params.items()}
    v = {k: np.zeros_like(a) for k, a in params.items()}
    ts = {k: torch.tensor(a, requires_grad=True) for k, a in params.items()}
    opt = torch.optim.Adam([{"params": [ts[k]], "lr": hp.lr(k)} for k in ts], betas=(hp.beta1, hp.beta2),
                           eps=hp.eps)
    for step in range(1, 4):
        grads = {k: rng.normal(size=a.shape) for k, a in params.items()}
        params, m, v = optim.map_step(params, grads, m, v, step, hp)
        opt.zero_grad()
        for k in ts:
            ts[k].grad = torch.tensor(grads[k])
        opt.step()
        for k in ts:
            np.testing.assert_allclose(params[k], ts[k].detach().numpy(), rtol=1e-14, atol=1e-16)


def test_pose_identities():
    rng = np.random.default_rng(9)
    for _ in range(5):
        q = rng.normal(size=4) * rng.uniform(0.5, 2.0)
        t = rng.normal(size=3)
        C = optim.centre_of(q, t)
        np.testing.assert_allclose(optim.trans_of(q, C), t, atol=1e-14)
        # the centre maps to the camera origin
        np.testing.assert_allclose(optim.rot(q) @ C + t, 0.0, atol=1e-14)
        # the renderer's rotation agrees (it normalises q the same way)
        np.testing.assert_allclose(optim.rot(q), oracle.quat_to_rot(q), atol=1e-14)
    assert np.allclose(optim.centre_of([1.0, 0, 0, 0], [0.3, -0.2, 0.1]), [-0.3, 0.2, -0.1])


def test_decoupled_step_invariants():
    rng = np.random.default_rng(10)
    hp = optim.PoseAdam()
    st = optim.PoseState.from_pose(rng.normal(size=4), rng.normal(size=3))
    # no centre gradient: the camera turns in place (C fixed, t changes)
    s1 = optim.pose_step(st, rng.normal(size=4), np.zeros(3), hp)
    assert np.array_equal(s1.C, st.C) and not np.allclose(s1.pose()[1], st.pose()[1])
    # no rotation gradient: the orientation is unchanged and the centre moves by lr per axis
    dc = np.array([1.0, -2.0, 0.5])
    s2 = optim.pose_step(st, np.zeros(4), dc, hp)
    assert np.array_equal(s2.q, st.q)
    np.testing.assert_allclose(s2.C - st.C, -hp.lr_pos * np.sign(dc), rtol=1e-7)


def test_tracking_loop_converges_config1():
    """From the 2 degree / 2 cm perturbed start of the tiny tracking scene the
    oracle's loop reduces the loss and moves toward the true pose."""
    w = scenes.config1()
    tv = w.target_views
    r = oracle.run(w.truth, tv)
    tg = oracle.Targets(r.rgb, r.depth, r.sil)
    hp = optim.PoseAdam(lr_rot=1e-3, lr_pos=1e-3)
    hist, losses = optim.track(w.gaussians, w.views.cams, np.asarray(w.views.quat), np.asarray(w.views.trans), tg,
                               oracle.Options(**w.weights), hp, 25)

    def err(st):
        q, t = st.pose()
        dq = abs(float(np.dot(q / np.linalg.norm(q), tv.quat[0] / np.linalg.norm(tv.quat[0]))))
        return 2 * np.degrees(np.arccos(min(1.0, dq))), float(np.linalg.norm(optim.centre_of(q, t)
                                                                            - optim.centre_of(tv.quat[0], tv.trans[0])))
    e0 = err(optim.PoseState.from_pose(w.views.quat[0], w.views.trans[0]))
    e1 = err(hist[-1][0])
    print(f"rotation {e0[0]:.3f} -> {e1[0]:.3f} deg, centre {e0[1] * 100:.2f} -> {e1[1] * 100:.2f} cm, "
          f"loss {losses[0, 0]:.5f} -> {losses[-1, 0]:.5f}")
    assert losses[-1, 0] < 0.7 * losses[0, 0]
    assert e1[0] < e0[0] and e1[1] < e0[1]


@pytest.mark.parametrize("iso", [True, False])
def test_new_gaussians_project_back_to_their_pixels(iso):
    cam = scenes.Camera(40, 30, 35.0, 36.0, 19.5, 14.5)
    rng = np.random.default_rng(11)
    P = cam.width * cam.height
    depth = rng.uniform(0.5, 4.0, size=P)
    depth[rng.random(P) < 0.1] = 0.0        # missing depth
    sil = rng.random(P).astype(np.float32)
    rgb = rng.random((3, P))
    q = np.array([0.9, 0.1, -0.2, 0.15])
    t = np.array([0.2, -0.1, 0.3])
    pix, g = optim.new_gaussians(cam, q, t, rgb, depth, sil, 0.5, isotropic=iso)
    assert pix.size == int(((depth > 0) & (sil < 0.5)).sum()) and np.all(np.diff(pix) > 0)

    class G:
        pass
    gg = G()
    for k, a in g.items():
        setattr(gg, k, a)
    views = optim.Views([cam], q[None], t[None])
    pr = oracle.project_view(gg, views, 0, oracle.Options(blur2d=0.0))
    u, v = pix % cam.width, pix // cam.width
    np.testing.assert_allclose(pr.mean2d[:, 0], u, atol=1e-9)
    np.testing.assert_allclose(pr.mean2d[:, 1], v, atol=1e-9)
    np.testing.assert_allclose(pr.Xc[:, 2], depth[pix], rtol=1e-12)
    # one-pixel radius: scale * f / depth = 1; opacity 0.5; the pixel's colour
    np.testing.assert_allclose(np.exp(g["log_scales"][:, 0]) * 0.5 * (cam.fx + cam.fy) / depth[pix], 1.0, rtol=1e-12)
    assert np.all(g["opacity_logits"] == 0.0)
    np.testing.assert_array_equal(g["rgb"], rgb[:, pix].T)
    # initialisation (no silhouette): every pixel with depth
    pix0, _ = optim.new_gaussians(cam, q, t, rgb, depth, None)
    assert np.array_equal(pix0, np.nonzero(depth > 0)[0])
