"""Warm-start machinery on tiny data: the network trains (loss falls), a warm
start reaches the same steady state as a cold start (and, on a geometry with
a node whose y links are all solid, only does so after the prediction is
projected onto the invariants of a start from rest), and a prediction that
blows up falls back to a cold start."""
import numpy as np
import pytest

from paper_1703_08015_amd import inputs, warmstart

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def trained(torch):
    rng = np.random.default_rng(0)
    masks, gs = [], []
    for k in range(6):
        m, _ = inputs.spheres_3d(16, float(rng.uniform(0.4, 0.7)), 2.0, 4.0, seed=100 + k)
        d = rng.normal(size=3)
        masks.append(m)
        gs.append((1e-6 * d / np.linalg.norm(d)).tolist())
    data, steps, res = warmstart.steady_dataset(torch, masks, gs, tau=0.8)
    assert np.all(steps > 0)
    scale = warmstart.make_targets(torch, data, 0.8)
    net = warmstart.make_net(levels=2, base=8, seed=1, out_scale=scale)
    hist = warmstart.train(torch, net, data, epochs=40, lr=3e-3)
    return net, data, hist


def test_training_reduces_loss(torch, trained):
    net, data, hist = trained
    assert hist[-1] < 0.5 * hist[0], hist


def test_warm_start_reaches_cold_steady_state(torch, trained):
    net, data, _ = trained
    rows = warmstart.evaluate(torch, net, data[:2], 0.8)
    for r in rows:
        print(r, flush=True)
        assert r["warm_steps"] > 0 and r["cold_steps"] > 0
        assert r["warm_vs_cold_u_rel_l2"] <= 1e-4
        assert r["prediction_u_rel_l2"] < 1.0
    # data[0] holds a node whose y momentum is a one-node invariant: the raw
    # prediction keeps its own value of it and settles elsewhere
    raw = warmstart.evaluate(torch, net, data[:1], 0.8, project=False)[0]
    print("raw", raw, flush=True)
    assert raw["warm_vs_cold_u_rel_l2"] > 1e-4


def test_blown_up_prediction_falls_back_to_cold(torch, trained):
    _, data, _ = trained
    sm = data[0]
    rho = torch.full(sm.shape, float("nan"), dtype=torch.float64, device="cuda")
    u = torch.zeros((3,) + sm.shape, dtype=torch.float64, device="cuda")
    steps, _, u_out, fell_back = warmstart.solve(torch, sm, 0.8, init=(rho, u))
    assert fell_back and steps > 0 and torch.isfinite(u_out).all()


def test_warm_start_matches_the_fp64_oracle_steady_state(torch, trained):
    """The FP32 warm-started solve ends within 1e-3 (velocity rel-L2) of the
    FP64 CPU oracle's steady state of the same geometry and force."""
    from oracle import dense
    net, data, _ = trained
    for sm in data[:2]:
        init = warmstart.predict_fields(torch, net, sm, 0.8)
        steps, _, u_warm, fell_back = warmstart.solve(torch, sm, 0.8, init=init)
        assert steps > 0 and not fell_back
        mask = sm.solid.cpu().numpy().astype(bool)
        f = dense.init(19, mask)
        prev = None
        for _ in range(300):
            f = dense.step(19, mask, f, 0.8, sm.g, 100, nthreads=4)
            _, u_ref = dense.moments(19, mask, f, sm.g)
            if prev is not None and np.linalg.norm(u_ref - prev) < 1e-10 * np.linalg.norm(u_ref):
                break
            prev = u_ref
        u = u_warm.cpu().numpy()
        fl = ~mask
        err = np.linalg.norm(u[:, fl] - u_ref[:, fl]) / np.linalg.norm(u_ref[:, fl])
        print("warm FP32 vs FP64 oracle", err, flush=True)
        assert err <= 1e-3


def test_gain_on_held_out_samples(torch, trained):
    """What the trained network gains on geometries it never saw, and the
    ceiling of any (rho, u) start.  On held-out 16^3 samples the network's
    projected prediction reaches the cold start's steady state in no more
    steps than a start from rest, to within one residual check (20 steps) on
    average.  On a held-out 128^3 sample of the evaluation workload (spheres
    r 4-12) the exact steady fields, put through f_eq and projected, reach it
    in fewer steps than a start from rest (on the 16^3 packings they do not)."""
    net, _, _ = trained
    rng = np.random.default_rng(7)
    cold, warm, errs = [], [], []
    for k in range(4):
        m, _ = inputs.spheres_3d(16, float(rng.uniform(0.4, 0.7)), 2.0, 4.0, seed=900 + k)
        d = rng.normal(size=3)
        sm = warmstart.Sample(torch, m, (1e-6 * d / np.linalg.norm(d)).tolist())
        r = warmstart.evaluate(torch, net, [sm], 0.8, check_every=20)[0]
        print("held-out 16^3 sample %d: cold %d, warm %d steps; prediction error %.3f, agreement %.1e"
              % (k, r["cold_steps"], r["warm_steps"], r["prediction_u_rel_l2"], r["warm_vs_cold_u_rel_l2"]),
              flush=True)
        assert r["warm_steps"] > 0 and not r["fell_back"] and r["warm_vs_cold_u_rel_l2"] <= 1e-4
        cold.append(r["cold_steps"])
        warm.append(r["warm_steps"])
        errs.append(r["prediction_u_rel_l2"])
    print("16^3 mean steps: cold %.0f, warm %.0f; mean prediction error %.3f"
          % (np.mean(cold), np.mean(warm), np.mean(errs)), flush=True)
    assert np.mean(warm) <= np.mean(cold) + 20
    m, _ = inputs.spheres_3d(128, 0.5, 4.0, 12.0, seed=950)
    sm = warmstart.Sample(torch, m, (1e-6, 0.0, 0.0))
    base, pts = warmstart.error_curve(torch, net, sm, 0.8, scales=(0.0, 1.0), check_every=20)
    print("held-out 128^3: cold %d, exact fields %d, network %d steps (prediction error %.3f)"
          % (base["cold_steps"], pts[0]["steps"], pts[1]["steps"], pts[1]["start_u_rel_l2"]), flush=True)
    assert 0 < pts[0]["steps"] < base["cold_steps"]
