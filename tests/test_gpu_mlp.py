"""GPU parity of the predictor's HIP kernels against the FP64 reference MLP
(oracle/mlp.py): forward logits, softmax, loss, every layer's gradients and
the Adam update, at FP32 tolerances."""
import numpy as np
import pytest

from oracle import mlp as ref
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

hdc = pytest.importorskip("paper_2306_10016_amd")


def _setup(sizes, B, seed):
    import torch
    from paper_2306_10016_amd.mlp import MLP, he_init
    params = he_init(sizes, seed)
    r = synth.rng(500, seed, 0)
    params = [(W, r.normal(0, 0.1, b.shape)) for W, b in params]
    X = r.normal(0, 1, (B, sizes[0]))
    y = r.integers(0, sizes[-1], B)
    net = MLP(sizes, params=params)
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    yt = torch.tensor(y, dtype=torch.int32, device="cuda")
    # the reference sees the float32-rounded inputs and weights
    params64 = [(W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)) for W, b in params]
    return net, Xt, yt, params64, X.astype(np.float32).astype(np.float64), y


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("sizes,B", [([11, 128, 128, 128, 16], 300), ([5, 7, 7, 7, 3], 17), ([11, 128, 128, 128, 16], 1)])
def test_forward_loss_gradients(sizes, B):
    import torch
    say(f"mlp sizes={sizes} B={B}")
    net, Xt, yt, params64, X64, y = _setup(sizes, B, seed=B)
    Z, _ = net.forward(Xt)
    _, z_ref = ref.forward(params64, X64)
    assert _rel(Z.cpu().numpy(), z_ref) < 1e-5
    P = net.probs(Xt).cpu().numpy()
    assert np.allclose(P.sum(1), 1.0, atol=1e-5)
    assert _rel(P, ref.softmax(z_ref)) < 1e-5
    loss, grads = net.gradients(Xt, yt)
    g_ref, l_ref = ref.backward(params64, X64, y)
    assert abs(float(loss) - l_ref) <= 1e-5 * max(1.0, abs(l_ref))
    for li, ((dW, db), (rW, rb)) in enumerate(zip(grads, g_ref)):
        assert _rel(dW.cpu().numpy(), rW) < 1e-4, li
        assert _rel(db.cpu().numpy(), rb) < 1e-4, li


def test_adam_step_matches_reference():
    net, Xt, yt, params64, X64, y = _setup([6, 16, 16, 16, 4], 32, seed=3)
    m = ref.zeros_like(params64)
    v = ref.zeros_like(params64)
    p = params64
    for t in range(1, 4):
        _, grads = net.gradients(Xt, yt)
        g_host = [(dW.cpu().numpy().astype(np.float64), db.cpu().numpy().astype(np.float64)) for dW, db in grads]
        net.adam(grads, lr=1e-2)
        p, m, v = ref.adam_step(p, g_host, m, v, t, lr=1e-2)
        for (W, b), (rW, rb) in zip(net.host_params(), p):
            assert _rel(W, rW) < 1e-5 and _rel(b, rb) < 1e-5


def test_training_learns_a_separable_rule():
    from paper_2306_10016_amd.mlp import MLP
    r = synth.rng(501, 0, 0)
    X = r.normal(0, 1, (2000, 11)).astype(np.float32)
    A = r.normal(0, 1, (11, 6))
    y = np.argmax(X @ A, axis=1).astype(np.int32)
    net = MLP([11, 128, 128, 128, 6], seed=1)
    hist = net.train(X, y, epochs=40, batch=128, lr=2e-3)
    acc = float(np.mean(np.argmax(net.predict_proba(X), 1) == y))
    say(f"mlp toy: loss {hist[0]:.3f} -> {hist[-1]:.3f}, accuracy {acc:.3f}")
    assert hist[-1] < 0.3 * hist[0] and acc > 0.9


def test_soft_targets_match_reference():
    import torch
    net, Xt, yt, params64, X64, y = _setup([11, 32, 32, 32, 16], 64, seed=7)
    r = synth.rng(502, 0, 0)
    T = r.random((64, 16))
    T /= T.sum(1, keepdims=True)
    Tt = torch.tensor(T, dtype=torch.float32, device="cuda")
    loss, grads = net.gradients(Xt, T=Tt)
    g_ref, l_ref = ref.backward(params64, X64, T=T.astype(np.float32).astype(np.float64))
    assert abs(float(loss) - l_ref) <= 1e-5 * max(1.0, abs(l_ref))
    for (dW, db), (rW, rb) in zip(grads, g_ref):
        assert _rel(dW.cpu().numpy(), rW) < 1e-4 and _rel(db.cpu().numpy(), rb) < 1e-4


def test_trained_predictor_gains_over_the_default_on_a_known_cost_model():
    """What the trained network adds to the method without it (p = 1, all residues),
    on a synthetic separable cost model whose optimum is known: an axis of length L
    costs q (m log2(2m) (1.6 if m > 2048) + 2e4), 1.25 times more with D < q, so the
    best m is the next power of two up to L = 2048 and 2048 beyond.  The network is
    tuned and trained exactly as the predictor pipeline does on hardware timings (the
    training problems of at most 2^20 elements, soft targets, the HIP training
    kernels).  On 65 held-out problems inside the training range (1D lengths it has
    not seen, long rectangles and long 3D bars) its top-1 choice must be within 3 % of
    the exhaustive optimum on average and within 10 % on at least 90 % of them, where
    the default is about 34 % off on average (the misses sit at class boundaries,
    where two scale-free classes give different m for lengths between training sizes).
    The 2D/3D evaluation problems lie outside that range (no training problem has two
    axes above 1024): their top-1 and verified top-2 regrets are reported, not asserted."""
    import itertools
    import math
    from paper_2306_10016_amd import predict

    def axis_cost(L, M, m, D):
        q = -(-M // m)
        c = q * (m * math.log2(2 * m) * (1.6 if m > 2048 else 1.0) + 2.0e4)
        return c * (1.25 if D < q else 1.0)

    def timer(Ls, Ms, ms, Ds, dtype, batch=1):
        tot = 0.0
        for a in range(len(Ls)):
            w = float(np.prod([Ls[b] for b in range(len(Ls)) if b != a])) if len(Ls) > 1 else 1.0
            tot += w * axis_cost(Ls[a], Ms[a], ms[a], Ds[a])
        return tot * batch * 1e-6

    def t_of(Ls, Ms, params, dt):
        return timer(Ls, Ms, [p[0] for p in params], [p[1] for p in params], dt)

    train = predict.training_problems()
    X, T = [], []
    for Ls, batch, dt in train:
        Ms = [2 * L - 1 for L in Ls]
        _, tables, _ = predict.tune_separable(Ls, Ms, dt, timer, batch)
        for a in range(len(Ls)):
            X.append(predict.features(Ls, a, dt, batch))
            T.append(predict.soft_target(Ls[a], Ms[a], tables[a], outer=a < len(Ls) - 1))
    pred = predict.Predictor(seed=0)
    hist = pred.fit(np.stack(X), np.stack(T), epochs=300)
    say(f"predictor on the cost model: loss {hist[0]:.3f} -> {hist[-1]:.3f}")

    seen = {(tuple(Ls), dt) for Ls, _, dt in train}
    r = synth.rng(503, 0, 0)
    held = [([int(L)], "c64") for L in r.choice(predict.smooth_sides(2500, 1 << 20), 40, replace=False)
            if ((int(L),), "c64") not in seen]
    for L in (3000, 5000, 6000, 7000, 10000, 12000, 15000):
        held += [([L, 32], "c64"), ([32, L], "c64"), ([L, 16], "c128")]
    for L in (3000, 3500, 4000):
        held += [([16, 16, L], "c64"), ([L, 16, 16], "c64")]
    r_pred, r_def = [], []
    for Ls, dt in held:
        Ms = [2 * L - 1 for L in Ls]
        _, _, t_best = predict.tune_separable(Ls, Ms, dt, timer)  # separable cost: the joint optimum
        r_pred.append(t_of(Ls, Ms, pred.predict_axes(Ls, Ms, dt)[0], dt) / t_best - 1)
        r_def.append(t_of(Ls, Ms, predict.default_params(Ls, Ms), dt) / t_best - 1)
    say(f"  {len(held)} held-out problems: top-1 regret mean {np.mean(r_pred):.4f} max {max(r_pred):.4f}; "
        f"default mean {np.mean(r_def):.4f} max {max(r_def):.4f}")
    worst = sorted(zip(r_pred, [h[0] for h in held], r_def), reverse=True)[:3]
    say(f"  worst top-1: {[(round(a, 3), b, round(c, 3)) for a, b, c in worst]} (regret, L, default regret)")
    assert len(held) >= 60
    assert np.mean(r_pred) <= 0.03 and np.mean(np.asarray(r_pred) <= 0.10) >= 0.9
    assert np.mean(r_def) - np.mean(r_pred) >= 0.2

    for Ls, dt in predict.EVAL_PROBLEMS:
        Ms = [2 * L - 1 for L in Ls]
        joint = predict.tune_joint(Ls, Ms, dt, timer)
        params, conf, _ = pred.predict_axes(Ls, Ms, dt)
        combos = list(itertools.product(*pred.shortlist(Ls, Ms, dt, k=2)))
        verified = min(combos, key=lambda c: t_of(Ls, Ms, c, dt))
        say(f"  {Ls} (outside the training range): top-1 {params} regret "
            f"{t_of(Ls, Ms, params, dt) / joint[0][1] - 1:.3f}; top-2 verified regret "
            f"{t_of(Ls, Ms, verified, dt) / joint[0][1] - 1:.3f} in {len(combos)} timings (joint {len(joint)}); "
            f"default regret {t_of(Ls, Ms, predict.default_params(Ls, Ms), dt) / joint[0][1] - 1:.3f}")
