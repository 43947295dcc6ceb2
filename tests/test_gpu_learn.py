"""The learned cost model on the GPU: its FP32 forward/backward/Adam kernels
against the FP64 NumPy oracle, and the learned plan choice against the plain
policies on a held-out batch (results must stay exact, time must not get
worse)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    from paper_1604_06460_amd import qs
    return qs


def _split(flat):
    shapes = [(24, 64), (64,), (64, 64), (64,), (64, 4), (4,)]
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(flat[o:o + k].reshape(s).astype(np.float64))
        o += k
    return out


def _data(rng, n):
    X = rng.standard_normal((n, 24)).astype(np.float32)
    T = rng.standard_normal((n, 4)).astype(np.float32)
    mask = (rng.random((n, 4)) < 0.7).astype(np.float32)
    mask[:, 0] = 1
    return X, T, mask


def test_forward_loss_and_gradient_vs_fp64_oracle(Q, O):
    rng = np.random.default_rng(3)
    m = Q.Mlp(seed=11)
    p = m.params()
    # nonzero biases so every gradient path is exercised
    p = p + 0.05 * rng.standard_normal(p.size).astype(np.float32)
    m.free()
    m = Q.Mlp(params=p)
    X, T, mask = _data(rng, 777)
    ref = O.MLP(_split(p.astype(np.float64)))
    y = m.forward(X)
    y_ref, _ = ref.forward(X.astype(np.float64))
    assert np.abs(y - y_ref).max() < 1e-4 * max(1.0, np.abs(y_ref).max())
    loss, g = m.loss_grad(X, T, mask)
    l_ref = ref.loss(X.astype(np.float64), T, mask)
    g_ref = np.concatenate([a.reshape(-1) for a in ref.grads(X.astype(np.float64), T, mask)])
    assert abs(loss - l_ref) < 1e-4 * max(1.0, abs(l_ref))
    rel = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    assert rel < 1e-4, rel


def test_adam_six_steps_vs_oracle(Q, O):
    """Six gradient+Adam steps of the GPU kernels against six FP64 oracle
    steps from the same numpy-drawn start, each side on its own trajectory
    (the oracle computes its own gradients). Targets near 100 keep every
    gradient entry a sum of like-signed terms, so FP32 rounding cannot flip
    a step's sign; the bias corrections of steps 2..6 are what is checked."""
    rng = np.random.default_rng(14)
    p0 = np.concatenate([a.reshape(-1) for a in O.MLP.init(21)])
    p0 = (p0 + 0.05 * rng.standard_normal(p0.size)).astype(np.float32)
    m = Q.Mlp(params=p0)
    ref = O.MLP(_split(p0.astype(np.float64)))
    mom = [np.zeros_like(a) for a in ref.p]
    vel = [np.zeros_like(a) for a in ref.p]
    lr = 1e-3
    for t in range(1, 7):
        X, T, mask = _data(rng, 300)
        T = (T + 100.0).astype(np.float32)
        m.loss_grad(X, T, mask)
        m.adam_step(lr)
        g = ref.grads(X.astype(np.float64), T.astype(np.float64), mask.astype(np.float64))
        O.MLP.adam(ref.p, g, mom, vel, t, lr=lr)
        want = np.concatenate([a.reshape(-1) for a in ref.p])
        err = np.abs(m.params().astype(np.float64) - want).max()
        assert err < 2e-6, (t, err)
    m.free()


def test_training_fits_a_smooth_target(Q):
    rng = np.random.default_rng(6)
    X = rng.standard_normal((4000, 24)).astype(np.float32)
    W = rng.standard_normal((24, 4)) * 0.3
    T = (np.tanh(X @ W) + 0.1 * X[:, :4] ** 2).astype(np.float32)
    mask = np.ones_like(T)
    m = Q.Mlp(seed=1)
    l0, _ = m.loss_grad(X, T, mask)
    lf = m.train(X, T, mask, epochs=30, batch=128, lr=3e-3, seed=2)
    assert lf < 0.1 * l0, (l0, lf)


def test_learned_plan_choice_on_held_out_batch(Q, O, S):
    """Train on timings of one batch, choose plans for a disjoint batch of
    the same mix: the learned plans give the oracle's states and run no
    slower than the best plain policy (median of 5 launches each)."""
    from paper_1604_06460_amd import learn
    train = Q.Batch(S.batch_mix(256, S.SEED_BASE * 1000 + 500000, d_range=(10, 40)))
    X, T, mask = learn.collect(train, runs=8, seed=1)
    train.free()
    model, loss = learn.fit(X, T, mask, epochs=60)
    assert np.isfinite(loss)
    circuits = S.batch_mix(512, S.SEED_BASE * 1000 + 7, d_range=(10, 40))
    ev = Q.Batch(circuits)
    res, plans = learn.wall_times(ev, model, repeats=5)
    ratio, best = learn.learned_vs_plain(res)
    stats = model.choose_stats()
    print("wall ms per policy:", res, "learned / best plain (%s) = %.3f, margin %.1f%%; choices %s"
          % (best, ratio, 100 * (1 - ratio), stats))
    assert ratio <= 1.0, (ratio, res)
    # results are exact under the learned plan
    ev.set_plan(plans["learned"])
    ev.run()
    from test_gpu_batch import oracle_circuit
    for c in range(0, len(circuits), 41):
        if circuits[c].n <= 16:
            ref = oracle_circuit(O, S, circuits[c])
            assert np.abs(ev.state(c).astype(np.complex128) - ref).max() < 1e-5
    ev.free()
    model.free()


def test_learned_policy_falls_back_to_the_heuristic(Q, S):
    """Segments whose features lie outside the model's training range, or
    whose predictions are not finite, are planned by the paper's rules
    (the heuristic policy); inside the range the model decides."""
    small = Q.Batch(S.batch_mix(24, 501, n_range=(10, 12), d_range=(4, 8)))
    big = Q.Batch(S.batch_mix(24, 502, n_range=(18, 20), d_range=(4, 8)))
    fs = small.features()
    m = Q.Mlp(seed=3)
    m.set_range(fs.min(0), fs.max(0))
    heur = Q.choose(big, Q.QS_POLICY_HEURISTIC)
    got = Q.choose(big, Q.QS_POLICY_LEARNED, m)
    st = m.choose_stats()
    assert st["fallback_range"] == big.n_segments and st["learned"] == 0, st
    assert np.array_equal(got, heur)
    # inside its own range the model is consulted (learned or margin fallback)
    Q.choose(small, Q.QS_POLICY_LEARNED, m)
    st = m.choose_stats()
    assert st["fallback_range"] == 0 and st["learned"] + st["fallback_margin"] == small.n_segments, st
    # non-finite predictions
    bad = Q.Mlp(params=np.full(Q.QS_MLP_PARAMS, np.nan, dtype=np.float32))
    got = Q.choose(big, Q.QS_POLICY_LEARNED, bad)
    st = bad.choose_stats()
    assert st["fallback_nonfinite"] == big.n_segments, st
    assert np.array_equal(got, heur)
    with pytest.raises(Q.QSError):
        m.set_range(fs.max(0) + 1, fs.min(0))     # lo > hi
    for x in (m, bad, small, big):
        x.free()
