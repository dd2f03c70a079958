"""The learned warm start end to end on small four-roll lattices: steady
states from a batch train the network, the network initialises held-out
lattices, and the fallback rule replaces a bad prediction by the cold run.
Also the settling steps: from the exact steady fields they remove the
transient that an equilibrium-only start excites."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_13072_amd import vflb as V
    from paper_2506_13072_amd import warmstart as W
    from paper_2506_13072_amd.workloads import ensemble_draws
    draws = ensemble_draws(28, seed=4242)
    specs = [dict(side=64, Re=1.0, Wi=min(d["Wi"], 1.0), beta=d["beta"], U0=0.01) for d in draws]
    run = W.cold_runs(V, specs[:24], tol=1e-5)
    ok = [i for i in range(24) if run["status"][i] == V.RUN_CONVERGED]
    assert len(ok) >= 20
    X, T = W.training_set(V, run, specs, ok)
    model = W.ColdModel(specs[:24], run)
    mlp = V.Mlp(max_batch=8192, seed=3, sigma=1.5)
    hist = W.train(mlp, X, T, iters=1500, rows=8192, lr=2e-3, log_every=500)
    return dict(V=V, W=W, specs=specs, run=run, mlp=mlp, hist=hist, model=model, X=X, T=T)


def test_training_fits_the_steady_states(env):
    first, last = env["hist"][0][1], env["hist"][-1][1]
    assert last < 0.02 * first, env["hist"]


def test_trained_network_predicts_the_training_states(env):
    # the library folded the target standardisation into the output layer:
    # the network's raw outputs are the normalised fields themselves
    X, T = env["X"], env["T"]
    y = env["mlp"].forward(X[:4096]).cpu().numpy()
    err = np.linalg.norm(y - T[:4096]) / np.linalg.norm(T[:4096])
    assert err < 0.1, err


def test_warm_start_lowers_the_early_residual(env):
    V, W = env["V"], env["W"]
    res = W.warm_vs_cold(V, env["mlp"], env["specs"][24:], env["model"], tol=1e-5, K0=1000,
                         ref_tol=1e-8)
    better = res["R_warm_K0"] < res["R_cold_K0"]
    assert better.sum() >= 3, (res["R_warm_K0"], res["R_cold_K0"])
    keep = ~res["fallback"]
    assert np.all(res["effective_warm_steps"][keep] == res["warm_steps"][keep])
    fb = res["fallback"]
    assert np.all(res["effective_warm_steps"][fb] == res["abandoned"][fb] + res["cold_steps"][fb])
    # both runs stop at R < 1e-5, so both stand about as far from the tightly
    # converged reference
    assert np.all(res["err_warm"] < 1e-2) and np.all(res["err_cold"] < 1e-2)


def test_bad_prediction_falls_back_to_the_cold_run(env):
    V, W = env["V"], env["W"]
    specs = env["specs"][24:]
    res = W.warm_vs_cold(V, env["mlp"], specs, env["model"], tol=1e-5, K0=1000,
                         u_scale_factor=100.0, ref_tol=1e-6)
    assert np.all(res["fallback"])
    assert np.all(res["abandoned"] == 1000)
    assert np.all(res["effective_warm_steps"] == 1000 + res["cold_steps"])
    for i in range(len(specs)):
        assert not res["warm"].is_active(i)
        assert res["warm_status"][i] == V.RUN_SKIPPED


def test_settling_removes_the_initial_transient(env):
    V, W = env["V"], env["W"]
    specs, run = env["specs"][:4], env["run"]
    fields = [(run["batch"][i].read(V.FIELD_U), run["batch"][i].read(V.FIELD_TAU))
              for i in range(4)]
    r = {}
    for settle in (0, 1000):
        b, _ = W.four_roll_batch(V, specs)
        for i, (u, tau) in enumerate(fields):
            b[i].init_fields(u, tau, None)
            if settle:
                b[i].settle(u, tau, settle, V.SETTLE_U | V.SETTLE_A)
        b.reduce()
        b.step(100)
        r[settle] = b.reduce()[:, 0]
    assert np.all(r[1000] < 0.1 * r[0]), r


# ------------------------------------------------------------ channel
# The Poiseuille half of the warm start: 4 x 128 channels (the flow does not
# depend on x), networks trained on steady states the batched LB generated,
# held-out channels judged at the same final accuracy as their cold runs
# against an FP64 run converged to R < 1e-9.

@pytest.fixture(scope="module")
def channel_env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_13072_amd import vflb as V
    from paper_2506_13072_amd import warmstart as W
    from paper_2506_13072_amd.workloads import ensemble_draws
    draws = ensemble_draws(52, seed=777)
    specs = [dict(side=128, Re=1.0, Wi=d["Wi"], beta=d["beta"], U0=0.01, geometry="channel")
             for d in draws]
    run = W.cold_runs(V, specs[:48], tol=1e-6, storage="f64")
    ok = [i for i in range(48) if run["status"][i] == V.RUN_CONVERGED]
    X, T = W.training_set(V, run, specs, ok)
    model = W.ColdModel(specs[:48], run)
    mlp = V.Mlp(max_batch=8192, seed=5, sigma=1.5)
    W.train(mlp, X, T, iters=4000, rows=8192, lr=2e-3)
    return dict(V=V, W=W, specs=specs, mlp=mlp, model=model, ok=ok)


@pytest.mark.timeout(600)
def test_channel_warm_start_reaches_the_same_accuracy_sooner(channel_env):
    V, W = channel_env["V"], channel_env["W"]
    assert len(channel_env["ok"]) >= 44
    test = channel_env["specs"][48:]
    res = W.warm_vs_cold(V, channel_env["mlp"], test, channel_env["model"], tol=1e-6,
                         storage="f64")
    assert np.all(res["cold_status"] == V.RUN_CONVERGED)
    cold, warm = res["cold_steps"].sum(), res["warm_steps_same_accuracy"].sum()
    print("cold", res["cold_steps"], "warm (same accuracy)", res["warm_steps_same_accuracy"])
    assert warm < 0.8 * cold, (warm, cold)
    # the analytic steady state, the upper bound of any equilibrium-only start
    ref = [(res["ref"][i].read(V.FIELD_U), res["ref"][i].read(V.FIELD_TAU))
           for i in range(len(test))]
    an = W.steps_to_accuracy(V, W.analytic_batch(V, test), ref, res["err_cold"].max(1),
                             [3 * W.step_cap(V, sp) for sp in test])
    assert an.sum() < cold
