"""GPU parity of the surrogate kernels (BF16 matrix-core GEMMs, alignment and
its derivative, training step, fallback step) against the FP64 oracle
(oracle/mlp.py, which rounds GEMM operands to BF16 where the kernels do).

Tolerances: products accumulate in FP32 on the GPU and in FP64 in the
oracle, so a pre-activation differs by ~1e-6 relative; when such a value
sits next to a BF16 rounding boundary the two sides round one activation
to neighbouring BF16 values (0.4 % apart).  Outputs therefore agree to a
few 1e-4 of their scale; the bounds below allow 2e-3 (values) and 1e-2
(gradients, which pass three BF16-rounded backward signals)."""
import numpy as np
import pytest

import workloads as wl
from oracle import mlp as om
from oracle.close import CloseStructure
from oracle.path import landmark_lambda, path_cv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _setup(n=20, hidden=64, seed=1, max_batch=64):
    import paper_1801_02362_amd as pcv
    s = wl.small_path(n, 30, 50 + seed, dtype=np.float32)
    ref = s.landmarks[0].astype(np.float64)
    sizes = wl.mlp_sizes(n, hidden)
    params = wl.mlp_init(sizes, seed)
    sur = pcv.Surrogate(ref, hidden=hidden, max_batch=max_batch, use_graph=False)
    sur.set_params(params)
    W, b = wl.mlp_unflatten(params.astype(np.float64), sizes)
    net = om.MLP(W, b, mean=np.array([12.0, 0.002]), std=np.array([6.0, 0.003]))
    sur.set_scaling(net.mean, net.std)
    return s, ref, sur, net, params, sizes


def _bf16_values(t):
    """Float64 values of a tensor of BF16 bit patterns (int16)."""
    b = t.detach().cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def _frames(s, k, seed, sigma=0.03):
    rng = np.random.default_rng(seed)
    base = s.waypoints[0]
    return (base[None] + rng.normal(0, sigma, (k,) + base.shape)).astype(np.float32)


def test_alignment_matches_oracle(torch):
    from gpu_util import dev, host
    s, ref, sur, net, _, _ = _setup()
    X = _frames(s, 5, 2)
    _, xa = sur.align(dev(X, torch.float32), bf16=False, f32=True)
    xa = host(xa)
    for k in range(5):
        xp, _ = om.align(X[k].astype(np.float64), ref)
        assert np.abs(xa[k] - xp.reshape(-1)).max() < 2e-6
    sur.close()


def test_forward_matches_oracle(torch):
    from gpu_util import dev, host
    s, ref, sur, net, _, _ = _setup(n=40, hidden=128, seed=3)
    X = _frames(s, 33, 4)
    xb, _ = sur.align(dev(X, torch.float32))
    y = host(sur.forward(xb))
    inputs = _bf16_values(xb)
    ref_y = om.forward(net, inputs, rounded=True)["y"]
    scale = np.abs(ref_y).max()
    assert np.abs(y - ref_y).max() <= 2e-3 * scale
    sur.close()


@pytest.mark.parametrize("n,hidden", [(20, 64), (37, 96)])
def test_values_and_gradients_match_oracle(torch, n, hidden):
    from gpu_util import dev, host
    s, ref, sur, net, _, _ = _setup(n=n, hidden=hidden, seed=5)
    X = _frames(s, 4, 6)
    o = sur.eval(dev(X, torch.float32))
    sz, gs, gz = host(o["sz"]), host(o["ds_dx"]), host(o["dz_dx"])
    for k in range(4):
        rs, rz, rgs, rgz = om.surrogate(net, X[k].astype(np.float64), ref, rounded=True)
        assert abs(sz[k, 0] - rs) <= 2e-3 * net.std[0]
        assert abs(sz[k, 1] - rz) <= 2e-3 * net.std[1]
        assert np.abs(gs[k] - rgs).max() <= 1e-2 * np.abs(rgs).max()
        assert np.abs(gz[k] - rgz).max() <= 1e-2 * np.abs(rgz).max()
        # a function of the aligned structure: no net force, no net torque
        xc = X[k] - X[k].mean(0)
        for g in (gs[k], gz[k]):
            assert np.abs(g.sum(0)).max() <= 1e-4 * np.abs(g).max() * n
            assert np.abs(np.cross(xc, g).sum(0)).max() <= 1e-3 * np.abs(g).max() * n
    sur.close()


def test_graph_replay_matches_eager(torch):
    import paper_1801_02362_amd as pcv
    from gpu_util import dev, host
    s, ref, sur, net, params, _ = _setup(n=20, hidden=64, seed=7)
    X = dev(_frames(s, 3, 8), torch.float32)
    eager = sur.eval(X)
    g = pcv.Surrogate(ref, hidden=64, max_batch=64, use_graph=True)
    g.set_params(params)
    g.set_scaling(net.mean, net.std)
    out = {"sz": torch.empty(3, 2, dtype=torch.float64, device="cuda"),
           "ds_dx": torch.empty_like(X), "dz_dx": torch.empty_like(X)}
    for _ in range(3):
        r = g.eval(X, out=out)
        for key in ("sz", "ds_dx", "dz_dx"):
            assert np.array_equal(host(r[key]), host(eager[key]))
    g.close()
    sur.close()


def test_training_step_matches_oracle(torch):
    from gpu_util import dev, host
    s, ref, sur, net, params, sizes = _setup(n=24, hidden=64, seed=9)
    X = _frames(s, 48, 10)
    xb, _ = sur.align(dev(X, torch.float32))
    rng = np.random.default_rng(11)
    T = rng.normal(0, 1, (48, 2)).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    lr = 1e-3
    sur.train_step(xb, dev(T, torch.float32), lr, loss)
    inputs = _bf16_values(xb)
    cache = om.forward(net, inputs, rounded=True)
    ref_loss, dy = om.loss_and_grad(cache["y"], T)
    assert abs(host(loss)[0] - ref_loss) <= 2e-3 * ref_loss
    dW, db = om.param_grads(net, cache, dy, rounded=True)
    gW, gb = wl.mlp_unflatten(sur.grads().astype(np.float64), sizes)
    for l in range(4):
        assert np.abs(gW[l] - dW[l]).max() <= 1e-2 * np.abs(dW[l]).max()
        assert np.abs(gb[l] - db[l]).max() <= 1e-2 * np.abs(db[l]).max() + 1e-7
    # Adam's first step moves each weight by lr * sign(g) where |g| >> eps
    newW, newb = wl.mlp_unflatten(sur.params().astype(np.float64), sizes)
    for l in range(4):
        w1, _, _ = om.adam_step(net.W[l], dW[l], 0.0 * dW[l], 0.0 * dW[l], 1, lr)
        big = np.abs(dW[l]) > 1e-3 * np.abs(dW[l]).max()
        assert np.abs(newW[l][big] - w1[big]).max() <= 1e-6 + 1e-6 * np.abs(w1[big]).max()
    sur.close()


def test_training_reduces_the_loss(torch):
    from gpu_util import dev, host
    s, ref, sur, net, params, sizes = _setup(n=24, hidden=64, seed=12, max_batch=256)
    X = _frames(s, 256, 13, sigma=0.05)
    xb, _ = sur.align(dev(X, torch.float32))
    # a smooth target of the aligned coordinates
    xa = _bf16_values(xb)
    T = np.stack([np.tanh(xa[:, :6].sum(1)), np.cos(xa[:, 6:12].sum(1))], 1).astype(np.float32)
    T = (T - T.mean(0)) / T.std(0)
    Td = dev(T, torch.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    for it in range(300):
        sur.train_step(xb, Td, 3e-3, loss)
        if it % 50 == 0 or it == 299:
            losses.append(float(host(loss)[0]))
    assert losses[-1] < 0.1 * losses[0], losses
    sur.close()


def test_fallback_step_follows_the_drift_test(torch):
    import paper_1801_02362_amd as pcv
    from gpu_util import TOL32, dev, host
    n, L = 20, 30
    s, ref, sur, net, params, _ = _setup(n=n, hidden=64, seed=14)
    lam = landmark_lambda(s.landmarks)
    eps = 0.002
    exact = pcv.PathCV(dev(s.landmarks, torch.float32), lam, eps=eps)
    walk = wl.random_walk(s.waypoints[0].astype(np.float32), 120, rng=np.random.default_rng(15))
    orc = CloseStructure(s.landmarks.astype(np.float64), lam, eps)
    x = torch.empty(n, 3, dtype=torch.float32, device="cuda")
    used_steps = exact_steps = 0
    errs = []
    anchor = None   # exact(y) - f(y) at the last exact step
    for t in range(len(walk)):
        x.copy_(torch.as_tensor(walk[t]))
        o = sur.step(exact, x)
        step = orc.step(walk[t].astype(np.float64))
        used = int(host(o["used"])[0])
        assert used == (0 if step.recomputed else 1), t
        rs, rz, rgs, _ = om.surrogate(net, walk[t].astype(np.float64), ref, rounded=True)
        if used:
            used_steps += 1
            ps = rs + (anchor[0] if anchor is not None else 0.0)
            assert abs(host(o["sz"])[0] - ps) <= 4e-3 * net.std[0]
            assert np.abs(host(o["ds_dx"]) - rgs).max() <= 1e-2 * np.abs(rgs).max()
        else:
            exact_steps += 1
            ref_ex = path_cv(walk[t].astype(np.float64), s.landmarks.astype(np.float64), lam)
            assert abs(host(o["sz"])[0] - ref_ex.s) <= TOL32["sz"]
            if anchor is not None:
                errs.append(abs(rs + anchor[0] - ref_ex.s))
            anchor = (ref_ex.s - rs, ref_ex.z - rz)
    st = sur.stats()
    assert st["steps"] == len(walk)
    assert st["surrogate_steps"] == used_steps and st["exact_steps"] == exact_steps
    assert st["judged_steps"] == len(errs)
    assert exact_steps >= 2 and used_steps >= 1
    assert abs(st["max_abs_ds"] - max(errs)) <= 4e-3 * net.std[0]
    ex = exact.stats()
    assert ex["recomputes"] == exact_steps
    exact.close()
    sur.close()


def test_full_size_network_single_structure(torch):
    """300 atoms, H = 512 (the surrogate's production shape): one structure
    takes the split-K products; it must agree with the oracle and with the
    same structure evaluated inside a 65-row batch (no split)."""
    import paper_1801_02362_amd as pcv
    from gpu_util import dev, host
    n, H = 300, 512
    s = wl.small_path(n, 4, 77, dtype=np.float32)
    ref = s.landmarks[0].astype(np.float64)
    sizes = wl.mlp_sizes(n, H)
    params = wl.mlp_init(sizes, 21)
    W, b = wl.mlp_unflatten(params.astype(np.float64), sizes)
    net = om.MLP(W, b, mean=np.array([250.0, 0.05]), std=np.array([120.0, 0.04]))
    sur = pcv.Surrogate(ref, hidden=H, max_batch=65, use_graph=False)
    sur.set_params(params)
    sur.set_scaling(net.mean, net.std)
    X = _frames(s, 65, 78, sigma=0.05)
    one = sur.eval(dev(X[:1], torch.float32))
    rs, rz, rgs, rgz = om.surrogate(net, X[0].astype(np.float64), ref, rounded=True)
    assert abs(host(one["sz"])[0, 0] - rs) <= 2e-3 * net.std[0]
    assert abs(host(one["sz"])[0, 1] - rz) <= 2e-3 * net.std[1]
    assert np.abs(host(one["ds_dx"])[0] - rgs).max() <= 1e-2 * np.abs(rgs).max()
    assert np.abs(host(one["dz_dx"])[0] - rgz).max() <= 1e-2 * np.abs(rgz).max()
    many = sur.eval(dev(X, torch.float32))
    assert abs(host(many["sz"])[0, 0] - host(one["sz"])[0, 0]) <= 2e-3 * net.std[0]
    assert np.abs(host(many["ds_dx"])[0] - host(one["ds_dx"])[0]).max() <= 1e-2 * np.abs(rgs).max()
    sur.close()


def test_fallback_step_with_replaced_exact_handles(torch):
    """Exact handles destroyed and recreated between fallback steps (their
    host addresses may repeat) while the surrogate replays cached graphs:
    every step must use the live handle's buffers.  Each run starts with an
    exact step (a new handle has no close structure), which resets the
    anchor, so every run equals the same run on a fresh surrogate."""
    import paper_1801_02362_amd as pcv
    from gpu_util import dev, host
    n, hidden = 20, 64
    s, ref, _, net, params, _ = _setup(n=n, hidden=hidden, seed=21)
    lam = landmark_lambda(s.landmarks)
    lm = dev(s.landmarks, torch.float32)
    walk = wl.random_walk(s.waypoints[0].astype(np.float32), 12, rng=np.random.default_rng(22))
    x = torch.empty(n, 3, dtype=torch.float32, device="cuda")

    def surrogate():
        m = pcv.Surrogate(ref, hidden=hidden, max_batch=64, use_graph=True)
        m.set_params(params)
        m.set_scaling(net.mean, net.std)
        return m

    def run(m, eps):
        h = pcv.PathCV(lm, lam, eps=eps)
        out = []
        for f in walk:
            x.copy_(torch.as_tensor(f))
            o = m.step(h, x)
            out.append(np.concatenate([host(o["sz"]), host(o["ds_dx"]).ravel()]))
        h.close()
        return np.array(out)

    shared = surrogate()
    for eps in (0.002, 0.001, 0.002, 0.0005):
        got = run(shared, eps)
        fresh = surrogate()
        want = run(fresh, eps)
        fresh.close()
        assert np.array_equal(got, want), eps
    shared.close()


def test_trained_network_learns_s_on_held_out_frames(torch):
    """What training gains: after minibatch Adam on exact labels (all on the
    GPU), the network's error on frames it never saw is a small fraction of
    the spread of (s, z), where the untrained network (or the label mean)
    is off by the whole spread."""
    import paper_1801_02362_amd as pcv
    from paper_1801_02362_amd import surrogate as sg
    from gpu_util import dev, say
    n, L, hidden = 30, 60, 128
    s = wl.small_path(n, L, 81, dtype=np.float32, n_waypoints=3)
    lam = landmark_lambda(s.landmarks)
    frames = wl.surrogate_training_walks(40, 500, system=s)
    frames = frames[wl.minibatch_order(frames.shape[0], 1)]
    lm = dev(s.landmarks, torch.float32)
    fd = dev(frames, torch.float32)
    labels = sg.exact_labels(lm, lam, fd)
    n_tr = frames.shape[0] - 2000
    mean, sd = sg.standardise(labels[:n_tr])
    targets = ((labels - torch.as_tensor(mean, device="cuda")) / torch.as_tensor(sd, device="cuda")).float().contiguous()
    sur = pcv.Surrogate(s.landmarks[0].astype(np.float64), hidden=hidden, max_batch=1024)
    sur.set_params(wl.mlp_init(wl.mlp_sizes(n, hidden), 2))
    sur.set_scaling(mean, sd)
    inputs = sg.aligned_inputs(sur, fd)
    before = sg.test_loss(sur, inputs[n_tr:], targets[n_tr:])
    hist = sg.train(sur, inputs[:n_tr], targets[:n_tr], epochs=40, batch=512, lr=3e-3, lr_final=3e-4)
    after = sg.test_loss(sur, inputs[n_tr:], targets[n_tr:])
    say(f"[surrogate] held-out loss {before:.3e} -> {after:.3e} (training {hist[0]:.3e} -> {hist[-1]:.3e})")
    assert after < 0.05, after                # the label mean scores 2.0 (one per output)
    assert after < 0.02 * before
    y = torch.cat([sur.forward(inputs[t0:t0 + 1000]).clone() for t0 in range(n_tr, inputs.shape[0], 1000)])
    s_pred = y[:, 0].double() * sd[0] + mean[0]
    err = (s_pred - labels[n_tr:, 0]).abs()
    assert float(err.pow(2).mean().sqrt()) < 0.2 * float(labels[n_tr:, 0].std())
    sur.close()


def test_batched_surrogate_outpaces_the_exact_batch(torch):
    """What the trained network gains in throughput, at the accuracy it
    has: the full-size network (900-512-512-512-2) trained on exact labels of
    random walks on the 300-atom, 500-landmark path, then one batched
    evaluation of 1,024 held-out frames of the same walks against the exact
    batched-walker launch over the same structures.  The surrogate's error
    on those frames is asserted (in distribution; the test walk of the bench
    lies outside the training frames' reach, see the bench's overlap
    report) together with the speed-up."""
    import time
    import paper_1801_02362_amd as pcv
    from paper_1801_02362_amd import surrogate as sg
    from gpu_util import dev, say
    sysm, _ = wl.path_300x500(1)
    lam = landmark_lambda(sysm.landmarks)
    frames = wl.surrogate_training_walks(40, 1000, system=sysm)
    frames = frames[wl.minibatch_order(frames.shape[0], 2)]
    lm = dev(sysm.landmarks, torch.float32)
    fd = dev(frames, torch.float32)
    labels = sg.exact_labels(lm, lam, fd)
    n_tr = frames.shape[0] - 1024
    mean, sd = sg.standardise(labels[:n_tr])
    targets = ((labels - torch.as_tensor(mean, device="cuda")) / torch.as_tensor(sd, device="cuda")).float().contiguous()
    sur = pcv.Surrogate(sysm.landmarks[0].astype(np.float64), hidden=512, max_batch=1024)
    sur.set_params(wl.mlp_init(wl.mlp_sizes(300, 512), 3))
    sur.set_scaling(mean, sd)
    inputs = sg.aligned_inputs(sur, fd)
    sg.train(sur, inputs[:n_tr], targets[:n_tr], epochs=8, batch=1024, lr=2e-3, lr_final=1e-4)
    xb = fd[n_tr:].contiguous()
    ob = sur.eval(xb)
    err = (ob["sz"][:, 0] - labels[n_tr:, 0]).abs()
    rms, spread = float(err.pow(2).mean().sqrt()), float(labels[n_tr:, 0].std())
    say(f"[surrogate] held-out |ds| rms {rms:.3f} max {float(err.max()):.3f} (s spread {spread:.1f})")
    assert rms < 0.1 * spread
    bx = pcv.BatchPathCV([lm] * 1024, [lam] * 1024)
    xall = xb.reshape(1024 * 300, 3)
    sz_ex, _, _ = bx.eval(xall)
    assert float((sz_ex[:, 0] - labels[n_tr:, 0]).abs().max()) < 1e-6
    torch.cuda.synchronize()

    def rate(fn):
        t0 = time.perf_counter()
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        return 10 * 1024 / (time.perf_counter() - t0)

    r_sur = rate(lambda: sur.eval(xb, out=ob))
    r_ex = rate(lambda: bx.eval(xall))
    say(f"[surrogate] batched frames/s: surrogate {r_sur:,.0f}, exact {r_ex:,.0f}")
    assert r_sur > 1.5 * r_ex
    bx.close()
    sur.close()


def test_training_state_checkpoint_resumes_bit_for_bit(torch):
    """pcv_mlp_save_state / pcv_mlp_load_state: train, save, train three
    more steps; load the saved state into a fresh surrogate and take the
    same three steps: parameters, Adam moments (through the next steps) and
    outputs agree bit for bit."""
    import paper_1801_02362_amd as pcv
    from gpu_util import dev, host
    s, ref, sur, net, params, sizes = _setup(n=24, hidden=64, seed=21, max_batch=128)
    X = _frames(s, 128, 22, sigma=0.05)
    xb, _ = sur.align(dev(X, torch.float32))
    rng = np.random.default_rng(23)
    T = dev(rng.normal(0, 1, (128, 2)).astype(np.float32), torch.float32)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for _ in range(4):
        sur.train_step(xb, T, 1e-3, loss)
    blob = sur.save_state()
    for _ in range(3):
        sur.train_step(xb, T, 1e-3, loss)
    want = sur.params()
    y_want = host(sur.forward(xb))
    other = pcv.Surrogate(ref, hidden=64, max_batch=128, use_graph=False)
    other.load_state(blob)
    for _ in range(3):
        other.train_step(xb, T, 1e-3, loss)
    assert np.array_equal(other.params(), want)
    assert np.array_equal(host(other.forward(xb)), y_want)
    with pytest.raises(pcv.PcvError):
        pcv.Surrogate(ref, hidden=96, max_batch=8, use_graph=False).load_state(blob)
    with pytest.raises(pcv.PcvError):
        other.load_state(blob[:-4])
    other.close()
    sur.close()
