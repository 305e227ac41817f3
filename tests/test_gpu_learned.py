"""The learned initial guess on the GPU: the network's BF16 forward pass,
gradients and Adam step against the FP64 oracle network, training progress,
the fallback of the guess, and the gain over the zero guess.

Tolerances: activations and weights are rounded to BF16 (8 significant
bits, relative error 2^-9 per rounding) before each FP32-accumulated
product, so the forward output and the last layer's gradient agree with
FP64 to a few 1e-3 in relative L2 norm (bound 2e-2).  Each layer the
gradient passes back through adds one BF16 rounding of the propagated
gradient and of the weights, and ReLU masks that differ where a
pre-activation lies within rounding of zero; the bound grows by 1e-2 per
layer traversed (2e-2 + 1e-2 * depth).  Replaying the oracle's layers on
operands rounded to BF16 at the same points reproduces the kernels'
gradients up to FP32 summation order (bound 3e-3), which pins the
remaining FP64 difference on BF16 rounding.  A wrong tap flip, channel
transpose or missing mask gives errors of order one.  Adam runs in FP32:
1e-5 relative to the step.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import nn as onn  # noqa: E402
from paper_2310_14649_amd import binding as B  # noqa: E402
from paper_2310_14649_amd.learned import LearnedGuess, draw_params, init_params  # noqa: E402


def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rl2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _bf16(x):
    """Round to the nearest BF16 (ties to even), as the kernels store operands."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16_replay(params, X, T, env, osc):
    """The oracle's layers evaluated on BF16-rounded operands at the points
    where the kernels round (weights, inputs, activations, propagated
    gradients); everything else in FP64."""
    Pb = [(_bf16(Wt), b) for Wt, b in params]
    acts = [_bf16(X)]
    A = acts[0]
    for l, (Wt, b) in enumerate(Pb):
        Z = onn.conv3x3(A, Wt, b)
        if l + 1 < len(Pb):
            A = _bf16(np.maximum(Z, 0.0))
            acts.append(A)
    E = env[None, :, :, None] * Z - T / osc[None, None, None, :]
    dZ = _bf16(2.0 * env[None, :, :, None] * E / E.size)
    grads = [None] * len(Pb)
    for l in range(len(Pb) - 1, -1, -1):
        dA, dW, db = onn.conv3x3_backward(acts[l], Pb[l][0], dZ)
        grads[l] = (dW, db)
        if l > 0:
            dZ = _bf16(dA * (acts[l] > 0.0))
    return grads


def _setup(channels, H, W, Bn, seed=0):
    rng = np.random.default_rng(seed)
    p = init_params(channels, seed + 1).astype(np.float64)
    # non-zero biases so that every term of the gradient is exercised
    params = onn.unflatten(p, channels)
    params = [(Wt, 0.05 * rng.standard_normal(b.shape)) for Wt, b in params]
    X = rng.standard_normal((Bn, H, W, channels[0]))
    T = rng.standard_normal((Bn, H, W, channels[-1]))
    env = rng.uniform(0.3, 1.0, (H, W))
    osc = rng.uniform(0.5, 2.0, channels[-1])
    return params, X, T, env, osc


@pytest.mark.parametrize("channels,H,W,Bn", [([5, 16, 16, 16, 7], 11, 13, 3),
                                             ([5, 64, 64, 64, 35], 9, 10, 2),
                                             ([3, 24, 40], 17, 5, 4)])
def test_forward_and_gradients_match_oracle(channels, H, W, Bn):
    _cuda()
    params, X, T, env, osc = _setup(channels, H, W, Bn)
    nn = B.nn_create(channels, H, W, Bn)
    try:
        B.nn_set_params(nn, onn.flatten(params))
        B.nn_set_output_map(nn, env, osc)
        Xd = torch.from_numpy(X).cuda()
        Td = torch.from_numpy(T).cuda()
        U = torch.empty((Bn, H * W * channels[-1]), dtype=torch.float64, device="cuda")
        B.nn_forward(nn, Xd, Bn, U)
        U = U.cpu().numpy().reshape(Bn, H, W, channels[-1])
        U_ref = onn.predict(params, X, env, osc)
        assert _rl2(U, U_ref) < 2e-2
        loss = B.nn_loss_grad(nn, Xd, Td, Bn)
        loss_ref, grads_ref = onn.loss_and_grads(params, X, T, env, osc)
        assert abs(loss - loss_ref) / loss_ref < 2e-2
        _, g = B.nn_get_params(nn)
        g_ref = onn.flatten(grads_ref)
        # per layer, weights and biases separately
        q = 0
        L = len(params)
        errs = []
        for l, ((Wr, br), (gWr, gbr)) in enumerate(zip(params, grads_ref)):
            nw, nb = Wr.size, br.size
            ew, eb = _rl2(g[q:q + nw], gWr.ravel()), _rl2(g[q + nw:q + nw + nb], gbr)
            errs.append((ew, eb))
            bound = 2e-2 + 1e-2 * (L - 1 - l)
            assert ew < bound and eb < bound, (l, ew, eb)
            q += nw + nb
        print(f"[learned] gradient rel. L2 per layer (W, b): {errs}", flush=True)
        assert q == g_ref.size
        # the same rounding replayed on the CPU: only FP32 summation order differs
        g_bf = onn.flatten(_bf16_replay(params, X, T, env, osc))
        q = 0
        for (Wr, br), (gWb, gbb) in zip(params, _bf16_replay(params, X, T, env, osc)):
            nw, nb = Wr.size, br.size
            assert _rl2(g[q:q + nw], gWb.ravel()) < 3e-3
            assert _rl2(g[q + nw:q + nw + nb], gbb) < 3e-3
            q += nw + nb
        assert q == g_bf.size
        # Adam with the device gradient against the oracle's update, over
        # three steps with a new gradient each time (other targets), the
        # oracle carrying its moments and step count as the device does
        p0, _ = B.nn_get_params(nn)
        state, ref = {}, onn.unflatten(p0.astype(np.float64), channels)
        rng = np.random.default_rng(9)
        for step in range(3):
            if step:
                B.nn_loss_grad(nn, Xd, torch.from_numpy(rng.standard_normal(T.shape)).cuda(), Bn)
                _, g = B.nn_get_params(nn)
            B.nn_adam_step(nn, 1e-3)
            p1, _ = B.nn_get_params(nn)
            ref = onn.adam_step(ref, onn.unflatten(g.astype(np.float64), channels), state, 1e-3)
            # FP32 master weights: an update of size <= lr per step, rounded to FP32
            assert np.abs(p1 - onn.flatten(ref)).max() <= 1e-5 * 1e-3 + 1e-6 * np.abs(p0).max(), step
        assert state["t"] == 3
    finally:
        B.nn_destroy(nn)


def test_input_fields_and_output_map_match_oracle():
    """nn_input_fields against the oracle's channels; nn_fit_output_map read
    back through a network whose output is one everywhere (last weights
    zero, last bias one), so that U = env (x) oscale in FP32."""
    _cuda()
    rng = np.random.default_rng(5)
    H, W, M, P, Bn = 9, 7, 4, 6, 3
    g0 = 0.1 * rng.standard_normal(H * W)
    g = 0.5 * rng.standard_normal((M, H * W))
    X = torch.empty((H * W, M + 1), dtype=torch.float64, device="cuda")
    B.nn_input_fields(H * W, M, torch.from_numpy(g0).cuda(), torch.from_numpy(g).cuda(), X)
    assert _rl2(X.cpu().numpy(), onn.input_channels(g0, g)) < 1e-15
    channels = [M + 1, 8, P]
    nn = B.nn_create(channels, H, W, Bn)
    try:
        params = onn.unflatten(np.zeros(int(B.nn_param_count(nn))), channels)
        params[-1] = (params[-1][0], np.ones(P))
        B.nn_set_params(nn, onn.flatten(params).astype(np.float32))
        shape = rng.uniform(0.1, 2.0, H * W)
        T = rng.standard_normal((Bn, H * W, P)) * np.arange(1, P + 1)
        B.nn_fit_output_map(nn, torch.from_numpy(shape).cuda(), torch.from_numpy(T).cuda(), Bn)
        U = torch.empty(H * W * P, dtype=torch.float64, device="cuda")
        B.nn_forward(nn, X.view(1, H, W, M + 1), 1, U)
        env, osc = onn.output_map(shape, T)
        ref = env.astype(np.float32).astype(np.float64)[:, None] * \
            osc.astype(np.float32).astype(np.float64)[None, :]
        assert np.allclose(U.cpu().numpy().reshape(H * W, P), ref, rtol=1e-6, atol=0)
    finally:
        B.nn_destroy(nn)


def test_nn_rejects_bad_arguments():
    _cuda()
    with pytest.raises(B.SgError):
        B.nn_create([5, 80, 3], 8, 8, 1)
    nn = B.nn_create([2, 8, 3], 8, 8, 2)
    try:
        X = torch.zeros((3, 8, 8, 2), dtype=torch.float64, device="cuda")
        U = torch.zeros(3 * 8 * 8 * 3, dtype=torch.float64, device="cuda")
        with pytest.raises(B.SgError):       # batch beyond max_batch
            B.nn_forward(nn, X, 3, U)
        with pytest.raises(B.SgError):       # output map not set
            B.nn_forward(nn, X, 1, U)
    finally:
        B.nn_destroy(nn)


@pytest.fixture(scope="module")
def small_model():
    """Config-4 structure on a 32 x 32 grid: 96 training draws, 8 held out."""
    _cuda()
    lg = LearnedGuess("c4", nc=32, max_batch=16, seed=0)
    train = lg.generate(draw_params(96, seed=0))
    lg.fit_output_scale(train)
    losses, _ = lg.train(train, steps=1500, batch=16, lr=2e-3, lr_final=2e-5)
    yield lg, train, losses
    lg.close()


def test_training_reduces_the_loss(small_model):
    lg, train, losses = small_model
    first = np.mean(losses[:5])
    last = np.mean(losses[-10:])
    print(f"[learned] loss {first:.3e} -> {last:.3e}", flush=True)
    assert last < 0.2 * first


def test_guess_falls_back_to_zero_for_a_bad_prediction(small_model):
    lg, train, _ = small_model
    s, e = draw_params(1, seed=7)[0]
    lg.set_draw(s, e)
    N = lg.H * lg.W * lg.P
    bad = torch.full((N,), 50.0, dtype=torch.float64, device="cuda")
    U0 = torch.empty_like(bad)
    choice, rel = B.newton_guess(lg.solver.nl, bad, U0, lg.guess_ws)
    assert choice == 0 and rel[1] > 1.0
    assert float(U0.abs().max()) == 0.0
    # an exact solution is kept (its residual is at the solve tolerance)
    U, info = lg.solver.solve(tol=1e-10)
    choice, rel = B.newton_guess(lg.solver.nl, U, U0, lg.guess_ws)
    assert choice in (1, 2) and min(rel[1], rel[2]) < 1e-9


def test_learned_guess_lowers_the_starting_residual(small_model):
    """What the trained network gains on held-out draws: the starting
    residual ||R(U_0)||/||F|| of the learned guess against the zero guess's 1
    (strictly below 1 on every draw, and on average by at least 10 %), with
    the same converged solution.  Newton steps and Krylov iterations are
    reported beside it; on this mildly nonlinear problem, whose zero-guess
    Newton converges in three steps, the lower start saves at most a few
    Krylov iterations, so those are only bounded (no Newton step more, at
    most one Krylov iteration more on average)."""
    lg, train, _ = small_model
    held = draw_params(8, seed=1)
    its_nn, its_zero, steps_nn, steps_zero, rel = [], [], [], [], []
    for s, e in held:
        U0, i0 = lg.solve(s, e, use_nn=False)
        U1, i1 = lg.solve(s, e, use_nn=True)
        assert i0["converged"] and i1["converged"]
        assert i1["guess_choice"] in (0, 1, 2)
        chosen = [1.0, *i1["guess_relres"][1:]][i1["guess_choice"]]
        assert chosen < 1.0
        rel.append(chosen)
        # both meet ||R||/||F|| <= 1e-8; the iterates agree to the solve tolerance
        assert float(torch.linalg.norm(U1 - U0) / torch.linalg.norm(U0)) < 1e-6
        its_nn.append(i1["krylov_its"])
        its_zero.append(i0["krylov_its"])
        steps_nn.append(i1["steps"])
        steps_zero.append(i0["steps"])
        print(f"[learned] draw s={s:.3f} l={e:.3f}: zero {i0['steps']} steps/{i0['krylov_its']} its,"
              f" nn {i1['steps']} steps/{i1['krylov_its']} its, guess {i1['guess_relres']}",
              flush=True)
    print(f"[learned] mean: zero {np.mean(steps_zero):.2f} steps / {np.mean(its_zero):.2f} its, "
          f"nn {np.mean(steps_nn):.2f} steps / {np.mean(its_nn):.2f} its, "
          f"start residual {np.mean(rel):.3f}", flush=True)
    assert np.mean(rel) < 0.9
    assert np.mean(its_nn) <= np.mean(its_zero) + 1.0
    assert np.mean(steps_nn) <= np.mean(steps_zero)
