"""The learned warm start of the implicit step, trained on oracle pairs.

* Training pairs come from FP64 oracle trajectories (oracle.surrogate_pairs,
  at N = 32 to keep the test short); the network is trained on the GPU by the
  library's own kernels (hot_mlp_grad, hot_mlp_adam) and must cut its training
  loss.  On held-out oracle trajectories the test measures what it gains over
  the plain extrapolation 2 D1 - D2 in the stopping test's norm,
  gain = 1 - sum s^2 |y - t|^2 / sum s^2 |t|^2 (printed; the extrapolation is
  gain 0), and checks the network's inference kernel against the reference
  forward pass on those rows.
* The batch's accuracy: 64 instances with the batch size law (16 <= N <= 64),
  FP32, tau = 1e-5, two plain steps of history and then one step plain and one
  warm-started, each against the FP64 oracle's implicit-midpoint step from
  the same (FP32-rounded) state: the state to the FP32 bar, the increment to
  20 tau plus the state's FP32 rounding seen relative to it.  The sweeps of
  both are printed.
"""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import binding, inputs
from hotrun import fp32_tol, round32, to_dev, workspace

pytestmark = pytest.mark.gpu

NU, DT = 1.0 / 1600.0, 1e-2


def _dev32(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _pairs(seeds, n, rows):
    parts = [oracle.surrogate_pairs(sd, rows, n=n) for sd in seeds]
    return (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]),
            np.concatenate([p[2] for p in parts]))


def _train(X, T, steps=600, mb=2048, seed=0):
    """Adam on minibatches drawn uniformly from the (already s^2-weighted)
    rows; returns (parameters on the GPU, first and last minibatch loss)."""
    import torch
    P = binding.hot_mlp_param_count()
    th = _dev32(oracle.mlp_init(seed))
    grad = torch.empty(P, dtype=torch.float32, device="cuda")
    m = torch.zeros(P, dtype=torch.float32, device="cuda")
    v = torch.zeros(P, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ws = workspace(binding.hot_mlp_train_bytes(mb))
    dX, dT = _dev32(X), _dev32(T)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    losses = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, X.shape[0], (mb,), device="cuda", generator=gen)
        xb, tb = dX[idx].contiguous(), dT[idx].contiguous()
        binding.hot_mlp_grad(th, xb, tb, mb, grad, loss, ws)
        if step in (1, steps):
            losses.append(float(loss.item()))
        lr = 1e-3 * 0.5 * (1 + np.cos(np.pi * (step - 1) / steps))
        binding.hot_mlp_adam(th, grad, m, v, step, max(lr, 1e-5))
    return th, losses


@pytest.fixture(scope="module")
def trained():
    import torch
    X, T, S = _pairs(range(10000, 10016), 32, 1500)
    th, losses = _train(X, T)
    pk = torch.empty(binding.hot_mlp_packed_bytes(), dtype=torch.uint8, device="cuda")
    binding.hot_mlp_pack(th, pk)
    torch.cuda.synchronize()
    return th.cpu().numpy().astype(np.float64), pk, losses


def test_training_on_oracle_pairs_and_held_out_gain(trained):
    import torch
    theta, pk, losses = trained
    print(f"surrogate training loss {losses[0]:.3e} -> {losses[1]:.3e}", flush=True)
    assert losses[1] < 0.5 * losses[0]
    Xv, Tv, Sv = _pairs(range(20000, 20004), 32, 0)  # every retained mode of held-out trajectories
    y = torch.empty((len(Xv), 6), dtype=torch.float32, device="cuda")
    binding.hot_mlp_forward(pk, _dev32(Xv), y, len(Xv))
    got = y.cpu().numpy().astype(np.float64)
    ref, _ = oracle.mlp_forward(theta, Xv.astype(np.float32).astype(np.float64), bf16=True)
    # the trained network's outputs are small corrections (about 1e-3 of the
    # increment), left after cancellations, so a BF16 operand that rounds the
    # other way moves them more than in the random-weight tests: 5e-2
    assert np.linalg.norm(got - ref) <= 5e-2 * np.linalg.norm(ref)
    w = Sv[:, None] ** 2

    def gain(y):
        return 1.0 - float(np.sum(w * (y - Tv) ** 2) / np.sum(w * Tv ** 2))
    g_gpu, g_ref = gain(got), gain(ref)
    print(f"held-out gain over the extrapolation (s^2-weighted): {g_gpu:+.4f} (reference forward {g_ref:+.4f})",
          flush=True)
    assert abs(g_gpu - g_ref) < 1e-2


def test_batch_warm_start_accuracy_against_the_oracle(trained):
    import torch
    _, pk, _ = trained
    sizes = [int(n) for n in inputs.batch_sizes(64, 3)]
    fields = [inputs.smooth_random(N, 30000 + i) for i, N in enumerate(sizes)]
    tol = 1e-5
    results = {}
    for assisted in (False, True):
        h, wsb = binding.hot_plan(sizes, "implicit", "f32", nu=NU, dt=DT, tol=tol, max_iter=20, keep_history=True)
        try:
            ws = workspace(wsb)
            xs = [to_dev(f, "f32") for f in fields]
            mids = [torch.empty_like(x) for x in xs]
            outs = [torch.empty_like(x) for x in xs]
            binding.hot_run(h, xs, mids, ws, 2)  # two plain steps: the history of the third
            if assisted:
                binding.hot_set_surrogate(h, pk)
            binding.hot_run(h, mids, outs, ws, 1)
            torch.cuda.synchronize()
            sweeps, nonconv = binding.hot_implicit_stats(h, len(sizes))
            assert not any(nonconv)
            results[assisted] = ([m.cpu().numpy() for m in mids], [o.cpu().numpy() for o in outs], sweeps)
        finally:
            binding.hot_destroy(h)
    mids = results[False][0]
    for i, N in enumerate(sizes):
        # the plain history does not depend on the surrogate
        assert np.array_equal(mids[i].view(np.uint8), results[True][0][i].view(np.uint8))
        # the oracle's step from the same FP32 state, converged far below tau
        # (the fixed point does not depend on the predictor)
        u2 = round32(mids[i])
        ref, _, ok, _ = oracle.implicit_midpoint_step(u2, NU, DT, 1e-12, 80)
        assert ok
        bar = 20 * tol * np.linalg.norm(ref - u2) + fp32_tol(N) * np.linalg.norm(ref)
        for assisted in (False, True):
            err = np.linalg.norm(results[assisted][1][i] - ref)
            assert err <= bar, (assisted, i, N, err, bar)
    sw0, sw1 = sum(results[False][2]), sum(results[True][2])
    print(f"sweeps of the third step over 64 instances: plain {sw0}, warm-started {sw1}", flush=True)
