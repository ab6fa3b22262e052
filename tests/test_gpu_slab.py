"""z-slab shares of one field (hot_plan_slab / hot_slab_run), every share on
this one GPU with the all-to-all done by device copies (slab.exchange_local).

* Against the oracle: RK4 steps and right-hand sides, FP64 and FP32, with
  the tolerances of the single-field parity tests.
* Against the single-field path: bitwise equal.  Every column and z line is
  transformed by the same kernels with the same arithmetic; only the
  addresses differ.  At 512^3 FP32 over two shares (chunks of 86 retained
  kz at a 128-byte padded pitch of 96) and over eight (chunks of 22, the
  last share holding 17) this covers the blocked z-line loads and stores at
  a realistic size.
* Edge cases: one share (the phases alone), a last share with a single
  retained kz, dealias "none", a 3-smooth N.
* At the benchmark's shape (share 0 of 8 of 2048^3, FP32) one share alone:
  an x-independent band-limited field whose right-hand side the oracle gives
  exactly at 64^3 and whose exchange reduces to the share's own blocks.
"""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import binding, inputs, slab
from hotrun import CDT, fp32_tol, note, rel_l2, round32, run

pytestmark = pytest.mark.gpu

NU = 1.0 / 1600.0
DT = 1e-3


def _torch():
    import torch
    return torch


def run_shares(u, R, op, dtype, nsteps=1, dealias="two_thirds", nu=NU, dt=DT, on_device=False):
    """All R shares of the canonical field u ([3][N][N][N/2+1], numpy or a
    device tensor); returns the assembled canonical result (same kind)."""
    torch = _torch()
    N = u.shape[1]
    plans, lays, wss, ins, outs = [], [], [], [], []
    try:
        for r in range(R):
            h, wsb = binding.hot_plan_slab(N, op, R, r, dtype, dealias, nu, dt)
            plans.append(h)
            lay = binding.hot_slab_layout_of(h)
            lays.append(lay)
            wss.append(torch.zeros(wsb, dtype=torch.uint8, device="cuda"))
            part = u[..., lay.kz0:lay.kz0 + lay.nkz]
            if on_device:
                ins.append(part.contiguous())
            else:
                ins.append(torch.from_numpy(np.ascontiguousarray(part.astype(CDT[dtype]))).cuda())
            outs.append(torch.empty_like(ins[-1]))
        for r in range(R):
            binding.hot_slab_run(plans[r], binding.HOT_SLAB_GATHER, wss[r], inp=ins[r])
        stages = [4] if op == "rhs" else [s for _ in range(nsteps) for s in range(4)]
        for st in stages:
            for r in range(R):
                binding.hot_slab_run(plans[r], binding.HOT_SLAB_INVERSE, wss[r], stage=st)
            slab.exchange_local(wss, lays, forward=True)
            for r in range(R):
                binding.hot_slab_run(plans[r], binding.HOT_SLAB_CROSS, wss[r], stage=st)
            slab.exchange_local(wss, lays, forward=False)
            for r in range(R):
                binding.hot_slab_run(plans[r], binding.HOT_SLAB_FORWARD, wss[r], stage=st)
        for r in range(R):
            binding.hot_slab_run(plans[r], binding.HOT_SLAB_SCATTER, wss[r], out=outs[r])
        res = torch.cat(outs, dim=3)
        torch.cuda.synchronize()
        return res if on_device else res.cpu().numpy()
    finally:
        for h in plans:
            binding.hot_destroy(h)


CASES = [  # N, R, dtype, op, steps
    (32, 2, "f64", "rk4", 1),
    (48, 3, "f64", "rk4", 2),
    (64, 4, "f64", "rhs", 0),
    (64, 8, "f32", "rk4", 1),  # last share: one retained kz
    (54, 2, "f32", "rhs", 0),  # 3-smooth N
    (24, 1, "f64", "rk4", 1),  # one share: the phases alone
]


@pytest.mark.parametrize("N,R,dtype,op,steps", CASES)
def test_shares_match_oracle_and_single_field(N, R, dtype, op, steps):
    print(f"slab N={N} R={R} {dtype} {op} steps={steps}", flush=True)
    u = inputs.rough_random(N, 40 + N)
    got = run_shares(u, R, op, dtype, steps)
    x = round32(u) if dtype == "f32" else u
    ref = oracle.rhs(x, NU) if op == "rhs" else oracle.rk4(x, NU, DT, steps)
    assert rel_l2(got, ref) < (1e-12 if dtype == "f64" else fp32_tol(N))
    assert np.all(got[:, ~oracle.retained_mask(N)] == 0)
    (single,) = run(op, [u], dtype, nu=NU, dt=DT, nsteps=steps)
    assert np.array_equal(got, single)


def test_shares_dealias_none():
    N, R = 32, 4
    u = inputs.rough_random(N, 3, dealias="none")
    got = run_shares(u, R, "rhs", "f64", dealias="none", nu=0.01)
    assert rel_l2(got, oracle.rhs(u, 0.01, dealias="none")) < 1e-12
    (single,) = run("rhs", [u], "f64", dealias="none", nu=0.01)
    assert np.array_equal(got, single)


@pytest.mark.parametrize("R", [2, 8])
def test_shares_512_fp32_equal_the_single_field(R):
    torch = _torch()
    N = 512
    print(f"slab N={N} R={R} f32 rk4", flush=True)
    u = torch.from_numpy(inputs.smooth_random(N, 11).astype(np.complex64)).cuda()
    got = run_shares(u, R, "rk4", "f32", 1, on_device=True)
    h, wsb = binding.hot_plan(N, "rk4", "f32", "two_thirds", NU, DT)
    try:
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        single = torch.empty_like(u)
        binding.hot_run(h, [u], [single], ws, 1)
        torch.cuda.synchronize()
    finally:
        binding.hot_destroy(h)
    del ws
    assert torch.equal(got, single)
    assert float(torch.linalg.vector_norm(single)) > 0


def _x_independent_field(n, band, seed):
    """A real solenoidal field that does not depend on x, band-limited to
    |k_y|, |k_z| <= band, on an n^3 grid: u_x = phi(y, z), (u_y, u_z) =
    (d psi/dz, -d psi/dy) for random trigonometric phi and psi."""
    rng = np.random.default_rng(seed)
    g = 2 * np.pi * np.arange(n) / n
    Y, Z = np.meshgrid(g, g, indexing="ij")
    phi = np.zeros((n, n))
    uy = np.zeros((n, n))
    uz = np.zeros((n, n))
    for my in range(-band, band + 1):
        for mz in range(0, band + 1):
            if my == 0 and mz == 0:
                continue
            a, b, p, q = rng.standard_normal(4)
            arg = my * Y + mz * Z
            phi += a * np.cos(arg + p)
            # psi = b sin(arg + q): u_y = d psi/dz, u_z = -d psi/dy
            uy += b * mz * np.cos(arg + q)
            uz += -b * my * np.cos(arg + q)
    u = np.stack([phi, uy, uz])[:, None, :, :] * np.ones((1, n, 1, 1))
    return u / np.sqrt(np.mean(u * u))


def _share0_rhs_alone(h, lay, ws, x, R):
    """One right-hand side on share 0 alone, for an x-independent field whose
    modes and right-hand side lie in share 0's kz slab: every other share's
    slab is empty going out, and every x-plane's z pass gives the same values
    coming back, so the exchange reduces to share 0's own blocks."""
    torch = _torch()
    y = torch.empty_like(x)
    send = slab._blocks(ws, lay, lay.send_offset, 6)
    recv = slab._blocks(ws, lay, lay.recv_offset, 6)
    binding.hot_slab_run(h, binding.HOT_SLAB_GATHER, ws, inp=x)
    binding.hot_slab_run(h, binding.HOT_SLAB_INVERSE, ws, stage=4)
    recv[:, 0].copy_(send[:, 0])
    binding.hot_slab_run(h, binding.HOT_SLAB_CROSS, ws, stage=4)
    for q in range(R):
        send[:3, q].copy_(recv[:3, 0])
    binding.hot_slab_run(h, binding.HOT_SLAB_FORWARD, ws, stage=4)
    binding.hot_slab_run(h, binding.HOT_SLAB_SCATTER, ws, out=y)
    torch.cuda.synchronize()
    return y


def test_share_0_of_8_at_2048_rhs_fp32_matches_oracle_at_64():
    """One share at the benchmark's shape (2048^3 over 8 shares, share 0,
    FP32), checked alone.  The field does not depend on x and is band-limited
    to |k_y|, |k_z| <= 8, so its right-hand side only has k_x = 0 and
    |k_y|, k_z <= 16: it lies in share 0's kz slab, the oracle at 64^3 gives
    it exactly (alias-free, nothing truncated) up to the (2048/64)^3 scale of
    Eq. ffteq, and the exchange reduces to share 0's own blocks: every other
    share's slab is empty going out, and every x-plane's z pass returns the
    same values coming back."""
    torch = _torch()
    N, R, n = 2048, 8, 64
    print(f"slab share 0 of {R} at N={N} f32 rhs", flush=True)
    u = _x_independent_field(n, 8, 3)
    uh = oracle.forward(u)
    ref = oracle.rhs(round32(uh), NU)
    h, wsb = binding.hot_plan_slab(N, "rhs", R, 0, "f32", "two_thirds", NU, DT)
    try:
        lay = binding.hot_slab_layout_of(h)
        assert lay.kz0 == 0 and lay.nkz > 16
        ws = torch.zeros(wsb, dtype=torch.uint8, device="cuda")
        big = np.where(np.arange(n) <= n // 2, np.arange(n), np.arange(n) - n) % N

        def place(a, scale):
            # the field's modes (rounding noise elsewhere left out)
            nz = np.nonzero(np.abs(a).max(axis=0) > 1e-12 * np.abs(a).max())
            x = torch.zeros((3, N, N, lay.nkz), dtype=torch.complex64, device="cuda")
            idx = [torch.from_numpy(v).long().cuda() for v in (big[nz[0]], big[nz[1]], nz[2])]
            x[:, idx[0], idx[1], idx[2]] = torch.from_numpy(a[:, nz[0], nz[1], nz[2]] * scale).to(torch.complex64).cuda()
            return x, idx

        x, _ = place(uh, (N / n) ** 3)
        y = _share0_rhs_alone(h, lay, ws, x, R)
        del ws, x
        exp, idx = place(ref, (N / n) ** 3)
        assert int(idx[0].numel()) > 100
        err = float(torch.linalg.vector_norm(y - exp) / torch.linalg.vector_norm(exp))
        print(f"rel L2 {err:.3e}", flush=True)
        assert note(err) < fp32_tol(N)
    finally:
        binding.hot_destroy(h)


def test_one_share_plan_runs_whole_with_hot_run():
    """A one-share plan is the single-field plan: hot_run on it (tuned, so
    the fused passes may be chosen) gives the single-field result."""
    torch = _torch()
    N = 48
    u = inputs.rough_random(N, 12)
    x = torch.from_numpy(u.astype(np.complex64)).cuda()
    outs = []
    for slab_plan in (True, False):
        if slab_plan:
            h, wsb = binding.hot_plan_slab(N, "rk4", 1, 0, "f32", "two_thirds", NU, DT)
        else:
            h, wsb = binding.hot_plan(N, "rk4", "f32", "two_thirds", NU, DT)
        try:
            ws = torch.zeros(wsb, dtype=torch.uint8, device="cuda")
            binding.hot_tune(h, ws)
            for name in ("x_inv_curl", "y_inv", "y_fwd", "x_fwd"):
                binding.hot_set_variant(h, name, 1)
            binding.hot_set_variant(h, "x_fwd_rk", -1)
            binding.hot_set_variant(h, "yz_fused", -1)
            y = torch.empty_like(x)
            binding.hot_run(h, [x], [y], ws, 2)
            torch.cuda.synchronize()
            outs.append(y.cpu().numpy())
        finally:
            binding.hot_destroy(h)
    assert np.array_equal(outs[0], outs[1])
    assert rel_l2(outs[0], oracle.rk4(round32(u), NU, DT, 2)) < fp32_tol(N)


def test_share_0_of_8_at_2048_sparse_rhs_fp32_matches_triad_oracle():
    """The same share with an x-independent sparse field whose ky reach the
    retained limit +-682 and whose kz reach 42, so that its right-hand side
    (kz <= 84) stays in share 0's slab of 86 retained kz: the triad-sum
    oracle gives it exactly at 2048^3, and the column tiles at the edges of
    the retained ky range carry data."""
    torch = _torch()
    N, R = 2048, 8
    print(f"slab share 0 of {R} at N={N} f32 rhs, sparse", flush=True)
    ix, iy, iz, vals = inputs.plane_sparse_modes(N, 96, 8, kz_max=42)
    v32 = vals.astype(np.complex64)
    s = inputs.signed_index(N)
    kout, ref = oracle.rhs_triads(np.stack([s[ix], s[iy], iz], -1), v32.astype(np.complex128), N, NU)
    assert np.all(kout[:, 0] == 0) and kout[:, 2].max() <= 84 and np.abs(kout[:, 1]).max() == (N - 1) // 3
    h, wsb = binding.hot_plan_slab(N, "rhs", R, 0, "f32", "two_thirds", NU, DT)
    try:
        lay = binding.hot_slab_layout_of(h)
        assert lay.kz0 == 0 and lay.nkz > 84
        ws = torch.zeros(wsb, dtype=torch.uint8, device="cuda")

        def dense(k, v):
            d = torch.zeros((3, N, N, lay.nkz), dtype=torch.complex64, device="cuda")
            idx = [torch.from_numpy(np.asarray(a)).long().cuda() for a in (k[:, 0] % N, k[:, 1] % N, k[:, 2])]
            d[:, idx[0], idx[1], idx[2]] = torch.from_numpy(v).to(torch.complex64).cuda()
            return d

        x = dense(np.stack([ix, iy, iz], -1), v32)
        y = _share0_rhs_alone(h, lay, ws, x, R)
        del ws, x
        exp = dense(kout, ref)
        err = float(torch.linalg.vector_norm(y - exp) / torch.linalg.vector_norm(exp))
        print(f"rel L2 {err:.3e} over {len(kout)} modes", flush=True)
        assert note(err) < fp32_tol(N)
    finally:
        binding.hot_destroy(h)
