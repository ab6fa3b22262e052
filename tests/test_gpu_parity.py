"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (relative L2 over the whole output):
  FP64: 1e-12 for transforms, right-hand sides and single RK4 steps,
        1e-11 after 10 steps.
  FP32: 10 * eps32 * log2(N^3) against the oracle run on the FP32-rounded
        input (upcast to FP64).
Integer/index work (mask, compaction, layouts) is checked exactly: modes
outside the retained set must come back as exact zeros.
"""
import numpy as np
import pytest

import oracle
from paper_1607_00850_amd import inputs
from hotrun import fp32_tol, rel_l2, round32, run

pytestmark = pytest.mark.gpu

NU = 1.0 / 1600.0
DT = 1e-3
DTYPES = ["f64", "f32"]


def tol(dtype, N, f64=1e-12):
    return f64 if dtype == "f64" else fp32_tol(N)


def field(kind, N, seed=0):
    if kind == "tg":
        return inputs.taylor_green(N)
    if kind == "smooth":
        return inputs.smooth_random(N, seed)
    if kind == "rough":
        return inputs.rough_random(N, seed)
    raise ValueError(kind)


def ref_input(x, dtype):
    return round32(x) if dtype == "f32" else x


# -- plain transforms (Eq. ffteq) -------------------------------------------------

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [8, 16, 32, 64, 128])
def test_r2c_matches_oracle(N, dtype):
    print(f"r2c N={N} {dtype}", flush=True)
    u = np.random.default_rng(N).standard_normal((3, N, N, N))
    (got,) = run("r2c", [u], dtype)
    ref = oracle.forward(ref_input(u, dtype))
    assert rel_l2(got, ref) < tol(dtype, N, 1e-13)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [8, 16, 32, 64, 128])
def test_c2r_matches_oracle(N, dtype):
    print(f"c2r N={N} {dtype}", flush=True)
    rng = np.random.default_rng(1000 + N)
    # arbitrary (not Hermitian) coefficients: checks that only the imaginary
    # parts of the kz = 0 and N/2 coefficients are dropped, as numpy does
    uh = rng.standard_normal((3, N, N, N // 2 + 1)) + 1j * rng.standard_normal((3, N, N, N // 2 + 1))
    (got,) = run("c2r", [uh], dtype)
    ref = oracle.inverse(ref_input(uh, dtype), N)
    assert rel_l2(got, ref) < tol(dtype, N, 1e-13)


# -- right-hand side of Eq. NSfinal ---------------------------------------------

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kind", ["tg", "smooth", "rough"])
@pytest.mark.parametrize("N", [8, 16, 32, 64])
def test_rhs_matches_oracle(N, kind, dtype):
    print(f"rhs N={N} {kind} {dtype}", flush=True)
    uh = field(kind, N, seed=N)
    (got,) = run("rhs", [uh], dtype, nu=NU)
    ref = oracle.rhs(ref_input(uh, dtype), NU)
    assert rel_l2(got, ref) < tol(dtype, N)
    M = oracle.retained_mask(N)
    assert np.all(got[:, ~M] == 0)


@pytest.mark.parametrize("dtype", DTYPES)
def test_rhs_projects_input_onto_retained_modes(dtype):
    N = 16
    rng = np.random.default_rng(5)
    uh = rng.standard_normal((3, N, N, N // 2 + 1)) + 1j * rng.standard_normal((3, N, N, N // 2 + 1))
    uh = oracle.forward(oracle.inverse(uh, N))  # a real field with content everywhere
    (got,) = run("rhs", [uh], dtype, nu=0.01)
    ref = oracle.rhs(ref_input(uh, dtype), 0.01)
    assert rel_l2(got, ref) < tol(dtype, N)


def test_rhs_dealias_none():
    N = 16
    uh = inputs.rough_random(N, 3, dealias="none")
    (got,) = run("rhs", [uh], "f64", dealias="none", nu=0.01)
    ref = oracle.rhs(uh, 0.01, dealias="none")
    assert rel_l2(got, ref) < 1e-12
    M = oracle.retained_mask(N, "none")
    assert np.all(got[:, ~M] == 0)


def test_rhs_batch_of_uneven_instances():
    fields = [inputs.rough_random(16, 1), inputs.smooth_random(32, 2), inputs.taylor_green(8),
              inputs.rough_random(64, 4)]
    outs = run("rhs", fields, "f64", nu=0.01)
    for f, g in zip(fields, outs):
        assert rel_l2(g, oracle.rhs(f, 0.01)) < 1e-12


# -- RK4 steps --------------------------------------------------------------------

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [16, 32, 64])
def test_rk4_one_step_matches_oracle(N, dtype):
    print(f"rk4 N={N} {dtype}", flush=True)
    uh = inputs.rough_random(N, 7)
    (got,) = run("rk4", [uh], dtype, nu=NU, dt=DT, nsteps=1)
    ref = oracle.rk4(ref_input(uh, dtype), NU, DT, 1)
    assert rel_l2(got, ref) < tol(dtype, N)


def test_rk4_ten_steps_matches_oracle_fp64():
    N = 32
    uh = inputs.smooth_random(N, 9)
    (got,) = run("rk4", [uh], "f64", nu=0.01, dt=0.01, nsteps=10)
    ref = oracle.rk4(uh, 0.01, 0.01, 10)
    assert rel_l2(got, ref) < 1e-11


@pytest.mark.parametrize("kind", ["tg", "smooth", "rough"])
def test_rk4_ten_steps_at_64_fp64(kind):
    """The smallest configuration as the benchmark defines it: 64^3 FP64 at
    the paper's Re = 1600 and dt = 1e-3 (Sec. 4), Taylor-Green and the two
    random families, parity after 1 and after 10 steps."""
    N = 64
    print(f"rk4 10 steps N={N} {kind}", flush=True)
    uh = field(kind, N, seed=0)
    (one,) = run("rk4", [uh], "f64", nu=NU, dt=DT, nsteps=1)
    (ten,) = run("rk4", [uh], "f64", nu=NU, dt=DT, nsteps=10)
    ref1 = oracle.rk4(uh, NU, DT, 1)
    assert rel_l2(one, ref1) < 1e-12
    assert rel_l2(ten, oracle.rk4(ref1, NU, DT, 9)) < 1e-11


def test_rk4_one_step_at_128_fp64():
    """The paper's smallest whole mesh, 128^3 (Sec. 4), one FP64 RK4 step."""
    N = 128
    print(f"rk4 N={N} f64", flush=True)
    uh = inputs.smooth_random(N, 1)
    (got,) = run("rk4", [uh], "f64", nu=NU, dt=DT, nsteps=1)
    assert rel_l2(got, oracle.rk4(uh, NU, DT, 1)) < 1e-12


def test_rk4_in_place_and_zero_steps():
    N = 16
    uh = inputs.rough_random(N, 8, dealias="none")  # content outside the 2/3 set
    (same,) = run("rk4", [uh], "f64", nu=NU, dt=DT, nsteps=0)
    np.testing.assert_array_equal(same, uh * oracle.retained_mask(N))
    (got,) = run("rk4", [uh], "f64", nu=NU, dt=DT, nsteps=2, inplace=True)
    assert rel_l2(got, oracle.rk4(uh, NU, DT, 2)) < 1e-12


@pytest.mark.parametrize("dtype,N", [("f64", 64), ("f32", 128)])
def test_rk4_beltrami_exact_decay(dtype, N):
    K2, nu, dt, n = 9, 0.05, 0.01, 10
    assert nu * dt * 3 * ((N - 1) // 3) ** 2 < 2.78  # RK4 stable at the largest mode
    u0 = inputs.beltrami(N, K2, seed=1)
    (got,) = run("rk4", [u0], dtype, nu=nu, dt=dt, nsteps=n)
    z = -nu * K2 * dt
    R = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
    assert rel_l2(got, R**n * ref_input(u0, dtype)) < tol(dtype, N, 1e-12)


def test_runs_are_bitwise_deterministic():
    uh = inputs.rough_random(32, 11)
    a = run("rk4", [uh], "f32", nu=NU, dt=DT, nsteps=2)[0]
    b = run("rk4", [uh], "f32", nu=NU, dt=DT, nsteps=2)[0]
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("dtype,N", [("f64", 128), ("f32", 256)])
def test_rhs_with_padded_rows_matches_oracle(dtype, N):
    # sizes whose compact z rows are padded to whole 128-byte segments
    print(f"rhs padded N={N} {dtype}", flush=True)
    uh = inputs.smooth_random(N, 3)
    (got,) = run("rhs", [uh], dtype, nu=NU)
    ref = oracle.rhs(ref_input(uh, dtype), NU)
    assert rel_l2(got, ref) < tol(dtype, N)


def test_rk4_beltrami_exact_decay_padded_fp32():
    # nu dt |k|^2 stays inside RK4's stability interval at the largest mode
    N, K2, nu, dt, n = 256, 400, 0.005, 0.01, 3
    assert nu * dt * 3 * 85**2 < 2.78
    u0 = inputs.beltrami(N, K2, seed=2)
    (got,) = run("rk4", [u0], "f32", nu=nu, dt=dt, nsteps=n)
    z = -nu * K2 * dt
    R = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
    assert rel_l2(got, R**n * round32(u0)) < fp32_tol(N)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [18, 24, 36, 48, 54])
def test_radix3_sizes_match_oracle(N, dtype):
    # 2^a 3^b lengths (radix-3 and radix-6 stages); for N = 18, 36, 54 the 2/3
    # rule's strict inequality decides the edge mode (3K < N)
    print(f"radix3 N={N} {dtype}", flush=True)
    rng = np.random.default_rng(N)
    u = rng.standard_normal((3, N, N, N))
    (got,) = run("r2c", [u], dtype)
    assert rel_l2(got, oracle.forward(ref_input(u, dtype))) < tol(dtype, N, 1e-13)
    uh = rng.standard_normal((3, N, N, N // 2 + 1)) + 1j * rng.standard_normal((3, N, N, N // 2 + 1))
    (got,) = run("c2r", [uh], dtype)
    assert rel_l2(got, oracle.inverse(ref_input(uh, dtype), N)) < tol(dtype, N, 1e-13)
    uh = inputs.rough_random(N, N)
    (got,) = run("rhs", [uh], dtype, nu=NU)
    assert rel_l2(got, oracle.rhs(ref_input(uh, dtype), NU)) < tol(dtype, N)
    (got,) = run("rk4", [uh], dtype, nu=NU, dt=DT, nsteps=1)
    assert rel_l2(got, oracle.rk4(ref_input(uh, dtype), NU, DT, 1)) < tol(dtype, N)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [16, 64])
def test_row_forms_drop_the_imaginary_part_at_kz0(N, dtype):
    # a kz = 0 plane that is not Hermitian: the real inverse transform along z
    # (Eq. ffteq with a real field) uses only the real part of each (x, y)
    # line's k = 0 coefficient, as numpy's irfftn does in the oracle: each
    # row form of the y and z passes, and the fused y-z pass, must drop the
    # imaginary part there.
    print(f"kz0 plane N={N} {dtype}", flush=True)
    uh = inputs.rough_random(N, 400 + N)
    rng = np.random.default_rng(N)
    M = oracle.retained_mask(N)
    pert = (rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))) * np.abs(uh).max()
    uh[:, :, :, 0] += np.where(M[:, :, 0], pert, 0)
    ref = oracle.rhs(ref_input(uh, dtype), NU)
    for v in ({"z_cross": 1}, {"z_cross": 2}, {"z_cross": 0}, {"z_cross": 3}, {"z_cross": 1, "y_fwd": 4},
              {"yz_fused": 0}):
        (got,) = run("rhs", [uh], dtype, nu=NU, variants=v)
        assert rel_l2(got, ref) < tol(dtype, N), v


@pytest.mark.parametrize("dtype", DTYPES)
def test_x_inverse_with_six_blocks_per_tile(dtype):
    # x_inv_curl variants 3..5 (N > 64): one output per block instead of two
    N = 128
    print(f"x_inv_curl six blocks {dtype}", flush=True)
    uh = inputs.rough_random(N, 600)
    ref = oracle.rhs(ref_input(uh, dtype), NU)
    (a,) = run("rhs", [uh], dtype, nu=NU, variants={"x_inv_curl": 1})
    for v in (3, 4, 5):
        (b,) = run("rhs", [uh], dtype, nu=NU, variants={"x_inv_curl": v})
        assert rel_l2(b, ref) < tol(dtype, N), v
        assert rel_l2(b, a) < (1e-14 if dtype == "f64" else 1e-6), v  # the same arithmetic up to contraction


# -- the x pass fused with the stage update (x_fwd_rk) -----------------------------

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N,fused", [(16, 1), (32, 0), (64, 1), (24, 1), (128, 0)])
def test_rk4_with_fused_x_pass_matches_oracle(N, fused, dtype):
    print(f"rk4 fused={fused} N={N} {dtype}", flush=True)
    uh = inputs.rough_random(N, 70 + N)
    (got,) = run("rk4", [uh], dtype, nu=NU, dt=DT, nsteps=2, variants={"x_fwd_rk": fused})
    ref = oracle.rk4(ref_input(uh, dtype), NU, DT, 2)
    assert rel_l2(got, ref) < tol(dtype, N)
    M = oracle.retained_mask(N)
    assert np.all(got[:, ~M] == 0)


@pytest.mark.parametrize("dtype", DTYPES)
def test_rhs_with_fused_x_pass_matches_oracle(dtype):
    N = 48
    uh = inputs.smooth_random(N, 5)
    (got,) = run("rhs", [uh], dtype, nu=NU, variants={"x_fwd_rk": 1})
    assert rel_l2(got, oracle.rhs(ref_input(uh, dtype), NU)) < tol(dtype, N)


def test_fused_and_separate_x_pass_agree_on_a_batch():
    fields = [inputs.rough_random(16, 1), inputs.smooth_random(32, 2), inputs.rough_random(24, 4)]
    a = run("rk4", fields, "f32", nu=NU, dt=DT, nsteps=1, variants={"x_fwd_rk": -1})
    b = run("rk4", fields, "f32", nu=NU, dt=DT, nsteps=1, variants={"x_fwd_rk": 1})
    for x, y, f in zip(a, b, fields):
        assert rel_l2(y, x) < 1e-6
        assert rel_l2(y, oracle.rk4(round32(f), NU, DT, 1)) < fp32_tol(f.shape[1])


# -- the y and z passes on packed pair rows against six component rows -----------

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [16, 24, 64, 128])
def test_packed_and_component_rows_agree(N, dtype):
    # variant 1 (default): u and w travel as packed pairs of complex lines;
    # variant 0: six component rows, the z pass building the Hermitian halves
    print(f"packed rows N={N} {dtype}", flush=True)
    uh = inputs.rough_random(N, 90 + N)
    (a,) = run("rk4", [uh], dtype, nu=NU, dt=DT, nsteps=1, variants={"z_cross": 1})
    (b,) = run("rk4", [uh], dtype, nu=NU, dt=DT, nsteps=1, variants={"z_cross": 0})
    # the packed y forward pass with one output per block (variant 4)
    (c,) = run("rk4", [uh], dtype, nu=NU, dt=DT, nsteps=1, variants={"z_cross": 1, "y_fwd": 4})
    # packed rows into the z pass, c0 c1 c2 component rows out of it (variant 2)
    (d,) = run("rk4", [uh], dtype, nu=NU, dt=DT, nsteps=1, variants={"z_cross": 2})
    # component rows through the y passes, packed by the z pass on load (variant 3)
    (e,) = run("rk4", [uh], dtype, nu=NU, dt=DT, nsteps=1, variants={"z_cross": 3})
    ref = oracle.rk4(ref_input(uh, dtype), NU, DT, 1)
    for x in (a, b, c, d, e):
        assert rel_l2(x, ref) < tol(dtype, N)
        assert rel_l2(a, x) < tol(dtype, N)
    M = oracle.retained_mask(N)
    for x in (a, b, c, d, e):
        assert np.all(x[:, ~M] == 0)
