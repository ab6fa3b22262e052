"""Write ``oracle_rk4_r2_512_f32in.npz``: one RK4 step of a dense 512^3 field,
sampled.

Calls only the CPU oracle and the seeded input generator.  The input is R2
(every retained mode filled) with seed 512, rounded to FP32 and upcast, the
input the FP32 path sees; the oracle runs one classical RK4 step of
Eq. NSfinal (Sec. 2) at nu = 1/1600, dt = 1e-3 (Sec. 4) in FP64.  The whole
output (3.2 GB) is too large to keep, so the fixture holds the output at
8192 seeded retained modes plus the eight corners of the retained box, and
the L2 norm of the whole output.  About 5 minutes and 35 GB of host memory.

    python tests/golden/make_dense512_fixture.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1607_00850_amd import inputs  # noqa: E402

N, SEED, NU, DT, NSAMPLE = 512, 512, 1.0 / 1600.0, 1e-3, 8192


def sample_modes():
    """Canonical indices (ix, iy, iz) of the sampled retained modes."""
    K = (N - 1) // 3
    rng = np.random.default_rng(SEED)
    kx = rng.integers(-K, K + 1, NSAMPLE)
    ky = rng.integers(-K, K + 1, NSAMPLE)
    kz = rng.integers(0, K + 1, NSAMPLE)
    corners = np.array([(sx * K, sy * K, K) for sx in (-1, 1) for sy in (-1, 1)] +
                       [(sx * K, sy * K, 0) for sx in (-1, 1) for sy in (-1, 1)])
    k = np.concatenate([np.stack([kx, ky, kz], -1), corners])
    return k[:, 0] % N, k[:, 1] % N, k[:, 2]


def main():
    u0 = inputs.rough_random(N, SEED).astype(np.complex64).astype(np.complex128)
    u1 = oracle.rk4(u0, NU, DT, 1)
    del u0
    ix, iy, iz = sample_modes()
    np.savez(os.path.join(HERE, "oracle_rk4_r2_512_f32in.npz"), ix=ix.astype(np.int32), iy=iy.astype(np.int32),
             iz=iz.astype(np.int32), values=u1[:, ix, iy, iz], norm=np.linalg.norm(u1), nu=NU, dt=DT, seed=SEED)


if __name__ == "__main__":
    main()
