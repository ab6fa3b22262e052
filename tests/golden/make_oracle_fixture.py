"""Write the oracle regression fixture ``oracle_rk4_n8.npz``.

Calls only the CPU oracle and the seeded input generator.  The fixture locks
the oracle's output for one small case so that any later change to the
oracle's arithmetic shows up as a test failure.

    python tests/golden/make_oracle_fixture.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1607_00850_amd import inputs  # noqa: E402


def main():
    N, nu, dt, nsteps = 8, 0.01, 0.01, 3
    u0 = inputs.rough_random(N, seed=42)
    u1 = oracle.rk4(u0, nu, dt, nsteps)
    np.savez(os.path.join(HERE, "oracle_rk4_n8.npz"), u0=u0, u1=u1, nu=nu, dt=dt, nsteps=nsteps)


if __name__ == "__main__":
    main()
