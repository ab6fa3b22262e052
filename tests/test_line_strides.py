"""The per-line LDS strides of the FP32 z lines (LPz32 in csrc/impl.hpp) are
the ones the bank model in tests/zline_banks.py picks, and no stride lets two
lines overlap."""
import importlib.util
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1607_00850_amd", "csrc")


def _model():
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("zline_banks", os.path.join(here, "zline_banks.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _table():
    text = open(os.path.join(CSRC, "impl.hpp")).read()
    return {int(n): int(s) for n, s in re.findall(r"struct LPz32<(\d+)> \{ using P = StridedLines<LP<\d+>::P, (\d+)>; \};", text)}


def test_strides_are_the_model_optimum():
    zb = _model()
    table = _table()
    assert sorted(table) == sorted(zb.PLANS)
    for N, (R, rad) in zb.PLANS.items():
        SH = zb.ilog2(rad[0])
        slots = N if SH >= 4 else N + (N >> SH) + 1
        Mz = (N - 1) // 3 + 1
        best = min(range(slots, slots + 48), key=lambda s: (zb.cost(N, R, rad, s, Mz), s))
        assert table[N] == best, N
        assert table[N] >= slots  # lines never overlap
        assert zb.cost(N, R, rad, best, Mz) <= zb.cost(N, R, rad, slots, Mz)


def test_model_degree_counts_bank_conflicts():
    zb = _model()
    # 32 lanes reading consecutive 8-byte slots: conflict-free
    assert zb.degree(list(range(64))) == 1
    # 32 lanes on the same 256-byte stride: every lane on the same two banks
    assert zb.degree([32 * l for l in range(32)] + [None] * 32) == 32
    # inactive lanes do not count
    assert zb.degree([0, 32] + [None] * 62) == 2
