"""LDS bank model used to pick the per-line LDS strides of the FP32 z lines
(LPz32 in impl.hpp).

Model: 64 banks of 4 bytes; an 8-byte access by a wave is served 32 lanes at
a time, and a group costs as many cycles as the largest number of distinct
words any bank must deliver.  A z kernel packs 64 / Tl lines into a wave, line
l at l * stride complex slots, and a position p of a line sits at slot
sw(p) = p + (p >> SH) (SH < 4) or p ^ ((p >> SH) & 15) (SH >= 4), SH =
log2 of the first radix.  The cost of a stride is the summed conflict degree
(degree - 1) over the z pass's LDS accesses: every Stockham stage's writes and
reads of five transforms, the Hermitian completion of three, the final put
and the split reads.

    python zline_banks.py      # prints the line_slots cost and the best stride per length
"""


def degree(slots):
    worst = 1
    for g in (0, 32):
        banks = {}
        for a in slots[g:g + 32]:
            if a is None:
                continue
            for w in (2 * a, 2 * a + 1):
                banks.setdefault(w % 64, set()).add(w)
        if banks:
            worst = max(worst, max(len(v) for v in banks.values()))
    return worst


def ilog2(v):
    k = 0
    while (1 << (k + 1)) <= v:
        k += 1
    return k


def slot(p, SH):
    return p ^ ((p >> SH) & 15) if SH >= 4 else p + (p >> SH)


def stage_accesses(N, R, radices):
    """Positions lane j (0 <= j < Tl) writes and reads in each exchange of
    the Stockham engine (one list per register)."""
    Tl = N // R
    Ns = 1
    out = []
    for r in radices:
        last = Ns * r == N
        nb = R // r
        if not last:
            for m in range(nb):
                for q in range(r):
                    out.append([((j + m * Tl) // Ns) * Ns * r + (j + m * Tl) % Ns + q * Ns for j in range(Tl)])
            for s in range(R):
                out.append([j + s * Tl for j in range(Tl)])
        Ns *= r
    return out


def z_accesses(N, R, radices, Mz):
    Tl = N // R
    fft = stage_accesses(N, R, radices)
    KL = -(-Mz // Tl)
    completion = []
    for t in range(KL):
        completion.append([j + t * Tl if j + t * Tl < Mz else None for j in range(Tl)])
        completion.append([(N - (j + t * Tl)) % N if 0 < j + t * Tl < Mz else None for j in range(Tl)])
    reads = [[j + s * Tl for j in range(Tl)] for s in range(R)]
    split = [[(N - (j + s * Tl)) % N for j in range(Tl)] for s in range(R)]
    return 3 * (completion + reads + fft) + 2 * fft + reads + reads + split


def cost(N, R, radices, stride, Mz):
    Tl = N // R
    lpw = max(1, 64 // Tl)
    SH = ilog2(radices[0])
    total = 0
    for acc in z_accesses(N, R, radices, Mz):
        slots = [None if acc[j] is None else l * stride + slot(acc[j], SH) for l in range(lpw) for j in range(Tl)]
        slots += [None] * (64 - len(slots))
        total += degree(slots) - 1
    return total


# (R, radices) of the line plans of impl.hpp
PLANS = {16: (16, [16]), 18: (6, [6, 3]), 24: (12, [4, 6]), 32: (8, [8, 4]), 36: (6, [6, 6]),
         48: (12, [4, 4, 3]), 54: (6, [6, 3, 3]), 64: (8, [8, 8])}

if __name__ == "__main__":
    for N, (R, rad) in PLANS.items():
        SH = ilog2(rad[0])
        slots = N if SH >= 4 else N + (N >> SH) + 1
        Mz = (N - 1) // 3 + 1
        best = min(range(slots, slots + 48), key=lambda s: (cost(N, R, rad, s, Mz), s))
        print(f"N={N:3d} line_slots={slots:3d} cost={cost(N, R, rad, slots, Mz):5d}   "
              f"best stride={best:3d} cost={cost(N, R, rad, best, Mz):5d}")
