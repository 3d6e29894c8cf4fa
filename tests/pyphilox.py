"""Pure-Python Philox4x32-10 and the integer variate maps (a third,
independent implementation used only to pin the oracle and the device code).

Philox: Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as
1, 2, 3" (SC 2011)."""

MASK = 0xFFFFFFFF


def philox(ctr, key):
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for _ in range(10):
        p0 = 0xD2511F53 * c0
        p1 = 0xCD9E8D57 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0, p1 & MASK, (p0 >> 32) ^ c3 ^ k1, p0 & MASK)
        k0 = (k0 + 0x9E3779B9) & MASK
        k1 = (k1 + 0xBB67AE85) & MASK
    return (c0, c1, c2, c3)


def below(w, n):
    return (w * n) >> 32


def u53(wa, wb):
    return ((wa >> 5) * 67108864 + (wb >> 6)) / 9007199254740992.0


def threshold(p):
    if p <= 0.0:
        return 0
    if p >= 1.0:
        return 1 << 32
    import math
    return int(math.floor(p * 4294967296.0))


def words(i, gen, n_words, seed, run_id):
    out = []
    for blk in range((n_words + 3) // 4):
        out.extend(philox((i, blk, gen, 3), (seed, run_id)))
    return out[:n_words]
