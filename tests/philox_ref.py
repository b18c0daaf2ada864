"""Pure-Python Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), used to check the device generator."""

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform(seed, chain, step):
    """The sampler's coin: counter (chain lo, chain hi, step, 0), key (seed lo,
    seed hi); 53 bits from the first two output words."""
    x = philox4x32_10((chain & MASK, (chain >> 32) & MASK, step & MASK, 0), (seed & MASK, (seed >> 32) & MASK))
    b = (x[0] << 21) | (x[1] >> 11)
    return b * 2.0 ** -53
