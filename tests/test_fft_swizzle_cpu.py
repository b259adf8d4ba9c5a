"""CPU check of the FFT exchange swizzle's bank behaviour (a model of the
LDS, not a GPU run): for every stage of the kernel shapes the tuners use
(radix = P = 4, 8, 16; one to several problems per workgroup; complex and
split exchange), the stage's swizzle sigma = min(lns, bits - log2 RS) maps
the exchange buffer onto itself one to one, and the writes of every group of
lanes the LDS serves together (16 lanes of 8-byte words, 32 of 4-byte words)
fall on distinct banks from N = 256 up (and radix 8 with the complex
exchange from N = 128).  The
plain swizzle (sigma = 0) leaves 2-way conflicts in every radix-8 kernel.

The functions below restate the device formulas (stage_out_pos, swz_cs,
swz_fs in csrc/fft_device.h) for the model."""
import pytest


def stage_out_pos(t, lns, lrs, q):
    return ((t >> lns) << (lns + lrs)) + (t & ((1 << lns) - 1)) + (q << lns)


def swz(p, sigma, bits):
    m = (1 << bits) - 1
    return p ^ ((p >> (bits - sigma)) & ((m << sigma) & m))


def stages(log2n, r):
    lr = r.bit_length() - 1
    rem = log2n % lr
    out, lns = [], 0
    while lns < log2n:
        rs = (1 << rem) if (lns == 0 and rem) else r
        out.append((rs, lns))
        lns += rs.bit_length() - 1
    return out


def conflicts(log2n, r, p, g, split, plain=False):
    n = 1 << log2n
    t_per = n // p
    lanes = t_per * g
    bits, grp = (5, 32) if split else (4, 16)
    extra = 0
    for rs, lns in stages(log2n, r)[:-1]:  # every stage but the last exchanges
        lrs = rs.bit_length() - 1
        sg = 0 if plain else min(lns, bits - lrs)
        seen = set()
        for i in range(p // rs):
            for q in range(rs):
                for g0 in range(0, lanes, grp):
                    banks = []
                    for tx in range(g0, min(g0 + grp, lanes)):
                        w = swz((tx // t_per) * n + stage_out_pos(tx % t_per + i * t_per, lns, lrs, q), sg, bits)
                        seen.add(w)
                        banks.append(w % grp)
                    extra += max(banks.count(b) for b in set(banks)) - 1
        assert seen == set(range(g * n)), "the swizzle must permute the buffer"
    return extra


CASES = [(r, log2n) for r in (4, 8, 16) for log2n in range(7, 15) if not (r == 4 and log2n > 12)]


@pytest.mark.parametrize("r,log2n", CASES)
@pytest.mark.parametrize("split", [False, True])
def test_stage_swizzle_is_conflict_free(r, log2n, split):
    t_per = (1 << log2n) // r
    g = max(1, 256 // t_per)
    if log2n >= 8 or (r == 8 and not split):
        assert conflicts(log2n, r, r, g, split) == 0


def test_plain_swizzle_conflicts_at_radix_8():
    assert conflicts(13, 8, 8, 1, False, plain=True) > 0
    assert conflicts(13, 8, 8, 1, False) == 0
