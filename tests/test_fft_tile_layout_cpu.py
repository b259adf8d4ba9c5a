"""CPU check of the large-N FFT tile layout in LDS (a model of the LDS, not a
GPU run).  For every tile shape the two-pass kernels instantiate with a
column of at least 64 threads (T = len / R >= 64), the layout

    slot(c, e) = swz_c(c * len + (e ^ px(c))),   px(c) = c * max(1, 16 / TC) mod 16

* maps the tile's TC * len values one to one onto TC * len slots;
* puts the 16 lanes that the LDS serves together (8-byte words) on 16
  distinct banks for the row accesses (lane l on column l mod TC, row
  e0 + l div TC), and for the column reads of 64 consecutive threads;
* has the offset form the kernels use: slot(c, e + k) equals
  (swz_c(c * len + (e ^ px(c))) ^ ((k >> 4) & 15)) + k for e < 2^m and k a
  multiple of 2^m, m >= 6, and the last stage's writes (thread index XORed
  with px) land where the column reads expect them.

The formulas restate TileLayout in csrc/fft_large.hip and swz_c in
csrc/fft_device.h for the model.  The padded layout the kernels used before
(c * (len + 1) + e, swizzled) is checked to conflict, as the counters showed.
"""
import random

import pytest


def swz_c(p):
    return p ^ ((p >> 4) & 15)


def px(c, tc):
    return (c * (16 // tc if tc < 16 else 1)) & 15


def slot(c, e, ln, tc):
    return swz_c(c * ln + (e ^ px(c, tc)))


def slot_k(c, e, k, ln, tc):
    return (swz_c(c * ln + (e ^ px(c, tc))) ^ ((k >> 4) & 15)) + k


# (radix, log2 len, tile width): the shapes with T >= 64 that fit the tile
# kernels' limits (at most 1024 threads, TC * len values in 160 KiB)
SHAPES = [(r, ll, tc) for r in (8, 16) for ll in range(9, 14) for tc in (2, 4, 8, 16, 32, 64)
          if (1 << ll) // r >= 64 and tc * (1 << ll) // r <= 1024 and tc * (1 << ll) * 8 <= 160 * 1024]


def extra_cycles(words):
    """Extra LDS cycles of one 64-lane access: per group of 16 lanes, the
    largest number of lanes on one bank (word mod 16), minus one."""
    extra = 0
    for g in range(0, 64, 16):
        banks = [w % 16 for w in words[g:g + 16]]
        extra += max(banks.count(b) for b in set(banks)) - 1
    return extra


@pytest.mark.parametrize("r,ll,tc", SHAPES)
def test_tile_layout_is_a_permutation(r, ll, tc):
    ln = 1 << ll
    slots = {slot(c, e, ln, tc) for c in range(tc) for e in range(ln)}
    assert slots == set(range(tc * ln))


@pytest.mark.parametrize("r,ll,tc", SHAPES)
def test_tile_row_and_column_accesses_are_conflict_free(r, ll, tc):
    ln, t = 1 << ll, (1 << ll) // r
    rows_per_wave = 64 // tc if tc <= 64 else 1
    for e0 in range(0, min(ln, 1024), rows_per_wave):
        words = [slot(l % tc, e0 + l // tc, ln, tc) for l in range(64)]
        assert extra_cycles(words) == 0, e0
    for c in range(tc):
        for j in range(r):
            for w in range(t // 64):
                words = [slot(c, w * 64 + l + j * t, ln, tc) for l in range(64)]
                assert extra_cycles(words) == 0


def test_padded_layout_conflicts():
    ln, tc = 4096, 4
    words = [swz_c((l % tc) * (ln + 1) + l // tc) for l in range(64)]
    assert extra_cycles(words) > 0


@pytest.mark.parametrize("r,ll,tc", SHAPES)
def test_tile_slot_offset_form(r, ll, tc):
    ln, t = 1 << ll, (1 << ll) // r
    nt = t * tc
    rng = random.Random(ll * 100 + tc)
    for c in rng.sample(range(tc), min(tc, 6)):
        # column reads: e = tid < T, k = j T; the tile's loads: the same with
        # e = thread div TC; pass A's row stores: e = thread < NT, k = r NT
        for e, step, count in ((rng.randrange(t), t, r), (rng.randrange(nt), nt, max(1, ln // nt))):
            for j in range(count):
                k = j * step
                assert slot_k(c, e, k, ln, tc) == slot(c, e + k, ln, tc)
        # the last stage writes output position tid + q T through the thread
        # index XORed with px: the same slot as slot(c, tid + q T)
        tid = rng.randrange(t)
        base = swz_c(c * ln + (tid ^ px(c, tc)))
        for q in range(r):
            assert (base ^ (((q * t) >> 4) & 15)) + q * t == slot(c, tid + q * t, ln, tc)


def tile_order(b, tc):
    lg = 16 // tc if tc < 16 else 1
    x, w = b & 7, b >> 3
    return (w // lg) * (8 * lg) + lg * x + (w % lg)


@pytest.mark.parametrize("tc", [2, 4, 8, 16, 32, 64])
def test_tile_order(tc):
    """tile_order (csrc/fft_large.hip) permutes each run of 8 * LG
    workgroups onto as many consecutive tiles, and the LG tiles that share a
    row's 128-byte lines land on one XCD (workgroup index mod 8)."""
    lg = 16 // tc if tc < 16 else 1
    g = 8 * lg * 5
    order = [tile_order(b, tc) for b in range(g)]
    assert sorted(order) == list(range(g))
    for run in range(0, g, 8 * lg):
        assert sorted(order[run:run + 8 * lg]) == list(range(run, run + 8 * lg))
    for b, t in enumerate(order):
        assert (t // lg) % 8 == b % 8


def tile_step_order(u, g, tiles, tc):
    lg = 16 // tc if tc < 16 else 1
    m = tiles // g
    if m < 2 or tiles % g or g % lg:
        return u
    row, p = divmod(u, tiles)
    grp, i = divmod(p, lg)
    ng = g // lg
    return row * tiles + ((grp % ng) * m + grp // ng) * lg + i


@pytest.mark.parametrize("tc,tiles", [(4, 512), (8, 512), (2, 1024), (4, 1024), (16, 512), (4, 256), (8, 128)])
def test_tile_step_order(tc, tiles):
    """The step order of the persistent tiles (TileWalk in
    csrc/fft_large.hip) permutes each problem's tiles, keeps the 16 / TC
    tiles of a line group together, and, where a row holds m >= 2 steps of
    the grid's G tiles, gives every step line groups spread over the whole
    row (step h: groups h, h + m, ...).  The kernel walks it incrementally
    (+LG, or +tiles - (m - 1) LG where h wraps, from the first tile
    (t0 div LG) m LG + t0 mod LG): checked against the definition here."""
    g = 256
    lg = 16 // tc if tc < 16 else 1
    total = 3 * tiles
    order = [tile_step_order(u, g, tiles, tc) for u in range(total)]
    assert sorted(order) == list(range(total))
    for u in range(0, total, lg):
        assert order[u:u + lg] == list(range(order[u], order[u] + lg))
    m = tiles // g
    if m >= 2:
        groups = sorted({order[u] // lg for u in range(g)})  # the first step
        assert groups == list(range(0, tiles // lg, m))
    reorder = tiles >= 2 * g and tiles % g == 0 and g % lg == 0
    mm = tiles // g if reorder else 1
    wrap = tiles - (mm - 1) * lg
    for t0 in range(g):
        tile = (t0 // lg) * mm * lg + t0 % lg if reorder else t0
        h = 0
        for t in range(t0, total, g):
            assert tile == order[t]
            tile += (lg if h + 1 < mm else wrap) if reorder else g
            h = h + 1 if h + 1 < mm else 0
