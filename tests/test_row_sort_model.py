"""Host model of the in-place row sort's networks (no GPU): the lane permutations its
cross-lane exchanges are built from, and the grouped bitonic network (a group of G lanes, 16
entries per lane, one row per group) run on every group size with ragged row lengths.

The lane maps follow the published DPP / swizzle definitions of the GCN and CDNA ISA:
quad_perm selects inside groups of 4 lanes, row_mirror reverses each row of 16 lanes,
row_half_mirror each half row of 8, and the bit-mode swizzle maps lane l of a 32-lane half
to ((l & and) | or) ^ xor."""
import numpy as np
import pytest

LANES = 64


def quad_perm(sel):
    return [4 * (l // 4) + sel[l % 4] for l in range(LANES)]


def row_mirror():
    return [16 * (l // 16) + 15 - l % 16 for l in range(LANES)]


def row_half_mirror():
    return [8 * (l // 8) + 7 - l % 8 for l in range(LANES)]


def swizzle_bitmode(and_mask, or_mask, xor_mask):
    return [32 * (l // 32) + (((l % 32) & and_mask) | or_mask) ^ xor_mask for l in range(LANES)]


def then(first, second):
    """lane l reads, after `first` then `second` (each a source-lane map), the value of lane
    first[second[l]]"""
    return [first[second[l]] for l in range(LANES)]


def test_lane_exchange_identities():
    xor = lambda k: [l ^ k for l in range(LANES)]
    assert quad_perm([1, 0, 3, 2]) == xor(1)
    assert quad_perm([2, 3, 0, 1]) == xor(2)
    assert then(row_half_mirror(), quad_perm([3, 2, 1, 0])) == xor(4)
    assert then(row_mirror(), row_half_mirror()) == xor(8)
    assert swizzle_bitmode(0x1F, 0, 0x10) == xor(16)
    # the DPP control words of these moves: quad_perm packs the 4 selectors, 2 bits each
    enc = lambda sel: sum(s << (2 * i) for i, s in enumerate(sel))
    assert (enc([1, 0, 3, 2]), enc([2, 3, 0, 1]), enc([3, 2, 1, 0])) == (0xB1, 0x4E, 0x1B)
    # the swizzle offset: and mask in bits 0-4, or in 5-9, xor in 10-14
    assert 0x1F | (0 << 5) | (0x10 << 10) == 0x401F


def group_sort(rows, G, E=16):
    """The kernel's grouped network on one wave: group q = lanes q G .. q G + G - 1 holds row
    q (len <= G E) padded with the maximum, lane g of the group positions g E .. g E + E - 1;
    strides below E compare inside a lane, the others exchange with lane g ^ (stride / E)."""
    P = G * E
    per = LANES // G
    assert len(rows) <= per
    v = np.full((LANES, E), np.iinfo(np.uint32).max, dtype=np.uint64)
    for q, row in enumerate(rows):
        assert len(row) <= P
        for i, x in enumerate(row):
            v[q * G + i // E, i % E] = x
    lane = np.arange(LANES)
    g = lane % G
    k = 2
    while k <= P:
        st = k // 2
        while st:
            if st >= E:
                ls = st // E
                partner = lane ^ ls
                y = v[partner].copy()
                i = g[:, None] * E + np.arange(E)[None, :]
                lower = (i & st) == 0
                asc = (i & k) == 0
                v = np.where(lower == asc, np.minimum(v, y), np.maximum(v, y))
            else:
                for j in range(E):
                    q = j ^ st
                    if q > j:
                        i = g * E + j
                        a, b = v[:, j].copy(), v[:, q].copy()
                        up = (i & k) == 0
                        v[:, j] = np.where(up, np.minimum(a, b), np.maximum(a, b))
                        v[:, q] = np.where(up, np.maximum(a, b), np.minimum(a, b))
            st //= 2
        k *= 2
    return [[int(x) for x in v[q * G:(q + 1) * G].reshape(-1)[:len(row)]]
            for q, row in enumerate(rows)]


@pytest.mark.parametrize("C", range(7))
def test_grouped_bitonic_network_sorts_every_class(C):
    """Groups of G = 2^C lanes sort rows of up to 16 G entries: full, ragged and one-entry
    rows, repeated values, all groups of the wave busy."""
    G = 1 << C
    rng = np.random.default_rng(C)
    cap = 16 * G
    lengths = [cap, 1, max(1, cap // 2 + 1), max(1, cap - 3)]
    rows = []
    for q in range(LANES // G):
        n = lengths[q % len(lengths)]
        rows.append(rng.integers(0, 1 << 23, n).tolist() if q % 3 else
                    rng.integers(0, 5, n).tolist())
    out = group_sort(rows, G)
    for row, got in zip(rows, out):
        assert got == sorted(row)


def test_size_classes_cover_the_wave_rows():
    """The class of a row of L entries (1 <= L <= 1024) is the smallest C with 16 * 2^C >= L,
    computed in the kernel as 32 - clz(L - 1) - 4 above 16 entries."""
    def cls(L):
        return 0 if L <= 16 else 32 - (32 - (L - 1).bit_length()) - 4
    for L in range(1, 1025):
        C = cls(L)
        assert 16 << C >= L and (C == 0 or 16 << (C - 1) < L), L
        assert C <= 6
