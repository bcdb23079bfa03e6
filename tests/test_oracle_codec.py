"""Pins of the oracle's indexed-map codec (Appendix B).

A map's distinct count values form an index file; pixels are replaced by the
index of their value and written with the fewest bits that hold every index.
The size rules are pinned to the paper's Tables 'max' and 'bits' (stored
under tests/golden with their citation); the encoding itself to an
independent numpy bit-packing and to exact round trips.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "appendix_b_tables.json")))


def bits_for(n_distinct):
    """Fewest bits b >= 1 with 2^b >= n_distinct (indices 0 .. n_distinct-1)."""
    return max(1, math.ceil(math.log2(n_distinct))) if n_distinct > 1 else 1


def test_bits_table_sizes_and_ranges():
    t = GOLDEN["bits_table"]
    pix = 10000 * 10000
    for b, mx, mb, tb in zip(t["bits"], t["max_integer"], t["map_size_megabytes_10000sq"],
                             t["size_70000_maps_terabytes"]):
        size = pix * b / 8
        assert round(size / 2 ** 20) == mb                     # Megabytes = 2^20 bytes
        assert abs(70000 * size / 2 ** 40 - tb) <= 0.1        # Terabytes = 2^40 bytes, rounded
        if b == 22:
            # the table prints 2^22; the largest 22-bit integer is 2^22 - 1
            assert mx == 2 ** 22 and 2 ** b - 1 == mx - 1
        else:
            assert 2 ** b - 1 == mx


def test_max_table_bit_requirements():
    """GD1's 58042 distinct values need 16-bit indices (the text's example), the
    largest ray counts need 20 bits as raw counts, and every dataset fits the
    24-bit representation the text calls sufficient."""
    m = GOLDEN["max_table"]
    assert bits_for(m["GD1"]["max_distinct_values"]) == GOLDEN["indexed_map_example"]["bits"] == 16
    assert bits_for(m["GD0"]["max_distinct_values"]) == 14
    for d in m.values():
        raw_bits = bits_for(d["max_ray_count"] + 1)
        assert raw_bits <= 24 and bits_for(d["max_distinct_values"]) <= 16
    assert bits_for(m["GD1"]["max_ray_count"] + 1) == 20
    ex = GOLDEN["index_file_example"]
    size = ex["distinct_values"] * (ex["index_bits"] + ex["value_bits"]) / 8
    assert abs(size / 1e6 - ex["megabytes"]) < 0.01


def numpy_pack(indices, b):
    """Independent packing: each index as b bits, least significant first,
    concatenated and cut into little-endian 32-bit words."""
    bits = ((indices[:, None] >> np.arange(b)[None, :]) & 1).astype(np.uint8).ravel()
    pad = (-bits.size) % 32
    bits = np.concatenate([bits, np.zeros(pad, np.uint8)])
    by = np.packbits(bits, bitorder="little")
    return by.view("<u4")


@pytest.mark.parametrize("seed,hi,shape", [(1, 1, (7, 5)), (2, 3, (64, 64)), (3, 300, (97, 33)),
                                           (4, 70000, (128, 100)), (5, 2 ** 31 - 1, (50, 41))])
def test_encode_matches_unique_and_independent_packing(seed, hi, shape):
    rng = np.random.default_rng(seed)
    c = rng.integers(0, hi, size=shape, endpoint=True).astype(np.int32)
    values, b, packed = oracle.codec_encode(c)
    u, inv = np.unique(c.ravel(), return_inverse=True)
    assert (values == u).all()
    assert b == bits_for(u.size)
    assert (packed == numpy_pack(inv.astype(np.int64), b)).all()
    back = oracle.codec_decode(packed, c.size, b, values)
    assert (back == c.ravel()).all()


def test_single_value_map_uses_one_bit():
    c = np.full((33, 17), 16, np.int32)
    values, b, packed = oracle.codec_encode(c)
    assert values.tolist() == [16] and b == 1 and not packed.any()
    assert (oracle.codec_decode(packed, c.size, b, values) == 16).all()


def test_shot_map_round_trip_and_size():
    from paper_1406_0559_amd import inputs
    spec = inputs.config_small()
    f = spec.lenses()
    c, _ = oracle.shoot(f.x1, f.x2, f.m, spec.kappa, spec.gamma, spec.s, spec.n1, spec.n2, spec.c1,
                        spec.c2, spec.h1, spec.h2, spec.p1, spec.p2, spec.w1, spec.w2, spec.W1, spec.W2)
    values, b, packed = oracle.codec_encode(c)
    assert (oracle.codec_decode(packed, c.size, b, values) == c.ravel()).all()
    assert packed.size * 4 < c.size * 4 * b / 32 + 4
    assert b < 32


def test_decode_rejects_bad_streams():
    with pytest.raises(ValueError):
        oracle.codec_decode(np.zeros(1, np.uint32), 40, 2, np.array([1], np.int32))
    packed = np.array([0xFFFFFFFF], np.uint32)
    with pytest.raises(ValueError):      # index 3 with only two values
        oracle.codec_decode(packed, 4, 2, np.array([1, 2], np.int32))
