"""Pins of the shared seeded generator (no TFHE arithmetic lives there)."""
import numpy as np

import seeded_inputs as si


def test_splitmix64_published_vector():
    # SplitMix64 from state 1234567: the first five outputs of the reference
    # implementation (Vigna's splitmix64.c).
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    s, got = 1234567, []
    for _ in range(5):
        s = (s + si.GAMMA) & si.MASK64
        got.append(si.mix64_int(s))
    assert got == expect


def test_counter_form_matches_sequential():
    key = si.stream_key(77, 5)
    s, seq = key, []
    for _ in range(10):
        s = (s + si.GAMMA) & si.MASK64
        seq.append(si.mix64_int(s))
    assert [int(v) for v in si.raw(77, 5, 10)] == seq
    assert [int(v) for v in si.raw(77, 5, 4, start=6)] == seq[6:]


def test_chunking_is_invisible():
    n = (1 << 19) + 1234
    a = si.raw(3, 9, n)
    b = si.raw(3, 9, 1000, start=(1 << 19) - 500)
    assert np.array_equal(a[(1 << 19) - 500:(1 << 19) + 500], b)


def test_noise_moments():
    q, s = 32, 20
    e = si.noise(11, 4, 200000, q, s).astype(np.int64)
    e = np.where(e >= (1 << 31), e - (1 << 32), e)
    sd = 2.0 ** (q - s)
    assert abs(e.mean()) < 0.02 * sd
    assert abs(e.std() / sd - 1.0) < 0.01
    assert np.abs(e).max() <= 6 * sd + 1
    # 64-bit torus with a left scale
    e64 = si.noise(11, 4, 50000, 64, 20)
    v = np.array([int(x) - (1 << 64) if int(x) >= (1 << 63) else int(x) for x in e64[:5000]], dtype=float)
    assert abs(v.std() / 2.0 ** 44 - 1.0) < 0.05


def test_bits_and_ints_uniform():
    b = si.bits(5, 1, 100000)
    assert set(np.unique(b)) <= {0, 1} and abs(b.mean() - 0.5) < 0.01
    u = si.uniform_ints(5, 9, 100000, 8)
    assert u.max() <= 255 and abs(u.mean() - 127.5) < 1.5


def test_uneven_tables_shape():
    rows, ops = si.uneven_tables(si.DATA_SEED_BASE + 3)
    assert len(rows) == 16 and rows.min() >= 100 and rows.max() <= 65536
    assert set(ops.tolist()) <= {0, 1, 2}
