"""Test helpers: encryption and decryption of bit-encoded values with the
oracle (test infrastructure), and plain-Python reference polynomials."""
import numpy as np

import oracle
import seeded_inputs as si


def enc_bits(p, keys, bits, seed, tag_hi=0):
    """Encrypt bits with the gate encoding (2b - 1)/8 under the LWE key."""
    bits = np.asarray(bits, dtype=np.uint64).ravel()
    masks, errs = si.lwe_randomness(p, seed, bits.size, tag_hi=tag_hi)
    eighth = 1 << (p.q - 3)
    mus = np.where(bits == 1, eighth, (-eighth) & ((1 << p.q) - 1)).astype(np.uint64)
    return oracle.lwe_encrypt(p, keys.s, masks, errs, mus)


def dec_bits(p, keys, cts):
    cts = np.asarray(cts, dtype=np.uint64)
    flat = cts.reshape(-1, p.n + 1)
    out = np.array([oracle.decrypt_bit(p.q, keys.s, c) for c in flat], dtype=np.int64)
    return out.reshape(cts.shape[:-1])


def bits_to_int(bits):
    return sum(int(b) << j for j, b in enumerate(bits))


def py_monomial(q, N, e, poly):
    """X^e * poly mod (X^N + 1, 2^q), written from the exponent rule
    X^(j+e) = (-1)^floor((j+e)/N) X^((j+e) mod N)."""
    out = [0] * N
    for j, c in enumerate(poly):
        t = j + int(e)
        sign = -1 if (t // N) % 2 else 1
        out[t % N] = (out[t % N] + sign * int(c)) % (1 << q)
    return out


def torus_dist(q, a, b):
    d = (int(a) - int(b)) % (1 << q)
    return min(d, (1 << q) - d)
