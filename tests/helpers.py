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


def edge_lwe(p, seed):
    """Small LWE inputs on the method's boundaries (TFHE bootstrapping, the
    modulus switch rounds half up): an all-zero ciphertext; noiseless bodies
    at exactly +-1/8 with a zero mask; a body with bbar = 0; masks whose
    every coefficient switches to 0, N or 2N-1 exactly; masks and bodies on
    exact modulus-switch ties k * 2^(q-lg) + 2^(q-lg-1), lg = log2(2N)
    (including 2N-1 plus a half, which rounds up to 2N = 0); the largest
    word; and mixtures of those with uniform words."""
    import numpy as np
    import seeded_inputs as si
    q, n, N = p.q, p.n, p.N
    M = (1 << q) - 1
    lg = (2 * N).bit_length() - 1
    unit, half = 1 << (q - lg), 1 << (q - lg - 1)
    rnd = si.torus(seed, 97, 64 * (n + 1), q).reshape(64, n + 1)
    pick = si.uniform_ints(seed, 98, 64 * (n + 1), 32).reshape(64, n + 1)
    rows = []
    rows.append(np.zeros(n + 1, dtype=np.uint64))
    for b in (1 << (q - 3), (-(1 << (q - 3))) & M):
        r = np.zeros(n + 1, dtype=np.uint64)
        r[n] = b
        rows.append(r)
    r = rnd[0].copy()
    r[n] = 0
    rows.append(r)
    for t in range(6):  # every mask coefficient switches to 0, N or 2N-1 exactly
        ks = np.array([(0, N, 2 * N - 1)[int(x) % 3] for x in pick[t, :n]], dtype=np.uint64)
        r = np.empty(n + 1, dtype=np.uint64)
        r[:n] = (ks * np.uint64(unit)) & np.uint64(M)
        r[n] = rnd[t + 1, n]
        rows.append(r)
    for t in range(10):  # every word on a tie
        ks = pick[10 + t] % np.uint64(2 * N)
        rows.append(((ks * np.uint64(unit) + np.uint64(half)) & np.uint64(M)).astype(np.uint64))
    r = np.full(n + 1, ((2 * N - 1) * unit + half) & M, dtype=np.uint64)  # 2N-1 + half -> 0
    rows.append(r)
    rows.append(np.full(n + 1, M, dtype=np.uint64))
    for t in range(8):  # each word a tie, an exact multiple or uniform
        sel = pick[30 + t] % np.uint64(3)
        ks = pick[40 + t] % np.uint64(2 * N)
        exact = (ks * np.uint64(unit)) & np.uint64(M)
        tie = (exact + np.uint64(half)) & np.uint64(M)
        rows.append(np.where(sel == 0, exact, np.where(sel == 1, tie, rnd[20 + t])).astype(np.uint64))
    return np.stack(rows)


def edge_big(p, seed):
    """Big LWE inputs (dimension kN) of the key switch on its rounding
    boundaries: coefficients exactly on ties of the t*b-bit rounding
    (k * 2^(q-tb) + 2^(q-tb-1)), the tie just below 2^q (rounds up to 0),
    exact multiples, zero, the largest word, and mixtures with uniform words."""
    import numpy as np
    import seeded_inputs as si
    q, d = p.q, p.k * p.N
    M = (1 << q) - 1
    tb = p.ks_t * p.ks_bits
    if tb >= q:
        unit, half = 1, 0
    else:
        unit, half = 1 << (q - tb), 1 << (q - tb - 1)
    rnd = si.torus(seed, 95, 24 * (d + 1), q).reshape(24, d + 1)
    pick = si.uniform_ints(seed, 96, 24 * (d + 1), 32).reshape(24, d + 1)
    K = 1 << min(tb, 32)
    rows = [np.zeros(d + 1, dtype=np.uint64), np.full(d + 1, M, dtype=np.uint64)]
    rows.append(np.full(d + 1, (M - half + 1) & M, dtype=np.uint64))  # 2^q - half: rounds to 2^(tb) = 0
    for t in range(6):
        ks = pick[t] % np.uint64(K)
        rows.append(((ks * np.uint64(unit) + np.uint64(half)) & np.uint64(M)).astype(np.uint64))
    for t in range(4):
        ks = pick[6 + t] % np.uint64(K)
        rows.append(((ks * np.uint64(unit)) & np.uint64(M)).astype(np.uint64))
    for t in range(6):
        sel = pick[12 + t] % np.uint64(3)
        ks = pick[18 + t % 6] % np.uint64(K)
        exact = (ks * np.uint64(unit)) & np.uint64(M)
        tie = (exact + np.uint64(half)) & np.uint64(M)
        rows.append(np.where(sel == 0, exact, np.where(sel == 1, tie, rnd[t])).astype(np.uint64))
    return np.stack(rows)
