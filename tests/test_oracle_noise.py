"""Statistical pin: empirical output-noise variances of the oracle's blind
rotation (+ sample extraction) and key switching against the variances the
TFHE noise analysis predicts for these definitions (binary keys, gadget digits
in [-Bg/2, Bg/2), unsigned key-switch digits, every table entry noisy).

  Var_BR = n (k+1) l N E[d^2] s_glwe^2 + h_s (1 + h_S) 2^(-2 l b) / 12,
           E[d^2] = (Bg^2 + 2) / 12 (mean square of a digit),
  Var_KS = k N t s_lwe^2 + h_s' 2^(-2 t b_ks) / 12,
with h the Hamming weights of the actual keys and variances in torus units."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from helpers import enc_bits


def _signed_torus(q, x):
    x = int(x) % (1 << q)
    if x >= 1 << (q - 1):
        x -= 1 << q
    return x / float(1 << q)


@pytest.mark.slow
def test_noise_variances_toy(toy_keys):
    p = si.TOY
    K = toy_keys
    samples = 2000
    cts = enc_bits(p, K, si.bits(17, 1, samples), 900)
    tv = oracle.gate_testv(p)
    eighth = 1 << (p.q - 3)

    def one(i):
        ct = cts[i]
        big = oracle.bootstrap(p, K.bsk, ct, tv)
        out = oracle.keyswitch(p, K.ksk, big)
        phi = (oracle.mod_switch(p.q, p.N, ct[p.n])
               - sum(oracle.mod_switch(p.q, p.N, ct[j]) * int(K.s[j]) for j in range(p.n))) % (2 * p.N)
        expect = eighth if phi < p.N else (1 << p.q) - eighth
        ph_big = oracle.lwe_phase(p.q, K.sx, big)
        ph_out = oracle.lwe_phase(p.q, K.s, out)
        return (_signed_torus(p.q, ph_big - expect), _signed_torus(p.q, ph_out - ph_big))

    res = np.array(oracle.parallel_map(one, range(samples)))
    e_br, e_ks = res[:, 0], res[:, 1]
    hs, hS = int(K.s.sum()), int(K.S.sum())
    bg = 1 << p.bg_bits
    var_br = (p.n * (p.k + 1) * p.l * p.N * (bg * bg + 2) / 12.0 * 2.0 ** (-2 * p.glwe_sigma_log2)
              + hs * (1 + hS) * 2.0 ** (-2 * p.l * p.bg_bits) / 12.0)
    var_ks = (p.k * p.N * p.ks_t * 2.0 ** (-2 * p.lwe_sigma_log2)
              + hS * 2.0 ** (-2 * p.ks_t * p.ks_bits) / 12.0)
    assert abs(e_br.var() / var_br - 1) < 0.2, (e_br.var(), var_br)
    assert abs(e_ks.var() / var_ks - 1) < 0.2, (e_ks.var(), var_ks)
    assert abs(e_br.mean()) < 4 * np.sqrt(var_br / samples)


def test_forced_phase_flip_is_predicted(toy_keys):
    """Host-forced failure: moving the body of an encryption of TRUE by
    -(1/8 + d) puts its phase at about -d.  For d = +2^-5 the decryption and
    the bootstrapped copy both flip to FALSE; for d = -2^-5 both stay TRUE
    (2^-5 is about ten standard deviations of the modulus-switch rounding at
    N = 256, and the fresh noise is 2^-20)."""
    p = si.TOY
    K = toy_keys
    cts = enc_bits(p, K, [1, 1, 1, 1], 950)
    eighth = 1 << (p.q - 3)
    tv = oracle.gate_testv(p)
    for d_sign, want in ((+1, 0), (-1, 1)):
        for ct in cts:
            c = ct.copy()
            shift = eighth + d_sign * (1 << (p.q - 5))
            c[p.n] = (int(c[p.n]) - shift) % (1 << p.q)
            assert oracle.decrypt_bit(p.q, K.s, c) == want
            out = oracle.keyswitch(p, K.ksk, oracle.bootstrap(p, K.bsk, c, tv))
            assert oracle.decrypt_bit(p.q, K.s, out) == want
