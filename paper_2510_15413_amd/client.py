"""Client-side helpers on the device: bit encoding, seeded encryption and
decryption of bit-wise encrypted integers and the filtering of the returned
rows (the client steps of Algorithm 1: EncryptQuery, Decrypt and
FilterZeroRows), built on the library's kernels."""
from __future__ import annotations

import torch

from . import _lib


def bit_mu(p, bits: torch.Tensor) -> torch.Tensor:
    """Gate encoding (2b - 1)/8 of a tensor of bits, as torus words."""
    e = 1 << (p.q - 3)
    dt = _lib.torch_dtype(p.q)
    bits = bits.to(device="cuda", dtype=torch.int64)
    mu = torch.where(bits != 0, torch.tensor(e, dtype=torch.int64, device="cuda"),
                     torch.tensor(-e, dtype=torch.int64, device="cuda"))
    return mu.to(dt) if p.q == 32 else mu


def value_bits(values: torch.Tensor, w: int) -> torch.Tensor:
    """[rows][w] bits, least significant first."""
    v = values.to(device="cuda", dtype=torch.int64)
    sh = torch.arange(w, device="cuda", dtype=torch.int64)
    return (v[:, None] >> sh[None, :]) & 1


def encrypt_bits(p, seed, key, bits: torch.Tensor, tag_hi=0, start=0) -> torch.Tensor:
    """Encrypt a [..] tensor of bits: result [.., n+1]."""
    mu = bit_mu(p, bits.reshape(-1))
    out = _lib.tfhe_lwe_encrypt(p, seed, key, mu, start=start, tag_hi=tag_hi)
    return out.reshape(*bits.shape, p.n + 1)


def decrypt_bits(p, key, cts: torch.Tensor, dim=None) -> torch.Tensor:
    """Bit = 1 iff the phase read as a signed q-bit integer is > 0."""
    ph = _lib.tfhe_lwe_phase(p, key, cts, dim=dim)
    return (ph > 0).to(torch.int64)


def bits_to_values(bits: torch.Tensor) -> torch.Tensor:
    w = bits.shape[-1]
    sh = torch.arange(w, device=bits.device, dtype=torch.int64)
    return (bits.to(torch.int64) << sh).sum(-1)


def decrypt_values(p, key, cts: torch.Tensor) -> torch.Tensor:
    """Integers of bit-wise encrypted values [.., w, n+1] -> [..]."""
    return bits_to_values(decrypt_bits(p, key, cts))


def filter_zero_rows(p, key, selected: torch.Tensor):
    """FilterZeroRows after Decrypt: the server returns If-Then-Else(mask, v,
    enc(0)) for every row, so unmatched rows decrypt to zero.  selected:
    [rows, w, n+1] (one column) or [rows, cols, w, n+1].  Returns (indices of
    rows with a non-zero value in some column, their decrypted values)."""
    vals = decrypt_values(p, key, selected)
    if vals.dim() == 1:
        vals = vals[:, None]
    keep = (vals != 0).any(dim=1).nonzero().flatten()
    return keep, vals[keep]
