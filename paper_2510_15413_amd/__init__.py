"""MI355X (gfx950) TFHE oblivious selection for FHE-SQL.

The library (``libfhesql.so``, C ABI in ``include/fhesql.h``) runs the server
hot path of FHE-SQL's oblivious selection on one GPU: TFHE gate bootstrapping
(blind rotation with an exact limb-split int8 MFMA external product, sample
extraction, key switching) inside the boolean circuits of the WHERE mask (one
predicate, many tables in one batch, or a whole expression tree), the masked
select and the masked SUM; 64-bit programmable bootstrapping over radix
blocks; and a continuous-batching query server.  This package is its thin
Python binding (``Context``, ``Server``), with client helpers (``client``:
device encryption and decryption; ``query``: WHERE syntax tree to expression
nodes), the executor autotuner (``autotune``) and the serving loop driver
(``serve``).
"""
from ._lib import (Context, Server, FheError, load, tfhe_keygen, tfhe_lwe_encrypt, tfhe_lwe_phase,  # noqa: F401
                   tfhe_rng_fill, sum_width, SQL_OPS, GATE_OPS, LIB_PATH)
