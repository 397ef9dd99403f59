"""MI355X (gfx950) TFHE oblivious selection for FHE-SQL.

The library (``libfhesql.so``, C ABI in ``include/fhesql.h``) runs the server
hot path of FHE-SQL's oblivious selection on one GPU: TFHE gate bootstrapping
(blind rotation with an exact limb-split int8 MFMA external product, sample
extraction, key switching) inside the boolean circuits of the WHERE mask, the
masked select and the masked SUM.  This package is its thin Python binding.
"""
from ._lib import (Context, Server, FheError, load, tfhe_keygen, tfhe_lwe_encrypt, tfhe_lwe_phase,  # noqa: F401
                   tfhe_rng_fill, sum_width, SQL_OPS, GATE_OPS, LIB_PATH)
