"""CPU oracle of the Hough track finder -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product (``paper_2511_02742_amd``)
never imports it, and it never imports the product.
"""
from .oracle import (OracleConfig, TwConfig, build_oracle, cand_dtype, oracle_acc_after, oracle_bin,
                     oracle_fill, oracle_find, oracle_find_batch, oracle_peaks, oracle_tables,
                     oracle_tw_find_batch, track_dtype)

__all__ = ["OracleConfig", "TwConfig", "build_oracle", "cand_dtype", "oracle_acc_after", "oracle_bin",
           "oracle_fill", "oracle_find", "oracle_find_batch", "oracle_peaks", "oracle_tables",
           "oracle_tw_find_batch", "track_dtype"]
