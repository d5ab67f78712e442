"""Plain CPU reference of full-RNS CKKS.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product library never imports it.
"""
from .ckks import OracleCtx, Ct, load_params  # noqa: F401
