"""FP64 CPU oracle of JPEG XL VarDCT reconstruction -- test infrastructure only.

Only tests/, the smoke check and the CPU-baseline leg of bench.py may import
this package; the product path never does.
"""
