"""ORACLE -- test infrastructure only.

A plain, slow, FP64 CPU implementation of what the GPU path computes, written
from the paper: Algorithm 1 (solver-free componentwise ADMM) in `admm`, and an
independently assembled centralised LP of the same model for brute-force
checks in `central`.  Only tests, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product library never does, and the two share
no code.
"""
