"""LCP particle compressor (arXiv 2411.00761) on MI355X: LCP-S / LCP-T in HIP.

The compute path is the HIP library liblcp_hip.so behind the C ABI in
include/lcp.h; `lcp` is its Python binding and `datagen` the seeded synthetic
workloads.
"""
__all__ = ["lcp", "datagen"]
