"""MI355X (gfx950) library for exhaustive, incrementally bounded checking of
quantized MLPs and their neuron-pair coverage (after arXiv 1907.12933).

The compute path is libibmc.so (hand-written HIP kernels behind the C ABI in
include/ibmc.h); paper_1907_12933_amd.ibmc is its ctypes binding and
paper_1907_12933_amd.inputs holds the seeded synthetic workloads.
"""
