"""Seeded synthetic workloads: BG-shaped QC-LDPC graphs, GF(2) encoders,
BPSK/AWGN channel and int8 quantiser. Inputs only -- no decoding arithmetic;
shared by the CPU oracle's tests and the GPU path's tests and benchmark."""
from .channel import (Batch, LLR_SCALE, make_batch, make_batch_parallel, noiseless_q, quantize,
                      sigma2)
from .encoder import ElimEncoder, encode, syndrome
from .graph import GRAPH_SEED, LIFTS, BaseGraph, full_shape, make_graph, make_toy_graph

__all__ = [
    "Batch", "LLR_SCALE", "make_batch", "make_batch_parallel", "noiseless_q", "quantize", "sigma2",
    "ElimEncoder", "encode", "syndrome", "GRAPH_SEED", "LIFTS", "BaseGraph",
    "full_shape", "make_graph", "make_toy_graph",
]
