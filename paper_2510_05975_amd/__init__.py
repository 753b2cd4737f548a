"""MI355X (gfx950) alpha-CNG: exact-candidate alpha-convergent graph build and
batched beam search behind the C ABI of libcng.so (include/cng.h)."""
from ._lib import (BF16, F32, FP8, NONE, CngError, Graph, Server, Store, backward, build, connect,
                   entry_point, graph_candidates, knn, lib, nndescent, prune, quantize, search,
                   search_quantized, u32, version)

__all__ = ["BF16", "F32", "FP8", "NONE", "CngError", "Graph", "Server", "Store", "backward", "build",
           "connect",
           "entry_point", "graph_candidates", "knn", "lib", "nndescent", "prune", "quantize", "search", "search_quantized", "u32",
           "version"]
