"""MI355X (gfx950) alpha-CNG: exact-candidate alpha-convergent graph build and
batched beam search behind the C ABI of libcng.so (include/cng.h)."""
from ._lib import (NONE, CngError, Graph, build, connect, entry_point, knn, lib, prune, search,
                   u32, version)

__all__ = ["NONE", "CngError", "Graph", "build", "connect", "entry_point", "knn", "lib", "prune",
           "search", "u32", "version"]
