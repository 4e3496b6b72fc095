"""The oracle: a plain, slow CPU FP64 bidiagonal divide-and-conquer SVD.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or run anything in this package; the library and
its Python binding never do, and the oracle imports nothing from them.  It is
written from Section 4.2.1 of the paper (Algorithm 2 and the equations of the
merge step) and the published methods it cites (Gu & Eisenstat's
recomputation of z; Golub-Kahan QR for the leaves; R.-C. Li's rational
iteration for the secular equation), in NumPy float64 without fused
multiply-add.

Pinned (tests marked "not gpu") against closed forms, invariants, brute force
and library routines; see tests/test_oracle_*.py.
"""

from .bdc import (  # noqa: F401
    DEFL_CLOSE,
    DEFL_SMALL_Z,
    DEFL_ZERO_D,
    SURVIVOR,
    Node,
    Prep,
    bdsdc,
    build_tree,
    dense,
    deflate,
    merge_prep,
    merge_sort_order,
    merge_values,
    scale_of,
    tree_nodes,
)
from .leaf import leaf_svd  # noqa: F401
from .secular import lowner_z, secular_roots, vectors  # noqa: F401
from . import learned  # noqa: F401
