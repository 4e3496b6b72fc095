"""MI355X bidiagonal divide-and-conquer SVD (B = U Sigma V^T, FP64, full
vectors) on hand-written HIP kernels for gfx950.

``Solver`` / ``svd`` (module ``api``) call the C ABI of libbdc.so; importing
this package does not load the library or torch, so the ``inputs`` submodule
can be used alone.
"""

__all__ = ["Solver", "svd"]


def __getattr__(name):
    if name in ("Solver", "svd"):
        import importlib

        api = importlib.import_module(__name__ + ".api")
        return getattr(api, name)
    raise AttributeError(name)
